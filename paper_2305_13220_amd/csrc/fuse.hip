// Producing the voxels of a grid: depth, colour and semantic fusion
// (Sec. 3.4.2) -- each voxel is projected into every frame and the
// associated observations are averaged (the closed-form minimisers of the
// per-voxel squared losses) -- and the Gaussian de-noising of Sec. 3.4.3.
#include <climits>
#include <cmath>

#include "common.h"

namespace sg {

// One lane per voxel; frames in order, so the sums (and the result bits) do
// not depend on the launch.  Camera rows are read with scalar loads (the
// frame index is uniform).  The association decisions are float32 with no
// fused multiply-add, in the order written.
template <int C>
__global__ __launch_bounds__(256) void k_fuse(const int32_t* __restrict__ coords, int64_t n_vox,
                                              float h, float ox, float oy, float oz,
                                              const float* __restrict__ cams, int32_t F,
                                              const float* __restrict__ depth,
                                              const float* __restrict__ feat, int32_t W,
                                              int32_t H, float trunc, int32_t n_sem,
                                              float* __restrict__ vox,
                                              float* __restrict__ weight) {
#pragma clang fp contract(off)
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_vox) return;
  const int64_t b = v >> 9;
  const int l = (int)(v & 511);
  const int li[3] = {l & 7, (l >> 3) & 7, l >> 6};
  const float org[3] = {ox, oy, oz};
  float X[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float fi = (float)(8 * coords[3 * b + a] + li[a]);
    const float step = fi * h;
    X[a] = org[a] + step;
  }
  float sd = 0.0f, acc[C > 0 ? C : 1];
#pragma unroll
  for (int ch = 0; ch < C; ++ch) acc[ch] = 0.0f;
  int32_t cnt = 0;
  const int64_t plane = (int64_t)W * H;
  for (int32_t f = 0; f < F; ++f) {
    const float* K = cams + 16 * (int64_t)f;
    const float dd[3] = {X[0] - K[7], X[1] - K[11], X[2] - K[15]};
    float c[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float p0 = K[4 + j] * dd[0];
      const float p1 = K[8 + j] * dd[1];
      const float p2 = K[12 + j] * dd[2];
      c[j] = (p0 + p1) + p2;
    }
    const float z = c[2];
    if (!(z > 0.0f)) continue;
    const float qx = c[0] / z, qy = c[1] / z;
    const float uf = K[0] * qx + K[2];
    const float vf = K[1] * qy + K[3];
    if (!(uf >= 0.0f && uf < (float)W && vf >= 0.0f && vf < (float)H)) continue;
    const int64_t pix = f * plane + (int64_t)(int32_t)floorf(vf) * W + (int32_t)floorf(uf);
    const float D = depth[pix];
    if (!(isfinite(D) && D > 0.0f)) continue;
    const float s = D - z;
    if (!(s >= -trunc)) continue;  // occluded: more than trunc behind the surface
    sd += fminf(s, trunc);
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] += feat[pix * C + ch];
    ++cnt;
  }
  float* o = vox + v * (1 + C);
  if (weight) weight[v] = (float)cnt;
  if (cnt == 0) {
    o[0] = trunc;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) o[1 + ch] = 0.0f;
    return;
  }
  const float inv = 1.0f / (float)cnt;
  o[0] = sd * inv;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) acc[ch] *= inv;
  float nrm = 0.0f;
#pragma unroll
  for (int ch = 0; ch < C; ++ch)
    if (ch >= C - n_sem) nrm += acc[ch] * acc[ch];
  nrm = sqrtf(nrm);
#pragma unroll
  for (int ch = 0; ch < C; ++ch) {
    float val = acc[ch];
    if (ch >= C - n_sem) val = nrm > 0.0f ? val / nrm : 0.0f;
    o[1 + ch] = val;
  }
}

// Gaussian blur over allocated voxels (Sec. 3.4.3): one workgroup per block,
// one lane per voxel.  The 27 blocks around the block (radius <= 8 keeps
// every neighbourhood within them) are resolved once into LDS; each voxel
// then sums w(d) theta(v + d) and w(d) over the offsets whose block exists
// and divides (the weights renormalise where the neighbourhood leaves the
// grid).  Reads of neighbouring voxels are shared through the caches.
template <int C>
__global__ __launch_bounds__(512) void k_denoise(GridView g, const int32_t* __restrict__ coords,
                                                 const float* __restrict__ vox, int32_t radius,
                                                 float inv_2s2, float* __restrict__ out) {
  constexpr int V = 1 + C;
  __shared__ int32_t nb[27];
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x;
  const int32_t bc[3] = {coords[3 * b], coords[3 * b + 1], coords[3 * b + 2]};
  if (t < 27) {
    const int32_t x = bc[0] + t % 3 - 1, y = bc[1] + (t / 3) % 3 - 1, z = bc[2] + t / 9 - 1;
    int32_t idx = -1, nm = 0, dist = 0;
    if (x >= g.bmin[0] && x <= g.bmax[0] && y >= g.bmin[1] && y <= g.bmax[1] && z >= g.bmin[2] &&
        z <= g.bmax[2])
      block_state(g, x, y, z, idx, nm, dist);
    nb[t] = idx;
  }
  __syncthreads();
  const int l[3] = {t & 7, (t >> 3) & 7, t >> 6};
  float acc[V], wsum = 0.0f;
#pragma unroll
  for (int ch = 0; ch < V; ++ch) acc[ch] = 0.0f;
  for (int dz = -radius; dz <= radius; ++dz)
    for (int dy = -radius; dy <= radius; ++dy)
      for (int dx = -radius; dx <= radius; ++dx) {
        const int jx = l[0] + dx, jy = l[1] + dy, jz = l[2] + dz;
        // block offset in {-1, 0, 1} per axis (floor division by 8)
        const int ox = (jx >> 3) + 1, oy = (jy >> 3) + 1, oz = (jz >> 3) + 1;
        const int32_t n = nb[ox + 3 * oy + 9 * oz];
        if (n < 0) continue;
        const float w = expf(-(float)(dx * dx + dy * dy + dz * dz) * inv_2s2);
        const float* th = vox + ((int64_t)n * SG_BLOCK_VOXELS + (jx & 7) + 8 * (jy & 7) +
                                 64 * (jz & 7)) * V;
        wsum += w;
#pragma unroll
        for (int ch = 0; ch < V; ++ch) acc[ch] += w * th[ch];
      }
  float* o = out + (b * SG_BLOCK_VOXELS + t) * V;
  const float inv = 1.0f / wsum;  // > 0: the voxel itself is allocated
#pragma unroll
  for (int ch = 0; ch < V; ++ch) o[ch] = acc[ch] * inv;
}

// The same blur, separably, through an LDS tile (radius <= kTileR).  The
// Gaussian weight of an offset is the product of three 1-D weights, and the
// two sums of the renormalised blur, of m theta and of the allocation mask
// m, are both convolutions with it: each is taken as three 1-D passes.  The
// tile holds the block and its halo, side^3 voxels (side = 8 + 2 radius),
// four channels at a time (one 16-byte load per voxel when 1 + C is a
// multiple of four, with consecutive lanes on consecutive voxels); the x
// pass reduces it to an (8, side, side) slab, the y pass to (8, 8, side)
// (written over the tile), the z pass to the block's 512 voxels, one per
// lane.  The mask is filtered the same way once, before the channels.
// `vec`: both arrays are 16-byte aligned, so a voxel's channels c0..c0+3 are
// one 16-byte access when 1 + C is a multiple of four.
// Results equal k_denoise's up to rounding order.
constexpr int kTileR = 2;

__host__ __device__ constexpr int denoise_side(int radius) { return 8 + 2 * radius; }

// LDS bytes of the separable kernel: the tile (side^3) and the slab of the
// x pass (8 side^2), float4 each.
static size_t denoise_lds_bytes(int radius) {
  const size_t side = (size_t)denoise_side(radius);
  return (side * side * side + 8 * side * side) * sizeof(float4);
}

template <int C>
__global__ __launch_bounds__(512) void k_denoise_sep(GridView g, const int32_t* __restrict__ coords,
                                                     const float* __restrict__ vox, int32_t radius,
                                                     float inv_2s2, float* __restrict__ out,
                                                     bool vec) {
  constexpr int V = 1 + C;
  extern __shared__ float4 lds4[];
  __shared__ int32_t nb[27];
  __shared__ float w1[2 * kTileR + 1];
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x;
  const int side = denoise_side(radius), kw = 2 * radius + 1;
  const int n_tile = side * side * side, n_x = 8 * side * side, n_y = 64 * side;
  float4* A = lds4;           // tile, then the y pass
  float4* B = lds4 + n_tile;  // x pass
  float* Am = reinterpret_cast<float*>(A);
  float* Bm = reinterpret_cast<float*>(B);
  const int32_t bc[3] = {coords[3 * b], coords[3 * b + 1], coords[3 * b + 2]};
  if (t < 27) {
    const int32_t x = bc[0] + t % 3 - 1, y = bc[1] + (t / 3) % 3 - 1, z = bc[2] + t / 9 - 1;
    int32_t idx = -1, nm = 0, dist = 0;
    if (x >= g.bmin[0] && x <= g.bmax[0] && y >= g.bmin[1] && y <= g.bmax[1] && z >= g.bmin[2] &&
        z <= g.bmax[2])
      block_state(g, x, y, z, idx, nm, dist);
    nb[t] = idx;
  }
  if (t < kw) {
    const int d = t - radius;
    w1[t] = expf(-(float)(d * d) * inv_2s2);
  }
  __syncthreads();
  // Block index of tile voxel e ((x, y, z), x fastest, at offset -radius) and
  // the element offset of that voxel, or -1 where its block is absent.
  auto tile_voxel = [&](int e) -> int64_t {
    const int x = e % side - radius, y = (e / side) % side - radius, z = e / (side * side) - radius;
    const int32_t n = nb[((x >> 3) + 1) + 3 * ((y >> 3) + 1) + 9 * ((z >> 3) + 1)];
    return n < 0 ? -1 : (int64_t)n * SG_BLOCK_VOXELS + (x & 7) + 8 * (y & 7) + 64 * (z & 7);
  };
  const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
  // The mask: tile, x, y and z passes; wsum > 0 (the voxel itself is allocated).
  for (int e = t; e < n_tile; e += 512) Am[e] = tile_voxel(e) >= 0 ? 1.0f : 0.0f;
  __syncthreads();
  for (int e = t; e < n_x; e += 512) {
    const int xo = e & 7, yz = e >> 3;
    float a = 0.0f;
    for (int i = 0; i < kw; ++i) a += w1[i] * Am[xo + i + side * yz];
    Bm[e] = a;
  }
  __syncthreads();
  for (int e = t; e < n_y; e += 512) {
    const int xo = e & 7, yo = (e >> 3) & 7, z = e >> 6;
    float a = 0.0f;
    for (int i = 0; i < kw; ++i) a += w1[i] * Bm[xo + 8 * ((yo + i) + side * z)];
    Am[e] = a;
  }
  __syncthreads();
  float wsum = 0.0f;
  for (int i = 0; i < kw; ++i) wsum += w1[i] * Am[lx + 8 * (ly + 8 * (lz + i))];
  const float inv = 1.0f / wsum;
  float* o = out + (b * SG_BLOCK_VOXELS + t) * V;
  for (int c0 = 0; c0 < V; c0 += 4) {
    __syncthreads();  // the previous passes' reads of A are done
    for (int e = t; e < n_tile; e += 512) {
      const int64_t off = tile_voxel(e);
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (off >= 0) {
        const float* th = vox + off * V + c0;
        if (V % 4 == 0 && vec) {
          v = *reinterpret_cast<const float4*>(th);
        } else {
          v.x = th[0];
          if (c0 + 1 < V) v.y = th[1];
          if (c0 + 2 < V) v.z = th[2];
          if (c0 + 3 < V) v.w = th[3];
        }
      }
      A[e] = v;
    }
    __syncthreads();
    for (int e = t; e < n_x; e += 512) {
      const int xo = e & 7, yz = e >> 3;
      float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (int i = 0; i < kw; ++i) {
        const float w = w1[i];
        const float4 v = A[xo + i + side * yz];
        a.x += w * v.x;
        a.y += w * v.y;
        a.z += w * v.z;
        a.w += w * v.w;
      }
      B[e] = a;
    }
    __syncthreads();
    for (int e = t; e < n_y; e += 512) {
      const int xo = e & 7, yo = (e >> 3) & 7, z = e >> 6;
      float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (int i = 0; i < kw; ++i) {
        const float w = w1[i];
        const float4 v = B[xo + 8 * ((yo + i) + side * z)];
        a.x += w * v.x;
        a.y += w * v.y;
        a.z += w * v.z;
        a.w += w * v.w;
      }
      A[e] = a;
    }
    __syncthreads();
    float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int i = 0; i < kw; ++i) {
      const float w = w1[i];
      const float4 v = A[lx + 8 * (ly + 8 * (lz + i))];
      a.x += w * v.x;
      a.y += w * v.y;
      a.z += w * v.z;
      a.w += w * v.w;
    }
    if (V % 4 == 0 && vec) {
      *reinterpret_cast<float4*>(o + c0) = make_float4(a.x * inv, a.y * inv, a.z * inv, a.w * inv);
    } else {
      o[c0] = a.x * inv;
      if (c0 + 1 < V) o[c0 + 1] = a.y * inv;
      if (c0 + 2 < V) o[c0 + 2] = a.z * inv;
      if (c0 + 3 < V) o[c0 + 3] = a.w * inv;
    }
  }
}

static bool fuse_C(int C) {
  return C == 0 || C == 1 || C == 2 || C == 3 || C == 4 || C == 8 || C == 16 || C == 19 ||
         C == 32;
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_fuse(const sg_grid* grid, const float* d_cams, int32_t n_frames, const float* d_depth,
            const float* d_feat, int32_t C, int32_t W, int32_t H, float trunc, int32_t n_sem,
            float* d_vox, float* d_weight, sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!fuse_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_sem < 0 || n_sem > C) return fail(SG_EINVAL, "n_sem must be in [0, C]");
  if (n_frames < 0 || W < 0 || H < 0) return fail(SG_EINVAL, "sizes must be >= 0");
  if ((int64_t)W * H > (int64_t)INT_MAX) return fail(SG_EINVAL, "frame larger than 2^31-1 pixels");
  if (!(trunc > 0.0f) || !std::isfinite(trunc)) return fail(SG_EINVAL, "trunc must be finite and > 0");
  if (!d_vox) return fail(SG_EINVAL, "d_vox is NULL");
  if (n_frames > 0 && (!d_cams || !d_depth || (C > 0 && !d_feat)))
    return fail(SG_EINVAL, "a required pointer is NULL");
  const int64_t n_vox = grid->n_blocks * SG_BLOCK_VOXELS;
  if (n_vox == 0) return SG_OK;
  const int64_t blocks = (n_vox + 255) / 256;
  if (blocks > INT_MAX) return fail(SG_EINVAL, "too many voxels for one launch");
  hipStream_t s = (hipStream_t)stream;
  switch (C) {
#define SG_FUSE_CASE(CC)                                                                        \
  case CC:                                                                                      \
    hipLaunchKernelGGL(k_fuse<CC>, dim3((unsigned)blocks), dim3(256), 0, s, grid->d_coords,      \
                       n_vox, grid->h, grid->org[0], grid->org[1], grid->org[2], d_cams,        \
                       n_frames, d_depth, d_feat, W, H, trunc, n_sem, d_vox, d_weight);         \
    break;
    SG_FUSE_CASE(0)
    SG_FUSE_CASE(1)
    SG_FUSE_CASE(2)
    SG_FUSE_CASE(3)
    SG_FUSE_CASE(4)
    SG_FUSE_CASE(8)
    SG_FUSE_CASE(16)
    SG_FUSE_CASE(19)
    SG_FUSE_CASE(32)
#undef SG_FUSE_CASE
    default:
      break;
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_denoise(const sg_grid* grid, const float* d_vox, int32_t C, int32_t radius, float sigma,
               float* d_out, sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!fuse_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (radius < 0 || radius > 8) return fail(SG_EINVAL, "radius must be in [0, 8]");
  if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fail(SG_EINVAL, "sigma must be finite and > 0");
  if (!d_vox || !d_out) return fail(SG_EINVAL, "a required pointer is NULL");
  if (d_vox == d_out) return fail(SG_EINVAL, "d_out must not be d_vox (the blur is not in place)");
  if (grid->n_blocks == 0) return SG_OK;
  if (grid->n_blocks > INT_MAX) return fail(SG_EINVAL, "too many blocks for one launch");
  const GridView g = view_of(grid);
  const float inv_2s2 = (float)(1.0 / (2.0 * (double)sigma * (double)sigma));
  const bool vec = reinterpret_cast<uintptr_t>(d_vox) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(d_out) % 16 == 0;
  hipStream_t s = (hipStream_t)stream;
  switch (C) {
#define SG_DENOISE_CASE(CC)                                                                 \
  case CC:                                                                                  \
    if (radius <= kTileR)                                                                   \
      hipLaunchKernelGGL(k_denoise_sep<CC>, dim3((unsigned)grid->n_blocks), dim3(512),      \
                         denoise_lds_bytes(radius), s, g, grid->d_coords, d_vox, radius,    \
                         inv_2s2, d_out, vec);                                              \
    else                                                                                    \
      hipLaunchKernelGGL(k_denoise<CC>, dim3((unsigned)grid->n_blocks), dim3(512), 0, s, g,  \
                         grid->d_coords, d_vox, radius, inv_2s2, d_out);                    \
    break;
    SG_DENOISE_CASE(0)
    SG_DENOISE_CASE(1)
    SG_DENOISE_CASE(2)
    SG_DENOISE_CASE(3)
    SG_DENOISE_CASE(4)
    SG_DENOISE_CASE(8)
    SG_DENOISE_CASE(16)
    SG_DENOISE_CASE(19)
    SG_DENOISE_CASE(32)
#undef SG_DENOISE_CASE
    default:
      break;
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

}  // extern "C"
