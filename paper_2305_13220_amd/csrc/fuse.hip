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
// G channels at a time (all of a voxel's channels when they fit, so that a
// voxel's contiguous record is read once, with consecutive lanes on
// consecutive floats); each pass runs in place, one lane per line of the
// tile and channel: along x over side^2 lines, along y over 8 side (the x
// range left by the first pass), and along z over the block's 8 x 8 columns,
// which write the output (or, with several channel groups where LDS allows,
// hold it until whole records are written after the last group, as
// denoise_held below describes).  The mask goes through the same passes once, and
// each voxel's weight sum is kept for the renormalisation.  Results equal
// k_denoise's up to rounding order.
constexpr int kTileR = 2;

__host__ __device__ constexpr int denoise_side(int radius) { return 8 + 2 * radius; }

// Channels per tile pass: as many as fit a 79 KiB LDS budget (two
// 1024-lane workgroups per CU, so that one loads while the other filters),
// balanced over the passes, and a multiple of four when the voxel record is
// (16-byte loads).
constexpr int kDenoiseT = 1024;
__host__ __device__ constexpr int denoise_group(int V, int radius) {
  const int n3 = denoise_side(radius) * denoise_side(radius) * denoise_side(radius);
  const int gmax = (73 * 1024) / (4 * n3);
  const int g4 = (V % 4 == 0 && gmax >= 4) ? gmax / 4 * 4 : gmax;
  const int passes = (V + g4 - 1) / g4;
  const int gb = (V + passes - 1) / passes;
  return (V % 4 == 0 && gmax >= 4) ? (gb + 3) / 4 * 4 : gb;
}

// Channels a voxel record keeps in LDS until its last group is filtered:
// with several groups, the outputs of all but the last are held back and
// every record is written once, whole, after the last group (written group
// by group, the partly written lines of a block's output left the L2 between
// the groups and went to memory twice).  Only where it stays within the
// 80 KiB of two workgroups per CU; otherwise each group writes directly.
__host__ __device__ constexpr int denoise_held(int V, int radius) {
  const int G = denoise_group(V, radius), n3 = denoise_side(radius) * denoise_side(radius) *
                                                denoise_side(radius);
  const int ng = (V + G - 1) / G, last = V - (ng - 1) * G;
  const int held = ng > 1 ? V - last : 0;
  const int bytes = 4 * (n3 * G + n3 + SG_BLOCK_VOXELS + SG_BLOCK_VOXELS * held);
  return held > 0 && bytes <= 80 * 1024 && SG_BLOCK_VOXELS * V <= n3 * G &&
                 64 * last <= 1024
             ? held
             : 0;
}

template <int C, int R>
static size_t denoise_lds_bytes() {
  constexpr int side = denoise_side(R), n3 = side * side * side;
  return sizeof(float) * ((size_t)n3 * denoise_group(1 + C, R) + n3 + SG_BLOCK_VOXELS +
                          (size_t)SG_BLOCK_VOXELS * denoise_held(1 + C, R));
}

// One 1-D pass of width 2R + 1 in place over a line of side values at
// stride st: out[o] = sum_i w[i] in[o + i], o < 8.
template <int R>
__device__ __forceinline__ void denoise_line(float* p, int st, const float* w) {
  constexpr int side = denoise_side(R);
  float v[side];
#pragma unroll
  for (int x = 0; x < side; ++x) v[x] = p[x * st];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    float a = 0.0f;
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) a += w[i] * v[o + i];
    p[o * st] = a;
  }
}

template <int C, int R>
__global__ __launch_bounds__(kDenoiseT) void k_denoise_sep(GridView g,
                                                           const int32_t* __restrict__ coords,
                                                           const float* __restrict__ vox,
                                                           float inv_2s2, float* __restrict__ out,
                                                           bool vec) {
  constexpr int V = 1 + C;
  constexpr int side = denoise_side(R), n2 = side * side, n3 = n2 * side;
  constexpr int G = denoise_group(V, R);
  extern __shared__ float4 lds_q4[];  // 16-byte aligned: the tile takes 16-byte accesses
  float* lds = reinterpret_cast<float*>(lds_q4);
  float* tile = lds;               // [n3][G]: voxel (x, y, z) at x + side (y + side z)
  float* mk = lds + n3 * G;        // [n3] the mask, then its passes
  float* inv = mk + n3;            // [512] 1 / weight sum of each voxel of the block
  constexpr int HELD = denoise_held(V, R);
  float* held = inv + SG_BLOCK_VOXELS;  // [512][HELD] outputs of the earlier groups
  __shared__ int32_t nb[27];
  __shared__ float w1[2 * R + 1];
  // Workgroups are dealt to the 8 XCDs round-robin and each XCD has its own
  // L2: XCD x takes the x-th eighth of the blocks, in their index order
  // (allocation order, which follows the frames and so keeps neighbours
  // close), so the halo a block reads was mostly just read by its neighbours
  // on the same L2.  Every block costs the same, so the eighths balance.
  const int64_t nb_all = gridDim.x, xcd = blockIdx.x % 8, per = nb_all / 8, rem = nb_all % 8;
  const int64_t b = xcd * per + (xcd < rem ? xcd : rem) + blockIdx.x / 8;
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
  if (t <= 2 * R) {
    const int d = t - R;
    w1[t] = expf(-(float)(d * d) * inv_2s2);
  }
  __syncthreads();
  // element offset of tile voxel e (at voxel offset -R), or -1 where its block is absent
  auto tile_voxel = [&](int e) -> int64_t {
    const int x = e % side - R, y = (e / side) % side - R, z = e / n2 - R;
    const int32_t n = nb[((x >> 3) + 1) + 3 * ((y >> 3) + 1) + 9 * ((z >> 3) + 1)];
    return n < 0 ? -1 : (int64_t)n * SG_BLOCK_VOXELS + (x & 7) + 8 * (y & 7) + 64 * (z & 7);
  };
  for (int e = t; e < n3; e += kDenoiseT) mk[e] = tile_voxel(e) >= 0 ? 1.0f : 0.0f;
  __syncthreads();
  for (int l = t; l < n2; l += kDenoiseT) denoise_line<R>(mk + l * side, 1, w1);
  __syncthreads();
  for (int l = t; l < 8 * side; l += kDenoiseT) denoise_line<R>(mk + (l & 7) + n2 * (l >> 3), side, w1);
  __syncthreads();
  if (t < SG_BLOCK_VOXELS) {
    const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    float a = 0.0f;
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) a += w1[i] * mk[lx + side * (ly + side * (lz + i))];
    inv[t] = 1.0f / a;  // > 0: the voxel itself is allocated
  }
  for (int c0 = 0; c0 < V; c0 += G) {
    const int gc = min(G, V - c0);
    __syncthreads();  // the previous group's reads of the tile are done
    if (V % 4 == 0 && G % 4 == 0 && vec) {
      // 16-byte pieces of the voxel records (c0 and gc are multiples of 4)
      const int gq = gc / 4;
      for (int f = t; f < n3 * gq; f += kDenoiseT) {
        const int e = f / gq, q = f - e * gq;
        const int64_t off = tile_voxel(e);
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (off >= 0) v = *reinterpret_cast<const float4*>(vox + off * V + c0 + 4 * q);
        *reinterpret_cast<float4*>(tile + e * G + 4 * q) = v;
      }
    } else {
      for (int f = t; f < n3 * gc; f += kDenoiseT) {
        const int e = f / gc, j = f - e * gc;
        const int64_t off = tile_voxel(e);
        tile[e * G + j] = off >= 0 ? vox[off * V + c0 + j] : 0.0f;
      }
    }
    __syncthreads();
    for (int f = t; f < n2 * gc; f += kDenoiseT) {
      const int l = f / gc, j = f - l * gc;
      denoise_line<R>(tile + l * side * G + j, G, w1);
    }
    __syncthreads();
    for (int f = t; f < 8 * side * gc; f += kDenoiseT) {
      const int l = f / gc, j = f - l * gc;
      denoise_line<R>(tile + ((l & 7) + n2 * (l >> 3)) * G + j, side * G, w1);
    }
    __syncthreads();
    if (HELD > 0 && c0 + gc == V) {
      // last group: each lane's column (at most one per lane) into registers,
      // then the whole records assembled over the tile and stored once
      const bool has = t < 64 * gc;
      const int l = has ? t / gc : 0, j = has ? t - (t / gc) * gc : 0;
      const int lx = l & 7, ly = l >> 3;
      float v[side];
#pragma unroll
      for (int z = 0; z < side; ++z) v[z] = has ? tile[(lx + side * (ly + side * z)) * G + j] : 0.0f;
      __syncthreads();  // every column read: the tile becomes the records
      float* rec = tile;  // [512][V]
      if (has) {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          float a = 0.0f;
#pragma unroll
          for (int i = 0; i <= 2 * R; ++i) a += w1[i] * v[o + i];
          const int vi = lx + 8 * ly + 64 * o;
          rec[vi * V + c0 + j] = a * inv[vi];
        }
      }
      for (int f = t; f < SG_BLOCK_VOXELS * HELD; f += kDenoiseT) {
        const int vi = f / HELD;
        rec[vi * V + (f - vi * HELD)] = held[f];
      }
      __syncthreads();
      float* ob = out + b * SG_BLOCK_VOXELS * V;
      if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {
        for (int f = t; f < SG_BLOCK_VOXELS * V / 4; f += kDenoiseT)
          reinterpret_cast<float4*>(ob)[f] = reinterpret_cast<const float4*>(rec)[f];
      } else {
        for (int f = t; f < SG_BLOCK_VOXELS * V; f += kDenoiseT) ob[f] = rec[f];
      }
      continue;
    }
    for (int f = t; f < 64 * gc; f += kDenoiseT) {
      const int l = f / gc, j = f - l * gc;
      const int lx = l & 7, ly = l >> 3;
      float v[side];
#pragma unroll
      for (int z = 0; z < side; ++z) v[z] = tile[(lx + side * (ly + side * z)) * G + j];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) a += w1[i] * v[o + i];
        const int vi = lx + 8 * ly + 64 * o;
        if (HELD > 0)
          held[vi * HELD + c0 + j] = a * inv[vi];
        else
          out[(b * SG_BLOCK_VOXELS + vi) * V + c0 + j] = a * inv[vi];
      }
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
  const bool vec = reinterpret_cast<uintptr_t>(d_vox) % 16 == 0;
  int dev = 0, lds_max = 0;
  SG_HIP_CHECK(hipGetDevice(&dev));
  SG_HIP_CHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  hipStream_t s = (hipStream_t)stream;
  switch (C) {
#define SG_DENOISE_CASE(CC)                                                                 \
  case CC:                                                                                  \
    if (radius == 0)                                                                        \
      hipLaunchKernelGGL((k_denoise_sep<CC, 0>), dim3((unsigned)grid->n_blocks), dim3(kDenoiseT), \
                         (denoise_lds_bytes<CC, 0>()), s, g, grid->d_coords, d_vox, inv_2s2,  \
                         d_out, vec);                                                       \
    else if (radius == 1 && (denoise_lds_bytes<CC, 1>()) <= (size_t)lds_max)         \
      hipLaunchKernelGGL((k_denoise_sep<CC, 1>), dim3((unsigned)grid->n_blocks), dim3(kDenoiseT), \
                         (denoise_lds_bytes<CC, 1>()), s, g, grid->d_coords, d_vox, inv_2s2,  \
                         d_out, vec);                                                       \
    else if (radius == 2 && (denoise_lds_bytes<CC, 2>()) <= (size_t)lds_max)         \
      hipLaunchKernelGGL((k_denoise_sep<CC, 2>), dim3((unsigned)grid->n_blocks), dim3(kDenoiseT), \
                         (denoise_lds_bytes<CC, 2>()), s, g, grid->d_coords, d_vox, inv_2s2,  \
                         d_out, vec);                                                       \
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
