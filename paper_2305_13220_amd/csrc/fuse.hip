// Depth, colour and semantic fusion into the voxels of a grid (Sec. 3.4.2):
// each voxel is projected into every frame and the associated observations
// are averaged (the closed-form minimisers of the per-voxel squared losses).
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
    if (!(fabsf(s) < trunc)) continue;
    sd += s;
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

}  // extern "C"
