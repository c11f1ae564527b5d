// The rest of the training step around the renderer: camera rays (inverse
// pinhole projection, the camera model of Eq. 3), the squared-L2 rendering
// losses of Eq. 12-14 and their gradient, and an in-place optimiser step on
// the voxel parameters (Sec. 3.5.4).
#include <cmath>

#include "common.h"

namespace sg {

__global__ void k_rays_pinhole(const float* __restrict__ cams, int32_t n_cams,
                               const int32_t* __restrict__ pix, int64_t R, float* __restrict__ rays) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int32_t c = pix[3 * r];
  float* out = rays + 6 * r;
  if (c < 0 || c >= n_cams) {
    for (int a = 0; a < 6; ++a) out[a] = __int_as_float(0x7fc00000);
    return;
  }
  float ray[6];
  pinhole_ray(cams + 16 * (int64_t)c, pix[3 * r + 1], pix[3 * r + 2], ray);
#pragma unroll
  for (int a = 0; a < 6; ++a) out[a] = ray[a];
}

__global__ void k_l2_grad(const float* __restrict__ feat, const float* __restrict__ feat_ref,
                          const float* __restrict__ depth, const float* __restrict__ depth_ref,
                          const float* __restrict__ normal, const float* __restrict__ normal_ref,
                          int64_t R, int32_t C, float lambda_d, float lambda_n,
                          float* __restrict__ g_feat, float* __restrict__ g_depth,
                          float* __restrict__ g_normal) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const float s = 2.0f / (float)R;
  for (int ch = 0; ch < C; ++ch)
    g_feat[(int64_t)C * r + ch] = s * (feat[(int64_t)C * r + ch] - feat_ref[(int64_t)C * r + ch]);
  g_depth[r] = s * lambda_d * (depth[r] - depth_ref[r]);
  for (int a = 0; a < 3; ++a) g_normal[3 * r + a] = s * lambda_n * (normal[3 * r + a] - normal_ref[3 * r + a]);
}

// Loss value: one workgroup, fixed summation order (deterministic).
__global__ void k_l2_loss(const float* __restrict__ feat, const float* __restrict__ feat_ref,
                          const float* __restrict__ depth, const float* __restrict__ depth_ref,
                          const float* __restrict__ normal, const float* __restrict__ normal_ref,
                          int64_t R, int32_t C, float lambda_d, float lambda_n,
                          float* __restrict__ loss) {
  __shared__ float part[1024 / kWave];
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < R; r += blockDim.x) {
    float a = 0.0f;
    for (int ch = 0; ch < C; ++ch) {
      const float d = feat[(int64_t)C * r + ch] - feat_ref[(int64_t)C * r + ch];
      a += d * d;
    }
    const float dd = depth[r] - depth_ref[r];
    float an = 0.0f;
    for (int k = 0; k < 3; ++k) {
      const float d = normal[3 * r + k] - normal_ref[3 * r + k];
      an += d * d;
    }
    acc += (double)(a + lambda_d * dd * dd + lambda_n * an);
  }
  float v = (float)acc;
  v = wave_sum(v);
  if (lane_id() == 0) part[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += part[w];
    *loss = t / (float)R;
  }
}

__global__ void k_optim(int32_t kind, float* __restrict__ p, const float* __restrict__ g,
                        float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1,
                        float b2, float eps, float bc1, float bc2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float gi = g[i];
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    v[i] = vi;
    if (kind == 0) {
      const float mi = b1 * m[i] + (1.0f - b1) * gi;
      m[i] = mi;
      p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    } else {
      p[i] -= lr * gi / (sqrtf(vi) + eps);
    }
  }
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_rays_pinhole(const float* d_cams, int32_t n_cams, const int32_t* d_pix, int64_t n_rays,
                    float* d_rays, sg_stream stream) {
  if (n_rays < 0 || n_cams < 0) return fail(SG_EINVAL, "n_rays / n_cams must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_cams || !d_pix || !d_rays) return fail(SG_EINVAL, "a required pointer is NULL");
  hipLaunchKernelGGL(k_rays_pinhole, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, d_cams, n_cams, d_pix, n_rays, d_rays);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_l2_loss_grad(const float* d_feat, const float* d_feat_ref, const float* d_depth,
                    const float* d_depth_ref, const float* d_normal, const float* d_normal_ref,
                    int64_t n_rays, int32_t C, float lambda_d, float lambda_n, float* d_g_feat,
                    float* d_g_depth, float* d_g_normal, float* d_loss, sg_stream stream) {
  if (n_rays < 1) return fail(SG_EINVAL, "n_rays must be >= 1");
  if (C < 0) return fail(SG_EINVAL, "C must be >= 0");
  if (!std::isfinite(lambda_d) || !std::isfinite(lambda_n))
    return fail(SG_EINVAL, "lambda_d / lambda_n must be finite");
  if (!d_depth || !d_depth_ref || !d_normal || !d_normal_ref || !d_g_depth || !d_g_normal ||
      (C > 0 && (!d_feat || !d_feat_ref || !d_g_feat)))
    return fail(SG_EINVAL, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_l2_grad, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, s, d_feat,
                     d_feat_ref, d_depth, d_depth_ref, d_normal, d_normal_ref, n_rays, C, lambda_d,
                     lambda_n, d_g_feat, d_g_depth, d_g_normal);
  if (d_loss)
    hipLaunchKernelGGL(k_l2_loss, dim3(1), dim3(1024), 0, s, d_feat, d_feat_ref, d_depth,
                       d_depth_ref, d_normal, d_normal_ref, n_rays, C, lambda_d, lambda_n, d_loss);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_optim_step(int32_t kind, float* d_param, const float* d_grad, float* d_m, float* d_v,
                  int64_t n, float lr, float b1, float b2, float eps, int32_t t, sg_stream stream) {
  if (kind != 0 && kind != 1) return fail(SG_EINVAL, "kind must be 0 (Adam) or 1 (RMSProp)");
  if (n < 0) return fail(SG_EINVAL, "n must be >= 0");
  if (n == 0) return SG_OK;
  if (!d_param || !d_grad || !d_v || (kind == 0 && !d_m))
    return fail(SG_EINVAL, "a required pointer is NULL");
  if (t < 1) return fail(SG_EINVAL, "t must be >= 1");
  if (!(lr >= 0.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps >= 0.0f) ||
      (kind == 0 && !(b1 >= 0.0f && b1 < 1.0f)))
    return fail(SG_EINVAL, "optimiser hyper-parameters out of range");
  const float bc1 = kind == 0 ? (float)(1.0 - std::pow((double)b1, (double)t)) : 1.0f;
  const float bc2 = kind == 0 ? (float)(1.0 - std::pow((double)b2, (double)t)) : 1.0f;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_optim, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, kind,
                     d_param, d_grad, d_m, d_v, n, lr, b1, b2, eps, bc1, bc2);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

}  // extern "C"
