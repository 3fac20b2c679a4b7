// Support kernel, not part of the sampling method: an analytic radiance field
// (Gaussian density blobs, optional background shell, colour maps) that plays
// the user's NeRF of Algorithm 1 so the whole pipeline runs on the GPU.
#include "txs_common.h"

namespace txs {
namespace {

constexpr int kFieldBlock = 256;

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

__global__ __launch_bounds__(kFieldBlock) void blob_field_kernel(
    const float* __restrict__ p, int32_t nb, const float* __restrict__ ro, const float* __restrict__ rd,
    const float* __restrict__ t0, const float* __restrict__ t1, const int32_t* __restrict__ rid,
    int32_t fixed, int32_t n_rays, int64_t n, float* __restrict__ sigma,
    float* __restrict__ rgb) {
  const int64_t i = (int64_t)blockIdx.x * kFieldBlock + threadIdx.x;
  if (i >= n) return;
  int64_t r = rid ? (int64_t)rid[i] : i / fixed;
  if (r < 0 || r >= n_rays) r = 0;  // out-of-range ray index: defined, not faulting
  const float tm = 0.5f * (t0[i] + t1[i]);
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = ro[3 * r + a] + tm * rd[3 * r + a];
  const float peak = p[1], wd = p[2];
  // exp(-r2/(2w^2)) = exp2(-r2 k2), k2 = log2(e)/(2w^2); with s = sqrt(k2) the
  // exponent is -|x s - c s|^2, each difference one fused x s - c s
  const float k2 = 1.4426950408889634f / (2.0f * wd * wd);
  const float sk = sqrtf(k2);
  const float xs[3] = {x[0] * sk, x[1] * sk, x[2] * sk};
  const float* cen = p + 32;
  // Blobs in order, four centres per group of (wave-uniform) loads.  The
  // hardware exp2 has no subnormal results, so each factor is taken as
  // 2^(y + 32) and the sum scaled by 2^-32 at the end: factors down to 2^-158
  // stay normal until that final (exact or once-rounded) scaling, as with a
  // subnormal-preserving exp2.
  float sb = 0.0f;
  int b = 0;
  for (; b + 4 <= nb; b += 4) {
    float c[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = cen[3 * b + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float dx = fmaf(-c[3 * k], sk, xs[0]), dy = fmaf(-c[3 * k + 1], sk, xs[1]),
                  dz = fmaf(-c[3 * k + 2], sk, xs[2]);
      sb += __builtin_amdgcn_exp2f(fmaf(-dz, dz, fmaf(-dy, dy, fmaf(-dx, dx, 32.0f))));
    }
  }
  for (; b < nb; ++b) {
    const float dx = fmaf(-cen[3 * b], sk, xs[0]), dy = fmaf(-cen[3 * b + 1], sk, xs[1]),
                dz = fmaf(-cen[3 * b + 2], sk, xs[2]);
    sb += __builtin_amdgcn_exp2f(fmaf(-dz, dz, fmaf(-dy, dy, fmaf(-dx, dx, 32.0f))));
  }
  sb = (sb * peak) * 0x1p-32f;
  float ss = 0.0f;
  const float nrm = sqrtf(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  if (p[3] != 0.0f) {
    const float g = nrm - p[4];
    ss = p[6] * __expf(-g * g / (2.0f * p[5] * p[5]));
  }
  const float tot = sb + ss;
  sigma[i] = tot;
  if (rgb) {
    const float* A = p + 7;
    const float* bb = p + 16;
    const float* A2 = p + 19;
    const float* b2 = p + 28;
    const float inv_n = nrm > 0.0f ? 1.0f / nrm : 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float z = bb[c] + A[3 * c] * x[0] + A[3 * c + 1] * x[1] + A[3 * c + 2] * x[2];
      const float cb = sigmoidf(z);
      float out = cb;
      if (tot > 0.0f && ss > 0.0f) {
        const float z2 = b2[c] + (A2[3 * c] * x[0] + A2[3 * c + 1] * x[1] + A2[3 * c + 2] * x[2]) *
                                     inv_n;
        out = (sb * cb + ss * sigmoidf(z2)) / tot;
      }
      rgb[3 * i + c] = out;
    }
  }
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_blob_field(const float* params, int32_t n_blobs, const float* rays_o,
                                     const float* rays_d, int32_t n_rays, const float* t0,
                                     const float* t1, const int32_t* ray_id, int32_t fixed_count,
                                     int64_t n, float* sigma, float* rgb, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n >= 0 && n_blobs >= 0 && n_rays >= 0, "txs_blob_field: bad size");
  if (n == 0) return TXS_OK;
  TXS_REQUIRE(n_rays > 0, "txs_blob_field: samples but no rays");
  TXS_REQUIRE(params && rays_o && rays_d && t0 && t1 && sigma, "txs_blob_field: null array");
  TXS_REQUIRE(ray_id || fixed_count > 0, "txs_blob_field: need ray_id or fixed_count > 0");
  hipLaunchKernelGGL(blob_field_kernel, dim3(grid_1d(n, kFieldBlock)), dim3(kFieldBlock), 0,
                     as_stream(stream), params, n_blobs, rays_o, rays_d, t0, t1, ray_id,
                     fixed_count, n_rays, n, sigma, rgb);
  return launch_status("txs_blob_field");
}
