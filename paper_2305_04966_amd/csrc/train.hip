// Estimator update by gradient descent (Eq. 4 with an SGD update; Section 3.1
// "PDF Approaches"): the PDF-matching loss between the radiance field's
// rendering weights and the proposal's, and the Adam step on the proposal
// network's parameters.
#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kMaxBins = 1024;
constexpr int kLossWaves = 4;

// Bins of the proposal overlapping the open interval (a, b):
// j in [first j with e[j+1] > a, last j with e[j] < b].
__device__ __forceinline__ void bin_range(const float* e, int nb, float a, float b, int& jlo,
                                          int& jhi) {
  int lo = 0, hi = nb;  // first j in [0, nb) with e[j+1] > a (nb if none)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (e[mid + 1] > a) hi = mid;
    else lo = mid + 1;
  }
  jlo = lo;
  lo = -1;
  hi = nb - 1;  // last j in [0, nb) with e[j] < b (-1 if none)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (e[mid] < b) lo = mid;
    else hi = mid - 1;
  }
  jhi = lo;
}

// gap = w - (proposal mass over the bins overlapping the target interval)
__device__ __forceinline__ float target_gap(const float* e, const float* pw, int nb, float a,
                                            float b, float w) {
  int jlo, jhi;
  bin_range(e, nb, a, b, jlo, jhi);
  float bound = 0.0f;
  for (int j = jlo; j <= jhi; ++j) bound += pw[j];
  return w - bound;
}

// One wave per ray: the ray's proposal edges and weights in LDS; the loss
// sums over the ray's target intervals; the gradient of each bin sums, in
// target order, over the contiguous run of targets that overlap it.
__global__ __launch_bounds__(kWave* kLossWaves) void hist_loss_kernel(
    const int32_t* __restrict__ info, const float* __restrict__ t0, const float* __restrict__ t1,
    const float* __restrict__ w, int32_t n_rays, int64_t n_targets, int32_t nb,
    const float* __restrict__ edges, const float* __restrict__ prop, float eps, float inv_n,
    float* __restrict__ loss, float* __restrict__ d_prop) {
  __shared__ float sE[kLossWaves][kMaxBins + 1];
  __shared__ float sP[kLossWaves][kMaxBins];
  const int wv = threadIdx.x / kWave, ln = lane();
  const int64_t r = (int64_t)blockIdx.x * kLossWaves + wv;
  if (r >= n_rays) return;
  float* e = sE[wv];
  float* pw = sP[wv];
  for (int j = ln; j <= nb; j += kWave) e[j] = edges[r * (nb + 1) + j];
  for (int j = ln; j < nb; j += kWave) pw[j] = prop[r * nb + j];
  wave_sync();
  int64_t st = info[2 * r], ct = info[2 * r + 1];
  if (st < 0 || ct < 0 || st + ct > n_targets) ct = 0;  // malformed row: no targets
  float acc = 0.0f;
  for (int64_t i = st + ln; i < st + ct; i += kWave) {
    const float g = target_gap(e, pw, nb, t0[i], t1[i], w[i]);
    if (g > 0.0f) acc += g * g / (w[i] + eps);
  }
#pragma unroll
  for (int s = kWave / 2; s >= 1; s >>= 1) acc += __shfl_xor(acc, s, kWave);
  if (ln == 0) loss[r] = acc;
  if (!d_prop) return;
  for (int j = ln; j < nb; j += kWave) {
    const float lo = e[j], hi = e[j + 1];
    // targets overlapping (lo, hi): t1_i > lo and t0_i < hi (sorted, disjoint)
    int64_t a = st, b = st + ct;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (t1[mid] > lo) b = mid;
      else a = mid + 1;
    }
    float g = 0.0f;
    for (int64_t i = a; i < st + ct && t0[i] < hi; ++i) {
      const float gap = target_gap(e, pw, nb, t0[i], t1[i], w[i]);
      if (gap > 0.0f) g += -2.0f * gap / (w[i] + eps) * inv_n;
    }
    d_prop[r * nb + j] = g;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v,
                                                   const float* __restrict__ g, int64_t n,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_hist_loss(const int32_t* packed_info, int32_t n_rays, int64_t n_targets,
                                    const float* t0, const float* t1, const float* w,
                                    int32_t n_bins, const float* edges, const float* prop_w,
                                    float eps, float* loss, float* d_prop, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && n_targets >= 0, "txs_hist_loss: negative size");
  TXS_REQUIRE(n_bins >= 1 && n_bins <= kMaxBins, "txs_hist_loss: n_bins must be in [1,%d]",
              kMaxBins);
  TXS_REQUIRE(eps >= 0.0f, "txs_hist_loss: eps must be >= 0");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(packed_info && edges && prop_w && loss, "txs_hist_loss: null array");
  TXS_REQUIRE(n_targets == 0 || (t0 && t1 && w), "txs_hist_loss: null target array");
  const int64_t blocks = ((int64_t)n_rays + kLossWaves - 1) / kLossWaves;
  hipLaunchKernelGGL(hist_loss_kernel, dim3((unsigned)blocks), dim3(kWave * kLossWaves), 0,
                     as_stream(stream), packed_info, t0, t1, w, n_rays, n_targets, n_bins, edges,
                     prop_w, eps, 1.0f / (float)n_rays, loss, d_prop);
  return launch_status("txs_hist_loss");
}

extern "C" txs_status txs_adam_step(float* params, float* m, float* v, const float* grad,
                                    int64_t n, float lr, float beta1, float beta2, float eps,
                                    int32_t step, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n >= 0 && step >= 1, "txs_adam_step: bad size or step");
  TXS_REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f,
              "txs_adam_step: betas must be in [0,1)");
  if (n == 0) return TXS_OK;
  TXS_REQUIRE(params && m && v && grad, "txs_adam_step: null array");
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, as_stream(stream), params,
                     m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
  return launch_status("txs_adam_step");
}
