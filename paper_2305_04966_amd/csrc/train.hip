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

constexpr int kChunk = 512;  // targets staged per pass

// LDS of one wave: edges [nb+1], proposal weights [nb], and for a chunk of
// targets their gradient coefficient and overlapping bin range.
__host__ __device__ inline size_t loss_lds_bytes(int nb) {
  return ((size_t)(2 * nb + 1) * 4 + 15) / 16 * 16 + (size_t)kChunk * (4 + 2 + 2);
}

// One wave per ray.  Each target's bin range (two binary searches over the
// edges in LDS), gap w - bound and loss term are computed once, by the lane
// that owns the target; its gradient coefficient c_i = -2 gap/(w + eps)/n (0
// when gap <= 0) and bin range go to LDS in target order.  Targets are sorted
// and disjoint, so bin ranges are non-decreasing in the target index and the
// targets overlapping a bin form a contiguous run: the lane of bin j finds its
// run by a binary search over the staged ranges and sums it in target order.
// Rays with more than kChunk targets are staged in chunks, each bin carrying
// its partial sum across them (same order).  kBinsPerLane = ceil(nb / 64)
// rounded up to 1, 4 or 16: the bins' partial sums a lane carries.
template <int kBinsPerLane, int kRegEdges>
__global__ __launch_bounds__(kWave* kLossWaves) void hist_loss_kernel(
    const int32_t* __restrict__ info, const float* __restrict__ t0, const float* __restrict__ t1,
    const float* __restrict__ w, int32_t n_rays, int64_t n_targets, int32_t nb,
    const float* __restrict__ edges, const float* __restrict__ prop, float eps, float inv_n,
    float* __restrict__ loss, float* __restrict__ d_prop) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const int wv = threadIdx.x / kWave, ln = lane();
  const int64_t r = (int64_t)blockIdx.x * kLossWaves + wv;
  if (r >= n_rays) return;
  unsigned char* base = lds_raw + (size_t)wv * loss_lds_bytes(nb);
  float* e = reinterpret_cast<float*>(base);
  float* pw = e + nb + 1;
  float* cc = reinterpret_cast<float*>(base + ((size_t)(2 * nb + 1) * 4 + 15) / 16 * 16);
  int16_t* jl = reinterpret_cast<int16_t*>(cc + kChunk);
  int16_t* jh = jl + kChunk;
  // The ray's packed row, its edges and proposal weights load together, and
  // the first targets as soon as the row is in: two memory latencies before
  // the first target is processed instead of three in a row.
  int64_t st = info[2 * r], ct = info[2 * r + 1];
  float ev[kBinsPerLane + 1], pv[kBinsPerLane];
#pragma unroll
  for (int q = 0; q <= kBinsPerLane; ++q) {
    const int j = ln + q * kWave;
    ev[q] = j <= nb ? edges[r * (nb + 1) + j] : 0.0f;
    if (q < kBinsPerLane) pv[q] = j < nb ? prop[r * nb + j] : 0.0f;
  }
  if (st < 0 || ct < 0 || st + ct > n_targets) ct = 0;  // malformed row: no targets
  // each lane's next target loads while its current one is processed; the
  // first targets of a chunk load before the previous chunk's bin sums
  float na = 0.0f, nb_ = 0.0f, nw = 0.0f;
  auto first_targets = [&](int64_t c0) {
    if (ln < min<int64_t>(kChunk, ct - c0)) {
      const int64_t i = st + c0 + ln;
      na = t0[i];
      nb_ = t1[i];
      nw = w[i];
    }
  };
  first_targets(0);
#pragma unroll
  for (int q = 0; q <= kBinsPerLane; ++q) {
    const int j = ln + q * kWave;
    if (j <= nb) e[j] = ev[q];
    if (q < kBinsPerLane && j < nb) pw[j] = pv[q];
  }
  wave_sync();
  // rows of at most kRegEdges bins: every lane holds the row's edges
  float er[kRegEdges + 1];
  float e_last = 0.0f;
  if (kRegEdges > 0) {
#pragma unroll
    for (int m = 0; m <= kRegEdges; ++m) er[m] = m <= nb ? e[m] : INFINITY;
    e_last = e[nb];
  }
  float gacc[kBinsPerLane];
#pragma unroll
  for (int q = 0; q < kBinsPerLane; ++q) gacc[q] = 0.0f;
  float acc = 0.0f;
  for (int64_t c0 = 0; c0 < ct || c0 == 0; c0 += kChunk) {
    const int n = (int)min<int64_t>(kChunk, ct - c0);
    for (int k = ln; k < n; k += kWave) {
      const float a = na, b = nb_, wi = nw;
      if (k + kWave < n) {
        const int64_t i = st + c0 + k + kWave;
        na = t0[i];
        nb_ = t1[i];
        nw = w[i];
      }
      int jlo, jhi;
      if (kRegEdges > 0) {
        // the same bounds as counts over the edges held in registers (sorted
        // edges; +inf past e[nb]): jlo = #{m in [1, nb]: !(e[m] > a)}, jhi =
        // #{m in [0, nb - 1]: e[m] < b} - 1
        int cl = 0, ch = 0;
#pragma unroll
        for (int m = 0; m <= kRegEdges; ++m) {
          if (m > 0) cl += !(er[m] > a);
          ch += er[m] < b;
        }
        jlo = min(cl, nb);
        jhi = ch - (e_last < b) - 1;
      } else {
        bin_range(e, nb, a, b, jlo, jhi);
      }
      float bound = 0.0f;
      for (int j = jlo; j <= jhi; ++j) bound += pw[j];
      const float gap = wi - bound;
      float c = 0.0f;
      if (gap > 0.0f) {
        acc += gap * gap / (wi + eps);
        c = -2.0f * gap / (wi + eps) * inv_n;
      }
      cc[k] = c;
      jl[k] = (int16_t)jlo;
      jh[k] = (int16_t)jhi;
    }
    wave_sync();
    if (c0 + kChunk < ct) first_targets(c0 + kChunk);
    if (d_prop) {
#pragma unroll
      for (int q = 0; q < kBinsPerLane; ++q) {
        const int j = ln + q * kWave;
        if (j >= nb) break;
        int lo = 0, hi = n;  // first staged target with jhi >= j
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (jh[mid] >= j) hi = mid;
          else lo = mid + 1;
        }
        int end = lo;  // first staged target at or after lo with jlo > j
        hi = n;
        while (end < hi) {
          const int mid = (end + hi) >> 1;
          if (jl[mid] > j) hi = mid;
          else end = mid + 1;
        }
        // the run [lo, end) in target order; its length is known, so the
        // LDS reads of the run are issued ahead of the (sequential) sum
        float g = gacc[q];
#pragma unroll 8
        for (int k = lo; k < end; ++k) g += cc[k];
        gacc[q] = g;
      }
    }
    wave_sync();
    if (ct == 0) break;
  }
#pragma unroll
  for (int s = kWave / 2; s >= 1; s >>= 1) acc += __shfl_xor(acc, s, kWave);
  if (ln == 0) loss[r] = acc;
  if (d_prop) {
#pragma unroll
    for (int q = 0; q < kBinsPerLane; ++q) {
      const int j = ln + q * kWave;
      if (j < nb) d_prop[r * nb + j] = gacc[q];
    }
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
  if (n_targets >= ((int64_t)1 << 31)) {
    set_error("txs_hist_loss: %lld targets do not fit the int32 packed layout",
              (long long)n_targets);
    return TXS_EOVERFLOW;
  }
  TXS_REQUIRE(n_bins >= 1 && n_bins <= kMaxBins, "txs_hist_loss: n_bins must be in [1,%d]",
              kMaxBins);
  TXS_REQUIRE(eps >= 0.0f, "txs_hist_loss: eps must be >= 0");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(packed_info && edges && prop_w && loss, "txs_hist_loss: null array");
  TXS_REQUIRE(n_targets == 0 || (t0 && t1 && w), "txs_hist_loss: null target array");
  const int64_t blocks = ((int64_t)n_rays + kLossWaves - 1) / kLossWaves;
  const size_t lds = kLossWaves * loss_lds_bytes(n_bins);
  const auto kern = n_bins <= 16          ? hist_loss_kernel<1, 16>
                    : n_bins <= kWave       ? hist_loss_kernel<1, 0>
                    : n_bins <= 4 * kWave ? hist_loss_kernel<4, 0>
                                          : hist_loss_kernel<kMaxBins / kWave, 0>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kWave * kLossWaves), lds,
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
