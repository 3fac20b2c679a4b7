// Shared engine of the packed volume-rendering kernels (Eq. 2 discretised;
// Section 4.2 packed tensors and no-gradient filtering).
//
// Work decomposition.  A wave owns 64 consecutive rays (one per lane) and
// walks the sample range of those rays in windows of W = 64*K samples held in
// registers, K contiguous samples per lane (blocked layout, 16-byte vector
// loads and stores).  Ray boundaries inside a window are marked in LDS; the
// per-ray scans are segmented scans: a serial pass inside each lane plus a
// wave-wide Hillis-Steele scan over the 64 lane aggregates, gated by the lane
// of the nearest segment boundary.  The forward direction walks the windows
// left to right with a carry; the adjoint walks them right to left, so its
// suffix sums are exact reverse scans.  Optical depths are accumulated in
// binary64: the transmittance exp(-P) needs P to ~1e-6 absolute.
#pragma once

#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int K = 8;               // samples per lane per window
constexpr int W = kWave * K;       // samples per window
constexpr int kWaves = 4;          // waves per block
constexpr int kBlock = kWave * kWaves;
constexpr int kMarks = W + kWave;  // marks for window positions 0..W (cleared 64 at a time)

enum Mode { kFwd = 0, kPrefix = 1, kTotal = 2, kBwd = 3, kWBwd = 4 };

struct Args {
  const int32_t* info;
  int32_t fixed;
  int32_t n_rays;
  int64_t n_samples;
  const float* t0;
  const float* t1;
  const float* sigma;
  const float* rgb;
  const float* bg;
  // forward outputs
  float* out_rgb;
  float* out_opacity;
  float* out_depth;
  float* out_w;
  double* out_optical;
  // filter
  double p_max;  // keep while sum_{j<i} tau_j <= p_max
  int32_t* kept;
  // adjoint
  const double* optical;  // per-ray total optical depth (NULL: recomputed)
  const float* g_rgb;
  const float* g_op;
  const float* g_depth;
  const float* g_w;
  float* d_sigma;
  float* d_rgb;
};

// Per-wave LDS: boundary marks of the current window, per-ray cotangents and
// total optical depths (adjoint).
struct WaveLds {
  int marks[kMarks];
  float cot[kWave][8];  // g_rgb(3), h, q, bg(3) of each owned ray
  double ptot[kWave];
};

// mark value: 0 none, lane+1 = first sample of that lane's ray, -1 = sample
// after the end of a ray (dead until the next head).
__device__ __forceinline__ int decode_mark(int m) { return m > 0 ? m - 1 : -1; }

__device__ __forceinline__ void ray_row(const Args& a, int32_t r, int64_t& st, int32_t& ct) {
  if (r >= a.n_rays) {
    st = 0;
    ct = 0;
  } else if (a.info) {
    const int2 v = reinterpret_cast<const int2*>(a.info)[r];
    st = v.x;
    ct = v.y;
    if (v.x < 0 || v.y < 0) {  // malformed row: treated as an empty ray
      st = 0;
      ct = 0;
    }
  } else {
    st = (int64_t)r * a.fixed;
    ct = a.fixed;
  }
}

// ----------------------------------------------------------- wave scans
__device__ __forceinline__ int max_scan_incl(int v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = shfl_up(v, d);
    if (lane() >= d) v = max(v, t);
  }
  return v;
}

__device__ __forceinline__ int min_scan_rev_incl(int v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = shfl_down(v, d);
    if (lane() + d < kWave) v = min(v, t);
  }
  return v;
}

// Inclusive segmented scan over lanes; hl = last lane <= this one that starts
// a segment (-1 if none).
template <typename T>
__device__ __forceinline__ T seg_scan(T v, int hl) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T t = shfl_up(v, d);
    if (lane() >= d && lane() - d >= hl) v += t;
  }
  return v;
}

// Reverse inclusive segmented scan; fl = first lane >= this one that ends the
// chain (64 if none).
template <typename T>
__device__ __forceinline__ T seg_scan_rev(T v, int fl) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T t = shfl_down(v, d);
    if (lane() + d < kWave && lane() + d <= fl) v += t;
  }
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  return __shfl(v, l, kWave);
}

struct Acc5 {
  float r, g, b, o, d;
};
__device__ __forceinline__ Acc5 seg_scan(Acc5 v, int hl) {
  return {seg_scan(v.r, hl), seg_scan(v.g, hl), seg_scan(v.b, hl), seg_scan(v.o, hl),
          seg_scan(v.d, hl)};
}
__device__ __forceinline__ Acc5 shfl_up1(Acc5 v) {
  return {shfl_up(v.r, 1), shfl_up(v.g, 1), shfl_up(v.b, 1), shfl_up(v.o, 1), shfl_up(v.d, 1)};
}

// ----------------------------------------------------------- loads / stores
__device__ __forceinline__ void load_k(const float* __restrict__ src, int64_t pos0, int64_t lim,
                                       float (&v)[K]) {
  if (pos0 + K <= lim) {
    const float4* p = reinterpret_cast<const float4*>(src + pos0);
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
      const float4 x = p[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = (pos0 + j < lim) ? src[pos0 + j] : 0.0f;
  }
}

__device__ __forceinline__ void load_rgb(const float* __restrict__ src, int64_t pos0, int64_t lim,
                                         float (&c)[K][3]) {
  if (pos0 + K <= lim) {
    const float4* p = reinterpret_cast<const float4*>(src + 3 * pos0);
    float f[3 * K];
#pragma unroll
    for (int q = 0; q < 3 * K / 4; ++q) {
      const float4 x = p[q];
      f[4 * q] = x.x;
      f[4 * q + 1] = x.y;
      f[4 * q + 2] = x.z;
      f[4 * q + 3] = x.w;
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) c[j][c3] = f[3 * j + c3];
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3)
        c[j][c3] = (pos0 + j < lim) ? src[3 * (pos0 + j) + c3] : 0.0f;
  }
}

// Stores v[j] where own[j]; a full vector store when every element is owned.
__device__ __forceinline__ void store_k(float* __restrict__ dst, int64_t pos0, const float (&v)[K],
                                        const bool (&own)[K]) {
  bool all = true;
#pragma unroll
  for (int j = 0; j < K; ++j) all = all && own[j];
  if (all) {
    float4* p = reinterpret_cast<float4*>(dst + pos0);
#pragma unroll
    for (int q = 0; q < K / 4; ++q)
      p[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (own[j]) dst[pos0 + j] = v[j];
  }
}

// ----------------------------------------------------------- window marks
// Marks, for window start p, the first sample (lane+1) and the end (-1) of
// every ray in the set that falls in window positions [0, W].
__device__ __forceinline__ void write_marks(WaveLds& L, int64_t p, int64_t st, int64_t en,
                                            bool in_set) {
  const int ln = lane();
#pragma unroll
  for (int j = 0; j < kMarks / kWave; ++j) L.marks[ln + kWave * j] = 0;
  wave_sync();
  const int64_t e_off = en - p, s_off = st - p;
  if (in_set && en > st && e_off >= 0 && e_off <= W) L.marks[e_off] = -1;
  wave_sync();
  if (in_set && en > st && s_off >= 0 && s_off <= W) L.marks[s_off] = ln + 1;
  wave_sync();
}

__device__ __forceinline__ void read_marks(const WaveLds& L, int (&mk)[K + 1]) {
  const int base = K * lane();
#pragma unroll
  for (int j = 0; j <= K; ++j) mk[j] = L.marks[base + j];
}

// Sample range [lo, hi) of the wave's rays (hi clipped to n_samples); the
// per-lane row (st, en) with en clipped likewise; active = non-empty row.
struct WaveRange {
  int64_t st, en, lo, hi;
  bool active;
};

__device__ __forceinline__ WaveRange wave_range(const Args& a, int32_t r) {
  WaveRange w;
  int32_t ct;
  ray_row(a, r, w.st, ct);
  w.en = min(w.st + (int64_t)ct, a.n_samples);
  w.active = r < a.n_rays && w.en > w.st;
  w.lo = wave_min(w.active ? w.st : INT64_MAX);
  w.hi = wave_max(w.active ? w.en : (int64_t)0);
  return w;
}

txs_status check_common(const char* who, const int32_t* info, int32_t fixed, int32_t n_rays,
                        int64_t n_samples, const float* t0, const float* t1,
                        const float* sigma) {
  TXS_REQUIRE(n_rays >= 0 && n_samples >= 0, "%s: negative size", who);
  TXS_REQUIRE(n_samples < ((int64_t)1 << 31), "%s: n_samples must be < 2^31", who);
  if (!info) {
    TXS_REQUIRE(fixed >= 0, "%s: fixed_count must be >= 0", who);
    TXS_REQUIRE((int64_t)fixed * n_rays <= n_samples,
                "%s: dense layout needs n_rays*fixed_count <= n_samples", who);
  }
  TXS_REQUIRE(n_samples == 0 || (t0 && t1 && sigma), "%s: null sample array", who);
  return TXS_OK;
}

template <typename Kern>
txs_status launch(Kern kern, const Args& a, void* stream, const char* who) {
  const int64_t waves = ((int64_t)a.n_rays + kWave - 1) / kWave;
  const int64_t blocks = (waves + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(kern, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0,
                     as_stream(stream), a);
  return launch_status(who);
}

}  // namespace
}  // namespace txs
