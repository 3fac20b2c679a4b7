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

// Samples per lane per window (a multiple of 4): 8 in the forward kernels, 4
// in the adjoint, whose per-sample state is larger (its translation unit
// defines TXS_RENDER_ADJOINT before including this header).
#ifdef TXS_RENDER_ADJOINT
constexpr int K = 4;
#else
constexpr int K = 8;
#endif
constexpr int W = kWave * K;       // samples per window
constexpr int kWaves = 8;          // waves per block
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

// Per-wave LDS: boundary marks of the current window (every kernel), and for
// the adjoint the per-ray cotangents and total optical depths.  The forward
// kernels hold the marks alone (33 KB per block with the colour staging).
struct MarkLds {
  int marks[kMarks];
};
struct WaveLds : MarkLds {
  float cot[kWave][8];  // g_rgb(3), h, q, bg(3) of each owned ray
  double ptot[kWave];
};

// Per-wave LDS staging of a window's [W][3] colour rows (colours on the way
// in, colour gradients on the way out), so that HBM sees whole-row float4
// accesses at consecutive lanes.  Only the modes that move colours have it.
template <int kMode>
struct StageSize {
  static constexpr int value = (kMode == kFwd || kMode == kBwd) ? 3 * W / 4 : 1;
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
// Lane scans run inside each 16-lane row with DPP row shifts (VALU latency),
// then the three row-end values are read into scalars and carried into the
// later rows.  They must be called with all 64 lanes active.

// Inclusive max over lanes <= this one: max_scan_incl (txs_common.h).
// Inclusive min over lanes >= this one.
__device__ __forceinline__ int min_scan_rev_incl(int v) {
  const int ri = lane() & 15, row = lane() >> 4;
  int t;
  t = dpp<kRowShl1>(v, v); if (ri + 1 < 16) v = min(v, t);
  t = dpp<kRowShl2>(v, v); if (ri + 2 < 16) v = min(v, t);
  t = dpp<kRowShl4>(v, v); if (ri + 4 < 16) v = min(v, t);
  t = dpp<kRowShl8>(v, v); if (ri + 8 < 16) v = min(v, t);
  const int e1 = readlane(v, 16), e2 = readlane(v, 32), e3 = readlane(v, 48);
  const int c2 = e3, c1 = min(e2, c2), c0 = min(e1, c1);
  const int c = row == 0 ? c0 : row == 1 ? c1 : row == 2 ? c2 : v;
  return min(v, c);
}

// Inclusive segmented scan over lanes; hl = last lane <= this one that starts
// a segment (-1 if none): the sum over lanes [max(hl, 0), lane].
template <typename T>
__device__ __forceinline__ T seg_scan(T v, int hl) {
  const int ln = lane(), ri = ln & 15, row = ln >> 4;
  const T z = T(0);
  T t;
  t = dpp<kRowShr1>(z, v); if (ri >= 1 && ln - 1 >= hl) v += t;
  t = dpp<kRowShr2>(z, v); if (ri >= 2 && ln - 2 >= hl) v += t;
  t = dpp<kRowShr4>(z, v); if (ri >= 4 && ln - 4 >= hl) v += t;
  t = dpp<kRowShr8>(z, v); if (ri >= 8 && ln - 8 >= hl) v += t;
  // carry of row r = value at the end of row r-1, chained while that row
  // holds no segment start
  const T e0 = readlane(v, 15), e1 = readlane(v, 31), e2 = readlane(v, 47);
  const int h1 = readlane(hl, 31), h2 = readlane(hl, 47);
  const T c1 = e0;
  const T c2 = e1 + (h1 < 16 ? c1 : z);
  const T c3 = e2 + (h2 < 32 ? c2 : z);
  const T c = row == 1 ? c1 : row == 2 ? c2 : c3;
  if (row > 0 && hl < 16 * row) v += c;
  return v;
}

// Reverse inclusive segmented scan; fl = first lane >= this one that ends the
// chain (64 if none): the sum over lanes [lane, min(fl, 63)].
template <typename T>
__device__ __forceinline__ T seg_scan_rev(T v, int fl) {
  const int ln = lane(), ri = ln & 15, row = ln >> 4;
  const T z = T(0);
  T t;
  t = dpp<kRowShl1>(z, v); if (ri + 1 < 16 && ln + 1 <= fl) v += t;
  t = dpp<kRowShl2>(z, v); if (ri + 2 < 16 && ln + 2 <= fl) v += t;
  t = dpp<kRowShl4>(z, v); if (ri + 4 < 16 && ln + 4 <= fl) v += t;
  t = dpp<kRowShl8>(z, v); if (ri + 8 < 16 && ln + 8 <= fl) v += t;
  // carry of row r = value at the start of row r+1, chained while that row
  // holds no chain end
  const T e1 = readlane(v, 16), e2 = readlane(v, 32), e3 = readlane(v, 48);
  const int f1 = readlane(fl, 16), f2 = readlane(fl, 32);
  const T c2 = e3;
  const T c1 = e2 + (f2 > 47 ? c2 : z);
  const T c0 = e1 + (f1 > 31 ? c1 : z);
  const T c = row == 0 ? c0 : row == 1 ? c1 : c2;
  if (row < 3 && fl > 16 * row + 15) v += c;
  return v;
}

// Value of the previous / next lane (lane 0 / 63 receive `fill`).
template <typename T>
__device__ __forceinline__ T lane_prev(T v, T fill) { return dpp<kWaveShr1>(fill, v); }
template <typename T>
__device__ __forceinline__ T lane_next(T v, T fill) { return dpp<kWaveShl1>(fill, v); }

__device__ __forceinline__ double readlane_d(double v, int l) { return readlane(v, l); }

// exp(-x) from a binary64 argument: -x log2(e) = n + f with n an integer and
// f in [0,1), so exp(-x) = 2^f 2^n; 2^f comes from the hardware exp2 on a
// binary32 f, whose rounding (2^-24 absolute) is the only error besides the
// exp2 itself, for any x.  Results below 2^-250 flush to zero.
__device__ __forceinline__ float exp_neg(double x) {
  // x < 16: rounding x and x log2(e) to binary32 costs < 2e-6 relative in the
  // result, so the exponent is formed in binary32
  if (x < 16.0) return __builtin_amdgcn_exp2f((float)x * -1.44269504f);
  const double y = -x * 1.4426950408889634;
  if (!(y > -250.0)) return 0.0f;
  const double n = floor(y);
  return ldexpf(__builtin_amdgcn_exp2f((float)(y - n)), (int)n);
}

// 1 - exp(-t) for t >= 0 without cancellation: for t < 1/4 the nested Taylor
// form t (1 - t/2 (1 - t/3 (1 - ... (1 - t/7)))) (truncation < 1e-9
// relative), otherwise 1 - exp(-t) with exp(-t) <= 0.78.  (Inputs are finite
// and >= 0; an infinite t gives 1.)
__device__ __forceinline__ float one_minus_exp_neg(float t) {
  if (t < 0.25f) {
    float r = 1.0f - t * (1.0f / 7.0f);
    r = 1.0f - t * (1.0f / 6.0f) * r;
    r = 1.0f - t * (1.0f / 5.0f) * r;
    r = 1.0f - t * 0.25f * r;
    r = 1.0f - t * (1.0f / 3.0f) * r;
    r = 1.0f - t * 0.5f * r;
    return t * r;
  }
  // exp(-t) <= 0.78 here: its binary32 error is < 6e-7 of 1 - exp(-t)
  return 1.0f - __builtin_amdgcn_exp2f(t * -1.44269504f);
}

struct Acc5 {
  float r, g, b, o, d;
};
__device__ __forceinline__ Acc5 seg_scan(Acc5 v, int hl) {
  return {seg_scan(v.r, hl), seg_scan(v.g, hl), seg_scan(v.b, hl), seg_scan(v.o, hl),
          seg_scan(v.d, hl)};
}
__device__ __forceinline__ Acc5 shfl_up1(Acc5 v) {
  return {lane_prev(v.r, 0.0f), lane_prev(v.g, 0.0f), lane_prev(v.b, 0.0f), lane_prev(v.o, 0.0f),
          lane_prev(v.d, 0.0f)};
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

// load_k for a lane whose K samples all lie below the window's limit.
__device__ __forceinline__ void load_k_whole(const float* __restrict__ src, int64_t pos0,
                                             float (&v)[K]) {
  const float4* p = reinterpret_cast<const float4*>(src + pos0);
#pragma unroll
  for (int q = 0; q < K / 4; ++q) {
    const float4 x = p[q];
    v[4 * q] = x.x;
    v[4 * q + 1] = x.y;
    v[4 * q + 2] = x.z;
    v[4 * q + 3] = x.w;
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

// A window's rgb rows [p, p+W) loaded as consecutive-lane float4s (rg[q] =
// float4 q*64 + lane of the window: consecutive lanes, consecutive 16 bytes)
// to each lane's own K rows, through LDS.
__device__ __forceinline__ void unstage_rgb(const float4 (&rg)[3 * K / 4], float4* stage,
                                            float (&c)[K][3]) {
  const int ln = lane();
#pragma unroll
  for (int q = 0; q < 3 * K / 4; ++q) stage[q * kWave + ln] = rg[q];
  wave_sync();
  float f[3 * K];
#pragma unroll
  for (int q = 0; q < 3 * K / 4; ++q) {
    const float4 x = stage[(3 * K / 4) * ln + q];
    f[4 * q] = x.x;
    f[4 * q + 1] = x.y;
    f[4 * q + 2] = x.z;
    f[4 * q + 3] = x.w;
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) c[j][c3] = f[3 * j + c3];
  wave_sync();
}

// Writes the staged [W][3] rows to dst rows [p, p+W) as consecutive-lane float4s.
__device__ __forceinline__ void store_rgb_staged(float* __restrict__ dst, int64_t p,
                                                 const float4* stage) {
  const int ln = lane();
  wave_sync();
  float4* d4 = reinterpret_cast<float4*>(dst + 3 * p);
#pragma unroll
  for (int q = 0; q < 3 * K / 4; ++q) d4[q * kWave + ln] = stage[q * kWave + ln];
  wave_sync();
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
__device__ __forceinline__ void write_marks(MarkLds& L, int64_t p, int64_t st, int64_t en,
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

__device__ __forceinline__ void read_marks(const MarkLds& L, int (&mk)[K + 1]) {
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
  if (n_samples >= ((int64_t)1 << 31)) {
    set_error("%s: %lld samples do not fit the int32 packed layout", who, (long long)n_samples);
    return TXS_EOVERFLOW;
  }
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
