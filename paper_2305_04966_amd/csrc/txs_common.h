// Shared host/device helpers of the txs HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "txs.h"

namespace txs {

// ---------------------------------------------------------------- host side
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

// Status of the kernel launches enqueued since the last check.
txs_status launch_status(const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

#define TXS_REQUIRE(cond, ...)           \
  do {                                   \
    if (!(cond)) {                       \
      ::txs::set_error(__VA_ARGS__);     \
      return TXS_EINVAL;                 \
    }                                    \
  } while (0)

inline unsigned grid_1d(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// -------------------------------------------------------------- device side
constexpr int kWave = 64;

__device__ __forceinline__ int lane() { return static_cast<int>(__lane_id()); }

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, d, kWave); }
template <typename T>
__device__ __forceinline__ T shfl_down(T v, int d) { return __shfl_down(v, d, kWave); }
template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t t = __shfl_xor((long long)v, d, kWave);
    v = v > t ? v : t;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_min(int64_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t t = __shfl_xor((long long)v, d, kWave);
    v = v < t ? v : t;
  }
  return v;
}

// ---- DPP lane moves (data-parallel primitives of the GFX9 family) ----------
// A VALU move that reads another lane of the same wave: no LDS round trip.
// Lanes whose source lane is outside the row (row_*) or the wave (wave_*)
// receive `old`.
enum DppCtrl : int {
  kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108,
  kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118,
  kWaveShl1 = 0x130, kWaveShr1 = 0x138,
};

template <int kCtrl>
__device__ __forceinline__ int dpp(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, kCtrl, 0xf, 0xf, false);
}
template <int kCtrl>
__device__ __forceinline__ float dpp(float old, float src) {
  return __int_as_float(dpp<kCtrl>(__float_as_int(old), __float_as_int(src)));
}
template <int kCtrl>
__device__ __forceinline__ double dpp(double old, double src) {
  const int lo = dpp<kCtrl>(__double2loint(old), __double2loint(src));
  const int hi = dpp<kCtrl>(__double2hiint(old), __double2hiint(src));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Unsigned 32-bit division by a divisor d >= 1 fixed at launch, by a
// multiply-high and two shifts (Granlund and Montgomery 1994, Sec. 4): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n),
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) for every n < 2^32.
struct FastDiv {
  uint32_t m = 1;
  int s1 = 0, s2 = 0;
  FastDiv() = default;
  __host__ __device__ explicit FastDiv(uint32_t d) {
    int l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    m = (uint32_t)(((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d) + 1);
    s1 = l < 1 ? l : 1;
    s2 = l > 1 ? l - 1 : 0;
  }
  __host__ __device__ uint32_t div(uint32_t n) const {
    const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

// Keeps the compiler from moving memory operations across this point; the
// hardware already executes one wave's LDS operations in order.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Inclusive sum over lanes <= this one (same scheme as max_scan_incl).
__device__ __forceinline__ float add_scan_incl(float v) {
  const int ri = lane() & 15, row = lane() >> 4;
  float t;
  t = dpp<kRowShr1>(v, v); if (ri >= 1) v += t;
  t = dpp<kRowShr2>(v, v); if (ri >= 2) v += t;
  t = dpp<kRowShr4>(v, v); if (ri >= 4) v += t;
  t = dpp<kRowShr8>(v, v); if (ri >= 8) v += t;
  const float e0 = readlane(v, 15), e1 = readlane(v, 31), e2 = readlane(v, 47);
  const float c1 = e0, c2 = c1 + e1, c3 = c2 + e2;
  return row == 1 ? v + c1 : row == 2 ? v + c2 : row == 3 ? v + c3 : v;
}

// Inclusive max over lanes <= this one: DPP row shifts inside each 16-lane row,
// then the three row carries by readlane.
__device__ __forceinline__ int max_scan_incl(int v) {
  const int ri = lane() & 15, row = lane() >> 4;
  int t;
  t = dpp<kRowShr1>(v, v); if (ri >= 1) v = max(v, t);
  t = dpp<kRowShr2>(v, v); if (ri >= 2) v = max(v, t);
  t = dpp<kRowShr4>(v, v); if (ri >= 4) v = max(v, t);
  t = dpp<kRowShr8>(v, v); if (ri >= 8) v = max(v, t);
  const int e0 = readlane(v, 15), e1 = readlane(v, 31), e2 = readlane(v, 47);
  const int c1 = e0, c2 = max(c1, e1), c3 = max(c2, e2);
  const int c = row == 1 ? c1 : row == 2 ? c2 : row == 3 ? c3 : v;
  return max(v, c);
}

}  // namespace txs
