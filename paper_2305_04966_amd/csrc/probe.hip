// Measurement support, not part of the method: the memory traffic of the
// render kernels without their arithmetic.  stream_probe: the adjoint's.  A wave owns a contiguous range of
// samples and walks it in windows of 512 (8 consecutive samples per lane,
// 16-byte loads; colour rows as consecutive-lane float4s), reading t0, t1,
// sigma and rgb and writing one float and one float3 per sample, as the
// adjoint does.  Its time bounds what any kernel with that traffic and layout
// can reach on the device.
#include "txs_common.h"
#include "txs_measure.h"

namespace txs {
namespace {

constexpr int kPK = 8, kPW = kWave * kPK, kPWaves = 4;

__global__ __launch_bounds__(kWave* kPWaves) void stream_probe_kernel(
    int64_t n, int64_t per_wave, const float* __restrict__ t0, const float* __restrict__ t1,
    const float* __restrict__ sg, const float* __restrict__ rgb, float* __restrict__ oa,
    float* __restrict__ ob) {
  const int ln = lane();
  const int64_t wave = (int64_t)blockIdx.x * kPWaves + threadIdx.x / kWave;
  const int64_t lo = wave * per_wave, hi = min(lo + per_wave, n);
  int64_t p = lo;
  for (; p + kPW <= hi; p += kPW) {
    const int64_t q0 = p + (int64_t)kPK * ln;
    const float4* a = reinterpret_cast<const float4*>(t0 + q0);
    const float4* b = reinterpret_cast<const float4*>(t1 + q0);
    const float4* c = reinterpret_cast<const float4*>(sg + q0);
    float4* o = reinterpret_cast<float4*>(oa + q0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float4 x = a[h], y = b[h], z = c[h];
      o[h] = make_float4(x.x + y.x + z.x, x.y + y.y + z.y, x.z + y.z + z.z, x.w + y.w + z.w);
    }
    const float4* r = reinterpret_cast<const float4*>(rgb + 3 * p);
    float4* s = reinterpret_cast<float4*>(ob + 3 * p);
#pragma unroll
    for (int q = 0; q < 3 * kPK / 4; ++q) {
      const float4 v = r[q * kWave + ln];
      s[q * kWave + ln] = make_float4(v.x + v.x, v.y + v.y, v.z + v.z, v.w + v.w);
    }
  }
  for (int64_t i = p + ln; i < hi; i += kWave) {  // tail of the range
    oa[i] = t0[i] + t1[i] + sg[i];
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) ob[3 * i + c3] = rgb[3 * i + c3] + rgb[3 * i + c3];
  }
}

// The forward render's reads in its layout: each wave walks its range in
// windows of 512 samples, t0, t1 and sigma as 8 consecutive samples per lane
// (two 16-byte loads each), rgb rows as consecutive-lane float4s; a per-lane
// sum keeps every load live and is written once per lane at the end.
__global__ __launch_bounds__(kWave* kPWaves) void read_probe_kernel(
    int64_t n, int64_t per_wave, const float* __restrict__ t0, const float* __restrict__ t1,
    const float* __restrict__ sg, const float* __restrict__ rgb, float* __restrict__ out) {
  const int ln = lane();
  const int64_t wave = (int64_t)blockIdx.x * kPWaves + threadIdx.x / kWave;
  const int64_t lo = wave * per_wave, hi = min(lo + per_wave, n);
  if (lo >= n) return;  // a wave past the last range (the launch rounds up to blocks)
  float acc = 0.0f;
  int64_t p = lo;
  for (; p + kPW <= hi; p += kPW) {
    const int64_t q0 = p + (int64_t)kPK * ln;
    const float4* a = reinterpret_cast<const float4*>(t0 + q0);
    const float4* b = reinterpret_cast<const float4*>(t1 + q0);
    const float4* c = reinterpret_cast<const float4*>(sg + q0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float4 x = a[h], y = b[h], z = c[h];
      acc += (x.x + y.x + z.x) + (x.y + y.y + z.y) + (x.z + y.z + z.z) + (x.w + y.w + z.w);
    }
    const float4* r = reinterpret_cast<const float4*>(rgb + 3 * p);
#pragma unroll
    for (int q = 0; q < 3 * kPK / 4; ++q) {
      const float4 v = r[q * kWave + ln];
      acc += (v.x + v.y) + (v.z + v.w);
    }
  }
  for (int64_t i = p + ln; i < hi; i += kWave)  // tail of the range
    acc += t0[i] + t1[i] + sg[i] + rgb[3 * i] + rgb[3 * i + 1] + rgb[3 * i + 2];
  out[wave * kWave + ln] = acc;
}

}  // namespace
}  // namespace txs

extern "C" int64_t txs_read_probe_out_size(void) { return (int64_t)16384 * txs::kWave; }

extern "C" txs_status txs_read_probe(int64_t n_samples, const float* t0, const float* t1,
                                     const float* sigma, const float* rgb, float* out,
                                     void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_samples >= 0, "txs_read_probe: negative size");
  if (n_samples == 0) return TXS_OK;
  TXS_REQUIRE(t0 && t1 && sigma && rgb && out, "txs_read_probe: null array");
  const int64_t waves = 16384;  // as many as the forward's 2^20-ray launch
  const int64_t per_wave = ((n_samples + waves - 1) / waves + kPW - 1) / kPW * kPW;
  const int64_t used = (n_samples + per_wave - 1) / per_wave;
  hipLaunchKernelGGL(read_probe_kernel, dim3((unsigned)((used + kPWaves - 1) / kPWaves)),
                     dim3(kWave * kPWaves), 0, as_stream(stream), n_samples, per_wave, t0, t1,
                     sigma, rgb, out);
  return launch_status("txs_read_probe");
}

extern "C" txs_status txs_stream_probe(int64_t n_samples, const float* t0, const float* t1,
                                       const float* sigma, const float* rgb, float* out_a,
                                       float* out_b, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_samples >= 0, "txs_stream_probe: negative size");
  if (n_samples == 0) return TXS_OK;
  TXS_REQUIRE(t0 && t1 && sigma && rgb && out_a && out_b, "txs_stream_probe: null array");
  const int64_t waves = 16384;  // as many as the adjoint's 2^20-ray launch
  const int64_t per_wave = ((n_samples + waves - 1) / waves + kPW - 1) / kPW * kPW;
  const int64_t used = (n_samples + per_wave - 1) / per_wave;
  hipLaunchKernelGGL(stream_probe_kernel, dim3((unsigned)((used + kPWaves - 1) / kPWaves)),
                     dim3(kWave * kPWaves), 0, as_stream(stream), n_samples, per_wave, t0, t1,
                     sigma, rgb, out_a, out_b);
  return launch_status("txs_stream_probe");
}
