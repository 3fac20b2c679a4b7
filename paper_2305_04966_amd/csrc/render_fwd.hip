// Forward direction of the packed rendering engine: compositing (Eq. 2) and
// the transmittance-prefix filter (Section 4.2, no-gradient filtering).
#include "render_window.h"

namespace txs {
namespace {

template <int kMode, bool kColour>
__global__ __launch_bounds__(kBlock) void fwd_kernel(Args a) {
  __shared__ MarkLds lds[kWaves];
  __shared__ float4 stage_mem[kWaves][StageSize<kMode>::value];
  MarkLds& L = lds[threadIdx.x / kWave];
  float4* stage = stage_mem[threadIdx.x / kWave];
  const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  const int32_t r0 = (int32_t)(wave * kWave);
  if (r0 >= a.n_rays) return;
  const int32_t r = r0 + lane();
  const WaveRange R = wave_range(a, r);
  if (r < a.n_rays && !R.active) {
    emit_ray<kMode>(a, r, Acc5{0.f, 0.f, 0.f, 0.f, 0.f}, 0);
    if (kMode == kFwd && a.out_optical) a.out_optical[r] = 0.0;
  }
  FwdCarry carry{-1, 0.0, Acc5{0.f, 0.f, 0.f, 0.f, 0.f}, 0};
  for (int64_t p = R.lo & ~int64_t(3); p < R.hi; p += W) {
    write_marks(L, p, R.st, R.en, R.active);
    if (R.hi - p >= W)  // a whole window (no overflow: p < R.hi)
      carry = fwd_window<kMode, kColour, true>(a, L, stage, r0, p, p + W, carry);
    else
      carry = fwd_window<kMode, kColour, false>(a, L, stage, r0, p, R.hi, carry);
  }
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_render_fwd(const int32_t* packed_info, int32_t fixed_count,
                                     int32_t n_rays, int64_t n_samples, const float* t0,
                                     const float* t1, const float* sigma, const float* rgb,
                                     const float* bg, float* out_rgb, float* out_opacity,
                                     float* out_depth, float* out_weights,
                                     double* out_optical_depth, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_common("txs_render_fwd", packed_info, fixed_count, n_rays, n_samples,
                                  t0, t1, sigma))
    return s;
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(out_rgb && out_opacity && out_depth, "txs_render_fwd: null output");
  Args a{};
  a.info = packed_info;
  a.fixed = fixed_count;
  a.n_rays = n_rays;
  a.n_samples = n_samples;
  a.t0 = t0;
  a.t1 = t1;
  a.sigma = sigma;
  a.rgb = rgb;
  a.bg = bg;
  a.out_rgb = out_rgb;
  a.out_opacity = out_opacity;
  a.out_depth = out_depth;
  a.out_w = out_weights;
  a.out_optical = out_optical_depth;
  return rgb ? launch(fwd_kernel<kFwd, true>, a, stream, "txs_render_fwd")
             : launch(fwd_kernel<kFwd, false>, a, stream, "txs_render_fwd");
}

extern "C" txs_status txs_transmittance_prefix(const int32_t* packed_info, int32_t n_rays,
                                               int64_t n_samples, const float* t0,
                                               const float* t1, const float* sigma, float t_min,
                                               int32_t* kept_counts, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(packed_info || n_rays == 0, "txs_transmittance_prefix: null packed_info");
  if (txs_status s = check_common("txs_transmittance_prefix", packed_info, 0, n_rays, n_samples,
                                  t0, t1, sigma))
    return s;
  TXS_REQUIRE(t_min > 0.0f && t_min <= 1.0f, "txs_transmittance_prefix: t_min must be in (0,1]");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(kept_counts, "txs_transmittance_prefix: null output");
  Args a{};
  a.info = packed_info;
  a.n_rays = n_rays;
  a.n_samples = n_samples;
  a.t0 = t0;
  a.t1 = t1;
  a.sigma = sigma;
  a.p_max = -std::log((double)t_min);
  a.kept = kept_counts;
  return launch(fwd_kernel<kPrefix, false>, a, stream, "txs_transmittance_prefix");
}
