// Forward direction of the packed rendering engine: compositing (Eq. 2) and
// the transmittance-prefix filter (Section 4.2, no-gradient filtering).
#include "render_common.h"

namespace txs {
namespace {

// ----------------------------------------------------------- forward window
struct FwdCarry {
  int seg;  // ray lane of the segment running into the window, -1 = dead
  float P;  // optical depth accumulated by that segment
  Acc5 acc; // fwd: partial sums of that segment
  int cnt;  // prefix: kept samples of that segment
};

template <int kMode>
__device__ __forceinline__ void emit_ray(const Args& a, int32_t r, const Acc5& s, int cnt) {
  if (kMode == kFwd) {
    float br = 0.f, bgc = 0.f, bb = 0.f;
    if (a.bg) {
      const float one_minus = 1.0f - s.o;
      br = one_minus * a.bg[3 * (int64_t)r];
      bgc = one_minus * a.bg[3 * (int64_t)r + 1];
      bb = one_minus * a.bg[3 * (int64_t)r + 2];
    }
    a.out_rgb[3 * (int64_t)r] = s.r + br;
    a.out_rgb[3 * (int64_t)r + 1] = s.g + bgc;
    a.out_rgb[3 * (int64_t)r + 2] = s.b + bb;
    a.out_opacity[r] = s.o;
    a.out_depth[r] = s.d;
  } else {
    a.kept[r] = cnt;
  }
}

// One window of the forward direction (render forward / prefix filter).
// Samples [p, p+W) clipped to lim; the window's marks are already in LDS.
template <int kMode>
__device__ FwdCarry fwd_window(const Args& a, const WaveLds& L, int32_t r0, int64_t p,
                               int64_t lim, const FwdCarry& cin) {
  const int ln = lane();
  const int64_t pos0 = p + (int64_t)K * ln;
  float t0v[K], t1v[K], sg[K];
  load_k(a.t0, pos0, lim, t0v);
  load_k(a.t1, pos0, lim, t1v);
  load_k(a.sigma, pos0, lim, sg);
  int mk[K + 1];
  read_marks(L, mk);

  // pass 1: optical depth per sample and the lane's tail aggregate
  float tau[K];
  float run = (ln == 0) ? cin.P : 0.0f;
  int lastm = -1;
  bool has_mark = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    tau[j] = sg[j] * (t1v[j] - t0v[j]);
    if (mk[j] != 0) {
      run = 0.0f;
      has_mark = true;
      lastm = K * ln + j;
    }
    run += tau[j];
  }
  const int hl = max_scan_incl(has_mark ? ln : -1);
  const float incl_tau = seg_scan(run, hl);
  float P = shfl_up(incl_tau, 1);
  if (ln == 0) P = cin.P;
  int cp = shfl_up(max_scan_incl(lastm), 1);
  if (ln == 0) cp = -1;
  int cur = (cp >= 0) ? decode_mark(L.marks[cp]) : cin.seg;

  // pass 2: transmittance, weights, per-ray sums
  Acc5 acc = (ln == 0) ? cin.acc : Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
  int cnt = (ln == 0) ? cin.cnt : 0;
  bool first = true;
  Acc5 first_acc{0.f, 0.f, 0.f, 0.f, 0.f};
  int first_cnt = 0, first_ray = -1;
  float wv[K];
  bool own[K];
  float c[K][3];
  if (kMode == kFwd) load_rgb(a.rgb, pos0, lim, c);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (mk[j] != 0) {
      cur = decode_mark(mk[j]);
      P = 0.0f;
      acc = Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
      cnt = 0;
      first = false;
    }
    const bool live = cur >= 0 && (pos0 + j) < lim;
    own[j] = live;
    if (kMode == kFwd) {
      const float T = expf(-P);
      const float alpha = -expm1f(-tau[j]);
      const float w = live ? T * alpha : 0.0f;
      wv[j] = w;
      const float mid = 0.5f * (t0v[j] + t1v[j]);
      acc.r += w * c[j][0];
      acc.g += w * c[j][1];
      acc.b += w * c[j][2];
      acc.o += w;
      acc.d += w * mid;
    } else {
      if (live && P <= a.p_max) ++cnt;
    }
    P += tau[j];
    if (mk[j + 1] != 0 && cur >= 0) {
      if (first) {
        first_acc = acc;
        first_cnt = cnt;
        first_ray = cur;
      } else {
        emit_ray<kMode>(a, r0 + cur, acc, cnt);
      }
    }
  }
  if (kMode == kFwd && a.out_w) store_k(a.out_w, pos0, wv, own);

  FwdCarry cout;
  cout.P = readlane(incl_tau, kWave - 1);
  cout.seg = readlane(cur, kWave - 1);
  if (kMode == kFwd) {
    const Acc5 incl = seg_scan(acc, hl);
    Acc5 carry = shfl_up1(incl);
    if (first_ray >= 0) {
      if (ln > 0) {
        first_acc.r += carry.r;
        first_acc.g += carry.g;
        first_acc.b += carry.b;
        first_acc.o += carry.o;
        first_acc.d += carry.d;
      }
      emit_ray<kMode>(a, r0 + first_ray, first_acc, 0);
    }
    cout.acc = Acc5{readlane(incl.r, kWave - 1), readlane(incl.g, kWave - 1),
                    readlane(incl.b, kWave - 1), readlane(incl.o, kWave - 1),
                    readlane(incl.d, kWave - 1)};
    cout.cnt = 0;
  } else {
    const int incl = seg_scan(cnt, hl);
    const int carry = shfl_up(incl, 1);
    if (first_ray >= 0) emit_ray<kMode>(a, r0 + first_ray, Acc5{}, first_cnt + (ln > 0 ? carry : 0));
    cout.cnt = readlane(incl, kWave - 1);
    cout.acc = Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
  }
  return cout;
}

template <int kMode>
__global__ __launch_bounds__(kBlock) void fwd_kernel(Args a) {
  __shared__ WaveLds lds[kWaves];
  WaveLds& L = lds[threadIdx.x / kWave];
  const int ln = lane();
  const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  const int32_t r0 = (int32_t)(wave * kWave);
  if (r0 >= a.n_rays) return;
  const int32_t r = r0 + ln;
  int64_t st;
  int32_t ct;
  ray_row(a, r, st, ct);
  if (r < a.n_rays && ct <= 0) emit_ray<kMode>(a, r, Acc5{0.f, 0.f, 0.f, 0.f, 0.f}, 0);
  const bool active = r < a.n_rays && ct > 0;
  // wave-wide sample range [lo, hi) of the owned rays
  const int64_t lo = wave_min(active ? st : INT64_MAX);
  int64_t hi = wave_max(active ? st + ct : (int64_t)0);
  if (hi <= lo) return;
  hi = min(hi, a.n_samples);
  FwdCarry carry{-1, 0.0f, Acc5{0.f, 0.f, 0.f, 0.f, 0.f}, 0};
  for (int64_t p = lo & ~int64_t(3); p < hi; p += W) {
    write_marks(L, p, st, ct, active);
    carry = fwd_window<kMode>(a, L, r0, p, min(p + W, hi), carry);
  }
}

}  // namespace
}  // namespace txs

using txs::Args;

extern "C" txs_status txs_render_fwd(const int32_t* packed_info, int32_t fixed_count,
                                     int32_t n_rays, int64_t n_samples, const float* t0,
                                     const float* t1, const float* sigma, const float* rgb,
                                     const float* bg, float* out_rgb, float* out_opacity,
                                     float* out_depth, float* out_weights, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_common("txs_render_fwd", packed_info, fixed_count, n_rays, n_samples,
                                  t0, t1, sigma))
    return s;
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(out_rgb && out_opacity && out_depth, "txs_render_fwd: null output");
  TXS_REQUIRE(n_samples == 0 || rgb, "txs_render_fwd: null rgb");
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
  return launch(fwd_kernel<kFwd>, a, stream, "txs_render_fwd");
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
  a.p_max = (float)(-std::log((double)t_min));
  a.kept = kept_counts;
  return launch(fwd_kernel<kPrefix>, a, stream, "txs_transmittance_prefix");
}

