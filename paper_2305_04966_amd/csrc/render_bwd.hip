// Backward direction of the packed rendering engine: the adjoint of the
// compositing of Eq. 2 (the gradients that reach the radiance field in
// Algorithm 1) and the adjoint of the weights alone.
//
// For the samples i of one ray, with v_i = dL/dw_i,
//   dL/dsigma_i = Delta_i (T_{i+1} v_i - sum_{j>i} w_j v_j).
// A wave walks its sample range right to left, so both suffix sums it needs
// -- Q_i = sum_{j>=i} tau_j and S_i = sum_{j>i} w_j v_j -- are reverse
// segmented scans with carries (binary64).  The exclusive optical depth is
// P_i = P_total - Q_i, with P_total the ray's total optical depth from the
// forward (or from a tau-only pre-pass), so T_i = exp(-P_i) needs no forward
// walk and nothing per sample is stored between the two directions.
// Windows of 4 samples per lane: the adjoint's state per sample is larger
// than the forward's, and half the window keeps three waves per SIMD.
#define TXS_RENDER_ADJOINT
#include "render_window.h"

namespace txs {
namespace {

// One window, right to left.  Samples [p, p+W) clipped to lim; marks in LDS;
// seg_in = ray lane whose segment covers position p (-1: none).  cQ, cS: the
// sums entering from the right for the chain that crosses the window end;
// replaced by the sums leaving to the left.
//
// xt0, xt1, xsg hold this window's t0, t1, sigma and rg its colour rows
// (whole windows only), all loaded one window ahead: when p_next >= 0 they are
// refilled with those of the window [p_next, lim_next) -- always whole --
// while this one computes.
template <int kMode>
__device__ void bwd_window(const Args& a, WaveLds& L, float4* stage, int64_t p, int64_t lim,
                           int seg_in, double& cQ, double& cS, float (&xt0)[K],
                           float (&xt1)[K], float (&xsg)[K], float4 (&rg)[3 * K / 4],
                           int64_t p_next, int64_t lim_next) {
  const int ln = lane();
  const int64_t pos0 = p + (int64_t)K * ln;
  float tau[K], delta[K], mid[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    delta[j] = xt1[j] - xt0[j];
    tau[j] = xsg[j] * delta[j];
    mid[j] = 0.5f * (xt0[j] + xt1[j]);
  }
  const bool full = p + W <= lim;  // wave-uniform
  if (p_next >= 0) {
    const int64_t pn = p_next + (int64_t)K * ln;
    load_k(a.t0, pn, lim_next, xt0);
    load_k(a.t1, pn, lim_next, xt1);
    load_k(a.sigma, pn, lim_next, xsg);
  }
  int mk[K + 1];
  read_marks(L, mk);

  // ray of each element: nearest mark to the left (within the window) or seg_in
  int lastm = -1;
  bool has_mark = false;
  double Bq = 0.0;  // tau over the lane's elements before its first mark
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (mk[j] != 0) {
      has_mark = true;
      lastm = K * ln + j;
    }
    if (!has_mark) Bq += (double)tau[j];
  }
  const int cp = lane_prev(max_scan_incl(lastm), -1);
  const int seg_lane = (cp >= 0) ? decode_mark(L.marks[cp]) : seg_in;
  int cur_[K];
  bool own[K];
  bool all_own = true;
  {
    int cur = seg_lane;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (mk[j] != 0) cur = decode_mark(mk[j]);
      cur_[j] = cur;
      own[j] = cur >= 0 && (pos0 + j) < lim;
      all_own = all_own && own[j];
    }
  }

  // reverse scan of tau: suffix optical depth entering each lane from the right
  const int fl = min_scan_rev_incl(has_mark ? ln : kWave);
  double Rq = seg_scan_rev(Bq, fl);
  if (fl == kWave) Rq += cQ;
  double q = lane_next(Rq, cQ);

  // right to left: P_i = P_total - Q_i; weights, v, u = w v, T_{i+1} v; d_rgb
  float u[K], tv[K];
  double Bs = 0.0;  // u over the lane's elements before its first mark
  {
    float c[K][3];
    float gwv[K];
    if (kMode == kBwd) {
      if (full) unstage_rgb(rg, stage, c);
      else load_rgb(a.rgb, pos0, lim, c);
      if (p_next >= 0) {  // the next window's colour rows, while this one computes
        const float4* s4 = reinterpret_cast<const float4*>(a.rgb + 3 * p_next);
#pragma unroll
        for (int q = 0; q < 3 * K / 4; ++q) rg[q] = s4[q * kWave + ln];
      }
    } else {
      load_k(a.g_w, pos0, lim, gwv);
    }
    // whole window owned by this wave's rays: colour gradients leave through LDS
    const bool staged = kMode == kBwd && a.d_rgb && __ballot(!all_own) == 0;
    float* st = reinterpret_cast<float*>(stage) + 3 * K * ln;
    float T_right = 0.0f;  // T of element j+1 (same lane)
    // the ray's total optical depth and cotangent row change only where a ray
    // starts inside the lane: loaded once per ray, not per element
    int cs = cur_[K - 1] < 0 ? 0 : cur_[K - 1];
    double ptot = L.ptot[cs];
    float4 g4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b4 = g4;
    if (kMode == kBwd) {
      g4 = *reinterpret_cast<const float4*>(&L.cot[cs][0]);
      b4 = *reinterpret_cast<const float4*>(&L.cot[cs][4]);
    }
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      if (j < K - 1 && mk[j + 1] != 0) {  // element j belongs to an earlier ray
        cs = cur_[j] < 0 ? 0 : cur_[j];
        ptot = L.ptot[cs];
        if (kMode == kBwd) {
          g4 = *reinterpret_cast<const float4*>(&L.cot[cs][0]);
          b4 = *reinterpret_cast<const float4*>(&L.cot[cs][4]);
        }
      }
      q += (double)tau[j];  // Q_j, inclusive
      const double P = ptot - q;
      const float T = exp_neg(P);
      // T_{j+1} is the next element's T unless j ends its lane or its ray
      const float Tn = (j == K - 1 || mk[j + 1] != 0) ? exp_neg(P + (double)tau[j]) : T_right;
      T_right = T;
      const float w = T * one_minus_exp_neg(tau[j]);
      float v;
      if (kMode == kBwd) {
        // cot row: g0 g1 g2 h | q bg0 bg1 bg2
        v = g4.x * (c[j][0] - b4.y) + g4.y * (c[j][1] - b4.z) + g4.z * (c[j][2] - b4.w) + g4.w +
            b4.x * mid[j];
        if (staged) {
          st[3 * j] = w * g4.x;
          st[3 * j + 1] = w * g4.y;
          st[3 * j + 2] = w * g4.z;
        } else if (a.d_rgb && own[j]) {
          a.d_rgb[3 * (pos0 + j)] = w * g4.x;
          a.d_rgb[3 * (pos0 + j) + 1] = w * g4.y;
          a.d_rgb[3 * (pos0 + j) + 2] = w * g4.z;
        }
      } else {
        v = gwv[j];
      }
      u[j] = own[j] ? w * v : 0.0f;
      tv[j] = own[j] ? Tn * v : 0.0f;
      if (mk[j] != 0) q = 0.0;
    }
    if (staged) store_rgb_staged(a.d_rgb, p, stage);
    bool before_first = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (mk[j] != 0) before_first = false;
      if (before_first) Bs += (double)u[j];
    }
  }

  // reverse scan of u: the suffix sum entering each lane from the right
  double Rs = seg_scan_rev(Bs, fl);
  if (fl == kWave) Rs += cS;
  double s = lane_next(Rs, cS);
  // the difference T_{j+1} v_j - S_j in binary32: its rounding is relative to
  // the larger term, which is within the adjoint's own conditioning scale
  float ds[K];
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    ds[j] = delta[j] * (tv[j] - (float)s);
    s += (double)u[j];
    if (mk[j] != 0) s = 0.0;
  }
  store_k(a.d_sigma, pos0, ds, own);
  cQ = readlane_d(Rq, 0);
  cS = readlane_d(Rs, 0);
}

template <int kMode>
__global__ __launch_bounds__(kBlock) void bwd_kernel(Args a) {
  __shared__ WaveLds lds[kWaves];
  __shared__ float4 stage_mem[kWaves][StageSize<kMode>::value];
  WaveLds& L = lds[threadIdx.x / kWave];
  float4* stage = stage_mem[threadIdx.x / kWave];
  const int ln = lane();
  const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  const int32_t r0 = (int32_t)(wave * kWave);
  if (r0 >= a.n_rays) return;
  const int32_t r = r0 + ln;
  const WaveRange R = wave_range(a, r);
  if (R.hi <= R.lo) return;
  if (kMode == kBwd) {
    float* row = L.cot[ln];
    if (r < a.n_rays) {
      row[0] = a.g_rgb[3 * (int64_t)r];
      row[1] = a.g_rgb[3 * (int64_t)r + 1];
      row[2] = a.g_rgb[3 * (int64_t)r + 2];
      row[3] = a.g_op ? a.g_op[r] : 0.0f;
      row[4] = a.g_depth ? a.g_depth[r] : 0.0f;
      row[5] = a.bg ? a.bg[3 * (int64_t)r] : 0.0f;
      row[6] = a.bg ? a.bg[3 * (int64_t)r + 1] : 0.0f;
      row[7] = a.bg ? a.bg[3 * (int64_t)r + 2] : 0.0f;
    }
  }
  if (a.optical) {
    L.ptot[ln] = (r < a.n_rays) ? a.optical[r] : 0.0;
    wave_sync();
  } else {
    wave_optical_depth(a, L, r0, R);
  }
  const int64_t p0 = R.lo & ~int64_t(3);
  const int64_t nwin = (R.hi - p0 + W - 1) / W;
  double cQ = 0.0, cS = 0.0;
  float xt0[K], xt1[K], xsg[K];
  float4 rg[3 * K / 4];
#pragma unroll
  for (int q = 0; q < 3 * K / 4; ++q) rg[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  {
    const int64_t p = p0 + (nwin - 1) * W, lim = min(p + W, R.hi);
    load_k(a.t0, p + (int64_t)K * ln, lim, xt0);
    load_k(a.t1, p + (int64_t)K * ln, lim, xt1);
    load_k(a.sigma, p + (int64_t)K * ln, lim, xsg);
    if (kMode == kBwd && p + W <= lim) {
      const float4* s4 = reinterpret_cast<const float4*>(a.rgb + 3 * p);
#pragma unroll
      for (int q = 0; q < 3 * K / 4; ++q) rg[q] = s4[q * kWave + ln];
    }
  }
  for (int64_t i = nwin - 1; i >= 0; --i) {
    const int64_t p = p0 + i * W;
    const uint64_t cover = __ballot(R.active && R.st < p && p < R.en);
    const int seg_in = cover ? __builtin_ctzll(cover) : -1;
    write_marks(L, p, R.st, R.en, R.active);
    // the window to the left, [p - W, p), is whole and inside [p0, R.hi)
    bwd_window<kMode>(a, L, stage, p, min(p + W, R.hi), seg_in, cQ, cS, xt0, xt1, xsg, rg,
                      i > 0 ? p - W : -1, p);
  }
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_render_bwd(const int32_t* packed_info, int32_t fixed_count,
                                     int32_t n_rays, int64_t n_samples, const float* t0,
                                     const float* t1, const float* sigma, const float* rgb,
                                     const float* bg, const double* optical_depth,
                                     const float* g_rgb, const float* g_opacity,
                                     const float* g_depth, float* d_sigma, float* d_rgb,
                                     void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_common("txs_render_bwd", packed_info, fixed_count, n_rays, n_samples,
                                  t0, t1, sigma))
    return s;
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(g_rgb, "txs_render_bwd: null g_rgb");
  TXS_REQUIRE(n_samples == 0 || (rgb && d_sigma), "txs_render_bwd: null rgb or d_sigma");
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
  a.optical = optical_depth;
  a.g_rgb = g_rgb;
  a.g_op = g_opacity;
  a.g_depth = g_depth;
  a.d_sigma = d_sigma;
  a.d_rgb = d_rgb;
  return launch(bwd_kernel<kBwd>, a, stream, "txs_render_bwd");
}

extern "C" txs_status txs_weights_bwd(const int32_t* packed_info, int32_t fixed_count,
                                      int32_t n_rays, int64_t n_samples, const float* t0,
                                      const float* t1, const float* sigma,
                                      const double* optical_depth, const float* g_w,
                                      float* d_sigma, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_common("txs_weights_bwd", packed_info, fixed_count, n_rays,
                                  n_samples, t0, t1, sigma))
    return s;
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(n_samples == 0 || (g_w && d_sigma), "txs_weights_bwd: null g_w or d_sigma");
  Args a{};
  a.info = packed_info;
  a.fixed = fixed_count;
  a.n_rays = n_rays;
  a.n_samples = n_samples;
  a.t0 = t0;
  a.t1 = t1;
  a.sigma = sigma;
  a.optical = optical_depth;
  a.g_w = g_w;
  a.d_sigma = d_sigma;
  return launch(bwd_kernel<kWBwd>, a, stream, "txs_weights_bwd");
}
