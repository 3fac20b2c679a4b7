// Forward window of the packed rendering engine, shared by the forward
// kernels and by the adjoint's optical-depth pre-pass.
#pragma once

#include "render_common.h"

namespace txs {
namespace {

struct FwdCarry {
  int seg;     // ray lane of the segment running into the window, -1 = dead
  double P;    // optical depth accumulated by that segment
  Acc5 acc;    // render: partial sums of that segment
  int cnt;     // filter: kept samples of that segment
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
  } else if (kMode == kPrefix) {
    a.kept[r] = cnt;
  }
}

// One window of the forward direction: samples [p, p+W) clipped to lim, the
// window's marks already in LDS, cin the state entering the window.
// kColour: the render reads colours (a.rgb non-null); kFull: the window is
// whole (lim = p + W).  A whole window issues all of its loads (t0, t1, sigma
// and the colour rows) in one branch-free run, so the first wait covers them
// together instead of the colours' latency following pass 1.
template <int kMode, bool kColour, bool kFull, class Lds>
__device__ FwdCarry fwd_window(const Args& a, Lds& L, float4* stage, int32_t r0, int64_t p,
                               int64_t lim, const FwdCarry& cin) {
  const int ln = lane();
  const int64_t pos0 = p + (int64_t)K * ln;
  float t0v[K], t1v[K], sg[K];
  // (zeroed: left undefined on the paths that do not load it, the compiler
  // kept the array in scratch memory)
  float4 rg[3 * K / 4];
#pragma unroll
  for (int q = 0; q < 3 * K / 4; ++q) rg[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (kFull) {
    load_k_whole(a.t0, pos0, t0v);
    load_k_whole(a.t1, pos0, t1v);
    load_k_whole(a.sigma, pos0, sg);
    if (kMode == kFwd && kColour) {
      // consecutive-lane float4s of the window's rows, unstaged after pass 1
      const float4* s4 = reinterpret_cast<const float4*>(a.rgb + 3 * p);
#pragma unroll
      for (int q = 0; q < 3 * K / 4; ++q) rg[q] = s4[q * kWave + ln];
    }
    // keep the scheduler from sinking the colour loads to their use
    __builtin_amdgcn_sched_barrier(0);
  } else {
    load_k(a.t0, pos0, lim, t0v);
    load_k(a.t1, pos0, lim, t1v);
    load_k(a.sigma, pos0, lim, sg);
  }
  int mk[K + 1];
  read_marks(L, mk);

  // pass 1: optical depth per sample and the lane's tail aggregate
  float tau[K];
  double run = (ln == 0) ? cin.P : 0.0;
  int lastm = -1;
  bool has_mark = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    tau[j] = sg[j] * (t1v[j] - t0v[j]);
    if (mk[j] != 0) {
      run = 0.0;
      has_mark = true;
      lastm = K * ln + j;
    }
    run += (double)tau[j];
  }
  const int hl = max_scan_incl(has_mark ? ln : -1);
  const double incl_tau = seg_scan(run, hl);
  double P = lane_prev(incl_tau, cin.P);
  const int cp = lane_prev(max_scan_incl(lastm), -1);
  int cur = (cp >= 0) ? decode_mark(L.marks[cp]) : cin.seg;

  // pass 2: transmittance, weights, per-ray sums.  Inside the lane the
  // optical depth of sample j is P_s + loc_j: P_s (binary64) where the lane's
  // current segment starts, loc_j (binary32) the sum of the segment's taus in
  // this lane before j, at most K of them.  The transmittance takes
  // fl(fl(P_s) + loc_j): at most K + 2 binary32 roundings, each < 2^-24 P, and
  // one more in the scaling by log2(e), so T is within (K + 3) 2^-24 P
  // relative besides the exp2's own rounding (6.6e-7 P for K = 8), which the
  // weights' relative bar admits wherever T is not negligible.  The per-ray
  // totals (the adjoint subtracts suffix sums from them) and the filter's
  // decisions keep the binary64 sum P per sample.
  float Psf = (float)P, loc = 0.0f;
  Acc5 acc = (ln == 0) ? cin.acc : Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
  int cnt = (ln == 0) ? cin.cnt : 0;
  bool first = true;
  Acc5 first_acc{0.f, 0.f, 0.f, 0.f, 0.f};
  int first_cnt = 0, first_ray = -1;
  float wv[K];
  bool own[K];
  float c[K][3];
  if (kMode == kFwd) {
    if (kColour) {
      if (kFull) unstage_rgb(rg, stage, c);
      else load_rgb(a.rgb, pos0, lim, c);
    } else {  // colourless: weights, opacity and depth only
#pragma unroll
      for (int j = 0; j < K; ++j) c[j][0] = c[j][1] = c[j][2] = 0.0f;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (mk[j] != 0) {
      cur = decode_mark(mk[j]);
      P = 0.0;
      Psf = 0.0f;
      loc = 0.0f;
      acc = Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
      cnt = 0;
      first = false;
    }
    const bool live = cur >= 0 && (kFull || (pos0 + j) < lim);
    own[j] = live;
    if (kMode == kFwd) {
      const float T = __builtin_amdgcn_exp2f((Psf + loc) * -1.44269504f);
      const float alpha = one_minus_exp_neg(tau[j]);
      const float w = live ? T * alpha : 0.0f;
      wv[j] = w;
      const float mid = 0.5f * (t0v[j] + t1v[j]);
      acc.r += w * c[j][0];
      acc.g += w * c[j][1];
      acc.b += w * c[j][2];
      acc.o += w;
      acc.d += w * mid;
    } else if (kMode == kPrefix) {
      if (live && P <= a.p_max) ++cnt;
    }
    P += (double)tau[j];
    loc += tau[j];
    if (mk[j + 1] != 0 && cur >= 0) {  // last sample of ray `cur`
      if (kMode == kFwd && a.out_optical) a.out_optical[r0 + cur] = P;
      if constexpr (kMode == kTotal) L.ptot[cur] = P;
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
  cout.P = readlane_d(incl_tau, kWave - 1);
  cout.seg = readlane(cur, kWave - 1);
  cout.acc = Acc5{0.f, 0.f, 0.f, 0.f, 0.f};
  cout.cnt = 0;
  if (kMode == kFwd) {
    const Acc5 incl = seg_scan(acc, hl);
    const Acc5 carry = shfl_up1(incl);
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
  } else if (kMode == kPrefix) {
    const int incl = seg_scan(cnt, hl);
    const int carry = lane_prev(incl, 0);
    if (first_ray >= 0)
      emit_ray<kMode>(a, r0 + first_ray, Acc5{}, first_cnt + (ln > 0 ? carry : 0));
    cout.cnt = readlane(incl, kWave - 1);
  }
  return cout;
}

// Per-ray total optical depth of the rays of one wave into L.ptot (the
// adjoint's pre-pass when the forward's optical depths are not supplied).
__device__ __forceinline__ void wave_optical_depth(const Args& a, WaveLds& L, int32_t r0, const WaveRange& R) {
  L.ptot[lane()] = 0.0;
  wave_sync();
  FwdCarry carry{-1, 0.0, Acc5{0.f, 0.f, 0.f, 0.f, 0.f}, 0};
  for (int64_t p = R.lo & ~int64_t(3); p < R.hi; p += W) {
    write_marks(L, p, R.st, R.en, R.active);
    if (R.hi - p >= W)  // a whole window (no overflow: p < R.hi)
      carry = fwd_window<kTotal, false, true>(a, L, nullptr, r0, p, p + W, carry);
    else
      carry = fwd_window<kTotal, false, false>(a, L, nullptr, r0, p, R.hi, carry);
  }
  wave_sync();
}

}  // namespace
}  // namespace txs
