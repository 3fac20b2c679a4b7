// Backward direction of the packed rendering engine: the adjoint of the
// compositing of Eq. 2 (gradients that reach the radiance field in
// Algorithm 1) and the adjoint of the weights alone.
//
// For the samples i of one ray, with v_i = dL/dw_i,
//   dL/dsigma_i = Delta_i (T_{i+1} v_i - sum_{j>i} w_j v_j).
// T and w are recomputed from the inputs; the suffix sums are an exact
// reverse segmented scan over a window that holds whole rays.  A ray longer
// than one window is processed in chunks: a forward pass stores the optical
// depth entering each chunk, then a reverse pass carries the suffix sum from
// chunk to chunk.
#include "render_common.h"

namespace txs {
namespace {

// One window (or one chunk of a long ray).  seg_in / P_in: segment running
// into the window and its optical depth; ext: suffix sum of w v beyond the
// window for the chain that reaches the window end.  Returns the suffix sum
// over the whole window of the chain that starts at its first sample (+ext).
template <int kMode>
__device__ float bwd_window(const Args& a, WaveLds& L, int64_t p, int64_t lim, int seg_in,
                            float P_in, float ext) {
  const int ln = lane();
  const int64_t pos0 = p + (int64_t)K * ln;
  int mk[K + 1];
  read_marks(L, mk);
  float tau[K], delta[K], mid[K];
  {
    float t0v[K], t1v[K], sg[K];
    load_k(a.t0, pos0, lim, t0v);
    load_k(a.t1, pos0, lim, t1v);
    load_k(a.sigma, pos0, lim, sg);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      delta[j] = t1v[j] - t0v[j];
      tau[j] = sg[j] * delta[j];
      mid[j] = 0.5f * (t0v[j] + t1v[j]);
    }
  }

  // forward segmented scan of the optical depth
  float run = (ln == 0) ? P_in : 0.0f;
  int lastm = -1;
  bool has_mark = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
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
  if (ln == 0) P = P_in;
  int cp = shfl_up(max_scan_incl(lastm), 1);
  if (ln == 0) cp = -1;
  const int seg_lane = (cp >= 0) ? decode_mark(L.marks[cp]) : seg_in;

  // ownership of each element (live sample of an owned ray)
  bool own[K];
  bool all_own = true;
  {
    int cur = seg_lane;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (mk[j] != 0) cur = decode_mark(mk[j]);
      own[j] = cur >= 0 && (pos0 + j) < lim;
      all_own = all_own && own[j];
    }
  }

  // recompute T_i, w_i; form u_i = w_i v_i and T_{i+1} v_i; write d_rgb
  float u[K], tv[K];
  float B = 0.0f;  // sum of u over the lane's elements before its first mark
  {
    float c[K][3];
    float gwv[K];
    if (kMode == kBwd) load_rgb(a.rgb, pos0, lim, c);
    else load_k(a.g_w, pos0, lim, gwv);
    int cur = seg_lane;
    int cached = -2;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, h = 0.f, q = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
    float T = expf(-P);
    bool before_first = true;
    float stage[4];
    const int64_t rgb_base = 3 * pos0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (mk[j] != 0) {
        cur = decode_mark(mk[j]);
        P = 0.0f;
        T = 1.0f;
        before_first = false;
      }
      const float Pn = P + tau[j];
      const float Tn = expf(-Pn);
      const float w = T * -expm1f(-tau[j]);
      float v;
      if (kMode == kBwd) {
        if (cur != cached && cur >= 0) {
          cached = cur;
          g0 = L.cot[cur][0];
          g1 = L.cot[cur][1];
          g2 = L.cot[cur][2];
          h = L.cot[cur][3];
          q = L.cot[cur][4];
          b0 = L.cot[cur][5];
          b1 = L.cot[cur][6];
          b2 = L.cot[cur][7];
        }
        v = g0 * (c[j][0] - b0) + g1 * (c[j][1] - b1) + g2 * (c[j][2] - b2) + h + q * mid[j];
        if (a.d_rgb) {
          const float d3[3] = {w * g0, w * g1, w * g2};
          // the lane's 3K floats go out as float4 groups once each is complete
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3) {
            const int f = 3 * j + c3;
            stage[f & 3] = d3[c3];
            if ((f & 3) == 3 && all_own)
              *reinterpret_cast<float4*>(a.d_rgb + rgb_base + (f - 3)) =
                  make_float4(stage[0], stage[1], stage[2], stage[3]);
          }
          if (!all_own && own[j]) {
            a.d_rgb[rgb_base + 3 * j] = d3[0];
            a.d_rgb[rgb_base + 3 * j + 1] = d3[1];
            a.d_rgb[rgb_base + 3 * j + 2] = d3[2];
          }
        }
      } else {
        v = gwv[j];
      }
      u[j] = own[j] ? w * v : 0.0f;
      tv[j] = own[j] ? Tn * v : 0.0f;
      if (before_first) B += u[j];
      P = Pn;
      T = Tn;
    }
  }

  // reverse segmented scan of the lanes' leading parts: the suffix sum that
  // enters each lane from the lanes after it
  const int fl = min_scan_rev_incl(has_mark ? ln : kWave);
  float R = seg_scan_rev(B, fl);
  if (fl == kWave) R += ext;
  float S = shfl_down(R, 1);
  if (ln == kWave - 1) S = ext;
  const float chain_total = readlane(R, 0);

  float ds[K];
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    ds[j] = delta[j] * (tv[j] - S);
    S += u[j];
    if (mk[j] != 0) S = 0.0f;
  }
  store_k(a.d_sigma, pos0, ds, own);
  return chain_total;
}

// Forward-only pass over one chunk of a long ray: the optical depth carried
// out of the chunk.
__device__ float tau_chunk(const Args& a, const WaveLds& L, int64_t p, int64_t lim, float P_in) {
  const int ln = lane();
  const int64_t pos0 = p + (int64_t)K * ln;
  float t0v[K], t1v[K], sg[K];
  load_k(a.t0, pos0, lim, t0v);
  load_k(a.t1, pos0, lim, t1v);
  load_k(a.sigma, pos0, lim, sg);
  int mk[K + 1];
  read_marks(L, mk);
  float run = (ln == 0) ? P_in : 0.0f;
  bool has_mark = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (mk[j] != 0) {
      run = 0.0f;
      has_mark = true;
    }
    run += sg[j] * (t1v[j] - t0v[j]);
  }
  const int hl = max_scan_incl(has_mark ? ln : -1);
  return readlane(seg_scan(run, hl), kWave - 1);
}

template <int kMode>
__global__ __launch_bounds__(kBlock) void bwd_kernel(Args a) {
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
  int64_t en = st + ct;
  if (en > a.n_samples) en = a.n_samples;
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
    wave_sync();
  }
  bool pending = r < a.n_rays && ct > 0 && en > st;
  while (true) {
    const uint64_t pend = __ballot(pending);
    if (pend == 0) break;
    const int ra = __builtin_ctzll(pend);
    const int64_t st_a = (int64_t)__shfl((long long)st, ra, kWave);
    const int64_t p = st_a & ~int64_t(3);
    // lanes >= ra whose rays end inside [p, p+W]; lanes without pending
    // samples (empty rays) do not break the run
    const uint64_t fit = __ballot(!pending || en <= p + W);
    const uint64_t run = ~(fit >> ra);
    const int nfit = run == 0 ? (kWave - ra) : __builtin_ctzll(run);
    if (nfit > 0) {
      const int rb = ra + nfit;
      const bool in_set = pending && ln >= ra && ln < rb;
      const int64_t e = wave_max(in_set ? en : (int64_t)0);
      write_marks(L, p, st, (int32_t)(en - st), in_set);
      bwd_window<kMode>(a, L, p, e, -1, 0.0f, 0.0f);
      if (in_set) pending = false;
    } else {
      // ray ra does not fit one window: chunked two-pass path
      const int64_t e = (int64_t)__shfl((long long)en, ra, kWave);
      const int64_t nchunks = (e - p + W - 1) / W;
      const bool is_ra = ln == ra;
      const int32_t ct_a = (int32_t)(en - st);
      float P = 0.0f;
      for (int64_t c = 0; c < nchunks && c < kLongCarries; ++c) {
        const int64_t pc = p + c * W;
        if (ln == 0) L.long_carry[c] = P;
        write_marks(L, pc, st, ct_a, is_ra);
        P = tau_chunk(a, L, pc, min(pc + W, e), P);
      }
      wave_sync();
      float ext = 0.0f;
      for (int64_t c = nchunks - 1; c >= 0; --c) {
        const int64_t pc = p + c * W;
        float Pc;
        if (c < kLongCarries) {
          Pc = L.long_carry[c];
        } else {  // carries of far chunks (rays beyond 32k samples) are recomputed
          Pc = 0.0f;
          for (int64_t q = 0; q < c; ++q) {
            const int64_t pq = p + q * W;
            write_marks(L, pq, st, ct_a, is_ra);
            Pc = tau_chunk(a, L, pq, min(pq + W, e), Pc);
          }
        }
        write_marks(L, pc, st, ct_a, is_ra);
        ext = bwd_window<kMode>(a, L, pc, min(pc + W, e), c == 0 ? -1 : ra, Pc, ext);
      }
      if (is_ra) pending = false;
    }
  }
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_render_bwd(const int32_t* packed_info, int32_t fixed_count,
                                     int32_t n_rays, int64_t n_samples, const float* t0,
                                     const float* t1, const float* sigma, const float* rgb,
                                     const float* bg, const float* g_rgb, const float* g_opacity,
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
  a.g_rgb = g_rgb;
  a.g_op = g_opacity;
  a.g_depth = g_depth;
  a.d_sigma = d_sigma;
  a.d_rgb = d_rgb;
  return launch(bwd_kernel<kBwd>, a, stream, "txs_render_bwd");
}

extern "C" txs_status txs_weights_bwd(const int32_t* packed_info, int32_t fixed_count,
                                      int32_t n_rays, int64_t n_samples, const float* t0,
                                      const float* t1, const float* sigma, const float* g_w,
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
  a.g_w = g_w;
  a.d_sigma = d_sigma;
  return launch(bwd_kernel<kWBwd>, a, stream, "txs_weights_bwd");
}
