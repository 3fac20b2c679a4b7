// Inverse transform sampling from a transmittance estimator (Eqs. 1-3,
// Section 3.1): the CDF of the rendering weights is 1 - T, so a piecewise-
// constant density estimate gives its CDF in closed form and new interval
// edges come from inverting it.  Also the uniform estimator (Table 1, first
// row) that seeds a proposal round.
#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kMaxBins = 1024;
constexpr int kRsWaves = 4;

// Persistent waves, one ray at a time: edges to LDS, wave-wide scan of the
// bin masses into the CDF (LDS), then one binary search per output edge.  LDS
// per wave is 2 (n_bins + 1) floats (dynamic).  Rows of 64 to
// kRegChunks * 64 - 1 bins are held in registers (64 consecutive bins per
// chunk, one per lane), and the wave loads its next ray's row while it
// resamples the current one (128 bins -> 32: 0.19 -> 0.16 ms for 2^18 rays);
// rows of at most 32 bins go two to a wave (one per half-wave), rows of at
// most 16 four to a wave; other rows are read in place.  Every kind does the
// same arithmetic in the same order.
//
// out != NULL: edges [n_rays, n_out+1]; otherwise the intervals between them,
// t0o[r*n_out + k] = edge k and t1o[r*n_out + k] = edge k+1.
constexpr int kRegChunks = 4;

struct RsArgs {
  int32_t n_rays, n_bins;
  const float* edges;
  const float* vals;
  int32_t mode, n_out;
  const float* u;
  float* out;
  float* t0o;
  float* t1o;
};

// Inclusive sum over the lanes <= this one within its half-wave: the scheme of
// add_scan_incl without the carry from lane 31 into lanes 32..63, so each
// half's sums are bit for bit those of a whole-wave scan of its values alone.
__device__ __forceinline__ float half_scan_incl(float v) {
  const int ri = lane() & 15, row = lane() >> 4;
  float t;
  t = dpp<kRowShr1>(v, v); if (ri >= 1) v += t;
  t = dpp<kRowShr2>(v, v); if (ri >= 2) v += t;
  t = dpp<kRowShr4>(v, v); if (ri >= 4) v += t;
  t = dpp<kRowShr8>(v, v); if (ri >= 8) v += t;
  const float e0 = readlane(v, 15), e2 = readlane(v, 47);
  return row == 1 ? v + e0 : row == 3 ? v + e2 : v;
}

// The same within each 16-lane row (the row steps of add_scan_incl alone).
__device__ __forceinline__ float row_scan_incl(float v) {
  const int ri = lane() & 15;
  float t;
  t = dpp<kRowShr1>(v, v); if (ri >= 1) v += t;
  t = dpp<kRowShr2>(v, v); if (ri >= 2) v += t;
  t = dpp<kRowShr4>(v, v); if (ri >= 4) v += t;
  t = dpp<kRowShr8>(v, v); if (ri >= 8) v += t;
  return v;
}

// CDF of a ray into F[0..n_bins] (its edges already in e) by kLanes lanes
// (the whole wave, or one half-wave per ray when n_bins <= 32); ln is the
// lane within them, valid false for a half-wave without a ray (it still
// takes part in the wave's scan, with zeros).  Returns F_n and whether the
// uniform estimator replaced a massless row.  vi(c, i) is the value of bin
// i = kLanes c + ln (i < n_bins).
template <int kLanes, class Val>
__device__ __forceinline__ float ray_cdf(const RsArgs& a, float* F, const float* e, Val vi,
                                         bool& uniform, int ln, bool valid) {
  float carry = 0.0f;
  if (ln == 0 && valid) F[0] = 0.0f;
  for (int base = 0, c = 0; base < a.n_bins; base += kLanes, ++c) {
    const int i = base + ln;
    float m = 0.0f;
    if (valid && i < a.n_bins)
      m = (a.mode != TXS_PDF_WEIGHTS) ? vi(c, i) * (e[i + 1] - e[i]) : vi(c, i);
    const float incl = (kLanes == kWave ? add_scan_incl(m)
                        : kLanes == 32  ? half_scan_incl(m)
                                        : row_scan_incl(m)) + carry;
    if (valid && i < a.n_bins) F[i + 1] = (a.mode != TXS_PDF_WEIGHTS) ? -expm1f(-incl) : incl;
    if (kLanes == kWave) carry = readlane(incl, kWave - 1);  // one chunk for half-waves
  }
  wave_sync();
  float Fn = valid ? F[a.n_bins] : 1.0f;
  uniform = !(Fn > 1e-12f);
  if (uniform) {
    for (int i = ln; i <= a.n_bins; i += kLanes) F[i] = (float)i / (float)a.n_bins;
    wave_sync();
    Fn = 1.0f;
  }
  return Fn;
}

// Output edges of ray r from its CDF F and edges e (both in LDS), kLanes
// lanes, ln the lane within them.
template <int kLanes>
__device__ __forceinline__ void ray_invert(const RsArgs& a, int64_t r, const float* F,
                                           const float* e, float Fn, bool uniform, int ln) {
  const float* vr = a.vals + r * a.n_bins;
  for (int k = ln; k <= a.n_out; k += kLanes) {
    const float uk = a.u ? a.u[r * (a.n_out + 1) + k] : (float)k / (float)a.n_out;
    const float up = uk * Fn;
    // largest i in [0, n_bins] with F[i] <= up (F[0] = 0 <= up).  u' = F_n
    // (u = 1) is i = n_bins: F is non-decreasing, but its binary32 lane scan
    // may put a bin of zero mass an ulp above F_n, which the search would
    // otherwise stop at
    int lo = up >= Fn ? a.n_bins : 0, hi = a.n_bins;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (F[mid] <= up) lo = mid;
      else hi = mid - 1;
    }
    float t;
    if (lo >= a.n_bins) {
      t = e[a.n_bins];
    } else {
      const float f0 = F[lo], f1 = F[lo + 1];
      const float frac = (up - f0) / (f1 - f0);
      const float width = e[lo + 1] - e[lo];
      if (a.mode == TXS_PDF_SIGMA_EXP && !uniform) {
        // constant density in the bin: the share x of the transmittance at
        // the bin's start used up by u' is frac (1 - exp(-tau)); then
        // t - e = -log(1 - x) / sigma, and t stays inside the bin
        const float tau = vr[lo] * width;
        const float x = frac * -expm1f(-tau);
        t = fminf(e[lo] + width * (-log1pf(-x) / tau), e[lo + 1]);
      } else {
        t = e[lo] + frac * width;
      }
    }
    if (a.out) {
      a.out[r * (a.n_out + 1) + k] = t;
    } else {
      if (k < a.n_out) a.t0o[r * a.n_out + k] = t;
      if (k > 0) a.t1o[r * a.n_out + k - 1] = t;
    }
  }
}

// Kernel kinds: rows read in place by the whole wave, rows of 64..255 bins in
// registers with the next ray prefetched, two rays per wave (one per
// half-wave) for rows of at most 32 bins, four (one per 16-lane row) for rows
// of at most 16.
enum RsKind { kInPlace = 0, kRegRows = 1, kHalfWaves = 2, kQuarterWaves = 3 };

template <int kKind>
__global__ __launch_bounds__(kWave* kRsWaves) void resample_kernel(RsArgs a) {
  extern __shared__ float lds_rs[];
  const int w = threadIdx.x / kWave, ln = lane();
  float* F = lds_rs + (size_t)w * 2 * (a.n_bins + 1);
  float* e = F + (a.n_bins + 1);
  const int64_t stride = (int64_t)gridDim.x * kRsWaves;
  const int64_t r0 = (int64_t)blockIdx.x * kRsWaves + w;
  if constexpr (kKind == kHalfWaves || kKind == kQuarterWaves) {
    // kParts rays per wave, kLanes lanes each; each part has its own F and e
    constexpr int kParts = kKind == kHalfWaves ? 2 : 4, kLanes = kWave / kParts;
    const int pl = ln % kLanes, part = ln / kLanes;
    float* Fh = lds_rs + (size_t)(kParts * w + part) * 2 * (a.n_bins + 1);
    float* eh = Fh + (a.n_bins + 1);
    for (int64_t pr = r0; kParts * pr < a.n_rays; pr += stride) {  // wave-uniform group index
      const int64_t r = kParts * pr + part;
      const bool valid = r < a.n_rays;
      const float* er = a.edges + r * (a.n_bins + 1);
      const float* vr = a.vals + r * a.n_bins;
      if (valid)
        for (int i = pl; i <= a.n_bins; i += kLanes) eh[i] = er[i];
      wave_sync();
      bool uniform;
      const float Fn = ray_cdf<kLanes>(a, Fh, eh, [&](int, int i) { return vr[i]; }, uniform, pl,
                                       valid);
      if (valid) ray_invert<kLanes>(a, r, Fh, eh, Fn, uniform, pl);
      wave_sync();  // this group's LDS reads are done before the next group overwrites it
    }
    return;
  }
  if constexpr (kKind == kRegRows) {
    // row c-chunk values of ray rr: edge 64c + lane (<= n_bins), bin 64c + lane
    auto fetch = [&](int64_t rr, float (&fe)[kRegChunks], float (&fv)[kRegChunks]) {
#pragma unroll
      for (int c = 0; c < kRegChunks; ++c) {
        const int i = kWave * c + ln;
        fe[c] = (rr < a.n_rays && i <= a.n_bins) ? a.edges[rr * (a.n_bins + 1) + i] : 0.0f;
        fv[c] = (rr < a.n_rays && i < a.n_bins) ? a.vals[rr * a.n_bins + i] : 0.0f;
      }
    };
    float ce[kRegChunks], cv[kRegChunks];
    fetch(r0, ce, cv);
    for (int64_t r = r0; r < a.n_rays; r += stride) {
      float ne[kRegChunks], nv[kRegChunks];
      fetch(r + stride, ne, nv);
#pragma unroll
      for (int c = 0; c < kRegChunks; ++c)
        if (kWave * c + ln <= a.n_bins) e[kWave * c + ln] = ce[c];
      wave_sync();
      bool uniform;
      const float Fn = ray_cdf<kWave>(a, F, e,
                                      [&](int c, int) {
                                        float v = cv[0];
#pragma unroll
                                        for (int q = 1; q < kRegChunks; ++q) v = (c == q) ? cv[q] : v;
                                        return v;
                                      },
                                      uniform, ln, true);
      ray_invert<kWave>(a, r, F, e, Fn, uniform, ln);
      wave_sync();  // this ray's LDS reads are done before the next ray overwrites it
#pragma unroll
      for (int c = 0; c < kRegChunks; ++c) {
        ce[c] = ne[c];
        cv[c] = nv[c];
      }
    }
    return;
  }
  for (int64_t r = r0; r < a.n_rays; r += stride) {
    const float* er = a.edges + r * (a.n_bins + 1);
    const float* vr = a.vals + r * a.n_bins;
    for (int i = ln; i <= a.n_bins; i += kWave) e[i] = er[i];
    wave_sync();
    bool uniform;
    const float Fn = ray_cdf<kWave>(a, F, e, [&](int, int i) { return vr[i]; }, uniform, ln, true);
    ray_invert<kWave>(a, r, F, e, Fn, uniform, ln);
    wave_sync();  // this ray's LDS reads are done before the next ray overwrites it
  }
}

// grid of persistent resample blocks
inline unsigned resample_blocks(int32_t n_rays) {
  const int64_t need = ((int64_t)n_rays + kRsWaves - 1) / kRsWaves;
  return (unsigned)std::min<int64_t>(need, 256 * 16);
}

// one instantiation per kernel kind, so that each keeps its own register
// budget and occupancy
inline void launch_resample(const RsArgs& a, hipStream_t s) {
  const unsigned blocks = resample_blocks(a.n_rays);
  const size_t lds = kRsWaves * 2 * (a.n_bins + 1) * sizeof(float);
  if (a.n_bins <= 16)  // four rays per wave: four times the LDS per wave
    hipLaunchKernelGGL(resample_kernel<kQuarterWaves>,
                       dim3(resample_blocks((a.n_rays + 3) / 4)), dim3(kWave * kRsWaves), 4 * lds,
                       s, a);
  else if (a.n_bins <= 32)  // two rays per wave: twice the LDS per wave, half the waves
    hipLaunchKernelGGL(resample_kernel<kHalfWaves>, dim3(resample_blocks((a.n_rays + 1) / 2)),
                       dim3(kWave * kRsWaves), 2 * lds, s, a);
  else if (a.n_bins >= kWave && a.n_bins < kRegChunks * kWave)
    hipLaunchKernelGGL(resample_kernel<kRegRows>, dim3(blocks), dim3(kWave * kRsWaves), lds, s, a);
  else
    hipLaunchKernelGGL(resample_kernel<kInPlace>, dim3(blocks), dim3(kWave * kRsWaves), lds, s, a);
}

// Equally spaced edges e_k = lo + (hi - lo) * (k / n_bins) over per-ray
// intervals.  A block writes whole rows: the endpoints of its rays go to LDS
// first (thread per ray), then its threads store the block's contiguous run
// of edges (a fixed divisor maps a position in the run to its row).
constexpr int kEdgeBlock = 256;
constexpr int kEdgeWords = 4096;  // edges per block, at least one row

inline int32_t edge_rows(int32_t n_bins) { return std::max(1, kEdgeWords / (n_bins + 1)); }

// chord of the ray through the outermost cube, clipped to [near, far]
struct ChordEnds {
  txs_grid g;
  float near_plane, far_plane;
  const float* ro;
  const float* rd;
  __device__ void operator()(int64_t r, float& lo, float& hi) const {
    const float h = g.half_extent0 * (float)(1 << (g.n_levels - 1));
    float tn = near_plane, tf = far_plane;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float inv = 1.0f / rd[3 * r + a];
      const float o = ro[3 * r + a];
      const float tlo = ((g.center[a] - h) - o) * inv;
      const float thi = ((g.center[a] + h) - o) * inv;
      tn = fmaxf(tn, fminf(tlo, thi));
      tf = fminf(tf, fmaxf(tlo, thi));
    }
    if (!(tn < tf)) {
      tn = near_plane;
      tf = near_plane;
    }
    lo = tn;
    hi = tf;
  }
};

// a given span per ray
struct SpanEnds {
  const float* span;
  __device__ void operator()(int64_t r, float& lo, float& hi) const {
    lo = span[2 * r];
    hi = span[2 * r + 1];
  }
};

// Spacing of the edges between a ray's endpoints: equal steps in t, or equal
// steps in disparity 1/t (e_k = 1 / (1/lo + (1/hi - 1/lo) k/n), lo > 0; the
// end edges are lo and hi themselves).
enum Spacing : int { kLinearT = 0, kDisparity = 1 };

template <int kSpacing, class Ends>
__global__ __launch_bounds__(kEdgeBlock) void edges_kernel(Ends ends, int32_t n_rays,
                                                          int32_t n_bins, int32_t rows,
                                                          FastDiv per_row,
                                                          float* __restrict__ out) {
  __shared__ float s_lo[kEdgeWords / 2], s_hi[kEdgeWords / 2];  // rows <= 2048 (n_bins >= 1)
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int nr = (int)std::min<int64_t>(rows, (int64_t)n_rays - r0);
  for (int j = threadIdx.x; j < nr; j += kEdgeBlock) ends(r0 + j, s_lo[j], s_hi[j]);
  __syncthreads();
  const int E = n_bins + 1;
  const int cnt = nr * E;
  float* o = out + r0 * E;
  for (int j = threadIdx.x; j < cnt; j += kEdgeBlock) {
    const int rr = (int)per_row.div((uint32_t)j);
    const int k = j - rr * E;
    const float lo = s_lo[rr], hi = s_hi[rr];
    if (kSpacing == kLinearT) {
      o[j] = lo + (hi - lo) * ((float)k / (float)n_bins);
    } else {
      const float a = 1.0f / lo, b = 1.0f / hi;
      o[j] = k == 0 ? lo : (k == n_bins ? hi : 1.0f / (a + (b - a) * ((float)k / (float)n_bins)));
    }
  }
}

template <int kSpacing = kLinearT, class Ends>
void launch_edges(const Ends& ends, int32_t n_rays, int32_t n_bins, float* out,
                  hipStream_t stream) {
  const int32_t rows = edge_rows(n_bins);
  const int64_t blocks = ((int64_t)n_rays + rows - 1) / rows;
  hipLaunchKernelGGL((edges_kernel<kSpacing, Ends>), dim3((unsigned)blocks), dim3(kEdgeBlock), 0,
                     stream, ends, n_rays, n_bins, rows, FastDiv((uint32_t)(n_bins + 1)), out);
}

// t0[r*n + k] = e[r][k], t1[r*n + k] = e[r][k+1]: thread per output pair
__global__ __launch_bounds__(256) void intervals_kernel(const float* __restrict__ edges,
                                                        int64_t total, int32_t n,
                                                        float* __restrict__ t0,
                                                        float* __restrict__ t1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / n;
  const float* e = edges + i + r;  // row r starts at r*(n+1) = i - k + r
  t0[i] = e[0];
  t1[i] = e[1];
}

// Sorted union of two sorted edge rows per ray, a [na] and b [nb] ->
// out [na+nb] (the fine pass of the coarse-to-fine PDF estimator renders the
// coarse and the fine edges together).  Output rank of a_i = i + #{b < a_i},
// of b_j = j + #{a <= b_j}: a stable merge, a first among equal values.  A
// block stages whole rows of a and b in LDS; each thread places elements by
// a binary search in the other row.
constexpr int kMergeWords = 4096;  // LDS words per block, at least one row
constexpr int kMaxMergeRow = 4096;

inline int32_t merge_rows(int32_t na, int32_t nb) {
  return std::max(1, kMergeWords / (na + nb));
}

__device__ __forceinline__ int count_below(const float* row, int n, float v, bool or_equal) {
  int lo = 0, hi = n;  // first index whose value is >= v (> v with or_equal)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool before = or_equal ? (row[mid] <= v) : (row[mid] < v);
    if (before) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void merge_kernel(int32_t n_rays, int32_t na, int32_t nb,
                                                    int32_t rows, FastDiv div_a, FastDiv div_b,
                                                    const float* __restrict__ a,
                                                    const float* __restrict__ b,
                                                    float* __restrict__ out) {
  extern __shared__ float s_rows[];
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int nr = (int)std::min<int64_t>(rows, (int64_t)n_rays - r0);
  float* sa = s_rows;
  float* sb = s_rows + (size_t)rows * na;
  for (int j = threadIdx.x; j < nr * na; j += blockDim.x) sa[j] = a[r0 * na + j];
  for (int j = threadIdx.x; j < nr * nb; j += blockDim.x) sb[j] = b[r0 * nb + j];
  __syncthreads();
  const int W = na + nb;
  float* o = out + r0 * W;
  for (int j = threadIdx.x; j < nr * na; j += blockDim.x) {
    const int rr = (int)div_a.div((uint32_t)j);
    const int i = j - rr * na;
    const float v = sa[j];
    o[rr * W + i + count_below(sb + rr * nb, nb, v, false)] = v;
  }
  for (int j = threadIdx.x; j < nr * nb; j += blockDim.x) {
    const int rr = (int)div_b.div((uint32_t)j);
    const int i = j - rr * nb;
    const float v = sb[j];
    o[rr * W + i + count_below(sa + rr * na, na, v, true)] = v;
  }
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_edges_to_intervals(const float* edges, int32_t n_rays, int32_t n,
                                             float* t0, float* t1, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && n >= 1, "txs_edges_to_intervals: bad size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(edges && t0 && t1, "txs_edges_to_intervals: null array");
  const int64_t total = (int64_t)n_rays * n;
  hipLaunchKernelGGL(intervals_kernel, dim3(grid_1d(total, 256)), dim3(256), 0,
                     as_stream(stream), edges, total, n, t0, t1);
  return launch_status("txs_edges_to_intervals");
}

extern "C" txs_status txs_resample(int32_t n_rays, int32_t n_bins, const float* edges,
                                   const float* vals, int32_t mode, int32_t n_out,
                                   const float* u, float* out_edges, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0, "txs_resample: n_rays < 0");
  TXS_REQUIRE(n_bins >= 1 && n_bins <= kMaxBins, "txs_resample: n_bins must be in [1,%d]",
              kMaxBins);
  TXS_REQUIRE(n_out >= 1, "txs_resample: n_out must be >= 1");
  TXS_REQUIRE(mode == TXS_PDF_SIGMA || mode == TXS_PDF_WEIGHTS || mode == TXS_PDF_SIGMA_EXP,
              "txs_resample: bad mode %d",
              mode);
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(edges && vals && out_edges, "txs_resample: null array");
  launch_resample(RsArgs{n_rays, n_bins, edges, vals, mode, n_out, u, out_edges, nullptr, nullptr},
                  as_stream(stream));
  return launch_status("txs_resample");
}

extern "C" txs_status txs_resample_intervals(int32_t n_rays, int32_t n_bins, const float* edges,
                                             const float* vals, int32_t mode, int32_t n_out,
                                             const float* u, float* out_t0, float* out_t1,
                                             void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0, "txs_resample_intervals: n_rays < 0");
  TXS_REQUIRE(n_bins >= 1 && n_bins <= kMaxBins,
              "txs_resample_intervals: n_bins must be in [1,%d]", kMaxBins);
  TXS_REQUIRE(n_out >= 1, "txs_resample_intervals: n_out must be >= 1");
  TXS_REQUIRE(mode == TXS_PDF_SIGMA || mode == TXS_PDF_WEIGHTS || mode == TXS_PDF_SIGMA_EXP,
              "txs_resample_intervals: bad mode %d", mode);
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(edges && vals && out_t0 && out_t1, "txs_resample_intervals: null array");
  launch_resample(RsArgs{n_rays, n_bins, edges, vals, mode, n_out, u, nullptr, out_t0, out_t1},
                  as_stream(stream));
  return launch_status("txs_resample_intervals");
}

extern "C" txs_status txs_uniform_bins(const txs_grid* grid, float near_plane, float far_plane,
                                       const float* rays_o, const float* rays_d, int32_t n_rays,
                                       int32_t n_bins, float* out_edges, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(grid, "txs_uniform_bins: null grid");
  TXS_REQUIRE(grid->n_levels >= 1 && grid->n_levels <= 8, "txs_uniform_bins: bad n_levels");
  TXS_REQUIRE(std::isfinite(grid->half_extent0) && grid->half_extent0 > 0,
              "txs_uniform_bins: bad half_extent0");
  TXS_REQUIRE(n_rays >= 0 && n_bins >= 1 && n_bins <= (1 << 24), "txs_uniform_bins: bad size");
  TXS_REQUIRE(near_plane >= 0.0f && far_plane > near_plane, "txs_uniform_bins: bad planes");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && out_edges, "txs_uniform_bins: null array");
  launch_edges(ChordEnds{*grid, near_plane, far_plane, rays_o, rays_d}, n_rays, n_bins,
               out_edges, as_stream(stream));
  return launch_status("txs_uniform_bins");
}

extern "C" txs_status txs_disparity_bins(const txs_grid* grid, float near_plane,
                                         float far_plane, const float* rays_o,
                                         const float* rays_d, int32_t n_rays, int32_t n_bins,
                                         float* out_edges, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(grid, "txs_disparity_bins: null grid");
  TXS_REQUIRE(grid->n_levels >= 1 && grid->n_levels <= 8, "txs_disparity_bins: bad n_levels");
  TXS_REQUIRE(std::isfinite(grid->half_extent0) && grid->half_extent0 > 0,
              "txs_disparity_bins: bad half_extent0");
  TXS_REQUIRE(n_rays >= 0 && n_bins >= 1 && n_bins <= (1 << 24), "txs_disparity_bins: bad size");
  TXS_REQUIRE(near_plane > 0.0f && far_plane > near_plane,
              "txs_disparity_bins: near_plane must be > 0 and below far_plane");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && out_edges, "txs_disparity_bins: null array");
  launch_edges<kDisparity>(ChordEnds{*grid, near_plane, far_plane, rays_o, rays_d}, n_rays,
                           n_bins, out_edges, as_stream(stream));
  return launch_status("txs_disparity_bins");
}

extern "C" txs_status txs_span_bins(int32_t n_rays, const float* span, int32_t n_bins,
                                    float* out_edges, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && n_bins >= 1 && n_bins <= (1 << 24), "txs_span_bins: bad size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(span && out_edges, "txs_span_bins: null array");
  launch_edges(SpanEnds{span}, n_rays, n_bins, out_edges, as_stream(stream));
  return launch_status("txs_span_bins");
}

extern "C" txs_status txs_merge_edges(int32_t n_rays, int32_t na, const float* a, int32_t nb,
                                      const float* b, float* out, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && na >= 1 && nb >= 1 && na <= kMaxMergeRow && nb <= kMaxMergeRow,
              "txs_merge_edges: row lengths must be in [1,%d]", kMaxMergeRow);
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(a && b && out, "txs_merge_edges: null array");
  const int32_t rows = merge_rows(na, nb);
  const int64_t blocks = ((int64_t)n_rays + rows - 1) / rows;
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)blocks), dim3(256),
                     (size_t)rows * (na + nb) * sizeof(float), as_stream(stream), n_rays, na, nb,
                     rows, FastDiv((uint32_t)na), FastDiv((uint32_t)nb), a, b, out);
  return launch_status("txs_merge_edges");
}
