// Occupancy-grid ray marching (spatial-skipping estimator, Section 3.1 and
// Table 1 second row; cascaded levels for unbounded scenes, Section 3.2).
//
// One wave marches one ray: its 64 lanes test 64 consecutive lattice points
// at a time with the binary32 recipe of txs.h (contraction disabled in this
// file), a ballot collects the occupied ones and a lane-rank (mbcnt) packs
// them, so the fill pass writes each ray's samples as contiguous, coalesced
// runs.  Every lattice point is tested, so the emitted samples are the dense
// definition exactly.
#pragma clang fp contract(off)

#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kMaxLevels = 8;
constexpr int32_t kLatticeLimit = 1 << 24;  // k stays exact in binary32
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

struct MarchArgs {
  const uint32_t* bits;
  int32_t res;
  int32_t n_levels;
  int32_t level_words;
  float center[3];
  float half_extent0;
  float near_plane, far_plane, dt0;
  int32_t max_per_ray;
  float inv_scale;  // contracted lookup: 1 / contract_scale
};

// Level-l box and grid scale, evaluated exactly as the recipe defines them.
struct LevelBox {
  float bmin[3], bmax[3], scale[3];
};

__device__ __forceinline__ LevelBox level_box(const MarchArgs& g, int l) {
  LevelBox b;
  const float h = g.half_extent0 * (float)(1 << l);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    b.bmin[a] = g.center[a] - h;
    b.bmax[a] = g.center[a] + h;
    b.scale[a] = (float)g.res / (b.bmax[a] - b.bmin[a]);
  }
  return b;
}

// Slab clip; min/max ignore the NaN of 0*inf for rays lying in a slab plane.
__device__ __forceinline__ void clip_box(const float o[3], const float inv[3], const LevelBox& b,
                                         float near_plane, float far_plane, float& tn,
                                         float& tf) {
  float t_near = near_plane, t_far = far_plane;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float tlo = (b.bmin[a] - o[a]) * inv[a];
    const float thi = (b.bmax[a] - o[a]) * inv[a];
    t_near = fmaxf(t_near, fminf(tlo, thi));
    t_far = fminf(t_far, fmaxf(tlo, thi));
  }
  tn = t_near;
  tf = t_far;
}

// What a march pass produces: per-ray sample counts, the samples themselves,
// or the span [t0 of the first sample, t1 of the last] without the samples.
enum MarchMode : int { kCount = 0, kFill = 1, kSpan = 2 };

struct Emit {
  float* t0;
  float* t1;
  int32_t* ray_id;
  int64_t base;
  int32_t count;  // kFill: the table row's count; no write at or beyond it
  int64_t capacity;
  int32_t ray;
  float lo, hi;  // kSpan: the span so far (wave-uniform)
};

// Lattice point k of segment [a, b) on level l: its midpoint a + (k + 1/2) dt
// must lie before b; valid points issue the load of their cell's grid word.
struct Lattice {
  LevelBox box;
  const uint32_t* bits;
  float a, b, dt, resf;
  int res;
  float center[3], inv_scale;  // contracted lookup
};

template <bool kContract>
__device__ __forceinline__ Lattice lattice(const MarchArgs& g, float a, float b, int l) {
  Lattice p;
  p.box = level_box(g, l);
  p.bits = kContract ? g.bits : g.bits + (int64_t)l * g.level_words;
  p.a = a;
  p.b = b;
  p.dt = g.dt0 * (float)(1 << l);
  p.res = g.res;
  p.resf = (float)g.res;
#pragma unroll
  for (int c = 0; c < 3; ++c) p.center[c] = g.center[c];
  p.inv_scale = g.inv_scale;
  return p;
}

// Cell of point x in the grid over contracted space: y = (x - center) / scale
// (times the binary32 reciprocal), y' = y if |y|^2 <= 1, else y (2 - 1/|y|)/|y|
// (Mip-NeRF 360's contraction, into the ball of radius 2), then the cell of y'
// in [-2, 2]^3.  Every operation is one binary32 rounding, in this order.
__device__ __forceinline__ int32_t contracted_cell(const Lattice& p, const float x[3]) {
  float y[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) y[c] = (x[c] - p.center[c]) * p.inv_scale;
  const float r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  if (r2 > 1.0f) {
    const float r = sqrtf(r2);
    const float inv_r = 1.0f / r;
    const float f = (2.0f - inv_r) * inv_r;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c] = y[c] * f;
  }
  const float scale = p.resf * 0.25f;
  int cell[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    cell[c] = (int)__builtin_amdgcn_fmed3f(floorf((y[c] + 2.0f) * scale), 0.0f, p.resf - 1.0f);
  return cell[0] + p.res * (cell[1] + p.res * cell[2]);
}

template <bool kContract>
__device__ __forceinline__ bool probe(const Lattice& p, const float o[3], const float d[3],
                                      int32_t k, uint32_t& word, int32_t& sh) {
  const float m = p.a + ((float)k + 0.5f) * p.dt;
  const bool valid = (k >= 0) && (k < kLatticeLimit) && (m < p.b);
  word = 0u;
  sh = 0;
  if (valid) {
    int32_t idx;
    if (kContract) {
      float x[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c] = o[c] + m * d[c];
      idx = contracted_cell(p, x);
    } else {
      int cell[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float x = o[c] + m * d[c];
        const float u = (x - p.box.bmin[c]) * p.box.scale[c];
        // clamp of the floor to [0, res - 1] as one median-of-three (u is
        // never NaN here, so it equals min(max(floor(u), 0), res - 1))
        cell[c] = (int)__builtin_amdgcn_fmed3f(floorf(u), 0.0f, p.resf - 1.0f);
      }
      idx = cell[0] + p.res * (cell[1] + p.res * cell[2]);
    }
    word = p.bits[idx >> 5];
    sh = idx & 31;
  }
  return valid;
}

// One segment [a, b) on level l.  Each step tests kGroups groups of 64
// consecutive lattice points (one per lane), with all their grid-word loads in
// flight together, then emits the groups in k order.  n: samples so far
// (wave-uniform); returns the new count.  kSpan stops at the first occupied
// point, records its t0 in em.lo and returns a non-zero count.
constexpr int kGroups = 2;

template <int kMode, bool kContract>
__device__ __forceinline__ int32_t march_segment(const MarchArgs& g, const float o[3],
                                                 const float d[3], float a, float b, int l,
                                                 int32_t n, int32_t cap, Emit& em) {
  const Lattice p = lattice<kContract>(g, a, b, l);
  const int ln = lane();
  for (int32_t k0 = 0; k0 < kLatticeLimit; k0 += kWave * kGroups) {
    bool valid[kGroups], occ[kGroups];
    uint32_t word[kGroups];
    int32_t sh[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q)
      valid[q] = probe<kContract>(p, o, d, k0 + kWave * q + ln, word[q], sh[q]);
#pragma unroll
    for (int q = 0; q < kGroups; ++q) occ[q] = valid[q] && ((word[q] >> sh[q]) & 1u);
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      const int32_t k = k0 + kWave * q + ln;
      const uint64_t mask = __ballot(occ[q]);
      if (kMode == kSpan && mask != 0) {
        // the fill pass's binary32 t0 at the lowest occupied k
        const int32_t kf = k0 + kWave * q + (int32_t)__builtin_ctzll(mask);
        em.lo = a + (float)kf * p.dt;
        return n + __popcll(mask);
      }
      if (kMode == kFill && occ[q]) {
        const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const int64_t pos = em.base + n + rank;
        if ((cap == 0 || n + rank < cap) && n + rank < em.count && pos < em.capacity) {
          em.t0[pos] = a + (float)k * p.dt;
          em.t1[pos] = fminf(a + (float)(k + 1) * p.dt, b);
          if (em.ray_id) em.ray_id[pos] = em.ray;
        }
      }
      n += __popcll(mask);
      if (cap > 0 && n >= cap) return cap;
    }
    if (__ballot(valid[kGroups - 1]) != ~0ull) break;  // the segment ended in this step
  }
  return n;
}

// Last lattice point of segment [a, b): the largest k < kLatticeLimit with
// a + (k + 1/2) dt < b in binary32, or -1.  That midpoint is non-decreasing in
// k, so the segment's points are exactly k = 0 .. kmax (the forward pass
// visits the same set); the quotient estimate is off by a few units at most.
__device__ __forceinline__ int32_t last_lattice_point(float a, float b, float dt) {
  auto inside = [&](int32_t k) { return a + ((float)k + 0.5f) * dt < b; };
  const float e = floorf((b - a) / dt - 0.5f);
  int32_t k = !(e >= 0.0f) ? -1 : (e >= (float)(kLatticeLimit - 1) ? kLatticeLimit - 1 : (int32_t)e);
  while (k + 1 < kLatticeLimit && inside(k + 1)) ++k;
  while (k >= 0 && !inside(k)) --k;
  return k;
}

// Highest occupied lattice point of segment [a, b) on level l, scanning k
// downwards from the last point kGroups groups of 64 at a time; on success
// em.hi = the fill pass's binary32 t1 of that sample.
template <bool kContract>
__device__ __forceinline__ bool span_back(const MarchArgs& g, const float o[3], const float d[3],
                                          float a, float b, int l, Emit& em) {
  const Lattice p = lattice<kContract>(g, a, b, l);
  const int32_t kmax = last_lattice_point(a, b, p.dt);
  const int ln = lane();
  for (int32_t k0 = 0; k0 <= kmax; k0 += kWave * kGroups) {
    bool occ[kGroups];
    uint32_t word[kGroups];
    int32_t sh[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q)
      occ[q] = probe<kContract>(p, o, d, kmax - (k0 + kWave * q + ln), word[q], sh[q]);
#pragma unroll
    for (int q = 0; q < kGroups; ++q) occ[q] = occ[q] && ((word[q] >> sh[q]) & 1u);
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      const uint64_t mask = __ballot(occ[q]);
      if (mask != 0) {
        const int32_t kl = kmax - (k0 + kWave * q + (int32_t)__builtin_ctzll(mask));
        em.hi = fminf(a + (float)(kl + 1) * p.dt, b);
        return true;
      }
    }
  }
  return false;
}

template <int kMode, bool kContract>
__device__ __forceinline__ int32_t march_ray(const MarchArgs& g, const float o[3], const float d[3],
                                             Emit& em) {
  float inv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) inv[c] = 1.0f / d[c];
  const int L = g.n_levels;
  // lane l holds the chord of level l's cube
  const int ln = lane();
  float tn_l = INFINITY, tf_l = -INFINITY;
  if (ln < L) clip_box(o, inv, level_box(g, ln), g.near_plane, g.far_plane, tn_l, tf_l);
  // an inner cube's chord lies inside the next outer one: max / min over l' >= l
#pragma unroll
  for (int s = 1; s < kMaxLevels; s <<= 1) {
    const float a_n = shfl_down(tn_l, s), a_f = shfl_down(tf_l, s);
    if (ln + s < L) {
      tn_l = fmaxf(tn_l, a_n);
      tf_l = fminf(tf_l, a_f);
    }
  }
  const uint32_t hit = (uint32_t)__ballot(ln < L && tn_l < tf_l);
  auto tn = [&](int l) { return readlane(tn_l, l); };
  auto tf = [&](int l) { return readlane(tf_l, l); };

  // segment s in increasing t: descend from the outermost level, then ascend;
  // false if the ray does not cross it
  auto segment = [&](int s, int& l, float& a, float& b) {
    if (s < L) {
      l = L - 1 - s;
      if (!((hit >> l) & 1u)) return false;
      a = tn(l);
      b = (l > 0 && ((hit >> (l - 1)) & 1u)) ? tn(l - 1) : tf(l);
    } else {
      l = s - L + 1;
      if (!((hit >> l) & 1u) || !((hit >> (l - 1)) & 1u)) return false;
      a = tf(l - 1);
      b = tf(l);
    }
    return true;
  };

  const int32_t cap = g.max_per_ray;
  int32_t n = 0;
  int l;
  float a, b;
  if (kMode == kSpan) {
    // the first occupied point going forward, then the last one going back
    int s_first = -1;
    for (int s = 0; s < 2 * L - 1 && s_first < 0; ++s)
      if (segment(s, l, a, b) && march_segment<kSpan, kContract>(g, o, d, a, b, l, 0, 0, em) > 0)
        s_first = s;
    if (s_first < 0) return 0;
    for (int s = 2 * L - 2; s >= s_first; --s)
      if (segment(s, l, a, b) && span_back<kContract>(g, o, d, a, b, l, em)) break;
    return 1;
  }
  for (int s = 0; s < 2 * L - 1; ++s) {
    if (!segment(s, l, a, b)) continue;
    n = march_segment<kMode, kContract>(g, o, d, a, b, l, n, cap, em);
    if (cap > 0 && n >= cap) break;
  }
  return n;
}

template <int kMode, bool kContract>
__global__ __launch_bounds__(kBlock) void march_kernel(MarchArgs g, const float* __restrict__ ro,
                                                       const float* __restrict__ rd,
                                                       int32_t n_rays, int32_t* counts,
                                                       const int32_t* __restrict__ info,
                                                       int64_t capacity, float* t0, float* t1,
                                                       int32_t* ray_id, float* span) {
  // one ray per wave; the ray index is wave-uniform
  const int32_t r = __builtin_amdgcn_readfirstlane(
      (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave));
  if (r >= n_rays) return;
  float o[3], d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[c] = ro[3 * (int64_t)r + c];
    d[c] = rd[3 * (int64_t)r + c];
  }
  Emit em{t0, t1, ray_id, 0, 0, capacity, r, 0.0f, 0.0f};
  if (kMode == kFill) {
    const int2 row = reinterpret_cast<const int2*>(info)[r];
    em.base = row.x;
    em.count = (row.x < 0 || row.y < 0) ? 0 : row.y;  // malformed row: nothing written
  }
  const int32_t n = march_ray<kMode, kContract>(g, o, d, em);
  if (kMode == kCount && lane() == 0) counts[r] = n;
  if (kMode == kSpan && lane() == 0) {
    span[2 * (int64_t)r] = em.lo;
    span[2 * (int64_t)r + 1] = em.hi;
    counts[r] = n > 0 ? 1 : 0;
  }
}

txs_status make_args(const txs_grid* grid, const txs_march_params* p, MarchArgs& g) {
  TXS_REQUIRE(grid && p, "txs_march: null grid or params");
  TXS_REQUIRE(grid->bits, "txs_march: null grid bits");
  const int res = grid->res;
  TXS_REQUIRE(res >= 2 && res <= 1024 && (res & (res - 1)) == 0,
              "txs_march: res must be a power of two in [2,1024], got %d", res);
  TXS_REQUIRE(grid->n_levels >= 1 && grid->n_levels <= kMaxLevels,
              "txs_march: n_levels must be in [1,%d], got %d", kMaxLevels, grid->n_levels);
  TXS_REQUIRE(std::isfinite(grid->half_extent0) && grid->half_extent0 > 0.0f,
              "txs_march: half_extent0 must be finite and > 0");
  for (int c = 0; c < 3; ++c)
    TXS_REQUIRE(std::isfinite(grid->center[c]), "txs_march: grid center must be finite");
  TXS_REQUIRE(std::isfinite(p->dt0) && p->dt0 > 0.0f, "txs_march: dt0 must be finite and > 0");
  TXS_REQUIRE(std::isfinite(p->near_plane) && p->near_plane >= 0.0f,
              "txs_march: near_plane must be finite and >= 0");
  TXS_REQUIRE(!std::isnan(p->far_plane) && p->far_plane > p->near_plane,
              "txs_march: far_plane must exceed near_plane");
  TXS_REQUIRE(p->max_per_ray >= 0, "txs_march: max_per_ray must be >= 0");
  g.bits = grid->bits;
  g.res = res;
  g.n_levels = grid->n_levels;
  g.level_words = (int32_t)(((int64_t)res * res * res + 31) / 32);
  for (int c = 0; c < 3; ++c) g.center[c] = grid->center[c];
  g.half_extent0 = grid->half_extent0;
  g.near_plane = p->near_plane;
  g.far_plane = p->far_plane;
  g.dt0 = p->dt0;
  g.max_per_ray = p->max_per_ray;
  g.inv_scale = 0.0f;
  return TXS_OK;
}

unsigned march_blocks(int32_t n_rays) {
  return grid_1d(((int64_t)n_rays + kWavesPerBlock - 1) / kWavesPerBlock, 1);
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_march_count(const txs_grid* grid, const txs_march_params* params,
                                      const float* rays_o, const float* rays_d, int32_t n_rays,
                                      int32_t* counts, void* stream) {
  using namespace txs;
  clear_error();
  MarchArgs g;
  if (txs_status s = make_args(grid, params, g)) return s;
  TXS_REQUIRE(n_rays >= 0, "txs_march_count: n_rays < 0");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && counts, "txs_march_count: null array");
  hipLaunchKernelGGL((march_kernel<kCount, false>), dim3(march_blocks(n_rays)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, counts, nullptr, 0, nullptr,
                     nullptr, nullptr, nullptr);
  return launch_status("txs_march_count");
}

extern "C" txs_status txs_march_fill(const txs_grid* grid, const txs_march_params* params,
                                     const float* rays_o, const float* rays_d, int32_t n_rays,
                                     const int32_t* packed_info, int64_t capacity, float* t0,
                                     float* t1, int32_t* ray_id, void* stream) {
  using namespace txs;
  clear_error();
  MarchArgs g;
  if (txs_status s = make_args(grid, params, g)) return s;
  TXS_REQUIRE(n_rays >= 0 && capacity >= 0, "txs_march_fill: negative size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && packed_info, "txs_march_fill: null array");
  TXS_REQUIRE(capacity == 0 || (t0 && t1), "txs_march_fill: null output");
  hipLaunchKernelGGL((march_kernel<kFill, false>), dim3(march_blocks(n_rays)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, nullptr, packed_info, capacity,
                     t0, t1, ray_id, nullptr);
  return launch_status("txs_march_fill");
}

extern "C" txs_status txs_march_span(const txs_grid* grid, const txs_march_params* params,
                                     const float* rays_o, const float* rays_d, int32_t n_rays,
                                     float* span, int32_t* hit, void* stream) {
  using namespace txs;
  clear_error();
  MarchArgs g;
  if (txs_status s = make_args(grid, params, g)) return s;
  TXS_REQUIRE(g.max_per_ray == 0, "txs_march_span: max_per_ray must be 0");
  TXS_REQUIRE(n_rays >= 0, "txs_march_span: n_rays < 0");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && span && hit, "txs_march_span: null array");
  hipLaunchKernelGGL((march_kernel<kSpan, false>), dim3(march_blocks(n_rays)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, hit, nullptr, 0, nullptr,
                     nullptr, nullptr, span);
  return launch_status("txs_march_span");
}

extern "C" txs_status txs_march_count_contracted(const txs_grid* grid,
                                                 const txs_march_params* params,
                                                 float contract_scale, const float* rays_o,
                                                 const float* rays_d, int32_t n_rays,
                                                 int32_t* counts, void* stream) {
  using namespace txs;
  clear_error();
  MarchArgs g;
  if (txs_status s = make_args(grid, params, g)) return s;
  TXS_REQUIRE(std::isfinite(contract_scale) && contract_scale > 0.0f,
              "txs_march_count_contracted: contract_scale must be finite and > 0");
  g.inv_scale = 1.0f / contract_scale;
  TXS_REQUIRE(n_rays >= 0, "txs_march_count_contracted: n_rays < 0");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && counts, "txs_march_count_contracted: null array");
  hipLaunchKernelGGL((march_kernel<kCount, true>), dim3(march_blocks(n_rays)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, counts, nullptr, 0, nullptr,
                     nullptr, nullptr, nullptr);
  return launch_status("txs_march_count_contracted");
}

extern "C" txs_status txs_march_fill_contracted(const txs_grid* grid,
                                                const txs_march_params* params,
                                                float contract_scale, const float* rays_o,
                                                const float* rays_d, int32_t n_rays,
                                                const int32_t* packed_info, int64_t capacity,
                                                float* t0, float* t1, int32_t* ray_id,
                                                void* stream) {
  using namespace txs;
  clear_error();
  MarchArgs g;
  if (txs_status s = make_args(grid, params, g)) return s;
  TXS_REQUIRE(std::isfinite(contract_scale) && contract_scale > 0.0f,
              "txs_march_fill_contracted: contract_scale must be finite and > 0");
  g.inv_scale = 1.0f / contract_scale;
  TXS_REQUIRE(n_rays >= 0 && capacity >= 0, "txs_march_fill_contracted: negative size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && packed_info, "txs_march_fill_contracted: null array");
  TXS_REQUIRE(capacity == 0 || (t0 && t1), "txs_march_fill_contracted: null output");
  hipLaunchKernelGGL((march_kernel<kFill, true>), dim3(march_blocks(n_rays)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, nullptr, packed_info, capacity,
                     t0, t1, ray_id, nullptr);
  return launch_status("txs_march_fill_contracted");
}
