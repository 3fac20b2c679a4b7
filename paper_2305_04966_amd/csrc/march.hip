// Occupancy-grid ray marching (spatial-skipping estimator, Section 3.1 and
// Table 1 second row; cascaded levels for unbounded scenes, Section 3.2).
//
// One lane marches one ray.  The decision "sample k is kept" is the binary32
// recipe of txs.h evaluated with contraction disabled (this file), so the
// emitted samples equal those of a dense test of every lattice point.  Runs
// of lattice points that provably fall in the same cell are handled at once:
// skipped when the cell is empty, counted (count pass) or written (fill
// pass) when it is occupied.
#pragma clang fp contract(off)

#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kMaxLevels = 8;
constexpr int32_t kLatticeLimit = 1 << 24;  // k stays exact in binary32
constexpr int kBlock = 256;

struct MarchArgs {
  const uint32_t* bits;
  int32_t res;
  int32_t n_levels;
  int32_t level_words;
  float center[3];
  float half_extent0;
  float near_plane, far_plane, dt0;
  int32_t max_per_ray;
};

// Level-l box and grid scale, evaluated exactly as the recipe defines them.
struct LevelBox {
  float bmin[3], bmax[3], scale[3];
};

__host__ __device__ __forceinline__ LevelBox level_box(const MarchArgs& g, int l) {
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
__host__ __device__ __forceinline__ void clip_box(const float o[3], const float inv[3], const LevelBox& b,
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

template <int N>
__host__ __device__ __forceinline__ float pick(const float (&v)[N], int i) {
  float r = v[0];
#pragma unroll
  for (int j = 1; j < N; ++j) r = (i == j) ? v[j] : r;
  return r;
}

struct Emit {
  float* t0;
  float* t1;
  int32_t* ray_id;
  int64_t base;
  int64_t capacity;
  int32_t ray;
};

// Marches one segment [a, b) on level l; returns the updated sample count.
template <bool kFill>
__host__ __device__ int32_t march_segment(const MarchArgs& g, const float o[3], const float d[3], float a,
                                 float b, int l, int32_t n, int32_t cap, const Emit& em) {
  const float dt = g.dt0 * (float)(1 << l);
  const float inv_dt = 1.0f / dt;
  const LevelBox box = level_box(g, l);
  const int res = g.res;
  const float resf = (float)res;
  const uint32_t* bits = g.bits + (int64_t)l * g.level_words;

  // Linear map of the ray into grid units, u_c(t) = u0_c + t v_c, and a margin
  // dl_c (grid units) that bounds, with a wide factor, the rounding of the
  // binary32 recipe and of the run computation below.
  const float T = fmaxf(fabsf(a), fabsf(b)) + dt;
  float u0[3], v[3], iv[3], dl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u0[c] = (o[c] - box.bmin[c]) * box.scale[c];
    v[c] = d[c] * box.scale[c];
    iv[c] = 1.0f / v[c];
    dl[c] = 0x1p-16f * (box.scale[c] * (fabsf(o[c]) + fabsf(box.bmin[c]) + T * fabsf(d[c])) +
                        resf + 1.0f);
  }

  int32_t last_word = -1;
  uint32_t word_bits = 0;
  int32_t k = 0;
  while (k < kLatticeLimit) {
    const float m = a + ((float)k + 0.5f) * dt;
    if (!(m < b)) break;
    int cell[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float x = o[c] + m * d[c];
      const float u = (x - box.bmin[c]) * box.scale[c];
      float f = floorf(u);
      f = fminf(fmaxf(f, 0.0f), resf - 1.0f);
      cell[c] = (int)f;
    }
    const int32_t idx = cell[0] + res * (cell[1] + res * cell[2]);
    const int32_t word = idx >> 5;
    if (word != last_word) {
      word_bits = bits[word];
      last_word = word;
    }
    const bool occ = (word_bits >> (idx & 31)) & 1u;

    // Lattice points k+1 .. k_end-1 provably share this cell: their exact
    // positions lie inside the cell shrunk by dl on every face, where the
    // recipe's rounding cannot move them out.  Point k_end is re-tested.
    float tb = -INFINITY, te = b;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float lo = (cell[c] == 0) ? -INFINITY : (float)cell[c] + dl[c];
      const float hi = (cell[c] == res - 1) ? INFINITY : (float)(cell[c] + 1) - dl[c];
      float t_lo, t_hi;
      if (v[c] > 0.0f) {
        t_lo = (lo - u0[c]) * iv[c];
        t_hi = (hi - u0[c]) * iv[c];
      } else if (v[c] < 0.0f) {
        t_lo = (hi - u0[c]) * iv[c];
        t_hi = (lo - u0[c]) * iv[c];
      } else {
        const bool inside = (u0[c] >= lo) && (u0[c] <= hi);
        t_lo = inside ? -INFINITY : INFINITY;
        t_hi = inside ? INFINITY : -INFINITY;
      }
      tb = fmaxf(tb, t_lo);
      te = fminf(te, t_hi);
    }
    int32_t k_end = k + 1;
    const float m_next = a + ((float)(k + 1) + 0.5f) * dt;
    if (m_next >= tb && m_next < te) {
      const float q = (te - a) * inv_dt - 0.5f;  // ~ last lattice index inside
      const int32_t kq = (q >= (float)kLatticeLimit) ? kLatticeLimit : (int32_t)floorf(q);
      k_end = max(k_end, kq);
    }

    if (occ) {
      int32_t run = k_end - k;
      if (cap > 0) run = min(run, cap - n);
      if (kFill) {
        for (int32_t j = 0; j < run; ++j) {
          const int64_t pos = em.base + n + j;
          if (pos < em.capacity) {
            const int32_t kk = k + j;
            em.t0[pos] = a + (float)kk * dt;
            em.t1[pos] = fminf(a + (float)(kk + 1) * dt, b);
            if (em.ray_id) em.ray_id[pos] = em.ray;
          }
        }
      }
      n += run;
      if (cap > 0 && n >= cap) return n;
    }
    k = k_end;
  }
  return n;
}

template <bool kFill>
__host__ __device__ int32_t march_ray(const MarchArgs& g, const float o[3], const float d[3],
                             const Emit& em) {
  float inv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) inv[c] = 1.0f / d[c];
  const int L = g.n_levels;
  float tn[kMaxLevels], tf[kMaxLevels];
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    tn[l] = INFINITY;
    tf[l] = -INFINITY;
    if (l < L) clip_box(o, inv, level_box(g, l), g.near_plane, g.far_plane, tn[l], tf[l]);
  }
  // an inner cube's chord lies inside the next outer one
#pragma unroll
  for (int l = kMaxLevels - 2; l >= 0; --l) {
    if (l + 1 < L) {
      tn[l] = fmaxf(tn[l], tn[l + 1]);
      tf[l] = fminf(tf[l], tf[l + 1]);
    }
  }
  uint32_t hit = 0;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l)
    if (l < L && tn[l] < tf[l]) hit |= 1u << l;

  const int32_t cap = g.max_per_ray;
  int32_t n = 0;
  // segments in increasing t: descend from the outermost level, then ascend
  for (int s = 0; s < 2 * L - 1; ++s) {
    int l;
    float a, b;
    if (s < L) {
      l = L - 1 - s;
      if (!((hit >> l) & 1u)) continue;
      a = pick(tn, l);
      b = (l > 0 && ((hit >> (l - 1)) & 1u)) ? pick(tn, l - 1) : pick(tf, l);
    } else {
      l = s - L + 1;
      if (!((hit >> l) & 1u) || !((hit >> (l - 1)) & 1u)) continue;
      a = pick(tf, l - 1);
      b = pick(tf, l);
    }
    n = march_segment<kFill>(g, o, d, a, b, l, n, cap, em);
    if (cap > 0 && n >= cap) break;
  }
  return n;
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void march_kernel(MarchArgs g, const float* __restrict__ ro,
                                                       const float* __restrict__ rd,
                                                       int32_t n_rays, int32_t* counts,
                                                       const int32_t* __restrict__ info,
                                                       int64_t capacity, float* t0, float* t1,
                                                       int32_t* ray_id) {
  const int32_t r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= n_rays) return;
  float o[3], d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[c] = ro[3 * (int64_t)r + c];
    d[c] = rd[3 * (int64_t)r + c];
  }
  Emit em{t0, t1, ray_id, kFill ? (int64_t)info[2 * (int64_t)r] : 0, capacity, r};
  const int32_t n = march_ray<kFill>(g, o, d, em);
  if (!kFill) counts[r] = n;
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
  return TXS_OK;
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
  hipLaunchKernelGGL(march_kernel<false>, dim3(grid_1d(n_rays, kBlock)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, counts, nullptr, 0, nullptr,
                     nullptr, nullptr);
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
  hipLaunchKernelGGL(march_kernel<true>, dim3(grid_1d(n_rays, kBlock)), dim3(kBlock), 0,
                     as_stream(stream), g, rays_o, rays_d, n_rays, nullptr, packed_info, capacity,
                     t0, t1, ray_id);
  return launch_status("txs_march_fill");
}
