// Occupancy-grid ray marching (spatial-skipping estimator, Section 3.1 and
// Table 1 second row; cascaded levels for unbounded scenes, Section 3.2).
//
// One wave marches one ray: its 64 lanes test 64 lattice points at a time
// with the binary32 recipe of txs.h (contraction disabled in this file), a
// ballot collects the occupied ones and a lane-rank (mbcnt) packs them, so the
// fill pass writes each ray's samples as contiguous, coalesced runs.
//
// Empty-space skipping.  Given the grid's brick occupancy (8^3-cell bricks,
// staged in LDS per block), a segment is first walked in runs of kChunk
// lattice points, one run per lane: the cell coordinates of a run's points
// lie between those of its two end points (the recipe's u is monotone in the
// midpoint m up to its rounding, which a per-axis margin covers), so a run
// whose bounding bricks are all empty holds no occupied point.  The points of
// the remaining runs are then tested one by one, four runs per 64 lanes, in k
// order (or, when most runs of the window remain, the window's points in
// order without the run list).  Skipped points are exactly points that are
// not occupied, so the emitted samples are those of testing every lattice
// point.  Without brick occupancy (or over contracted space, where the path
// bends in cell space) every point is tested.
//
// A block of four waves marches 64 consecutive rays (16 per wave); a wave
// copies a level's brick occupancy into its LDS the first time it skips on
// that level (1 KiB for a 128^3 level).  Skipping is chosen per segment: on
// levels with at most 5/16 of their bricks occupied, for segments of more
// than a few hundred lattice points.
#pragma clang fp contract(off)

#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kMaxLevels = 8;
constexpr int32_t kLatticeLimit = 1 << 24;  // k stays exact in binary32
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
// rays per block: waves live for several rays, so that the launch of waves
// (a fixed cost per wave) does not bound the march of short rays
constexpr int kRaysPerBlock = 64;
constexpr int kChunk = 16;                  // lattice points per run of the skipping pass
constexpr int kDenseRuns = 48;              // more maybe-occupied runs of 63: test the window in order
constexpr int kBrickShift = 3;              // bricks of 8^3 cells
// brick occupancy a wave may hold in LDS (four 128^3 levels: 1028 words);
// with the run list, 8 blocks of 4 waves fit a CU's LDS
constexpr int kCoarseLdsWords = 1088;
constexpr int kListLen = kWave + 16;        // run list per wave, sentinel-padded
constexpr int kSentinelRun = 1 << 21;       // a run beyond every segment's last point

struct MarchArgs {
  const uint32_t* bits;
  int32_t res;
  int32_t res_shift;  // log2(res)
  int32_t n_levels;
  int32_t level_words;
  float center[3];
  float half_extent0;
  float near_plane, far_plane, dt0;
  int32_t max_per_ray;
  float inv_scale;  // contracted lookup: 1 / contract_scale
  // brick occupancy (skipping kernels only)
  const uint32_t* coarse;
  int32_t cshift;       // log2(bricks per axis)
  int32_t coarse_half;  // words of one of a level's two arrays
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
  int res, res_shift;
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
  p.res_shift = g.res_shift;
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
      uint32_t cell[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float x = o[c] + m * d[c];
        const float u = (x - p.box.bmin[c]) * p.box.scale[c];
        // clamp(floor(u), 0, res - 1) as the truncation of the clamped u: for
        // a u that is not NaN both give floor(u) inside [0, res - 1] and the
        // bound outside it (one median-of-three and one conversion)
        cell[c] = (uint32_t)__builtin_amdgcn_fmed3f(u, 0.0f, p.resf - 1.0f);
      }
      idx = (int32_t)(cell[0] | ((cell[1] | (cell[2] << p.res_shift)) << p.res_shift));
    }
    word = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(p.bits) +
                                              (((uint32_t)idx >> 3) & ~3u));
    sh = idx & 31;
  }
  return valid;
}

// Grid word of the lattice point with (float)k + 1/2 = kh on a cascade level
// (the recipe of probe()); bit = the cell's bit position in the word.  The
// clamp keeps the address inside the level's grid for any k, so the load
// needs no branch; the caller decides whether the point belongs to the
// segment.  The word's byte offset fits 32 bits: a scalar base and a 32-bit
// lane offset.
__device__ __forceinline__ uint32_t cell_word(const Lattice& p, const float o[3],
                                              const float d[3], float kh, uint32_t& bit,
                                              float& m) {
  m = p.a + kh * p.dt;
  uint32_t cell[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float x = o[c] + m * d[c];
    const float u = (x - p.box.bmin[c]) * p.box.scale[c];
    cell[c] = (uint32_t)__builtin_amdgcn_fmed3f(u, 0.0f, p.resf - 1.0f);
  }
  const uint32_t idx = cell[0] | ((cell[1] | (cell[2] << p.res_shift)) << p.res_shift);
  bit = idx & 31u;
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(p.bits) +
                                            ((idx >> 3) & ~3u));
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
  const float lane_h = (float)ln + 0.5f;
  // kLatticeLimit is a multiple of 64 kGroups, so every k of a step is below it
  static_assert(kLatticeLimit % (kWave * kGroups) == 0, "lattice limit");
  for (int32_t k0 = 0; k0 < kLatticeLimit; k0 += kWave * kGroups) {
    bool valid[kGroups], occ[kGroups];
    uint32_t word[kGroups];
    int32_t sh[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      if (kContract) {
        valid[q] = probe<kContract>(p, o, d, k0 + kWave * q + ln, word[q], sh[q]);
      } else {
        // (float)k + 1/2 as a scalar plus a lane constant: exact below 2^24
        const float kh = (float)(k0 + kWave * q) + lane_h;
        uint32_t bt;
        float m;
        word[q] = cell_word(p, o, d, kh, bt, m);
        sh[q] = (int32_t)bt;
        valid[q] = m < p.b;
      }
    }
#pragma unroll
    for (int q = 0; q < kGroups; ++q) occ[q] = valid[q] && ((word[q] >> sh[q]) & 1u);
    // every group's ballot before any early exit: the loads of all groups
    // then stay in flight together (a convergent ballot is not sunk into a
    // branch)
    uint64_t masks[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) masks[q] = __ballot(occ[q]);
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      const int32_t k = k0 + kWave * q + ln;
      const uint64_t mask = masks[q];
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

// Brick occupancy of one level as staged in LDS: the plain array, then the
// 2x2x2-block array.
struct Bricks {
  const uint32_t* plain;
  const uint32_t* block;
  int cshift;
};

// Skipping pays where the bricks are mostly empty; on a level with more than
// 5/16 of its bricks occupied the points are tested one by one (measured on
// MI355X, one 128^3 level, 2^20 camera rays: 44% occupied, skipping 5% slower
// than testing every point; 19% occupied, 13% faster)...
constexpr uint32_t kSkipNum = 5, kSkipDen = 16;
// ... and on segments long enough for the run pass to pay (a few hundred
// lattice points; the unbounded rig's short middle-level segments march
// faster point by point)
constexpr int kSkipMinPoints = 256;

// One segment [a, b) on level l with empty-space skipping (see the top of the
// file).  Pass 1: lane j < 63 bounds run c0 + j (lattice points
// [kChunk (c0 + j), kChunk (c0 + j + 1))) by the recipe's u at its first
// point and at the next run's first point (lane j + 1's); lane 63 only
// supplies that bound.  Every u of the run lies within 2 delta of the
// interval between the two, delta the rounding bound of one evaluation of the
// recipe, so the clamped floors of the widened interval bound the run's
// cells.  The run may hold an occupied point only if the brick of those
// bounds (one brick) or the 2x2x2 block starting at the lower brick (when the
// bounds span at most two bricks per axis) is occupied; wider bounds count as
// occupied.  Pass 2 tests the points of the maybe-occupied runs, four runs
// per 64 lanes, in k order, exactly as the dense march does; a window where
// more than kDenseRuns of its 63 runs remain is tested point by point in
// order instead.
template <int kMode>
__device__ __forceinline__ int32_t march_segment_skip(const MarchArgs& g, const Bricks& br,
                                                      int* list, const float o[3],
                                                      const float d[3], float a, float b, int l,
                                                      int32_t n, int32_t cap, Emit& em) {
  const Lattice p = lattice<false>(g, a, b, l);
  const int ln = lane();
  // The bounds need not follow the recipe, only enclose it.  With U(m) =
  // (o + m d - bmin) scale in exact arithmetic on the binary32 inputs and
  // u_r = 2^-24: the recipe's u at a point is within u_r scale (4|m d| + 3|o|
  // + 2|bmin|) 1.01 of U(m_k) (four roundings); the bound's u~ = fma(B, m, A)
  // with A = fl(fl(o - bmin) scale), B = fl(d scale), at the recipe's m of a
  // run's first point, is within u_r scale (3.02|m d| + 3.02(|o| + |bmin|))
  // of U(m).  U is monotone in m and m_k is non-decreasing in k, so every
  // point of a run lies within the sum of the two of the interval between
  // its first point's and the next run's u~.  marg = 2^-19 (scale (2 m_max|d|
  // + 2|o| + 2|bmin|) + res) exceeds that sum at least fivefold for any m of
  // this segment's runs.
  const float m_max = fmaxf(fabsf(a), fabsf(b) + (float)(kChunk + 2) * p.dt);
  float marg[3], A[3], B[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    marg[c] = 2.0f * 0x1p-20f *
              (p.box.scale[c] * (2.0f * m_max * fabsf(d[c]) + 2.0f * fabsf(o[c]) +
                                 2.0f * fabsf(p.box.bmin[c])) + p.resf);
    A[c] = (o[c] - p.box.bmin[c]) * p.box.scale[c];
    B[c] = d[c] * p.box.scale[c];
  }
  const int sh = br.cshift;
  constexpr uint64_t kRunLanes = ~0ull >> 1;  // lanes 0..62 own runs, lane 63 bounds
  // one step: two groups of 64 points, kq[q] the lane's point of group q
  // (valid when a point of the segment, below 2^24 and below k_end); their
  // grid-word loads stay in flight together.  Returns true when the ray is
  // done.
  auto step = [&](const int32_t (&kq)[kGroups], int32_t k_end) -> bool {
    bool valid[kGroups];
    uint32_t word[kGroups], bit[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      float m;
      word[q] = cell_word(p, o, d, (float)kq[q] + 0.5f, bit[q], m);
      valid[q] = kq[q] < k_end && m < b;
    }
    bool occs[kGroups];
    uint64_t masks[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      occs[q] = valid[q] && ((word[q] >> bit[q]) & 1u);
      masks[q] = __ballot(occs[q]);  // all ballots first: loads stay in flight together
    }
#pragma unroll
    for (int q = 0; q < kGroups; ++q) {
      const uint64_t mask = masks[q];
      if (kMode == kSpan && mask != 0) {
        const int32_t kf = readlane(kq[q], (int)__builtin_ctzll(mask));
        em.lo = a + (float)kf * p.dt;
        n += __popcll(mask);
        return true;
      }
      if (kMode == kFill && occs[q]) {
        const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const int64_t pos = em.base + n + rank;
        if ((cap == 0 || n + rank < cap) && n + rank < em.count && pos < em.capacity) {
          const float kf = (float)kq[q];
          em.t0[pos] = a + kf * p.dt;
          em.t1[pos] = fminf(a + (kf + 1.0f) * p.dt, b);
          if (em.ray_id) em.ray_id[pos] = em.ray;
        }
      }
      n += __popcll(mask);
      if (cap > 0 && n >= cap) {
        n = cap;
        return true;
      }
    }
    return false;
  };
  for (int32_t c0 = 0; c0 < kLatticeLimit / kChunk; c0 += kWave - 1) {
    const int32_t ks = kChunk * (c0 + ln);
    // the recipe's midpoint of the run's first point: the run holds points of
    // the segment iff it lies before b (midpoints grow with k)
    const float m0 = a + ((float)ks + 0.5f) * p.dt;
    const bool live = ks < kLatticeLimit && m0 < b;
    float u[3], un[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = __builtin_fmaf(B[c], m0, A[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) un[c] = dpp<kWaveShl1>(u[c], u[c]);  // lane + 1's u
    bool maybe = false;
    if (ln < kWave - 1 && live) {
      int lo[3], hi[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float u0 = fminf(u[c], un[c]) - marg[c], u1 = fmaxf(u[c], un[c]) + marg[c];
        lo[c] = (int)__builtin_amdgcn_fmed3f(u0, 0.0f, p.resf - 1.0f) >> kBrickShift;
        hi[c] = (int)__builtin_amdgcn_fmed3f(u1, 0.0f, p.resf - 1.0f) >> kBrickShift;
      }
      const int j = lo[0] | ((lo[1] | (lo[2] << sh)) << sh);
      const int w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
      if ((w0 | w1 | w2) == 0) maybe = (br.plain[j >> 5] >> (j & 31)) & 1u;
      else if (w0 <= 1 && w1 <= 1 && w2 <= 1) maybe = (br.block[j >> 5] >> (j & 31)) & 1u;
      else maybe = true;
    }
    const bool last_window = (__ballot(live) & kRunLanes) != kRunLanes;
    const uint64_t runs = __ballot(maybe);
    const int nr = __popcll(runs);
    if (nr > kDenseRuns) {
      // most runs of the window may hold samples: its points in order, as
      // the dense march does (no list)
      const int32_t k_end = kChunk * (c0 + kWave - 1);
      for (int32_t k0 = kChunk * c0; k0 < k_end; k0 += kWave * kGroups) {
        int32_t kq[kGroups];
#pragma unroll
        for (int q = 0; q < kGroups; ++q) kq[q] = k0 + kWave * q + ln;
        if (step(kq, k_end)) return n;
        if (__ballot(kq[kGroups - 1] < k_end && a + ((float)kq[kGroups - 1] + 0.5f) * p.dt < b) !=
            ~0ull)
          break;  // the segment ended in this step
      }
    } else if (nr > 0) {
      // the maybe-occupied runs in k order at list[0, nr), every other lane's
      // sentinel after them (entries kWave.. hold the sentinel already), so
      // the steps read the list without a branch
      const int rank = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(runs >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)runs, 0u));
      list[maybe ? rank : nr + ln - rank] = maybe ? c0 + ln : kSentinelRun;
      wave_sync();
      constexpr int kRunsPerGroup = kWave / kChunk;
      for (int i0 = 0; i0 < nr; i0 += kGroups * kRunsPerGroup) {
        int32_t kq[kGroups];
#pragma unroll
        for (int q = 0; q < kGroups; ++q)
          kq[q] = kChunk * list[i0 + kRunsPerGroup * q + ln / kChunk] + (ln % kChunk);
        if (step(kq, kLatticeLimit)) {
          wave_sync();
          return n;
        }
      }
      wave_sync();  // the list is rewritten by the next run window
    }
    if (last_window) break;
  }
  return n;
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

template <int kMode, bool kContract, bool kSkip>
__device__ __forceinline__ int32_t march_ray(const MarchArgs& g, uint32_t* coarse_lds,
                                             uint32_t& staged, int* list, const float o[3],
                                             const float d[3], Emit& em) {
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
  auto forward = [&](int l, float a, float b, int32_t n, int32_t cap) {
    if (kSkip) {
      const int lw = 2 * g.coarse_half + 1;
      const uint32_t occupied = g.coarse[l * lw + 2 * g.coarse_half];  // scalar load
      if (kSkipDen * occupied <= kSkipNum * (1u << (3 * g.cshift)) &&
          b - a > (float)kSkipMinPoints * (g.dt0 * (float)(1 << l))) {
        uint32_t* lv = coarse_lds + l * lw;
        if (!((staged >> l) & 1u)) {
          // first skip on this level: this wave copies its bricks into LDS
          for (int i = lane(); i < 2 * g.coarse_half; i += kWave) lv[i] = g.coarse[l * lw + i];
          wave_sync();
          staged |= 1u << l;
        }
        const Bricks br{lv, lv + g.coarse_half, g.cshift};
        return march_segment_skip<kMode>(g, br, list, o, d, a, b, l, n, cap, em);
      }
    }
    return march_segment<kMode, kContract>(g, o, d, a, b, l, n, cap, em);
  };

  const int32_t cap = g.max_per_ray;
  int32_t n = 0;
  int l;
  float a, b;
  if (kMode == kSpan) {
    // the first occupied point going forward, then the last one going back
    int s_first = -1;
    for (int s = 0; s < 2 * L - 1 && s_first < 0; ++s)
      if (segment(s, l, a, b) && forward(l, a, b, 0, 0) > 0) s_first = s;
    if (s_first < 0) return 0;
    for (int s = 2 * L - 2; s >= s_first; --s)
      if (segment(s, l, a, b) && span_back<kContract>(g, o, d, a, b, l, em)) break;
    return 1;
  }
  for (int s = 0; s < 2 * L - 1; ++s) {
    if (!segment(s, l, a, b)) continue;
    n = forward(l, a, b, n, cap);
    if (cap > 0 && n >= cap) break;
  }
  return n;
}

// Dynamic LDS of a march block: the brick occupancy of every level (skipping
// kernels), then one 64-entry run list per wave.
template <int kMode, bool kContract, bool kSkip>
__global__ __launch_bounds__(kBlock) void march_kernel(MarchArgs g, const float* __restrict__ ro,
                                                       const float* __restrict__ rd,
                                                       int32_t n_rays, int32_t* counts,
                                                       const int32_t* __restrict__ info,
                                                       int64_t capacity, float* t0, float* t1,
                                                       int32_t* ray_id, float* span) {
  extern __shared__ uint32_t lds[];
  // per wave: the brick occupancy of every level (copied on the first skip
  // on that level) and the run list
  const int coarse_words = kSkip ? g.n_levels * (2 * g.coarse_half + 1) : 0;
  const int w = threadIdx.x / kWave;
  uint32_t* coarse_lds = lds + (coarse_words + kListLen) * w;
  int* list = reinterpret_cast<int*>(coarse_lds + coarse_words);
  if (kSkip && lane() < kListLen - kWave) list[kWave + lane()] = kSentinelRun;
  uint32_t staged = 0u;  // levels whose bricks this wave holds (wave-uniform)
  // a block marches kRaysPerBlock consecutive rays, its waves taking every
  // kWavesPerBlock-th of them (neighbouring rays cost alike, so the waves
  // finish together); the next ray's origin and direction load while the
  // current one marches.  Ray indices are wave-uniform.
  const int64_t base = (int64_t)blockIdx.x * kRaysPerBlock;
  const int64_t end = min(base + kRaysPerBlock, (int64_t)n_rays);
  int64_t r64 = base + w;
  float on[3] = {0.0f, 0.0f, 0.0f}, dn[3] = {0.0f, 0.0f, 0.0f};
  if (r64 < end) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      on[c] = ro[3 * r64 + c];
      dn[c] = rd[3 * r64 + c];
    }
  }
  for (; r64 < end; r64 += kWavesPerBlock) {
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)r64);
    float o[3], d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o[c] = on[c];
      d[c] = dn[c];
    }
    const int64_t rn = r64 + kWavesPerBlock;
    if (rn < end) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        on[c] = ro[3 * rn + c];
        dn[c] = rd[3 * rn + c];
      }
    }
    Emit em{t0, t1, ray_id, 0, 0, capacity, r, 0.0f, 0.0f};
    if (kMode == kFill) {
      const int2 row = reinterpret_cast<const int2*>(info)[r];
      em.base = row.x;
      em.count = (row.x < 0 || row.y < 0) ? 0 : row.y;  // malformed row: nothing written
    }
    const int32_t n = march_ray<kMode, kContract, kSkip>(g, coarse_lds, staged, list, o, d, em);
    if (kMode == kCount && lane() == 0) counts[r] = n;
    if (kMode == kSpan && lane() == 0) {
      span[2 * (int64_t)r] = em.lo;
      span[2 * (int64_t)r + 1] = em.hi;
      counts[r] = n > 0 ? 1 : 0;
    }
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
  g.res_shift = __builtin_ctz((unsigned)res);
  g.n_levels = grid->n_levels;
  g.level_words = (int32_t)(((int64_t)res * res * res + 31) / 32);
  for (int c = 0; c < 3; ++c) g.center[c] = grid->center[c];
  g.half_extent0 = grid->half_extent0;
  g.near_plane = p->near_plane;
  g.far_plane = p->far_plane;
  g.dt0 = p->dt0;
  g.max_per_ray = p->max_per_ray;
  g.inv_scale = 0.0f;
  // brick occupancy: used when given, res >= 8 and small enough for LDS
  g.coarse = nullptr;
  g.cshift = 0;
  g.coarse_half = 0;
  const int64_t cw = txs_grid_coarse_words(res);
  if (grid->coarse && cw > 0 && cw * grid->n_levels <= kCoarseLdsWords) {
    g.coarse = grid->coarse;
    g.cshift = g.res_shift - kBrickShift;
    g.coarse_half = (int32_t)((cw - 1) / 2);
  }
  return TXS_OK;
}

unsigned march_blocks(int32_t n_rays) {
  return grid_1d(((int64_t)n_rays + kRaysPerBlock - 1) / kRaysPerBlock, 1);
}

// Launches one march kernel (skipping when the grid carries brick occupancy).
template <int kMode, bool kContract>
txs_status launch_march(const MarchArgs& g, void* stream, const float* ro, const float* rd,
                        int32_t n_rays, int32_t* counts, const int32_t* info, int64_t capacity,
                        float* t0, float* t1, int32_t* ray_id, float* span, const char* who) {
  const bool skip = !kContract && g.coarse != nullptr;
  const size_t lds = sizeof(uint32_t) * kWavesPerBlock *
                     ((skip ? g.n_levels * (2 * g.coarse_half + 1) : 0) + kListLen);
  if (skip)
    hipLaunchKernelGGL((march_kernel<kMode, kContract, !kContract>), dim3(march_blocks(n_rays)),
                       dim3(kBlock), lds, as_stream(stream), g, ro, rd, n_rays, counts, info,
                       capacity, t0, t1, ray_id, span);
  else
    hipLaunchKernelGGL((march_kernel<kMode, kContract, false>), dim3(march_blocks(n_rays)),
                       dim3(kBlock), lds, as_stream(stream), g, ro, rd, n_rays, counts, info,
                       capacity, t0, t1, ray_id, span);
  return launch_status(who);
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
  return launch_march<kCount, false>(g, stream, rays_o, rays_d, n_rays, counts, nullptr, 0,
                                     nullptr, nullptr, nullptr, nullptr, "txs_march_count");
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
  return launch_march<kFill, false>(g, stream, rays_o, rays_d, n_rays, nullptr, packed_info,
                                    capacity, t0, t1, ray_id, nullptr, "txs_march_fill");
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
  return launch_march<kSpan, false>(g, stream, rays_o, rays_d, n_rays, hit, nullptr, 0, nullptr,
                                    nullptr, nullptr, span, "txs_march_span");
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
  return launch_march<kCount, true>(g, stream, rays_o, rays_d, n_rays, counts, nullptr, 0,
                                    nullptr, nullptr, nullptr, nullptr,
                                    "txs_march_count_contracted");
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
  return launch_march<kFill, true>(g, stream, rays_o, rays_d, n_rays, nullptr, packed_info,
                                   capacity, t0, t1, ray_id, nullptr,
                                   "txs_march_fill_contracted");
}
