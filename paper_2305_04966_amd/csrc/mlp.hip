// Proposal network of the learned transmittance estimator (Section 3.1 "PDF
// Approaches", Table 1 third row; Section 3.2 "Choice of Representations"):
// x -> Fourier features -> H ReLU -> H ReLU -> 1 -> softplus, evaluated at the
// midpoints of each ray's bins, on the bf16 matrix cores with fp32 accumulation.
//
// MFMA formulation (v_mfma_f32_16x16x32_bf16, wave64).  Every layer computes
// its output transposed: rows = hidden units (M), columns = 16 points (N),
// K = input units.  In that form the 16x16 fp32 fragment a lane holds after a
// layer (one point column, four consecutive unit rows per 16-lane group) is,
// once rounded to bf16, exactly the lane's share of the next layer's B operand,
// provided the next layer's K order is the matching permutation of its input
// units; that permutation is applied once, when the weights are packed into
// operand tiles (txs_mlp_pack), so no activation moves between lanes.  The
// three 16-lane groups g = 0,1,2 each encode the 13 features of axis g.
#include <cmath>

#include "txs_common.h"

namespace txs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kNF = 39;  // x_hat (3) + 3 axes x 6 octaves x (sin, cos)

// ---------------------------------------------------------------- layout
// Parameter vector: W1 [H,39], b1 [H], W2 [H,H], b2 [H], w3 [H], b3.
struct ParamOffsets {
  int64_t W1, b1, W2, b2, w3, b3, total;
  __host__ __device__ explicit ParamOffsets(int H)
      : W1(0), b1(39 * H), W2(40 * H), b2(40 * H + (int64_t)H * H), w3(41 * H + (int64_t)H * H),
        b3(42 * H + (int64_t)H * H), total(42 * H + (int64_t)H * H + 1) {}
};

// Packed operand tiles (bf16), each tile = 64 lanes x 8 values:
//   A1[m][s]  layer 1 (W1; b1 in the constant-1 slots), m < H/16, s < 2
//   A2[m][s]  layer 2 (W2), s < H/32
//   A2t[T][s] W2^T for the adjoint, B operand: K = layer-2 units in the order
//             of K-step s, N = layer-1 units in the order of point-major tile T
//   w3 (H values, unit order)
struct PackOffsets {
  int64_t A1, A2, A2t, w3, total;  // in bf16 elements
  __host__ __device__ explicit PackOffsets(int H)
      : A1(0), A2((int64_t)(H / 16) * 2 * 512), A2t(A2 + (int64_t)(H / 16) * (H / 32) * 512),
        w3(A2t + (int64_t)(H / 16) * (H / 32) * 512), total(w3 + H) {}
};

// Feature slot q (0..15) of lane group g: q < 12 -> sin/cos of octave q/2 of
// axis g, q = 12 -> x_hat_g; slots 13..15 of group 0 hold the constant 1 that
// carries the layer-1 bias, the rest are zero.  Canonical feature index or -1.
__host__ __device__ inline int feature_of(int g, int q) {
  if (g > 2) return -1;
  if (q < 12) return 3 + 12 * g + q;
  return q == 12 ? g : -1;
}

// K position i (0..7) of K-step s for lane group g of a layer whose input is a
// previous layer's fragments: input unit 16 (2s + i/4) + 4g + i%4.
__host__ __device__ inline int unit_of(int s, int g, int i) {
  return 16 * (2 * s + i / 4) + 4 * g + (i % 4);
}

// Unit in column n of point-major tile T: the transpose of K-step T/2 of a
// unit-major fragment, half T%2 of its K range.
__host__ __device__ inline int pm_unit(int T, int n) {
  return unit_of(T / 2, 2 * (T % 2) + n / 8, n % 8);
}

// Canonical feature (or -1) in column n of point-major feature tile F:
// F = 0: axes 0,1 slots 0..7; F = 1: axes 0,1 slots 8..15; F = 2: axis 2.
__host__ __device__ inline int pm_feature(int F, int n) {
  return F == 2 ? feature_of(2, n) : feature_of(n / 8, 8 * F + n % 8);
}

__global__ void pack_kernel(const float* __restrict__ p, int H, __bf16* __restrict__ out) {
  const ParamOffsets po(H);
  const PackOffsets ko(H);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ko.total) return;
  float v = 0.0f;
  if (e < ko.A2) {  // A1[m][s][lane][i]
    const int64_t t = e / 512, r = e % 512;
    const int m = (int)(t / 2), s = (int)(t % 2), l = (int)(r / 8), i = (int)(r % 8);
    const int q = 8 * s + i, f = feature_of(l / 16, q);
    const int row = 16 * m + l % 16;
    if (f >= 0) {
      v = p[po.W1 + (int64_t)row * kNF + f];
    } else if (l / 16 == 0 && q >= 13) {
      // b1 as three bf16 pieces (hi + mid + lo = b1 to binary32 precision),
      // multiplied by the constant-1 feature slots 13..15 of lane group 0
      const float b = p[po.b1 + row];
      const float hi = (float)(__bf16)b, mid = (float)(__bf16)(b - hi);
      v = q == 13 ? hi : q == 14 ? mid : (b - hi) - mid;
    }
  } else if (e < ko.A2t) {  // A2[m][s][lane][i] = W2[out][in]
    const int64_t t = (e - ko.A2) / 512, r = (e - ko.A2) % 512;
    const int m = (int)(t / (H / 32)), s = (int)(t % (H / 32)), l = (int)(r / 8), i = (int)(r % 8);
    v = p[po.W2 + (int64_t)(16 * m + l % 16) * H + unit_of(s, l / 16, i)];
  } else if (e < ko.w3) {  // A2t[T][s][lane][i] = W2[out = K order of s][in = pm_unit(T, n)]
    const int64_t t = (e - ko.A2t) / 512, r = (e - ko.A2t) % 512;
    const int T = (int)(t / (H / 32)), s = (int)(t % (H / 32)), l = (int)(r / 8), i = (int)(r % 8);
    v = p[po.W2 + (int64_t)unit_of(s, l / 16, i) * H + pm_unit(T, l % 16)];
  } else {  // w3 in unit order
    v = p[po.w3 + (e - ko.w3)];
  }
  out[e] = (__bf16)v;
}

// ---------------------------------------------------------------- forward
struct FwdArgs {
  const __bf16* packed;
  const float* params;
  float inv_scale;  // 1 / scale
  int32_t contract;
  const float* ro;
  const float* rd;
  int32_t n_rays, n_bins;
  FastDiv bins_div;   // division by n_bins
  int32_t small;      // n_rays * n_bins < 2^32: point -> ray by FastDiv
  const float* edges;
  float* sigma;
};

__device__ __forceinline__ bf16x8 pack8(const float (&v)[8]) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];
  return r;
}

// softplus(z) = log(1 + e^z): e = 2^(z log2 e) by the hardware exp2; for
// e < 1/16 the series e (1 - e/2 + e^2/3 - e^3/4 + e^4/5) (truncation < 2e-7
// relative), else log2(1 + e) ln 2 (rounding of 1 + e costs < 1e-6 relative).
// bf16 of relu(v), eight at a time.  Round-to-nearest-even keeps the sign, so
// relu after rounding equals rounding after relu; on the packed halves it is
// one arithmetic shift (sign -> all-ones mask) and one masked clear per pair,
// where fmaxf costs a NaN-quieting max plus the max per value.
__device__ __forceinline__ bf16x8 pack8_relu(const float (&v)[8]) {
  typedef unsigned uint4v __attribute__((ext_vector_type(4)));
  uint4v w = __builtin_bit_cast(uint4v, pack8(v));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // as signed 16-bit integers, bf16 values with the sign bit set are negative
    unsigned r;
    asm("v_pk_max_i16 %0, %1, 0" : "=v"(r) : "v"(w[q]));
    w[q] = r;
  }
  return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ float softplus(float z) {
  if (z > 20.0f) return z;
  const float e = __builtin_amdgcn_exp2f(z * 1.44269504f);
  if (e < 0.0625f)
    return e * (1.0f - e * (0.5f - e * (1.0f / 3.0f - e * (0.25f - e * 0.2f))));
  return __builtin_amdgcn_logf(1.0f + e) * 0.693147181f;
}

// Raw inputs of one point (its bin's edges, its ray's origin and direction),
// loaded apart from their use so that a kernel can fetch them a step ahead.
struct PointIn {
  float e0, e1, o[3], d[3];
};

template <class Args>
__device__ __forceinline__ PointIn load_point(const Args& a, int64_t p) {
  int64_t r;
  if (a.small) r = a.bins_div.div((uint32_t)p);
  else r = p / a.n_bins;
  const int64_t j = p - r * a.n_bins;
  const float* e = a.edges + r * (a.n_bins + 1) + j;
  PointIn in;
  in.e0 = e[0];
  in.e1 = e[1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    in.o[c] = a.ro[3 * r + c];
    in.d[c] = a.rd[3 * r + c];
  }
  return in;
}

// x_hat of a bin midpoint: x / scale, optionally contracted into the unit ball
template <class Args>
__device__ __forceinline__ void encode_loaded(const Args& a, const PointIn& in, float (&y)[3]) {
  const float tm = 0.5f * (in.e0 + in.e1);
#pragma unroll
  for (int c = 0; c < 3; ++c) y[c] = (in.o[c] + tm * in.d[c]) * a.inv_scale;
  if (a.contract) {
    const float n = sqrtf(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const float rn = 1.0f / n;
    const float f = n <= 1.0f ? 0.5f : 0.5f * (2.0f - rn) * rn;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c] *= f;
  }
}

// Lane group g's 16 feature slots of a point, as the two K-steps of layer 1.
// Octave 0 from the hardware sine (argument in revolutions: sin(pi x) at x/2,
// cos at x/2 + 1/4); each further octave by the double-angle identities
// sin 2a = 2 sin a cos a, cos 2a = 1 - 2 sin^2 a (absolute error grows about
// 2x per octave: ~1e-6 at octave 5, far below a bf16 step).
__device__ __forceinline__ void features(float xa, int g, bf16x8& b0, bf16x8& b1) {
  float f[16];
  float sn = __builtin_amdgcn_sinf(0.5f * xa);
  float cs = __builtin_amdgcn_sinf(0.5f * xa + 0.25f);
  f[0] = sn;
  f[1] = cs;
#pragma unroll
  for (int k = 1; k < 6; ++k) {
    const float s2 = 2.0f * sn * cs;
    const float c2 = 1.0f - 2.0f * sn * sn;
    sn = s2;
    cs = c2;
    f[2 * k] = sn;
    f[2 * k + 1] = cs;
  }
  f[12] = xa;
  f[13] = f[14] = f[15] = g == 0 ? 1.0f : 0.0f;
  float lo[8], hi[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    lo[i] = f[i];
    hi[i] = f[8 + i];
  }
  b0 = pack8(lo);
  b1 = pack8(hi);
}

// Layer 3 (w3 . h2) also runs on the matrix cores: an A operand whose row 0
// is w3 (in the K order of the h2 fragments) and whose other rows are zero,
// times the bf16 h2 fragments as B, accumulates z in row 0 of a 16x16 tile
// (lanes 0..15, element 0), one point per column.
// kThreads = 512 (eight waves sharing one LDS copy of the weights) for the
// hidden-128 network: its 54 KB of weights allow three 256-thread blocks per
// CU (three waves per SIMD); two 512-thread blocks at the 128 registers of a
// four-wave target give four.
template <int H, int NT, int kThreads = 256>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kThreads == 512 ? 4 : 1))) void mlp_fwd_kernel(FwdArgs a) {
  constexpr int MT = H / 16, KS = H / 32;
  const PackOffsets ko(H);
  const ParamOffsets po(H);
  __shared__ bf16x8 sA1[MT * 2 * 64];
  __shared__ bf16x8 sA2[MT * KS * 64];
  __shared__ bf16x8 sA3[KS * 64];
  __shared__ float sb1[H], sb2[H];
  // per wave: the encoded coordinates of its NT * 16 points, axis-major
  __shared__ float sY[kThreads / kWave][3][kWave];
  // weights to LDS once per block
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(a.packed);
    for (int i = threadIdx.x; i < MT * 2 * 64; i += blockDim.x) sA1[i] = src[i];
    const bf16x8* src2 = reinterpret_cast<const bf16x8*>(a.packed + ko.A2);
    for (int i = threadIdx.x; i < MT * KS * 64; i += blockDim.x) sA2[i] = src2[i];
    for (int i = threadIdx.x; i < KS * 64; i += blockDim.x) {
      const int s3 = i / 64, l = i % 64;
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        v[e] = (l % 16 == 0) ? a.packed[ko.w3 + unit_of(s3, l / 16, e)] : (__bf16)0.0f;
      sA3[i] = v;
    }
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      sb1[i] = a.params[po.b1 + i];
      sb2[i] = a.params[po.b2 + i];
    }
    __syncthreads();
  }
  const float b3 = a.params[po.b3];
  const int ln = lane(), g = ln >> 4, col = ln & 15;
  const int64_t n_points = (int64_t)a.n_rays * a.n_bins;
  const int64_t n_tiles = (n_points + 15) / 16;
  const int wv = threadIdx.x / kWave;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  // A group of NT tiles holds NT * 16 <= 64 points: lane l loads and encodes
  // point l of the group (once, where the lanes of a tile column would each
  // repeat it), fetched one group ahead; the coordinates reach the lanes
  // that form the features through LDS.
  static_assert(NT * 16 <= kWave, "one point per lane");
  const bool loads = ln < NT * 16;
  PointIn in{};
  {
    const int64_t p = wave * NT * 16 + ln;
    if (loads && p < n_points) in = load_point(a, p);
  }
  for (int64_t t0 = wave * NT; t0 < n_tiles; t0 += n_waves * NT) {
    if (loads) {
      float y[3] = {0.0f, 0.0f, 0.0f};
      if (t0 * 16 + ln < n_points) encode_loaded(a, in, y);
#pragma unroll
      for (int c = 0; c < 3; ++c) sY[wv][c][ln] = y[c];
      const int64_t pn = (t0 + n_waves * NT) * 16 + ln;
      if (pn < n_points) in = load_point(a, pn);
    }
    wave_sync();
    bf16x8 B1[NT][2];
    bool valid[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t p = (t0 + t) * 16 + col;
      valid[t] = p < n_points;
      const float xa = sY[wv][g < 2 ? g : 2][16 * t + col];
      features(xa, g, B1[t][0], B1[t][1]);
    }
    wave_sync();  // the slots are rewritten by the next group
    // layer 1; B operand of layer 2's K-step s = fragments 2s and 2s+1
    bf16x8 B2[NT][KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      f32x4 hh[NT][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * s + h;
        const bf16x8 w0 = sA1[(m * 2 + 0) * 64 + ln], w1 = sA1[(m * 2 + 1) * 64 + ln];
        const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};  // b1 arrives through K
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, B1[t][0], zero, 0, 0, 0);
          hh[t][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, B1[t][1], c, 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float v[8] = {hh[t][0][0], hh[t][0][1], hh[t][0][2], hh[t][0][3],
                            hh[t][1][0], hh[t][1][1], hh[t][1][2], hh[t][1][3]};
        B2[t][s] = pack8_relu(v);
      }
    }
    // layers 2 and 3: two row tiles of h2 at a time make one K-step of layer 3
    f32x4 zt[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) zt[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int s3 = 0; s3 < KS; ++s3) {
      f32x4 c[NT][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * s3 + h;
        const f32x4 bias = {sb2[16 * m + 4 * g], sb2[16 * m + 4 * g + 1], sb2[16 * m + 4 * g + 2],
                            sb2[16 * m + 4 * g + 3]};
#pragma unroll
        for (int t = 0; t < NT; ++t) c[t][h] = bias;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const bf16x8 w = sA2[(m * KS + s) * 64 + ln];
#pragma unroll
          for (int t = 0; t < NT; ++t)
            c[t][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, B2[t][s], c[t][h], 0, 0, 0);
        }
      }
      const bf16x8 w3 = sA3[s3 * 64 + ln];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float v[8] = {c[t][0][0], c[t][0][1], c[t][0][2], c[t][0][3],
                            c[t][1][0], c[t][1][1], c[t][1][2], c[t][1][3]};
        zt[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, pack8_relu(v), zt[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t p = (t0 + t) * 16 + col;
      if (g == 0 && valid[t]) a.sigma[p] = softplus(zt[t][0] + b3);
    }
  }
}

// ---------------------------------------------------------------- adjoint
// Gradient of sum_p d_sigma[p] sigma(x_p) w.r.t. the parameters.  Rounding
// points: gamma, h1, h2, the weights, and the adjoints d2 = dL/da2 and
// d1 = dL/da1 are bf16 (matrix-core operands); every sum is fp32.
//
// Two orientations of a 16x16 tile.  Unit-major: a lane holds 8 units of one
// point (the layout the forward layers consume as K).  Point-major: a lane
// holds 8 points of one unit -- 4 from each of two 16-point tiles -- which is
// the operand layout of the weight gradients, whose K runs over points.  An
// MFMA's A and B operands share one lane layout, so a unit-major fragment fed
// as A against a 0/1 selector B comes out of the accumulator point-major,
// exactly (one nonzero product per output); this transposes h1, d2 and gamma
// on the matrix cores.  d1 is produced point-major directly, with d2 as the A
// operand and W2^T tiles as B (their N order matching the transposed h1).
//
// Each wave takes 32 points (one chunk) per iteration and keeps its own fp32
// dW2 tiles for the whole launch (H^2/64 values per lane: the accumulation
// registers).  dW1 is shared out instead: each wave writes its chunk's d1 and
// gamma fragments to an LDS slot, and wave w accumulates dW1's row tiles
// [w H/64, (w+1) H/64) over the four slots, in slot order, one iteration
// later.  At the end the block's waves add their dW2 tiles in LDS in a fixed
// order and the block writes one partial; a second kernel sums the blocks in
// index order (deterministic, no float atomics).
constexpr int kBwdWaves = 4;  // waves per block

__host__ __device__ inline int bwd_blocks(int H) { return H == 64 ? 512 : 256; }

struct BwdArgs {
  const __bf16* packed;
  const float* params;
  float inv_scale;  // 1 / scale
  int32_t contract;
  const float* ro;
  const float* rd;
  int32_t n_rays, n_bins;
  FastDiv bins_div;   // division by n_bins
  int32_t small;      // n_rays * n_bins < 2^32: point -> ray by FastDiv
  const float* edges;
  const float* d_sigma;
  float* partial;  // [gridDim.x][param count]
};

__device__ __forceinline__ bf16x8 pack_pair(const f32x4& x, const f32x4& y) {
  const float v[8] = {x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
  return pack8(v);
}

// x where the matching value of m (a relu output, never negative) is
// positive, else +0; both eight bf16 wide.  Per 16-bit half: min(m, 1) is 1
// or 0 and multiplies x's bits.
__device__ __forceinline__ bf16x8 mask_positive(bf16x8 x, bf16x8 m) {
  typedef unsigned uint4v __attribute__((ext_vector_type(4)));
  const uint4v xv = __builtin_bit_cast(uint4v, x), mv = __builtin_bit_cast(uint4v, m);
  uint4v r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    unsigned one;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(one) : "v"(mv[q]), "s"(0x00010001u));
    asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(r[q]) : "v"(xv[q]), "v"(one));
  }
  return __builtin_bit_cast(bf16x8, r);
}

// acc[q] += a b[q] (q < N) with acc held in the accumulation registers.  The
// compiler places an MFMA's accumulator in one register file for the whole
// kernel; written out here, dW2's N^2/4 x 64 values sit in AGPRs while the
// other products keep their results in VGPRs for the VALU work that follows.
// Being opaque to the hazard checks, the block pads itself: 4 wait states for
// VALU writes of a and b before it, 8 for its own operand reads after it.
template <int N>
__device__ __forceinline__ void mfma_agpr_row(f32x4 (&acc)[N], const bf16x8& a,
                                              const bf16x8 (&b)[N]);
template <>
__device__ __forceinline__ void mfma_agpr_row<8>(f32x4 (&acc)[8], const bf16x8& a,
                                                 const bf16x8 (&b)[8]) {
  asm volatile(
      "s_nop 3\n\t"
      "v_mfma_f32_16x16x32_bf16 %0, %8, %9, %0\n\t"
      "v_mfma_f32_16x16x32_bf16 %1, %8, %10, %1\n\t"
      "v_mfma_f32_16x16x32_bf16 %2, %8, %11, %2\n\t"
      "v_mfma_f32_16x16x32_bf16 %3, %8, %12, %3\n\t"
      "v_mfma_f32_16x16x32_bf16 %4, %8, %13, %4\n\t"
      "v_mfma_f32_16x16x32_bf16 %5, %8, %14, %5\n\t"
      "v_mfma_f32_16x16x32_bf16 %6, %8, %15, %6\n\t"
      "v_mfma_f32_16x16x32_bf16 %7, %8, %16, %7\n\t"
      "s_nop 7"
      : "+a"(acc[0]), "+a"(acc[1]), "+a"(acc[2]), "+a"(acc[3]), "+a"(acc[4]), "+a"(acc[5]),
        "+a"(acc[6]), "+a"(acc[7])
      : "v"(a), "v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(b[3]), "v"(b[4]), "v"(b[5]), "v"(b[6]),
        "v"(b[7]));
}
template <>
__device__ __forceinline__ void mfma_agpr_row<4>(f32x4 (&acc)[4], const bf16x8& a,
                                                 const bf16x8 (&b)[4]) {
  asm volatile(
      "s_nop 3\n\t"
      "v_mfma_f32_16x16x32_bf16 %0, %4, %5, %0\n\t"
      "v_mfma_f32_16x16x32_bf16 %1, %4, %6, %1\n\t"
      "v_mfma_f32_16x16x32_bf16 %2, %4, %7, %2\n\t"
      "v_mfma_f32_16x16x32_bf16 %3, %4, %8, %3\n\t"
      "s_nop 7"
      : "+a"(acc[0]), "+a"(acc[1]), "+a"(acc[2]), "+a"(acc[3])
      : "v"(a), "v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(b[3]));
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int H>
__global__ __launch_bounds__(kBwdWaves * kWave)
__attribute__((amdgpu_waves_per_eu(H == 64 ? 2 : 1, H == 64 ? 2 : 1)))
void mlp_bwd_kernel(BwdArgs a) {
  constexpr int MT = H / 16, KS = H / 32;
  const PackOffsets ko(H);
  const ParamOffsets po(H);
  // operand tiles and the d1 / gamma exchange slots, then (after the loop)
  // the block's reduction buffer
  constexpr int kTiles = MT * 2 + 2 * MT * KS + KS + 4;
  constexpr int kSlot = MT + 3;  // fragments per wave: d1 row tiles, gamma tiles
  constexpr int RT = MT / kBwdWaves;  // dW1 row tiles owned by each wave
  constexpr int kBytes = (kTiles + kBwdWaves * kSlot) * 64 * 16 + 2 * H * 4;
  static_assert(kBwdWaves * 16 * H * 4 <= kTiles * 64 * 16, "reduction buffer");
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  bf16x8* sA1 = reinterpret_cast<bf16x8*>(smem);  // layer 1, A operand
  bf16x8* sA2 = sA1 + MT * 2 * 64;                 // layer 2, A operand
  bf16x8* sA2t = sA2 + MT * KS * 64;               // W2^T, B operand of d1
  bf16x8* sA3 = sA2t + MT * KS * 64;               // w3 in row 0
  bf16x8* sSel = sA3 + KS * 64;                    // 0/1 selectors
  float* sb2 = reinterpret_cast<float*>(sSel + 4 * 64);
  float* sw3 = sb2 + H;  // w3 at unit_of(s, g, j), as [s][g][j]
  bf16x8* sX = reinterpret_cast<bf16x8*>(sw3 + H);  // [wave][kSlot][64]
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(a.packed);
    for (int i = threadIdx.x; i < MT * 2 * 64; i += blockDim.x) sA1[i] = src[i];
    const bf16x8* src2 = reinterpret_cast<const bf16x8*>(a.packed + ko.A2);
    for (int i = threadIdx.x; i < 2 * MT * KS * 64; i += blockDim.x) sA2[i] = src2[i];
    for (int i = threadIdx.x; i < KS * 64; i += blockDim.x) {
      const int s3 = i / 64, l = i % 64;
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        v[e] = (l % 16 == 0) ? a.packed[ko.w3 + unit_of(s3, l / 16, e)] : (__bf16)0.0f;
      sA3[i] = v;
    }
    // selector k of lane (n, g), element j: B[8g + j][n] = 1 where
    //   k = 0: 8g + j == n        (K rows 0..15)
    //   k = 1: 8g + j == 16 + n   (K rows 16..31)
    //   k = 2: n < 8 and 8g + j == 16 + n
    //   k = 3: n >= 8 and 8g + j == 8 + n
    for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
      const int k = i / 64, l = i % 64, n = l % 16, gg = l / 16;
      const int row = k == 0 ? n : k == 1 ? 16 + n : k == 2 ? (n < 8 ? 16 + n : -1)
                                                            : (n >= 8 ? 8 + n : -1);
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)(8 * gg + e == row ? 1.0f : 0.0f);
      sSel[i] = v;
    }
    const bf16x8 zero8 = {};
    for (int i = threadIdx.x; i < kBwdWaves * kSlot * 64; i += blockDim.x) sX[i] = zero8;
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      sb2[i] = a.params[po.b2 + i];
      const int s = i / 32, gg = (i / 8) % 4, j = i % 8;
      sw3[i] = (float)a.packed[ko.w3 + unit_of(s, gg, j)];
    }
    __syncthreads();
  }
  const float b3 = a.params[po.b3];
  const int ln = lane(), g = ln >> 4, col = ln & 15, w = threadIdx.x / kWave;
  const int64_t n_points = (int64_t)a.n_rays * a.n_bins;
  const int64_t n_chunks = (n_points + 31) / 32;
  // chunk groups of kBwdWaves chunks: block b takes groups b, b + gridDim.x,
  // ...; wave w takes chunk kBwdWaves group + w (past the end: no valid points,
  // so the wave still meets the block's barriers and adds zeros)
  const int64_t n_groups = (n_chunks + kBwdWaves - 1) / kBwdWaves;

  f32x4 acc2[MT][MT], acc1[RT][3];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int q = 0; q < MT; ++q) acc2[m][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < RT; ++m)
#pragma unroll
    for (int q = 0; q < 3; ++q) acc1[m][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // dW1 += d1 gamma^T for this wave's row tiles, over every wave's points of
  // the last group (slots in wave order: a fixed summation order)
  const auto consume = [&]() {
    bf16x8 q[2][3 + RT];  // one source wave's fragments, the next one's in flight
    const auto load = [&](int v, bf16x8 (&d)[3 + RT]) {
      const bf16x8* slot = sX + v * kSlot * 64;
#pragma unroll
      for (int F = 0; F < 3; ++F) d[F] = slot[(MT + F) * 64 + ln];
#pragma unroll
      for (int r = 0; r < RT; ++r) d[3 + r] = slot[(RT * w + r) * 64 + ln];
    };
    load(0, q[0]);
#pragma unroll
    for (int v = 0; v < kBwdWaves; ++v) {
      if (v + 1 < kBwdWaves) load(v + 1, q[(v + 1) % 2]);
      const bf16x8(&d)[3 + RT] = q[v % 2];
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int F = 0; F < 3; ++F) acc1[r][F] = mfma(d[3 + r], d[F], acc1[r][F]);
    }
  };
  // dw3 and db2 partials of unit pm_unit(m, col), over this lane's points
  float acc3[MT], db2p[MT], db3p = 0.0f;
#pragma unroll
  for (int m = 0; m < MT; ++m) acc3[m] = db2p[m] = 0.0f;

  // Per chunk: the raw inputs and features, then the phases below.  The
  // previous group's dW1 products run beside the d2 arithmetic.  Lane l < 32
  // loads point l of a chunk (clamped to the last point, so no branch splits
  // the scheduling regions) one chunk ahead and encodes it once; the
  // coordinates and d_sigma reach the feature lanes through LDS, out-of-range
  // points as zeros.  Weight tiles are read two steps ahead of their products
  // (the wq, w1q, wtq rings): LDS latency is then covered by the products in
  // between, which with one wave per SIMD nothing else covers.
  const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  bf16x8* slot_w = sX + w * kSlot * 64;
  __shared__ float sPt[kBwdWaves][4][32];  // x, y, z, d_sigma of the chunk's points
  PointIn in;
  float dsig;
  const auto fetch = [&](int64_t chunk) {
    const int64_t p = min(chunk * 32 + (ln & 31), n_points - 1);
    in = load_point(a, p);
    dsig = a.d_sigma[p];
  };
  bf16x8 B1[2][2];
  float ds[2];
  const auto encode_chunk = [&](int64_t chunk) {
    wave_sync();  // the previous chunk's reads of the slots are done
    if (ln < 32) {
      const bool valid = chunk * 32 + ln < n_points;
      float y[3];
      encode_loaded(a, in, y);
#pragma unroll
      for (int k = 0; k < 3; ++k) sPt[w][k][ln] = valid ? y[k] : 0.0f;
      sPt[w][3][ln] = valid ? dsig : 0.0f;
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      features(sPt[w][g < 2 ? g : 2][16 * t + col], g, B1[t][0], B1[t][1]);
      ds[t] = sPt[w][3][16 * t + col];
    }
  };

  // the four 0/1 selectors stay in registers for the whole loop
  const bf16x8 sel[4] = {sSel[ln], sSel[64 + ln], sSel[128 + ln], sSel[192 + ln]};
  for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int64_t c = grp * kBwdWaves + w;
    // The operand tiles never change, so their LDS reads are loop-invariant:
    // hoisted, they would pin ~5H registers for the whole loop.  An offset of
    // zero the compiler cannot see through keeps each read next to its use.
    int opaque;
    asm volatile("v_mov_b32 %0, 0" : "=v"(opaque));
    const int li = ln + opaque;
    if (grp == blockIdx.x) fetch(c);
    encode_chunk(c);
    fetch(c + (int64_t)gridDim.x * kBwdWaves);  // the next group's chunk, while this one computes
    // gamma point-major, and layer 1 unit-major (K-step s of layer 2 = row
    // tiles 2s and 2s+1)
    bf16x8 G[3];
    {
      const bf16x8 e0 = sel[0], e2 = sel[2], e3 = sel[3];
      f32x4 c0[2], c1[2], c2[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        c0[t] = mfma(B1[t][0], e0, zero);
        c1[t] = mfma(B1[t][1], e0, zero);
        c2[t] = mfma(B1[t][1], e3, mfma(B1[t][0], e2, zero));
      }
      G[0] = pack_pair(c0[0], c0[1]);
      G[1] = pack_pair(c1[0], c1[1]);
      G[2] = pack_pair(c2[0], c2[1]);
    }
    bf16x8 B2[2][KS];
    bf16x8 w1q[4];
    w1q[0] = sA1[li];
    w1q[1] = sA1[64 + li];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      f32x4 hh[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * s + h;
        if (m + 1 < MT) {
          w1q[(2 * m + 2) % 4] = sA1[(2 * m + 2) * 64 + li];
          w1q[(2 * m + 3) % 4] = sA1[(2 * m + 3) * 64 + li];
        }
        const bf16x8 w0 = w1q[(2 * m) % 4], w1 = w1q[(2 * m + 1) % 4];
#pragma unroll
        for (int t = 0; t < 2; ++t) hh[t][h] = mfma(w1, B1[t][1], mfma(w0, B1[t][0], zero));
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float v[8] = {hh[t][0][0], hh[t][0][1], hh[t][0][2], hh[t][0][3],
                            hh[t][1][0], hh[t][1][1], hh[t][1][2], hh[t][1][3]};
        B2[t][s] = pack8_relu(v);
      }
    }
    // layer 2, unit-major, as bf16 h2
    bf16x8 H2[2][KS];
    bf16x8 wq[3];
    wq[0] = sA2[li];
    wq[1] = sA2[64 + li];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      f32x4 cc[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * s + h;
        const f32x4 bias = *reinterpret_cast<const f32x4*>(&sb2[16 * m + 4 * g + opaque]);
        cc[0][h] = bias;
        cc[1][h] = bias;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int idx = m * KS + k;
          if (idx + 2 < MT * KS) wq[(idx + 2) % 3] = sA2[(idx + 2) * 64 + li];
          const bf16x8 wv = wq[idx % 3];
#pragma unroll
          for (int t = 0; t < 2; ++t) cc[t][h] = mfma(wv, B2[t][k], cc[t][h]);
        }
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float v[8] = {cc[t][0][0], cc[t][0][1], cc[t][0][2], cc[t][0][3],
                            cc[t][1][0], cc[t][1][1], cc[t][1][2], cc[t][1][3]};
        H2[t][s] = pack8_relu(v);
      }
    }
    // z = w3 . h2 + b3 on the matrix cores (row 0 of the product), then dz;
    // beside it, h1 point-major
    float dz[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x4 zt = zero;
#pragma unroll
      for (int s = 0; s < KS; ++s) zt = mfma(sA3[s * 64 + li], H2[t][s], zt);
      const float z = __shfl(zt[0], col, kWave);
      dz[t] = ds[t] / (1.0f + expf(-(z + b3)));
    }
    if (g == 0) db3p += dz[0] + dz[1];
    bf16x8 H1p[MT];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const bf16x8 e = sel[hf];
        H1p[2 * s + hf] = pack_pair(mfma(B2[0][s], e, zero), mfma(B2[1][s], e, zero));
      }
    // d2 = [a2 > 0] dz w3 (unit-major, bf16); dw3 += h2 dz with h2
    // point-major (unit col, points 4g + r) and dz of those points; beside
    // them, dW1 from the previous group's slots
    bf16x8 D2[2][KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const f32x4 wlo = *reinterpret_cast<const f32x4*>(&sw3[(4 * s + g) * 8 + opaque]);
      const f32x4 whi = *reinterpret_cast<const f32x4*>(&sw3[(4 * s + g) * 8 + 4 + opaque]);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float v[8] = {dz[t] * wlo[0], dz[t] * wlo[1], dz[t] * wlo[2], dz[t] * wlo[3],
                            dz[t] * whi[0], dz[t] * whi[1], dz[t] * whi[2], dz[t] * whi[3]};
        D2[t][s] = mask_positive(pack8(v), H2[t][s]);
      }
    }
    {
      float dzp[2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) dzp[t][r] = __shfl(dz[t], 4 * g + r, kWave);
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          const bf16x8 e = sel[hf];
          const f32x4 x = mfma(H2[0][s], e, zero), y = mfma(H2[1][s], e, zero);
          float v = acc3[2 * s + hf];
#pragma unroll
          for (int r = 0; r < 4; ++r) v = fmaf(x[r], dzp[0][r], fmaf(y[r], dzp[1][r], v));
          acc3[2 * s + hf] = v;
        }
    }
    consume();  // the first group's slots hold zeros
    // d1 = [a1 > 0] W2^T d2, point-major, into this wave's slot with gamma
    __syncthreads();  // every wave has consumed the slots of the last group
#pragma unroll
    for (int F = 0; F < 3; ++F) slot_w[(MT + F) * 64 + ln] = G[F];
    bf16x8 wtq[3];
    wtq[0] = sA2t[li];
    wtq[1] = sA2t[64 + li];
#pragma unroll
    for (int T = 0; T < MT; ++T) {
      f32x4 cc[2] = {zero, zero};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int idx = T * KS + s;
        if (idx + 2 < MT * KS) wtq[(idx + 2) % 3] = sA2t[(idx + 2) * 64 + li];
        const bf16x8 wt = wtq[idx % 3];
#pragma unroll
        for (int t = 0; t < 2; ++t) cc[t] = mfma(D2[t][s], wt, cc[t]);
      }
      slot_w[T * 64 + ln] = mask_positive(pack_pair(cc[0], cc[1]), H1p[T]);
    }
    // d2 point-major; db2 += its column sums; dW2 += d2 h1^T; beside them,
    // the next chunk's features
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const bf16x8 e = sel[hf];
        const f32x4 x = mfma(D2[0][s], e, zero), y = mfma(D2[1][s], e, zero);
        const int To = 2 * s + hf;
        db2p[To] += ((x[0] + x[1]) + (x[2] + x[3])) + ((y[0] + y[1]) + (y[2] + y[3]));
        const bf16x8 d2p = pack_pair(x, y);
        mfma_agpr_row<MT>(acc2[To], d2p, H1p);
      }
    __syncthreads();  // this group's slots are complete
  }
  if (n_groups > blockIdx.x) consume();

  // the last accumulation MFMAs' results before any read of them
  asm volatile("s_nop 15\n\ts_nop 15" ::: "memory");
  // ---------------- the block's partial: waves added in LDS in index order
  float* red = reinterpret_cast<float*>(smem);
  float* out = a.partial + (int64_t)blockIdx.x * po.total;
  // db2, dw3: sums over the lane groups
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    db2p[m] += __shfl_xor(db2p[m], 16, kWave);
    db2p[m] += __shfl_xor(db2p[m], 32, kWave);
    acc3[m] += __shfl_xor(acc3[m], 16, kWave);
    acc3[m] += __shfl_xor(acc3[m], 32, kWave);
  }
  db3p += __shfl_xor(db3p, 1, kWave);
  db3p += __shfl_xor(db3p, 2, kWave);
  db3p += __shfl_xor(db3p, 4, kWave);
  db3p += __shfl_xor(db3p, 8, kWave);
  __syncthreads();  // every wave is past its last read of the operand tiles
  // One 16-unit row tile at a time: each wave stores its values for the tile
  // into a region of its own (row n = 4g + r of the accumulator, so only
  // stores), then the block sums the regions in wave order and writes the
  // tile's rows.  Rows of point-major tile T: pm_unit(T, n).
  constexpr int kSlab = 16 * H;  // floats per wave region
  float* mine = red + w * kSlab;
#pragma unroll
  for (int To = 0; To < MT; ++To) {
#pragma unroll
    for (int Ti = 0; Ti < MT; ++Ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) mine[(4 * g + r) * H + pm_unit(Ti, col)] = acc2[To][Ti][r];
    __syncthreads();
    for (int e = threadIdx.x; e < kSlab; e += blockDim.x) {
      const float v = ((red[e] + red[kSlab + e]) + red[2 * kSlab + e]) + red[3 * kSlab + e];
      out[po.W2 + (int64_t)pm_unit(To, e / H) * H + e % H] = v;
    }
    __syncthreads();
  }
  // dW1 and db1: this wave's row tiles, each owned by one wave of the block
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int F = 0; F < 3; ++F) {
      const int f = pm_feature(F, col);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = pm_unit(RT * w + r, 4 * g + q);
        if (f >= 0) out[po.W1 + o * kNF + f] = acc1[r][F][q];
        // column 5 of tile 1 is slot 13 of axis 0, the constant 1 that
        // carries b1: its dW1 column is db1
        if (F == 1 && col == 5) out[po.b1 + o] = acc1[r][F][q];
      }
    }
  // b2, w3, b3 as one vector [b2 | w3 | b3] per wave
  if (g == 0) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      mine[pm_unit(m, col)] = db2p[m];
      mine[H + pm_unit(m, col)] = acc3[m];
    }
  }
  if (ln == 0) mine[2 * H] = db3p;
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * H + 1; e += blockDim.x)
    out[po.b2 + e] = ((red[e] + red[kSlab + e]) + red[2 * kSlab + e]) + red[3 * kSlab + e];
}

// grad[i] = sum over blocks of partial[b][i] in binary64, in a fixed order:
// a block takes 64 parameters; its thread (g, i) sums blocks b = g (mod 4) in
// increasing order, and the four sums are added in g order.
constexpr int kSumLanes = 64, kSumGroups = 4;
__global__ __launch_bounds__(kSumLanes* kSumGroups) void sum_partials_kernel(
    const float* __restrict__ partial, int n_blocks, int64_t P, float* __restrict__ grad) {
  __shared__ double part[kSumGroups][kSumLanes];
  const int li = threadIdx.x % kSumLanes, g = threadIdx.x / kSumLanes;
  const int64_t i = (int64_t)blockIdx.x * kSumLanes + li;
  double s = 0.0;
  if (i < P)
    for (int b = g; b < n_blocks; b += kSumGroups) s += (double)partial[(int64_t)b * P + i];
  part[g][li] = s;
  __syncthreads();
  if (g == 0 && i < P)
    grad[i] = (float)(((part[0][li] + part[1][li]) + part[2][li]) + part[3][li]);
}

txs_status check_mlp(const txs_mlp* m) {
  TXS_REQUIRE(m, "txs_mlp: null descriptor");
  TXS_REQUIRE(m->hidden == 64 || m->hidden == 128, "txs_mlp: hidden must be 64 or 128, got %d",
              m->hidden);
  TXS_REQUIRE(m->packed && m->params, "txs_mlp: null packed weights or params");
  TXS_REQUIRE(std::isfinite(m->scale) && m->scale > 0.0f, "txs_mlp: scale must be > 0");
  return TXS_OK;
}

}  // namespace
}  // namespace txs

extern "C" size_t txs_mlp_param_count(int32_t hidden) {
  return (size_t)txs::ParamOffsets(hidden).total;
}

extern "C" size_t txs_mlp_packed_bytes(int32_t hidden) {
  return (size_t)txs::PackOffsets(hidden).total * 2;
}

extern "C" txs_status txs_mlp_pack(const float* params, int32_t hidden, void* packed,
                                   void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(hidden == 64 || hidden == 128, "txs_mlp_pack: hidden must be 64 or 128");
  TXS_REQUIRE(params && packed, "txs_mlp_pack: null pointer");
  const int64_t n = PackOffsets(hidden).total;
  hipLaunchKernelGGL(pack_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, as_stream(stream), params,
                     (int)hidden, static_cast<__bf16*>(packed));
  return launch_status("txs_mlp_pack");
}

extern "C" txs_status txs_prop_mlp_fwd(const txs_mlp* mlp, const float* rays_o,
                                       const float* rays_d, int32_t n_rays, int32_t n_bins,
                                       const float* edges, float* sigma, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_mlp(mlp)) return s;
  TXS_REQUIRE(n_rays >= 0 && n_bins >= 1, "txs_prop_mlp_fwd: bad size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(rays_o && rays_d && edges && sigma, "txs_prop_mlp_fwd: null array");
  FwdArgs a{static_cast<const __bf16*>(mlp->packed), mlp->params, 1.0f / mlp->scale,
            mlp->contract, rays_o, rays_d, n_rays, n_bins, FastDiv((uint32_t)n_bins),
            (int64_t)n_rays * n_bins < ((int64_t)1 << 32), edges, sigma};
  const int64_t n_tiles = ((int64_t)n_rays * n_bins + 15) / 16;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  if (mlp->hidden == 64) {
    constexpr int NT = 4;
    const int64_t blocks = std::min<int64_t>((n_tiles + 4 * NT - 1) / (4 * NT), (int64_t)cus * 8);
    hipLaunchKernelGGL((mlp_fwd_kernel<64, NT>), dim3((unsigned)blocks), dim3(256), 0,
                       as_stream(stream), a);
  } else {
    constexpr int NT = 2;
    const int64_t blocks = std::min<int64_t>((n_tiles + 8 * NT - 1) / (8 * NT), (int64_t)cus * 4);
    hipLaunchKernelGGL((mlp_fwd_kernel<128, NT, 512>), dim3((unsigned)blocks), dim3(512), 0,
                       as_stream(stream), a);
  }
  return launch_status("txs_prop_mlp_fwd");
}

extern "C" size_t txs_mlp_bwd_workspace_size(int32_t hidden) {
  if (hidden != 64 && hidden != 128) return 0;
  return (size_t)txs::bwd_blocks(hidden) * (size_t)txs::ParamOffsets(hidden).total * sizeof(float);
}

extern "C" txs_status txs_prop_mlp_bwd(const txs_mlp* mlp, const float* rays_o,
                                       const float* rays_d, int32_t n_rays, int32_t n_bins,
                                       const float* edges, const float* d_sigma, float* grad,
                                       void* workspace, size_t workspace_bytes, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status s = check_mlp(mlp)) return s;
  TXS_REQUIRE(n_rays >= 0 && n_bins >= 1, "txs_prop_mlp_bwd: bad size");
  TXS_REQUIRE(grad, "txs_prop_mlp_bwd: null grad");
  const int H = mlp->hidden;
  const int64_t P = ParamOffsets(H).total;
  const int64_t n_points = (int64_t)n_rays * n_bins;
  const int64_t n_chunks = (n_points + 31) / 32;  // 32 points per wave iteration
  const int blocks =
      (int)std::min<int64_t>((n_chunks + kBwdWaves - 1) / kBwdWaves, bwd_blocks(H));
  if (blocks > 0) {
    TXS_REQUIRE(rays_o && rays_d && edges && d_sigma, "txs_prop_mlp_bwd: null array");
    TXS_REQUIRE(workspace, "txs_prop_mlp_bwd: null workspace");
    TXS_REQUIRE(workspace_bytes >= txs_mlp_bwd_workspace_size(H),
                "txs_prop_mlp_bwd: workspace of %zu bytes, need %zu", workspace_bytes,
                txs_mlp_bwd_workspace_size(H));
    BwdArgs a{static_cast<const __bf16*>(mlp->packed), mlp->params, 1.0f / mlp->scale,
              mlp->contract, rays_o, rays_d, n_rays, n_bins, FastDiv((uint32_t)n_bins),
              n_points < ((int64_t)1 << 32), edges, d_sigma, static_cast<float*>(workspace)};
    if (H == 64)
      hipLaunchKernelGGL(mlp_bwd_kernel<64>, dim3(blocks), dim3(kBwdWaves * kWave), 0,
                         as_stream(stream), a);
    else
      hipLaunchKernelGGL(mlp_bwd_kernel<128>, dim3(blocks), dim3(kBwdWaves * kWave), 0,
                         as_stream(stream), a);
    if (txs_status s = launch_status("txs_prop_mlp_bwd")) return s;
  }
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((P + kSumLanes - 1) / kSumLanes)),
                     dim3(kSumLanes * kSumGroups), 0, as_stream(stream),
                     static_cast<const float*>(workspace), blocks, P, grad);
  return launch_status("txs_prop_mlp_bwd");
}
