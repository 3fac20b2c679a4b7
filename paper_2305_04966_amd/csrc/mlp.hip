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
//   A2t[m][s] layer 2 transposed (W2^T, for the adjoint), s < H/32
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
  } else if (e < ko.w3) {  // A2t[m][s][lane][i] = W2[out = permuted K][in = row]
    const int64_t t = (e - ko.A2t) / 512, r = (e - ko.A2t) % 512;
    const int m = (int)(t / (H / 32)), s = (int)(t % (H / 32)), l = (int)(r / 8), i = (int)(r % 8);
    v = p[po.W2 + (int64_t)unit_of(s, l / 16, i) * H + (16 * m + l % 16)];
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
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  // inputs of the current tile group, fetched one group ahead
  PointIn in[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int64_t p = (wave * NT + t) * 16 + col;
    if (p < n_points) in[t] = load_point(a, p);
  }
  for (int64_t t0 = wave * NT; t0 < n_tiles; t0 += n_waves * NT) {
    bf16x8 B1[NT][2];
    bool valid[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t p = (t0 + t) * 16 + col;
      valid[t] = p < n_points;
      float y[3] = {0.0f, 0.0f, 0.0f};
      if (valid[t]) encode_loaded(a, in[t], y);
      const float xa = g == 0 ? y[0] : g == 1 ? y[1] : y[2];
      features(xa, g, B1[t][0], B1[t][1]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t pn = (t0 + n_waves * NT + t) * 16 + col;
      if (pn < n_points) in[t] = load_point(a, pn);
    }
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
// A block of 4 waves takes 64 points at a time, 16 per wave.  Phase A: each
// wave recomputes its tile's forward in the transposed orientation (rows =
// units, columns = points), forms dz, d2 = [a2 > 0] dz w3 and
// d1 = [a1 > 0] W2^T d2 (W2^T from the A2t tiles, whose K order matches the
// fragments of d2), and stores bf16 gamma, h1, d2, d1 into LDS as
// [unit][point] rows.  Phase B: the weight gradients contract over points, so
// each operand lane needs 8 consecutive points of one unit -- one 16-byte LDS
// read from those rows; wave w owns rows [RO w, RO w + RO) of the 16-unit row
// tiles of dW2 and dW1 and accumulates them over every batch in registers.
// Per-block partial gradients go to a workspace; a second kernel sums the
// blocks in a fixed order (deterministic, no float atomics).
constexpr int kBwdBlocks = 256;  // one block per CU (LDS-limited)
constexpr int kBwdBatch = 64;    // points per block iteration
constexpr int kRowStride = kBwdBatch + 8;  // bf16 elements per staged row (144 B)

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

__device__ __forceinline__ float bf16_round(float v) { return (float)(__bf16)v; }

template <int H>
__global__ __launch_bounds__(256) void mlp_bwd_kernel(BwdArgs a) {
  constexpr int MT = H / 16, KS = H / 32, RO = MT / 4, RS = kRowStride;
  const PackOffsets ko(H);
  const ParamOffsets po(H);
  __shared__ bf16x8 sA1[MT * 2 * 64];
  __shared__ bf16x8 sA2[MT * KS * 64];
  __shared__ bf16x8 sA2t[MT * KS * 64];
  __shared__ float sb1[H], sb2[H], sw3[H];
  __shared__ __attribute__((aligned(16))) __bf16 sH1[H * RS];
  __shared__ __attribute__((aligned(16))) __bf16 sD2[H * RS];
  __shared__ __attribute__((aligned(16))) __bf16 sD1[H * RS];
  __shared__ __attribute__((aligned(16))) __bf16 sG[48 * RS];
  __shared__ float sRed[4][H + 1];
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(a.packed);
    for (int i = threadIdx.x; i < MT * 2 * 64; i += blockDim.x) sA1[i] = src[i];
    const bf16x8* src2 = reinterpret_cast<const bf16x8*>(a.packed + ko.A2);
    for (int i = threadIdx.x; i < MT * KS * 64; i += blockDim.x) sA2[i] = src2[i];
    const bf16x8* src3 = reinterpret_cast<const bf16x8*>(a.packed + ko.A2t);
    for (int i = threadIdx.x; i < MT * KS * 64; i += blockDim.x) sA2t[i] = src3[i];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      sb1[i] = a.params[po.b1 + i];
      sb2[i] = a.params[po.b2 + i];
      sw3[i] = (float)a.packed[ko.w3 + i];
    }
    __syncthreads();
  }
  const float b3 = a.params[po.b3];
  const int ln = lane(), g = ln >> 4, col = ln & 15, w = threadIdx.x / kWave;
  const int64_t n_points = (int64_t)a.n_rays * a.n_bins;
  const int64_t n_batches = (n_points + kBwdBatch - 1) / kBwdBatch;

  f32x4 acc2[RO][MT], acc1[RO][3];
#pragma unroll
  for (int r = 0; r < RO; ++r) {
#pragma unroll
    for (int m = 0; m < MT; ++m) acc2[r][m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int m = 0; m < 3; ++m) acc1[r][m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  float db2p[RO];
#pragma unroll
  for (int r = 0; r < RO; ++r) db2p[r] = 0.0f;
  float acc3[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc3[m][i] = 0.0f;
  float acc_b3 = 0.0f;

  const int pc = 16 * w + col;  // column of this lane's point in the staged rows
  // inputs of the current batch, fetched one batch ahead (before phase B)
  PointIn in{};
  float dsig = 0.0f;
  {
    const int64_t p = (int64_t)blockIdx.x * kBwdBatch + pc;
    if (p < n_points) {
      in = load_point(a, p);
      dsig = a.d_sigma[p];
    }
  }
  for (int64_t batch = blockIdx.x; batch < n_batches; batch += gridDim.x) {
    // ---------------- phase A: this wave's 16 points
    const int64_t p = batch * kBwdBatch + pc;
    const bool valid = p < n_points;
    bf16x8 B1[2];
    {
      float y[3] = {0.0f, 0.0f, 0.0f};
      if (valid) encode_loaded(a, in, y);
      const float xa = g == 0 ? y[0] : g == 1 ? y[1] : y[2];
      features(xa, g, B1[0], B1[1]);
      if (g < 3) {
#pragma unroll
        for (int q = 0; q < 16; ++q) sG[(16 * g + q) * RS + pc] = B1[q / 8][q % 8];
      }
    }
    bf16x8 B2[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      f32x4 hh[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * s + h;
        const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};  // b1 arrives through K
        f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sA1[(m * 2 + 0) * 64 + ln], B1[0], zero,
                                                           0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sA1[(m * 2 + 1) * 64 + ln], B1[1], c, 0, 0, 0);
        hh[h] = c;
      }
      const float v[8] = {hh[0][0], hh[0][1], hh[0][2], hh[0][3],
                          hh[1][0], hh[1][1], hh[1][2], hh[1][3]};
      B2[s] = pack8_relu(v);
#pragma unroll
      for (int j = 0; j < 8; ++j) sH1[(16 * (2 * s + j / 4) + 4 * g + j % 4) * RS + pc] = B2[s][j];
    }
    // layer 2, all row tiles kept for the masks
    f32x4 a2[MT];
    float z = 0.0f;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      f32x4 c = {sb2[16 * m + 4 * g], sb2[16 * m + 4 * g + 1], sb2[16 * m + 4 * g + 2],
                 sb2[16 * m + 4 * g + 3]};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sA2[(m * KS + s) * 64 + ln], B2[s], c, 0, 0, 0);
      a2[m] = c;
#pragma unroll
      for (int i = 0; i < 4; ++i) z = fmaf(bf16_round(fmaxf(c[i], 0.0f)), sw3[16 * m + 4 * g + i], z);
    }
    z += __shfl_xor(z, 16, kWave);
    z += __shfl_xor(z, 32, kWave);
    const float dz = valid ? dsig / (1.0f + expf(-(z + b3))) : 0.0f;
    if (g == 0) acc_b3 += dz;
    bf16x8 D2B[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int m = 2 * s + j / 4, i = j % 4, u = 16 * m + 4 * g + i;
        const float h2 = bf16_round(fmaxf(a2[m][i], 0.0f));
        acc3[m][i] = fmaf(dz, h2, acc3[m][i]);
        v[j] = a2[m][i] > 0.0f ? dz * sw3[u] : 0.0f;
      }
      D2B[s] = pack8(v);
#pragma unroll
      for (int j = 0; j < 8; ++j) sD2[(16 * (2 * s + j / 4) + 4 * g + j % 4) * RS + pc] = D2B[s][j];
    }
    // d1 = [a1 > 0] W2^T d2, K over layer-2 units in the fragments' order
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sA2t[(m * KS + s) * 64 + ln], D2B[s], c, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool on = (float)B2[m / 2][4 * (m % 2) + i] > 0.0f;
        sD1[(16 * m + 4 * g + i) * RS + pc] = (__bf16)(on ? c[i] : 0.0f);
      }
    }
    __syncthreads();
    {
      const int64_t pn = (batch + gridDim.x) * kBwdBatch + pc;
      if (pn < n_points) {
        in = load_point(a, pn);
        dsig = a.d_sigma[pn];
      }
    }
    // ---------------- phase B: contract over the batch's 64 points
#pragma unroll
    for (int ks = 0; ks < kBwdBatch / 32; ++ks) {
      const int kp = 32 * ks + 8 * g;
      bf16x8 AD2[RO], AD1[RO];
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        const int row = 16 * (RO * w + r) + col;
        AD2[r] = *reinterpret_cast<const bf16x8*>(&sD2[row * RS + kp]);
        AD1[r] = *reinterpret_cast<const bf16x8*>(&sD1[row * RS + kp]);
#pragma unroll
        for (int j = 0; j < 8; ++j) db2p[r] += (float)AD2[r][j];
      }
#pragma unroll
      for (int mf = 0; mf < MT; ++mf) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sH1[(16 * mf + col) * RS + kp]);
#pragma unroll
        for (int r = 0; r < RO; ++r)
          acc2[r][mf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AD2[r], bh, acc2[r][mf], 0, 0, 0);
      }
#pragma unroll
      for (int gf = 0; gf < 3; ++gf) {
        const bf16x8 bg = *reinterpret_cast<const bf16x8*>(&sG[(16 * gf + col) * RS + kp]);
#pragma unroll
        for (int r = 0; r < RO; ++r)
          acc1[r][gf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AD1[r], bg, acc1[r][gf], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---------------- per-block partial gradients
  const int64_t P = po.total;
  float* out = a.partial + (int64_t)blockIdx.x * P;
#pragma unroll
  for (int r = 0; r < RO; ++r) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * (RO * w + r) + 4 * g + i;
#pragma unroll
      for (int mf = 0; mf < MT; ++mf) out[po.W2 + (int64_t)o * H + 16 * mf + col] = acc2[r][mf][i];
#pragma unroll
      for (int gf = 0; gf < 3; ++gf) {
        const int f = feature_of(gf, col);
        if (f >= 0) out[po.W1 + (int64_t)o * kNF + f] = acc1[r][gf][i];
      }
      // feature slot 13 of lane group 0 is the constant 1 that carries b1, so
      // its column of dW1 is db1 = sum over points of d1
      if (col == 13) out[po.b1 + o] = acc1[r][0][i];
    }
    float s2 = db2p[r];
    s2 += __shfl_xor(s2, 16, kWave);
    s2 += __shfl_xor(s2, 32, kWave);
    if (g == 0) out[po.b2 + 16 * (RO * w + r) + col] = s2;
  }
  // dw3, db3: sum over the 16 point columns, then over the 4 waves in order
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = acc3[m][i];
      v += __shfl_xor(v, 1, kWave);
      v += __shfl_xor(v, 2, kWave);
      v += __shfl_xor(v, 4, kWave);
      v += __shfl_xor(v, 8, kWave);
      if (col == 0) sRed[w][16 * m + 4 * g + i] = v;
    }
  {
    float v = acc_b3;
    v += __shfl_xor(v, 1, kWave);
    v += __shfl_xor(v, 2, kWave);
    v += __shfl_xor(v, 4, kWave);
    v += __shfl_xor(v, 8, kWave);
    if (ln == 0) sRed[w][H] = v;
  }
  __syncthreads();
  for (int u = threadIdx.x; u <= H; u += blockDim.x) {
    const float v = ((sRed[0][u] + sRed[1][u]) + sRed[2][u]) + sRed[3][u];
    out[u < H ? po.w3 + u : po.b3] = v;
  }
}

// grad[i] = sum over blocks of partial[b][i], blocks in index order
__global__ void sum_partials_kernel(const float* __restrict__ partial, int n_blocks, int64_t P,
                                    float* __restrict__ grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  double s = 0.0;
  for (int b = 0; b < n_blocks; ++b) s += (double)partial[(int64_t)b * P + i];
  grad[i] = (float)s;
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
  return (size_t)txs::kBwdBlocks * (size_t)txs::ParamOffsets(hidden).total * sizeof(float);
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
  const int64_t n_batches = (n_points + kBwdBatch - 1) / kBwdBatch;
  const int blocks = (int)std::min<int64_t>(n_batches, kBwdBlocks);
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
      hipLaunchKernelGGL(mlp_bwd_kernel<64>, dim3(blocks), dim3(256), 0, as_stream(stream), a);
    else
      hipLaunchKernelGGL(mlp_bwd_kernel<128>, dim3(blocks), dim3(256), 0, as_stream(stream), a);
    if (txs_status s = launch_status("txs_prop_mlp_bwd")) return s;
  }
  hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_1d(P, 256)), dim3(256), 0, as_stream(stream),
                     static_cast<const float*>(workspace), blocks, P, grad);
  return launch_status("txs_prop_mlp_bwd");
}
