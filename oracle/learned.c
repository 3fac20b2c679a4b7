/*
 * learned.c -- reference of the learned transmittance estimator (proposal
 * network) of the method: a small MLP that predicts density along each ray,
 * whose rendering weights are fitted to those of the radiance field by a
 * PDF-matching (histogram) loss, updated by SGD (Section 3.1 "PDF
 * Approaches", Table 1 third row, Eq. 4; Section 3.2 "Choice of
 * Representations"; Appendix B hyper-parameters F_Theta and N).
 *
 * TEST INFRASTRUCTURE ONLY (same rules as txs_oracle.c).  binary64
 * throughout; the "bf16" variants round the MLP operands to bfloat16
 * (round-to-nearest-even) at the points the GPU path stores them in bfloat16,
 * to serve as the emulated reference of a bfloat16 matrix-core forward.
 *
 * Network (hidden width H):
 *   x_hat = x / s                                   (bounded scene, s = half extent)
 *   x_hat = contract(x / s) / 2,  contract(y) = y if |y| <= 1 else (2 - 1/|y|) y/|y|
 *   gamma = [x_hat_0..2, then per axis a, octave k = 0..5: sin(2^k pi x_hat_a), cos(2^k pi x_hat_a)]
 *   h1 = relu(W1 gamma + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3, sigma = softplus(z)
 * Parameter vector (row-major): W1 [H,39], b1 [H], W2 [H,H], b2 [H], w3 [H], b3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))
#define NF 39

/* bfloat16 round-to-nearest-even of a value (through binary32, as a GPU
 * holding binary32 data rounds it). */
static double bf16(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static void encode(const double x[3], double s, int contract, double* g, int emulate) {
  double y[3] = {x[0] / s, x[1] / s, x[2] / s};
  if (contract) {
    double n = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double f = (n <= 1.0) ? 1.0 : (2.0 - 1.0 / n) / n;
    for (int a = 0; a < 3; ++a) y[a] = 0.5 * f * y[a];
  }
  for (int a = 0; a < 3; ++a) g[a] = y[a];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 6; ++k) {
      double arg = ldexp(3.14159265358979323846, k) * y[a];
      g[3 + 12 * a + 2 * k] = sin(arg);
      g[3 + 12 * a + 2 * k + 1] = cos(arg);
    }
  if (emulate)
    for (int f = 0; f < NF; ++f) g[f] = bf16(g[f]);
}

/* The parameters as binary64, the weight matrices and w3 rounded to bf16 when
 * emulating (biases stay exact: the matrix-core path adds them in fp32). */
typedef struct {
  double* buf;
  const double* W1;
  const double* b1;
  const double* W2;
  const double* b2;
  const double* w3;
  const double* b3;
} mlp_view;

static mlp_view view(const float* p, int H, int emulate) {
  const int64_t P = (int64_t)H * H + 42 * H + 1;
  mlp_view m;
  m.buf = (double*)malloc((size_t)P * sizeof(double));
  for (int64_t i = 0; i < P; ++i) m.buf[i] = (double)p[i];
  m.W1 = m.buf;
  m.b1 = m.W1 + H * NF;
  m.W2 = m.b1 + H;
  m.b2 = m.W2 + H * H;
  m.w3 = m.b2 + H;
  m.b3 = m.w3 + H;
  if (emulate) {
    for (int64_t i = 0; i < H * NF; ++i) m.buf[i] = bf16(m.buf[i]);
    for (int64_t i = 0; i < (int64_t)H * H; ++i) m.buf[40 * H + i] = bf16(m.buf[40 * H + i]);
    for (int64_t i = 0; i < H; ++i) m.buf[41 * H + (int64_t)H * H + i] = bf16(m.buf[41 * H + (int64_t)H * H + i]);
  }
  return m;
}

static double softplus(double z) { return z > 30.0 ? z + log1p(exp(-z)) : log1p(exp(z)); }
static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Forward at points x [n,3]; optional outputs: z [n] (pre-softplus). */
EXPORT void oracle_mlp_fwd(int64_t n, const double* x, const float* params, int32_t H,
                           double scale, int32_t contract, int32_t emulate, double* sigma,
                           double* zout) {
  const mlp_view m = view(params, H, emulate);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double g[NF], h1[512], h2[512];
    encode(x + 3 * i, scale, contract, g, emulate);
    for (int o = 0; o < H; ++o) {
      double acc = 0.0;
      for (int f = 0; f < NF; ++f) acc += m.W1[o * NF + f] * g[f];
      acc += m.b1[o];
      h1[o] = acc > 0.0 ? acc : 0.0;
      if (emulate) h1[o] = bf16(h1[o]);
    }
    for (int o = 0; o < H; ++o) {
      double acc = 0.0;
      for (int f = 0; f < H; ++f) acc += m.W2[o * H + f] * h1[f];
      acc += m.b2[o];
      h2[o] = acc > 0.0 ? acc : 0.0;
      if (emulate) h2[o] = bf16(h2[o]);
    }
    double z = m.b3[0];
    for (int f = 0; f < H; ++f) z += m.w3[f] * h2[f];
    sigma[i] = softplus(z);
    if (zout) zout[i] = z;
  }
  free(m.buf);
}

/* Gradient of sum_i d_sigma[i] * sigma(x_i) w.r.t. the parameter vector
 * (same layout); binary64 reverse mode, per point then summed in point order.
 * With emulate set, the adjoint operands of the two hidden layers
 * (d2 = dL/da2 and d1 = dL/da1) are rounded to bfloat16 as well, since a
 * matrix-core backward multiplies them in bfloat16; the bias gradients sum the
 * rounded values.  Optional grad_abs receives the same sums taken over the
 * absolute values of every term (the scale against which a reordered fp32
 * summation is judged). */
EXPORT void oracle_mlp_bwd(int64_t n, const double* x, const float* params, int32_t H,
                           double scale, int32_t contract, int32_t emulate, const double* d_sigma,
                           double* grad, double* grad_abs) {
  const mlp_view m = view(params, H, emulate);
  const int64_t P = (int64_t)H * H + 42 * H + 1;
  double* out[2] = {grad, grad_abs};
  for (int k = 0; k < 2; ++k)
    if (out[k]) memset(out[k], 0, (size_t)P * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    double g[NF], a1[512], h1[512], a2[512], h2[512], d2[512], d1[512];
    encode(x + 3 * i, scale, contract, g, emulate);
    for (int o = 0; o < H; ++o) {
      double acc = m.b1[o];
      for (int f = 0; f < NF; ++f) acc += m.W1[o * NF + f] * g[f];
      a1[o] = acc;
      h1[o] = acc > 0.0 ? acc : 0.0;
      if (emulate) h1[o] = bf16(h1[o]);
    }
    for (int o = 0; o < H; ++o) {
      double acc = m.b2[o];
      for (int f = 0; f < H; ++f) acc += m.W2[o * H + f] * h1[f];
      a2[o] = acc;
      h2[o] = acc > 0.0 ? acc : 0.0;
      if (emulate) h2[o] = bf16(h2[o]);
    }
    double z = m.b3[0];
    for (int f = 0; f < H; ++f) z += m.w3[f] * h2[f];
    const double dz = d_sigma[i] * sigm(z);
    for (int f = 0; f < H; ++f) {
      d2[f] = a2[f] > 0.0 ? dz * m.w3[f] : 0.0;
      if (emulate) d2[f] = bf16(d2[f]);
    }
    for (int f = 0; f < H; ++f) {
      double acc = 0.0;
      for (int o = 0; o < H; ++o) acc += m.W2[o * H + f] * d2[o];
      d1[f] = a1[f] > 0.0 ? acc : 0.0;
      if (emulate) d1[f] = bf16(d1[f]);
    }
    for (int k = 0; k < 2; ++k) {
      if (!out[k]) continue;
      /* k = 0: the gradient; k = 1: the same sums of |term| */
#define T(v) (k ? fabs(v) : (v))
      double* gW1 = out[k];
      double* gb1 = gW1 + H * NF;
      double* gW2 = gb1 + H;
      double* gb2 = gW2 + H * H;
      double* gw3 = gb2 + H;
      double* gb3 = gw3 + H;
      gb3[0] += T(dz);
      for (int f = 0; f < H; ++f) gw3[f] += T(dz * h2[f]);
      for (int o = 0; o < H; ++o) {
        gb2[o] += T(d2[o]);
        for (int f = 0; f < H; ++f) gW2[o * H + f] += T(d2[o] * h1[f]);
      }
      for (int o = 0; o < H; ++o) {
        gb1[o] += T(d1[o]);
        for (int f = 0; f < NF; ++f) gW1[o * NF + f] += T(d1[o] * g[f]);
      }
#undef T
    }
  }
  free(m.buf);
}

/*
 * PDF-matching loss between a target histogram (the rendering weights of the
 * radiance field on its own intervals, packed) and a proposal histogram
 * (weights on dense bins), the proposal's outer measure bounding the target:
 *   bound_i = sum of proposal weights whose bin overlaps (t0_i, t1_i)
 *   loss_r  = sum_i max(0, w_i - bound_i)^2 / (w_i + eps)
 * (the proposal loss of Mip-NeRF 360, which the paper's proposal estimator
 * uses).  Bins overlap an interval iff e_j < t1_i and e_{j+1} > t0_i.
 * Outputs: loss per ray; d_prop = d(mean_r loss_r)/d(proposal weights).
 */
EXPORT void oracle_hist_loss(int32_t n_rays, const int32_t* packed_info, const float* t0,
                             const float* t1, const float* w, int32_t n_bins, const float* edges,
                             const float* wp, double eps, double* loss, double* d_prop) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t r = 0; r < n_rays; ++r) {
    const int64_t s0 = packed_info[2 * r], cnt = packed_info[2 * r + 1];
    const float* e = edges + (int64_t)r * (n_bins + 1);
    const float* p = wp + (int64_t)r * n_bins;
    double* dp = d_prop ? d_prop + (int64_t)r * n_bins : NULL;
    if (dp)
      for (int j = 0; j < n_bins; ++j) dp[j] = 0.0;
    double L = 0.0;
    for (int64_t i = s0; i < s0 + cnt; ++i) {
      double bound = 0.0;
      for (int j = 0; j < n_bins; ++j)
        if (e[j] < t1[i] && e[j + 1] > t0[i]) bound += (double)p[j];
      const double gap = (double)w[i] - bound;
      if (gap > 0.0) {
        L += gap * gap / ((double)w[i] + eps);
        if (dp) {
          const double c = -2.0 * gap / ((double)w[i] + eps) / n_rays;
          for (int j = 0; j < n_bins; ++j)
            if (e[j] < t1[i] && e[j + 1] > t0[i]) dp[j] += c;
        }
      }
    }
    loss[r] = L;
  }
}

/* Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  In place, binary64. */
EXPORT void oracle_adam(int64_t n, double* p, double* m, double* v, const double* g, double lr,
                        double b1, double b2, double eps, int32_t step) {
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
