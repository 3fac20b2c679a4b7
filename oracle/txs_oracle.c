/*
 * txs_oracle.c -- plain, slow, obviously-correct CPU reference of the
 * transmittance-estimator sampling and packed volume-rendering path
 * (Li, Gao, Tancik, Kanazawa, "NerfAcc: Efficient Sampling Accelerates
 * NeRFs", 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only on the
 * seeded inputs of the `scenes` module.
 *
 * Precision contract:
 *  - geometric decisions (box clip, lattice points, occupancy cell, sample
 *    counts) are evaluated in IEEE binary32 following one written recipe,
 *    with contraction disabled (build with -ffp-contract=off);
 *  - everything continuous (transmittance, weights, colours, gradients, the
 *    inverse CDF, the field) is evaluated in binary64 from the float inputs.
 *
 * Each function names the passage of the paper it follows.  Loops run one
 * ray at a time, in sample order, with no blocking or reordering.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Ray / axis-aligned box clip (slab method).  The paper samples each ray on a
 * bounded range [t_n, t_f] (Section 3.1); for the occupancy-grid estimator
 * that range is the ray's chord through the grid's box.
 *
 * binary32 recipe, per axis a:
 *   inv = 1/d_a;  tlo = (bmin_a - o_a)*inv;  thi = (bmax_a - o_a)*inv
 *   t_near = max(near, min(tlo,thi) over axes), t_far = min(far, max(...))
 * min/max ignore NaN (0*inf from a ray lying in a slab plane).  The ray hits
 * iff t_near < t_far.                                                        */
static void clip_box(const float o[3], const float d[3], const float bmin[3],
                     const float bmax[3], float near_plane, float far_plane,
                     float* tn, float* tf) {
  float t_near = near_plane, t_far = far_plane;
  for (int a = 0; a < 3; ++a) {
    float inv = 1.0f / d[a];
    float tlo = (bmin[a] - o[a]) * inv;
    float thi = (bmax[a] - o[a]) * inv;
    t_near = fmaxf(t_near, fminf(tlo, thi));
    t_far = fminf(t_far, fmaxf(tlo, thi));
  }
  *tn = t_near;
  *tf = t_far;
}

EXPORT void oracle_clip(int32_t n, const float* o, const float* d, const float* bmin,
                        const float* bmax, float near_plane, float far_plane,
                        float* t_near, float* t_far) {
  for (int32_t r = 0; r < n; ++r) clip_box(o + 3 * r, d + 3 * r, bmin, bmax,
                                           near_plane, far_plane, t_near + r, t_far + r);
}

/* ------------------------------------------------------------------------- */
/* Occupancy-grid ray marching, dense definition.
 *
 * The spatial-skipping estimator (Section 3.1, "Spatial Skipping"; Table 1,
 * second row) binarises density on a grid and samples uniformly inside the
 * occupied cells.  Samples live on a per-segment lattice of step dt:
 *   t_k  = a + k*dt,  midpoint m_k = a + (k + 1/2)*dt,  k = 0,1,... while m_k < b
 * and sample k is kept iff the grid cell holding x(m_k) = o + m_k d is
 * occupied.  A sample is the interval (Section 4.2, "Sample as Interval")
 *   [t_k, min(a + (k+1)*dt, b)].
 * The test that decides occupancy is the binary32 recipe:
 *   m   = a + ((float)k + 0.5f)*dt
 *   x_c = o_c + m*d_c;  u_c = (x_c - bmin_c)*scale_c,  scale_c = res/(bmax_c-bmin_c)
 *   cell_c = clamp(floor(u_c), 0, res-1);  index = cx + res*(cy + res*cz)
 * This function tests every lattice point; it skips nothing.
 *
 * Unbounded scenes (Section 3.2, "Handling Unbounded Scenes") sample more
 * coarsely with distance.  With n_levels > 1 the grid is a cascade of nested
 * cubes of half-extent h0*2^l; the ray is cut into constant-level segments at
 * the cube faces (at most 2L-1 of them); a level-l segment uses the level-l
 * grid and the step dt0*2^l, its lattice anchored at the segment start.
 * With n_levels == 1 this is the plain bounded march over [t_near, t_far).
 * ------------------------------------------------------------------------- */
typedef struct {
  const uint32_t* bits;
  int32_t res, n_levels;
  float center[3];
  float half_extent0;
  float near_plane, far_plane, dt0;
  int32_t max_per_ray; /* 0 = no cap */
  float inv_scale;     /* > 0: one grid over contracted space, 1/contract_scale */
} march_cfg;

/* Occupancy in the grid over contracted space: the point, relative to the
 * centre and divided by the scene scale, is contracted into the ball of
 * radius 2 (Mip-NeRF 360: unchanged inside the unit ball, radius 2 - 1/|y|
 * outside), and the bit of its cell in the res^3 grid over [-2, 2]^3 is read.
 * binary32, one rounding per operation, in the order written. */
static int occupied_contracted(const march_cfg* c, const float o[3], const float d[3],
                               float m) {
  const int res = c->res;
  float y[3];
  for (int a = 0; a < 3; ++a) {
    float x = o[a] + m * d[a];
    y[a] = (x - c->center[a]) * c->inv_scale;
  }
  float r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  if (r2 > 1.0f) {
    float r = sqrtf(r2);
    float q = 1.0f / r;
    float f = (2.0f - q) * q;
    for (int a = 0; a < 3; ++a) y[a] = y[a] * f;
  }
  const float scale = (float)res * 0.25f;
  int cell[3];
  for (int a = 0; a < 3; ++a) {
    float u = floorf((y[a] + 2.0f) * scale);
    u = fminf(fmaxf(u, 0.0f), (float)(res - 1));
    cell[a] = (int)u;
  }
  int64_t idx = (int64_t)cell[0] + (int64_t)res * ((int64_t)cell[1] + (int64_t)res * cell[2]);
  return (int)((c->bits[idx >> 5] >> (idx & 31)) & 1u);
}

#define LATTICE_LIMIT (1 << 24) /* k stays exactly representable in binary32 */

static int occupied(const march_cfg* c, int level, const float o[3], const float d[3],
                    float m) {
  const float h = c->half_extent0 * (float)(1 << level);
  const int res = c->res;
  int cell[3];
  for (int a = 0; a < 3; ++a) {
    float bmin = c->center[a] - h;
    float bmax = c->center[a] + h;
    float scale = (float)res / (bmax - bmin);
    float x = o[a] + m * d[a];
    float u = (x - bmin) * scale;
    float f = floorf(u);
    f = fminf(fmaxf(f, 0.0f), (float)(res - 1));
    cell[a] = (int)f;
  }
  int64_t idx = (int64_t)cell[0] + (int64_t)res * ((int64_t)cell[1] + (int64_t)res * cell[2]);
  int64_t word = (int64_t)level * (((int64_t)res * res * res) >> 5) + (idx >> 5);
  return (int)((c->bits[word] >> (idx & 31)) & 1u);
}

/* Emits the samples of one ray; when t0 == NULL it only counts. */
static int32_t march_one(const march_cfg* c, const float o[3], const float d[3], float* t0,
                         float* t1, int32_t* lvl) {
  const int L = c->n_levels;
  float tn[8], tf[8];
  int hit[8];
  for (int l = 0; l < L; ++l) {
    const float h = c->half_extent0 * (float)(1 << l);
    float bmin[3], bmax[3];
    for (int a = 0; a < 3; ++a) { bmin[a] = c->center[a] - h; bmax[a] = c->center[a] + h; }
    clip_box(o, d, bmin, bmax, c->near_plane, c->far_plane, tn + l, tf + l);
  }
  /* nesting: an inner cube's chord lies inside the next outer one */
  for (int l = L - 2; l >= 0; --l) {
    tn[l] = fmaxf(tn[l], tn[l + 1]);
    tf[l] = fminf(tf[l], tf[l + 1]);
  }
  for (int l = 0; l < L; ++l) hit[l] = tn[l] < tf[l];

  /* segments in increasing t: descend from the outer level, then ascend */
  float sa[16], sb[16];
  int sl[16], ns = 0;
  for (int l = L - 1; l >= 0; --l) {
    if (!hit[l]) continue;
    sa[ns] = tn[l];
    sb[ns] = (l > 0 && hit[l - 1]) ? tn[l - 1] : tf[l];
    sl[ns++] = l;
  }
  for (int l = 1; l < L; ++l) {
    if (!hit[l] || !hit[l - 1]) continue;
    sa[ns] = tf[l - 1];
    sb[ns] = tf[l];
    sl[ns++] = l;
  }

  int32_t n = 0;
  for (int s = 0; s < ns; ++s) {
    const float a = sa[s], b = sb[s];
    const int l = sl[s];
    const float dt = c->dt0 * (float)(1 << l);
    for (int32_t k = 0; k < LATTICE_LIMIT; ++k) {
      float m = a + ((float)k + 0.5f) * dt;
      if (!(m < b)) break;
      if (c->inv_scale > 0.0f ? !occupied_contracted(c, o, d, m) : !occupied(c, l, o, d, m))
        continue;
      if (t0) {
        t0[n] = a + (float)k * dt;
        t1[n] = fminf(a + (float)(k + 1) * dt, b);
        if (lvl) lvl[n] = l;
      }
      ++n;
      if (c->max_per_ray > 0 && n >= c->max_per_ray) return n;
    }
  }
  return n;
}

/* counts[r] = number of samples of ray r.  If offsets != NULL, also writes the
 * packed samples of ray r at offsets[r] (ray-major, t ascending). */
EXPORT void oracle_march(int32_t n_rays, const float* o, const float* d, const uint32_t* bits,
                         int32_t res, int32_t n_levels, const float* center,
                         float half_extent0, float near_plane, float far_plane, float dt0,
                         int32_t max_per_ray, float contract_scale, int32_t* counts,
                         const int64_t* offsets, float* t0, float* t1, int32_t* ray_id,
                         int32_t* level) {
  march_cfg c = {bits, res, n_levels, {center[0], center[1], center[2]}, half_extent0,
                 near_plane, far_plane, dt0, max_per_ray,
                 contract_scale > 0.0f ? 1.0f / contract_scale : 0.0f};
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t r = 0; r < n_rays; ++r) {
    if (offsets) {
      int64_t s = offsets[r];
      int32_t n = march_one(&c, o + 3 * r, d + 3 * r, t0 + s, t1 + s, level ? level + s : NULL);
      for (int32_t i = 0; i < n; ++i) ray_id[s + i] = r;
      counts[r] = n;
    } else {
      counts[r] = march_one(&c, o + 3 * r, d + 3 * r, NULL, NULL, NULL);
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Volume rendering of packed samples (Eq. 2 discretised; Section 4.2
 * "Packed Tensor").  For the samples i of one ray, in order:
 *   Delta_i = t1_i - t0_i,  tau_i = sigma_i * Delta_i,
 *   T_i = exp(-sum_{j<i} tau_j)              (exclusive transmittance)
 *   alpha_i = 1 - exp(-tau_i),  w_i = T_i * alpha_i
 *   rgb = sum w_i c_i,  opacity = sum w_i,  depth = sum w_i (t0_i + t1_i)/2
 * With a background colour bg: rgb += (1 - opacity) * bg.
 * packed_info[r] = (start, count).                                           */
EXPORT void oracle_render_fwd(int32_t n_rays, const int32_t* packed_info, const float* t0,
                              const float* t1, const float* sigma, const float* rgb,
                              const float* bg, double* out_rgb, double* out_opacity,
                              double* out_depth, double* out_weights) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t r = 0; r < n_rays; ++r) {
    const int64_t s0 = packed_info[2 * r], n = packed_info[2 * r + 1];
    double acc[3] = {0, 0, 0}, op = 0, dep = 0, optical = 0;
    for (int64_t i = s0; i < s0 + n; ++i) {
      const double delta = (double)t1[i] - (double)t0[i];
      const double tau = (double)sigma[i] * delta;
      const double T = exp(-optical);
      const double alpha = -expm1(-tau);
      const double w = T * alpha;
      for (int c = 0; c < 3; ++c) acc[c] += w * (double)rgb[3 * i + c];
      op += w;
      dep += w * 0.5 * ((double)t0[i] + (double)t1[i]);
      if (out_weights) out_weights[i] = w;
      optical += tau;
    }
    for (int c = 0; c < 3; ++c)
      out_rgb[3 * r + c] = acc[c] + (bg ? (1.0 - op) * (double)bg[3 * r + c] : 0.0);
    out_opacity[r] = op;
    out_depth[r] = dep;
  }
}

/* Adjoint of oracle_render_fwd.  With v_i = dL/dw_i
 *   = g.(c_i - bg) + h + q*(t0_i+t1_i)/2,
 *   dL/dc_i     = w_i g
 *   dL/dsigma_i = Delta_i ( T_{i+1} v_i - sum_{j>i} w_j v_j ),  T_{i+1} = T_i e^{-tau_i}
 * obtained from dw_i/dtau_k = -w_i (k<i), T_{i+1} (k=i), 0 (k>i).  The suffix
 * sum is accumulated by a sequential reverse loop.  The sample intervals carry
 * no gradient (Section 4.2).  g_opacity, g_depth, bg may be NULL.             */
static void render_bwd_ray(int64_t s0, int64_t n, const float* t0, const float* t1,
                           const float* sigma, const float* rgb, const double g[3],
                           double h, double q, const double bgc[3], const float* g_w,
                           double* d_sigma, double* d_rgb) {
  if (n <= 0) return;
  /* exclusive optical depth before each sample, by a forward pass */
  double* excl = (double*)malloc((size_t)n * sizeof(double));
  double optical = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    excl[i] = optical;
    optical += (double)sigma[s0 + i] * ((double)t1[s0 + i] - (double)t0[s0 + i]);
  }
  /* suffix sum of w_j v_j by a reverse pass */
  double suffix = 0.0;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int64_t i = s0 + k;
    const double delta = (double)t1[i] - (double)t0[i];
    const double tau = (double)sigma[i] * delta;
    const double T = exp(-excl[k]);
    const double T_next = exp(-(excl[k] + tau));
    const double w = T * -expm1(-tau);
    double v;
    if (g_w) {
      v = (double)g_w[i];
    } else {
      const double mid = 0.5 * ((double)t0[i] + (double)t1[i]);
      v = h + q * mid;
      for (int c = 0; c < 3; ++c) v += g[c] * ((double)rgb[3 * i + c] - bgc[c]);
      for (int c = 0; c < 3; ++c) d_rgb[3 * i + c] = w * g[c];
    }
    d_sigma[i] = delta * (T_next * v - suffix);
    suffix += w * v;
  }
  free(excl);
}

EXPORT void oracle_render_bwd(int32_t n_rays, const int32_t* packed_info, const float* t0,
                              const float* t1, const float* sigma, const float* rgb,
                              const float* bg, const float* g_rgb, const float* g_opacity,
                              const float* g_depth, double* d_sigma, double* d_rgb) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t r = 0; r < n_rays; ++r) {
    double g[3], bgc[3];
    for (int c = 0; c < 3; ++c) {
      g[c] = g_rgb[3 * r + c];
      bgc[c] = bg ? (double)bg[3 * r + c] : 0.0;
    }
    const double h = g_opacity ? (double)g_opacity[r] : 0.0;
    const double q = g_depth ? (double)g_depth[r] : 0.0;
    render_bwd_ray(packed_info[2 * r], packed_info[2 * r + 1], t0, t1, sigma, rgb, g, h, q, bgc,
                   NULL, d_sigma, d_rgb);
  }
}

/* Adjoint of the weights alone: given v_i = dL/dw_i per sample, dL/dsigma_i. */
EXPORT void oracle_weights_bwd(int32_t n_rays, const int32_t* packed_info, const float* t0,
                               const float* t1, const float* sigma, const float* g_w,
                               double* d_sigma) {
  const double zero[3] = {0, 0, 0};
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t r = 0; r < n_rays; ++r)
    render_bwd_ray(packed_info[2 * r], packed_info[2 * r + 1], t0, t1, sigma, NULL, zero, 0.0,
                   0.0, zero, g_w, d_sigma, NULL);
}

/* ------------------------------------------------------------------------- */
/* No-gradient filtering (Section 4.2): samples whose transmittance is below
 * t_min are disregarded.  T_i = exp(-sum_{j<i} tau_j) is non-increasing, so the
 * kept samples are a prefix; kept[r] = #{i : T_i >= t_min}.
 * band[r] = 1 when some T_i lies within relative 1e-5 of t_min (a decision a
 * binary32 evaluation may legitimately take either way).                    */
EXPORT void oracle_transmittance_prefix(int32_t n_rays, const int32_t* packed_info,
                                        const float* t0, const float* t1, const float* sigma,
                                        double t_min, int32_t* kept, int32_t* band) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t r = 0; r < n_rays; ++r) {
    const int64_t s0 = packed_info[2 * r], n = packed_info[2 * r + 1];
    double optical = 0.0;
    int32_t k = 0, b = 0;
    for (int64_t i = s0; i < s0 + n; ++i) {
      const double T = exp(-optical);
      if (fabs(T - t_min) <= 1e-5 * t_min) b = 1;
      if (T >= t_min) ++k;
      optical += (double)sigma[i] * ((double)t1[i] - (double)t0[i]);
    }
    kept[r] = k;
    if (band) band[r] = b;
  }
}

/* ------------------------------------------------------------------------- */
/* Inverse transform sampling (Eq. 1) of a piecewise-constant estimator on
 * n_bins bins with edges e_0..e_n.  The CDF is read off the transmittance
 * estimator, F = 1 - T (Eq. 3):
 *   mode 0 (density):  F_0 = 0, F_{i+1} = 1 - exp(-sum_{j<=i} sigma_j (e_{j+1}-e_j))
 *   mode 1 (weights):  F_{i+1} = sum_{j<=i} w_j
 * Within a bin the estimator's T is linear (Table 1), so the inverse is linear:
 *   u' = u F_n;  i = largest i in [0, n] with F_i <= u'
 *   t  = e_i + (u' - F_i)/(F_{i+1} - F_i) (e_{i+1} - e_i)   if i < n, else t = e_n
 * mode 2 (density, exponential in the bin): the CDF of mode 0, inverted
 * exactly for a density that is constant inside each bin (T decays
 * exponentially there): with P_i = sum_{j<i} sigma_j (e_{j+1}-e_j),
 *   t = e_i + (-log(1 - u') - P_i) / sigma_i, kept inside [e_i, e_{i+1}].
 * When F_n <= 1e-12 the uniform estimator (Table 1, first row) is used
 * instead (F_i = i/n, linear in every mode).  u defaults to k/n_out,
 * k = 0..n_out, giving n_out+1 edges, i.e. n_out contiguous intervals.
 * out_bin records the chosen bin; band flags an edge whose u' lies within
 * relative 1e-5 of a CDF knot.                                              */
EXPORT void oracle_resample(int32_t n_rays, int32_t n_bins, const float* edges, const float* vals,
                            int32_t mode, int32_t n_out, const float* u_in, double* out_edges,
                            int32_t* out_bin, int32_t* band) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t r = 0; r < n_rays; ++r) {
    const float* e = edges + (int64_t)r * (n_bins + 1);
    const float* v = vals + (int64_t)r * n_bins;
    double* F = (double*)malloc((size_t)(2 * (n_bins + 1)) * sizeof(double));
    double* P = F + n_bins + 1; /* optical depth before each edge (modes 0 and 2) */
    F[0] = 0.0;
    P[0] = 0.0;
    double acc = 0.0;
    for (int i = 0; i < n_bins; ++i) {
      if (mode == 0 || mode == 2) {
        acc += (double)v[i] * ((double)e[i + 1] - (double)e[i]);
        F[i + 1] = -expm1(-acc);
        P[i + 1] = acc;
      } else {
        acc += (double)v[i];
        F[i + 1] = acc;
      }
    }
    const int uniform = !(F[n_bins] > 1e-12);
    if (uniform)
      for (int i = 0; i <= n_bins; ++i) F[i] = (double)i / n_bins;
    const double Fn = F[n_bins];
    int b = 0;
    for (int k = 0; k <= n_out; ++k) {
      const double u = u_in ? (double)u_in[(int64_t)r * (n_out + 1) + k] : (double)k / n_out;
      const double up = u * Fn;
      int i = 0; /* largest i in [0, n] with F_i <= u' */
      for (int j = 1; j <= n_bins; ++j)
        if (F[j] <= up) i = j;
      for (int j = 1; j < n_bins; ++j)
        if (fabs(up - F[j]) <= 1e-5 * Fn) b = 1;
      double t;
      if (i == n_bins) {
        t = (double)e[n_bins];
      } else if (mode == 2 && !uniform) {
        /* density constant in the bin: T(t) = exp(-P_i - sigma_i (t - e_i));
           solve 1 - T(t) = u' exactly, kept inside the bin against rounding */
        t = (double)e[i] + (-log1p(-up) - P[i]) / (double)v[i];
        if (t < (double)e[i]) t = (double)e[i];
        if (t > (double)e[i + 1]) t = (double)e[i + 1];
      } else { /* F_i <= u' < F_{i+1}: linear in the bin */
        t = (double)e[i] + (up - F[i]) / (F[i + 1] - F[i]) * ((double)e[i + 1] - (double)e[i]);
      }
      out_edges[(int64_t)r * (n_out + 1) + k] = t;
      if (out_bin) out_bin[(int64_t)r * (n_out + 1) + k] = i;
    }
    if (band) band[r] = b;
    free(F);
  }
}

/* ------------------------------------------------------------------------- */
/* Analytic stand-in radiance field (not part of the paper's method; it plays
 * the user's NeRF of Algorithm 1).  Parameter layout as documented in the
 * scenes module: [0] n_blobs, [1] peak, [2] width, [3] shell flag, [4] shell
 * radius, [5] shell width, [6] shell peak, [7:16] A, [16:19] b, [19:28] A2,
 * [28:31] b2, [32:] centres.
 *   sigma_blob = sum_b peak exp(-|x - c_b|^2/(2 w^2))
 *   sigma_shell = shell_peak exp(-(|x| - R)^2/(2 ws^2))
 *   rgb = (sigma_blob sig(Ax+b) + sigma_shell sig(A2 x/|x| + b2))/(sigma_blob+sigma_shell)
 * (rgb = sig(Ax+b) when the total density is zero).                          */
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

EXPORT void oracle_field(int64_t n, const double* x, const double* p, double* sigma, double* rgb) {
  const int nb = (int)p[0];
  const double peak = p[1], wdt = p[2];
  const int shell = p[3] != 0.0;
  const double R = p[4], ws = p[5], speak = p[6];
  const double* A = p + 7;
  const double* bb = p + 16;
  const double* A2 = p + 19;
  const double* b2 = p + 28;
  const double* cen = p + 32;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double* xi = x + 3 * i;
    double sb = 0.0;
    for (int b = 0; b < nb; ++b) {
      double r2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        double dd = xi[a] - cen[3 * b + a];
        r2 += dd * dd;
      }
      sb += peak * exp(-r2 / (2.0 * wdt * wdt));
    }
    double ss = 0.0, nrm = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    if (shell) {
      double g = nrm - R;
      ss = speak * exp(-g * g / (2.0 * ws * ws));
    }
    double cb[3], cs[3];
    for (int c = 0; c < 3; ++c) {
      double z = bb[c], z2 = b2[c];
      for (int a = 0; a < 3; ++a) {
        z += A[3 * c + a] * xi[a];
        z2 += A2[3 * c + a] * (nrm > 0 ? xi[a] / nrm : 0.0);
      }
      cb[c] = sigmoid(z);
      cs[c] = sigmoid(z2);
    }
    const double tot = sb + ss;
    sigma[i] = tot;
    for (int c = 0; c < 3; ++c)
      rgb[3 * i + c] = (tot > 0.0) ? (sb * cb[c] + ss * cs[c]) / tot : cb[c];
  }
}

EXPORT int32_t oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads the loops over rays use from now on (timing of the oracle with one
 * thread and with all cores; no effect on any result). */
EXPORT void oracle_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/*
 * Update of the occupancy-grid estimator (Section 3.1 "Spatial Skipping";
 * the update column of Table 1's occupancy-grid row): the density cached per
 * cell is blended with the radiance field's density at a point of the cell by
 * an exponential moving average over updates,
 *   D_c <- gamma D_c + (1 - gamma) sigma_c,
 * and the cell is occupied iff D_c > tau (the binarisation of the estimator).
 *
 * Cells are indexed as the grid's bits: level-major, i = x + res (y + res z).
 * The point of cell (x, y, z) on level l is
 *   bmin_l + (index + u) * (2 h0 2^l / res),   u in [0, 1)^3,
 * with u = (1/2, 1/2, 1/2) (the cell centre) when no jitter is given.
 */
EXPORT void oracle_grid_points(int32_t res, int32_t n_levels, const float* center, double h0,
                               const float* u, double* out) {
  const int64_t n_cell = (int64_t)res * res * res;
  for (int l = 0; l < n_levels; ++l) {
    const double h = h0 * (double)(1 << l);
    const double cs = 2.0 * h / res;
    for (int64_t i = 0; i < n_cell; ++i) {
      const int64_t c = (int64_t)l * n_cell + i;
      const int64_t idx[3] = {i % res, (i / res) % res, i / ((int64_t)res * res)};
      for (int a = 0; a < 3; ++a) {
        const double ua = u ? (double)u[3 * c + a] : 0.5;
        out[3 * c + a] = ((double)center[a] - h) + ((double)idx[a] + ua) * cs;
      }
    }
  }
}

/* Cell points of a grid over contracted space: the cell point in [-2, 2]^3
 * mapped back through the contraction (inverse radius 1 / (2 - r) for
 * 1 < r < 2), scaled and centred; cells with r >= 2 go 1e4 scale out.      */
EXPORT void oracle_grid_points_contracted(int32_t res, const float* center, double scale,
                                          const float* u, double* out) {
  const int64_t n = (int64_t)res * res * res;
  const double cs = 4.0 / res;
  for (int64_t c = 0; c < n; ++c) {
    const int64_t idx[3] = {c % res, (c / res) % res, c / ((int64_t)res * res)};
    double z[3];
    for (int a = 0; a < 3; ++a) z[a] = -2.0 + ((double)idx[a] + (u ? (double)u[3 * c + a] : 0.5)) * cs;
    const double r = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    const double f = r <= 1.0 ? 1.0 : (r < 2.0 ? 1.0 / ((2.0 - r) * r) : 1.0e4 / r);
    for (int a = 0; a < 3; ++a) out[3 * c + a] = (double)center[a] + z[a] * f * scale;
  }
}

EXPORT void oracle_grid_ema(int64_t n, double* density, const double* sigma, double gamma,
                            double tau, uint8_t* occupied) {
  for (int64_t c = 0; c < n; ++c) {
    density[c] = gamma * density[c] + (1.0 - gamma) * sigma[c];
    occupied[c] = density[c] > tau;
  }
}
