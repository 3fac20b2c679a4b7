/*
 * txs.h -- C ABI of the MI355X (gfx950) library for transmittance-estimator
 * ray sampling and packed volume rendering.
 *
 * The method follows Li, Gao, Tancik, Kanazawa, "NerfAcc: Efficient Sampling
 * Accelerates NeRFs" (2023): every sampler is an estimator of transmittance T,
 * whose complement 1 - T is the CDF used for importance sampling (Section 3.1,
 * Eqs. 1-3); samples are intervals (t0, t1, ray) stored in packed tensors with
 * a per-ray (start, count) table (Section 4.2); samples with T < 1e-4 are
 * dropped before the differentiable pass (Section 4.2, "No Gradient
 * Filtering").  Algorithm 1 of the paper is the call sequence this ABI serves:
 * sample (march -> field density -> filter), render forward, render backward,
 * estimator update.
 *
 * Conventions for every entry point
 *  - Array pointers are DEVICE pointers owned by the caller; the library never
 *    allocates or frees them and keeps no reference after the call returns.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = the default stream)
 *    and is asynchronous: no entry point synchronises the device.
 *  - Return value: TXS_OK (0) or a negative txs_status.  On error nothing is
 *    enqueued and txs_last_error() returns a message (thread-local).  No C++
 *    exception crosses the ABI.
 *  - Results are bitwise deterministic run to run (no floating-point atomics).
 *  - Layouts: float = IEEE binary32, rows are contiguous (row-major), "[N,3]"
 *    means 3 consecutive floats per row.  packed_info is int32 [n_rays, 2]
 *    = (start, count); starts are non-decreasing and the ray segments
 *    [start, start+count) do not overlap (gaps between them are allowed).
 *  - Sample counts are int64 on the host side; packed starts are int32, so a
 *    packed tensor holds fewer than 2^31 samples (TXS_EOVERFLOW otherwise).
 */
#ifndef TXS_H_
#define TXS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t txs_status;
#define TXS_OK 0
#define TXS_EINVAL (-1)    /* bad argument (null pointer, size, layout) */
#define TXS_ECAPACITY (-2) /* an output buffer is smaller than required */
#define TXS_EHIP (-3)      /* a HIP runtime call or kernel launch failed */
#define TXS_EOVERFLOW (-4) /* a count does not fit the int32 packed layout */

#define TXS_ABI_VERSION 2

/* Message of the last error on the calling thread ("" if none). */
const char* txs_last_error(void);
int32_t txs_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Occupancy grid (the spatial-skipping estimator of Section 3.1 and Table 1,
 * second row).  Level l is the cube center +- half_extent0 * 2^l, divided into
 * res^3 cells; its occupancy bits start at bit l*res^3 of `bits`; the bit of
 * cell (x, y, z) is bit (i & 31) of word i >> 5 with i = x + res*(y + res*z).
 * n_levels > 1 is the cascade used for unbounded scenes (Section 3.2): each
 * level doubles the extent and the marching step.
 *
 * `coarse` (nullable) is the brick occupancy that lets the march skip empty
 * space (the point of the spatial-skipping estimator, Section 3.1): bricks of
 * 8^3 cells, cb = res/8 per axis, brick (bx, by, bz) holding the cells
 * [8bx, 8bx+8) x [8by, 8by+8) x [8bz, 8bz+8).  Per level
 * txs_grid_coarse_words(res) words: two bit arrays of h = ceil(cb^3 / 32)
 * words each, brick index j = bx + cb (by + cb bz), bit (j & 31) of word
 * j >> 5 -- first "some cell of the brick is occupied", then "some cell of
 * the 2x2x2 bricks (bx..bx+1, by..by+1, bz..bz+1) is occupied" -- then one
 * word holding the number of occupied bricks.  txs_grid_coarsen writes it
 * from `bits`; it must describe the current bits (rebuild it after every
 * change of bits), or the march may skip occupied cells.  NULL: every
 * lattice point is tested.                                                   */
typedef struct {
  const uint32_t* bits; /* device, n_levels * res^3 / 32 words */
  int32_t res;          /* cells per axis: a power of two in [2, 1024] */
  int32_t n_levels;     /* 1 .. 8 */
  float center[3];
  float half_extent0;   /* > 0 */
  const uint32_t* coarse; /* device, n_levels * txs_grid_coarse_words(res) words, or NULL */
} txs_grid;

/*
 * Words of brick occupancy per level for a grid of res cells per axis:
 * 2 * ceil((res/8)^3 / 32) + 1, or 0 for res < 8 (no bricks).
 */
int64_t txs_grid_coarse_words(int32_t res);

/*
 * Writes the brick occupancy of grid->bits into `coarse` (device,
 * n_levels * txs_grid_coarse_words(res) words; grid->coarse is not read).
 * res >= 8.
 */
txs_status txs_grid_coarsen(const txs_grid* grid, uint32_t* coarse, void* stream);

typedef struct {
  float near_plane; /* rays start at max(near_plane, box entry); >= 0 */
  float far_plane;  /* and end at min(far_plane, box exit); may be +inf */
  float dt0;        /* lattice step on level 0 (> 0); level l uses dt0 * 2^l */
  int32_t max_per_ray; /* keep at most this many samples per ray; 0 = no cap */
} txs_march_params;

/*
 * Occupancy-grid marching (Section 3.1 "Spatial Skipping"; Section 4.2
 * "Sample as Interval").  For each ray, each constant-level segment [a, b)
 * of its chord through the grid carries the lattice t_k = a + k*dt
 * (midpoints m_k = a + (k+1/2)*dt < b); sample k is emitted iff the cell that
 * holds o + m_k*d is occupied, as the interval [t_k, min(a+(k+1)*dt, b)].
 * The occupancy test is evaluated in binary32 with the fixed operation order
 *   m = a + ((float)k + 0.5f)*dt,  u = ((o + m*d) - bmin) * (res / (bmax - bmin)),
 *   cell = clamp(floor(u), 0, res-1)
 * (no fused multiply-add), so the emitted samples are a deterministic
 * function of the inputs that any binary32 evaluation of the same recipe at
 * every lattice point reproduces bit for bit.
 *
 * Empty-space skipping: with grid->coarse set (res >= 8 and at most 1088
 * words of brick occupancy over all levels, so that a wave holds it in LDS:
 * up to four 128^3 levels; otherwise it is ignored), on segments of more than
 * 256 lattice points of levels with at most 5/16 of their bricks occupied,
 * runs of 16 lattice points are first bounded in cell space from their end
 * points (with a margin that covers every rounding of the recipe) and
 * skipped when every brick the bound touches is empty; the points of the
 * other runs are tested one by one.  Other segments test every point.  The
 * emitted samples are those of testing every point either way.
 *
 * txs_march_count writes counts[n_rays] (int32).
 * rays_o, rays_d: float [n_rays, 3]; rays_d need not be normalised (the
 * paper's rays are unit vectors; t is measured in units of |d|).
 */
txs_status txs_march_count(const txs_grid* grid, const txs_march_params* params,
                           const float* rays_o, const float* rays_d, int32_t n_rays,
                           int32_t* counts, void* stream);

/*
 * Exclusive scan of per-ray counts into the packed table (Section 4.2,
 * "Packed Tensor"): packed_info[r] = (sum_{q<r} counts[q], counts[r]) and
 * *d_total (device int64) = sum of all counts.  The scan runs on the device,
 * so it cannot refuse a total it has not yet computed: a row whose end
 * start + count would pass INT32_MAX is written as the empty row
 * (INT32_MAX, 0), which every entry point of this library reads as a ray
 * with no samples, while *d_total stays the exact int64 sum.  The caller reads
 * *d_total (the one host read of a sampling pass) and treats a total
 * >= 2^31 as TXS_EOVERFLOW before sizing the packed tensors.  workspace:
 * device scratch of at least txs_scan_workspace_size(n_rays) bytes (contents
 * need not be zero).
 */
size_t txs_scan_workspace_size(int32_t n_rays);
txs_status txs_exclusive_scan(const int32_t* counts, int32_t n_rays, int32_t* packed_info,
                              int64_t* d_total, void* workspace, size_t workspace_bytes,
                              void* stream);

/*
 * Allocation-free variant of txs_exclusive_scan, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments minus the workspace, same
 * results bit for bit.  Its tile sums live in a fixed device array of the
 * library (128 KiB, one copy per GPU, held until the process ends), so
 * n_rays <= txs_exclusive_scan_noalloc_max_rays() (2^26); larger inputs return
 * TXS_ECAPACITY.  The call allocates nothing.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller; calls on one stream are ordered.
 */
int32_t txs_exclusive_scan_noalloc_max_rays(void);
txs_status txs_exclusive_scan_noalloc(const int32_t* counts, int32_t n_rays,
                                      int32_t* packed_info, int64_t* d_total, void* stream);

/*
 * Second marching pass: writes the samples of ray r at packed_info[r].start,
 * ray-major and t-ascending: t0, t1 (float [capacity]) and ray_id (int32
 * [capacity], may be NULL).  packed_info must come from counts produced by
 * txs_march_count with the same grid, params and rays.  No write goes at or
 * beyond `capacity` samples, nor past packed_info[r].count samples of ray r
 * (a row with a negative start or count is written as empty).
 */
txs_status txs_march_fill(const txs_grid* grid, const txs_march_params* params,
                          const float* rays_o, const float* rays_d, int32_t n_rays,
                          const int32_t* packed_info, int64_t capacity, float* t0, float* t1,
                          int32_t* ray_id, void* stream);

/*
 * Grid estimator over contracted space (a variant for unbounded scenes, next
 * to the cascade of nested cubes; Section 3.2, "Handling Unbounded Scenes",
 * leaves the parameterisation of far space to the works it cites, of which
 * Mip-NeRF 360's contraction is one): the same lattice,
 * segments, steps, outputs and errors as txs_march_count / txs_march_fill,
 * but the occupancy of a sample is read from ONE grid of res^3 bits
 * (grid->bits, x fastest) covering the contracted cube [-2, 2]^3 around
 * grid->center.  The midpoint x of a sample maps, in binary32 and in this
 * order, to
 *   y  = (x - center) * s,  s = 1 / contract_scale (one rounding),
 *   r2 = y0 y0 + y1 y1 + y2 y2;  if r2 > 1: r = sqrt(r2), q = 1 / r,
 *        y = y * ((2 - q) * q)   (Mip-NeRF 360's contraction into radius 2),
 *   cell_c = clamp(floor((y_c + 2) * (res / 4)), 0, res - 1),
 * with correctly rounded division and square root.  grid->n_levels and
 * grid->half_extent0 still define the cubes whose segments set the lattice
 * steps (dt0 2^l on level l); contract_scale > 0.
 */
txs_status txs_march_count_contracted(const txs_grid* grid, const txs_march_params* params,
                                      float contract_scale, const float* rays_o,
                                      const float* rays_d, int32_t n_rays, int32_t* counts,
                                      void* stream);
txs_status txs_march_fill_contracted(const txs_grid* grid, const txs_march_params* params,
                                     float contract_scale, const float* rays_o,
                                     const float* rays_d, int32_t n_rays,
                                     const int32_t* packed_info, int64_t capacity, float* t0,
                                     float* t1, int32_t* ray_id, void* stream);

/*
 * No-gradient filtering (Section 4.2): with tau_i = sigma_i (t1_i - t0_i) and
 * T_i = exp(-sum_{j<i} tau_j) over the samples of a ray, kept_counts[r] is
 * the number of leading samples with T_i >= t_min (the paper uses 1e-4).
 * T is non-increasing, so the kept samples are a prefix of the ray.  The
 * decision is taken in binary64: the optical depth sum_{j<i} tau_j is summed
 * in binary64 from the binary32 tau_j = sigma_j (t1_j - t0_j) and compared
 * with -log((double)t_min); sample i is kept iff it is <= that bound.
 * sigma: float [n_samples] (density from the radiance field, no gradient).
 * TXS_EOVERFLOW if n_samples >= 2^31.
 */
txs_status txs_transmittance_prefix(const int32_t* packed_info, int32_t n_rays,
                                    int64_t n_samples, const float* t0, const float* t1,
                                    const float* sigma, float t_min, int32_t* kept_counts,
                                    void* stream);

/*
 * Repacks the first packed_info_out[r].count samples of every ray r from the
 * input packed tensor (t0, t1: float [n_in], rows packed_info_in) to
 * packed_info_out[r].start of the output tensor: t0o, t1o (float
 * [capacity]) and ray_ido (int32 [capacity] = r, may be NULL).  A row whose
 * copy would read at or beyond n_in or write at or beyond capacity copies
 * nothing.  Typical use: packed_info_out = txs_exclusive_scan(kept_counts).
 */
txs_status txs_gather_prefix(const int32_t* packed_info_in, const int32_t* packed_info_out,
                             int32_t n_rays, int64_t n_in, const float* t0, const float* t1,
                             int64_t capacity, float* t0o, float* t1o, int32_t* ray_ido,
                             void* stream);

/*
 * Packed volume rendering forward (Eq. 2, discretised):
 *   tau_i = sigma_i (t1_i - t0_i),  T_i = exp(-sum_{j<i} tau_j),
 *   w_i = T_i (1 - exp(-tau_i)),
 *   out_rgb = sum w_i rgb_i + (1 - sum w_i) * bg,  out_opacity = sum w_i,
 *   out_depth = sum w_i (t0_i + t1_i)/2   (unnormalised expected depth).
 * packed_info may be NULL: then ray r owns samples [r*fixed_count,
 * (r+1)*fixed_count) (dense layout, e.g. proposal resampling output).
 * sigma float [n_samples], rgb float [n_samples, 3] or NULL (colour taken as
 * zero: weights, opacity and depth only), bg float [n_rays, 3] or NULL
 * (black).  Outputs: out_rgb [n_rays,3], out_opacity [n_rays],
 * out_depth [n_rays], out_weights [n_samples] or NULL, and
 * out_optical_depth double [n_rays] or NULL = sum_i tau_i per ray.
 * Optical depths are accumulated in binary64.  TXS_EOVERFLOW if
 * n_samples >= 2^31 (the same holds for txs_render_bwd and txs_weights_bwd).
 */
txs_status txs_render_fwd(const int32_t* packed_info, int32_t fixed_count, int32_t n_rays,
                          int64_t n_samples, const float* t0, const float* t1,
                          const float* sigma, const float* rgb, const float* bg,
                          float* out_rgb, float* out_opacity, float* out_depth,
                          float* out_weights, double* out_optical_depth, void* stream);

/*
 * Adjoint of txs_render_fwd (the gradients that reach the radiance field in
 * Algorithm 1; the intervals carry none, Section 4.2).  With
 *   v_i = g.(rgb_i - bg) + h + q (t0_i + t1_i)/2,
 *   d_rgb_i   = w_i g,
 *   d_sigma_i = (t1_i - t0_i) (T_{i+1} v_i - sum_{j>i} w_j v_j),
 * where g = g_rgb[r] (float [n_rays,3]), h = g_opacity[r], q = g_depth[r]
 * (both may be NULL = 0).  T and w are recomputed from the inputs; the only
 * forward state used is optical_depth (double [n_rays], the forward's
 * out_optical_depth of the same inputs), or NULL to recompute it here at the
 * cost of one more read of t0, t1, sigma.  The samples are walked last to
 * first so both suffix sums are exact reverse scans.
 * d_sigma float [n_samples], d_rgb float [n_samples,3] (may be NULL).
 * Samples outside every ray's segment (gaps between rows, or the tail of a
 * dense layout with n_rays * fixed_count < n_samples) are left unchanged:
 * a caller whose rows do not tile [0, n_samples) clears those outputs first.
 */
txs_status txs_render_bwd(const int32_t* packed_info, int32_t fixed_count, int32_t n_rays,
                          int64_t n_samples, const float* t0, const float* t1,
                          const float* sigma, const float* rgb, const float* bg,
                          const double* optical_depth, const float* g_rgb,
                          const float* g_opacity, const float* g_depth, float* d_sigma,
                          float* d_rgb, void* stream);

/*
 * Adjoint of the weights alone: given g_w[i] = dL/dw_i (float [n_samples]),
 *   d_sigma_i = (t1_i - t0_i) (T_{i+1} g_w_i - sum_{j>i} w_j g_w_j).
 * Used to train a proposal estimator through its rendering weights.
 * optical_depth as for txs_render_bwd (may be NULL).
 */
txs_status txs_weights_bwd(const int32_t* packed_info, int32_t fixed_count, int32_t n_rays,
                           int64_t n_samples, const float* t0, const float* t1,
                           const float* sigma, const double* optical_depth, const float* g_w,
                           float* d_sigma, void* stream);

/*
 * Inverse transform sampling (Eq. 1) of a piecewise-constant estimator whose
 * CDF is read off the transmittance, F = 1 - T (Eq. 3):
 *   mode TXS_PDF_SIGMA:   F_{i+1} = 1 - exp(-sum_{j<=i} vals_j (e_{j+1} - e_j))
 *   mode TXS_PDF_WEIGHTS: F_{i+1} = sum_{j<=i} vals_j
 * Per ray: u' = u * F_n, i = the largest i in [0, n_bins] with F_i <= u',
 * t = e_i + (u' - F_i) / (F_{i+1} - F_i) * (e_{i+1} - e_i)  (t = e_n if
 * i = n_bins, in particular for u = 1 even when trailing bins carry no
 * mass): the transmittance is taken linear inside a bin (Table 1).
 *   mode TXS_PDF_SIGMA_EXP: the CDF of TXS_PDF_SIGMA inverted exactly for a
 *   density constant inside each bin (T exponential there): with
 *   x = (u' - F_i) / (F_{i+1} - F_i) * (1 - exp(-tau_i)), tau_i = vals_i
 *   (e_{i+1} - e_i), t = min(e_i + (e_{i+1} - e_i) * (-log(1 - x) / tau_i),
 *   e_{i+1}).
 * A ray whose F_n <= 1e-12 uses the uniform estimator (F_i = i/n_bins,
 * Table 1, first row; linear in every mode).  u is float [n_rays, n_out+1] with
 * values in [0,1], non-decreasing per ray, or NULL for u_k = k/n_out.
 * edges float [n_rays, n_bins+1] (non-decreasing), vals float
 * [n_rays, n_bins] (>= 0); out_edges float [n_rays, n_out+1] are the
 * n_out+1 edges of n_out contiguous intervals.  n_bins <= 1024.
 */
#define TXS_PDF_SIGMA 0
#define TXS_PDF_WEIGHTS 1
#define TXS_PDF_SIGMA_EXP 2
txs_status txs_resample(int32_t n_rays, int32_t n_bins, const float* edges, const float* vals,
                        int32_t mode, int32_t n_out, const float* u, float* out_edges,
                        void* stream);

/*
 * txs_resample with the n_out intervals between consecutive output edges
 * written in the dense layout of the renderer and the field instead of the
 * edges: out_t0[r*n_out + k] = edge k, out_t1[r*n_out + k] = edge k+1
 * (float [n_rays*n_out] each).  Same arguments, rules and errors otherwise.
 */
txs_status txs_resample_intervals(int32_t n_rays, int32_t n_bins, const float* edges,
                                  const float* vals, int32_t mode, int32_t n_out, const float* u,
                                  float* out_t0, float* out_t1, void* stream);

/*
 * Uniform estimator (Table 1, first row): n_bins+1 equally spaced edges per
 * ray over its chord through the outermost cube of `grid` (bits unused),
 *   e_k = t_near + (t_far - t_near) * (k / n_bins),   out: float [n_rays, n_bins+1].
 * A ray that misses gets all edges equal to max(near_plane, 0) and t_far = t_near.
 * 1 <= n_bins <= 2^24.
 */
txs_status txs_uniform_bins(const txs_grid* grid, float near_plane, float far_plane,
                            const float* rays_o, const float* rays_d, int32_t n_rays,
                            int32_t n_bins, float* out_edges, void* stream);

/*
 * Uniform estimator in disparity: the chord of txs_uniform_bins (same clip,
 * same handling of rays that miss) split into n_bins bins of equal width in
 * 1/t, e_k = 1 / (1/t_near + (1/t_far - 1/t_near) * (k / n_bins)) in
 * binary32, with e_0 = t_near and e_n = t_far exactly: finer near the ray's
 * origin, coarser far away (the spacing Mip-NeRF 360 gives the proposal
 * network's first samples on unbounded scenes, Section 3.2 of the paper
 * cites it).  near_plane must be > 0 (1/t stays finite).
 */
txs_status txs_disparity_bins(const txs_grid* grid, float near_plane, float far_plane,
                              const float* rays_o, const float* rays_d, int32_t n_rays,
                              int32_t n_bins, float* out_edges, void* stream);

/*
 * Dense interval layout of per-ray edges (the input layout of the renderer
 * and the field for a fixed number of samples per ray): for edges float
 * [n_rays, n+1], writes t0[r*n + k] = e_k and t1[r*n + k] = e_{k+1}
 * (float [n_rays*n] each).
 */
txs_status txs_edges_to_intervals(const float* edges, int32_t n_rays, int32_t n, float* t0,
                                  float* t1, void* stream);

/*
 * Sorted union of two ascending edge rows per ray (the coarse-to-fine PDF
 * estimator of Table 1's third row, as vanilla NeRF runs it, renders its fine
 * pass on the coarse edges and the inverse-CDF edges together):
 * a float [n_rays, na], b float [n_rays, nb], out float [n_rays, na+nb], the
 * values of both rows in ascending order (stable: a before equal b).  Rows
 * must be ascending (not checked; an unsorted row leaves unspecified values in
 * its own output row and writes nothing outside it).  1 <= na, nb <= 4096.
 */
txs_status txs_merge_edges(int32_t n_rays, int32_t na, const float* a, int32_t nb, const float* b,
                           float* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Learned transmittance estimator: the proposal network (Section 3.1 "PDF
 * Approaches", Table 1 third row; Section 3.2 "Choice of Representations").
 *   x_hat = x / scale, or contract(x / scale) / 2 with contract(y) = y for
 *           |y| <= 1 and (2 - 1/|y|) y/|y| beyond (unbounded scenes)
 *   gamma = [x_hat, sin(2^k pi x_hat_a), cos(2^k pi x_hat_a)], a = 0..2, k = 0..5
 *   h1 = relu(W1 gamma + b1), h2 = relu(W2 h1 + b2), sigma = softplus(w3.h2 + b3)
 * Parameters: one float vector W1 [H,39], b1 [H], W2 [H,H], b2 [H], w3 [H], b3
 * (txs_mlp_param_count(H) values, row-major).  The matrix cores read bf16
 * operand tiles made from it by txs_mlp_pack (gamma, h1, h2 and the weights
 * are rounded to bf16, round-to-nearest-even; accumulation is fp32; biases
 * stay fp32).  H is 64 or 128.                                              */
typedef struct {
  const void* packed;  /* device, txs_mlp_packed_bytes(hidden), from txs_mlp_pack */
  const float* params; /* device, the float parameter vector (biases read here) */
  int32_t hidden;      /* 64 or 128 */
  float scale;         /* > 0 */
  int32_t contract;    /* 0: bounded scene, 1: contracted unbounded scene */
} txs_mlp;

size_t txs_mlp_param_count(int32_t hidden);
size_t txs_mlp_packed_bytes(int32_t hidden);
txs_status txs_mlp_pack(const float* params, int32_t hidden, void* packed, void* stream);

/*
 * Proposal density at the midpoints of n_bins bins per ray:
 * x = o + (e_j + e_{j+1})/2 d with edges float [n_rays, n_bins+1];
 * sigma float [n_rays, n_bins].
 */
txs_status txs_prop_mlp_fwd(const txs_mlp* mlp, const float* rays_o, const float* rays_d,
                            int32_t n_rays, int32_t n_bins, const float* edges, float* sigma,
                            void* stream);

/*
 * Adjoint of txs_prop_mlp_fwd for the estimator's update (Eq. 4): given
 * d_sigma float [n_rays, n_bins] = dL/dsigma at the same points, writes
 * grad float [txs_mlp_param_count(hidden)] = dL/dparams (overwritten, same
 * layout as params).  The forward is recomputed, not stored.  Besides the
 * forward's rounding points, dL/da2 and dL/da1 (the pre-activation adjoints of
 * the two hidden layers) are rounded to bf16 before the matrix-core products
 * that consume them; bias gradients sum those rounded values; all sums are
 * fp32, reduced in a fixed order (bitwise deterministic).
 * workspace: device, >= txs_mlp_bwd_workspace_size(hidden) bytes, caller-owned
 * scratch (per-block partial gradients); EINVAL if smaller.
 */
size_t txs_mlp_bwd_workspace_size(int32_t hidden);
txs_status txs_prop_mlp_bwd(const txs_mlp* mlp, const float* rays_o, const float* rays_d,
                            int32_t n_rays, int32_t n_bins, const float* edges,
                            const float* d_sigma, float* grad, void* workspace,
                            size_t workspace_bytes, void* stream);

/*
 * PDF-matching loss of the proposal estimator (its update by gradient descent,
 * Eq. 4 and Section 3.1 "PDF Approaches"; the proposal loss of Mip-NeRF 360,
 * on which the paper's proposal network rests).  Targets are the radiance
 * field's rendering weights on its own intervals, packed per ray
 * (packed_info, t0, t1, w; n_targets samples, sorted and disjoint per ray);
 * the proposal has n_bins dense bins per ray (edges [n_rays, n_bins+1],
 * weights prop_w [n_rays, n_bins]).  For each target interval,
 *   bound_i = sum of prop_w over the bins overlapping (t0_i, t1_i)
 *             (e_j < t1_i and e_{j+1} > t0_i),
 *   loss[r] = sum_i max(0, w_i - bound_i)^2 / (w_i + eps).
 * d_prop (may be NULL) = d(mean_r loss[r]) / d prop_w, float [n_rays, n_bins];
 * each bin sums its overlapping targets in target order (deterministic).
 * n_bins <= 1024.  TXS_EOVERFLOW if n_targets >= 2^31.
 */
txs_status txs_hist_loss(const int32_t* packed_info, int32_t n_rays, int64_t n_targets,
                         const float* t0, const float* t1, const float* w, int32_t n_bins,
                         const float* edges, const float* prop_w, float eps, float* loss,
                         float* d_prop, void* stream);

/*
 * One Adam step (Kingma & Ba 2015) on n fp32 parameters, in place:
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),  step >= 1.
 * Re-run txs_mlp_pack afterwards to refresh the bf16 operand tiles.
 */
txs_status txs_adam_step(float* params, float* m, float* v, const float* grad, int64_t n,
                         float lr, float beta1, float beta2, float eps, int32_t step,
                         void* stream);

/*
 * Support (not part of the method): an analytic radiance field standing in for
 * the user's NeRF of Algorithm 1, evaluated at interval midpoints
 * x = o[ray] + (t0+t1)/2 * d[ray]:
 *   sigma(x) = sum_b peak exp(-|x-c_b|^2/(2 w^2)) + shell_peak exp(-(|x|-R)^2/(2 ws^2))
 *   rgb(x)   = density-weighted mix of sigmoid(A x + b) and sigmoid(A2 x/|x| + b2).
 * params: device float array of 32 + 3*n_blobs values in the layout
 * [0] (unused), [1] peak, [2] width, [3] shell flag, [4] R, [5] ws,
 * [6] shell_peak, [7:16] A, [16:19] b, [19:28] A2, [28:31] b2,
 * [32:32+3*n_blobs] centres.
 * rays_o, rays_d: float [n_rays, 3].  ray_id int32 [n] or NULL with
 * fixed_count > 0 (ray = i / fixed_count); a ray index outside [0, n_rays)
 * reads ray 0.  rgb may be NULL (density only).
 */
txs_status txs_blob_field(const float* params, int32_t n_blobs, const float* rays_o,
                          const float* rays_d, int32_t n_rays, const float* t0, const float* t1,
                          const int32_t* ray_id, int32_t fixed_count, int64_t n, float* sigma,
                          float* rgb, void* stream);

/* ------------------------------------------------------------------------ */
/* Update of the occupancy-grid estimator (Section 3.1 "Spatial Skipping";
 * Table 1, occupancy-grid row, EMA update): the density cached per cell is
 * blended with the radiance field's density at one point of the cell,
 *   D_c <- gamma D_c + (1 - gamma) sigma_c,
 * and the grid bit of the cell is set iff D_c > tau.  Cells are ordered as
 * the grid's bits (level-major, i = x + res (y + res z)); n_cells =
 * n_levels res^3.  The caller evaluates its field at the points of
 * txs_grid_points and passes the densities to txs_grid_ema.
 *
 * txs_grid_points: points float [n_cells, 3], the point of cell (x, y, z) on
 * level l being bmin_l + (index + u) (2 half_extent0 2^l / res) per axis, in
 * binary32; u float [n_cells, 3] in [0, 1) (per-cell jitter) or NULL for the
 * cell centres (u = 1/2).  grid->bits is not read.
 *
 * txs_grid_ema: density float [n_cells] (in/out, the cache), sigma float
 * [n_cells], 0 <= gamma <= 1; writes the n_cells / 32 grid words of bits.
 * n_cells must be a multiple of 32 (res >= 4).  Binary32 arithmetic.
 */
txs_status txs_grid_points(const txs_grid* grid, const float* u, float* points, void* stream);

/*
 * Cell points of a grid over contracted space (the grid that
 * txs_march_count_contracted reads; update it with txs_grid_ema as any
 * other): for cell (x, y, z) of the res^3 grid over [-2, 2]^3, the point
 * z = -2 + (index + u) (4 / res) per axis, mapped back through the
 * contraction -- unchanged for |z| <= 1, radius 1 / (2 - |z|) for
 * 1 < |z| < 2 -- then scaled by contract_scale and moved to grid->center.
 * Cells with |z| >= 2 have no preimage and are never read by the march; their
 * point is placed 1e4 contract_scale out along z.  points float [res^3, 3],
 * binary32; u float [res^3, 3] in [0, 1) or NULL (cell centres).
 */
txs_status txs_grid_points_contracted(const txs_grid* grid, float contract_scale, const float* u,
                                      float* points, void* stream);
txs_status txs_grid_ema(int64_t n_cells, float* density, const float* sigma, float gamma,
                        float tau, uint32_t* bits, void* stream);

/* ------------------------------------------------------------------------ */
/* Combined estimator (Section 3.3 "Insights from Unified Formulation";
 * Section 4.4 "Combined Sampling"): the occupancy grid's transmittance comes
 * first -- rays that cross no occupied cell are dropped and every other ray is
 * narrowed to its occupied span -- and the proposal network refines inside
 * that span (uniform bins -> proposal density -> inverse CDF).
 *
 * txs_march_span: the march of txs_march_count / txs_march_fill (same grid,
 * params, recipe and errors; params->max_per_ray must be 0) without its
 * samples: span float [n_rays, 2] = (t0 of the ray's first sample, t1 of its
 * last), bit-identical to those samples' t0 and t1; hit int32 [n_rays] = 1 if
 * the ray has a sample, else 0 (and span = (0, 0)).
 *
 * Compaction table: table int32 [n_rays, 2] = txs_exclusive_scan of hit, i.e.
 * (slot_r, hit_r); the rays that hit own rows 0 .. total-1 of the compacted
 * set in ray order.
 * txs_compact_rows: dst row slot_r = src row r for every ray with hit_r = 1;
 *   rows of `width` 32-bit words (any type; 1 <= width <= 64), src
 *   [n_rays, width], dst [total, width].  Other memory is not written.
 * txs_expand_rows: dst row r = src row slot_r if hit_r, else `fill` in every
 *   word; src float [total, width] (may be NULL when total = 0), dst float
 *   [n_rays, width].
 * txs_span_bins: n_bins+1 equally spaced edges over each span,
 *   e_k = lo + (hi - lo) * (k / n_bins) in binary32 (the recipe of
 *   txs_uniform_bins), span float [n_rays, 2], out float [n_rays, n_bins+1],
 *   1 <= n_bins <= 2^24.
 */
txs_status txs_march_span(const txs_grid* grid, const txs_march_params* params,
                          const float* rays_o, const float* rays_d, int32_t n_rays, float* span,
                          int32_t* hit, void* stream);
txs_status txs_compact_rows(int32_t n_rays, const int32_t* table, int32_t width, const void* src,
                            void* dst, void* stream);
txs_status txs_expand_rows(int32_t n_rays, const int32_t* table, int32_t width, const float* src,
                           float fill, float* dst, void* stream);
txs_status txs_span_bins(int32_t n_rays, const float* span, int32_t n_bins, float* out_edges,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TXS_H_ */
