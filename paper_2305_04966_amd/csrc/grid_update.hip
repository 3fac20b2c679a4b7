// Update of the occupancy-grid estimator (Section 3.1 "Spatial Skipping";
// Table 1, occupancy-grid row, update column): an exponential moving average
// of the radiance field's density at one point per cell, binarised at a
// threshold into the grid the marcher reads.
#include "txs_common.h"

namespace txs {
namespace {

// point of every cell: bmin_l + (index + u) * cell size, u = 1/2 without jitter
__global__ __launch_bounds__(256) void grid_points_kernel(int32_t res, int32_t n_levels,
                                                          float cx, float cy, float cz, float h0,
                                                          const float* __restrict__ u,
                                                          float* __restrict__ out) {
  const int64_t n_cell = (int64_t)res * res * res;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell * n_levels) return;
  const int l = (int)(c / n_cell);
  const int64_t i = c - (int64_t)l * n_cell;
  const float h = h0 * (float)(1 << l);
  const float cs = 2.0f * h / (float)res;
  const int64_t idx[3] = {i % res, (i / res) % res, i / ((int64_t)res * res)};
  const float ctr[3] = {cx, cy, cz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float ua = u ? u[3 * c + a] : 0.5f;
    out[3 * c + a] = (ctr[a] - h) + ((float)idx[a] + ua) * cs;
  }
}

// point of every cell of a grid over contracted space: the cell point
// z = -2 + (index + u) * 4 / res, mapped back through the contraction
// (|z| <= 1: unchanged; 1 < |z| < 2: radius 1 / (2 - |z|)), scaled and
// centred.  Cells with |z| >= 2 have no preimage (no sample ever reads them):
// their point is put kFar scene units out along z.
constexpr float kFar = 1.0e4f;

__global__ __launch_bounds__(256) void grid_points_contracted_kernel(
    int32_t res, float cx, float cy, float cz, float scale, const float* __restrict__ u,
    float* __restrict__ out) {
  const int64_t n = (int64_t)res * res * res;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int64_t idx[3] = {c % res, (c / res) % res, c / ((int64_t)res * res)};
  const float cs = 4.0f / (float)res;
  float z[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) z[a] = -2.0f + ((float)idx[a] + (u ? u[3 * c + a] : 0.5f)) * cs;
  const float r = sqrtf(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
  const float f = r <= 1.0f ? 1.0f : (r < 2.0f ? 1.0f / ((2.0f - r) * r) : kFar / r);
  const float ctr[3] = {cx, cy, cz};
#pragma unroll
  for (int a = 0; a < 3; ++a) out[3 * c + a] = ctr[a] + z[a] * f * scale;
}

// D <- gamma D + (1 - gamma) sigma; bit c of the grid = D_c > tau.  One lane
// per cell; a wave's 64 decisions become two grid words by ballot.
__global__ __launch_bounds__(256) void grid_ema_kernel(int64_t n, float* __restrict__ density,
                                                       const float* __restrict__ sigma,
                                                       float gamma, float tau,
                                                       uint32_t* __restrict__ bits) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool occ = false;
  if (c < n) {
    const float d = gamma * density[c] + (1.0f - gamma) * sigma[c];
    density[c] = d;
    occ = d > tau;
  }
  const uint64_t m = __ballot(occ);
  const int64_t c0 = c - lane();  // first cell of this wave (multiple of 64)
  if (lane() == 0 && c0 < n) bits[c0 >> 5] = (uint32_t)m;
  if (lane() == 32 && c < n) bits[c0 >> 5 | 1] = (uint32_t)(m >> 32);
}

// Brick occupancy of the grid (the march's empty-space skipping): bricks of
// 8^3 cells, per level a plain array (some cell of the brick occupied), a
// block array (some cell of the 2x2x2 bricks starting at the brick occupied)
// and the number of occupied bricks.
constexpr int kBrickShift = 3;

__global__ __launch_bounds__(256) void clear_words_kernel(int64_t n, uint32_t* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 0u;
}

// One thread per brick: the OR of its 64 rows of 8 cells (8-aligned runs of
// x, so each row is one byte of one grid word); an occupied brick sets its
// plain bit and the block bit of every brick whose 2x2x2 block holds it.
// Integer OR is order-independent, so the result is deterministic.
__global__ __launch_bounds__(256) void coarsen_kernel(const uint32_t* __restrict__ bits,
                                                      int32_t res_shift, int32_t n_levels,
                                                      int64_t half_words,
                                                      uint32_t* __restrict__ coarse) {
  const int cs = res_shift - kBrickShift;
  const int64_t per_level = (int64_t)1 << (3 * cs);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per_level * n_levels) return;
  const int l = (int)(i >> (3 * cs));
  const int64_t j = i & (per_level - 1);
  const int cmask = (1 << cs) - 1;
  const int bx = (int)(j & cmask), by = (int)((j >> cs) & cmask), bz = (int)(j >> (2 * cs));
  const int64_t cells = (int64_t)1 << (3 * res_shift);
  const uint32_t* lv = bits + ((l * cells) >> 5);
  uint32_t any = 0u;
  for (int z = 0; z < 8; ++z)
    for (int y = 0; y < 8; ++y) {
      const int64_t c = ((int64_t)(8 * bx)) |
                        ((((int64_t)(8 * by + y)) | ((int64_t)(8 * bz + z) << res_shift))
                         << res_shift);
      any |= (lv[c >> 5] >> (c & 31)) & 0xffu;
    }
  if (!any) return;
  uint32_t* plain = coarse + l * (2 * half_words + 1);
  uint32_t* block = plain + half_words;
  atomicOr(&plain[j >> 5], 1u << (j & 31));
  atomicAdd(&block[half_words], 1u);  // the level's count of occupied bricks
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int x = bx - dx, y = by - dy, z = bz - dz;
        if (x < 0 || y < 0 || z < 0) continue;
        const int64_t k = x | ((y | ((int64_t)z << cs)) << cs);
        atomicOr(&block[k >> 5], 1u << (k & 31));
      }
}

}  // namespace
}  // namespace txs

extern "C" int64_t txs_grid_coarse_words(int32_t res) {
  if (res < 8 || res > 1024 || (res & (res - 1)) != 0) return 0;
  const int64_t b = (int64_t)(res / 8) * (res / 8) * (res / 8);
  return 2 * ((b + 31) / 32) + 1;
}

extern "C" txs_status txs_grid_coarsen(const txs_grid* grid, uint32_t* coarse, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(grid && grid->bits && coarse, "txs_grid_coarsen: null pointer");
  const int res = grid->res;
  TXS_REQUIRE(res >= 8 && res <= 1024 && (res & (res - 1)) == 0,
              "txs_grid_coarsen: res must be a power of two in [8,1024], got %d", res);
  TXS_REQUIRE(grid->n_levels >= 1 && grid->n_levels <= 8, "txs_grid_coarsen: bad n_levels");
  const int64_t words = txs_grid_coarse_words(res) * grid->n_levels;
  hipLaunchKernelGGL(clear_words_kernel, dim3(grid_1d(words, 256)), dim3(256), 0,
                     as_stream(stream), words, coarse);
  const int shift = __builtin_ctz((unsigned)res);
  const int64_t bricks = ((int64_t)1 << (3 * (shift - kBrickShift))) * grid->n_levels;
  hipLaunchKernelGGL(coarsen_kernel, dim3(grid_1d(bricks, 256)), dim3(256), 0,
                     as_stream(stream), grid->bits, shift, grid->n_levels,
                     (txs_grid_coarse_words(res) - 1) / 2, coarse);
  return launch_status("txs_grid_coarsen");
}

extern "C" txs_status txs_grid_points(const txs_grid* grid, const float* u, float* points,
                                      void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(grid, "txs_grid_points: null grid");
  const int res = grid->res;
  TXS_REQUIRE(res >= 2 && res <= 1024 && (res & (res - 1)) == 0,
              "txs_grid_points: res must be a power of two in [2,1024], got %d", res);
  TXS_REQUIRE(grid->n_levels >= 1 && grid->n_levels <= 8, "txs_grid_points: bad n_levels");
  TXS_REQUIRE(grid->half_extent0 > 0.0f, "txs_grid_points: bad half_extent0");
  TXS_REQUIRE(points, "txs_grid_points: null points");
  const int64_t n = (int64_t)res * res * res * grid->n_levels;
  hipLaunchKernelGGL(grid_points_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, as_stream(stream),
                     res, grid->n_levels, grid->center[0], grid->center[1], grid->center[2],
                     grid->half_extent0, u, points);
  return launch_status("txs_grid_points");
}

extern "C" txs_status txs_grid_ema(int64_t n_cells, float* density, const float* sigma,
                                   float gamma, float tau, uint32_t* bits, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_cells >= 0 && n_cells % 32 == 0, "txs_grid_ema: n_cells must be a multiple of 32");
  TXS_REQUIRE(gamma >= 0.0f && gamma <= 1.0f, "txs_grid_ema: gamma must be in [0,1]");
  if (n_cells == 0) return TXS_OK;
  TXS_REQUIRE(density && sigma && bits, "txs_grid_ema: null array");
  hipLaunchKernelGGL(grid_ema_kernel, dim3(grid_1d(n_cells, 256)), dim3(256), 0,
                     as_stream(stream), n_cells, density, sigma, gamma, tau, bits);
  return launch_status("txs_grid_ema");
}

extern "C" txs_status txs_grid_points_contracted(const txs_grid* grid, float contract_scale,
                                                 const float* u, float* points, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(grid, "txs_grid_points_contracted: null grid");
  const int res = grid->res;
  TXS_REQUIRE(res >= 2 && res <= 1024 && (res & (res - 1)) == 0,
              "txs_grid_points_contracted: res must be a power of two in [2,1024], got %d", res);
  TXS_REQUIRE(contract_scale > 0.0f, "txs_grid_points_contracted: contract_scale must be > 0");
  TXS_REQUIRE(points, "txs_grid_points_contracted: null points");
  const int64_t n = (int64_t)res * res * res;
  hipLaunchKernelGGL(grid_points_contracted_kernel, dim3(grid_1d(n, 256)), dim3(256), 0,
                     as_stream(stream), res, grid->center[0], grid->center[1], grid->center[2],
                     contract_scale, u, points);
  return launch_status("txs_grid_points_contracted");
}
