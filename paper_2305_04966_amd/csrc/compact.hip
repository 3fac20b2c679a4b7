// Combined estimator plumbing (Section 3.3, "Insights from Unified
// Formulation"; Section 4.4, "Combined Sampling"): the occupancy grid removes the
// rays that cross no occupied cell and shrinks every other ray's interval to
// its occupied span; the proposal network then bins only that span
// (txs_span_bins, beside the uniform bins).  These kernels move per-ray rows
// between the full ray set and the compacted set of rays that hit.
//
// A compaction table is the exclusive scan of 0/1 hit flags, packed as
// (slot, flag) pairs: ray r with flag 1 owns row `slot` of the compacted set.
#include "txs_common.h"

namespace txs {
namespace {

// thread per (ray, word): dst[slot_r] = src[r] for rays that hit
__global__ __launch_bounds__(256) void compact_kernel(int64_t total, int32_t width,
                                                      const int32_t* __restrict__ info,
                                                      const uint32_t* __restrict__ src,
                                                      uint32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / width;
  const int32_t c = (int32_t)(i - r * width);
  if (info[2 * r + 1] > 0) dst[(int64_t)info[2 * r] * width + c] = src[i];
}

// thread per (ray, word): dst[r] = src[slot_r] for rays that hit, else fill
__global__ __launch_bounds__(256) void expand_kernel(int64_t total, int32_t width,
                                                     const int32_t* __restrict__ info,
                                                     const float* __restrict__ src, float fill,
                                                     float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / width;
  const int32_t c = (int32_t)(i - r * width);
  dst[i] = info[2 * r + 1] > 0 ? src[(int64_t)info[2 * r] * width + c] : fill;
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_compact_rows(int32_t n_rays, const int32_t* table, int32_t width,
                                       const void* src, void* dst, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && width >= 1 && width <= 64, "txs_compact_rows: bad size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(table && src && dst, "txs_compact_rows: null array");
  const int64_t total = (int64_t)n_rays * width;
  hipLaunchKernelGGL(compact_kernel, dim3(grid_1d(total, 256)), dim3(256), 0, as_stream(stream),
                     total, width, table, static_cast<const uint32_t*>(src),
                     static_cast<uint32_t*>(dst));
  return launch_status("txs_compact_rows");
}

extern "C" txs_status txs_expand_rows(int32_t n_rays, const int32_t* table, int32_t width,
                                      const float* src, float fill, float* dst, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && width >= 1 && width <= 64, "txs_expand_rows: bad size");
  if (n_rays == 0) return TXS_OK;
  TXS_REQUIRE(table && dst, "txs_expand_rows: null array");
  const int64_t total = (int64_t)n_rays * width;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_1d(total, 256)), dim3(256), 0, as_stream(stream),
                     total, width, table, src, fill, dst);
  return launch_status("txs_expand_rows");
}
