// Test-only build of the library's marching core for the host CPU, so that its
// DDA can be compared with the oracle's dense lattice test without a GPU.  It
// includes the product source unchanged and adds one C entry point.
#include "../../paper_2305_04966_amd/csrc/march.hip"

extern "C" int host_march(const float* o, const float* d, int32_t n, const uint32_t* bits,
                          int32_t res, int32_t n_levels, const float* center, float h0,
                          float near_plane, float far_plane, float dt0, int32_t max_per_ray,
                          int32_t* counts, const int64_t* offsets, int64_t capacity, float* t0,
                          float* t1) {
  txs_grid grid{bits, res, n_levels, {center[0], center[1], center[2]}, h0};
  txs_march_params p{near_plane, far_plane, dt0, max_per_ray};
  txs::MarchArgs g;
  if (txs::make_args(&grid, &p, g) != TXS_OK) return -1;
  for (int32_t r = 0; r < n; ++r) {
    txs::Emit em{t0, t1, nullptr, offsets ? offsets[r] : 0, capacity, r};
    if (offsets)
      counts[r] = txs::march_ray<true>(g, o + 3 * r, d + 3 * r, em);
    else
      counts[r] = txs::march_ray<false>(g, o + 3 * r, d + 3 * r, em);
  }
  return 0;
}
