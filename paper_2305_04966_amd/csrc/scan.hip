// Packed-tensor bookkeeping (Section 4.2 "Packed Tensor"): exclusive scan of
// per-ray counts into (start, count) rows, and the prefix repack that follows
// no-gradient filtering.
#include <mutex>

#include "txs_common.h"

namespace txs {
namespace {

constexpr int kScanBlock = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kScanBlock * kPerThread;  // counts per tile
constexpr int kTopBlock = 1024;

// Block-wide exclusive scan of one int64 per thread; returns the block total.
__device__ int64_t block_exclusive_scan(int64_t& v, int64_t* lds_wave) {
  const int ln = lane(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t t = shfl_up(incl, d);
    if (ln >= d) incl += t;
  }
  if (ln == kWave - 1) lds_wave[w] = incl;
  __syncthreads();
  int64_t wave_off = 0, total = 0;
  for (int i = 0; i < nw; ++i) {
    const int64_t s = lds_wave[i];
    if (i < w) wave_off += s;
    total += s;
  }
  __syncthreads();
  v = incl - v + wave_off;
  return total;
}

// Pass 1: per-tile sums of the counts.
__global__ __launch_bounds__(kScanBlock) void tile_sums(const int32_t* __restrict__ counts,
                                                        int32_t n, int64_t* __restrict__ sums) {
  __shared__ int64_t lds[kScanBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kPerThread;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j)
    if (base + j < n) s += counts[base + j];
  const int64_t total = block_exclusive_scan(s, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass 2: one block scans the tile sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(kTopBlock) void scan_tile_sums(int64_t* sums, int32_t n_tiles,
                                                            int64_t* d_total) {
  __shared__ int64_t lds[kTopBlock / kWave];
  int64_t carry = 0;
  for (int32_t base = 0; base < n_tiles; base += kTopBlock) {
    const int32_t i = base + threadIdx.x;
    int64_t v = (i < n_tiles) ? sums[i] : 0;
    const int64_t total = block_exclusive_scan(v, lds);
    if (i < n_tiles) sums[i] = v + carry;
    carry += total;
  }
  if (threadIdx.x == 0) *d_total = carry;
}

// Pass 3: per-tile exclusive scan plus tile offset -> packed_info rows.
__global__ __launch_bounds__(kScanBlock) void write_packed(const int32_t* __restrict__ counts,
                                                           int32_t n,
                                                           const int64_t* __restrict__ offs,
                                                           int32_t* __restrict__ info) {
  __shared__ int64_t lds[kScanBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kPerThread;
  int32_t c[kPerThread];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    c[j] = (base + j < n) ? counts[base + j] : 0;
    s += c[j];
  }
  block_exclusive_scan(s, lds);
  int64_t start = s + offs[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    if (base + j < n) {
      // a row that does not end below 2^31 cannot be addressed by int32
      // starts: it is written as the empty row (INT32_MAX, 0), which keeps the
      // starts non-decreasing and leaves every consumer nothing to read or
      // write; the int64 total stays exact for the caller's overflow check
      const bool fits = start + c[j] <= (int64_t)INT32_MAX;
      info[2 * (base + j)] = fits ? (int32_t)start : INT32_MAX;
      info[2 * (base + j) + 1] = fits ? c[j] : 0;
    }
    start += c[j];
  }
}

// Repack: a wave owns 64 consecutive rays and copies the kept prefix of each
// with all lanes (contiguous loads and stores).
constexpr int kGatherWaves = 8;

// The wave's 64 rays are copied as one walk over their output positions in
// steps of kGatherSpan (kGatherUnroll chunks of 64 consecutive positions, one
// per lane): stores are contiguous and coalesced, loads contiguous within a
// ray, and the loads of a step's chunks are in flight together.  A step that
// lies inside the ray carried from the previous step (rays are hundreds of
// samples long) takes a wave-uniform path; otherwise each lane finds the ray
// of each of its positions from the ray starts that fall in the step (marked
// in LDS; inclusive max scan over lanes per chunk, the ray of a chunk's last
// position carried into the next chunk).  Rows are in ray-major order, so a
// later start belongs to a higher lane and the max is the latest ray started.
constexpr int kGatherUnroll = 8;
constexpr int kGatherSpan = kWave * kGatherUnroll;

__global__ __launch_bounds__(kWave* kGatherWaves) void gather_prefix_kernel(
    const int32_t* __restrict__ info_in, const int32_t* __restrict__ info_out, int32_t n_rays,
    int64_t n_in, const float* __restrict__ t0, const float* __restrict__ t1, int64_t capacity,
    float* __restrict__ t0o, float* __restrict__ t1o, int32_t* __restrict__ rido) {
  __shared__ int marks[kGatherWaves][kGatherSpan];
  const int ln = lane(), wv = threadIdx.x / kWave;
  const int64_t r0 = ((int64_t)blockIdx.x * kGatherWaves + wv) * kWave;
  if (r0 >= n_rays) return;
  const int64_t r = r0 + ln;
  int32_t si = 0, so = 0, cnt = 0;
  if (r < n_rays) {
    const int2 a = reinterpret_cast<const int2*>(info_in)[r];
    const int2 b = reinterpret_cast<const int2*>(info_out)[r];
    si = a.x;
    so = b.x;
    cnt = min(b.y, a.y);
    // rows that would read or write out of range copy nothing
    if (a.x < 0 || b.x < 0 || cnt < 0 || (int64_t)si + cnt > n_in ||
        (int64_t)so + cnt > capacity)
      cnt = 0;
  }
  // output span of the wave's non-empty rows
  const int64_t lo = wave_min(cnt > 0 ? (int64_t)so : INT64_MAX);
  if (lo == INT64_MAX) return;
  const int64_t hi = wave_max(cnt > 0 ? (int64_t)so + cnt : INT64_MIN);
  // ray carried into the next step (lane index, -1 none) and its row, uniform
  int cur = -1;
  int64_t c_so = 0, c_si = 0, c_end = 0;  // c_end = c_so + count
  int64_t base = lo;
  while (base < hi) {
    if (cur >= 0 && c_end > base) {
      // positions [base, end) all belong to the carried ray (wave-uniform)
      const int64_t end = min(min(c_end, hi), base + (int64_t)kGatherSpan);
      float v0[kGatherUnroll], v1[kGatherUnroll];
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        const int64_t p = base + (int64_t)kWave * u + ln;
        if (p < end) {
          const int64_t src = c_si + (p - c_so);
          v0[u] = t0[src];
          v1[u] = t1[src];
        }
      }
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        const int64_t p = base + (int64_t)kWave * u + ln;
        if (p < end) {
          t0o[p] = v0[u];
          t1o[p] = v1[u];
          if (rido) rido[p] = (int32_t)(r0 + cur);
        }
      }
      base = end;
      continue;
    }
    // a step where rays start (or a gap): ray of each position by lane scans
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) marks[wv][kWave * u + ln] = -1;
    wave_sync();
    {
      const int64_t d = (int64_t)so - base;
      if (cnt > 0 && d >= 0 && d < kGatherSpan) marks[wv][d] = ln;
    }
    wave_sync();
    int m[kGatherUnroll];
    int carry = cur;
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      int mu = max_scan_incl(marks[wv][kWave * u + ln]);
      if (mu < 0) mu = carry;
      m[u] = mu;
      carry = readlane(mu, kWave - 1);
    }
    float v0[kGatherUnroll], v1[kGatherUnroll];
    bool ok[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int q = m[u] < 0 ? 0 : m[u];
      const int32_t so_r = __shfl(so, q, kWave), si_r = __shfl(si, q, kWave),
                    c_r = __shfl(cnt, q, kWave);
      const int64_t p = base + (int64_t)kWave * u + ln;
      ok[u] = m[u] >= 0 && p < (int64_t)so_r + c_r;
      if (ok[u]) {
        const int64_t src = (int64_t)si_r + (p - so_r);
        v0[u] = t0[src];
        v1[u] = t1[src];
      }
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int64_t p = base + (int64_t)kWave * u + ln;
      if (ok[u]) {
        t0o[p] = v0[u];
        t1o[p] = v1[u];
        if (rido) rido[p] = (int32_t)(r0 + m[u]);
      }
    }
    // carry the ray of the step's last position
    cur = carry;
    if (cur >= 0) {
      c_so = readlane(so, cur);
      c_si = readlane(si, cur);
      c_end = c_so + readlane(cnt, cur);
    }
    wave_sync();
    base += kGatherSpan;
  }
}

}  // namespace
}  // namespace txs

extern "C" size_t txs_scan_workspace_size(int32_t n_rays) {
  const int64_t tiles = n_rays > 0 ? ((int64_t)n_rays + txs::kTile - 1) / txs::kTile : 1;
  return (size_t)tiles * sizeof(int64_t);
}

namespace txs {
namespace {

// The three passes of the scan, with the tile sums in `sums` (one int64 per
// tile of kTile counts; every pass-1 tile overwrites its own entry, so the
// buffer needs no clearing).
void launch_scan(const int32_t* counts, int32_t n_rays, int32_t* packed_info, int64_t* d_total,
                 int64_t* sums, hipStream_t s) {
  const int32_t tiles = (int32_t)((int64_t)std::max<int32_t>(n_rays, 1) + kTile - 1) / kTile;
  if (n_rays > 0)
    hipLaunchKernelGGL(tile_sums, dim3(tiles), dim3(kScanBlock), 0, s, counts, n_rays, sums);
  else
    hipLaunchKernelGGL(tile_sums, dim3(1), dim3(kScanBlock), 0, s, counts, 0, sums);
  hipLaunchKernelGGL(scan_tile_sums, dim3(1), dim3(kTopBlock), 0, s, sums, tiles, d_total);
  if (n_rays > 0)
    hipLaunchKernelGGL(write_packed, dim3(tiles), dim3(kScanBlock), 0, s, counts, n_rays, sums,
                       packed_info);
}

txs_status check_scan_args(const char* who, const int32_t* counts, int32_t n_rays,
                           const int32_t* packed_info, const int64_t* d_total) {
  TXS_REQUIRE(n_rays >= 0, "%s: n_rays < 0", who);
  TXS_REQUIRE(d_total, "%s: null d_total", who);
  TXS_REQUIRE(n_rays == 0 || (counts && packed_info), "%s: null array", who);
  return TXS_OK;
}

// Tile sums of the allocation-free scan: a fixed array in device memory
// (every GPU the library runs on holds its own copy until the process ends).
constexpr int32_t kScratchTiles = 16384;  // 128 KiB: up to 2^26 rays per call
static __device__ __align__(256) int64_t scratch[kScratchTiles];

// Device address of `scratch` on each device, taken once per device with that
// device current.  In host code the array's name is only a stand-in for the
// symbol, never a device address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch_ptr[kMaxDevices] = {};

txs_status scratch_on_current_device(const char* who, int64_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error("%s: hipGetDevice failed: %s", who, hipGetErrorString(e));
    return TXS_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("%s: device %d beyond the %d the library tracks", who, dev, kMaxDevices);
    return TXS_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("%s: hipGetSymbolAddress(scratch) failed: %s", who, hipGetErrorString(e));
      return TXS_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<int64_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return TXS_OK;
}

}  // namespace
}  // namespace txs

extern "C" txs_status txs_exclusive_scan(const int32_t* counts, int32_t n_rays,
                                         int32_t* packed_info, int64_t* d_total,
                                         void* workspace, size_t workspace_bytes, void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status st = check_scan_args("txs_exclusive_scan", counts, n_rays, packed_info, d_total))
    return st;
  const size_t need = txs_scan_workspace_size(n_rays);
  if (!workspace || workspace_bytes < need) {
    set_error("txs_exclusive_scan: workspace needs %zu bytes, got %zu", need, workspace_bytes);
    return TXS_ECAPACITY;
  }
  launch_scan(counts, n_rays, packed_info, d_total, static_cast<int64_t*>(workspace),
              as_stream(stream));
  return launch_status("txs_exclusive_scan");
}

extern "C" int32_t txs_exclusive_scan_noalloc_max_rays(void) {
  return (int32_t)((int64_t)txs::kScratchTiles * txs::kTile);
}

extern "C" txs_status txs_exclusive_scan_noalloc(const int32_t* counts, int32_t n_rays,
                                                 int32_t* packed_info, int64_t* d_total,
                                                 void* stream) {
  using namespace txs;
  clear_error();
  if (txs_status st = check_scan_args("txs_exclusive_scan_noalloc", counts, n_rays, packed_info,
                                      d_total))
    return st;
  if ((int64_t)n_rays > (int64_t)kScratchTiles * kTile) {
    set_error("txs_exclusive_scan_noalloc: %d rays exceed the static scratch's limit of %lld",
              n_rays, (long long)kScratchTiles * kTile);
    return TXS_ECAPACITY;
  }
  int64_t* sums = nullptr;
  if (txs_status st = scratch_on_current_device("txs_exclusive_scan_noalloc", &sums)) return st;
  launch_scan(counts, n_rays, packed_info, d_total, sums, as_stream(stream));
  return launch_status("txs_exclusive_scan_noalloc");
}

extern "C" txs_status txs_gather_prefix(const int32_t* packed_info_in,
                                        const int32_t* packed_info_out, int32_t n_rays,
                                        int64_t n_in, const float* t0, const float* t1,
                                        int64_t capacity, float* t0o, float* t1o,
                                        int32_t* ray_ido, void* stream) {
  using namespace txs;
  clear_error();
  TXS_REQUIRE(n_rays >= 0 && n_in >= 0 && capacity >= 0, "txs_gather_prefix: negative size");
  if (n_rays == 0 || n_in == 0 || capacity == 0) return TXS_OK;
  TXS_REQUIRE(packed_info_in && packed_info_out && t0 && t1, "txs_gather_prefix: null input");
  TXS_REQUIRE(t0o && t1o, "txs_gather_prefix: null output");
  const int64_t waves = ((int64_t)n_rays + kWave - 1) / kWave;
  const int64_t blocks = (waves + kGatherWaves - 1) / kGatherWaves;
  hipLaunchKernelGGL(gather_prefix_kernel, dim3((unsigned)blocks), dim3(kWave * kGatherWaves), 0,
                     as_stream(stream), packed_info_in, packed_info_out, n_rays, n_in, t0, t1,
                     capacity, t0o, t1o, ray_ido);
  return launch_status("txs_gather_prefix");
}
