// Fill and exclusive-scan primitives.
#include <algorithm>

#include "kernels.h"

namespace lm {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* p, T v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_iota(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) p[i] = (uint32_t)i;
}

static int fill_grid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

// Work counter `unit` += the sum of len[i] (or len[idx[i]]) over i < n.
__global__ __launch_bounds__(kBlock) void k_count_units(const uint32_t* len, const uint32_t* idx, uint64_t n,
                                                        unsigned long long* parts, uint32_t unit) {
  __shared__ unsigned long long red[kBlock / kWave];
  unsigned long long e = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
    e += len[idx ? idx[i] : i];
  e = block_sum(e, red);
  if (threadIdx.x == 0) add_units(parts, unit, e);
}

void count_units(hipStream_t s, const uint32_t* len, const uint32_t* idx, uint64_t n, unsigned long long* parts,
                 uint32_t unit) {
  if (n && parts) hipLaunchKernelGGL(k_count_units, dim3(std::min<size_t>(fill_grid(n), 1024)), dim3(kBlock), 0, s,
                                     len, idx, n, parts, unit);
}

void fill_u32(hipStream_t s, uint32_t* p, uint32_t v, size_t n) {
  if (n) hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void fill_u8(hipStream_t s, uint8_t* p, uint8_t v, size_t n) {
  if (n) hipLaunchKernelGGL(k_fill<uint8_t>, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void fill_i64(hipStream_t s, int64_t* p, int64_t v, size_t n) {
  if (n) hipLaunchKernelGGL(k_fill<int64_t>, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void fill_u64(hipStream_t s, uint64_t* p, uint64_t v, size_t n) {
  if (n) hipLaunchKernelGGL(k_fill<uint64_t>, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void iota_u32(hipStream_t s, uint32_t* p, size_t n) {
  if (n) hipLaunchKernelGGL(k_iota, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n);
}

// ---------------------------------------------------------------------------
// Exclusive scan: tiles of 1024 items (256 threads x 4); tile sums are
// scanned by one block, then every tile scans itself from its offset.
// ---------------------------------------------------------------------------
constexpr int kTile = 1024;
constexpr int kPerThread = kTile / kBlock;

__device__ inline unsigned long long wave_incl_scan(unsigned long long x) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    unsigned long long y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan across the block; `sh` holds one value per wave + 1.
template <int NT>
__device__ inline unsigned long long block_excl_scan(unsigned long long x, unsigned long long* sh,
                                                     unsigned long long* block_total) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  unsigned long long incl = wave_incl_scan(x);
  if (lane == kWave - 1) sh[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int i = 0; i < NT / kWave; ++i) {
      unsigned long long t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[NT / kWave] = run;
  }
  __syncthreads();
  unsigned long long r = sh[wid] + incl - x;
  *block_total = sh[NT / kWave];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_reduce(const T* in, size_t n, unsigned long long* tile_sums) {
  __shared__ unsigned long long red[kBlock / kWave];
  const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kPerThread;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if (base + k < n) s += (unsigned long long)in[base + k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(unsigned long long* sums, size_t ntiles, uint64_t* total) {
  __shared__ unsigned long long sh[1024 / kWave + 1];
  unsigned long long carry = 0;
  for (size_t chunk = 0; chunk < ntiles; chunk += 1024) {
    const size_t i = chunk + threadIdx.x;
    const unsigned long long v = i < ntiles ? sums[i] : 0;
    unsigned long long bt;
    const unsigned long long ex = block_excl_scan<1024>(v, sh, &bt);
    if (i < ntiles) sums[i] = carry + ex;
    carry += bt;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const T* in, size_t n, const unsigned long long* tile_off,
                                                      uint64_t* out) {
  __shared__ unsigned long long sh[kBlock / kWave + 1];
  const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kPerThread;
  unsigned long long v[kPerThread];
  unsigned long long tsum = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    v[k] = base + k < n ? (unsigned long long)in[base + k] : 0;
    tsum += v[k];
  }
  unsigned long long bt;
  unsigned long long run = block_excl_scan<kBlock>(tsum, sh, &bt) + tile_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

size_t scan_tmp_bytes(size_t n) { return ((n + kTile - 1) / kTile + 1) * sizeof(unsigned long long); }

template <typename T>
static void exclusive_scan(hipStream_t s, const T* in, uint64_t* out, size_t n, uint64_t* total, void* tmp) {
  if (n == 0) {
    if (total) hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, total, (uint64_t)0);
    return;
  }
  const size_t ntiles = (n + kTile - 1) / kTile;
  unsigned long long* sums = (unsigned long long*)tmp;
  hipLaunchKernelGGL(k_tile_reduce<T>, dim3(ntiles), dim3(kBlock), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, sums, ntiles, total);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(ntiles), dim3(kBlock), 0, s, in, n, sums, out);
}

// Per-thread pinned host buffer for small device-to-host reads: a copy into
// pageable memory is staged by the runtime and returns only when done, so a
// few reads in a row cost a round trip each; into pinned memory they queue
// behind the kernels and one synchronisation covers them all.
namespace {
struct PinnedStage {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local PinnedStage tl_stage;
}  // namespace

void* pinned_stage(size_t bytes) {
  if (bytes > tl_stage.bytes) {
    if (tl_stage.p) (void)hipHostFree(tl_stage.p);
    tl_stage.p = nullptr;
    tl_stage.bytes = 0;
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&tl_stage.p, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      tl_stage.p = nullptr;
      return nullptr;
    }
    tl_stage.bytes = want;
  }
  return tl_stage.p;
}

void exclusive_scan_u32(hipStream_t s, const uint32_t* in, uint64_t* out, size_t n, uint64_t* total, void* tmp) {
  exclusive_scan<uint32_t>(s, in, out, n, total, tmp);
}
void exclusive_scan_u64(hipStream_t s, const uint64_t* in, uint64_t* out, size_t n, uint64_t* total, void* tmp) {
  exclusive_scan<uint64_t>(s, in, out, n, total, tmp);
}

}  // namespace lm
