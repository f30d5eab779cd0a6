// Block-privatised scatter reductions.  Community sizes are very skewed
// (a few communities can hold a large share of all vertices), so a plain
// atomic per vertex on out[C[i]] serialises on the hot addresses.  Each block
// first reduces a tile of 1024 items in an LDS hash table and then issues one
// global atomic per distinct key of the tile.
#include "kernels.h"

namespace lm {

constexpr int kScTile = 1024;           // items per block iteration
constexpr int kScSlots = 2 * kScTile;   // LDS hash slots

static int grid_tiles(uint64_t n) {
  uint64_t b = (n + kScTile - 1) / kScTile;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

// out[key[i]] += val[i] (val == null: += 1) for i < n.
template <typename V, typename O>
__global__ __launch_bounds__(kBlock) void k_scatter_add(const uint32_t* key, const V* val, uint64_t n, O* out) {
  __shared__ uint32_t hk[kScSlots];
  __shared__ unsigned long long hv[kScSlots];
  for (uint64_t base = (uint64_t)blockIdx.x * kScTile; base < n; base += (uint64_t)gridDim.x * kScTile) {
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      hk[s] = kNone;
      hv[s] = 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kScTile; t += kBlock) {
      const uint64_t i = base + t;
      if (i < n) table_add(hk, hv, kScSlots - 1, key[i], val ? (unsigned long long)val[i] : 1ull);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      const uint32_t k = hk[s];
      if (k != kNone) atomicAdd((unsigned long long*)&out[k], hv[s]);
    }
    __syncthreads();
  }
}

// 32-bit counts
template <typename V>
__global__ __launch_bounds__(kBlock) void k_scatter_count(const uint32_t* key, uint64_t n, uint32_t* out) {
  __shared__ uint32_t hk[kScSlots];
  __shared__ unsigned long long hv[kScSlots];
  for (uint64_t base = (uint64_t)blockIdx.x * kScTile; base < n; base += (uint64_t)gridDim.x * kScTile) {
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      hk[s] = kNone;
      hv[s] = 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kScTile; t += kBlock) {
      const uint64_t i = base + t;
      if (i < n) table_add(hk, hv, kScSlots - 1, key[i], 1ull);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      const uint32_t k = hk[s];
      if (k != kNone) atomicAdd(&out[k], (uint32_t)hv[s]);
    }
    __syncthreads();
  }
}

// out[key[i]] = min(out[key[i]], i): the smallest index per key.  Inside a
// tile the first index of a key is its minimum, so one atomicMin per key and
// tile suffices.
__global__ __launch_bounds__(kBlock) void k_scatter_min_index(const uint32_t* key, uint64_t n, uint32_t* out) {
  __shared__ uint32_t hk[kScSlots];
  __shared__ uint32_t hmin[kScSlots];
  for (uint64_t base = (uint64_t)blockIdx.x * kScTile; base < n; base += (uint64_t)gridDim.x * kScTile) {
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      hk[s] = kNone;
      hmin[s] = kNone;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kScTile; t += kBlock) {
      const uint64_t i = base + t;
      if (i >= n) continue;
      const uint32_t k = key[i];
      uint32_t h = slot_hash(k, kScSlots - 1);
      while (true) {
        const uint32_t o = atomicCAS(&hk[h], kNone, k);
        if (o == kNone || o == k) break;
        h = (h + 1) & (kScSlots - 1);
      }
      atomicMin(&hmin[h], (uint32_t)i);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kScSlots; s += kBlock) {
      const uint32_t k = hk[s];
      if (k != kNone) atomicMin(&out[k], hmin[s]);
    }
    __syncthreads();
  }
}

void scatter_add_i64(hipStream_t s, const uint32_t* key, const int64_t* val, uint64_t n, int64_t* out) {
  if (n) hipLaunchKernelGGL((k_scatter_add<int64_t, int64_t>), dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, val, n, out);
}

void scatter_add_u32_to_u64(hipStream_t s, const uint32_t* key, const uint32_t* val, uint64_t n, uint64_t* out) {
  if (n)
    hipLaunchKernelGGL((k_scatter_add<uint32_t, uint64_t>), dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, val, n, out);
}

void scatter_count(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out) {
  if (n) hipLaunchKernelGGL(k_scatter_count<uint32_t>, dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, n, out);
}

void scatter_min_index(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out) {
  if (n) hipLaunchKernelGGL(k_scatter_min_index, dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, n, out);
}

}  // namespace lm
