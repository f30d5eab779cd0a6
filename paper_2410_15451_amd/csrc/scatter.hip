// Scatter reductions out[key[i]] (+)= val[i] or min= i.  Community sizes are
// very skewed (a few communities can hold a large share of all vertices), so
// a plain atomic per vertex on out[C[i]] serialises on the hot addresses.
//
// Small inputs: each block reduces a tile of 1024 items in an LDS hash table
// and issues one global atomic per distinct key of the tile.
//
// Large inputs (a workspace is set): the same tile reduction writes each
// tile's distinct (key, value) pairs to a staging array instead; the pairs
// are then counted per key bucket (4096 consecutive keys) and block, the
// counts scanned, the pairs placed bucket by bucket, and one block per bucket
// combines its pairs in a dense LDS array and updates its 4096 outputs with
// plain stores.  No global atomics, every pass streams.
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

// ---------------------------------------------------------------------------
// Bucketed form.  Op::kMin: value = item index, combine = min; otherwise sum.
// ---------------------------------------------------------------------------
constexpr int kBkBits = 12;
constexpr uint32_t kBkKeys = 1u << kBkBits;
constexpr int kBkBlocks = 256;  // blocks of the counting and placing passes
constexpr uint64_t kBkMinItems = 1u << 18;

enum class Op { kSum, kCount, kMin };

// Phase A: tile t's distinct pairs go to stage[t * kScTile ...], their count
// to tile_cnt[t].
template <Op OP, typename V>
__global__ __launch_bounds__(kBlock) void k_bk_tiles(const uint32_t* key, const V* val, uint64_t n, uint32_t* sk,
                                                     unsigned long long* sv, uint32_t* tile_cnt) {
  __shared__ uint32_t hk[kScSlots];
  __shared__ unsigned long long hv[kScSlots];
  __shared__ unsigned int used;
  const uint64_t ntiles = (n + kScTile - 1) / kScTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = t * kScTile;
    for (int q = threadIdx.x; q < kScSlots; q += kBlock) {
      hk[q] = kNone;
      hv[q] = OP == Op::kMin ? ~0ull : 0ull;
    }
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < kScTile; q += kBlock) {
      const uint64_t i = base + q;
      if (i >= n) continue;
      const uint32_t k = key[i];
      uint32_t h = slot_hash(k, kScSlots - 1);
      while (true) {
        const uint32_t o = atomicCAS(&hk[h], kNone, k);
        if (o == kNone || o == k) break;
        h = (h + 1) & (kScSlots - 1);
      }
      if (OP == Op::kMin)
        atomicMin(&hv[h], (unsigned long long)i);
      else if (OP == Op::kCount)
        atomicAdd(&hv[h], 1ull);
      else
        atomicAdd(&hv[h], (unsigned long long)val[i]);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kScSlots; q += kBlock) {
      const uint32_t k = hk[q];
      if (k == kNone) continue;
      const unsigned int pos = atomicAdd(&used, 1u);
      sk[base + pos] = k;
      sv[base + pos] = hv[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[t] = used;
    __syncthreads();
  }
}

// Phases B and D share the partition of tiles over kBkBlocks blocks.
__device__ inline void bk_tile_range(uint64_t ntiles, uint64_t* t0, uint64_t* t1) {
  const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  *t0 = min(ntiles, (uint64_t)blockIdx.x * per);
  *t1 = min(ntiles, *t0 + per);
}

// Phase B: mat[bucket * kBkBlocks + block] = pairs of that bucket in the block's tiles.
__global__ __launch_bounds__(kBlock) void k_bk_count(const uint32_t* sk, const uint32_t* tile_cnt, uint64_t ntiles,
                                                     uint32_t nb, uint32_t* mat) {
  extern __shared__ unsigned int hist[];
  for (uint32_t b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0;
  __syncthreads();
  uint64_t t0, t1;
  bk_tile_range(ntiles, &t0, &t1);
  for (uint64_t t = t0; t < t1; ++t) {
    const uint32_t c = tile_cnt[t];
    for (uint32_t q = threadIdx.x; q < c; q += kBlock) atomicAdd(&hist[sk[t * kScTile + q] >> kBkBits], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += kBlock) mat[(size_t)b * kBkBlocks + blockIdx.x] = hist[b];
}

// Phase D: place the pairs bucket by bucket.
__global__ __launch_bounds__(kBlock) void k_bk_place(const uint32_t* sk, const unsigned long long* sv,
                                                     const uint32_t* tile_cnt, uint64_t ntiles, uint32_t nb,
                                                     const uint64_t* off, uint32_t* bk, unsigned long long* bv) {
  extern __shared__ unsigned int cur[];
  for (uint32_t b = threadIdx.x; b < nb; b += kBlock) cur[b] = (unsigned int)off[(size_t)b * kBkBlocks + blockIdx.x];
  __syncthreads();
  uint64_t t0, t1;
  bk_tile_range(ntiles, &t0, &t1);
  for (uint64_t t = t0; t < t1; ++t) {
    const uint32_t c = tile_cnt[t];
    for (uint32_t q = threadIdx.x; q < c; q += kBlock) {
      const uint32_t k = sk[t * kScTile + q];
      const unsigned int pos = atomicAdd(&cur[k >> kBkBits], 1u);
      bk[pos] = k;
      bv[pos] = sv[t * kScTile + q];
    }
  }
}

// Phase E: work items of at most kBkSlice pairs: a bucket with more pairs is
// cut into equal slices.  Renumbered community IDs fill only the first
// buckets, so one block per bucket left a few blocks with all the pairs.
// item_start[b] is the first item of bucket b (item_start[nb] = items).
constexpr uint64_t kBkSlice = 8192;

__global__ __launch_bounds__(kBlock) void k_bk_items(const uint64_t* off, const uint64_t* total, uint32_t nb,
                                                     uint32_t* item_start) {
  __shared__ uint32_t wsum[kBlock / kWave];
  const uint32_t per = (nb + kBlock - 1) / kBlock;
  const uint32_t b0 = min(nb, threadIdx.x * per), b1 = min(nb, b0 + per);
  auto start = [&](uint32_t b) { return b < nb ? off[(size_t)b * kBkBlocks] : *total; };
  auto slices = [&](uint32_t b) { return (uint32_t)((start(b + 1) - start(b) + kBkSlice - 1) / kBkSlice); };
  uint32_t mine = 0;
  for (uint32_t b = b0; b < b1; ++b) mine += slices(b);
  // exclusive block scan of the per-thread sums
  const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  uint32_t inc = mine;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if ((int)lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  uint32_t base = inc - mine;
  for (uint32_t q = 0; q < wv; ++q) base += wsum[q];
  for (uint32_t b = b0; b < b1; ++b) {
    item_start[b] = base;
    base += slices(b);
  }
  if (threadIdx.x == kBlock - 1) item_start[nb] = base;  // the last thread's range ends at nb
}

template <Op OP, typename O>
__global__ __launch_bounds__(kBlock) void k_bk_reduce(const uint32_t* bk, const unsigned long long* bv,
                                                      const uint64_t* off, const uint64_t* total, uint32_t nb,
                                                      const uint32_t* item_start, uint64_t key_range, O* out) {
  __shared__ unsigned long long acc[kBkKeys];
  __shared__ uint32_t sb;
  const uint32_t it = blockIdx.x;
  if (it >= item_start[nb]) return;  // block-uniform
  if (threadIdx.x == 0) {            // last bucket whose first item is <= it
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (item_start[mid] <= it)
        lo = mid;
      else
        hi = mid;
    }
    sb = lo;
  }
  for (uint32_t q = threadIdx.x; q < kBkKeys; q += kBlock) acc[q] = OP == Op::kMin ? ~0ull : 0ull;
  __syncthreads();
  const uint32_t b = sb;
  const uint32_t s = it - item_start[b], ns = item_start[b + 1] - item_start[b];
  const uint64_t lo = off[(size_t)b * kBkBlocks];
  const uint64_t len = (b + 1 < nb ? off[(size_t)(b + 1) * kBkBlocks] : *total) - lo;
  const uint64_t x0 = lo + len * s / ns, x1 = lo + len * (s + 1) / ns;
  for (uint64_t x = x0 + threadIdx.x; x < x1; x += kBlock) {
    const uint32_t k = bk[x] & (kBkKeys - 1);
    if (OP == Op::kMin)
      atomicMin(&acc[k], bv[x]);
    else
      atomicAdd(&acc[k], bv[x]);
  }
  __syncthreads();
  const uint64_t k0 = (uint64_t)b << kBkBits;
  for (uint32_t q = threadIdx.x; q < kBkKeys; q += kBlock) {
    const uint64_t k = k0 + q;
    if (k >= key_range) break;
    const unsigned long long a = acc[q];
    if (OP == Op::kMin) {
      if (a == ~0ull) continue;
      if (ns > 1) {
        static_assert(OP != Op::kMin || sizeof(O) == 4, "minimum index outputs are 32-bit");
        atomicMin((unsigned int*)&out[k], (unsigned int)a);
      } else if ((O)a < out[k]) {
        out[k] = (O)a;
      }
    } else {
      if (!a) continue;
      if (ns == 1)
        out[k] = (O)((unsigned long long)out[k] + a);
      else if (sizeof(O) == 8)
        atomicAdd((unsigned long long*)&out[k], a);
      else
        atomicAdd((unsigned int*)&out[k], (unsigned int)a);
    }
  }
}

// Workspace layout for n items and keys below key_range.
struct BkLayout {
  uint64_t ntiles;
  uint32_t nb;
  size_t o_sk, o_sv, o_tc, o_bk, o_bv, o_mat, o_off, o_tot, o_items, o_tmp, bytes;
};

BkLayout bk_layout(uint64_t n, uint64_t key_range) {
  BkLayout L;
  L.ntiles = (n + kScTile - 1) / kScTile;
  L.nb = (uint32_t)((key_range + kBkKeys - 1) / kBkKeys);
  const size_t nm = (size_t)L.nb * kBkBlocks;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 0;
  L.o_sk = o;
  o = al(o + L.ntiles * kScTile * 4);
  L.o_sv = o;
  o = al(o + L.ntiles * kScTile * 8);
  L.o_tc = o;
  o = al(o + L.ntiles * 4);
  L.o_bk = o;
  o = al(o + n * 4);
  L.o_bv = o;
  o = al(o + n * 8);
  L.o_mat = o;
  o = al(o + nm * 4);
  L.o_off = o;
  o = al(o + (nm + 1) * 8);
  L.o_tot = o;
  o = al(o + 8);
  L.o_items = o;
  o = al(o + ((size_t)L.nb + 1) * 4);
  L.o_tmp = o;
  o = al(o + scan_tmp_bytes(nm) + 64);
  L.bytes = o;
  return L;
}

template <Op OP, typename V, typename O>
bool bucketed(hipStream_t s, const uint32_t* key, const V* val, uint64_t n, uint64_t key_range, O* out) {
  const ScatterWs* ws = tl_scatter_ws;
  if (!ws || n < kBkMinItems || key_range == 0) return false;
  const BkLayout L = bk_layout(n, key_range);
  if (L.bytes > ws->bytes || (size_t)L.nb * 4 > 64 * 1024) return false;
  char* p = (char*)ws->p;
  uint32_t* sk = (uint32_t*)(p + L.o_sk);
  unsigned long long* sv = (unsigned long long*)(p + L.o_sv);
  uint32_t* tc = (uint32_t*)(p + L.o_tc);
  uint32_t* bk = (uint32_t*)(p + L.o_bk);
  unsigned long long* bv = (unsigned long long*)(p + L.o_bv);
  uint32_t* mat = (uint32_t*)(p + L.o_mat);
  uint64_t* off = (uint64_t*)(p + L.o_off);
  uint64_t* tot = (uint64_t*)(p + L.o_tot);
  uint32_t* items = (uint32_t*)(p + L.o_items);
  void* tmp = p + L.o_tmp;
  const size_t lds = (size_t)L.nb * 4;
  hipLaunchKernelGGL((k_bk_tiles<OP, V>), dim3(std::min<uint64_t>(L.ntiles, 4096)), dim3(kBlock), 0, s, key, val, n,
                     sk, sv, tc);
  hipLaunchKernelGGL(k_bk_count, dim3(kBkBlocks), dim3(kBlock), lds, s, sk, tc, L.ntiles, L.nb, mat);
  exclusive_scan_u32(s, mat, off, (size_t)L.nb * kBkBlocks, tot, tmp);
  hipLaunchKernelGGL(k_bk_place, dim3(kBkBlocks), dim3(kBlock), lds, s, sk, sv, tc, L.ntiles, L.nb, off, bk, bv);
  hipLaunchKernelGGL(k_bk_items, dim3(1), dim3(kBlock), 0, s, off, tot, L.nb, items);
  // at most one item per bucket plus one per kBkSlice pairs (pairs <= n)
  const uint64_t max_items = (uint64_t)L.nb + n / kBkSlice + 1;
  hipLaunchKernelGGL((k_bk_reduce<OP, O>), dim3((uint32_t)max_items), dim3(kBlock), 0, s, bk, bv, off, tot, L.nb,
                     items, key_range, out);
  return true;
}

size_t scatter_ws_bytes(uint64_t n, uint64_t key_range) { return bk_layout(n, key_range).bytes; }

void scatter_add_i64(hipStream_t s, const uint32_t* key, const int64_t* val, uint64_t n, int64_t* out,
                     uint64_t key_range) {
  if (!n || bucketed<Op::kSum>(s, key, val, n, key_range, out)) return;
  hipLaunchKernelGGL((k_scatter_add<int64_t, int64_t>), dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, val, n, out);
}

void scatter_add_u32_to_u64(hipStream_t s, const uint32_t* key, const uint32_t* val, uint64_t n, uint64_t* out,
                            uint64_t key_range) {
  if (!n || bucketed<Op::kSum>(s, key, val, n, key_range, out)) return;
  hipLaunchKernelGGL((k_scatter_add<uint32_t, uint64_t>), dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, val, n, out);
}

void scatter_count(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out, uint64_t key_range) {
  if (!n || bucketed<Op::kCount, uint32_t>(s, key, nullptr, n, key_range, out)) return;
  hipLaunchKernelGGL(k_scatter_count<uint32_t>, dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, n, out);
}

void scatter_min_index(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out, uint64_t key_range) {
  if (!n || bucketed<Op::kMin, uint32_t>(s, key, nullptr, n, key_range, out)) return;
  hipLaunchKernelGGL(k_scatter_min_index, dim3(grid_tiles(n)), dim3(kBlock), 0, s, key, n, out);
}

}  // namespace lm
