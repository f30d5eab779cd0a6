// Shared definitions of the gfx950 Leiden kernels and their host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace lm {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kBlock = 256;     // threads per block of every list kernel
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kMaxClasses = 32; // vertex classes / refinement colours
constexpr int kBins = 6;        // degree bins of the hash kernels

// Degree bins: lanes per vertex and hash slots per vertex.  A vertex of
// degree d goes to the first bin b with d <= max_deg[b]; the last bin (hubs)
// keeps its tables in global memory.  The thresholds are tunable up to the
// capacity of each bin's table (kBinCap: slots - 1, so a table never fills);
// they change where a vertex is decided, never the decision.
struct BinCfg {
  uint32_t max_deg[kBins];
};
// Default thresholds: each bin up to its table's capacity (measured on R-MAT
// 2^22 against lower thresholds: 3% faster static runs, 5% faster DF updates).
constexpr BinCfg kDefaultBins = {{15, 63, 255, 1023, 4095, 0xFFFFFFFFu}};
constexpr uint32_t kBinCap[kBins - 1] = {15, 63, 255, 1023, 4095};

__host__ __device__ inline int bin_of_degree(uint32_t d, const BinCfg& cfg) {
  int b = 0;
  while (b < kBins - 1 && d > cfg.max_deg[b]) ++b;
  return b;
}

// A decided move of the local-moving or refinement phase.
struct Mover {
  uint32_t v;
  uint32_t c;
  double dq;
};

// Row view of one level of the graph: row i holds entries
// [start[i], start[i] + len[i]) of cols / w.
template <typename W>
struct Rows {
  const int64_t* start;
  const uint32_t* len;
  const uint32_t* cols;
  const W* w;
};

// Counters and scalars that live on the device during one call.
struct Ctl {
  unsigned long long dq_fixed;       // int64 fixed-point gain sum of the iteration (2^56 scale)
  unsigned long long moves;          // moves of the current sub-round
  unsigned long long edges;          // edge scans of the call
  unsigned long long total_moves;    // local-moving moves of the call
  unsigned long long refine_moves;   // refinement moves of the call
  unsigned int next_count;           // vertices unprocessed for the next iteration
  unsigned int iter_count;           // vertices unprocessed at the start of this iteration
  unsigned int cls_count[kMaxClasses];
  unsigned int bin_count[kBins];
  unsigned int mover_count;
  unsigned int refined_any;          // some vertex lies in a refined bound
  unsigned int split_count;          // vertices of split-marked communities
  unsigned int split_wide;           // split vertices with long rows (wider sample)
  unsigned int split_rest;           // split vertices outside their community's main tree
  unsigned int hub_items;            // (hub, chunk) work items of the current sub-round
  unsigned int error;                // batch validation error code
  unsigned int touched;              // rows touched by the batch
  unsigned int init_count;           // vertices marked affected by the batch
  unsigned long long overflow_need;  // entries to relocate into the overflow area
  unsigned int mark_items;           // neighbour-marking work items of the current sub-round
  unsigned int sort_count[2];        // batch segments left to the block sorts (LDS, merge)
  unsigned int misc[8];
  unsigned long long kt_units[4];    // work units of the timed kernels (indexed by leiden_kernel)
  unsigned long long units[16];      // work counters of the call (WorkUnit), folded at its end
  // A forest of independent graphs in one block-diagonal level graph (all
  // null for one graph): the graph of every vertex of the level, each
  // graph's first vertex at the level, each graph's Eq. 2 constants (1/m,
  // 1/(2 m^2)) and iteration gain sum, per graph whether it still iterates
  // local moving and whether it is still in the pass loop, and per graph
  // whether it marked a community for refinement in the current pass.
  const uint32_t* f_gid;
  const uint32_t* f_base;
  const double* f_inv;
  unsigned long long* f_dq;
  const uint8_t* f_move;
  const uint8_t* f_pass;
  uint8_t* f_refined;
  unsigned int f_live;    // graphs still in the pass loop
  unsigned int f_moving;  // graphs still iterating local moving
};

// The forest fields of a control block, read once per kernel.
struct ForestView {
  const uint32_t* gid;
  const uint32_t* base;
  const double* inv;
  unsigned long long* dq;
  const uint8_t* move;
  const uint8_t* pass;
  uint8_t* refined;
  // v's ID inside its graph (the schedules hash graph-local IDs, so that
  // every graph is processed as it would be alone)
  __device__ uint32_t local(uint32_t v) const { return gid ? v - base[gid[v]] : v; }
  // v's graph still iterates local moving
  __device__ bool moving(uint32_t v) const { return !move || move[gid[v]]; }
  // v's graph is still in the pass loop
  __device__ bool live(uint32_t v) const { return !pass || pass[gid[v]]; }
};
__device__ inline ForestView forest_view(const Ctl* c) {
  return ForestView{c->f_gid, c->f_base, c->f_inv, c->f_dq, c->f_move, c->f_pass, c->f_refined};
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// MurmurHash3 32-bit finaliser (Appleby, public domain).
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Class of vertex v in local-moving iteration t with P classes.
__host__ __device__ inline uint32_t vertex_class(uint32_t v, uint32_t t, uint32_t P) {
  return fmix32(v + t * 0x9e3779b9u) % P;
}

// Colour of vertex v in the R synchronous refinement rounds.
__host__ __device__ inline uint32_t vertex_colour(uint32_t v, uint32_t R) { return fmix32(v) % R; }

// Eq. 2, delta-modularity of moving a vertex i from community d to c:
//   (K_{i->c} - K_{i->d}) / m - K_i (K_i + Sigma_c - Sigma_d) / (2 m^2),
// with inv_m = 1/m and inv_2m2 = 1/(2 m^2) precomputed on the host.  Integer
// parts are exact; every product and difference below is rounded on its own
// (no contraction into fused multiply-add).
__device__ inline double delta_q(int64_t kic, int64_t kid, int64_t ki, int64_t sc, int64_t sd, double inv_m,
                                 double inv_2m2) {
#pragma clang fp contract(off)
  double a = (double)(kic - kid);
  double b = (double)(ki + sc - sd);
  double first = a * inv_m;
  double kb = (double)ki * b;
  double second = kb * inv_2m2;
  return first - second;
}

// Gain as int64 fixed point with 2^56 scale (truncation toward zero).
__device__ inline long long gain_fixed(double dq) {
#pragma clang fp contract(off)
  return (long long)(dq * 72057594037927936.0);
}

// Reads of locations that other threads of the same launch write.
//  peek: a hint read in front of an atomic or a store that decides by itself
//    (a stale value only costs a redundant atomic or store: the flags and
//    maxima it guards only grow during a launch); a plain load, so that it may
//    hit in the caches.  System-scope atomic loads bypass them, and thousands
//    of lanes reading one hot word (the flag of a large community) then queue
//    at one memory channel.
//  ld_sys / st_sys: system-scope relaxed accesses, for values a loop acts on
//    (live state of the asynchronous schedule, partial results of other
//    blocks).  Device-scope loads may be
//    served by the issuing XCD's own L2, which does not see the other XCDs'
//    writes during the launch; a retry loop can then read the same stale
//    value forever.
template <typename T>
__device__ inline T peek(const T* p) {
  return *p;
}
template <typename T>
__device__ inline T ld_sys(const T* p) {
  return __atomic_load_n(p, __ATOMIC_RELAXED);
}
template <typename T>
__device__ inline void st_sys(T* p, T v) {
  __atomic_store_n(p, v, __ATOMIC_RELAXED);
}
//  ld_near / st_near: workgroup-scope relaxed accesses, served by the nearest
//    cache.  For loops whose progress does not rest on fresh values: each
//    retry is driven by the value an atomic returned (atomics act at memory
//    and are coherent across XCDs), and a stale value only costs a retry
//    (union-find parents; keys of a hash table, written once per launch, so a
//    stale read shows a taken slot empty and the compare-and-swap that follows
//    returns its key).
template <typename T>
__device__ inline T ld_near(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ inline void st_near(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Raise a flag that many threads may raise at once (e.g. one per member of a
// large community): read first, since stores to one line from every CU
// queue on it.
template <typename T>
__device__ inline void raise_flag(T* a, size_t i) {
  if (!peek(&a[i])) a[i] = 1;
}

// (dq, c) order of the best-community choice: larger gain first, then lower ID.
__device__ inline bool better(double dq, uint32_t c, double bdq, uint32_t bc) {
  return dq > bdq || (dq == bdq && c < bc);
}

// Home slot of a key: the low bits of a full-avalanche mixing.  (The low bits
// of a plain multiplicative hash depend only on the key's low bits, and the
// labels of aggregated levels often share few low-bit patterns: such a table
// degenerates into probe chains of hundreds of slots.)
__device__ inline uint32_t slot_hash(uint32_t key, uint32_t mask) { return fmix32(key) & mask; }

// Salt of the tables whose slot order becomes the order of an aggregated row.
// A row listed in slot order is sorted by that table's hash: a table of the
// same hash filled from a run of such a row (a hub chunk) would see keys of
// nearly equal home slots and degenerate into long probe chains, so rows are
// ordered by a differently salted hash than every table that reads them.
constexpr uint32_t kRowSalt = 0x9e3779b9u;

// Open-addressing insert-or-add into a table of `mask + 1` slots (keys kNone
// when free); the table always has more slots than distinct keys.
template <typename KeyPtr, typename ValPtr>
__device__ inline void table_add(KeyPtr keys, ValPtr vals, uint32_t mask, uint32_t key, unsigned long long w,
                                 uint32_t salt = 0) {
  uint32_t h = slot_hash(key ^ salt, mask);
  while (true) {
    uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
    if (k == key) {
      atomicAdd(&vals[h], w);
      return;
    }
    if (k == kNone) {
      uint32_t o = atomicCAS(&keys[h], kNone, key);
      if (o == kNone || o == key) {
        atomicAdd(&vals[h], w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

// Streamed table_add over a lane's entries e = e, e + step, ... < e1:
// entry(e, key, w) yields the key and weight of entry e, or key kNone for an
// entry that is not inserted.  Entries are fetched kStreamBatch at a time
// (all lanes together, so the loads overlap), then inserted with a lane whose
// probe has ended taking its next fetched entry at once: a long probe holds
// up only its own lane, where a plain loop over table_add runs every entry
// at the pace of the wavefront's longest probe.
constexpr int kStreamBatch = 4;
template <typename KeyPtr, typename ValPtr, typename Entry>
__device__ inline void table_accumulate(KeyPtr keys, ValPtr vals, uint32_t mask, uint32_t e, uint32_t e1,
                                        uint32_t step, Entry entry) {
  for (; e < e1; e += kStreamBatch * step) {
    uint32_t kk[kStreamBatch];
    unsigned long long ww[kStreamBatch];
#pragma unroll
    for (int u = 0; u < kStreamBatch; ++u) {
      kk[u] = kNone;
      ww[u] = 0;
      const uint32_t x = e + u * step;
      if (x < e1) entry(x, kk[u], ww[u]);
    }
    int next = 0;
    uint32_t key = kNone, h = 0;
    unsigned long long w = 0;
    while (true) {
      if (key == kNone) {
        // the next fetched entry to insert (unrolled selection keeps kk / ww in registers)
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
          if (key == kNone && u >= next && kk[u] != kNone) {
            key = kk[u];
            w = ww[u];
            next = u + 1;
          }
        }
        if (key == kNone) break;
        h = slot_hash(key, mask);
      }
      const uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
      if (k == key) {
        atomicAdd(&vals[h], (std::remove_cv_t<std::remove_pointer_t<ValPtr>>)w);
        key = kNone;
        continue;
      }
      if (k == kNone) {
        const uint32_t o = atomicCAS(&keys[h], kNone, key);
        if (o == kNone || o == key) {
          atomicAdd(&vals[h], (std::remove_cv_t<std::remove_pointer_t<ValPtr>>)w);
          key = kNone;
          continue;
        }
      }
      h = (h + 1) & mask;
    }
  }
}

// table_accumulate that also lists the slots it takes (list[*nlist] = slot,
// LDS counter; the first `cap` of them), so that the table can be read and
// cleared by its used slots instead of all of them (when *nlist <= cap).
template <typename KeyPtr, typename ValPtr, typename Entry>
__device__ inline void table_accumulate_listed(KeyPtr keys, ValPtr vals, uint32_t mask, uint32_t e, uint32_t e1,
                                               uint32_t step, uint16_t* list, unsigned int* nlist, uint32_t cap,
                                               Entry entry) {
  for (; e < e1; e += kStreamBatch * step) {
    uint32_t kk[kStreamBatch];
    unsigned long long ww[kStreamBatch];
#pragma unroll
    for (int u = 0; u < kStreamBatch; ++u) {
      kk[u] = kNone;
      ww[u] = 0;
      const uint32_t x = e + u * step;
      if (x < e1) entry(x, kk[u], ww[u]);
    }
    int next = 0;
    uint32_t key = kNone, h = 0;
    unsigned long long w = 0;
    while (true) {
      if (key == kNone) {
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
          if (key == kNone && u >= next && kk[u] != kNone) {
            key = kk[u];
            w = ww[u];
            next = u + 1;
          }
        }
        if (key == kNone) break;
        h = slot_hash(key, mask);
      }
      const uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
      if (k == key) {
        atomicAdd(&vals[h], (std::remove_cv_t<std::remove_pointer_t<ValPtr>>)w);
        key = kNone;
        continue;
      }
      if (k == kNone) {
        const uint32_t o = atomicCAS(&keys[h], kNone, key);
        if (o == kNone) {
          const unsigned int x = atomicAdd(nlist, 1u);
          if (x < cap) list[x] = (uint16_t)h;
        }
        if (o == kNone || o == key) {
          atomicAdd(&vals[h], (std::remove_cv_t<std::remove_pointer_t<ValPtr>>)w);
          key = kNone;
          continue;
        }
      }
      h = (h + 1) & mask;
    }
  }
}

// table_add that gives up after probing every slot once: false when the key
// found no slot (the table is full), and the sum of that key is then missing.
template <typename KeyPtr, typename ValPtr>
__device__ inline bool table_add_bounded(KeyPtr keys, ValPtr vals, uint32_t mask, uint32_t key,
                                         unsigned long long w, uint32_t salt = 0) {
  uint32_t h = slot_hash(key ^ salt, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
    if (k == key) {
      atomicAdd(&vals[h], w);
      return true;
    }
    if (k == kNone) {
      const uint32_t o = atomicCAS(&keys[h], kNone, key);
      if (o == kNone || o == key) {
        atomicAdd(&vals[h], w);
        return true;
      }
    }
    h = (h + 1) & mask;
  }
  return false;
}

template <int G, typename T>
__device__ inline T group_sum(T x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

template <int G>
__device__ inline void group_best(double& dq, uint32_t& c) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    double odq = __shfl_xor(dq, o, G);
    uint32_t oc = __shfl_xor(c, o, G);
    if (better(odq, oc, dq, c)) {
      dq = odq;
      c = oc;
    }
  }
}

// Block-wide (kBlock threads) sum and best-choice through LDS.
template <typename T>
__device__ inline T block_sum(T x, T* red) {
  x = group_sum<kWave>(x);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) red[w] = x;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kBlock / kWave; ++i) r += red[i];
    red[0] = r;
  }
  __syncthreads();
  r = red[0];
  __syncthreads();
  return r;
}

__device__ inline void block_best(double& dq, uint32_t& c, double* rdq, uint32_t* rc) {
  group_best<kWave>(dq, c);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) {
    rdq[w] = dq;
    rc[w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / kWave; ++i)
      if (better(rdq[i], rc[i], rdq[0], rc[0])) {
        rdq[0] = rdq[i];
        rc[0] = rc[i];
      }
  }
  __syncthreads();
  dq = rdq[0];
  c = rc[0];
  __syncthreads();
}

// Append one item to a list with a device counter.
__device__ inline void list_push(uint32_t* list, unsigned int* count, uint32_t v) {
  unsigned int pos = atomicAdd(count, 1u);
  list[pos] = v;
}

// Wavefront-aggregated append to one of several lists: every active lane
// calls this together; a lane with key != kNone appends v to list `key`
// (list_of(key) gives the list base and its counter).  One atomic per
// distinct key in the wavefront instead of one per lane.
template <typename ListOf>
__device__ inline void wave_append(uint32_t key, uint32_t v, ListOf list_of) {
  const uint32_t lane = threadIdx.x % kWave;
  unsigned long long pending = __ballot(key != kNone);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t lk = __shfl(key, leader);
    const unsigned long long mask = __ballot(key == lk) & pending;
    uint32_t* list;
    unsigned int* count;
    list_of(lk, list, count);
    unsigned int base = 0;
    if ((int)lane == leader) base = atomicAdd(count, (unsigned int)__popcll(mask));
    base = __shfl(base, leader);
    if ((mask >> lane) & 1ull) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
    pending &= ~mask;
  }
}

// Wavefront-aggregated atomic adds keyed by address index: every active lane
// calls this together; the lanes sharing a key are summed and one of them
// adds the sums to a[key] and b[key].  Lanes with key == kNone add nothing.
__device__ inline void wave_add2_by_key(uint32_t key, long long va, long long vb, long long* a, long long* b) {
  const uint32_t lane = threadIdx.x % kWave;
  unsigned long long pending = __ballot(key != kNone);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t lk = __shfl(key, leader);
    const unsigned long long mask = __ballot(key == lk) & pending;
    const bool mine = (mask >> lane) & 1ull;
    long long sa = mine ? va : 0, sb = mine ? vb : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      sa += __shfl_xor(sa, o);
      sb += __shfl_xor(sb, o);
    }
    if ((int)lane == leader) {
      atomicAdd((unsigned long long*)&a[lk], (unsigned long long)sa);
      atomicAdd((unsigned long long*)&b[lk], (unsigned long long)sb);
    }
    pending &= ~mask;
  }
}

// wave_add2_by_key for one array.
__device__ inline void wave_add_by_key(uint32_t key, long long va, long long* a) {
  const uint32_t lane = threadIdx.x % kWave;
  unsigned long long pending = __ballot(key != kNone);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t lk = __shfl(key, leader);
    const unsigned long long mask = __ballot(key == lk) & pending;
    long long sa = ((mask >> lane) & 1ull) ? va : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) sa += __shfl_xor(sa, o);
    if ((int)lane == leader) atomicAdd((unsigned long long*)&a[lk], (unsigned long long)sa);
    pending &= ~mask;
  }
}

// Keyed append of a block's tile.  Every thread of the block calls this
// (block-uniform control flow) with U (key, value) pairs; key kNone appends
// nothing, any other key is below nk <= kBlock.  Per key the whole tile
// reserves one run of that key's list with a single global atomic: all
// atomics on one address are serialised device-wide, so per-wavefront
// reservations on a few shared counters cost far more than the writes.
// scnt[nk] must hold zeros on entry and holds zeros again on return; sbase[nk]
// is scratch.  list_of(key, list, count) names the key's list and counter.
template <int U, typename ListOf>
__device__ inline void tile_append(const uint32_t (&key)[U], const uint32_t (&val)[U], uint32_t nk,
                                   unsigned int* scnt, unsigned int* sbase, ListOf list_of) {
  uint32_t off[U];
#pragma unroll
  for (int u = 0; u < U; ++u) off[u] = key[u] == kNone ? 0u : atomicAdd(&scnt[key[u]], 1u);
  __syncthreads();
  if (threadIdx.x < nk) {
    const unsigned int c = scnt[threadIdx.x];
    if (c) {
      uint32_t* list;
      unsigned int* count;
      list_of(threadIdx.x, list, count);
      sbase[threadIdx.x] = atomicAdd(count, c);
    }
    scnt[threadIdx.x] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (key[u] == kNone) continue;
    uint32_t* list;
    unsigned int* count;
    list_of(key[u], list, count);
    list[sbase[key[u]] + off[u]] = val[u];
  }
}

// In-place exclusive scan of a[0, n) (n <= kPer * kBlock) by the whole block;
// returns the total.  wsum holds kBlock / kWave words.
template <uint32_t kPer>
__device__ inline uint32_t block_exclusive_scan(unsigned int* a, uint32_t n, unsigned int* wsum) {
  const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  unsigned int x[kPer], tot = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t i = threadIdx.x * kPer + q;
    x[q] = i < n ? a[i] : 0u;
    tot += x[q];
  }
  unsigned int incl = tot;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned int y = __shfl_up(incl, o);
    if ((int)lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  unsigned int run = incl - tot, total = 0;
#pragma unroll
  for (uint32_t q = 0; q < kBlock / kWave; ++q) {
    if (q < wv) run += wsum[q];
    total += wsum[q];
  }
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t i = threadIdx.x * kPer + q;
    if (i < n) a[i] = run;
    run += x[q];
  }
  __syncthreads();
  return total;
}

__host__ __device__ inline uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace lm
