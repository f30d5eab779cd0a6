// Local-moving (Alg. 6) and refinement (Alg. 8) kernels for gfx950.
//
// One synchronous sub-round is: bin the active vertices by degree, decide
// every active vertex against the current state with the degree-binned hash
// kernels (scanCommunities / scanBounded into a per-vertex open-addressing
// table, then the best community by Eq. 2), then apply all decided moves.
// Lists and counters live on the device; every list kernel is a grid-stride
// loop that reads its item count from device memory, so a sub-round needs no
// host round trip.
#include "kernels.h"

namespace lm {

static int grid_for(uint64_t items, int per_block, int cap);

__global__ void k_clear_misc6(Ctl* ctl) { ctl->misc[6] = 0; }

// ---------------------------------------------------------------------------
// Class distribution (start of a local-moving iteration)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_distribute(const uint32_t* in_list, const unsigned int* in_count,
                                                       uint32_t n_all, uint32_t li, uint32_t P, uint32_t stamp,
                                                       uint32_t* pend_mark, uint32_t* cls_lists, size_t stride,
                                                       Ctl* ctl) {
  __shared__ unsigned int lcount[kMaxClasses], lbase[kMaxClasses];
  const uint32_t cnt = in_count ? *in_count : n_all;
  for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += gridDim.x * kBlock) {
    if (threadIdx.x < kMaxClasses) lcount[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t i = base + threadIdx.x;
    uint32_t v = 0, k = 0, pos = 0;
    const bool ok = i < cnt;
    if (ok) {
      v = in_list ? in_list[i] : i;
      k = vertex_class(v, li, P);
      pend_mark[v] = stamp;
      pos = atomicAdd(&lcount[k], 1u);
    }
    __syncthreads();
    if (threadIdx.x < P && lcount[threadIdx.x] > 0)
      lbase[threadIdx.x] = atomicAdd(&ctl->cls_count[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (ok) cls_lists[(size_t)k * stride + lbase[k] + pos] = v;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Degree binning of one class list.  Vertices outside the affected range
// (Delta-screening, first pass) and vertices without entries are processed
// without a decision.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bin(const uint32_t* list, const unsigned int* count,
                                                const uint32_t* len, const uint8_t* in_range, uint32_t* bin_lists,
                                                size_t stride, Ctl* ctl) {
  __shared__ unsigned int lcount[kBins], lbase[kBins];
  const uint32_t cnt = *count;
  for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += gridDim.x * kBlock) {
    if (threadIdx.x < kBins) lcount[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t i = base + threadIdx.x;
    uint32_t v = 0, pos = 0;
    int b = -1;
    if (i < cnt) {
      v = list[i];
      const uint32_t d = len[v];
      if (d > 0 && (!in_range || in_range[v])) {
        b = bin_of_degree(d);
        pos = atomicAdd(&lcount[b], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x < kBins && lcount[threadIdx.x] > 0)
      lbase[threadIdx.x] = atomicAdd(&ctl->bin_count[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (b >= 0) bin_lists[(size_t)b * stride + lbase[b] + pos] = v;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Decision kernels.  REFINE selects Alg. 8 (bounded scan, isolated movers,
// targets that cannot move in the same colour round) instead of Alg. 6.
// ---------------------------------------------------------------------------
template <typename W, bool REFINE>
__device__ inline bool allowed_target(const DecideParams<W>& p, uint32_t c) {
  if (!REFINE) return true;
  return p.size[c] >= 2 || vertex_colour(c, p.R) != p.colour;
}

template <typename W, bool REFINE>
__device__ inline void emit_decision(const DecideParams<W>& p, uint32_t v, uint32_t d, double bdq, uint32_t bc) {
  if (bc == kNone || !(bdq > 0.0)) return;
  // two singletons of one class would swap forever: only the higher label moves
  if (!REFINE && p.size[d] == 1 && p.size[bc] == 1 && bc > d) return;
  const unsigned int pos = atomicAdd(&p.ctl->mover_count, 1u);
  p.movers[pos] = Mover{v, bc, bdq};
}

// G lanes per vertex (G <= 64, groups inside one wavefront), T slots each.
template <int G, int T, typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_decide_group(DecideParams<W> p) {
  constexpr int GPB = kBlock / G;
  __shared__ uint32_t keys[GPB * T];
  __shared__ unsigned long long vals[GPB * T];
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* tk = keys + g * T;
  unsigned long long* tv = vals + g * T;
  const uint32_t cnt = *p.count;
  unsigned long long edges = 0;
  for (uint32_t base = blockIdx.x * GPB; base < cnt; base += gridDim.x * GPB) {
    const uint32_t item = base + g;
    for (int s = lane; s < T; s += G) {
      tk[s] = kNone;
      tv[s] = 0;
    }
    __syncthreads();
    bool valid = item < cnt;
    uint32_t v = 0, d = 0;
    unsigned long long kid = 0;
    if (valid) {
      v = p.list[item];
      d = p.C[v];
      if (REFINE && p.size[d] != 1) valid = false;  // no longer isolated
    }
    if (valid) {
      const int64_t s0 = p.g.start[v];
      const uint32_t L = p.g.len[v];
      const uint32_t bnd = REFINE ? p.CB[v] : 0;
      if (!REFINE && lane == 0) edges += L;
      for (uint32_t e = lane; e < L; e += G) {
        const uint32_t j = p.g.cols[s0 + e];
        if (j == v) continue;
        if (REFINE && p.CB[j] != bnd) continue;
        const uint32_t c = p.C[j];
        const unsigned long long w = (unsigned long long)p.g.w[s0 + e];
        if (c == d)
          kid += w;
        else
          table_add(tk, tv, T - 1, c, w);
      }
    }
    __syncthreads();
    kid = group_sum<G>(kid);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    if (valid) {
      const int64_t ki = p.K[v], sd = p.S[d];
      for (int s = lane; s < T; s += G) {
        const uint32_t c = tk[s];
        if (c == kNone || !allowed_target<W, REFINE>(p, c)) continue;
        const double dq = delta_q((int64_t)tv[s], (int64_t)kid, ki, p.S[c], sd, p.inv_m, p.inv_2m2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    group_best<G>(bdq, bc);
    if (valid && lane == 0) emit_decision<W, REFINE>(p, v, d, bdq, bc);
    __syncthreads();
  }
  if (edges) atomicAdd(&p.ctl->edges, edges);
}

// One block (kBlock lanes) per vertex, T-slot table in LDS.
template <int T, typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_decide_block(DecideParams<W> p) {
  __shared__ uint32_t tk[T];
  __shared__ unsigned long long tv[T];
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ double rdq[kBlock / kWave];
  __shared__ uint32_t rc[kBlock / kWave];
  constexpr uint32_t mask = T - 1;
  const uint32_t cnt = *p.count;
  unsigned long long edges = 0;
  for (uint32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const uint32_t v = p.list[item];
    const uint32_t d = p.C[v];
    for (uint32_t s = threadIdx.x; s <= mask; s += kBlock) {
      tk[s] = kNone;
      tv[s] = 0;
    }
    __syncthreads();
    const bool valid = !(REFINE && p.size[d] != 1);
    unsigned long long kid = 0;
    if (valid) {
      const int64_t s0 = p.g.start[v];
      const uint32_t L = p.g.len[v];
      const uint32_t bnd = REFINE ? p.CB[v] : 0;
      if (!REFINE && threadIdx.x == 0) edges += L;
      for (uint32_t e = threadIdx.x; e < L; e += kBlock) {
        const uint32_t j = p.g.cols[s0 + e];
        if (j == v) continue;
        if (REFINE && p.CB[j] != bnd) continue;
        const uint32_t c = p.C[j];
        const unsigned long long w = (unsigned long long)p.g.w[s0 + e];
        if (c == d)
          kid += w;
        else
          table_add(tk, tv, mask, c, w);
      }
    }
    __syncthreads();
    kid = block_sum(kid, red);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    if (valid) {
      const int64_t ki = p.K[v], sd = p.S[d];
      for (uint32_t s = threadIdx.x; s <= mask; s += kBlock) {
        const uint32_t c = tk[s];
        if (c == kNone || !allowed_target<W, REFINE>(p, c)) continue;
        const double dq = delta_q((int64_t)tv[s], (int64_t)kid, ki, p.S[c], sd, p.inv_m, p.inv_2m2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    block_best(bdq, bc, rdq, rc);
    if (valid && threadIdx.x == 0) emit_decision<W, REFINE>(p, v, d, bdq, bc);
    __syncthreads();
  }
  if (edges) atomicAdd(&p.ctl->edges, edges);
}

// ---------------------------------------------------------------------------
// Hub bin: all blocks share every hub's row.  Each block sums a chunk of
// 2048 entries by community in LDS and adds each distinct community once to
// the hub's global table (and K_{i->d} to its accumulator); then one block per
// hub picks the best community from the table and clears it for the next use.
// ---------------------------------------------------------------------------
constexpr uint32_t kHubChunk = 2048, kHubSlots = 4096;

template <typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_hub_insert(DecideParams<W> p) {
  __shared__ uint32_t lk[kHubSlots];
  __shared__ unsigned long long lv[kHubSlots];
  __shared__ unsigned long long red[kBlock / kWave];
  for (int s = threadIdx.x; s < (int)kHubSlots; s += kBlock) {
    lk[s] = kNone;
    lv[s] = 0;
  }
  __syncthreads();
  const uint32_t cnt = *p.count;
  unsigned long long edges = 0;
  for (uint32_t h = 0; h < cnt; ++h) {
    const uint32_t v = p.list[h];
    const uint32_t d = p.C[v];
    if (REFINE && p.size[d] != 1) continue;  // block-uniform
    const uint32_t hi = p.hub_idx[v];
    uint32_t* tk = p.hub_keys + p.hub_off[hi];
    unsigned long long* tv = p.hub_vals + p.hub_off[hi];
    const uint32_t mask = p.hub_mask[hi];
    const int64_t s0 = p.g.start[v];
    const uint32_t L = p.g.len[v];
    const uint32_t bnd = REFINE ? p.CB[v] : 0;
    // chunk c of hub h goes to block (c + 97 h) mod grid, spreading the first
    // chunks of consecutive hubs over different blocks
    const uint32_t rot = (uint32_t)(((uint64_t)h * 97u) % gridDim.x);
    const uint32_t first = (blockIdx.x + gridDim.x - rot) % gridDim.x;
    for (uint32_t cb = first * kHubChunk; cb < L; cb += gridDim.x * kHubChunk) {
      const uint32_t ce = min(L, cb + kHubChunk);
      unsigned long long kid = 0;
      for (uint32_t e = cb + threadIdx.x; e < ce; e += kBlock) {
        const uint32_t j = p.g.cols[s0 + e];
        if (j == v) continue;
        if (REFINE && p.CB[j] != bnd) continue;
        const uint32_t c = p.C[j];
        const unsigned long long w = (unsigned long long)p.g.w[s0 + e];
        if (c == d)
          kid += w;
        else
          table_add(lk, lv, kHubSlots - 1, c, w);
      }
      if (!REFINE && threadIdx.x == 0) edges += ce - cb;
      kid = block_sum(kid, red);
      if (threadIdx.x == 0 && kid) atomicAdd(&p.hub_kid[hi], kid);
      for (int s = threadIdx.x; s < (int)kHubSlots; s += kBlock) {
        const uint32_t k = lk[s];
        if (k == kNone) continue;
        table_add(tk, tv, mask, k, lv[s]);
        lk[s] = kNone;
        lv[s] = 0;
      }
      __syncthreads();
    }
  }
  if (edges) atomicAdd(&p.ctl->edges, edges);
}

template <typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_hub_select(DecideParams<W> p) {
  __shared__ double rdq[kBlock / kWave];
  __shared__ uint32_t rc[kBlock / kWave];
  const uint32_t cnt = *p.count;
  for (uint32_t h = blockIdx.x; h < cnt; h += gridDim.x) {
    const uint32_t v = p.list[h];
    const uint32_t d = p.C[v];
    const bool valid = !(REFINE && p.size[d] != 1);
    const uint32_t hi = p.hub_idx[v];
    uint32_t* tk = p.hub_keys + p.hub_off[hi];
    unsigned long long* tv = p.hub_vals + p.hub_off[hi];
    const uint32_t mask = p.hub_mask[hi];
    const int64_t kid = (int64_t)p.hub_kid[hi];
    const int64_t ki = p.K[v], sd = p.S[d];
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    for (uint32_t s = threadIdx.x; s <= mask; s += kBlock) {
      const uint32_t c = tk[s];
      if (c == kNone) continue;
      const int64_t kic = (int64_t)tv[s];
      tk[s] = kNone;
      tv[s] = 0;
      if (!valid || !allowed_target<W, REFINE>(p, c)) continue;
      const double dq = delta_q(kic, kid, ki, p.S[c], sd, p.inv_m, p.inv_2m2);
      if (better(dq, c, bdq, bc)) {
        bdq = dq;
        bc = c;
      }
    }
    block_best(bdq, bc, rdq, rc);
    if (threadIdx.x == 0) {
      p.hub_kid[hi] = 0;
      if (valid) emit_decision<W, REFINE>(p, v, d, bdq, bc);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Hub bin, LDS-resident form.  The neighbour communities of a hub are split
// into P key partitions (P from the hub's distinct-community count at its
// last use, else from its degree); one 1024-thread block per (hub, partition)
// scans the whole row, sums the weights of its partition's communities in a
// 16384-slot LDS table and picks its best candidate.  The last block of a hub
// combines the partial results.  A table that reaches its capacity sends the
// hub to the global-table kernels above instead (no decision is emitted
// here), so the result never depends on the estimate.
// ---------------------------------------------------------------------------
constexpr int kHubThreads = 1024;
constexpr uint32_t kHubLdsSlots = 16384, kHubLdsCap = 12288;

__device__ inline uint32_t hub_parts(uint32_t est, uint32_t len) {
  const uint32_t d = est ? est + est / 4 : len;
  const uint32_t p = (d + kHubLdsCap - 1) / kHubLdsCap;
  return p < 1 ? 1 : (p > kHubMaxParts ? kHubMaxParts : p);
}

__device__ inline uint32_t key_part(uint32_t c, uint32_t P) { return P == 1 ? 0 : (fmix32(c) >> 4) % P; }

template <typename W>
__global__ __launch_bounds__(kBlock) void k_hub_items(DecideParams<W> p) {
  const uint32_t cnt = *p.count;
  for (uint32_t h = blockIdx.x * kBlock + threadIdx.x; h < cnt; h += gridDim.x * kBlock) {
    const uint32_t v = p.list[h];
    const uint32_t P = hub_parts(p.hub_est[v], p.g.len[v]);
    const unsigned int base = atomicAdd(&p.ctl->hub_items, P);
    for (uint32_t q = 0; q < P; ++q)
      p.hub_items[base + q] = ((unsigned long long)v << 32) | ((unsigned long long)P << 8) | q;
  }
}

template <typename T>
__device__ inline T hub_block_sum(T x, T* red) {
  x = group_sum<kWave>(x);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  T r = 0;
#pragma unroll
  for (int i = 0; i < kHubThreads / kWave; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ inline void hub_block_best(double& dq, uint32_t& c, double* rdq, uint32_t* rc) {
  group_best<kWave>(dq, c);
  if (threadIdx.x % kWave == 0) {
    rdq[threadIdx.x / kWave] = dq;
    rc[threadIdx.x / kWave] = c;
  }
  __syncthreads();
  dq = -INFINITY;
  c = kNone;
#pragma unroll
  for (int i = 0; i < kHubThreads / kWave; ++i)
    if (better(rdq[i], rc[i], dq, c)) {
      dq = rdq[i];
      c = rc[i];
    }
  __syncthreads();
}

template <typename W, bool REFINE>
__global__ __launch_bounds__(kHubThreads) void k_hub_lds(DecideParams<W> p) {
  __shared__ uint32_t tk[kHubLdsSlots];
  __shared__ uint32_t tv[kHubLdsSlots];
  __shared__ unsigned long long red[kHubThreads / kWave];
  __shared__ double rdq[kHubThreads / kWave];
  __shared__ uint32_t rc[kHubThreads / kWave];
  __shared__ unsigned int used, over, last;
  constexpr uint32_t mask = kHubLdsSlots - 1;
  const uint32_t items = p.ctl->hub_items;
  unsigned long long edges = 0;
  for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
    const unsigned long long item = p.hub_items[it];
    const uint32_t v = (uint32_t)(item >> 32), P = (uint32_t)(item >> 8) & 0xFFu, q = (uint32_t)item & 0xFFu;
    const uint32_t d = p.C[v];
    const uint32_t hi = p.hub_idx[v];
    const bool valid = !(REFINE && p.size[d] != 1);  // block-uniform
    for (uint32_t sl = threadIdx.x; sl < kHubLdsSlots; sl += kHubThreads) {
      tk[sl] = kNone;
      tv[sl] = 0;
    }
    if (threadIdx.x == 0) {
      used = 0;
      // 32-bit sums need K_i < 2^32; a heavier hub takes the global tables
      over = p.K[v] >= (int64_t)0xFFFFFFFFll ? 1u : 0u;
    }
    __syncthreads();
    unsigned long long kid = 0;
    if (valid && !over) {
      const int64_t s0 = p.g.start[v];
      const uint32_t L = p.g.len[v];
      const uint32_t bnd = REFINE ? p.CB[v] : 0;
      for (uint32_t e = threadIdx.x; e < L; e += kHubThreads) {
        const uint32_t j = p.g.cols[s0 + e];
        if (j == v) continue;
        if (REFINE && p.CB[j] != bnd) continue;
        const uint32_t c = p.C[j];
        const uint32_t w = (uint32_t)p.g.w[s0 + e];
        if (c == d) {
          kid += w;
          continue;
        }
        if (key_part(c, P) != q || __atomic_load_n(&over, __ATOMIC_RELAXED)) continue;
        uint32_t h = slot_hash(c, mask);
        while (true) {
          const uint32_t k = tk[h];
          if (k == c) {
            atomicAdd(&tv[h], w);
            break;
          }
          if (k == kNone) {
            const uint32_t o = atomicCAS(&tk[h], kNone, c);
            if (o == kNone) {
              atomicAdd(&tv[h], w);
              // at most kHubLdsCap + 2 * kHubThreads slots are ever claimed
              if (atomicAdd(&used, 1u) + 1 >= kHubLdsCap) atomicExch(&over, 1u);
              break;
            }
            if (o == c) {
              atomicAdd(&tv[h], w);
              break;
            }
          }
          h = (h + 1) & mask;
        }
      }
    }
    kid = hub_block_sum(kid, red);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    const bool ok = valid && !over;
    if (ok) {
      const int64_t ki = p.K[v], sd = p.S[d];
      for (uint32_t sl = threadIdx.x; sl < kHubLdsSlots; sl += kHubThreads) {
        const uint32_t c = tk[sl];
        if (c == kNone || !allowed_target<W, REFINE>(p, c)) continue;
        const double dq = delta_q((int64_t)tv[sl], (int64_t)kid, ki, p.S[c], sd, p.inv_m, p.inv_2m2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    hub_block_best(bdq, bc, rdq, rc);
    if (threadIdx.x == 0) {
      if (P == 1) {
        if (ok) {
          emit_decision<W, REFINE>(p, v, d, bdq, bc);
          p.hub_est[v] = used;
          if (!REFINE) edges += p.g.len[v];
        } else if (valid) {
          p.hub_over_list[atomicAdd(&p.ctl->hub_over, 1u)] = v;
        }
        last = 0;
      } else {
        const size_t slot = (size_t)hi * kHubMaxParts + q;
        p.hub_pdq[slot] = ok ? bdq : NAN;  // NaN marks an overflowed partition
        p.hub_pc[slot] = bc;
        p.hub_pkeys[slot] = used;
        __threadfence();
        last = atomicAdd(&p.hub_done[hi], 1u) == P - 1 ? 1u : 0u;
      }
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
      // every partition of this hub has finished: combine in partition order
      __threadfence();
      bool all_ok = true;
      double cdq = -INFINITY;
      uint32_t cc = kNone, keys = 0;
      const size_t base = (size_t)hi * kHubMaxParts;
      for (uint32_t r = 0; r < P; ++r) {
        const double x = __longlong_as_double((long long)__atomic_load_n(
            reinterpret_cast<unsigned long long*>(&p.hub_pdq[base + r]), __ATOMIC_RELAXED));
        const uint32_t xc = __atomic_load_n(&p.hub_pc[base + r], __ATOMIC_RELAXED);
        keys += __atomic_load_n(&p.hub_pkeys[base + r], __ATOMIC_RELAXED);
        if (x != x) {
          all_ok = false;
          continue;
        }
        if (better(x, xc, cdq, cc)) {
          cdq = x;
          cc = xc;
        }
      }
      p.hub_done[hi] = 0;
      if (all_ok) {
        emit_decision<W, REFINE>(p, v, d, cdq, cc);
        p.hub_est[v] = keys;
        if (!REFINE) edges += p.g.len[v];
      } else if (valid) {
        p.hub_over_list[atomicAdd(&p.ctl->hub_over, 1u)] = v;
      }
    }
    __syncthreads();
  }
  if (edges) {
    atomicAdd(&p.ctl->edges, edges);
    if (sizeof(W) == 4 && !REFINE) atomicAdd(&p.ctl->kt_units[LEIDEN_KT_HUB_INSERT], edges);
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_list(const uint32_t* len, uint32_t nl, uint32_t* list, Ctl* ctl) {
  __shared__ unsigned int s2[2];
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < nl; base += (uint64_t)gridDim.x * kBlock) {
    const uint64_t i = base + threadIdx.x;
    const bool hub = i < nl && len[i] > kBinMaxDeg[kBins - 2];
    block_append(list, &ctl->misc[6], hub, (uint32_t)i, s2);
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_sizes(const uint32_t* len, uint32_t cnt, HubLayout h) {
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < cnt; k += gridDim.x * kBlock) {
    const uint32_t v = h.list[k];
    const uint32_t t = pow2_at_least(2 * len[v]);
    h.size_tmp[k] = t;
    h.mask[k] = t - 1;
    h.idx[v] = k;
  }
}

int hub_layout(hipStream_t s, const uint32_t* len, uint32_t nl, HubLayout& h, Ctl* ctl, void* scan_tmp,
               uint64_t* total_dev, uint32_t* count_out, uint64_t* slots_out) {
  hipLaunchKernelGGL(k_clear_misc6, dim3(1), dim3(1), 0, s, ctl);
  hipLaunchKernelGGL(k_hub_list, dim3(grid_for(nl, kBlock, 4096)), dim3(kBlock), 0, s, len, nl, h.list, ctl);
  unsigned int cnt = 0;
  if (hipMemcpyAsync(&cnt, &ctl->misc[6], sizeof(cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  *count_out = cnt;
  *slots_out = 0;
  if (cnt == 0) return 0;
  hipLaunchKernelGGL(k_hub_sizes, dim3(grid_for(cnt, kBlock, 1024)), dim3(kBlock), 0, s, len, cnt, h);
  exclusive_scan_u64(s, h.size_tmp, h.off, cnt, total_dev, scan_tmp);
  uint64_t slots = 0;
  if (hipMemcpyAsync(&slots, total_dev, sizeof(slots), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  *slots_out = slots;
  return 0;
}

// ---------------------------------------------------------------------------
// Apply kernels
// ---------------------------------------------------------------------------

// A neighbour j of a mover in class k: if j's class comes later it joins
// that class's sub-round of this iteration, otherwise it is queued as
// unprocessed for the next iteration (each vertex at most once per list).
__device__ inline void mark_neighbour(const ApplyParams& p, uint32_t j) {
  const uint32_t kj = vertex_class(j, p.li, p.P);
  if (kj > p.k) {
    if (atomicExch(&p.pend_mark[j], p.stamp) != p.stamp)
      list_push(p.cls_lists + (size_t)kj * p.cls_stride, &p.ctl->cls_count[kj], j);
  } else {
    if (atomicExch(&p.unproc_mark[j], p.stamp + 1) != p.stamp + 1) list_push(p.next_list, &p.ctl->next_count, j);
  }
}

// Local-moving moves: one wavefront per mover.  Lane 0 moves the vertex
// (C, Sigma, member counts, gain sum, split flag of the source community);
// all lanes mark the neighbours: a neighbour of a later class joins that
// class's sub-round of this iteration, any other neighbour is queued as
// unprocessed for the next iteration.
__global__ __launch_bounds__(kBlock) void k_apply_moves(ApplyParams p) {
  const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  const uint32_t cnt = p.ctl->mover_count;
  long long dqsum = 0;
  for (uint32_t m = wave; m < cnt; m += nwaves) {
    const Mover mv = p.movers[m];
    const uint32_t v = mv.v;
    if (lane == 0) {
      const uint32_t d = p.C[v];
      const long long k = p.K[v];
      p.C[v] = mv.c;
      atomicAdd((unsigned long long*)&p.S[d], (unsigned long long)(-k));
      atomicAdd((unsigned long long*)&p.S[mv.c], (unsigned long long)k);
      atomicSub(&p.size[d], 1u);
      atomicAdd(&p.size[mv.c], 1u);
      dqsum += gain_fixed(mv.dq);
      if (p.dS) p.dS[d] = 1;
    }
    const uint32_t L = p.len[v];
    if (L > kBigRow) {
      if (lane == 0) list_push(p.big_list, &p.ctl->big_count, v);
      continue;
    }
    const int64_t s0 = p.start[v];
    for (uint32_t e = lane; e < L; e += kWave) mark_neighbour(p, p.cols[s0 + e]);
  }
  if (lane == 0 && dqsum != 0) atomicAdd(&p.ctl->dq_fixed, (unsigned long long)dqsum);
  if (lane == 0 && wave == 0) atomicAdd(&p.ctl->total_moves, (unsigned long long)cnt);
}

// Neighbour marking of movers with long rows: every block takes a share of
// each such row.
__global__ __launch_bounds__(kBlock) void k_mark_big(ApplyParams p) {
  const uint32_t nbig = p.ctl->big_count;
  for (uint32_t m = 0; m < nbig; ++m) {
    const uint32_t v = p.big_list[m];
    const int64_t s0 = p.start[v];
    const uint32_t L = p.len[v];
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < L; e += gridDim.x * kBlock) mark_neighbour(p, p.cols[s0 + e]);
  }
}

// Refinement moves: an isolated vertex joins its chosen sub-community.
__global__ __launch_bounds__(kBlock) void k_apply_refine(uint32_t* C, int64_t* S, const int64_t* K, uint32_t* size,
                                                         const Mover* movers, Ctl* ctl) {
  const uint32_t cnt = ctl->mover_count;
  for (uint32_t m = blockIdx.x * kBlock + threadIdx.x; m < cnt; m += gridDim.x * kBlock) {
    const Mover mv = movers[m];
    const uint32_t d = C[mv.v];
    const long long k = K[mv.v];
    C[mv.v] = mv.c;
    atomicAdd((unsigned long long*)&S[d], (unsigned long long)(-k));
    atomicAdd((unsigned long long*)&S[mv.c], (unsigned long long)k);
    atomicSub(&size[d], 1u);
    atomicAdd(&size[mv.c], 1u);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctl->refine_moves, (unsigned long long)cnt);
}

__global__ void k_subround_reset(Ctl* ctl) {
  if (threadIdx.x < kBins) ctl->bin_count[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ctl->mover_count = 0;
    ctl->big_count = 0;
    ctl->hub_items = 0;
    ctl->hub_over = 0;
  }
}

// Start of an iteration: the vertices queued as unprocessed become this
// iteration's input (the host swaps the two list buffers to match).
__global__ void k_iteration_reset(Ctl* ctl, uint32_t P) {
  if (threadIdx.x < kMaxClasses) ctl->cls_count[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ctl->dq_fixed = 0;
    ctl->iter_count = ctl->next_count;
    ctl->next_count = 0;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int grid_for(uint64_t items, int per_block, int cap) {
  uint64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap) b = cap;
  return (int)b;
}

void launch_distribute(hipStream_t s, const uint32_t* in_list, const unsigned int* in_count, uint32_t n_upper,
                       uint32_t li, uint32_t P, uint32_t stamp, uint32_t* pend_mark, uint32_t* cls_lists,
                       size_t stride, Ctl* ctl) {
  hipLaunchKernelGGL(k_distribute, dim3(grid_for(n_upper, kBlock, 4096)), dim3(kBlock), 0, s, in_list, in_count,
                     n_upper, li, P, stamp, pend_mark, cls_lists, stride, ctl);
}

void launch_bin(hipStream_t s, const uint32_t* list, const unsigned int* count, uint32_t n_upper, const uint32_t* len,
                const uint8_t* in_range, uint32_t* bin_lists, size_t stride, Ctl* ctl) {
  hipLaunchKernelGGL(k_bin, dim3(grid_for(n_upper, kBlock, 4096)), dim3(kBlock), 0, s, list, count, len, in_range,
                     bin_lists, stride, ctl);
}

template <typename W, bool REFINE>
void launch_decide_all(hipStream_t s, DecideParams<W> p, uint32_t* bin_lists, size_t stride, unsigned int* bin_counts,
                       const uint64_t* bin_upper, uint32_t maxdeg) {
  // bin 0: 8 lanes / 16 slots, bin 1: 32 / 64, bin 2: 64 / 256,
  // bin 3: block / 1024, bin 4: block / 4096, bin 5: hubs (all blocks per hub)
  for (int b = 0; b < kBins; ++b) {
    if (bin_upper[b] == 0) continue;
    DecideParams<W> q = p;
    q.list = bin_lists + (size_t)b * stride;
    q.count = bin_counts + b;
    switch (b) {
      case 0:
        hipLaunchKernelGGL((k_decide_group<8, 16, W, REFINE>), dim3(grid_for(bin_upper[b], kBlock / 8, 2048)),
                           dim3(kBlock), 0, s, q);
        break;
      case 1:
        hipLaunchKernelGGL((k_decide_group<32, 64, W, REFINE>), dim3(grid_for(bin_upper[b], kBlock / 32, 2048)),
                           dim3(kBlock), 0, s, q);
        break;
      case 2:
        hipLaunchKernelGGL((k_decide_group<64, 256, W, REFINE>), dim3(grid_for(bin_upper[b], kBlock / 64, 2048)),
                           dim3(kBlock), 0, s, q);
        break;
      case 3:
        hipLaunchKernelGGL((k_decide_block<1024, W, REFINE>), dim3(grid_for(bin_upper[b], 1, 2048)), dim3(kBlock), 0,
                           s, q);
        break;
      case 4:
        hipLaunchKernelGGL((k_decide_block<4096, W, REFINE>), dim3(grid_for(bin_upper[b], 1, 1024)), dim3(kBlock), 0,
                           s, q);
        break;
      default: {
        hipLaunchKernelGGL((k_hub_items<W>), dim3(grid_for(bin_upper[b], kBlock, 64)), dim3(kBlock), 0, s, q);
        if (sizeof(W) == 4 && !REFINE) kt_mark(LEIDEN_KT_HUB_INSERT, s);
        hipLaunchKernelGGL((k_hub_lds<W, REFINE>), dim3(grid_for(bin_upper[b] * kHubMaxParts, 1, 4096)),
                           dim3(kHubThreads), 0, s, q);
        if (sizeof(W) == 4 && !REFINE) kt_mark(LEIDEN_KT_HUB_INSERT, s);
        // hubs whose LDS tables overflowed (usually none)
        DecideParams<W> o = q;
        o.list = p.hub_over_list;
        o.count = &p.ctl->hub_over;
        hipLaunchKernelGGL((k_hub_insert<W, REFINE>), dim3(grid_for(bin_upper[b] * (maxdeg / kHubChunk + 1), 1, 1024)),
                           dim3(kBlock), 0, s, o);
        hipLaunchKernelGGL((k_hub_select<W, REFINE>), dim3(grid_for(bin_upper[b], 1, 1024)), dim3(kBlock), 0, s, o);
        break;
      }
    }
  }
}

template void launch_decide_all<uint32_t, false>(hipStream_t, DecideParams<uint32_t>, uint32_t*, size_t,
                                                 unsigned int*, const uint64_t*, uint32_t);
template void launch_decide_all<uint32_t, true>(hipStream_t, DecideParams<uint32_t>, uint32_t*, size_t,
                                                unsigned int*, const uint64_t*, uint32_t);
template void launch_decide_all<int64_t, false>(hipStream_t, DecideParams<int64_t>, uint32_t*, size_t,
                                                unsigned int*, const uint64_t*, uint32_t);
template void launch_decide_all<int64_t, true>(hipStream_t, DecideParams<int64_t>, uint32_t*, size_t, unsigned int*,
                                               const uint64_t*, uint32_t);

void launch_apply_moves(hipStream_t s, const ApplyParams& p, uint32_t n_upper, bool long_rows) {
  hipLaunchKernelGGL(k_apply_moves, dim3(grid_for(n_upper, kBlock / kWave, 2048)), dim3(kBlock), 0, s, p);
  if (long_rows) hipLaunchKernelGGL(k_mark_big, dim3(512), dim3(kBlock), 0, s, p);
}

void launch_apply_refine(hipStream_t s, uint32_t* C, int64_t* S, const int64_t* K, uint32_t* size,
                         const Mover* movers, Ctl* ctl, uint32_t n_upper) {
  hipLaunchKernelGGL(k_apply_refine, dim3(grid_for(n_upper, kBlock, 2048)), dim3(kBlock), 0, s, C, S, K, size, movers,
                     ctl);
}

void launch_subround_reset(hipStream_t s, Ctl* ctl) { hipLaunchKernelGGL(k_subround_reset, dim3(1), dim3(64), 0, s, ctl); }

void launch_iteration_reset(hipStream_t s, Ctl* ctl, uint32_t P) {
  hipLaunchKernelGGL(k_iteration_reset, dim3(1), dim3(64), 0, s, ctl, P);
}

__global__ void k_cls_reset(Ctl* ctl) {
  if (threadIdx.x < kMaxClasses) ctl->cls_count[threadIdx.x] = 0;
}

void launch_cls_reset(hipStream_t s, Ctl* ctl) { hipLaunchKernelGGL(k_cls_reset, dim3(1), dim3(64), 0, s, ctl); }

}  // namespace lm
