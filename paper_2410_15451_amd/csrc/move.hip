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
constexpr int kDistU = 8;  // list entries per thread of a tile
__global__ __launch_bounds__(kBlock) void k_distribute(const uint32_t* in_list, const unsigned int* in_count,
                                                       uint32_t n_all, uint32_t li, uint32_t P, uint32_t stamp,
                                                       uint32_t* pend_mark, uint32_t* cls_lists, size_t stride,
                                                       Ctl* ctl) {
  __shared__ unsigned int scnt[kMaxClasses], sbase[kMaxClasses];
  if (threadIdx.x < kMaxClasses) scnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t cnt = in_count ? *in_count : n_all;
  const ForestView F = forest_view(ctl);
  constexpr uint32_t tile = kBlock * kDistU;
  for (uint32_t base = blockIdx.x * tile; base < cnt; base += gridDim.x * tile) {
    uint32_t key[kDistU], val[kDistU];
#pragma unroll
    for (int u = 0; u < kDistU; ++u) {
      const uint32_t i = base + u * kBlock + threadIdx.x;
      key[u] = kNone;
      val[u] = 0;
      if (i < cnt) {
        const uint32_t v = in_list ? in_list[i] : i;
        if (F.moving(v)) {
          key[u] = vertex_class(F.local(v), li, P);
          val[u] = v;
          pend_mark[v] = stamp;
        }
      }
    }
    tile_append<kDistU>(key, val, P, scnt, sbase, [&](uint32_t k, uint32_t*& list, unsigned int*& count) {
      list = cls_lists + (size_t)k * stride;
      count = &ctl->cls_count[k];
    });
  }
}

// ---------------------------------------------------------------------------
// Degree binning of one class list.  Vertices outside the affected range
// (Delta-screening, first pass) and vertices without entries are processed
// without a decision.
// ---------------------------------------------------------------------------
// Hub vertices also queue their row chunks as work items of the hub kernels
// (hub_items, when given).

constexpr int kBinU = 4;  // list entries per thread of a tile
__global__ __launch_bounds__(kBlock) void k_bin(const uint32_t* list, const unsigned int* count,
                                                const uint32_t* len, const uint8_t* in_range, uint32_t* bin_lists,
                                                size_t stride, BinCfg cfg, unsigned long long* hub_items,
                                                Ctl* ctl) {
  __shared__ unsigned int scnt[kBins], sbase[kBins];
  if (threadIdx.x < kBins) scnt[threadIdx.x] = 0;
  // the previous sub-round's mover and marking counts (their readers, the
  // apply and marking kernels, have finished; nothing here reads them)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->mover_count = 0;
    ctl->mark_items = 0;
  }
  __syncthreads();
  const uint32_t cnt = *count;
  constexpr uint32_t tile = kBlock * kBinU;
  for (uint32_t base = blockIdx.x * tile; base < cnt; base += gridDim.x * tile) {
    uint32_t key[kBinU], val[kBinU];
#pragma unroll
    for (int u = 0; u < kBinU; ++u) {
      const uint32_t i = base + u * kBlock + threadIdx.x;
      key[u] = kNone;
      val[u] = 0;
      if (i < cnt) {
        const uint32_t v = list[i];
        const uint32_t d = len[v];
        if (d > 0 && (!in_range || in_range[v])) {
          const int b = bin_of_degree(d, cfg);
          key[u] = (uint32_t)b;
          val[u] = v;
          if (b == kBins - 1 && hub_items) {
            const uint32_t nch = (d + kHubChunk - 1) / kHubChunk;
            const unsigned int first = atomicAdd(&ctl->hub_items, nch);
            for (uint32_t k = 0; k < nch; ++k) hub_items[first + k] = ((unsigned long long)v << 32) | k;
          }
        }
      }
    }
    tile_append<kBinU>(key, val, kBins, scnt, sbase, [&](uint32_t b, uint32_t*& l, unsigned int*& c) {
      l = bin_lists + (size_t)b * stride;
      c = &ctl->bin_count[b];
    });
  }
}

// ---------------------------------------------------------------------------
// Decision kernels.  REFINE selects Alg. 8 (bounded scan, isolated movers,
// targets that cannot move in the same colour round) instead of Alg. 6.
// ---------------------------------------------------------------------------
template <typename W, bool REFINE>
__device__ inline bool allowed_target(const DecideParams<W>& p, const ForestView& F, uint32_t c) {
  if (!REFINE) return true;
  return p.size[c] >= 2 || vertex_colour(F.local(c), p.R) != p.colour;
}

// Eq. 2 constants of vertex v's graph.
template <typename W>
__device__ inline void eq2_consts(const DecideParams<W>& p, const ForestView& F, uint32_t v, double& im,
                                  double& i2) {
  im = p.inv_m;
  i2 = p.inv_2m2;
  if (F.gid) {
    const uint32_t q = F.gid[v];
    im = F.inv[2 * q];
    i2 = F.inv[2 * q + 1];
  }
}

// Asynchronous refinement move of isolated vertex v from its singleton d into
// c (Alg. 8 with the paper's compare-and-swap guard): v first empties its own
// community (only while nobody has joined it), then joins c unless c has been
// emptied meanwhile, in which case v takes its community back.  Members of
// communities with two or more vertices never move in this phase, so every
// community stays connected.
template <typename W>
__device__ inline void refine_move_async(const DecideParams<W>& p, uint32_t v, uint32_t d, uint32_t c) {
  uint32_t* size = const_cast<uint32_t*>(p.size);
  if (atomicCAS(&size[d], 1u, 0u) != 1u) return;
  uint32_t s = ld_sys(&size[c]);
  while (s != 0) {
    const uint32_t o = atomicCAS(&size[c], s, s + 1);
    if (o == s) break;
    s = o;
  }
  if (s == 0) {
    atomicExch(&size[d], 1u);
    return;
  }
  const long long k = p.K[v];
  st_sys(const_cast<uint32_t*>(&p.C[v]), c);
  atomicAdd((unsigned long long*)const_cast<int64_t*>(&p.S[d]), (unsigned long long)(-k));
  atomicAdd((unsigned long long*)const_cast<int64_t*>(&p.S[c]), (unsigned long long)k);
  atomicAdd(&p.ctl->refine_moves, 1ull);
}

// Asynchronous local move: applied at once against the live state; the mover
// is queued only for marking its neighbours.
template <typename W>
__device__ inline void local_move_async(const DecideParams<W>& p, uint32_t v, uint32_t d, double dq, uint32_t c) {
  const long long k = p.K[v];
  st_sys(const_cast<uint32_t*>(&p.C[v]), c);
  atomicAdd((unsigned long long*)const_cast<int64_t*>(&p.S[d]), (unsigned long long)(-k));
  atomicAdd((unsigned long long*)const_cast<int64_t*>(&p.S[c]), (unsigned long long)k);
  atomicSub(const_cast<uint32_t*>(&p.size[d]), 1u);
  atomicAdd(const_cast<uint32_t*>(&p.size[c]), 1u);
  if (p.dS) raise_flag(p.dS, d);
  const Ctl* ctl = p.ctl;
  atomicAdd(ctl->f_gid ? &ctl->f_dq[ctl->f_gid[v]] : &p.ctl->dq_fixed, (unsigned long long)gain_fixed(dq));
  const unsigned int pos = atomicAdd(&p.ctl->mover_count, 1u);
  p.movers[pos] = Mover{v, c, dq};
}

// Movers decided by one block gather in LDS and join the mover list a batch
// at a time: the list's counter sees one atomic per batch, where one per
// wavefront would queue tens of thousands on a single address per sub-round.
constexpr uint32_t kMoverStage = 256;
struct MoverStage {
  Mover m[kMoverStage];
  unsigned int n, base;
};

// Every thread of the block calls this (block-uniform), after a
// __syncthreads that follows the last push.
__device__ inline void stage_flush(MoverStage& st, Ctl* ctl, Mover* movers) {
  const unsigned int n = st.n;
  if (n == 0) return;
  if (threadIdx.x == 0) st.base = atomicAdd(&ctl->mover_count, n);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < n; t += kBlock) movers[st.base + t] = st.m[t];
  __syncthreads();
  if (threadIdx.x == 0) st.n = 0;
  __syncthreads();
}

// st: the block's stage (room for this call guaranteed by the caller), or
// null to append straight to the global list.
template <typename W, bool REFINE>
__device__ inline void emit_decision(const DecideParams<W>& p, uint32_t v, uint32_t d, double bdq, uint32_t bc,
                                     MoverStage* st = nullptr) {
  if (bc == kNone || !(bdq > 0.0)) return;
  // two singletons of one class would swap forever: only the higher label moves
  if (!REFINE && p.size[d] == 1 && p.size[bc] == 1 && bc > d) return;
  if (p.async) {
    if (REFINE)
      refine_move_async(p, v, d, bc);
    else
      local_move_async(p, v, d, bdq, bc);
    return;
  }
  if (st) {
    st->m[atomicAdd(&st->n, 1u)] = Mover{v, bc, bdq};
    return;
  }
  const unsigned int pos = atomicAdd(&p.ctl->mover_count, 1u);
  p.movers[pos] = Mover{v, bc, bdq};
}

// Work units of a decide kernel: local-moving scans and decisions, or
// refinement scans.
template <typename W, bool REFINE>
__device__ inline void add_decide_units(unsigned long long* parts, unsigned long long edges,
                                        unsigned long long verts) {
  if (REFINE) {
    add_units(parts, kWRefScan, edges);
  } else {
    add_edges<W>(parts, edges);
    add_units(parts, kWDecided, verts);
  }
}

// G lanes per vertex (G <= 64, groups inside one wavefront), T slots each;
// this block is block `blk` of `nblk` working on the list.
// LISTED: the tables start empty, each keeps a list of the slots it takes
// (slot_lists, T per group, counts in nslots), and a vertex reads and clears
// only those: a vertex of a few hundred entries has far fewer distinct
// communities than its table has slots.
template <int G, int T, typename W, bool REFINE, bool LISTED = false>
__device__ inline unsigned long long decide_group_body(const DecideParams<W>& p, const uint32_t* list, uint32_t cnt,
                                                       uint32_t blk, uint32_t nblk, uint32_t* keys,
                                                       unsigned long long* vals, MoverStage& st,
                                                       unsigned long long& verts, uint16_t* slot_lists = nullptr,
                                                       unsigned int* nslots = nullptr) {
  constexpr int GPB = kBlock / G;
  static_assert(GPB <= kMoverStage, "one round of decisions must fit the stage");
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* tk = keys + g * T;
  unsigned long long* tv = vals + g * T;
  uint16_t* sl = LISTED ? slot_lists + g * T : nullptr;
  unsigned int* nsl = LISTED ? nslots + g : nullptr;
  const ForestView F = forest_view(p.ctl);
  unsigned long long edges = 0;
  for (uint32_t base = blk * GPB; base < cnt; base += nblk * GPB) {
    const uint32_t item = base + g;
    if (!LISTED) {
      for (int s = lane; s < T; s += G) {
        tk[s] = kNone;
        tv[s] = 0;
      }
    }
    __syncthreads();
    bool valid = item < cnt;
    uint32_t v = 0, d = 0;
    unsigned long long kid = 0;
    if (valid) {
      v = list[item];
      d = p.C[v];
      if (REFINE && p.size[d] != 1) valid = false;  // no longer isolated
    }
    if (valid) {
      const int64_t s0 = p.g.start[v];
      const uint32_t L = p.g.len[v];
      const uint32_t bnd = REFINE ? p.CB[v] : 0;
      if (lane == 0) {
        edges += L;
        verts += 1;
      }
      auto entry = [&](uint32_t e, uint32_t& key, unsigned long long& w) {
        const uint32_t j = p.g.cols[s0 + e];
        if (j == v || (REFINE && p.CB[j] != bnd)) return;
        const uint32_t c = p.C[j];
        w = (unsigned long long)p.g.w[s0 + e];
        if (c == d)
          kid += w;
        else
          key = c;
      };
      if (LISTED)
        table_accumulate_listed(tk, tv, T - 1, lane, L, G, sl, nsl, (uint32_t)T, entry);
      else
        table_accumulate(tk, tv, T - 1, lane, L, G, entry);
    }
    __syncthreads();
    kid = group_sum<G>(kid);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    const uint32_t nused = LISTED ? *nsl : (uint32_t)T;
    if (valid) {
      const int64_t ki = p.K[v], sd = p.S[d];
      double im, i2;
      eq2_consts(p, F, v, im, i2);
      for (uint32_t x = lane; x < nused; x += G) {
        const uint32_t s = LISTED ? sl[x] : x;
        const uint32_t c = tk[s];
        if (c == kNone || !allowed_target<W, REFINE>(p, F, c)) continue;
        const double dq = delta_q((int64_t)tv[s], (int64_t)kid, ki, p.S[c], sd, im, i2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    group_best<G>(bdq, bc);
    if (valid && lane == 0) emit_decision<W, REFINE>(p, v, d, bdq, bc, &st);
    if (LISTED) {  // back to empty: only the slots this vertex took
      for (uint32_t x = lane; x < nused; x += G) {
        const uint32_t s = sl[x];
        tk[s] = kNone;
        tv[s] = 0;
      }
    }
    __syncthreads();
    if (LISTED && lane == 0) *nsl = 0;
    if (st.n + GPB > kMoverStage) stage_flush(st, p.ctl, p.movers);
  }
  __syncthreads();
  stage_flush(st, p.ctl, p.movers);
  return edges;
}

// The three wavefront bins in one launch: the first n0 blocks take bin 0
// (8 lanes, 16 slots per vertex), the next n1 bin 1 (32 / 64), the rest
// bin 2 (64 / 256).
struct SmallBins {
  const uint32_t* list[3];
  const unsigned int* count[3];
  uint32_t n0, n1, n2;
};

template <typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_decide_small(DecideParams<W> p, SmallBins sb) {
  __shared__ uint32_t keys[1024];
  __shared__ unsigned long long vals[1024];
  __shared__ MoverStage st;
  if (threadIdx.x == 0) st.n = 0;
  __syncthreads();
  unsigned long long edges = 0, verts = 0;
  const uint32_t b = blockIdx.x;
  if (b < sb.n0)
    edges = decide_group_body<8, 16, W, REFINE>(p, sb.list[0], *sb.count[0], b, sb.n0, keys, vals, st, verts);
  else if (b < sb.n0 + sb.n1)
    edges =
        decide_group_body<32, 64, W, REFINE>(p, sb.list[1], *sb.count[1], b - sb.n0, sb.n1, keys, vals, st, verts);
  else
    edges = decide_group_body<64, 256, W, REFINE>(p, sb.list[2], *sb.count[2], b - sb.n0 - sb.n1, sb.n2, keys,
                                                  vals, st, verts);
  add_decide_units<W, REFINE>(p.edge_parts, edges, verts);
}

// One block (kBlock lanes) per vertex, T-slot table in LDS.  The table
// starts empty and lists the slots it takes: a vertex reads and clears only
// those (its distinct communities are usually far fewer than the slots).
// V: the table's sums, 64-bit, or 32-bit when 2m < 2^32 (a 4096-slot table
// then takes 32 KB of LDS instead of 48 KB: four blocks per CU instead of
// three, and a block decides one vertex at a time)
template <int T, typename W, bool REFINE, typename V = unsigned long long>
__global__ __launch_bounds__(kBlock) void k_decide_block(DecideParams<W> p) {
  // slot list of at most LC entries (a vertex with more distinct communities
  // reads and clears the whole table); 512 keeps three 4096-slot blocks per CU
  constexpr uint32_t LC = T < 512 ? T : 512;
  __shared__ uint32_t tk[T];
  __shared__ V tv[T];
  __shared__ uint16_t used[LC];
  __shared__ unsigned int nused;
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ double rdq[kBlock / kWave];
  __shared__ uint32_t rc[kBlock / kWave];
  __shared__ MoverStage st;
  constexpr uint32_t mask = T - 1;
  const uint32_t cnt = *p.count;
  const ForestView F = forest_view(p.ctl);
  unsigned long long edges = 0, verts = 0;
  for (uint32_t s = threadIdx.x; s <= mask; s += kBlock) {
    tk[s] = kNone;
    tv[s] = 0;
  }
  if (threadIdx.x == 0) {
    st.n = 0;
    nused = 0;
  }
  __syncthreads();
  // the next vertex's community and row bounds are fetched while the current
  // one is summed (only the block deciding a vertex moves it, so its C entry
  // is the same when its turn comes)
  uint32_t nv = 0, nd = 0, nL = 0;
  int64_t ns0 = 0;
  if (blockIdx.x < cnt) {
    nv = p.list[blockIdx.x];
    nd = p.C[nv];
    ns0 = p.g.start[nv];
    nL = p.g.len[nv];
  }
  for (uint32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const uint32_t v = nv, d = nd;
    const int64_t s0 = ns0;
    const uint32_t L = nL;
    const uint32_t nx = item + gridDim.x;
    const uint32_t nv2 = nx < cnt ? p.list[nx] : 0u;
    const bool valid = !(REFINE && p.size[d] != 1);
    unsigned long long kid = 0;
    if (valid) {
      const uint32_t bnd = REFINE ? p.CB[v] : 0;
      if (threadIdx.x == 0) {
        edges += L;
        verts += 1;
      }
      table_accumulate_listed(tk, tv, mask, threadIdx.x, L, kBlock, used, &nused, LC,
                              [&](uint32_t e, uint32_t& key, unsigned long long& w) {
                                const uint32_t j = p.g.cols[s0 + e];
                                if (j == v || (REFINE && p.CB[j] != bnd)) return;
                                const uint32_t c = p.C[j];
                                w = (unsigned long long)p.g.w[s0 + e];
                                if (c == d)
                                  kid += w;
                                else
                                  key = c;
                              });
    }
    __syncthreads();
    if (nx < cnt) {
      nv = nv2;
      nd = p.C[nv];
      ns0 = p.g.start[nv];
      nL = p.g.len[nv];
    }
    kid = block_sum(kid, red);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    const bool listed = nused <= LC;
    const uint32_t nu = listed ? nused : T;
    if (valid) {
      const int64_t ki = p.K[v], sd = p.S[d];
      double im, i2;
      eq2_consts(p, F, v, im, i2);
      for (uint32_t x = threadIdx.x; x < nu; x += kBlock) {
        const uint32_t s = listed ? used[x] : x;
        const uint32_t c = tk[s];
        if (c == kNone || !allowed_target<W, REFINE>(p, F, c)) continue;
        const double dq = delta_q((int64_t)tv[s], (int64_t)kid, ki, p.S[c], sd, im, i2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    block_best(bdq, bc, rdq, rc);
    if (valid && threadIdx.x == 0) emit_decision<W, REFINE>(p, v, d, bdq, bc, &st);
    for (uint32_t x = threadIdx.x; x < nu; x += kBlock) {  // back to empty
      const uint32_t s = listed ? used[x] : x;
      tk[s] = kNone;
      tv[s] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) nused = 0;
    if (st.n == kMoverStage) stage_flush(st, p.ctl, p.movers);
    __syncthreads();  // the reset before the next vertex's inserts
  }
  __syncthreads();
  stage_flush(st, p.ctl, p.movers);
  add_decide_units<W, REFINE>(p.edge_parts, edges, verts);
}

// ---------------------------------------------------------------------------
// Hub bin (degree above the last LDS bin): a group-by over the hub's row with
// no global hash table and no global counters (global atomics are slow, and
// those on one address are serialised device-wide).  Rows are cut into
// chunks of kHubChunk entries and every (hub, chunk) pair is a work item of
// one block, which
//  - sums its chunk by community in an LDS table and adds its K_{i->d} share
//    to the hub's accumulator,
//  - sorts the chunk's distinct communities by bucket (top bits of
//    fmix32(community)) into the chunk's own staging slots, and writes the
//    bucket starts into the chunk's column of the hub's matrix.
// The pick then gives each block buckets of a hub: a bucket's runs in all
// chunks are summed in an LDS table and the communities found are evaluated;
// the hub's last block combines the blocks' best candidates in a fixed order
// and emits the decision.
// ---------------------------------------------------------------------------
__device__ inline uint32_t hub_bucket(uint32_t c, uint32_t rb) { return rb ? fmix32(c) >> (32 - rb) : 0u; }

// V: the chunk table's sums (32-bit when 2m < 2^32, as in the block decide)
template <typename W, bool REFINE, typename V = unsigned long long>
__global__ __launch_bounds__(kBlock) void k_hub_chunk(DecideParams<W> p) {
  constexpr uint32_t kNB = 1u << kHubMaxRbits;
  __shared__ uint32_t lk[kHubSlots];
  __shared__ V lv[kHubSlots];
  __shared__ unsigned int lcnt[kNB + 1];
  __shared__ unsigned int wsum[kBlock / kWave];
  __shared__ unsigned long long red[kBlock / kWave];
  for (uint32_t sl = threadIdx.x; sl < kHubSlots; sl += kBlock) {
    lk[sl] = kNone;
    lv[sl] = 0;
  }
  for (uint32_t b = threadIdx.x; b <= kNB; b += kBlock) lcnt[b] = 0;
  __syncthreads();
  const uint32_t items = p.ctl->hub_items;
  unsigned long long edges = 0, verts = 0;
  for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
    const unsigned long long item = p.hub_items[it];
    const uint32_t v = (uint32_t)(item >> 32), k = (uint32_t)item;
    const uint32_t d = p.C[v];
    if (REFINE && p.size[d] != 1) continue;  // block-uniform: only isolated vertices are refined
    const uint32_t hi = p.hub_idx[v];
    const int64_t s0 = p.g.start[v];
    const uint32_t L = p.g.len[v];
    const uint32_t cb = k * kHubChunk, ce = min(L, cb + kHubChunk);
    const uint32_t bnd = REFINE ? p.CB[v] : 0;
    unsigned long long kid = 0;
    table_accumulate(lk, lv, kHubSlots - 1, cb + threadIdx.x, ce, kBlock,
                     [&](uint32_t e, uint32_t& key, unsigned long long& w) {
                       const uint32_t j = p.g.cols[s0 + e];
                       if (j == v || (REFINE && p.CB[j] != bnd)) return;
                       const uint32_t c = p.C[j];
                       w = (unsigned long long)p.g.w[s0 + e];
                       if (c == d)
                         kid += w;
                       else
                         key = c;
                     });
    kid = block_sum(kid, red);
    if (threadIdx.x == 0) {
      if (kid) atomicAdd(&p.hub_kid[hi], kid);
      if (k == 0) {
        p.hub_live[hi] = 1;
        verts += 1;
      }
      edges += ce - cb;
    }
    __syncthreads();
    const uint32_t rb = p.hub_rbits[hi], R = 1u << rb;
    const uint32_t nch = (L + kHubChunk - 1) / kHubChunk;
    // counting sort of the chunk's distinct communities by bucket
    for (uint32_t sl = threadIdx.x; sl < kHubSlots; sl += kBlock) {
      const uint32_t c = lk[sl];
      if (c != kNone) atomicAdd(&lcnt[hub_bucket(c, rb)], 1u);
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan<kNB / kBlock>(lcnt, R, wsum);
    if (threadIdx.x == 0) lcnt[R] = total;
    __syncthreads();
    uint16_t* col = p.hub_mat + p.hub_moff[hi] + k;
    for (uint32_t b = threadIdx.x; b <= R; b += kBlock) col[(size_t)b * nch] = (uint16_t)lcnt[b];
    __syncthreads();
    uint32_t* tk = p.hub_keys + p.hub_off[hi] + cb;
    unsigned long long* tv = p.hub_vals + p.hub_off[hi] + cb;
    for (uint32_t sl = threadIdx.x; sl < kHubSlots; sl += kBlock) {
      const uint32_t c = lk[sl];
      if (c == kNone) continue;
      const unsigned int pos = atomicAdd(&lcnt[hub_bucket(c, rb)], 1u);
      tk[pos] = c;
      tv[pos] = lv[sl];
      lk[sl] = kNone;
      lv[sl] = 0;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b <= R; b += kBlock) lcnt[b] = 0;
  }
  if (edges) {
    add_decide_units<W, REFINE>(p.edge_parts, edges, verts);
    if (sizeof(W) == 4 && !REFINE) atomicAdd(&p.ctl->kt_units[LEIDEN_KT_HUB_INSERT], edges);
  }
}

// Pick: the hub's buckets are taken in G = 2^gb groups of consecutive
// buckets (top gb bits of the mixing), G the smallest power of two with about
// kHubBucket staged entries per group; block (x, y) of a grid with gridDim.y
// segments takes groups y, y + nseg, ... of the hubs x, x + gridDim.x, ...
// (nseg = min(G, gridDim.y)).  A group's runs are taken kPickWin chunks at a
// time (run lengths scanned in LDS, each entry found by binary search) and
// summed in an LDS table sized for the group.  Should a group hold more
// distinct communities than the table, it is taken in 2^q sub-groups by the
// next q bits of the same mixing (a bijection, so distinct communities
// eventually part).  Each segment's best candidate goes to the hub's partial results;
// the last segment to finish combines them in segment order.  Every block
// reads the hub's accumulators before it counts itself done, so they are
// stable until the last one resets them.
constexpr uint32_t kPickWin = 2048;

template <typename W, bool REFINE>
__global__ __launch_bounds__(kBlock) void k_hub_pick(DecideParams<W> p) {
  __shared__ uint32_t tk[kHubSlots];
  __shared__ unsigned long long tv[kHubSlots];
  __shared__ unsigned int rpre[kPickWin];  // exclusive prefix of the window's run lengths
  __shared__ uint16_t rst[kPickWin];       // run starts within their chunks
  __shared__ unsigned int wsum[kBlock / kWave];
  __shared__ double rdq[kBlock / kWave];
  __shared__ uint32_t rc[kBlock / kWave];
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ unsigned int last, full;
  bool clean = false;  // the table is cleared once, by blocks that get work
  const uint32_t cnt = *p.count;
  const uint32_t y = blockIdx.y;
  const ForestView F = forest_view(p.ctl);
  for (uint32_t h = blockIdx.x; h < cnt; h += gridDim.x) {
    const uint32_t v = p.list[h];
    const uint32_t d = p.C[v];
    const uint32_t hi = p.hub_idx[v];
    // taking part was settled by the chunk kernel: asynchronous refinement
    // moves made by this kernel may change community sizes meanwhile
    if (p.hub_live[hi] == 0) continue;  // block-uniform; nothing was summed
    const uint32_t rb = p.hub_rbits[hi], R = 1u << rb;
    const uint32_t nch = (p.g.len[v] + kHubChunk - 1) / kHubChunk;
    const uint16_t* mat = p.hub_mat + p.hub_moff[hi];
    // staged entries of the hub (row R of the matrix: the chunks' totals)
    // decide how many buckets one group of this pick takes
    unsigned long long tot = 0;
    for (uint32_t c = threadIdx.x; c < nch; c += kBlock) tot += mat[(size_t)R * nch + c];
    tot = block_sum(tot, red);
    uint32_t gb = 0;
    while (gb < rb && ((unsigned long long)kHubBucket << gb) < tot) ++gb;
    const uint32_t G = 1u << gb, span = rb - gb;
    const uint32_t nseg = min(G, gridDim.y);
    if (y >= nseg) continue;  // block-uniform; this block takes no part for this hub
    if (!clean) {
      for (uint32_t sl = threadIdx.x; sl < kHubSlots; sl += kBlock) {
        tk[sl] = kNone;
        tv[sl] = 0;
      }
      __syncthreads();
      clean = true;
    }
    const uint32_t* sk = p.hub_keys + p.hub_off[hi];
    const unsigned long long* sv = p.hub_vals + p.hub_off[hi];
    const int64_t kid = (int64_t)p.hub_kid[hi];
    const int64_t ki = p.K[v], sd = p.S[d];
    double im, i2;
    eq2_consts(p, F, v, im, i2);
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    for (uint32_t grp = y; grp < G; grp += nseg) {
      // buckets [b0, b1) of this group: contiguous in every chunk
      const uint32_t b0 = grp << span, b1 = (grp + 1) << span;
      for (uint32_t q = 0;; ++q) {  // sub-group bits
        bool fits = true;
        for (uint32_t sub = 0; sub < (1u << q) && fits; ++sub) {
          uint32_t mask = kHubSlots - 1;
          if (threadIdx.x == 0) full = 0;
          for (uint32_t c0 = 0; c0 < nch; c0 += kPickWin) {
            const uint32_t cw = min(kPickWin, nch - c0);
            for (uint32_t i = threadIdx.x; i < cw; i += kBlock) {
              const uint32_t s = mat[(size_t)b0 * nch + c0 + i], e = mat[(size_t)b1 * nch + c0 + i];
              rst[i] = (uint16_t)s;
              rpre[i] = e - s;
            }
            __syncthreads();
            const uint32_t n = block_exclusive_scan<kPickWin / kBlock>(rpre, cw, wsum);
            if (nch <= kPickWin) mask = min(kHubSlots, pow2_at_least(2 * n)) - 1;
            for (uint32_t x = threadIdx.x; x < n; x += kBlock) {
              // chunk i of the window with rpre[i] <= x < rpre[i + 1]
              uint32_t lo = 0, hi2 = cw - 1;
              while (lo < hi2) {
                const uint32_t mid = (lo + hi2 + 1) >> 1;
                if (rpre[mid] <= x)
                  lo = mid;
                else
                  hi2 = mid - 1;
              }
              const size_t pos = (size_t)(c0 + lo) * kHubChunk + rst[lo] + (x - rpre[lo]);
              const uint32_t c = sk[pos];
              if (q && ((fmix32(c) << gb) >> (32 - q)) != sub) continue;
              if (!table_add_bounded(tk, tv, mask, c, sv[pos])) full = 1;
            }
            __syncthreads();
          }
          fits = full == 0;
          for (uint32_t sl = threadIdx.x; sl <= mask; sl += kBlock) {
            const uint32_t c = tk[sl];
            if (c == kNone) continue;
            if (fits && allowed_target<W, REFINE>(p, F, c)) {
              const double dq = delta_q((int64_t)tv[sl], kid, ki, p.S[c], sd, im, i2);
              if (better(dq, c, bdq, bc)) {
                bdq = dq;
                bc = c;
              }
            }
            tk[sl] = kNone;
            tv[sl] = 0;
          }
          __syncthreads();
        }
        if (fits) break;
      }
    }
    block_best(bdq, bc, rdq, rc);
    if (threadIdx.x == 0) {
      if (nseg == 1) {
        last = 1;
      } else {
        const size_t slot = (size_t)hi * p.pick_segs + y;
        p.hub_pdq[slot] = bdq;
        p.hub_pc[slot] = bc;
        __threadfence();
        last = atomicAdd(&p.hub_done[hi], 1u) == nseg - 1 ? 1u : 0u;
        if (last) {
          __threadfence();
          bdq = -INFINITY;
          bc = kNone;
          for (uint32_t r = 0; r < nseg; ++r) {
            const size_t sr = (size_t)hi * p.pick_segs + r;
            const double x = __longlong_as_double(
                (long long)ld_sys(reinterpret_cast<const unsigned long long*>(&p.hub_pdq[sr])));
            const uint32_t xc = ld_sys(&p.hub_pc[sr]);
            if (better(x, xc, bdq, bc)) {
              bdq = x;
              bc = xc;
            }
          }
          p.hub_done[hi] = 0;
        }
      }
      if (last) {
        p.hub_kid[hi] = 0;
        p.hub_live[hi] = 0;
        emit_decision<W, REFINE>(p, v, d, bdq, bc);
      }
    }
    __syncthreads();
  }
}

constexpr int kListU = 8;  // elements per thread of a tile
__global__ __launch_bounds__(kBlock) void k_hub_list(const uint32_t* len, uint32_t nl, uint32_t hub_above,
                                                     uint32_t* list, Ctl* ctl) {
  __shared__ unsigned int scnt[1], sbase[1];
  if (threadIdx.x == 0) scnt[0] = 0;
  __syncthreads();
  constexpr uint32_t tile = kBlock * kListU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < nl; base += (uint64_t)gridDim.x * tile) {
    uint32_t key[kListU], val[kListU];
#pragma unroll
    for (int u = 0; u < kListU; ++u) {
      const uint64_t i = base + u * kBlock + threadIdx.x;
      key[u] = i < nl && len[i] > hub_above ? 0u : kNone;
      val[u] = (uint32_t)i;
    }
    tile_append<kListU>(key, val, 1, scnt, sbase, [&](uint32_t, uint32_t*& l, unsigned int*& c) {
      l = list;
      c = &ctl->misc[6];
    });
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_sizes(const uint32_t* len, uint32_t cnt, HubLayout h) {
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < cnt; k += gridDim.x * kBlock) {
    const uint32_t v = h.list[k];
    const uint32_t L = len[v];
    const uint32_t nch = (L + kHubChunk - 1) / kHubChunk;
    const uint32_t R = pow2_at_least((L + kHubBucket - 1) >> kHubBucketBits);
    uint32_t rb = 0;
    while ((1u << rb) < R && rb < kHubMaxRbits) ++rb;
    h.size_tmp[k] = (uint64_t)nch * kHubChunk;
    h.msize_tmp[k] = (uint64_t)((1u << rb) + 1) * nch;
    h.rbits[k] = rb;
    h.idx[v] = k;
  }
}

int hub_layout(hipStream_t s, const uint32_t* len, uint32_t nl, uint32_t hub_above, HubLayout& h, Ctl* ctl,
               void* scan_tmp, uint64_t* total_dev, uint32_t* count_out, uint64_t* slots_out,
               uint64_t* mat_out) {
  hipLaunchKernelGGL(k_clear_misc6, dim3(1), dim3(1), 0, s, ctl);
  hipLaunchKernelGGL(k_hub_list, dim3(grid_for(nl, kBlock * kListU, 4096)), dim3(kBlock), 0, s, len, nl, hub_above,
                     h.list, ctl);
  unsigned int* pc = (unsigned int*)pinned_stage(4);
  if (!pc || hipMemcpyAsync(pc, &ctl->misc[6], sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  const unsigned int cnt = *pc;
  *count_out = cnt;
  *slots_out = 0;
  *mat_out = 0;
  if (cnt == 0) return 0;
  hipLaunchKernelGGL(k_hub_sizes, dim3(grid_for(cnt, kBlock, 1024)), dim3(kBlock), 0, s, len, cnt, h);
  exclusive_scan_u64(s, h.size_tmp, h.off, cnt, total_dev, scan_tmp);
  exclusive_scan_u64(s, h.msize_tmp, h.moff, cnt, total_dev + 1, scan_tmp);
  uint64_t* ps = (uint64_t*)pinned_stage(16);
  if (!ps || hipMemcpyAsync(ps, total_dev, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  *slots_out = ps[0];
  *mat_out = ps[1];
  return 0;
}

// ---------------------------------------------------------------------------
// Apply kernels
// ---------------------------------------------------------------------------

// The list a marked neighbour j joins: a neighbour of a later class joins
// that class's sub-round of this iteration (key = its class), any other one
// is queued as unprocessed for the next iteration (key = P); kNone if it was
// marked already (each vertex at most once per list: the stamp is read first
// and claimed by exchange only when it is not set).
__device__ inline uint32_t mark_key(const ApplyParams& p, uint32_t j) {
  if (j == kNone) return kNone;
  const uint32_t kj = vertex_class(p.ctl->f_gid ? j - p.ctl->f_base[p.ctl->f_gid[j]] : j, p.li, p.P);
  if (kj > p.k) {
    if (peek(&p.pend_mark[j]) != p.stamp &&
        atomicExch(&p.pend_mark[j], p.stamp) != p.stamp)
      return kj;
  } else {
    if (peek(&p.unproc_mark[j]) != p.stamp + 1 &&
        atomicExch(&p.unproc_mark[j], p.stamp + 1) != p.stamp + 1)
      return p.P;
  }
  return kNone;
}

// Local-moving moves: one thread per mover moves the vertex (C, Sigma, member
// counts, gain sum, split flag of the source community) and cuts its row into
// chunks of kMarkChunk entries, queued as marking work items; then one
// wavefront per item marks the neighbours.  Long and short rows thus spread
// evenly over the machine.  Both kernels reserve list space once per block
// tile, not per wavefront.
constexpr uint32_t kMarkChunk = kWave;
constexpr int kMarkU = 8;  // marking items per wavefront of a tile

// Community deltas of a block's movers are summed in LDS and added once per
// community and iteration: movers gather in a few large communities, and
// atomics on one address are serialised device-wide.
constexpr uint32_t kApplySlots = 1024;
__device__ inline void apply_delta(uint32_t* tk, unsigned long long* ts, unsigned int* tn, uint32_t c, long long ds,
                                   int dn) {
  uint32_t h = slot_hash(c, kApplySlots - 1);
  while (true) {
    const uint32_t k = __atomic_load_n(&tk[h], __ATOMIC_RELAXED);
    if (k == c) break;
    if (k == kNone) {
      const uint32_t o = atomicCAS(&tk[h], kNone, c);
      if (o == kNone || o == c) break;
    }
    h = (h + 1) & (kApplySlots - 1);
  }
  atomicAdd(&ts[h], (unsigned long long)ds);
  atomicAdd(&tn[h], (unsigned int)dn);
}

// The sub-round's bin counts and hub items, cleared for the next sub-round
// by the apply kernel (its decide kernels, their only readers, have finished).
__device__ inline void clear_bins(Ctl* ctl) {
  if (blockIdx.x == 0) {
    if (threadIdx.x < kBins) ctl->bin_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) ctl->hub_items = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_apply_moves(ApplyParams p) {
  clear_bins(p.ctl);
  __shared__ unsigned int wtot[kBlock / kWave];
  __shared__ unsigned int sbase;
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ uint32_t tk[kApplySlots];
  __shared__ unsigned long long ts[kApplySlots];
  __shared__ unsigned int tn[kApplySlots];
  for (uint32_t sl = threadIdx.x; sl < kApplySlots; sl += kBlock) {
    tk[sl] = kNone;
    ts[sl] = 0;
    tn[sl] = 0;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const uint32_t cnt = p.ctl->mover_count;
  const uint32_t* fgid = p.ctl->f_gid;
  long long dqsum = 0;
  unsigned long long marks = 0;
  const uint32_t stride = gridDim.x * kBlock;
  // block-uniform loop: every thread runs every iteration
  for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += stride) {
    const uint32_t m = base + threadIdx.x;
    uint32_t nch = 0, v = 0;
    if (m < cnt) {
      const Mover mv = p.movers[m];
      v = mv.v;
      if (!p.applied) {
        const uint32_t d = p.C[v];
        const long long k = p.K[v];
        p.C[v] = mv.c;
        apply_delta(tk, ts, tn, d, -k, -1);
        apply_delta(tk, ts, tn, mv.c, k, 1);
        if (fgid)
          atomicAdd(&p.ctl->f_dq[fgid[v]], (unsigned long long)gain_fixed(mv.dq));
        else
          dqsum += gain_fixed(mv.dq);
        if (p.dS) raise_flag(p.dS, d);
      }
      nch = (p.len[v] + kMarkChunk - 1) / kMarkChunk;
      marks += p.len[v];
    }
    // wavefront prefix of the chunk counts, then one reservation per block
    uint32_t incl = nch;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if ((int)lane >= o) incl += y;
    }
    if (lane == kWave - 1) wtot[wv] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t q = 0; q < kBlock / kWave; ++q) {
      const uint32_t t = wtot[q];
      if (q < wv) before += t;
      total += t;
    }
    if (threadIdx.x == 0 && total) sbase = atomicAdd(&p.ctl->mark_items, total);
    // the iteration's community deltas (every insert happened before the barrier above)
    for (uint32_t sl = threadIdx.x; sl < kApplySlots; sl += kBlock) {
      const uint32_t c = tk[sl];
      if (c == kNone) continue;
      if (ts[sl]) atomicAdd((unsigned long long*)&p.S[c], ts[sl]);
      if (tn[sl]) atomicAdd(&p.size[c], tn[sl]);
      tk[sl] = kNone;
      ts[sl] = 0;
      tn[sl] = 0;
    }
    __syncthreads();
    const uint32_t first = sbase + before + incl - nch;
    for (uint32_t k = 0; k < nch; ++k) p.mark_items[first + k] = ((unsigned long long)v << 32) | k;
    __syncthreads();
  }
  dqsum = (long long)block_sum((unsigned long long)dqsum, red);
  if (threadIdx.x == 0 && dqsum != 0) atomicAdd(&p.ctl->dq_fixed, (unsigned long long)dqsum);
  marks = block_sum(marks, red);
  if (threadIdx.x == 0) add_units(p.parts, kWMarks, marks);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&p.ctl->total_moves, (unsigned long long)cnt);
}

__global__ __launch_bounds__(kBlock) void k_mark_items(ApplyParams p) {
  __shared__ unsigned int scnt[kMaxClasses + 1], sbase[kMaxClasses + 1];
  const uint32_t wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (threadIdx.x <= kMaxClasses) scnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t items = p.ctl->mark_items;
  constexpr uint32_t tile = kMarkU * (kBlock / kWave);
  for (uint32_t base = blockIdx.x * tile; base < items; base += gridDim.x * tile) {
    uint32_t key[kMarkU], val[kMarkU];
#pragma unroll
    for (int u = 0; u < kMarkU; ++u) {
      const uint32_t it = base + u * (kBlock / kWave) + wv;
      uint32_t j = kNone;
      if (it < items) {
        const unsigned long long item = p.mark_items[it];
        const uint32_t v = (uint32_t)(item >> 32), k = (uint32_t)item;
        const uint32_t e = k * kMarkChunk + lane;
        if (e < p.len[v]) j = p.cols[p.start[v] + e];
      }
      key[u] = mark_key(p, j);
      val[u] = j;
    }
    tile_append<kMarkU>(key, val, p.P + 1, scnt, sbase, [&](uint32_t k, uint32_t*& list, unsigned int*& count) {
      if (k < p.P) {
        list = p.cls_lists + (size_t)k * p.cls_stride;
        count = &p.ctl->cls_count[k];
      } else {
        list = p.next_list;
        count = &p.ctl->next_count;
      }
    });
  }
}

// Refinement moves: an isolated vertex joins its chosen sub-community.
__global__ __launch_bounds__(kBlock) void k_apply_refine(uint32_t* C, int64_t* S, const int64_t* K, uint32_t* size,
                                                         const Mover* movers, Ctl* ctl) {
  clear_bins(ctl);
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
    ctl->mark_items = 0;
    ctl->hub_items = 0;
  }
}

// Start of an iteration: the vertices queued as unprocessed become this
// iteration's input (the host swaps the two list buffers to match); the first
// sub-round's counters start at zero (later sub-rounds: the bin and apply
// kernels of the one before clear them).
__global__ void k_iteration_reset(Ctl* ctl, uint32_t P) {
  if (threadIdx.x < kBins) ctl->bin_count[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ctl->mover_count = 0;
    ctl->mark_items = 0;
    ctl->hub_items = 0;
  }
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
  hipLaunchKernelGGL(k_distribute, dim3(grid_for(n_upper, kBlock * kDistU, 4096)), dim3(kBlock), 0, s, in_list,
                     in_count, n_upper, li, P, stamp, pend_mark, cls_lists, stride, ctl);
}

void launch_bin(hipStream_t s, const uint32_t* list, const unsigned int* count, uint32_t n_upper, const uint32_t* len,
                const uint8_t* in_range, uint32_t* bin_lists, size_t stride, const BinCfg& cfg,
                unsigned long long* hub_items, Ctl* ctl) {
  hipLaunchKernelGGL(k_bin, dim3(grid_for(n_upper, kBlock * kBinU, 4096)), dim3(kBlock), 0, s, list, count, len,
                     in_range, bin_lists, stride, cfg, hub_items, ctl);
}

template <typename W, bool REFINE>
void launch_decide_all(hipStream_t s, DecideParams<W> p, uint32_t* bin_lists, size_t stride, unsigned int* bin_counts,
                       const uint64_t* bin_upper, uint32_t maxdeg, const DecideStreams* ds) {
  // bin 0: 8 lanes / 16 slots, bin 1: 32 / 64, bin 2: 64 / 256 (in one
  // launch on s); bin 3: block / 1024, bin 4: block / 4096, each on its own
  // side stream when ds is given; bin 5: hubs (all blocks per hub), on s
  // after the small bins.  The side streams fork before the small bins'
  // launch, so the three streams run together.  (With four hardware queues
  // per process a third side stream shared a queue with another one, and
  // the hubs then waited for the 4096 bin instead of the small bins, which
  // finish first.)
  bool forked = false;
  if (ds && (bin_upper[3] || bin_upper[4])) {
    (void)hipEventRecord(ds->fork, s);
    forked = true;
  }
  auto side = [&](int k) -> hipStream_t {
    if (!forked) return s;
    (void)hipStreamWaitEvent(ds->aux[k], ds->fork, 0);
    return ds->aux[k];
  };
  bool used[kDecideSide] = {false, false};
  {
    SmallBins sb{};
    uint32_t* nb[3] = {&sb.n0, &sb.n1, &sb.n2};
    const int lanes[3] = {8, 32, 64};
    for (int b = 0; b < 3; ++b) {
      sb.list[b] = bin_lists + (size_t)b * stride;
      sb.count[b] = bin_counts + b;
      *nb[b] = bin_upper[b] ? (uint32_t)grid_for(bin_upper[b], kBlock / lanes[b], 2048) : 0;
    }
    const uint32_t total = sb.n0 + sb.n1 + sb.n2;
    if (total) hipLaunchKernelGGL((k_decide_small<W, REFINE>), dim3(total), dim3(kBlock), 0, s, p, sb);
  }
  for (int b = 3; b < kBins; ++b) {
    if (bin_upper[b] == 0) continue;
    DecideParams<W> q = p;
    q.list = bin_lists + (size_t)b * stride;
    q.count = bin_counts + b;
    const hipStream_t t = b < 5 ? side(b - 3) : s;
    if (b < 5) used[b - 3] = forked;
    switch (b) {
      case 3:
        hipLaunchKernelGGL((k_decide_block<1024, W, REFINE>), dim3(grid_for(bin_upper[b], 1, 2048)), dim3(kBlock), 0,
                           t, q);
        break;
      case 4:
        if (p.narrow)
          hipLaunchKernelGGL((k_decide_block<4096, W, REFINE, unsigned int>), dim3(grid_for(bin_upper[b], 1, 1024)),
                             dim3(kBlock), 0, t, q);
        else
          hipLaunchKernelGGL((k_decide_block<4096, W, REFINE>), dim3(grid_for(bin_upper[b], 1, 1024)), dim3(kBlock),
                             0, t, q);
        break;
      default: {
        if (sizeof(W) == 4 && !REFINE) kt_mark(LEIDEN_KT_HUB_INSERT, t);
        if (p.narrow)
          hipLaunchKernelGGL((k_hub_chunk<W, REFINE, unsigned int>),
                             dim3(grid_for(bin_upper[b] * (maxdeg / kHubChunk + 1), 1, 1536)), dim3(kBlock), 0, t, q);
        else
          hipLaunchKernelGGL((k_hub_chunk<W, REFINE>), dim3(grid_for(bin_upper[b] * (maxdeg / kHubChunk + 1), 1, 1536)),
                             dim3(kBlock), 0, t, q);
        if (sizeof(W) == 4 && !REFINE) kt_mark(LEIDEN_KT_HUB_INSERT, t);
        hipLaunchKernelGGL((k_hub_pick<W, REFINE>), dim3(grid_for(bin_upper[b], 1, 512), p.pick_segs),
                           dim3(kBlock), 0, t, q);
        break;
      }
    }
  }
  if (forked)
    for (int k = 0; k < kDecideSide; ++k)
      if (used[k]) {
        (void)hipEventRecord(ds->join[k], ds->aux[k]);
        (void)hipStreamWaitEvent(s, ds->join[k], 0);
      }
}

template void launch_decide_all<uint32_t, false>(hipStream_t, DecideParams<uint32_t>, uint32_t*, size_t,
                                                 unsigned int*, const uint64_t*, uint32_t, const DecideStreams*);
template void launch_decide_all<uint32_t, true>(hipStream_t, DecideParams<uint32_t>, uint32_t*, size_t,
                                                unsigned int*, const uint64_t*, uint32_t, const DecideStreams*);
template void launch_decide_all<int64_t, false>(hipStream_t, DecideParams<int64_t>, uint32_t*, size_t,
                                                unsigned int*, const uint64_t*, uint32_t, const DecideStreams*);
template void launch_decide_all<int64_t, true>(hipStream_t, DecideParams<int64_t>, uint32_t*, size_t, unsigned int*,
                                               const uint64_t*, uint32_t, const DecideStreams*);

void launch_apply_moves(hipStream_t s, const ApplyParams& p, uint32_t n_upper, uint64_t items_upper) {
  hipLaunchKernelGGL(k_apply_moves, dim3(grid_for(n_upper, kBlock, 1024)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_mark_items, dim3(grid_for(items_upper, kMarkU * (kBlock / kWave), 2048)), dim3(kBlock), 0, s,
                     p);
}

void launch_apply_refine(hipStream_t s, uint32_t* C, int64_t* S, const int64_t* K, uint32_t* size,
                         const Mover* movers, Ctl* ctl, uint32_t n_upper) {
  hipLaunchKernelGGL(k_apply_refine, dim3(grid_for(n_upper, kBlock, 2048)), dim3(kBlock), 0, s, C, S, K, size, movers,
                     ctl);
}

void launch_subround_reset(hipStream_t s, Ctl* ctl) {
  hipLaunchKernelGGL(k_subround_reset, dim3(1), dim3(64), 0, s, ctl);
}

void launch_iteration_reset(hipStream_t s, Ctl* ctl, uint32_t P) {
  hipLaunchKernelGGL(k_iteration_reset, dim3(1), dim3(64), 0, s, ctl, P);
}

__global__ void k_cls_reset(Ctl* ctl) {
  if (threadIdx.x < kBins) ctl->bin_count[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ctl->mover_count = 0;
    ctl->mark_items = 0;
    ctl->hub_items = 0;
  }
  if (threadIdx.x < kMaxClasses) ctl->cls_count[threadIdx.x] = 0;
}

void launch_cls_reset(hipStream_t s, Ctl* ctl) { hipLaunchKernelGGL(k_cls_reset, dim3(1), dim3(64), 0, s, ctl); }

}  // namespace lm
