// Pass-level phases of Alg. 4 on gfx950: subset renumbering (Alg. 10),
// splitting (Alg. 7), the refinement reset (Alg. 8), dense renumbering and
// dendrogram lookup, aggregation (Alg. 9), modularity (Eq. 1), static output
// labels and community tracking (Alg. 12).  All are O(n) or O(|E|) sweeps with
// integer atomics, so their results do not depend on thread timing.
#include <cstring>

#include "kernels.h"

namespace lm {

constexpr int kTileU = 4;  // elements per thread of a list-building tile

static int grid_n(uint64_t n, int per_block = kBlock, int cap = 8192) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap) b = cap;
  return (int)b;
}

#define GRID_STRIDE(i, n) \
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < (uint64_t)(n); i += (uint64_t)gridDim.x * kBlock)

// ---------------------------------------------------------------------------
// Per-level helpers
// ---------------------------------------------------------------------------
// Each block adds its counts to one of kHistParts partial rows (own cache
// line each), summed by k_hist_fold: blocks that finish together and all add
// to the same few words queue on them.
constexpr uint32_t kHistParts = kWave, kHistStride = 16;
__global__ __launch_bounds__(kBlock) void k_degree_hist(const uint32_t* len, uint32_t n, BinCfg cfg,
                                                        unsigned long long* parts) {
  __shared__ unsigned int lb[kBins];
  __shared__ unsigned int lmax;
  if (threadIdx.x < kBins) lb[threadIdx.x] = 0;
  if (threadIdx.x == 0) lmax = 0;
  __syncthreads();
  GRID_STRIDE(i, n) {
    const uint32_t d = len[i];
    if (d > 0) {
      atomicAdd(&lb[bin_of_degree(d, cfg)], 1u);
      atomicMax(&lmax, d);
    }
  }
  __syncthreads();
  unsigned long long* part = parts + (size_t)(blockIdx.x % kHistParts) * kHistStride;
  if (threadIdx.x < kBins && lb[threadIdx.x]) atomicAdd(&part[threadIdx.x], (unsigned long long)lb[threadIdx.x]);
  if (threadIdx.x == 0 && lmax) atomicMax(&part[kBins], (unsigned long long)lmax);
}

// one wavefront, lane p reads partial row p
__global__ void k_hist_fold(const unsigned long long* parts, unsigned long long* bins, unsigned int* maxdeg) {
  const unsigned long long* row = parts + (size_t)threadIdx.x * kHistStride;
  for (int q = 0; q < kBins; ++q) {
    const unsigned long long c = group_sum<kWave>(row[q]);
    if (threadIdx.x == 0) bins[q] += c;
  }
  unsigned long long m = row[kBins];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o));
  if (threadIdx.x == 0 && m > *maxdeg) *maxdeg = (unsigned int)m;
}

void launch_degree_hist(hipStream_t s, const uint32_t* len, uint32_t n, const BinCfg& cfg, unsigned long long* bins_out,
                        unsigned int* maxdeg_out, unsigned long long* parts) {
  fill_u64(s, (uint64_t*)parts, 0, (size_t)kHistParts * kHistStride);
  hipLaunchKernelGGL(k_degree_hist, dim3(grid_n(n, kBlock, 2048)), dim3(kBlock), 0, s, len, n, cfg, parts);
  hipLaunchKernelGGL(k_hist_fold, dim3(1), dim3(kWave), 0, s, parts, bins_out, maxdeg_out);
}

// Row sweeps (weighted degrees, Eq. 1's intra-community sums) take one
// wavefront per row; a row of more than kWaveRowMax entries would hold its
// wavefront for a long serial chain of gathers (a hub of 10^5..10^6 entries
// for milliseconds), so the wavefront that meets one lists its chunks of
// kRowChunk entries instead (items[0] counts them, items[1 + q] = row << 32 |
// chunk) and a second launch sums every chunk with a whole block.
__device__ inline void list_row_chunks(unsigned long long* items, uint32_t i, uint32_t L, uint32_t lane) {
  const uint32_t nc = (L + kRowChunk - 1) / kRowChunk;
  unsigned int base = 0;
  if (lane == 0) base = (unsigned int)atomicAdd(&items[0], (unsigned long long)nc);
  base = __shfl(base, 0);
  for (uint32_t k = lane; k < nc; k += kWave) items[1 + (uint64_t)base + k] = ((unsigned long long)i << 32) | k;
}

// Weighted degree of every row.
__global__ __launch_bounds__(kBlock) void k_row_sums(Rows<uint32_t> g, uint32_t n, int64_t* K,
                                                     unsigned long long* items) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t i = wave; i < n; i += nwaves) {
    const int64_t s0 = g.start[i];
    const uint32_t L = g.len[i];
    if (L > kWaveRowMax) {  // wavefront-uniform
      if (lane == 0) K[i] = 0;
      list_row_chunks(items, (uint32_t)i, L, lane);
      continue;
    }
    unsigned long long k = 0;
    for (uint32_t e = lane; e < L; e += kWave) k += g.w[s0 + e];
    k = group_sum<kWave>(k);
    if (lane == 0) K[i] = (int64_t)k;
  }
}

// the listed chunks, one block each
__global__ __launch_bounds__(kBlock) void k_row_sums_long(Rows<uint32_t> g, int64_t* K,
                                                          const unsigned long long* items) {
  __shared__ unsigned long long red[kBlock / kWave];
  const unsigned long long cnt = items[0];
  for (unsigned long long q = blockIdx.x; q < cnt; q += gridDim.x) {
    const unsigned long long it = items[1 + q];
    const uint32_t i = (uint32_t)(it >> 32), e0 = (uint32_t)it * kRowChunk;
    const uint32_t e1 = min(g.len[i], e0 + kRowChunk);
    const int64_t s0 = g.start[i];
    unsigned long long k = 0;
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBlock) k += g.w[s0 + e];
    k = block_sum(k, red);
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)&K[i], k);
  }
}

void launch_row_sums_u32(hipStream_t s, Rows<uint32_t> g, uint32_t n, int64_t* K, unsigned long long* items) {
  if (n == 0) return;
  fill_u64(s, (uint64_t*)items, 0, 1);
  hipLaunchKernelGGL(k_row_sums, dim3(grid_n(n, kBlock / kWave, 16384)), dim3(kBlock), 0, s, g, n, K, items);
  hipLaunchKernelGGL(k_row_sums_long, dim3(kLongGrid), dim3(kBlock), 0, s, g, K, items);
}

void launch_count_members(hipStream_t s, const uint32_t* C, uint32_t n, uint32_t* size) {
  fill_u32(s, size, 0, n);
  scatter_count(s, C, n, size, n);
}

void launch_sigma_from(hipStream_t s, const uint32_t* C, const int64_t* K, uint32_t n, int64_t* S) {
  fill_i64(s, S, 0, n);
  scatter_add_i64(s, C, K, n, S, n);
}

// ---------------------------------------------------------------------------
// Alg. 10: each community takes the ID of its minimum member vertex; Sigma,
// member counts and the split / refine flags move with the label.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_move_by_label(uint32_t n, const uint32_t* rep, const int64_t* S,
                                                          const uint32_t* size, const uint8_t* dS, const uint8_t* dR,
                                                          int64_t* S2, uint32_t* size2, uint8_t* dS2, uint8_t* dR2,
                                                          Ctl* ctl) {
  unsigned int nsplit = 0, nref = 0;
  uint8_t* frefined = ctl->f_refined;
  const uint32_t* fgid = ctl->f_gid;
  GRID_STRIDE(c, n) {
    const uint32_t r = rep[c];
    if (r == kNone) continue;
    S2[r] = S[c];
    size2[r] = size[c];
    dS2[r] = dS[c];
    dR2[r] = dR[c];
    nsplit += (dS[c] && !dR[c]) ? 1u : 0u;
    nref += dR[c] ? 1u : 0u;
    if (frefined && dR[c]) raise_flag(frefined, fgid[r]);
  }
  // one atomic per block: per-thread (or per-wavefront) counts on these two
  // words queued one atomic after another
  __shared__ unsigned long long red[kBlock / kWave];
  const unsigned long long ns = block_sum((unsigned long long)nsplit, red);
  const unsigned long long nr = block_sum((unsigned long long)nref, red);
  if (threadIdx.x == 0) {
    if (ns) atomicAdd(&ctl->misc[0], (unsigned int)ns);
    if (nr) atomicAdd(&ctl->misc[1], (unsigned int)nr);
  }
}

__global__ __launch_bounds__(kBlock) void k_relabel(uint32_t* C, uint32_t n, const uint32_t* rep) {
  GRID_STRIDE(i, n) C[i] = rep[C[i]];
}

__global__ void k_clear_misc(Ctl* ctl) {
  if (threadIdx.x < 8) ctl->misc[threadIdx.x] = 0;
}

void subset_renumber(hipStream_t s, uint32_t n, uint32_t* C, int64_t*& S, uint32_t*& size, uint8_t*& dS,
                     uint8_t*& dR, RenumberBufs& b, Ctl* ctl) {
  hipLaunchKernelGGL(k_clear_misc, dim3(1), dim3(64), 0, s, ctl);
  if (n == 0) return;
  fill_u32(s, b.rep, kNone, n);
  fill_i64(s, b.S2, 0, n);
  fill_u32(s, b.size2, 0, n);
  fill_u8(s, b.dS2, 0, n);
  fill_u8(s, b.dR2, 0, n);
  scatter_min_index(s, C, n, b.rep, n);
  hipLaunchKernelGGL(k_move_by_label, dim3(grid_n(n, kBlock, 1024)), dim3(kBlock), 0, s, n, b.rep, S, size, dS, dR,
                     b.S2, b.size2, b.dS2, b.dR2, ctl);
  hipLaunchKernelGGL(k_relabel, dim3(grid_n(n)), dim3(kBlock), 0, s, C, n, b.rep);
  std::swap(S, b.S2);
  std::swap(size, b.size2);
  std::swap(dS, b.dS2);
  std::swap(dR, b.dR2);
}

// ---------------------------------------------------------------------------
// Alg. 7 by its definition: connected components of the subgraph induced by
// each community marked to be split and not refined, labelled by their
// minimum vertex.
//
// Concurrent union-find in which a union always hangs the larger root under
// the smaller one (so parent[x] <= x and every root is the minimum vertex of
// its tree), in the sampled form of Sutton et al., "Optimizing Parallel Graph
// Connectivity Computation via Subgraph Sampling" (IPDPS 2018):
//   1. union each split vertex with the same-community neighbours among the
//      first kSplitSample entries of its row (a vertex of more than
//      kSplitWideMin entries: the first kSplitSample + kWave), then compress;
//   2. per community one main tree (that of its highest-degree member, or of
//      its label vertex, the minimum member after subset renumbering); a
//      vertex already in it skips its row (each of its edges is either inside
//      the main tree or seen from the other endpoint);
//   3. every other split vertex unions all its same-community neighbours;
//   4. compress: the root of each vertex is its component's minimum vertex.
// ---------------------------------------------------------------------------
constexpr uint32_t kSplitSample = 4, kSplitWideMin = 64;
using UfNode = unsigned long long;
constexpr UfNode kUfComm = 0xFFFFFFFF00000000ull;
__device__ inline UfNode uf_node(uint32_t comm, uint32_t parent) { return ((UfNode)comm << 32) | parent; }

__global__ __launch_bounds__(kBlock) void k_split_init(uint32_t n, const uint32_t* C, const uint8_t* dS,
                                                       const uint8_t* dR, UfNode* lab, uint32_t* list,
                                                       uint32_t* wide, unsigned long long* main_key, Ctl* ctl,
                                                       const uint32_t* len, unsigned long long* parts) {
  __shared__ unsigned int scnt[2], sbase[2];
  __shared__ unsigned long long red[kBlock / kWave];
  if (threadIdx.x < 2) scnt[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long entries = 0;
  constexpr uint32_t tile = kBlock * kTileU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < n; base += (uint64_t)gridDim.x * tile) {
    uint32_t key[kTileU], val[kTileU];
#pragma unroll
    for (int u = 0; u < kTileU; ++u) {
      const uint64_t i = base + u * kBlock + threadIdx.x;
      key[u] = kNone;
      val[u] = (uint32_t)i;
      if (i < n) {
        const uint32_t c = C[i];
        lab[i] = uf_node(c, (uint32_t)i);
        const bool in = dS[c] && !dR[c];
        // the label of a community is its minimum member: one writer per community
        if (in && c == (uint32_t)i) main_key[c] = 0;
        if (in) {
          key[u] = 0;
          entries += len[i];
        }
      }
    }
    tile_append<kTileU>(key, val, 1, scnt, sbase, [&](uint32_t, uint32_t*& l, unsigned int*& cn) {
      l = list;
      cn = &ctl->split_count;
    });
    // the long rows again, in their own list
#pragma unroll
    for (int u = 0; u < kTileU; ++u)
      if (key[u] != kNone && len[val[u]] <= kSplitWideMin) key[u] = kNone;
    tile_append<kTileU>(key, val, 1, scnt + 1, sbase + 1, [&](uint32_t, uint32_t*& l, unsigned int*& cn) {
      l = wide;
      cn = &ctl->split_wide;
    });
  }
  entries = block_sum(entries, red);
  if (threadIdx.x == 0) add_units(parts, kWSplit, entries);
}

// A union-find node is one 64-bit word: the parent in the low half and the
// vertex's community, which stays fixed during the split, in the high half,
// so that one load gives both (the same-community test and the first step of
// a find read one line instead of two).  A tree only ever holds vertices of
// one community, so every word written into it carries that community.
//
// Every parent is below its child, and a parent pointer only ever moves to
// another ancestor, so a read of p[x], however stale, names an ancestor of x:
// a find ends (each step goes to a smaller ID) and returns an ancestor of x,
// which was a root when written.  Reads may therefore come from the nearest
// cache.  During the union launches a stale root only makes the union's
// compare-and-swap fail, and the union goes on from the parent the atomic
// returned; after them (compress, finish: separate launches) nothing links
// roots any more and every find reaches the true root.
// root of x, whose word wx was read before (the high half is its community)
__device__ inline uint32_t uf_find(UfNode* p, uint32_t x, UfNode wx) {
  // path halving: every pointer written is an ancestor of the node
  const UfNode comm = wx & kUfComm;
  uint32_t px = (uint32_t)wx;
  while (px != x) {
    const uint32_t gp = (uint32_t)ld_near(&p[px]);
    if (gp != px) st_near(&p[x], comm | gp);
    x = gp;
    px = (uint32_t)ld_near(&p[x]);
  }
  return x;
}

// a and b of one community, with their words wa and wb as read
__device__ inline void uf_union(UfNode* p, uint32_t a, UfNode wa, uint32_t b, UfNode wb) {
  const UfNode comm = wa & kUfComm;
  while (true) {
    a = uf_find(p, a, wa);
    b = uf_find(p, b, wb);
    if (a == b) return;
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    // hang root b under the smaller root a; if b stopped being a root, go on
    // from the parent the compare-and-swap found (a smaller ID), so that
    // every retry lowers max(a, b) whatever the loads above returned
    const UfNode o = atomicCAS(&p[b], comm | b, comm | a);
    if (o == (comm | b)) return;
    b = (uint32_t)o;
    wa = ld_near(&p[a]);
    wb = ld_near(&p[b]);
  }
}

// the union of u with its neighbour j when both are in one community
__device__ inline void uf_link(UfNode* lab, uint32_t u, uint32_t j) {
  if (j == u) return;
  const UfNode wj = ld_near(&lab[j]), wu = ld_near(&lab[u]);
  if ((wj ^ wu) & kUfComm) return;
  uf_union(lab, u, wu, j, wj);
}

template <typename W>
__global__ __launch_bounds__(kBlock) void k_split_sample(Rows<W> g, UfNode* lab, const uint32_t* list,
                                                         const Ctl* ctl) {
  // one thread per (vertex, sampled entry): the unions of a vertex run side
  // by side instead of one after another
  const uint64_t cnt = (uint64_t)ctl->split_count * kSplitSample;
  GRID_STRIDE(q, cnt) {
    const uint32_t u = list[q / kSplitSample];
    const uint32_t e = (uint32_t)(q % kSplitSample);
    if (e >= g.len[u]) continue;
    uf_link(lab, u, g.cols[g.start[u] + e]);
  }
}

// Long rows sample kSplitWide more entries: a high-degree vertex left
// outside its community's main tree would union its whole row.  One thread
// per (long-row vertex, extra entry), like the first sample.
constexpr uint32_t kSplitWide = 64;
template <typename W>
__global__ __launch_bounds__(kBlock) void k_split_sample_wide(Rows<W> g, UfNode* lab, const uint32_t* wide,
                                                              const Ctl* ctl) {
  const uint64_t cnt = (uint64_t)ctl->split_wide * kSplitWide;
  GRID_STRIDE(q, cnt) {
    const uint32_t u = wide[q / kSplitWide];
    const uint32_t e = kSplitSample + (uint32_t)(q % kSplitWide);
    if (e >= g.len[u]) continue;
    uf_link(lab, u, g.cols[g.start[u] + e]);
  }
}

__global__ __launch_bounds__(kBlock) void k_split_compress(UfNode* lab, const uint32_t* list, const Ctl* ctl) {
  const uint32_t cnt = ctl->split_count;
  GRID_STRIDE(it, cnt) {
    const uint32_t i = list[it];
    const UfNode w = ld_near(&lab[i]);
    lab[i] = (w & kUfComm) | uf_find(lab, i, w);
  }
}

// main tree of a community: that of its highest-degree member among those
// with more than kSplitMainDeg entries (lowest ID on ties), else that of its
// label vertex.  Launched once per degree band, highest band first: a large
// community's maximum is then set by its few hubs, and its many members of
// lower degree find it already above their key with a plain read instead of
// all racing to one address with atomics.
constexpr uint32_t kSplitMainDeg = 128;
constexpr uint32_t kSplitMainBands[] = {32768, 4096, 1024, kSplitMainDeg};
__global__ __launch_bounds__(kBlock) void k_split_main(const uint32_t* len, const uint32_t* C, const uint32_t* list,
                                                       unsigned long long* main_key, const Ctl* ctl, uint32_t lo,
                                                       uint32_t hi) {
  const uint32_t cnt = ctl->split_count;
  GRID_STRIDE(it, cnt) {
    const uint32_t u = list[it];
    const uint32_t L = len[u];
    if (L <= lo || L > hi) continue;
    const unsigned long long key = ((unsigned long long)L << 32) | (unsigned long long)(0xFFFFFFFFu - u);
    unsigned long long* slot = &main_key[C[u]];
    if (peek(slot) < key) atomicMax(slot, key);
  }
}

__global__ __launch_bounds__(kBlock) void k_split_rest(uint32_t n, const uint32_t* C, const UfNode* lab,
                                                       const uint32_t* list, const unsigned long long* main_key,
                                                       uint32_t* rest, Ctl* ctl) {
  __shared__ unsigned int scnt[1], sbase[1];
  if (threadIdx.x == 0) scnt[0] = 0;
  __syncthreads();
  const uint32_t cnt = ctl->split_count;
  constexpr uint32_t tile = kBlock * kTileU;
  for (uint32_t base = blockIdx.x * tile; base < cnt; base += gridDim.x * tile) {
    uint32_t kk[kTileU], val[kTileU];
#pragma unroll
    for (int q = 0; q < kTileU; ++q) {
      const uint32_t it = base + q * kBlock + threadIdx.x;
      kk[q] = kNone;
      val[q] = 0;
      if (it < cnt) {
        const uint32_t u = list[it];
        const uint32_t c = C[u];
        const unsigned long long key = main_key[c];
        uint32_t m = key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : c;
        if (m >= n || C[m] != c) m = c;  // any choice is correct; this one is always in range
        if (lab[u] != lab[m]) kk[q] = 0;  // both are roots after compression (same community half)
        val[q] = u;
      }
    }
    tile_append<kTileU>(kk, val, 1, scnt, sbase, [&](uint32_t, uint32_t*& l, unsigned int*& cn) {
      l = rest;
      cn = &ctl->split_rest;
    });
  }
}

// G lanes per vertex (G <= 64 inside a wavefront, G = kBlock for a block)
template <int G, typename W>
__global__ __launch_bounds__(kBlock) void k_split_union(Rows<W> g, const uint32_t* C, UfNode* lab,
                                                        const uint32_t* list, const unsigned int* count) {
  const uint32_t grp = threadIdx.x / G, lane = threadIdx.x % G;
  constexpr uint32_t GPB = kBlock / G;
  const uint32_t cnt = *count;
  for (uint32_t base = blockIdx.x * GPB; base < cnt; base += gridDim.x * GPB) {
    const uint32_t it = base + grp;
    if (it >= cnt) continue;
    const uint32_t u = list[it];
    const UfNode comm = (UfNode)C[u] << 32;
    const int64_t s0 = g.start[u];
    const uint32_t L = g.len[u];
    for (uint32_t e = lane; e < L; e += G) {
      const uint32_t j = g.cols[s0 + e];
      if (j == u) continue;
      const UfNode wj = ld_near(&lab[j]);
      if ((wj & kUfComm) == comm) uf_union(lab, u, ld_near(&lab[u]), j, wj);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_split_finish(uint32_t* C, UfNode* lab, const uint32_t* list, Ctl* ctl) {
  const uint32_t cnt = ctl->split_count;
  GRID_STRIDE(it, cnt) {
    const uint32_t i = list[it];
    C[i] = uf_find(lab, i, ld_near(&lab[i]));
  }
}

__global__ void k_split_reset(Ctl* ctl) {
  if (threadIdx.x == 0) {
    ctl->split_count = 0;
    ctl->split_rest = 0;
    ctl->split_wide = 0;
  }
}

void launch_split_init(hipStream_t s, uint32_t n, const uint32_t* C, const uint8_t* dS, const uint8_t* dR,
                       UfNode* lab, uint32_t* list, uint32_t* wide, unsigned long long* main_key, Ctl* ctl,
                       const uint32_t* len, unsigned long long* parts) {
  hipLaunchKernelGGL(k_split_reset, dim3(1), dim3(1), 0, s, ctl);
  if (n)
    hipLaunchKernelGGL(k_split_init, dim3(grid_n(n, kBlock * kTileU)), dim3(kBlock), 0, s, n, C, dS, dR, lab, list,
                       wide, main_key, ctl, len, parts);
}

template <typename W>
void launch_split_sample(hipStream_t s, Rows<W> g, const uint32_t* C, UfNode* lab, const uint32_t* list,
                         const uint32_t* wide, unsigned long long* main_key, uint32_t* rest, Ctl* ctl,
                         uint32_t n_upper) {
  hipLaunchKernelGGL((k_split_sample<W>), dim3(grid_n((uint64_t)n_upper * kSplitSample)), dim3(kBlock), 0, s, g, lab,
                     list, ctl);
  hipLaunchKernelGGL((k_split_sample_wide<W>), dim3(grid_n((uint64_t)n_upper * kSplitWide, kBlock, 4096)),
                     dim3(kBlock), 0, s, g, lab, wide, ctl);
  hipLaunchKernelGGL(k_split_compress, dim3(grid_n(n_upper)), dim3(kBlock), 0, s, lab, list, ctl);
  uint32_t hi = 0xFFFFFFFFu;
  for (const uint32_t lo : kSplitMainBands) {
    hipLaunchKernelGGL(k_split_main, dim3(grid_n(n_upper)), dim3(kBlock), 0, s, g.len, C, list, main_key, ctl, lo, hi);
    hi = lo;
  }
  hipLaunchKernelGGL(k_split_rest, dim3(grid_n(n_upper, kBlock * kTileU)), dim3(kBlock), 0, s, n_upper, C, lab, list,
                     main_key, rest, ctl);
}

// Full rows of the vertices outside their community's main tree, by degree
// bin (bins as in the local-moving kernels).
template <typename W>
void launch_split_union(hipStream_t s, Rows<W> g, const uint32_t* C, UfNode* lab, const uint32_t* bin_lists,
                        size_t stride, const unsigned int* bin_counts, const uint64_t* bin_upper) {
  for (int b = 0; b < kBins; ++b) {
    if (!bin_upper[b]) continue;
    const uint32_t* bl = bin_lists + (size_t)b * stride;
    const unsigned int* bc = bin_counts + b;
    if (b == 0)
      hipLaunchKernelGGL((k_split_union<8, W>), dim3(grid_n(bin_upper[b], kBlock / 8, 4096)), dim3(kBlock), 0, s,
                         g, C, lab, bl, bc);
    else if (b == 1)
      hipLaunchKernelGGL((k_split_union<32, W>), dim3(grid_n(bin_upper[b], kBlock / 32, 4096)), dim3(kBlock), 0, s,
                         g, C, lab, bl, bc);
    else if (b == 2)
      hipLaunchKernelGGL((k_split_union<64, W>), dim3(grid_n(bin_upper[b], kBlock / 64, 4096)), dim3(kBlock), 0, s,
                         g, C, lab, bl, bc);
    else
      hipLaunchKernelGGL((k_split_union<kBlock, W>), dim3(grid_n(bin_upper[b], 1, 4096)), dim3(kBlock), 0, s, g, C,
                         lab, bl, bc);
  }
}

void launch_split_finish(hipStream_t s, uint32_t* C, UfNode* lab, const uint32_t* list, Ctl* ctl, uint32_t n_upper) {
  hipLaunchKernelGGL(k_split_finish, dim3(grid_n(n_upper)), dim3(kBlock), 0, s, C, lab, list, ctl);
}

template void launch_split_sample<uint32_t>(hipStream_t, Rows<uint32_t>, const uint32_t*, UfNode*,
                                            const uint32_t*, const uint32_t*, unsigned long long*, uint32_t*, Ctl*,
                                            uint32_t);
template void launch_split_sample<int64_t>(hipStream_t, Rows<int64_t>, const uint32_t*, UfNode*, const uint32_t*,
                                           const uint32_t*, unsigned long long*, uint32_t*, Ctl*, uint32_t);
template void launch_split_union<uint32_t>(hipStream_t, Rows<uint32_t>, const uint32_t*, UfNode*, const uint32_t*,
                                           size_t, const unsigned int*, const uint64_t*);
template void launch_split_union<int64_t>(hipStream_t, Rows<int64_t>, const uint32_t*, UfNode*, const uint32_t*,
                                          size_t, const unsigned int*, const uint64_t*);

// ---------------------------------------------------------------------------
// Alg. 8, first loop: vertices of refined bounds become singletons; they are
// listed by refinement colour.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_refine_reset(uint32_t n, uint32_t* C, uint32_t* CB, int64_t* S,
                                                         const int64_t* K, uint32_t* size, const uint8_t* dR,
                                                         uint32_t R, uint32_t* col_lists, size_t stride, Ctl* ctl) {
  __shared__ unsigned int scnt[kMaxClasses], sbase[kMaxClasses];
  if (threadIdx.x < kMaxClasses) scnt[threadIdx.x] = 0;
  __syncthreads();
  bool any = false;
  const ForestView F = forest_view(ctl);
  constexpr uint32_t tile = kBlock * kTileU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < n; base += (uint64_t)gridDim.x * tile) {
    uint32_t key[kTileU], val[kTileU];
#pragma unroll
    for (int u = 0; u < kTileU; ++u) {
      const uint64_t i = base + u * kBlock + threadIdx.x;
      key[u] = kNone;
      val[u] = (uint32_t)i;
      if (i < n) {
        const uint32_t b = C[i];
        CB[i] = b;
        // a graph of a forest that left the pass loop keeps its communities
        if (dR[b] && F.live((uint32_t)i)) {
          C[i] = (uint32_t)i;
          S[i] = K[i];
          size[i] = 1;
          any = true;
          key[u] = vertex_colour(F.local((uint32_t)i), R);
        }
      }
    }
    tile_append<kTileU>(key, val, R, scnt, sbase, [&](uint32_t col, uint32_t*& l, unsigned int*& c) {
      l = col_lists + (size_t)col * stride;
      c = &ctl->cls_count[col];
    });
  }
  if (any) ctl->refined_any = 1;
}

void launch_refine_reset(hipStream_t s, uint32_t n, uint32_t* C, uint32_t* CB, int64_t* S, const int64_t* K,
                         uint32_t* size, const uint8_t* dR, uint32_t R, uint32_t* col_lists, size_t stride,
                         Ctl* ctl) {
  if (n)
    hipLaunchKernelGGL(k_refine_reset, dim3(grid_n(n, kBlock * kTileU)), dim3(kBlock), 0, s, n, C, CB, S, K, size, dR,
                       R, col_lists, stride, ctl);
}

// ---------------------------------------------------------------------------
// Dense renumbering in ascending label order, and dendrogram lookup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_flag_labels(const uint32_t* C, uint32_t n, uint32_t* flag) {
  GRID_STRIDE(i, n) raise_flag(flag, C[i]);
}

__global__ __launch_bounds__(kBlock) void k_apply_newid(uint32_t* C, uint32_t n, const uint64_t* newid) {
  GRID_STRIDE(i, n) C[i] = (uint32_t)newid[C[i]];
}

void dense_renumber(hipStream_t s, uint32_t n, uint32_t* C, uint32_t* flag, uint64_t* newid, uint64_t* total,
                    void* scan_tmp) {
  fill_u32(s, flag, 0, n);
  if (n) hipLaunchKernelGGL(k_flag_labels, dim3(grid_n(n)), dim3(kBlock), 0, s, C, n, flag);
  exclusive_scan_u32(s, flag, newid, n, total, scan_tmp);
  if (n) hipLaunchKernelGGL(k_apply_newid, dim3(grid_n(n)), dim3(kBlock), 0, s, C, n, newid);
}

__global__ __launch_bounds__(kBlock) void k_lookup(uint32_t* Ctop, const uint32_t* C, uint32_t n) {
  GRID_STRIDE(i, n) Ctop[i] = C[Ctop[i]];
}

void launch_lookup(hipStream_t s, uint32_t* Ctop, const uint32_t* C, uint32_t n) {
  if (n) hipLaunchKernelGGL(k_lookup, dim3(grid_n(n)), dim3(kBlock), 0, s, Ctop, C, n);
}

// ---------------------------------------------------------------------------
// Alg. 9: super-vertex graph.  w''(c, d) = sum of w_ij over entries with
// C[i] = c, C[j] = d (self-loops included).  Communities are grouped into a
// member CSR by counting sort; each community accumulates its neighbour
// communities in a hash table (LDS for total degree up to 2048, a global
// table above) and writes the distinct (d, w) pairs to its super row, whose
// capacity is min(total degree, number of communities).
// ---------------------------------------------------------------------------
// Counting-sort scatter of vertices into the member CSR.  Per tile, the
// vertices of one community reserve their range with a single atomic (ranks
// inside the tile come from the LDS counter), so large communities do not
// serialise on one global counter.
// Members of each community, short rows from the front of its range and rows
// of at least long_min entries from the back (fill_long counts them).
__global__ __launch_bounds__(kBlock) void k_comm_scatter(const uint32_t* C, uint32_t n, const uint64_t* off,
                                                         uint32_t* fill, uint32_t* members, const uint32_t* len,
                                                         uint32_t long_min, uint32_t* fill_long) {
  constexpr int kTile = 1024, kSlots = 2048, kPer = kTile / kBlock;
  constexpr unsigned long long kEmpty = ~0ull;
  __shared__ unsigned long long hk[kSlots];
  __shared__ uint32_t hc[kSlots];
  __shared__ uint32_t hb[kSlots];
  for (uint64_t base = (uint64_t)blockIdx.x * kTile; base < n; base += (uint64_t)gridDim.x * kTile) {
    for (int s = threadIdx.x; s < kSlots; s += kBlock) {
      hk[s] = kEmpty;
      hc[s] = 0;
    }
    __syncthreads();
    uint32_t slot[kPer], rank[kPer];
    unsigned long long key[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint64_t i = base + t * kBlock + threadIdx.x;
      if (i >= n) continue;
      const uint32_t c = C[i];
      const unsigned long long k = (unsigned long long)c | ((unsigned long long)(len[i] >= long_min) << 32);
      uint32_t h = slot_hash(c, kSlots - 1);
      while (true) {
        const unsigned long long o = atomicCAS(&hk[h], kEmpty, k);
        if (o == kEmpty || o == k) break;
        h = (h + 1) & (kSlots - 1);
      }
      key[t] = k;
      slot[t] = h;
      rank[t] = atomicAdd(&hc[h], 1u);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kSlots; s += kBlock) {
      const unsigned long long k = hk[s];
      if (k == kEmpty) continue;
      const uint32_t c = (uint32_t)k;
      hb[s] = (k >> 32) ? (uint32_t)(off[c + 1] - off[c]) - atomicAdd(&fill_long[c], hc[s]) - hc[s]
                        : atomicAdd(&fill[c], hc[s]);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint64_t i = base + t * kBlock + threadIdx.x;
      if (i < n) members[off[(uint32_t)key[t]] + hb[slot[t]] + rank[t]] = (uint32_t)i;
    }
    __syncthreads();
  }
}

// Row capacities and classification by entries: 0 = small (LDS, 64 lanes,
// 256 slots), 3 = medium (LDS, block, 1024 slots), 1 = large medium (LDS,
// block, 4096 slots), 2 = big (staging).  One block per community decides
// one community at a time, so the 1024-slot class (12 KB of LDS: eight
// blocks per CU instead of three) keeps more communities in flight.
constexpr uint64_t kAggSmall = 128, kAggMid = 512, kAggMedium = 2048;

__global__ __launch_bounds__(kBlock) void k_comm_classify(uint32_t nc, const uint64_t* deg, uint64_t* cap,
                                                          uint32_t* out_len, int64_t* Kout, uint32_t* lists,
                                                          size_t stride, Ctl* ctl) {
  __shared__ unsigned int scnt[4], sbase[4];
  if (threadIdx.x < 4) scnt[threadIdx.x] = 0;
  __syncthreads();
  constexpr uint32_t tile = kBlock * kTileU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < nc; base += (uint64_t)gridDim.x * tile) {
    uint32_t key[kTileU], val[kTileU];
#pragma unroll
    for (int u = 0; u < kTileU; ++u) {
      const uint64_t c = base + u * kBlock + threadIdx.x;
      key[u] = kNone;
      val[u] = (uint32_t)c;
      if (c < nc) {
        const uint64_t d = deg[c];
        cap[c] = d < nc ? d : nc;
        out_len[c] = 0;
        Kout[c] = 0;
        if (d > 0) key[u] = d <= kAggSmall ? 0u : (d <= kAggMid ? 3u : (d <= kAggMedium ? 1u : 2u));
      }
    }
    tile_append<kTileU>(key, val, 4, scnt, sbase, [&](uint32_t b, uint32_t*& l, unsigned int*& cn) {
      l = lists + (size_t)b * stride;
      cn = &ctl->misc[2 + b];
    });
  }
}

// Member ranges, row capacities and entry counts of the big communities (for
// host planning).
__global__ __launch_bounds__(kBlock) void k_big_info(const uint32_t* big, const unsigned int* nbig,
                                                     const uint64_t* moff, const uint64_t* cap, const uint64_t* deg,
                                                     const uint32_t* nlong, uint64_t* info) {
  const uint32_t cnt = *nbig;
  GRID_STRIDE(k, cnt) {
    const uint32_t c = big[k];
    info[4 * k] = moff[c];
    info[4 * k + 1] = moff[c + 1];
    info[4 * k + 2] = cap[c] | ((uint64_t)nlong[c] << 32);  // cap <= community count < 2^32
    info[4 * k + 3] = deg[c];
  }
}

__global__ __launch_bounds__(kBlock) void k_member_len(const uint32_t* members, uint32_t n, const uint32_t* len,
                                                       uint32_t* mlen) {
  GRID_STRIDE(m, n) mlen[m] = len[members[m]];
}

// Accumulate all entries of the members of community c into table (tk, tv).
// G lanes cooperate; members are taken G at a time and their entries are
// flattened so every lane has work whatever the member degrees.
template <int G, typename W, typename KP, typename VP>
__device__ inline void agg_accumulate(Rows<W> g, const uint32_t* C, const uint32_t* members, uint64_t m0, uint64_t m1,
                                      KP tk, VP tv, uint32_t mask, int lane, int64_t* sstart, uint32_t* spre) {
  for (uint64_t mb = m0; mb < m1; mb += G) {
    const uint64_t mi = mb + lane;
    uint32_t L = 0;
    int64_t st = 0;
    if (mi < m1) {
      const uint32_t v = members[mi];
      L = g.len[v];
      st = g.start[v];
    }
    if (G <= kWave) {
      // inclusive prefix of member lengths, kept in registers; every lane runs
      // the same number of steps so the shuffles stay converged
      uint32_t incl = L;
#pragma unroll
      for (int o = 1; o < G; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, G);
        if (lane >= o) incl += y;
      }
      const uint32_t total = __shfl(incl, G - 1, G);
      for (uint32_t xb = 0; xb < total; xb += G) {
        const uint32_t x = xb + lane;
        // p = number of members whose inclusive prefix is <= x (binary lifting)
        int p = 0;
#pragma unroll
        for (int step = G / 2; step > 0; step >>= 1) {
          const uint32_t v = __shfl(incl, p + step - 1, G);
          if (v <= x) p += step;
        }
        const uint32_t before = __shfl(incl, p > 0 ? p - 1 : 0, G);
        const long long sp = __shfl((long long)st, p, G);
        if (x < total) {
          const int64_t e = sp + (x - (p > 0 ? before : 0u));
          table_add(tk, tv, mask, C[g.cols[e]], (unsigned long long)g.w[e], kRowSalt);
        }
      }
    } else {
      sstart[lane] = st;
      spre[lane] = L;
      __syncthreads();
      if (lane == 0)
        for (int q = 1; q < G; ++q) spre[q] += spre[q - 1];
      __syncthreads();
      const uint32_t total = spre[G - 1];
      for (uint32_t x = lane; x < total; x += G) {
        // member p with spre[p-1] <= x < spre[p]
        int lo = 0, hi = G - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (spre[mid] > x)
            hi = mid;
          else
            lo = mid + 1;
        }
        const uint32_t before = lo > 0 ? spre[lo - 1] : 0;
        const int64_t e = sstart[lo] + (x - before);
        table_add(tk, tv, mask, C[g.cols[e]], (unsigned long long)g.w[e], kRowSalt);
      }
      __syncthreads();
    }
  }
}

// The table of a community takes min(T, 2 deg) slots (a power of two; at
// most deg distinct keys), so a community of a few hundred entries does not
// clear and scan all T.
template <int G, int T, typename W>
__global__ __launch_bounds__(kBlock) void k_agg_lds(Rows<W> g, const uint32_t* C, const uint32_t* members,
                                                    const uint64_t* moff, const uint32_t* list, const unsigned int* count,
                                                    const uint64_t* deg, const uint64_t* cap_off, uint32_t* out_len,
                                                    uint32_t* out_cols, int64_t* out_w, int64_t* Kout) {
  constexpr int GPB = kBlock / G;
  __shared__ uint32_t keys[GPB * T];
  __shared__ unsigned long long vals[GPB * T];
  __shared__ int64_t sstart[kBlock];
  __shared__ uint32_t spre[kBlock];
  __shared__ unsigned int wpos[GPB];
  __shared__ unsigned long long red[kBlock / kWave];
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* tk = keys + grp * T;
  unsigned long long* tv = vals + grp * T;
  const uint32_t cnt = *count;
  for (uint32_t base = blockIdx.x * GPB; base < cnt; base += gridDim.x * GPB) {
    const uint32_t item = base + grp;
    const bool valid = item < cnt;
    const uint32_t c = valid ? list[item] : 0;
    const uint32_t tn = valid ? min((uint32_t)T, pow2_at_least((uint32_t)min<uint64_t>(2 * deg[c], T))) : 1u;
    for (uint32_t s = lane; s < tn; s += G) {
      tk[s] = kNone;
      tv[s] = 0;
    }
    if (lane == 0) wpos[grp] = 0;
    __syncthreads();
    const uint64_t m0 = valid ? moff[c] : 0, m1 = valid ? moff[c + 1] : 0;
    agg_accumulate<G, W>(g, C, members, m0, m1, tk, tv, tn - 1, lane, sstart + grp * G, spre + grp * G);
    __syncthreads();
    unsigned long long ksum = 0;
    if (valid) {
      const uint64_t o = cap_off[c];
      for (uint32_t sl = lane; sl < tn; sl += G) {
        const uint32_t d = tk[sl];
        if (d == kNone) continue;
        const unsigned long long w = tv[sl];
        const unsigned int p = atomicAdd(&wpos[grp], 1u);
        out_cols[o + p] = d;
        out_w[o + p] = (int64_t)w;
        ksum += w;
      }
    }
    if (G <= kWave)
      ksum = group_sum<G>(ksum);
    else
      ksum = block_sum(ksum, red);
    __syncthreads();
    if (valid && lane == 0) {
      out_len[c] = wpos[grp];
      Kout[c] = (int64_t)ksum;
    }
    __syncthreads();
  }
}

// Big communities: a group-by of each community's entries with no global
// hash table (global atomics are slow, those on one address slowest).  Work
// items are parts of one community's entries; an item's entries are summed
// into stages of at most kBigStage entries.  Each stage is summed by key in an
// LDS table (the community's own key is summed in registers: most entries of
// a large community stay inside it), and its distinct keys are sorted by
// bucket (top bits of the salted mixing) into a stage column: the next nd
// slots of the community's staging area (nd distinct keys), with the bucket
// starts (and nd in row R) in column col of the community's (R + 1) x smax
// matrix.  The staging area thus needs one slot per entry at most.  The emit kernel then sums each group of
// buckets over all columns in an LDS table and writes the distinct keys into
// the super row.  At most 256 buckets (2^kBigMaxRbits): each stage column is
// R + 1 scattered 16-bit stores, and the counters' LDS then leaves room for
// three blocks per CU.
//
// XCD slices.  Workgroups are handed to the eight XCDs in turn (block b runs
// on XCD b mod 8), and each XCD has its own L2.  On a level whose rows are
// sorted by column (the input graph), the vertex IDs are cut into eight
// slices, and the long rows (kSliceMinLen entries or more, placed at the
// back of each community's member range) of a community of at least
// kSliceMinDeg entries are taken in runs of kSliceMembers members, one item
// per slice: it takes the part of each row whose columns lie in its slice,
// found by binary search.  The items of slice x are queued in list x, which
// the blocks of XCD x take in turn, so the C[j] gathers of the long rows hit
// the 1/8 of C that stays in that XCD's L2 instead of missing to memory.
// Items of whole rows are dealt over the lists in turn.  (Blocks taking items
// from shared counters instead were slower: the counters' atomics queue on
// one memory channel.)
constexpr uint32_t kBigStage = 2048, kBigSlots = 4096;
constexpr uint32_t kBigBucketBits = 10, kBigMaxRbits = 8, kEmitWin = 2048, kEmitSlices = 256;
constexpr uint32_t kSlices = 8, kSliceMembers = 128, kSliceMinLen = 128;
// Items of whole rows are ranges of kRangeEntries entries of the community's
// whole-row members in member order (found through the members' entry
// offsets), so that every item has the same work however long the rows are.
constexpr uint32_t kRange = 0xFFFFFFFEu;
constexpr uint64_t kRangeEntries = 8192;
constexpr uint64_t kSliceMinDeg = 1u << 16;
// a community's stage counter: columns used << kColShift | staging slots used
constexpr uint32_t kColShift = 40;

struct BigComm {
  uint32_t c;      // community
  uint32_t rbits;  // log2 of its bucket count
  uint32_t smax;   // stage columns reserved
  uint32_t pad;    // whole-row members (the first ones of its member range)
  uint64_t soff;   // first staging slot (one per entry of the community)
  uint64_t moff;   // first matrix entry ((R + 1) * smax entries)
};
struct AggItem {
  uint32_t big;
  uint32_t pad;   // stage items: the slice, or kRange; emit items: the slice of the community's groups
  uint64_t a, b;  // member range, or for kRange the entry range relative to the community's first entry
};

__device__ inline uint32_t big_mix(uint32_t c) { return fmix32(c ^ kRowSalt); }

// first position of a sorted row holding a column >= key
__device__ inline uint32_t row_lower_bound(const uint32_t* a, uint32_t L, uint32_t key) {
  uint32_t lo = 0, hi = L;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// sl: the kSlices + 1 list offsets into items; gridDim.x a multiple of kSlices
template <typename W>
__global__ __launch_bounds__(kBlock) void k_agg_stage(Rows<W> g, const uint32_t* C, const uint32_t* members,
                                                      const uint64_t* moff, const uint64_t* eoff,
                                                      const BigComm* bc, const AggItem* items, unsigned int* sl,
                                                      uint32_t slice_w, uint32_t* skeys, unsigned long long* svals,
                                                      uint16_t* smat, unsigned long long* stage_ctr,
                                                      unsigned long long* self_acc, unsigned long long* units) {
  constexpr uint32_t kNB = 1u << kBigMaxRbits;
  __shared__ int64_t sstart[kBlock];
  __shared__ uint32_t spre[kBlock];
  __shared__ uint32_t lk[kBigSlots];
  __shared__ unsigned long long lv[kBigSlots];
  __shared__ unsigned int lcnt[kNB + 1];
  __shared__ unsigned int wsum[kBlock / kWave];
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ unsigned int scol;
  __shared__ unsigned long long sbase;
  for (uint32_t q = threadIdx.x; q < kBigSlots; q += kBlock) {
    lk[q] = kNone;
    lv[q] = 0;
  }
  for (uint32_t q = threadIdx.x; q <= kNB; q += kBlock) lcnt[q] = 0;
  __syncthreads();
  unsigned long long entries = 0;
  auto run_item = [&](const AggItem x) {
    const BigComm b = bc[x.big];
    const uint32_t rb = b.rbits, R = 1u << rb;
    const uint32_t sx = x.pad;
    unsigned long long self = 0;
    // the stage's distinct keys per bucket, their starts, and a column
    auto flush = [&]() {
      for (uint32_t q = threadIdx.x; q < kBigSlots; q += kBlock) {
        const uint32_t c = lk[q];
        if (c != kNone) atomicAdd(&lcnt[rb ? big_mix(c) >> (32 - rb) : 0u], 1u);
      }
      __syncthreads();
      const uint32_t nd = block_exclusive_scan<kNB / kBlock>(lcnt, R, wsum);
      if (threadIdx.x == 0) {
        lcnt[R] = nd;
        // the next column and its nd slots, taken together: the columns'
        // slots follow one another in column order
        const unsigned long long o = atomicAdd(&stage_ctr[x.big], (1ull << kColShift) + nd);
        scol = (unsigned int)(o >> kColShift);
        sbase = o & ((1ull << kColShift) - 1);
      }
      __syncthreads();
      const uint32_t col = scol;
      for (uint32_t q = threadIdx.x; q <= R; q += kBlock) smat[b.moff + (size_t)q * b.smax + col] = (uint16_t)lcnt[q];
      __syncthreads();
      uint32_t* tk = skeys + b.soff + sbase;
      unsigned long long* tv = svals + b.soff + sbase;
      for (uint32_t q = threadIdx.x; q < kBigSlots; q += kBlock) {
        const uint32_t c = lk[q];
        if (c == kNone) continue;
        const unsigned int pos = atomicAdd(&lcnt[rb ? big_mix(c) >> (32 - rb) : 0u], 1u);
        tk[pos] = c;
        tv[pos] = lv[q];
        lk[q] = kNone;
        lv[q] = 0;
      }
      __syncthreads();
      for (uint32_t q = threadIdx.x; q <= R; q += kBlock) lcnt[q] = 0;
      __syncthreads();
    };
    uint32_t fill = 0;  // entries summed into the table since the last stage column
    // members [mfirst, mend); a range item takes the entries [lo, hi) of the
    // community's whole-row members in member order (eoff: entry offsets)
    uint64_t mfirst = x.a, mend = x.b, lo = 0, hi = 0;
    if (sx == kRange) {
      const uint64_t m0 = moff[b.c];
      mend = m0 + b.pad;
      const uint64_t e0 = eoff[m0];
      lo = e0 + x.a;
      hi = min(e0 + x.b, eoff[mend]);
      if (lo >= hi) return;  // block-uniform: past the members' entries
      // the member holding entry lo: the last m with eoff[m] <= lo
      uint64_t a = m0, z = mend - 1;
      while (a < z) {
        const uint64_t mid = (a + z + 1) >> 1;
        if (eoff[mid] <= lo)
          a = mid;
        else
          z = mid - 1;
      }
      mfirst = a;
    }
    for (uint64_t mb = mfirst; mb < mend; mb += kBlock) {
      const uint64_t mi = mb + threadIdx.x;
      uint32_t L = 0;
      int64_t st = 0;
      if (mi < mend) {
        const uint32_t v = members[mi];
        L = g.len[v];
        st = g.start[v];
        if (sx == kRange) {
          const uint64_t em = eoff[mi], a = max(em, lo), z = min(em + L, hi);
          st += (int64_t)(a - em);
          L = z > a ? (uint32_t)(z - a) : 0u;
        } else {  // the part of a long row in slice sx
          const uint32_t* row = g.cols + st;
          const uint32_t e0 = sx == 0 ? 0u : row_lower_bound(row, L, sx * slice_w);
          const uint32_t e1 = sx == kSlices - 1 ? L : row_lower_bound(row, L, (sx + 1) * slice_w);
          st += e0;
          L = e1 - e0;
        }
      }
      sstart[threadIdx.x] = st;
      // inclusive block scan of the row lengths (wavefront scans, then wavefront totals)
      uint32_t inc = L;
      const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if ((int)lane >= o) inc += y;
      }
      if (lane == kWave - 1) spre[wv] = inc;
      __syncthreads();
      uint32_t add = 0;
      for (uint32_t q = 0; q < wv; ++q) add += spre[q];
      __syncthreads();
      spre[threadIdx.x] = inc + add;
      __syncthreads();
      const uint32_t total = spre[kBlock - 1];
      entries += total;
      for (uint32_t xb = 0; xb < total;) {
        const uint32_t xe = xb + min(total - xb, kBigStage - fill);
        table_accumulate(lk, lv, kBigSlots - 1, xb + threadIdx.x, xe, kBlock,
                         [&](uint32_t xx, uint32_t& key, unsigned long long& w) {
                           int lo = 0, hi = kBlock - 1;
                           while (lo < hi) {
                             const int mid = (lo + hi) >> 1;
                             if (spre[mid] > xx)
                               hi = mid;
                             else
                               lo = mid + 1;
                           }
                           const uint32_t before = lo > 0 ? spre[lo - 1] : 0;
                           const int64_t e = sstart[lo] + (xx - before);
                           const uint32_t c = C[g.cols[e]];
                           w = (unsigned long long)g.w[e];
                           if (c == b.c)
                             self += w;
                           else
                             key = c;
                         });
        __syncthreads();
        fill += xe - xb;
        xb = xe;
        if (fill == kBigStage) {
          flush();
          fill = 0;
        }
      }
      if (sx == kRange && eoff[min(mb + kBlock, mend)] >= hi) break;  // block-uniform
    }
    if (fill) flush();
    self = block_sum(self, red);
    if (threadIdx.x == 0 && self) atomicAdd(&self_acc[x.big], self);
  };
  // the blocks of XCD x (a multiple of kSlices blocks) share list x
  const uint32_t li = blockIdx.x % kSlices, lo = sl[li], cnt = sl[li + 1] - lo;
  for (uint32_t k = blockIdx.x / kSlices; k < cnt; k += gridDim.x / kSlices) run_item(items[lo + k]);
  if (threadIdx.x == 0 && units && entries) atomicAdd(units, entries);
}

// Work items (community r, slice y of nseg): groups y, y + nseg, ... of
// community r, so a community with many groups gets many blocks.  A
// community's buckets are taken in G = 2^gb groups of
// consecutive buckets, G the smallest power of two with about 2^kBigBucketBits
// staged entries per group.  A group's runs (one per stage column) are summed
// in an LDS table of at most `cap` slots sized for the group; a sub-group
// holding more distinct keys than the table is split in two by the next bit of
// the same mixing (a bijection, so distinct keys eventually part), depth
// first, and only sub-groups that fit are written out, each exactly once.
// Each written sub-group reserves its part of the super row with one atomic;
// block y = 0 also adds the community's own key.
__global__ __launch_bounds__(kBlock) void k_agg_emit(const BigComm* bc, const AggItem* items, uint32_t nitems,
                                                     const uint32_t* skeys,
                                                     const unsigned long long* svals, const uint16_t* smat,
                                                     const unsigned long long* stage_ctr,
                                                     const unsigned long long* self_acc, const uint64_t* cap_off,
                                                     uint32_t* out_len, uint32_t* out_cols, int64_t* out_w,
                                                     int64_t* Kout, uint32_t cap) {
  __shared__ uint32_t tk[kBigSlots];
  __shared__ unsigned long long tv[kBigSlots];
  __shared__ unsigned int rpre[kEmitWin];
  __shared__ unsigned int cbase[kEmitWin];
  __shared__ uint16_t rst[kEmitWin];
  __shared__ unsigned int wsum[kBlock / kWave];
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ unsigned int full, nout, obase;
  bool clean = false;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const AggItem x = items[it];
    const uint32_t r = x.big, y = x.pad, nslice = (uint32_t)x.a;
    const BigComm b = bc[r];
    const uint32_t rb = b.rbits, R = 1u << rb;
    const uint32_t nst = (uint32_t)(stage_ctr[r] >> kColShift);
    const uint16_t* mat = smat + b.moff;
    const uint64_t o = cap_off[b.c];
    if (y == 0 && threadIdx.x == 0) {
      const unsigned long long self = self_acc[r];
      if (self) {
        const unsigned int p = atomicAdd(&out_len[b.c], 1u);
        out_cols[o + p] = b.c;
        out_w[o + p] = (int64_t)self;
        atomicAdd((unsigned long long*)&Kout[b.c], self);
      }
    }
    unsigned long long tot = 0;
    for (uint32_t c = threadIdx.x; c < nst; c += kBlock) tot += mat[(size_t)R * b.smax + c];
    tot = block_sum(tot, red);
    uint32_t gb = 0;
    while (gb < rb && ((unsigned long long)1 << (kBigBucketBits + gb)) < tot) ++gb;
    const uint32_t G = 1u << gb, span = rb - gb;
    const uint32_t nseg = min(G, nslice);
    if (y >= nseg) continue;  // block-uniform
    if (!clean) {
      for (uint32_t sl = threadIdx.x; sl < kBigSlots; sl += kBlock) {
        tk[sl] = kNone;
        tv[sl] = 0;
      }
      __syncthreads();
      clean = true;
    }
    for (uint32_t grp = y; grp < G; grp += nseg) {
      const uint32_t b0 = grp << span, b1 = (grp + 1) << span;
      // sub-group (q, sub): keys whose q mixing bits after the group's bits
      // equal sub; walked depth first over the leaves that fit
      uint32_t q = 0, sub = 0;
      for (;;) {
        uint32_t mask = cap - 1;
        if (threadIdx.x == 0) {
          full = 0;
          nout = 0;
        }
        uint64_t wbase = 0;  // staging slots of the columns before the window
        for (uint32_t c0 = 0; c0 < nst; c0 += kEmitWin) {
          const uint32_t cw = min(kEmitWin, nst - c0);
          for (uint32_t i = threadIdx.x; i < cw; i += kBlock) {
            const uint32_t s0 = mat[(size_t)b0 * b.smax + c0 + i], s1 = mat[(size_t)b1 * b.smax + c0 + i];
            rst[i] = (uint16_t)s0;
            rpre[i] = s1 - s0;
            cbase[i] = mat[(size_t)R * b.smax + c0 + i];
          }
          __syncthreads();
          const uint32_t n = block_exclusive_scan<kEmitWin / kBlock>(rpre, cw, wsum);
          const uint32_t wslots = block_exclusive_scan<kEmitWin / kBlock>(cbase, cw, wsum);
          if (nst <= kEmitWin) mask = min(cap, pow2_at_least(2 * n)) - 1;
          for (uint32_t xx = threadIdx.x; xx < n; xx += kBlock) {
            uint32_t lo = 0, hi = cw - 1;
            while (lo < hi) {
              const uint32_t mid = (lo + hi + 1) >> 1;
              if (rpre[mid] <= xx)
                lo = mid;
              else
                hi = mid - 1;
            }
            const size_t pos = b.soff + wbase + cbase[lo] + rst[lo] + (xx - rpre[lo]);
            const uint32_t c = skeys[pos];
            if (q && ((big_mix(c) << gb) >> (32 - q)) != sub) continue;
            if (!table_add_bounded(tk, tv, mask, c, svals[pos], kRowSalt)) full = 1;
          }
          __syncthreads();
          wbase += wslots;
        }
        const bool fits = full == 0;
        unsigned long long ksum = 0;
        if (fits) {
          for (uint32_t sl = threadIdx.x; sl <= mask; sl += kBlock)
            if (tk[sl] != kNone) {
              atomicAdd(&nout, 1u);
              ksum += tv[sl];
            }
        }
        ksum = block_sum(ksum, red);
        if (fits && threadIdx.x == 0 && nout) {
          obase = atomicAdd(&out_len[b.c], nout);
          atomicAdd((unsigned long long*)&Kout[b.c], ksum);
          nout = 0;
        }
        __syncthreads();
        for (uint32_t sl = threadIdx.x; sl <= mask; sl += kBlock) {
          const uint32_t c = tk[sl];
          if (c == kNone) continue;
          if (fits) {
            const unsigned int p = obase + atomicAdd(&nout, 1u);
            out_cols[o + p] = c;
            out_w[o + p] = (int64_t)tv[sl];
          }
          tk[sl] = kNone;
          tv[sl] = 0;
        }
        __syncthreads();
        if (!fits) {  // split: its first half next
          ++q;
          sub <<= 1;
          continue;
        }
        // written: the next leaf is the sibling of the nearest first half above
        while (q > 0 && (sub & 1u)) {
          sub >>= 1;
          --q;
        }
        if (q == 0) break;
        ++sub;
      }
    }
  }
}

__global__ void k_zero_misc_agg(Ctl* ctl) {
  if (threadIdx.x < 4) ctl->misc[2 + threadIdx.x] = 0;
}

template <typename W>
int aggregate(hipStream_t s, Rows<W> g, uint32_t n, const uint32_t* C, uint32_t nc, AggBufs& b, int64_t* out_start,
              uint32_t* out_len, uint32_t* out_cols, int64_t* out_w, int64_t* Kout, Ctl* ctl, bool sorted_rows) {
  fill_u32(s, b.comm_count, 0, nc);
  fill_u64(s, b.comm_deg, 0, nc);
  scatter_count(s, C, n, b.comm_count, n);
  scatter_add_u32_to_u64(s, C, g.len, n, b.comm_deg, n);
  exclusive_scan_u32(s, b.comm_count, b.comm_off, nc, b.total, b.scan_tmp);
  (void)hipMemcpyAsync(b.comm_off + nc, b.total, sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  fill_u32(s, b.comm_fill, 0, nc);
  fill_u32(s, b.comm_fill_long, 0, nc);
  hipLaunchKernelGGL(k_comm_scatter, dim3(grid_n(n, 1024, 4096)), dim3(kBlock), 0, s, C, n, b.comm_off, b.comm_fill,
                     b.members, g.len, sorted_rows ? kSliceMinLen : kNone, b.comm_fill_long);
  hipLaunchKernelGGL(k_zero_misc_agg, dim3(1), dim3(64), 0, s, ctl);
  // capacity per community -> super-row starts
  hipLaunchKernelGGL(k_comm_classify, dim3(grid_n(nc, kBlock * kTileU)), dim3(kBlock), 0, s, nc, b.comm_deg, b.cap_off,
                     out_len, Kout, b.small_lists, (size_t)nc, ctl);
  exclusive_scan_u64(s, b.cap_off, (uint64_t*)out_start, nc, b.total, b.scan_tmp);
  // kernel launches for small / medium communities read their counts on device
  hipLaunchKernelGGL((k_agg_lds<64, 256, W>), dim3(grid_n(nc, kBlock / 64, 2048)), dim3(kBlock), 0, s, g, C, b.members,
                     b.comm_off, b.small_lists, &ctl->misc[2], b.comm_deg, (const uint64_t*)out_start, out_len,
                     out_cols, out_w, Kout);
  hipLaunchKernelGGL((k_agg_lds<kBlock, 1024, W>), dim3(grid_n(nc, 1, 2048)), dim3(kBlock), 0, s, g, C, b.members,
                     b.comm_off, b.small_lists + 3 * (size_t)nc, &ctl->misc[5], b.comm_deg,
                     (const uint64_t*)out_start, out_len, out_cols, out_w, Kout);
  hipLaunchKernelGGL((k_agg_lds<kBlock, 4096, W>), dim3(grid_n(nc, 1, 2048)), dim3(kBlock), 0, s, g, C, b.members,
                     b.comm_off, b.small_lists + (size_t)nc, &ctl->misc[3], b.comm_deg, (const uint64_t*)out_start,
                     out_len, out_cols, out_w, Kout);
  // big communities: plan staging areas on the host
  unsigned int* pn = (unsigned int*)pinned_stage(4);
  if (!pn) return -1;
  (void)hipMemcpyAsync(pn, &ctl->misc[4], sizeof(unsigned int), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  const unsigned int nbig = *pn;
  if (nbig == 0) return 0;
  // entry offsets of the members in member order (lengths in comm_fill, free after the scatter)
  hipLaunchKernelGGL(k_member_len, dim3(grid_n(n)), dim3(kBlock), 0, s, b.members, n, g.len, b.comm_fill);
  exclusive_scan_u32(s, b.comm_fill, b.member_eoff, n, b.member_eoff + n, b.scan_tmp);
  const uint32_t* big = b.small_lists + 2 * (size_t)nc;
  hipLaunchKernelGGL(k_big_info, dim3(grid_n(nbig)), dim3(kBlock), 0, s, big, &ctl->misc[4], b.comm_off, b.cap_off,
                     b.comm_deg, b.comm_fill_long, b.big_info);
  const size_t ib = sizeof(uint64_t) * 4 * nbig, idb = sizeof(uint32_t) * nbig;
  char* st = (char*)pinned_stage(ib + idb);
  if (!st) return -1;
  (void)hipMemcpyAsync(st, b.big_info, ib, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(st + ib, big, idb, hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  const std::vector<uint64_t> info((const uint64_t*)st, (const uint64_t*)(st + ib));
  const std::vector<uint32_t> ids((const uint32_t*)(st + ib), (const uint32_t*)(st + ib + idb));
  uint32_t first = 0;
  while (first < nbig) {
    // a round: as many communities as their staging areas, matrices and
    // work items fit
    std::vector<BigComm> rc;
    std::vector<AggItem> lists[kSlices];
    uint64_t used = 0, mused = 0, nemitted = 0, nstage = 0, spread = 0;
    uint32_t last = first;
    while (last < nbig) {
      const uint64_t m0 = info[4 * last], m1 = info[4 * last + 1], deg = info[4 * last + 3];
      const uint64_t cap = info[4 * last + 2] & 0xFFFFFFFFull, nlong = info[4 * last + 2] >> 32;
      // long rows (at the back of the member range) by slices, the others whole
      const bool sliced = sorted_rows && deg >= kSliceMinDeg && nlong > 0;
      const uint64_t ml = sliced ? m1 - nlong : m1;
      // ranges over [0, deg), clipped on the device to the whole-row members' entries
      const uint64_t nrange = ml > m0 ? (deg + kRangeEntries - 1) / kRangeEntries : 0;
      const uint64_t nitems = nrange + (m1 - ml + kSliceMembers - 1) / kSliceMembers * kSlices;
      // stage columns: every item's stages hold at most kBigStage entries, so
      // deg / kBigStage + one partial stage per item
      const uint64_t smax = deg / kBigStage + nitems + 1;
      uint32_t rb = 0;
      while (rb < kBigMaxRbits && ((uint64_t)1 << (kBigBucketBits + rb)) < std::min(cap, deg)) ++rb;
      const uint64_t slots = deg, ment = (((uint64_t)1 << rb) + 1) * smax;
      const uint64_t nemit = std::min<uint64_t>(kEmitSlices, (uint64_t)1 << rb);
      if (slots > b.scap || ment > b.mcap || nitems + nemit > b.item_cap) return -2;
      if (last > first &&
          (used + slots > b.scap || mused + ment > b.mcap || nstage + nemitted + nitems + nemit > b.item_cap))
        break;
      const uint32_t r = (uint32_t)rc.size();
      rc.push_back(BigComm{ids[last], rb, (uint32_t)smax, (uint32_t)(ml - m0), used, mused});
      for (uint64_t j = 0; j < nrange; ++j)
        lists[spread++ % kSlices].push_back(
            AggItem{r, kRange, j * kRangeEntries, std::min(deg, (j + 1) * kRangeEntries)});
      for (uint64_t a = ml; a < m1; a += kSliceMembers)
        for (uint32_t x = 0; x < kSlices; ++x) lists[x].push_back(AggItem{r, x, a, std::min(m1, a + kSliceMembers)});
      used += slots;
      mused += ment;
      nemitted += nemit;
      nstage += nitems;
      ++last;
    }
    const uint32_t nr = (uint32_t)rc.size();
    // stage items list by list (list offsets in sl)
    std::vector<AggItem> ins;
    unsigned int sl[kSlices + 1] = {};
    size_t longest = 0;
    for (uint32_t x = 0; x < kSlices; ++x) {
      sl[x] = (unsigned int)ins.size();
      ins.insert(ins.end(), lists[x].begin(), lists[x].end());
      longest = std::max(longest, lists[x].size());
    }
    sl[kSlices] = (unsigned int)ins.size();
    const size_t nins = ins.size();
    // emit items: (community, slice of up to kEmitSlices) after the stage items
    for (uint32_t r = 0; r < nr; ++r) {
      const uint32_t ns = std::min<uint32_t>(kEmitSlices, 1u << rc[r].rbits);
      for (uint32_t y = 0; y < ns; ++y) ins.push_back(AggItem{r, y, ns, 0});
    }
    AggItem* di = (AggItem*)b.items;
    // through pinned memory: the copies queue behind the kernels instead of
    // each waiting for the stream (the round ends with a synchronisation)
    const size_t rb_bytes = sizeof(BigComm) * nr, ib2 = sizeof(AggItem) * ins.size();
    char* hs = (char*)pinned_stage(rb_bytes + ib2 + sizeof(sl));
    if (!hs) return -1;
    std::memcpy(hs, rc.data(), rb_bytes);
    std::memcpy(hs + rb_bytes, ins.data(), ib2);
    std::memcpy(hs + rb_bytes + ib2, sl, sizeof(sl));
    (void)hipMemcpyAsync(b.bigc, hs, rb_bytes, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(di, hs + rb_bytes, ib2, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(b.slice_ctl, hs + rb_bytes + ib2, sizeof(sl), hipMemcpyHostToDevice, s);
    fill_u64(s, (uint64_t*)b.stage_ctr, 0, nr);
    fill_u64(s, (uint64_t*)b.self_acc, 0, nr);
    // the input graph's big communities are timed as LEIDEN_KT_AGG_BIG
    const bool timed = sizeof(W) == 4;
    if (timed) kt_mark(LEIDEN_KT_AGG_BIG, s);
    hipLaunchKernelGGL(k_agg_stage<W>, dim3(kSlices * std::min<size_t>(longest, 512)), dim3(kBlock), 0, s, g, C, b.members,
                       (const uint64_t*)b.comm_off, (const uint64_t*)b.member_eoff, (const BigComm*)b.bigc, di, b.slice_ctl, (n + kSlices - 1) / kSlices, b.skeys, b.svals, b.smat,
                       b.stage_ctr, b.self_acc, timed ? &ctl->kt_units[LEIDEN_KT_AGG_BIG] : nullptr);
    if (timed) kt_mark(LEIDEN_KT_AGG_BIG, s);
    const size_t nemit = ins.size() - nins;
    const uint32_t ecap = (b.emit_cap >= 16 && b.emit_cap <= kBigSlots) ? b.emit_cap : kBigSlots;
    hipLaunchKernelGGL(k_agg_emit, dim3(std::min<size_t>(nemit, 8192)), dim3(kBlock), 0, s, (const BigComm*)b.bigc,
                       di + nins, (uint32_t)nemit, b.skeys, b.svals, b.smat, b.stage_ctr, b.self_acc,
                       (const uint64_t*)out_start, out_len, out_cols, out_w, Kout, ecap);
    if (hipStreamSynchronize(s) != hipSuccess) return -1;  // host vectors must outlive the copies
    first = last;
  }
  return 0;
}

template int aggregate<uint32_t>(hipStream_t, Rows<uint32_t>, uint32_t, const uint32_t*, uint32_t, AggBufs&, int64_t*,
                                 uint32_t*, uint32_t*, int64_t*, int64_t*, Ctl*, bool);
template int aggregate<int64_t>(hipStream_t, Rows<int64_t>, uint32_t, const uint32_t*, uint32_t, AggBufs&, int64_t*,
                                uint32_t*, uint32_t*, int64_t*, int64_t*, Ctl*, bool);

// ---------------------------------------------------------------------------
// Static output labels: dense, ordered by each community's minimum vertex.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_first_flag(const uint32_t* C, uint32_t n, const uint32_t* minv,
                                                       uint32_t* flag) {
  GRID_STRIDE(i, n) flag[i] = minv[C[i]] == (uint32_t)i ? 1u : 0u;
}

// In a forest every graph ranks its own communities from zero, and the label
// is offset by the graph's first vertex.
__global__ __launch_bounds__(kBlock) void k_rank_label(const uint32_t* C, uint32_t n, const uint32_t* minv,
                                                       const uint64_t* rank, uint32_t* out, const uint32_t* fgid,
                                                       const uint32_t* fbase) {
  GRID_STRIDE(i, n) {
    const uint32_t m = minv[C[i]];
    if (fgid) {
      const uint32_t b = fbase[fgid[i]];
      out[i] = b + (uint32_t)(rank[m] - rank[b]);
    } else {
      out[i] = (uint32_t)rank[m];
    }
  }
}

void launch_static_relabel(hipStream_t s, const uint32_t* C, uint32_t n, uint32_t* minv, uint32_t* flag,
                           uint64_t* rank, uint32_t* out, void* scan_tmp, uint64_t* total, const uint32_t* fgid,
                           const uint32_t* fbase) {
  if (n == 0) return;
  fill_u32(s, minv, kNone, n);
  scatter_min_index(s, C, n, minv, n);
  hipLaunchKernelGGL(k_first_flag, dim3(grid_n(n)), dim3(kBlock), 0, s, C, n, minv, flag);
  exclusive_scan_u32(s, flag, rank, n, total, scan_tmp);
  hipLaunchKernelGGL(k_rank_label, dim3(grid_n(n)), dim3(kBlock), 0, s, C, n, minv, rank, out, fgid, fbase);
}

// ---------------------------------------------------------------------------
// Eq. 1 parts: sigma (weight of entries inside communities), Sigma_c, and
// T = sum Sigma_c^2 as a 128-bit integer.  The host forms
// Q = sigma / 2m - T / (2m)^2.
// ---------------------------------------------------------------------------
// sigma partial sums, one wavefront per row (long rows: listed chunks)
__global__ __launch_bounds__(kBlock) void k_mod_sigma(Rows<uint32_t> g, uint32_t n, const uint32_t* C,
                                                      unsigned long long* partials, unsigned long long* items) {
  __shared__ unsigned long long red[kBlock / kWave];
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned long long sig = 0;
  for (uint64_t i = wave; i < n; i += nwaves) {
    const uint32_t c = C[i];
    const int64_t s0 = g.start[i];
    const uint32_t L = g.len[i];
    if (L > kWaveRowMax) {  // wavefront-uniform
      list_row_chunks(items, (uint32_t)i, L, lane);
      continue;
    }
    for (uint32_t e = lane; e < L; e += kWave)
      if (C[g.cols[s0 + e]] == c) sig += g.w[s0 + e];
  }
  sig = block_sum(sig, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = sig;
}

// the listed chunks, one block each; one partial sum per block
__global__ __launch_bounds__(kBlock) void k_mod_sigma_long(Rows<uint32_t> g, const uint32_t* C,
                                                           const unsigned long long* items,
                                                           unsigned long long* partials) {
  __shared__ unsigned long long red[kBlock / kWave];
  const unsigned long long cnt = items[0];
  unsigned long long sig = 0;
  for (unsigned long long q = blockIdx.x; q < cnt; q += gridDim.x) {
    const unsigned long long it = items[1 + q];
    const uint32_t i = (uint32_t)(it >> 32), e0 = (uint32_t)it * kRowChunk;
    const uint32_t e1 = min(g.len[i], e0 + kRowChunk);
    const int64_t s0 = g.start[i];
    const uint32_t c = C[i];
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBlock)
      if (C[g.cols[s0 + e]] == c) sig += g.w[s0 + e];
  }
  sig = block_sum(sig, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = sig;
}

__global__ __launch_bounds__(kBlock) void k_mod_square(uint32_t n, const int64_t* Sig, unsigned long long* partials) {
  __shared__ unsigned long long rhi[kBlock], rlo[kBlock];
  unsigned long long hi = 0, lo = 0;
  GRID_STRIDE(c, n) {
    const unsigned long long x = (unsigned long long)Sig[c];
    const unsigned long long plo = x * x;
    const unsigned long long phi = __umul64hi(x, x);
    lo += plo;
    hi += phi + (lo < plo ? 1ull : 0ull);
  }
  rhi[threadIdx.x] = hi;
  rlo[threadIdx.x] = lo;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long H = 0, L = 0;
    for (int t = 0; t < kBlock; ++t) {
      L += rlo[t];
      H += rhi[t] + (L < rlo[t] ? 1ull : 0ull);
    }
    partials[2 * blockIdx.x] = H;
    partials[2 * blockIdx.x + 1] = L;
  }
}

// Totals of the per-block parts: sigma of both sigma launches (nblocks each),
// and the 128-bit sum of squares with its carries.
__global__ __launch_bounds__(kBlock) void k_mod_final(const unsigned long long* sig_part,
                                                      const unsigned long long* sq_part,
                                                      const unsigned long long* long_part, int nblocks,
                                                      ModParts* out) {
  __shared__ unsigned long long rs[kBlock], rh[kBlock], rl[kBlock];
  unsigned long long sig = 0, H = 0, L = 0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    sig += sig_part[b] + long_part[b];
    L += sq_part[2 * b + 1];
    H += sq_part[2 * b] + (L < sq_part[2 * b + 1] ? 1ull : 0ull);
  }
  rs[threadIdx.x] = sig;
  rh[threadIdx.x] = H;
  rl[threadIdx.x] = L;
  __syncthreads();
  if (threadIdx.x == 0) {
    sig = H = L = 0;
    for (int t = 0; t < kBlock; ++t) {
      sig += rs[t];
      L += rl[t];
      H += rh[t] + (L < rl[t] ? 1ull : 0ull);
    }
    out->sigma = sig;
    out->T_hi = H;
    out->T_lo = L;
  }
}

void modularity_parts(hipStream_t s, Rows<uint32_t> g, uint32_t n, const uint32_t* C, const int64_t* K, int64_t* Sig,
                      unsigned long long* partials, int nblocks, ModParts* out_dev, unsigned long long* items) {
  fill_i64(s, Sig, 0, n);
  scatter_add_i64(s, C, K, n, Sig, n);
  fill_u64(s, (uint64_t*)items, 0, 1);
  hipLaunchKernelGGL(k_mod_sigma, dim3(nblocks), dim3(kBlock), 0, s, g, n, C, partials, items);
  hipLaunchKernelGGL(k_mod_sigma_long, dim3(nblocks), dim3(kBlock), 0, s, g, C, items, partials + 3 * nblocks);
  hipLaunchKernelGGL(k_mod_square, dim3(nblocks), dim3(kBlock), 0, s, n, Sig, partials + nblocks);
  hipLaunchKernelGGL(k_mod_final, dim3(1), dim3(kBlock), 0, s, partials, partials + nblocks, partials + 3 * nblocks,
                     nblocks, out_dev);
}

// ---------------------------------------------------------------------------
// Alg. 12 by its stated purpose: exact maximum overlap (total K^t of shared
// vertices) between old and current communities; ties go to the current
// community with the lowest minimum vertex, then to the lowest old ID;
// unmatched current communities take the smallest IDs that were not old
// labels, in ascending order of their minimum vertex.
// ---------------------------------------------------------------------------
constexpr unsigned long long kNone64 = ~0ull;

__device__ inline uint64_t pair_slot(unsigned long long key, uint64_t mask) {
  return ((key * 0x9E3779B97F4A7C15ull) >> 17) & mask;
}

__device__ inline uint64_t pair_insert(unsigned long long* hk, uint64_t mask, unsigned long long key) {
  uint64_t h = pair_slot(key, mask);
  while (true) {
    const unsigned long long k = ld_near(&hk[h]);
    if (k == key) return h;
    if (k == kNone64) {
      const unsigned long long o = atomicCAS(&hk[h], kNone64, key);
      if (o == kNone64 || o == key) return h;
    }
    h = (h + 1) & mask;
  }
}

// The community each old label continues in the first place: cb[x] =
// Ccur[head[x]], the current community of the old community's minimum vertex
// (kNone when x is not an old label).  Any choice is exact (it only decides
// which pairs are summed in place); this one holds most vertices of x.
__global__ __launch_bounds__(kBlock) void k_track_cb(uint32_t n, const uint32_t* head, const uint32_t* Ccur,
                                                     uint32_t* cb) {
  GRID_STRIDE(x, n) {
    const uint32_t h = head[x];
    cb[x] = h == kNone ? kNone : Ccur[h];
  }
}

// Pairs (old label b, current community c) of the vertices.  A vertex whose
// pair is (b, cb[b]) is common: its weight goes to Kc, summed per old label
// by a bucketed scatter.  The other (rare) pairs are summed per tile of 1024
// vertices in LDS and then added once per tile to the global pair table; the
// slots a tile creates are listed.
__global__ __launch_bounds__(kBlock) void k_track_split(uint32_t n, const uint32_t* Ccur, const uint32_t* Cprev,
                                                        const int64_t* K, const uint32_t* cb, int64_t* Kc,
                                                        unsigned long long* hk, long long* hv, uint64_t mask,
                                                        uint32_t* owners, unsigned int* owner_count) {
  constexpr int kTile = 1024, kSlots = 2048;
  __shared__ unsigned long long lk[kSlots];
  __shared__ unsigned long long lv[kSlots];
  __shared__ unsigned int nrare;
  for (uint64_t base = (uint64_t)blockIdx.x * kTile; base < n; base += (uint64_t)gridDim.x * kTile) {
    for (int s = threadIdx.x; s < kSlots; s += kBlock) {
      lk[s] = kNone64;
      lv[s] = 0;
    }
    if (threadIdx.x == 0) nrare = 0;
    __syncthreads();
    unsigned int mine = 0;
    for (int t = threadIdx.x; t < kTile; t += kBlock) {
      const uint64_t i = base + t;
      if (i >= n) continue;
      const uint32_t b = Cprev[i], c = Ccur[i];
      const bool common = cb[b] == c;
      Kc[i] = common ? K[i] : 0;
      if (common) continue;
      ++mine;
      const unsigned long long key = ((unsigned long long)b << 32) | c;
      uint32_t h = (uint32_t)pair_slot(key, kSlots - 1);
      while (true) {
        const unsigned long long o = atomicCAS(&lk[h], kNone64, key);
        if (o == kNone64 || o == key) break;
        h = (h + 1) & (kSlots - 1);
      }
      atomicAdd(&lv[h], (unsigned long long)K[i]);
    }
    if (mine) atomicAdd(&nrare, mine);
    __syncthreads();
    if (nrare) {  // block-uniform
      for (int s0 = 0; s0 < kSlots; s0 += kBlock) {
        const int s = s0 + threadIdx.x;
        const unsigned long long key = lk[s];
        uint32_t created = kNone, slot = 0;
        if (key != kNone64) {
          uint64_t h = pair_slot(key, mask);
          while (true) {
            const unsigned long long k = ld_near(&hk[h]);
            if (k == key) break;
            if (k == kNone64) {
              const unsigned long long o = atomicCAS(&hk[h], kNone64, key);
              if (o == kNone64) {
                created = 0;
                break;
              }
              if (o == key) break;
            }
            h = (h + 1) & mask;
          }
          atomicAdd((unsigned long long*)&hv[h], lv[s]);
          slot = (uint32_t)h;
        }
        wave_append(created, slot, [&](uint32_t, uint32_t*& l, unsigned int*& cnt) {
          l = owners;
          cnt = owner_count;
        });
      }
    }
    __syncthreads();
  }
}

// A pair of the two sources: item x < n is old label x's common pair (when x
// is an old label), item n + k the k-th listed rare pair.
struct TrackPair {
  uint32_t b, c;
  long long w;
  bool ok;
};
__device__ inline TrackPair track_pair(uint64_t x, uint32_t n, const uint32_t* cb, const int64_t* wb,
                                       const unsigned long long* hk, const long long* hv, const uint32_t* owners) {
  TrackPair p{0, 0, 0, false};
  if (x < n) {
    const uint32_t c = cb[x];
    if (c != kNone) p = TrackPair{(uint32_t)x, c, (long long)wb[x], true};
  } else {
    const uint32_t h = owners[x - n];
    const unsigned long long k = hk[h];
    p = TrackPair{(uint32_t)(k >> 32), (uint32_t)k, hv[h], true};
  }
  return p;
}

// The maxima of the overlap weights are taken in two launches, weights of at
// least kTrackHeavy first: a large community's maximum is then in place
// before its many light pairs arrive, and those find it with a plain read
// (atomics on one address are serialised device-wide).
constexpr long long kTrackHeavy = 1ll << 16;

__global__ __launch_bounds__(kBlock) void k_track_best_w(uint32_t n, const uint32_t* cb, const int64_t* wb,
                                                         const unsigned long long* hk, const long long* hv,
                                                         const uint32_t* owners, const unsigned int* owner_count,
                                                         long long* best_w, bool heavy) {
  const uint64_t items = (uint64_t)n + *owner_count;
  GRID_STRIDE(x, items) {
    const TrackPair p = track_pair(x, n, cb, wb, hk, hv, owners);
    if (!p.ok || (p.w >= kTrackHeavy) != heavy) continue;
    // read first: most updates would not raise the maximum
    long long* slot = &best_w[p.b];
    if (peek(slot) < p.w) atomicMax(slot, p.w);
  }
}

__global__ __launch_bounds__(kBlock) void k_track_best_c(uint32_t n, const uint32_t* cb, const int64_t* wb,
                                                         const unsigned long long* hk, const long long* hv,
                                                         const uint32_t* owners, const unsigned int* owner_count,
                                                         const uint32_t* minv, const long long* best_w,
                                                         uint32_t* best_vmin) {
  const uint64_t items = (uint64_t)n + *owner_count;
  GRID_STRIDE(x, items) {
    const TrackPair p = track_pair(x, n, cb, wb, hk, hv, owners);
    if (!p.ok) continue;
    const uint32_t vm = minv[p.c];
    if (p.w == best_w[p.b] && peek(&best_vmin[p.b]) > vm) atomicMin(&best_vmin[p.b], vm);
  }
}

__global__ __launch_bounds__(kBlock) void k_track_cand_w(uint32_t n, const uint32_t* Ccur, const long long* best_w,
                                                         const uint32_t* best_vmin, long long* cand_w, bool heavy) {
  GRID_STRIDE(b, n) {
    const uint32_t vm = best_vmin[b];
    if (vm == kNone) continue;
    const long long w = best_w[b];
    if ((w >= kTrackHeavy) != heavy) continue;
    long long* slot = &cand_w[Ccur[vm]];
    if (peek(slot) < w) atomicMax(slot, w);
  }
}

__global__ __launch_bounds__(kBlock) void k_track_cand_b(uint32_t n, const uint32_t* Ccur, const long long* best_w,
                                                         const uint32_t* best_vmin, const long long* cand_w,
                                                         uint32_t* cand_b) {
  GRID_STRIDE(b, n) {
    const uint32_t vm = best_vmin[b];
    if (vm == kNone) continue;
    const uint32_t c = Ccur[vm];
    if (best_w[b] == cand_w[c] && peek(&cand_b[c]) > b) atomicMin(&cand_b[c], (uint32_t)b);
  }
}

// flag[v] = v is the minimum vertex of an unmatched current community;
// freeflag[x] = x is not an old label
__global__ __launch_bounds__(kBlock) void k_track_flags(uint32_t n, const uint32_t* Ccur, const uint32_t* minv,
                                                        const uint32_t* cand_b, const uint32_t* head, uint32_t* flag,
                                                        uint32_t* freeflag) {
  GRID_STRIDE(i, n) {
    const uint32_t c = Ccur[i];
    flag[i] = (minv[c] == (uint32_t)i && cand_b[c] == kNone) ? 1u : 0u;
    freeflag[i] = head[i] == kNone ? 1u : 0u;
  }
}

// Position of the r-th item (by a scan over the whole level) of x's graph in
// that graph's segment of a per-vertex array: in a forest, every graph ranks
// its own free IDs and unmatched communities from zero, in its own ID range.
__device__ inline uint64_t graph_pos(const uint32_t* gid, const uint32_t* base, const uint64_t* rank, uint32_t x,
                                     uint64_t r) {
  if (!gid) return r;
  const uint32_t b = base[gid[x]];
  return b + (r - rank[b]);
}

__global__ __launch_bounds__(kBlock) void k_track_free(uint32_t n, const uint32_t* freeflag, const uint64_t* free_rank,
                                                       uint32_t* free_id, const uint32_t* fgid, const uint32_t* fbase) {
  GRID_STRIDE(x, n) if (freeflag[x]) free_id[graph_pos(fgid, fbase, free_rank, (uint32_t)x, free_rank[x])] = (uint32_t)x;
}

// The tracked label of community c: its matched old label, else the next
// free ID (by its minimum vertex).
__device__ inline uint32_t tracked_label(uint32_t c, uint32_t m, const uint32_t* cand_b, const uint64_t* rank,
                                         const uint32_t* free_id, const uint32_t* fgid, const uint32_t* fbase) {
  const uint32_t b = cand_b[c];
  return b != kNone ? b : free_id[graph_pos(fgid, fbase, rank, m, rank[m])];
}

__global__ __launch_bounds__(kBlock) void k_track_label(uint32_t n, const uint32_t* Ccur, const uint32_t* minv,
                                                        const uint32_t* cand_b, const uint64_t* rank,
                                                        const uint32_t* free_id, uint32_t* out, uint8_t* matched,
                                                        const uint32_t* fgid, const uint32_t* fbase) {
  GRID_STRIDE(i, n) {
    const uint32_t c = Ccur[i];
    const uint32_t b = cand_b[c];
    if (b != kNone) {
      out[i] = b;
      raise_flag(matched, b);
    } else {
      out[i] = tracked_label(c, minv[c], cand_b, rank, free_id, fgid, fbase);
    }
  }
}

// The minimum vertex of every community under its tracked label, for the
// next call (head must be all kNone before).
__global__ __launch_bounds__(kBlock) void k_track_heads(uint32_t n, const uint32_t* minv, const uint32_t* cand_b,
                                                        const uint64_t* rank, const uint32_t* free_id,
                                                        const uint32_t* fgid, const uint32_t* fbase, uint32_t* head) {
  GRID_STRIDE(c, n) {
    const uint32_t m = minv[c];
    if (m == kNone) continue;
    head[tracked_label((uint32_t)c, m, cand_b, rank, free_id, fgid, fbase)] = m;
  }
}

// The pair table's used slots back to empty (the table stays clean between calls).
__global__ __launch_bounds__(kBlock) void k_track_clear(unsigned long long* hk, long long* hv, const uint32_t* owners,
                                                        const unsigned int* owner_count) {
  GRID_STRIDE(k, *owner_count) {
    const uint32_t h = owners[k];
    hk[h] = kNone64;
    hv[h] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_track_minv_self(uint32_t n, const uint32_t* Ccur, uint32_t* minv) {
  GRID_STRIDE(v, n) if (Ccur[v] == (uint32_t)v) minv[v] = (uint32_t)v;
}

// head[label] = minimum vertex of the community of each label of C.
void track_heads_of(hipStream_t s, uint32_t n, const uint32_t* C, uint32_t* head) {
  fill_u32(s, head, kNone, n);
  scatter_min_index(s, C, n, head, n);
}

void track(hipStream_t s, uint32_t n, const uint32_t* Ccur, const uint32_t* Cprev, const int64_t* K, uint32_t* out,
           int64_t* S_out, bool labels_are_min, TrackBufs& b) {
  if (n == 0) return;
  // minimum vertex of each current community
  fill_u32(s, b.minv, kNone, n);
  if (labels_are_min)
    hipLaunchKernelGGL(k_track_minv_self, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Ccur, b.minv);
  else
    scatter_min_index(s, Ccur, n, b.minv, n);
  // overlap weights: common pairs per old label, rare pairs in the table
  hipLaunchKernelGGL(k_track_cb, dim3(grid_n(n)), dim3(kBlock), 0, s, n, b.head, Ccur, b.cb);
  fill_u32(s, b.owner_count, 0, 1);
  hipLaunchKernelGGL(k_track_split, dim3(grid_n(n, 1024, 4096)), dim3(kBlock), 0, s, n, Ccur, Cprev, K, b.cb, b.Kc,
                     b.hkeys, b.hvals, b.hmask, b.owners, b.owner_count);
  fill_i64(s, b.wb, 0, n);
  scatter_add_i64(s, Cprev, b.Kc, n, b.wb, n);
  // best current community of every old label, then the best old label of
  // every current community
  fill_i64(s, (int64_t*)b.best_w, -1, n);
  fill_u32(s, b.best_vmin, kNone, n);
  const int gp = grid_n(2 * (uint64_t)n);
  for (const bool heavy : {true, false})
    hipLaunchKernelGGL(k_track_best_w, dim3(gp), dim3(kBlock), 0, s, n, b.cb, b.wb, b.hkeys, b.hvals, b.owners,
                       b.owner_count, b.best_w, heavy);
  hipLaunchKernelGGL(k_track_best_c, dim3(gp), dim3(kBlock), 0, s, n, b.cb, b.wb, b.hkeys, b.hvals, b.owners,
                     b.owner_count, b.minv, b.best_w, b.best_vmin);
  fill_i64(s, (int64_t*)b.cand_w, -1, n);
  fill_u32(s, b.cand_b, kNone, n);
  for (const bool heavy : {true, false})
    hipLaunchKernelGGL(k_track_cand_w, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Ccur, b.best_w, b.best_vmin, b.cand_w,
                       heavy);
  hipLaunchKernelGGL(k_track_cand_b, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Ccur, b.best_w, b.best_vmin, b.cand_w,
                     b.cand_b);
  uint32_t* freeflag = b.label;  // scratch reuse
  hipLaunchKernelGGL(k_track_flags, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Ccur, b.minv, b.cand_b, b.head, b.flag,
                     freeflag);
  exclusive_scan_u32(s, b.flag, b.rank, n, b.total, b.scan_tmp);
  exclusive_scan_u32(s, freeflag, b.free_rank, n, b.total, b.scan_tmp);
  hipLaunchKernelGGL(k_track_free, dim3(grid_n(n)), dim3(kBlock), 0, s, n, freeflag, b.free_rank, b.free_id, b.f_gid,
                     b.f_base);
  fill_u8(s, b.matched, 0, n);
  hipLaunchKernelGGL(k_track_label, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Ccur, b.minv, b.cand_b, b.rank,
                     b.free_id, out, b.matched, b.f_gid, b.f_base);
  // the heads of the tracked labels, for the next call
  fill_u32(s, b.head, kNone, n);
  hipLaunchKernelGGL(k_track_heads, dim3(grid_n(n)), dim3(kBlock), 0, s, n, b.minv, b.cand_b, b.rank, b.free_id,
                     b.f_gid, b.f_base, b.head);
  // Sigma^t under the tracked labels
  launch_sigma_from(s, out, K, n, S_out);
  // the pair table back to empty
  hipLaunchKernelGGL(k_track_clear, dim3(grid_n(n)), dim3(kBlock), 0, s, b.hkeys, b.hvals, b.owners, b.owner_count);
}

// head[label] of dense static labels: the first vertex of every community
// (flag[i] = i is its community's minimum vertex) under its output label.
__global__ __launch_bounds__(kBlock) void k_heads_from_first(uint32_t n, const uint32_t* flag, const uint32_t* out,
                                                             uint32_t* head) {
  GRID_STRIDE(i, n) if (flag[i]) head[out[i]] = (uint32_t)i;
}

void static_heads(hipStream_t s, uint32_t n, const uint32_t* flag, const uint32_t* out, uint32_t* head) {
  if (n == 0) return;
  fill_u32(s, head, kNone, n);
  hipLaunchKernelGGL(k_heads_from_first, dim3(grid_n(n)), dim3(kBlock), 0, s, n, flag, out, head);
}

}  // namespace lm
