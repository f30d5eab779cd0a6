// Forests: many independent graphs as one block-diagonal graph, so that every
// phase of Alg. 4 (local moving, refinement, aggregation, and the dynamic
// marking, split and tracking steps) takes one launch for all of them.
//
// Vertex v of graph q is forest vertex first_q + v, and a community label of
// graph q is first_q + (its label inside q).  The level graphs stay block
// diagonal: aggregation keeps every community inside its graph, and dense
// renumbering keeps the graphs in order, so that a level's graphs are
// contiguous ranges again (their first super-vertices are the scan values at
// the graphs' first vertices).  What makes each graph's result equal to its
// result alone: the Eq. 2 constants are the graph's own (1/m, 1/(2 m^2)), the
// class and colour hashes of the schedules take graph-local IDs, and the
// stopping rules of Alg. 6 and Alg. 4 are evaluated per graph on its own gain
// sum, iteration count and refinement flag.  A graph that leaves the pass loop
// keeps its communities: it stays in the level graphs with every community a
// super-vertex of its own, takes no further moves, and so its final lookup
// equals the lookup through its refined labels at the pass where it stopped.
#include "kernels.h"

namespace lm {

static int grid_n(uint64_t n, int per_block = kBlock, int cap = 8192) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap) b = cap;
  return (int)b;
}

#define GRID_STRIDE(i, n) \
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < (uint64_t)(n); i += (uint64_t)gridDim.x * kBlock)

// Graph of every vertex of a level from the first vertices of its graphs
// (base has nq + 1 entries; the last is the vertex count): the last graph
// whose first vertex is at most v.
__global__ __launch_bounds__(kBlock) void k_forest_gid(uint32_t n, uint32_t nq, const uint32_t* base, uint32_t* gid) {
  GRID_STRIDE(v, n) {
    uint32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (base[mid] <= (uint32_t)v)
        lo = mid;
      else
        hi = mid - 1;
    }
    gid[v] = lo;
  }
}

void forest_gid(hipStream_t s, uint32_t n, uint32_t nq, const uint32_t* base, uint32_t* gid) {
  if (n && nq) hipLaunchKernelGGL(k_forest_gid, dim3(grid_n(n)), dim3(kBlock), 0, s, n, nq, base, gid);
}

// First super-vertex of every graph at the next level: the dense ID of the
// graph's first community, i.e. the scan of community flags at the graph's
// first vertex (labels of a graph lie in its vertex range).
__global__ void k_forest_next_base(uint32_t nq, uint32_t nl, const uint32_t* base, const uint64_t* newid,
                                   const uint64_t* total, uint32_t* next) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q <= nq; q += gridDim.x * blockDim.x)
    next[q] = (q < nq && base[q] < nl) ? (uint32_t)newid[base[q]] : (uint32_t)*total;
}

void forest_next_base(hipStream_t s, uint32_t nq, uint32_t nl, const uint32_t* base, const uint64_t* newid,
                      const uint64_t* total, uint32_t* next) {
  hipLaunchKernelGGL(k_forest_next_base, dim3(grid_n(nq + 1)), dim3(kBlock), 0, s, nq, nl, base, newid, total, next);
}

// Every entry of a row of graph q names a vertex of graph q (flag 1 if not).
__global__ __launch_bounds__(kBlock) void k_forest_check_rows(Rows<uint32_t> g, uint32_t n, const uint32_t* gid,
                                                              const uint32_t* base, unsigned int* flags) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned int f = 0;
  for (uint64_t i = wave; i < n; i += nwaves) {
    const uint32_t q = gid[i];
    const uint32_t lo = base[q], hi = base[q + 1];
    const int64_t s0 = g.start[i];
    for (uint32_t e = lane; e < g.len[i]; e += kWave) {
      const uint32_t j = g.cols[s0 + e];
      if (j < lo || j >= hi) f = 1;
    }
  }
  if (f) atomicOr(flags, f);
}

void forest_check_rows(hipStream_t s, Rows<uint32_t> g, uint32_t n, const uint32_t* gid, const uint32_t* base,
                       unsigned int* flags) {
  if (n) hipLaunchKernelGGL(k_forest_check_rows, dim3(grid_n(n, kBlock / kWave, 16384)), dim3(kBlock), 0, s, g, n, gid,
                            base, flags);
}

// Batch pairs join two vertices of one graph (flag 1 if not; vertex IDs out
// of range are left to the batch's own validation).  del holds (u, v) pairs,
// ins (u, v, w) triples.
__global__ __launch_bounds__(kBlock) void k_forest_check_batch(const uint32_t* del, uint64_t n_del, const uint32_t* ins,
                                                               uint64_t n_ins, uint32_t n, const uint32_t* gid,
                                                               unsigned int* flags) {
  unsigned int f = 0;
  GRID_STRIDE(t, n_del + n_ins) {
    const uint32_t u = t < n_del ? del[2 * t] : ins[3 * (t - n_del)];
    const uint32_t v = t < n_del ? del[2 * t + 1] : ins[3 * (t - n_del) + 1];
    if (u < n && v < n && gid[u] != gid[v]) f = 1;
  }
  if (f) atomicOr(flags, f);
}

void forest_check_batch(hipStream_t s, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                        uint32_t n, const uint32_t* gid, unsigned int* flags) {
  if (n_del + n_ins)
    hipLaunchKernelGGL(k_forest_check_batch, dim3(grid_n(n_del + n_ins)), dim3(kBlock), 0, s, del, n_del, ins, n_ins,
                       n, gid, flags);
}

// Labels inside each graph <-> forest labels.  to_forest flags labels that
// are not below the graph's vertex count (flag 1).
__global__ __launch_bounds__(kBlock) void k_forest_to_forest(uint32_t n, const uint32_t* gid, const uint32_t* base,
                                                             const uint32_t* local, uint32_t* out,
                                                             unsigned int* flags) {
  unsigned int f = 0;
  GRID_STRIDE(v, n) {
    const uint32_t q = gid[v];
    const uint32_t b = base[q], nq = base[q + 1] - b;
    const uint32_t x = local[v];
    if (x >= nq) {
      f = 1;
      out[v] = (uint32_t)v;
    } else {
      out[v] = b + x;
    }
  }
  if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kBlock) void k_forest_to_local(uint32_t n, const uint32_t* gid, const uint32_t* base,
                                                            const uint32_t* in, uint32_t* out) {
  GRID_STRIDE(v, n) out[v] = in[v] - base[gid[v]];
}

void forest_to_forest(hipStream_t s, uint32_t n, const uint32_t* gid, const uint32_t* base, const uint32_t* local,
                      uint32_t* out, unsigned int* flags) {
  if (n) hipLaunchKernelGGL(k_forest_to_forest, dim3(grid_n(n)), dim3(kBlock), 0, s, n, gid, base, local, out, flags);
}

void forest_to_local(hipStream_t s, uint32_t n, const uint32_t* gid, const uint32_t* base, const uint32_t* in,
                     uint32_t* out) {
  if (n) hipLaunchKernelGGL(k_forest_to_local, dim3(grid_n(n)), dim3(kBlock), 0, s, n, gid, base, in, out);
}

// Per-graph sums over a per-vertex (or per-label) array, where the graph of
// index x is gid[x]: every lane sums a contiguous run of indices and adds its
// partial sum to the graph's total whenever the graph changes (graphs are
// contiguous ranges, so a lane flushes about once per run).
__global__ __launch_bounds__(kBlock) void k_forest_sum(uint32_t n, const uint32_t* gid, const int64_t* x,
                                                       unsigned long long* out) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x, nt = (uint64_t)gridDim.x * kBlock;
  const uint64_t per = (n + nt - 1) / nt;
  const uint64_t a = t * per, e = a + per < n ? a + per : n;
  uint32_t cur = kNone;
  unsigned long long acc = 0;
  for (uint64_t i = a; i < e; ++i) {
    const uint32_t q = gid[i];
    if (q != cur) {
      if (cur != kNone && acc) atomicAdd(&out[cur], acc);
      cur = q;
      acc = 0;
    }
    acc += (unsigned long long)x[i];
  }
  if (cur != kNone && acc) atomicAdd(&out[cur], acc);
}

void forest_sum(hipStream_t s, uint32_t n, const uint32_t* gid, const int64_t* x, unsigned long long* out) {
  if (n) hipLaunchKernelGGL(k_forest_sum, dim3(grid_n(n, 16 * kBlock, 4096)), dim3(kBlock), 0, s, n, gid, x, out);
}

// Eq. 1 parts per graph: the weight of a graph's entries inside communities
// (one wavefront per row, contiguous rows per wavefront) ...
__global__ __launch_bounds__(kBlock) void k_forest_mod_rows(Rows<uint32_t> g, uint32_t n, const uint32_t* C,
                                                            const uint32_t* gid, unsigned long long* sig) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint64_t per = (n + nwaves - 1) / nwaves;
  const uint64_t a = wave * per, e = a + per < n ? a + per : n;
  uint32_t cur = kNone;
  unsigned long long acc = 0;
  for (uint64_t i = a; i < e; ++i) {
    const uint32_t q = gid[i];  // wavefront-uniform
    if (q != cur) {
      if (cur != kNone) {
        const unsigned long long t = group_sum<kWave>(acc);
        if (lane == 0 && t) atomicAdd(&sig[cur], t);
      }
      cur = q;
      acc = 0;
    }
    const uint32_t c = C[i];
    const int64_t s0 = g.start[i];
    for (uint32_t k = lane; k < g.len[i]; k += kWave)
      if (C[g.cols[s0 + k]] == c) acc += g.w[s0 + k];
  }
  if (cur != kNone) {
    const unsigned long long t = group_sum<kWave>(acc);
    if (lane == 0 && t) atomicAdd(&sig[cur], t);
  }
}

// ... and the sum of Sigma_c^2 over a graph's communities as a 128-bit integer
// (labels of a graph lie in its range, so label c belongs to graph gid[c]).
__device__ inline void add128(unsigned long long* hi, unsigned long long* lo, unsigned long long h,
                              unsigned long long l) {
  const unsigned long long old = atomicAdd(lo, l);
  atomicAdd(hi, h + (old + l < old ? 1ull : 0ull));
}

__global__ __launch_bounds__(kBlock) void k_forest_mod_square(uint32_t n, const int64_t* Sig, const uint32_t* gid,
                                                              unsigned long long* T_hi, unsigned long long* T_lo) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x, nt = (uint64_t)gridDim.x * kBlock;
  const uint64_t per = (n + nt - 1) / nt;
  const uint64_t a = t * per, e = a + per < n ? a + per : n;
  uint32_t cur = kNone;
  unsigned long long hi = 0, lo = 0;
  for (uint64_t c = a; c < e; ++c) {
    const uint32_t q = gid[c];
    if (q != cur) {
      if (cur != kNone && (hi | lo)) add128(&T_hi[cur], &T_lo[cur], hi, lo);
      cur = q;
      hi = lo = 0;
    }
    const unsigned long long x = (unsigned long long)Sig[c];
    const unsigned long long plo = x * x;
    const unsigned long long phi = __umul64hi(x, x);
    lo += plo;
    hi += phi + (lo < plo ? 1ull : 0ull);
  }
  if (cur != kNone && (hi | lo)) add128(&T_hi[cur], &T_lo[cur], hi, lo);
}

// parts: 4 x nq words (sigma, T_hi, T_lo, 2m), zeroed here
void forest_modularity_parts(hipStream_t s, Rows<uint32_t> g, uint32_t n, uint32_t nq, const uint32_t* C,
                             const int64_t* K, const uint32_t* gid, int64_t* Sig, unsigned long long* parts) {
  fill_u64(s, (uint64_t*)parts, 0, 4 * (size_t)nq);
  if (n == 0) return;
  launch_sigma_from(s, C, K, n, Sig);
  hipLaunchKernelGGL(k_forest_mod_rows, dim3(grid_n(n, 16 * (kBlock / kWave), 4096)), dim3(kBlock), 0, s, g, n, C,
                     gid, parts);
  hipLaunchKernelGGL(k_forest_mod_square, dim3(grid_n(n, 16 * kBlock, 4096)), dim3(kBlock), 0, s, n, Sig, gid,
                     parts + nq, parts + 2 * (size_t)nq);
  forest_sum(s, n, gid, K, parts + 3 * (size_t)nq);
}

// ---------------------------------------------------------------------------
// Per-graph control of the pass loop (one block; nq is at most a few 10^4).
// ---------------------------------------------------------------------------
__device__ inline unsigned int block_count(unsigned int x) {
  __shared__ unsigned long long red[kBlock / kWave];
  return (unsigned int)block_sum((unsigned long long)x, red);
}

// Start of a run: a graph with edges takes part; gain sums, flags and counts
// start at zero.
__global__ __launch_bounds__(kBlock) void k_forest_start(uint32_t nq, const unsigned long long* m2, uint8_t* move,
                                                         uint8_t* pass, uint8_t* refined, unsigned long long* dq,
                                                         uint32_t* cur_iters, uint32_t* passes, uint32_t* iters_hist,
                                                         Ctl* ctl) {
  unsigned int live = 0;
  for (uint32_t q = threadIdx.x; q < nq; q += kBlock) {
    const uint8_t on = m2[q] ? 1 : 0;
    move[q] = on;
    pass[q] = on;
    refined[q] = 0;
    dq[q] = 0;
    cur_iters[q] = 0;
    passes[q] = 0;
    for (uint32_t p = 0; p < kForestIterHist; ++p) iters_hist[(size_t)p * nq + q] = 0;
    live += on;
  }
  live = block_count(live);
  if (threadIdx.x == 0) {
    ctl->f_live = live;
    ctl->f_moving = live;
  }
}

// End of local-moving iteration li (Alg. 6): a graph whose gain sum of the
// iteration is at most tau, or that ran max_iters iterations, stops moving in
// this pass.  The same fixed-point-to-double conversion as for one graph.
__global__ __launch_bounds__(kBlock) void k_forest_iter_end(uint32_t nq, unsigned long long* dq, double tau,
                                                            uint32_t li, uint32_t max_iters, uint8_t* move,
                                                            uint32_t* cur_iters, Ctl* ctl) {
  unsigned int moving = 0;
  for (uint32_t q = threadIdx.x; q < nq; q += kBlock) {
    if (!move[q]) continue;
    const double g = (double)(long long)dq[q] / 72057594037927936.0;
    dq[q] = 0;
    cur_iters[q] = li + 1;
    if (g <= tau || li + 1 >= max_iters)
      move[q] = 0;
    else
      ++moving;
  }
  moving = block_count(moving);
  if (threadIdx.x == 0) ctl->f_moving = moving;
}

// End of pass `pass` (Alg. 4): a graph stops after a pass with at most one
// iteration, unless it is the first pass and some community was refined.
__global__ __launch_bounds__(kBlock) void k_forest_pass_end(uint32_t nq, uint32_t pass, uint32_t* cur_iters,
                                                            uint8_t* refined, uint8_t* pass_on, uint8_t* move,
                                                            uint32_t* passes, uint32_t* iters_hist, Ctl* ctl) {
  unsigned int live = 0;
  for (uint32_t q = threadIdx.x; q < nq; q += kBlock) {
    if (pass_on[q]) {
      const uint32_t it = cur_iters[q];
      passes[q] = pass + 1;
      if (pass < kForestIterHist) iters_hist[(size_t)pass * nq + q] = it;
      const bool stop = it <= 1 && (!refined[q] || pass > 0);
      if (stop) pass_on[q] = 0;
    }
    move[q] = pass_on[q];
    refined[q] = 0;
    cur_iters[q] = 0;
    live += pass_on[q];
  }
  live = block_count(live);
  if (threadIdx.x == 0) {
    ctl->f_live = live;
    ctl->f_moving = live;
  }
}

void forest_start(hipStream_t s, const ForestBufs& f, Ctl* ctl) {
  hipLaunchKernelGGL(k_forest_start, dim3(1), dim3(kBlock), 0, s, f.nq, f.m2, f.move, f.pass, f.refined, f.dq,
                     f.cur_iters, f.passes, f.iters_hist, ctl);
}

void forest_iter_end(hipStream_t s, const ForestBufs& f, double tau, uint32_t li, uint32_t max_iters, Ctl* ctl) {
  hipLaunchKernelGGL(k_forest_iter_end, dim3(1), dim3(kBlock), 0, s, f.nq, f.dq, tau, li, max_iters, f.move,
                     f.cur_iters, ctl);
}

void forest_pass_end(hipStream_t s, const ForestBufs& f, uint32_t pass, Ctl* ctl) {
  hipLaunchKernelGGL(k_forest_pass_end, dim3(1), dim3(kBlock), 0, s, f.nq, pass, f.cur_iters, f.refined, f.pass,
                     f.move, f.passes, f.iters_hist, ctl);
}

// The forest fields of the control block (the graph and first-vertex arrays
// of the current level).
__global__ void k_forest_bind(Ctl* ctl, const uint32_t* gid, const uint32_t* base, const double* inv,
                              unsigned long long* dq, const uint8_t* move, const uint8_t* pass, uint8_t* refined) {
  if (threadIdx.x != 0) return;
  ctl->f_gid = gid;
  ctl->f_base = base;
  ctl->f_inv = inv;
  ctl->f_dq = dq;
  ctl->f_move = move;
  ctl->f_pass = pass;
  ctl->f_refined = refined;
}

void forest_bind(hipStream_t s, Ctl* ctl, const ForestBufs& f, const uint32_t* gid, const uint32_t* base) {
  hipLaunchKernelGGL(k_forest_bind, dim3(1), dim3(kWave), 0, s, ctl, gid, base, (const double*)f.inv, f.dq,
                     (const uint8_t*)f.move, (const uint8_t*)f.pass, f.refined);
}

// Row lengths for aggregation: zero for the vertices of graphs that left the
// pass loop.  Their communities still become super-vertices (the lookup of
// their vertices goes through every level), but without entries: nothing of
// such a graph moves again, so its level graphs need no edges, and a forest
// whose graphs stop after different passes aggregates only the live ones.
__global__ __launch_bounds__(kBlock) void k_forest_live_len(uint32_t n, const uint32_t* gid, const uint8_t* pass,
                                                            const uint32_t* len, uint32_t* out) {
  GRID_STRIDE(v, n) out[v] = pass[gid[v]] ? len[v] : 0u;
}

void forest_live_len(hipStream_t s, uint32_t n, const uint32_t* gid, const uint8_t* pass, const uint32_t* len,
                     uint32_t* out) {
  if (n) hipLaunchKernelGGL(k_forest_live_len, dim3(grid_n(n)), dim3(kBlock), 0, s, n, gid, pass, len, out);
}

// Vertices of graphs without edges stay alone (as a graph without edges does).
__global__ __launch_bounds__(kBlock) void k_forest_isolate(uint32_t n, const uint32_t* gid, const uint8_t* pass,
                                                           uint32_t* C) {
  GRID_STRIDE(v, n) if (!pass[gid[v]]) C[v] = (uint32_t)v;
}

void forest_isolate(hipStream_t s, uint32_t n, const uint32_t* gid, const uint8_t* pass, uint32_t* C) {
  if (n) hipLaunchKernelGGL(k_forest_isolate, dim3(grid_n(n)), dim3(kBlock), 0, s, n, gid, pass, C);
}

}  // namespace lm
