// Batch update kernels: G^{t-1} -> G^t with set semantics (Section 3.5) on
// the device slack CSR, the auxiliary-state update of Alg. 11, the community
// marking of Alg. 5 and the vertex marking of Alg. 2 / Alg. 3.
//
// Every undirected update becomes its two directed entries.  Entries are
// grouped by source row (counting by row, one segment per touched row) and
// sorted by destination inside each segment; validation then checks each
// entry against the sorted old row.  Every row owns two spans of its
// capacity: the merge writes the new sorted row into the spare span (or a
// fresh pair of spans in the overflow area when the row outgrows its
// capacity) and the spans swap roles afterwards, so no merged row is copied
// back.  Nothing is written to the graph before validation has passed, so a
// rejected batch leaves the graph unchanged.
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

enum : unsigned int { kErrId = 1, kErrDup = 2, kErrPresent = 4, kErrAbsent = 8 };

// ---------------------------------------------------------------------------
// Expansion and grouping
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_expand(const uint32_t* del, uint64_t n_del, const uint32_t* ins,
                                                   uint64_t n_ins, uint32_t n, BatchBufs b, Ctl* ctl) {
  GRID_STRIDE(k, n_del + n_ins) {
    const bool is_del = k < n_del;
    const uint32_t u = is_del ? del[2 * k] : ins[3 * (k - n_del)];
    const uint32_t v = is_del ? del[2 * k + 1] : ins[3 * (k - n_del) + 1];
    const uint32_t w = is_del ? 0u : ins[3 * (k - n_del) + 2];
    if (u >= n || v >= n || u == v || (!is_del && w == 0)) {
      atomicOr(&ctl->error, kErrId);
      b.src[2 * k] = kNone;
      b.src[2 * k + 1] = kNone;
      continue;
    }
    for (int h = 0; h < 2; ++h) {
      const uint64_t e = 2 * k + h;
      const uint32_t a = h ? v : u, c = h ? u : v;
      const uint32_t sl = atomicAdd(&b.row_cnt[a], 1u);
      if (sl == 0) list_push(b.touched, &ctl->touched, a);
      b.slot[e] = sl;
      b.src[e] = a;
      b.dst[e] = c;
      b.w[e] = w;
      b.is_del[e] = is_del ? 1u : 0u;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_seg_setup(uint64_t nt, BatchBufs b) {
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    b.seg_cnt[t] = b.row_cnt[r];
    b.row_idx[r] = (uint32_t)t;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(uint64_t ne, BatchBufs b) {
  GRID_STRIDE(e, ne) {
    const uint32_t a = b.src[e];
    if (a == kNone) continue;
    const uint32_t t = b.row_idx[a];
    const uint64_t pos = b.seg_off[t] + b.slot[e];
    b.seg_src[pos] = a;
    b.seg_dst[pos] = b.dst[e];
    b.seg_w[pos] = b.w[e];
    b.seg_del[pos] = b.is_del[e];
    b.seg_id[pos] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_row_cnt_clear(uint64_t nt, BatchBufs b) {
  GRID_STRIDE(t, nt) b.row_cnt[b.touched[t]] = 0;
}

// ---------------------------------------------------------------------------
// Sorting each segment by destination (src is equal inside a segment).
// Short segments: one thread, insertion sort.  Medium: one block, bitonic
// sort in LDS.  Long: one block, bottom-up merge sort through scratch.  The
// short-segment pass lists the medium and long segments, so the block sorts
// visit only those.
// ---------------------------------------------------------------------------
__device__ inline void seg_swap(BatchBufs& b, uint64_t x, uint64_t y) {
  uint32_t t;
  t = b.seg_dst[x]; b.seg_dst[x] = b.seg_dst[y]; b.seg_dst[y] = t;
  t = b.seg_w[x]; b.seg_w[x] = b.seg_w[y]; b.seg_w[y] = t;
  t = b.seg_del[x]; b.seg_del[x] = b.seg_del[y]; b.seg_del[y] = t;
}

constexpr uint32_t kSortShort = 8, kSortLds = 2048;

__global__ __launch_bounds__(kBlock) void k_sort_short(uint64_t nt, BatchBufs b, Ctl* ctl) {
  GRID_STRIDE(t, nt) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint64_t L = s1 - s0;
    const uint32_t which = L > kSortLds ? 1u : (L > kSortShort ? 0u : kNone);
    wave_append(which, (uint32_t)t, [&](uint32_t k, uint32_t*& l, unsigned int*& c) {
      l = k ? b.sort_long : b.sort_mid;
      c = &ctl->sort_count[k];
    });
    if (which != kNone) continue;
    for (uint64_t i = s0 + 1; i < s1; ++i)
      for (uint64_t j = i; j > s0 && b.seg_dst[j - 1] > b.seg_dst[j]; --j) seg_swap(b, j - 1, j);
  }
}

__global__ __launch_bounds__(kBlock) void k_sort_lds(BatchBufs b, const Ctl* ctl) {
  __shared__ uint32_t key[kSortLds];
  __shared__ uint32_t idx[kSortLds];
  const unsigned int cnt = ctl->sort_count[0];
  for (unsigned int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const uint32_t t = b.sort_mid[it];
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint32_t L = (uint32_t)(s1 - s0);
    uint32_t P = 1;
    while (P < L) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
      key[i] = i < L ? b.seg_dst[s0 + i] : kNone;
      idx[i] = i;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
          const uint32_t l = i ^ j;
          if (l > i) {
            const bool up = (i & k) == 0;
            const bool gt = key[i] > key[l] || (key[i] == key[l] && idx[i] > idx[l]);
            if (gt == up) {
              uint32_t x = key[i]; key[i] = key[l]; key[l] = x;
              x = idx[i]; idx[i] = idx[l]; idx[l] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    // permute the payload through registers of this block (at most kSortLds / kBlock each)
    constexpr int kPer = kSortLds / kBlock;
    uint32_t pw[kPer], pd[kPer];
    int cnt = 0;
    for (uint32_t i = threadIdx.x; i < L; i += kBlock, ++cnt) {
      pw[cnt] = b.seg_w[s0 + idx[i]];
      pd[cnt] = b.seg_del[s0 + idx[i]];
    }
    __syncthreads();
    cnt = 0;
    for (uint32_t i = threadIdx.x; i < L; i += kBlock, ++cnt) {
      b.seg_dst[s0 + i] = key[i];
      b.seg_w[s0 + i] = pw[cnt];
      b.seg_del[s0 + i] = pd[cnt];
    }
    __syncthreads();
  }
}

// One block per long segment: merge runs of width 1, 2, 4, ... between the
// segment and its scratch copy; each thread merges one pair of runs.
__global__ __launch_bounds__(kBlock) void k_sort_long(BatchBufs b, const Ctl* ctl) {
  const unsigned int cnt = ctl->sort_count[1];
  for (unsigned int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const uint32_t t = b.sort_long[it];
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint64_t L = s1 - s0;
    uint32_t *ad = b.seg_dst + s0, *aw = b.seg_w + s0, *ax = b.seg_del + s0;
    uint32_t *bd = b.tmp_dst + s0, *bw = b.tmp_w + s0, *bx = b.tmp_del + s0;
    for (uint64_t width = 1; width < L; width <<= 1) {
      for (uint64_t lo = (uint64_t)threadIdx.x * 2 * width; lo < L; lo += (uint64_t)kBlock * 2 * width) {
        const uint64_t mid = lo + width < L ? lo + width : L;
        const uint64_t hi = lo + 2 * width < L ? lo + 2 * width : L;
        uint64_t i = lo, j = mid, o = lo;
        while (i < mid || j < hi) {
          const bool take_i = j >= hi || (i < mid && ad[i] <= ad[j]);
          const uint64_t s = take_i ? i++ : j++;
          bd[o] = ad[s];
          bw[o] = aw[s];
          bx[o] = ax[s];
          ++o;
        }
      }
      __syncthreads();
      uint32_t* x;
      x = ad; ad = bd; bd = x;
      x = aw; aw = bw; bw = x;
      x = ax; ax = bx; bx = x;
    }
    if (ad != b.seg_dst + s0) {
      for (uint64_t i = threadIdx.x; i < L; i += kBlock) {
        b.seg_dst[s0 + i] = ad[i];
        b.seg_w[s0 + i] = aw[i];
        b.seg_del[s0 + i] = ax[i];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Validation against G^{t-1}: no pair twice, deletions present (their old
// weight is recorded), insertions absent.
// ---------------------------------------------------------------------------
__device__ inline uint32_t row_lower_bound(const uint32_t* cols, int64_t s0, uint32_t L, uint32_t key) {
  uint32_t lo = 0, hi = L;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cols[s0 + mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Also records each entry's lower bound in its old row, which places it (and
// the old entries around it) in the merged row.
__global__ __launch_bounds__(kBlock) void k_validate(uint64_t ne, Rows<uint32_t> g, BatchBufs b, Ctl* ctl) {
  unsigned int err = 0;
  GRID_STRIDE(q, ne) {
    const uint32_t t = b.seg_id[q];
    const uint32_t d = b.seg_dst[q];
    if (q + 1 < b.seg_off[t + 1] && b.seg_dst[q + 1] == d) err |= kErrDup;
    const uint32_t r = b.seg_src[q];
    const int64_t s0 = g.start[r];
    const uint32_t L = g.len[r];
    const uint32_t lb = row_lower_bound(g.cols, s0, L, d);
    const bool present = lb < L && g.cols[s0 + lb] == d;
    b.seg_lb[q] = lb;
    if (b.seg_del[q]) {
      if (!present)
        err |= kErrAbsent;
      else
        b.seg_w[q] = g.w[s0 + lb];
    } else if (present) {
      err |= kErrPresent;
    }
  }
  if (err) atomicOr(&ctl->error, err);
}

// ---------------------------------------------------------------------------
// Merge planning, merge and commit
// ---------------------------------------------------------------------------
// capacity of each span of a row that outgrew its spans
__device__ inline uint32_t grown_cap(uint32_t nl) { return nl + (nl >> 2) + 4; }

__global__ __launch_bounds__(kBlock) void k_new_len(uint64_t nt, const uint32_t* len, const uint32_t* cap,
                                                    BatchBufs b, Ctl* ctl) {
  unsigned long long need = 0;
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint64_t dels = b.seg_pre[s1] - b.seg_pre[s0];
    const uint64_t inss = (s1 - s0) - dels;
    const uint32_t nl = (uint32_t)(len[r] - dels + inss);
    b.new_len[t] = nl;
    if (nl > cap[r]) need += 2 * (uint64_t)grown_cap(nl);
  }
  if (need) atomicAdd(&ctl->overflow_need, need);
}

// largest t in [lo, hi) with off[t] <= x, given off[lo] <= x
__device__ inline uint64_t row_in(const uint64_t* off, uint64_t lo, uint64_t hi, uint64_t x) {
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Destination span of each touched row: its spare span, or a fresh pair of
// spans above the bump pointer when the merged row outgrows the capacity.
__global__ __launch_bounds__(kBlock) void k_plan_rows(uint64_t nt, const int64_t* alt, const uint32_t* cap,
                                                      BatchBufs b, unsigned long long* edge_top) {
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    const uint32_t nl = b.new_len[t];
    if (nl > cap[r])
      b.dest[t] = (uint64_t)atomicAdd(edge_top, 2ull * grown_cap(nl));
    else
      b.dest[t] = (uint64_t)alt[r];
  }
}

// Runs of old entries.  Between two consecutive segment entries of a row the
// old entries keep their order and all move by the same amount: the
// insertions before them minus the deletions before them.  Run q + t ends at
// segment entry q (of touched row t); run seg_off[t + 1] + t is the row's
// tail.  A deleted entry is the old entry at its lower bound, so the next run
// starts just after it.
__device__ inline void run_plan(uint64_t i, uint64_t s0, uint64_t q, uint32_t end, int64_t src0, uint64_t dst0,
                                BatchBufs& b) {
  uint32_t a = 0;
  if (q > s0) a = b.seg_lb[q - 1] + (b.seg_del[q - 1] ? 1u : 0u);
  const uint64_t dels = b.seg_pre[q] - b.seg_pre[s0];
  const uint64_t inss = (q - s0) - dels;
  b.run_len[i] = end - a;
  b.run_src[i] = src0 + a;
  b.run_dst[i] = (int64_t)(dst0 + a + inss - dels);
}

__global__ __launch_bounds__(kBlock) void k_runs_seg(uint64_t ne, const int64_t* start, BatchBufs b) {
  GRID_STRIDE(q, ne) {
    const uint32_t t = b.seg_id[q];
    run_plan(q + t, b.seg_off[t], q, b.seg_lb[q], start[b.touched[t]], b.dest[t], b);
  }
}

__global__ __launch_bounds__(kBlock) void k_runs_tail(uint64_t nt, const int64_t* start, const uint32_t* len,
                                                      BatchBufs b) {
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    const uint64_t s1 = b.seg_off[t + 1];
    run_plan(s1 + t, b.seg_off[t], s1, len[r], start[r], b.dest[t], b);
  }
}

// Entry-parallel copy of the runs.  Each block takes one contiguous range of
// the entries; it keeps a window of kRunWin runs (offsets, sources and
// destinations) in LDS and loads the next window only when its entries run
// past the current one.  A thread finds the run of its entry in the window:
// the run of its previous entry if that still holds it (long runs), else by
// binary search.
constexpr uint32_t kRunWin = 512, kCopyU = 4, kCopyTile = kCopyU * kBlock;
// blocks of the run copy (the entry count is known on the device only)
constexpr int kCopyGrid = 2048;

__global__ __launch_bounds__(kBlock) void k_copy_runs(uint64_t nruns, const uint64_t* total, uint32_t* cols,
                                                      uint32_t* w, BatchBufs b) {
  __shared__ uint64_t woff[kRunWin + 1];
  __shared__ int64_t wsrc[kRunWin], wdst[kRunWin];
  __shared__ uint64_t sbase;
  const uint64_t tot = *total;
  const uint64_t per = (tot + gridDim.x - 1) / gridDim.x;
  const uint64_t xb = (uint64_t)blockIdx.x * per, xe = min(tot, xb + per);
  if (xb >= xe) return;  // block-uniform
  uint64_t base = 0;
  uint32_t wn = 0, j = 0;
  bool have = false;
  for (uint64_t x0 = xb; x0 < xe;) {
    if (!have || x0 >= woff[wn]) {
      // the run holding x0 lies at or after the end of the current window
      if (threadIdx.x == 0) sbase = row_in(b.run_off, have ? base + wn : 0, nruns, x0);
      __syncthreads();
      base = sbase;
      wn = (uint32_t)min((uint64_t)kRunWin, nruns - base);
      for (uint32_t k = threadIdx.x; k <= wn; k += kBlock) {
        const uint64_t t = base + k;
        woff[k] = t < nruns ? b.run_off[t] : tot;
        if (k < wn) {
          wsrc[k] = b.run_src[t];
          wdst[k] = b.run_dst[t];
        }
      }
      __syncthreads();
      have = true;
      j = 0;
    }
    const uint64_t x1 = min(min(x0 + kCopyTile, woff[wn]), xe);
    // all loads of the tile first, then the stores: sources and destinations
    // lie in different spans, so the loads need not wait for earlier stores
    uint32_t vc[kCopyU], vw[kCopyU];
    int64_t vd[kCopyU];
#pragma unroll
    for (uint32_t u = 0; u < kCopyU; ++u) {
      const uint64_t x = x0 + threadIdx.x + (uint64_t)u * kBlock;
      vd[u] = -1;
      if (x < x1) {
        if (woff[j + 1] <= x) {  // largest run j < wn with woff[j] <= x
          uint32_t lo = j + 1, hi = wn;
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (woff[mid] <= x)
              lo = mid;
            else
              hi = mid;
          }
          j = lo;
        }
        const uint64_t k = x - woff[j];
        const int64_t src = wsrc[j] + (int64_t)k;
        vd[u] = wdst[j] + (int64_t)k;
        vc[u] = cols[src];
        vw[u] = w[src];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kCopyU; ++u) {
      if (vd[u] < 0) continue;
      cols[vd[u]] = vc[u];
      w[vd[u]] = vw[u];
    }
    x0 = x1;
  }
}

// Inserted entries land at their lower bound, shifted like the run before.
__global__ __launch_bounds__(kBlock) void k_merge_ins(uint64_t ne, uint32_t* cols, uint32_t* w, BatchBufs b) {
  GRID_STRIDE(q, ne) {
    if (b.seg_del[q]) continue;
    const uint32_t t = b.seg_id[q];
    const uint64_t s0 = b.seg_off[t];
    const uint64_t dels = b.seg_pre[q] - b.seg_pre[s0];
    const uint64_t inss = (q - s0) - dels;
    const uint64_t pos = b.dest[t] + b.seg_lb[q] + inss - dels;
    cols[pos] = b.seg_dst[q];
    w[pos] = b.seg_w[q];
  }
}

// The spans swap roles (or the row moves to its fresh pair) and the new
// length is published.
__global__ __launch_bounds__(kBlock) void k_commit_rows(uint64_t nt, int64_t* start, int64_t* alt, uint32_t* len,
                                                        uint32_t* cap, BatchBufs b) {
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    const uint32_t nl = b.new_len[t];
    const int64_t d = (int64_t)b.dest[t];
    if (nl > cap[r]) {
      const uint32_t nc = grown_cap(nl);
      alt[r] = d + nc;
      cap[r] = nc;
    } else {
      alt[r] = start[r];
    }
    start[r] = d;
    len[r] = nl;
  }
}

// ---------------------------------------------------------------------------
// Host side of the batch pipeline
// ---------------------------------------------------------------------------
int batch_prepare(hipStream_t s, uint32_t n, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                  BatchBufs& b, Ctl* ctl, uint64_t* n_touched_host) {
  const uint64_t nb = n_del + n_ins;
  const uint64_t ne = 2 * nb;
  if (nb)
    hipLaunchKernelGGL(k_expand, dim3(grid_n(nb)), dim3(kBlock), 0, s, del, n_del, ins, n_ins, n, b, ctl);
  unsigned int* hv = (unsigned int*)pinned_stage(8);
  if (!hv) return -100;
  (void)hipMemcpyAsync(hv, &ctl->error, 2 * sizeof(unsigned int), hipMemcpyDeviceToHost, s);  // error, touched
  if (hipStreamSynchronize(s) != hipSuccess) return -100;
  const uint64_t nt = hv[1];
  *n_touched_host = nt;
  if (hv[0]) {
    if (nt) hipLaunchKernelGGL(k_row_cnt_clear, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, b);
    return (int)hv[0];
  }
  if (nt == 0) return 0;
  hipLaunchKernelGGL(k_seg_setup, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, b);
  exclusive_scan_u32(s, b.seg_cnt, b.seg_off, nt, b.total, b.scan_tmp);
  (void)hipMemcpyAsync(b.seg_off + nt, b.total, sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  hipLaunchKernelGGL(k_scatter, dim3(grid_n(ne)), dim3(kBlock), 0, s, ne, b);
  hipLaunchKernelGGL(k_row_cnt_clear, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, b);
  hipLaunchKernelGGL(k_sort_short, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, b, ctl);
  hipLaunchKernelGGL(k_sort_lds, dim3(grid_n(nt, 1, 1024)), dim3(kBlock), 0, s, b, ctl);
  hipLaunchKernelGGL(k_sort_long, dim3(grid_n(nt, 1, 256)), dim3(kBlock), 0, s, b, ctl);
  // prefix counts of deletions inside segments (for the merge positions)
  exclusive_scan_u32(s, b.seg_del, b.seg_pre, ne, b.total, b.scan_tmp);
  (void)hipMemcpyAsync(b.seg_pre + ne, b.total, sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  return 0;
}

int batch_validate(hipStream_t s, Rows<uint32_t> g, uint32_t n, uint64_t n_entries, uint64_t n_touched, BatchBufs& b,
                   Ctl* ctl) {
  (void)n;
  (void)n_touched;
  if (n_entries)
    hipLaunchKernelGGL(k_validate, dim3(grid_n(n_entries)), dim3(kBlock), 0, s, n_entries, g, b, ctl);
  unsigned int* err = (unsigned int*)pinned_stage(4);
  if (!err) return -100;
  (void)hipMemcpyAsync(err, &ctl->error, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -100;
  return (int)*err;
}

int batch_merge(hipStream_t s, int64_t* start, int64_t* alt, uint32_t* len, uint32_t* cap, uint32_t* cols,
                uint32_t* w, uint64_t n_touched, BatchBufs& b, unsigned long long* edge_top, uint64_t edge_cap,
                Ctl* ctl) {
  const uint64_t nt = n_touched;
  if (nt == 0) return 0;
  hipLaunchKernelGGL(k_new_len, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, len, cap, b, ctl);
  unsigned long long* hv = (unsigned long long*)pinned_stage(16);  // overflow need, bump pointer
  if (!hv) return -100;
  (void)hipMemcpyAsync(&hv[0], &ctl->overflow_need, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(&hv[1], edge_top, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -100;
  if (hv[1] + hv[0] > edge_cap) return 1;
  const uint64_t ne = b.n_entries, nruns = ne + nt;
  hipLaunchKernelGGL(k_plan_rows, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, alt, cap, b, edge_top);
  if (ne) hipLaunchKernelGGL(k_runs_seg, dim3(grid_n(ne)), dim3(kBlock), 0, s, ne, start, b);
  hipLaunchKernelGGL(k_runs_tail, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, start, len, b);
  exclusive_scan_u32(s, b.run_len, b.run_off, nruns, b.total, b.scan_tmp);
  hipLaunchKernelGGL(k_copy_runs, dim3(kCopyGrid), dim3(kBlock), 0, s, nruns, b.total, cols, w, b);
  if (ne) hipLaunchKernelGGL(k_merge_ins, dim3(grid_n(ne)), dim3(kBlock), 0, s, ne, cols, w, b);
  hipLaunchKernelGGL(k_commit_rows, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, start, alt, len, cap, b);
  return 0;
}

// ---------------------------------------------------------------------------
// Alg. 11: K and Sigma by the old memberships; DeltaSigma counts deletions and
// insertions alike.  Integer atomics, so the order of entries is irrelevant.
// ---------------------------------------------------------------------------
// A block sums a tile of kAuxTile entries per community in LDS first: a few
// large communities collect most entries, and atomics on one address are
// serialised device-wide, so per-wavefront sums still queued hundreds of
// microseconds on Sigma of the largest communities.
constexpr uint32_t kAuxTile = 1024, kAuxSlots = 2048;

__global__ __launch_bounds__(kBlock) void k_aux_update(uint64_t ne, BatchBufs b, const uint32_t* Cprev, int64_t* K,
                                                       int64_t* S, int64_t* dSig) {
  __shared__ uint32_t tk[kAuxSlots];
  __shared__ unsigned long long ts[kAuxSlots], tw[kAuxSlots];
  for (uint32_t sl = threadIdx.x; sl < kAuxSlots; sl += kBlock) {
    tk[sl] = kNone;
    ts[sl] = 0;
    tw[sl] = 0;
  }
  __syncthreads();
  for (uint64_t base = (uint64_t)blockIdx.x * kAuxTile; base < ne; base += (uint64_t)gridDim.x * kAuxTile) {
    for (uint64_t q = base + threadIdx.x; q < base + kAuxTile; q += kBlock) {
      uint32_t i = kNone, c = kNone;
      long long w = 0, sgn = 0;
      if (q < ne) {
        i = b.seg_src[q];
        c = Cprev[i];
        w = (long long)b.seg_w[q];
        sgn = b.seg_del[q] ? -w : w;
      }
      // entries are grouped by source: one atomic per vertex and wavefront
      wave_add_by_key(i, sgn, (long long*)K);
      if (c == kNone) continue;
      uint32_t h = slot_hash(c, kAuxSlots - 1);
      while (true) {
        const uint32_t k = __atomic_load_n(&tk[h], __ATOMIC_RELAXED);
        if (k == c) break;
        if (k == kNone) {
          const uint32_t o = atomicCAS(&tk[h], kNone, c);
          if (o == kNone || o == c) break;
        }
        h = (h + 1) & (kAuxSlots - 1);
      }
      atomicAdd(&ts[h], (unsigned long long)sgn);
      atomicAdd(&tw[h], (unsigned long long)w);
    }
    __syncthreads();
    for (uint32_t sl = threadIdx.x; sl < kAuxSlots; sl += kBlock) {
      const uint32_t c = tk[sl];
      if (c == kNone) continue;
      atomicAdd((unsigned long long*)&S[c], ts[sl]);
      atomicAdd((unsigned long long*)&dSig[c], tw[sl]);
      tk[sl] = kNone;
      ts[sl] = 0;
      tw[sl] = 0;
    }
    __syncthreads();
  }
}

void launch_aux_update(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev, int64_t* K,
                       int64_t* S, int64_t* dSig) {
  if (n_entries)
    hipLaunchKernelGGL(k_aux_update, dim3(grid_n(n_entries, kAuxTile, 2048)), dim3(kBlock), 0, s, n_entries, b, Cprev,
                       K, S, dSig);
}

// Alg. 5 (dynamic branch): split flags for intra-community deletions; refine
// flags for intra-community updates with DeltaSigma / Sigma > num / den
// (compared exactly as den * DeltaSigma > num * Sigma); then the cumulative
// change of every refine-marked community restarts from zero.
__device__ inline bool ratio_exceeds(unsigned long long dsig, unsigned long long sig, uint32_t num, uint32_t den) {
  const unsigned long long alo = dsig * den, ahi = __umul64hi(dsig, (unsigned long long)den);
  const unsigned long long blo = sig * num, bhi = __umul64hi(sig, (unsigned long long)num);
  return ahi > bhi || (ahi == bhi && alo > blo);
}

__global__ __launch_bounds__(kBlock) void k_mark_comm(uint64_t ne, BatchBufs b, const uint32_t* Cprev,
                                                      const int64_t* S, const int64_t* dSig, uint32_t num,
                                                      uint32_t den, uint8_t* dS, uint8_t* dR) {
  GRID_STRIDE(q, ne) {
    const uint32_t c = Cprev[b.seg_src[q]], d = Cprev[b.seg_dst[q]];
    if (c != d) continue;
    if (b.seg_del[q]) raise_flag(dS, c);
    const long long sg = S[c];
    if (ratio_exceeds((unsigned long long)dSig[c], (unsigned long long)(sg > 0 ? sg : 0), num, den)) raise_flag(dR, c);
  }
}

__global__ __launch_bounds__(kBlock) void k_mark_reset(uint64_t ne, BatchBufs b, const uint32_t* Cprev,
                                                       const uint8_t* dR, int64_t* dSig) {
  GRID_STRIDE(q, ne) {
    const uint32_t c = Cprev[b.seg_src[q]];
    if (dR[c]) dSig[c] = 0;
  }
}

void launch_mark_communities(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev,
                             const int64_t* S, int64_t* dSig, uint32_t num, uint32_t den, uint8_t* dS, uint8_t* dR) {
  if (!n_entries) return;
  hipLaunchKernelGGL(k_mark_comm, dim3(grid_n(n_entries)), dim3(kBlock), 0, s, n_entries, b, Cprev, S, dSig, num, den,
                     dS, dR);
  hipLaunchKernelGGL(k_mark_reset, dim3(grid_n(n_entries)), dim3(kBlock), 0, s, n_entries, b, Cprev, dR, dSig);
}

// Alg. 3: endpoints of intra-community deletions and inter-community
// insertions are affected; they form the first unprocessed list directly.
__global__ __launch_bounds__(kBlock) void k_mark_df(uint64_t ne, BatchBufs b, const uint32_t* Cprev, uint32_t* list,
                                                    unsigned int* count, uint32_t* mark, uint32_t stamp) {
  GRID_STRIDE(q, ne) {
    const uint32_t i = b.seg_src[q];
    const bool same = Cprev[i] == Cprev[b.seg_dst[q]];
    const bool push = (b.seg_del[q] ? same : !same) && atomicExch(&mark[i], stamp) != stamp;
    wave_append(push ? 0u : kNone, i, [&](uint32_t, uint32_t*& l, unsigned int*& c) {
      l = list;
      c = count;
    });
  }
}

void launch_mark_df(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev, uint32_t* list,
                    unsigned int* count, uint32_t* mark, uint32_t stamp) {
  if (n_entries)
    hipLaunchKernelGGL(k_mark_df, dim3(grid_n(n_entries)), dim3(kBlock), 0, s, n_entries, b, Cprev, list, count, mark,
                       stamp);
}

// Alg. 2: intra-community deletions mark the source, its neighbours and the
// community; each source of inter-community insertions marks itself, its
// neighbours and the community c* with the largest Eq. 2 gain over the
// communities of its inserted neighbours (K_{i->c} = inserted weight into c,
// K_{i->d} = 0, ties to the lowest ID).
__global__ __launch_bounds__(kBlock) void k_ds_del(uint64_t ne, BatchBufs b, const uint32_t* Cprev, uint8_t* dV,
                                                   uint8_t* dE, uint8_t* dC) {
  GRID_STRIDE(q, ne) {
    if (!b.seg_del[q]) continue;
    const uint32_t i = b.seg_src[q], j = b.seg_dst[q];
    if (Cprev[i] != Cprev[j]) continue;
    dV[i] = 1;
    dE[i] = 1;
    raise_flag(dC, Cprev[j]);
  }
}

// Short segments (at most kDsShort entries): one wavefront, one lane per entry;
// a lane sums the inserted weight of its community over the segment if it is
// the community's first insertion there.
constexpr uint32_t kDsShort = 64;
__global__ __launch_bounds__(kBlock) void k_ds_ins(uint64_t nt, BatchBufs b, const uint32_t* Cprev, const int64_t* K,
                                                   const int64_t* S, double inv_m, double inv_2m2, uint8_t* dV,
                                                   uint8_t* dE, uint8_t* dC) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t t = wave; t < nt; t += nwaves) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    if (s1 - s0 > kDsShort) continue;  // wavefront-uniform: k_ds_ins_long
    const uint32_t i = b.touched[t];
    const uint32_t d = Cprev[i];
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    const uint64_t q = s0 + lane;
    if (q < s1 && !b.seg_del[q]) {
      const uint32_t c = Cprev[b.seg_dst[q]];
      bool first = c != d;
      for (uint64_t p = s0; first && p < q; ++p)
        if (!b.seg_del[p] && Cprev[b.seg_dst[p]] == c) first = false;
      if (first) {
        long long h = 0;
        for (uint64_t p = s0; p < s1; ++p)
          if (!b.seg_del[p] && Cprev[b.seg_dst[p]] == c) h += b.seg_w[p];
        const double dq = b.f_gid ? delta_q(h, 0, K[i], S[c], S[d], b.f_inv[2 * b.f_gid[i]], b.f_inv[2 * b.f_gid[i] + 1])
                                  : delta_q(h, 0, K[i], S[c], S[d], inv_m, inv_2m2);
        if (better(dq, c, bdq, bc)) {
          bdq = dq;
          bc = c;
        }
      }
    }
    group_best<kWave>(bdq, bc);
    if (lane == 0 && bc != kNone) {
      dV[i] = 1;
      dE[i] = 1;
      dC[bc] = 1;
    }
  }
}

// Long segments: one block per segment sums the inserted weight per community
// in an LDS table, in 2^k partitions of the communities by hash (about
// kDsPart insertions each); a partition whose distinct communities overflow
// the table restarts the segment with twice the partitions.  The best
// community is the same whatever the partitioning (largest gain, then lowest
// ID), so the result equals the pairwise form's.
constexpr uint32_t kDsSlots = 2048, kDsPart = 1024;
__global__ __launch_bounds__(kBlock) void k_ds_ins_long(uint64_t nt, BatchBufs b, const uint32_t* Cprev,
                                                        const int64_t* K, const int64_t* S, double inv_m,
                                                        double inv_2m2, uint8_t* dV, uint8_t* dE, uint8_t* dC) {
  __shared__ uint32_t tk[kDsSlots];
  __shared__ unsigned long long tv[kDsSlots];
  __shared__ unsigned long long red[kBlock / kWave];
  __shared__ double rdq[kBlock / kWave];
  __shared__ uint32_t rc[kBlock / kWave];
  __shared__ unsigned int full;
  for (uint32_t sl = threadIdx.x; sl < kDsSlots; sl += kBlock) {
    tk[sl] = kNone;
    tv[sl] = 0;
  }
  __syncthreads();
  for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    if (s1 - s0 <= kDsShort) continue;  // block-uniform
    const uint32_t i = b.touched[t];
    const uint32_t d = Cprev[i];
    const double im = b.f_gid ? b.f_inv[2 * b.f_gid[i]] : inv_m;
    const double i2 = b.f_gid ? b.f_inv[2 * b.f_gid[i] + 1] : inv_2m2;
    unsigned long long nins = 0;
    for (uint64_t q = s0 + threadIdx.x; q < s1; q += kBlock) nins += b.seg_del[q] ? 0u : 1u;
    nins = block_sum(nins, red);
    uint32_t P = 1;
    while ((uint64_t)P * kDsPart < nins) P <<= 1;
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    for (uint32_t part = 0; part < P;) {
      if (threadIdx.x == 0) full = 0;
      __syncthreads();
      for (uint64_t q = s0 + threadIdx.x; q < s1; q += kBlock) {
        if (b.seg_del[q]) continue;
        const uint32_t c = Cprev[b.seg_dst[q]];
        if (c == d || (fmix32(c) & (P - 1)) != part) continue;
        // salted home slots: the partition already fixes the low bits of fmix32(c)
        if (!table_add_bounded(tk, tv, kDsSlots - 1, c, (unsigned long long)b.seg_w[q], kRowSalt)) full = 1;
      }
      __syncthreads();
      const bool ok = full == 0;
      for (uint32_t sl = threadIdx.x; sl < kDsSlots; sl += kBlock) {
        const uint32_t c = tk[sl];
        if (c == kNone) continue;
        if (ok) {
          const double dq = delta_q((int64_t)tv[sl], 0, K[i], S[c], S[d], im, i2);
          if (better(dq, c, bdq, bc)) {
            bdq = dq;
            bc = c;
          }
        }
        tk[sl] = kNone;
        tv[sl] = 0;
      }
      __syncthreads();
      if (ok) {
        ++part;
      } else {  // too many communities in one partition: start over, finer
        P <<= 1;
        part = 0;
        bdq = -INFINITY;
        bc = kNone;
      }
    }
    block_best(bdq, bc, rdq, rc);
    if (threadIdx.x == 0 && bc != kNone) {
      dV[i] = 1;
      dE[i] = 1;
      dC[bc] = 1;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_ds_neighbours(uint64_t nt, BatchBufs b, Rows<uint32_t> g,
                                                          const uint8_t* dE, uint8_t* dV) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t t = wave; t < nt; t += nwaves) {
    const uint32_t i = b.touched[t];
    if (!dE[i]) continue;
    const int64_t s0 = g.start[i];
    const uint32_t L = g.len[i];
    for (uint32_t e = lane; e < L; e += kWave) dV[g.cols[s0 + e]] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_ds_comm(uint32_t n, const uint32_t* Cprev, const uint8_t* dC, uint8_t* dV) {
  GRID_STRIDE(i, n) if (dC[Cprev[i]]) dV[i] = 1;
}

void launch_mark_ds(hipStream_t s, const BatchBufs& b, uint64_t n_entries, uint64_t n_touched, Rows<uint32_t> g,
                    uint32_t n, const uint32_t* Cprev, const int64_t* K, const int64_t* S, double inv_m,
                    double inv_2m2, uint8_t* dV, uint8_t* dE, uint8_t* dC) {
  if (n_entries) {
    hipLaunchKernelGGL(k_ds_del, dim3(grid_n(n_entries)), dim3(kBlock), 0, s, n_entries, b, Cprev, dV, dE, dC);
    hipLaunchKernelGGL(k_ds_ins, dim3(grid_n(n_touched, kBlock / kWave)), dim3(kBlock), 0, s, n_touched, b, Cprev, K,
                       S, inv_m, inv_2m2, dV, dE, dC);
    hipLaunchKernelGGL(k_ds_ins_long, dim3(grid_n(n_touched, 1, 2048)), dim3(kBlock), 0, s, n_touched, b, Cprev, K, S,
                       inv_m, inv_2m2, dV, dE, dC);
    hipLaunchKernelGGL(k_ds_neighbours, dim3(grid_n(n_touched, kBlock / kWave)), dim3(kBlock), 0, s, n_touched, b, g,
                       dE, dV);
  }
  if (n) hipLaunchKernelGGL(k_ds_comm, dim3(grid_n(n)), dim3(kBlock), 0, s, n, Cprev, dC, dV);
}

// Flag array -> vertex list (order irrelevant), stamping each listed vertex.
constexpr int kFlagsU = 8;  // flags per thread of a tile
__global__ __launch_bounds__(kBlock) void k_flags_to_list(const uint8_t* flags, uint32_t n, uint32_t* list,
                                                          unsigned int* count, uint32_t* mark, uint32_t stamp) {
  __shared__ unsigned int scnt[1], sbase[1];
  if (threadIdx.x == 0) scnt[0] = 0;
  __syncthreads();
  constexpr uint32_t tile = kBlock * kFlagsU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < n; base += (uint64_t)gridDim.x * tile) {
    uint32_t key[kFlagsU], val[kFlagsU];
#pragma unroll
    for (int u = 0; u < kFlagsU; ++u) {
      const uint64_t i = base + u * kBlock + threadIdx.x;
      const bool on = i < n && flags[i];
      if (on) mark[i] = stamp;
      key[u] = on ? 0u : kNone;
      val[u] = (uint32_t)i;
    }
    tile_append<kFlagsU>(key, val, 1, scnt, sbase, [&](uint32_t, uint32_t*& l, unsigned int*& c) {
      l = list;
      c = count;
    });
  }
}

void launch_flags_to_list(hipStream_t s, const uint8_t* flags, uint32_t n, uint32_t* list, unsigned int* count,
                          uint32_t* mark, uint32_t stamp) {
  if (n)
    hipLaunchKernelGGL(k_flags_to_list, dim3(grid_n(n, kBlock * kFlagsU)), dim3(kBlock), 0, s, flags, n, list, count,
                       mark, stamp);
}

}  // namespace lm
