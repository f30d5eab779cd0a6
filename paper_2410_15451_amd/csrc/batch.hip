// Batch update kernels: G^{t-1} -> G^t with set semantics (Section 3.5) on
// the device slack CSR, the auxiliary-state update of Alg. 11, the community
// marking of Alg. 5 and the vertex marking of Alg. 2 / Alg. 3.
//
// Every undirected update becomes its two directed entries.  Entries are
// grouped by source row (counting by row, one segment per touched row) and
// sorted by destination inside each segment; validation then checks each
// entry against the sorted old row, and the merge writes each new sorted row
// to scratch before it is committed in place (or into the overflow area when
// the row outgrows its capacity).  Nothing is written to the graph before
// validation has passed, so a rejected batch leaves the graph unchanged.
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
// sort in LDS.  Long: one block, bottom-up merge sort through scratch.
// ---------------------------------------------------------------------------
__device__ inline void seg_swap(BatchBufs& b, uint64_t x, uint64_t y) {
  uint32_t t;
  t = b.seg_dst[x]; b.seg_dst[x] = b.seg_dst[y]; b.seg_dst[y] = t;
  t = b.seg_w[x]; b.seg_w[x] = b.seg_w[y]; b.seg_w[y] = t;
  t = b.seg_del[x]; b.seg_del[x] = b.seg_del[y]; b.seg_del[y] = t;
}

constexpr uint32_t kSortShort = 32, kSortLds = 2048;

__global__ __launch_bounds__(kBlock) void k_sort_short(uint64_t nt, BatchBufs b) {
  GRID_STRIDE(t, nt) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    if (s1 - s0 > kSortShort) continue;
    for (uint64_t i = s0 + 1; i < s1; ++i)
      for (uint64_t j = i; j > s0 && b.seg_dst[j - 1] > b.seg_dst[j]; --j) seg_swap(b, j - 1, j);
  }
}

__global__ __launch_bounds__(kBlock) void k_sort_lds(uint64_t nt, BatchBufs b) {
  __shared__ uint32_t key[kSortLds];
  __shared__ uint32_t idx[kSortLds];
  for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint32_t L = (uint32_t)(s1 - s0);
    if (L <= kSortShort || L > kSortLds) continue;
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
__global__ __launch_bounds__(kBlock) void k_sort_long(uint64_t nt, BatchBufs b) {
  for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint64_t L = s1 - s0;
    if (L <= kSortLds) continue;
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
__device__ inline int64_t row_find(const uint32_t* cols, int64_t s0, uint32_t L, uint32_t key) {
  uint32_t lo = 0, hi = L;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cols[s0 + mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < L && cols[s0 + lo] == key) ? s0 + lo : -1;
}

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

__global__ __launch_bounds__(kBlock) void k_validate(uint64_t ne, Rows<uint32_t> g, BatchBufs b, Ctl* ctl) {
  unsigned int err = 0;
  GRID_STRIDE(q, ne) {
    const uint32_t t = b.seg_id[q];
    const uint32_t d = b.seg_dst[q];
    if (q + 1 < b.seg_off[t + 1] && b.seg_dst[q + 1] == d) err |= kErrDup;
    const uint32_t r = b.seg_src[q];
    const int64_t pos = row_find(g.cols, g.start[r], g.len[r], d);
    if (b.seg_del[q]) {
      if (pos < 0)
        err |= kErrAbsent;
      else
        b.seg_w[q] = g.w[pos];
    } else if (pos >= 0) {
      err |= kErrPresent;
    }
  }
  if (err) atomicOr(&ctl->error, err);
}

// ---------------------------------------------------------------------------
// Merge planning, merge and commit
// ---------------------------------------------------------------------------
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
    if (nl > cap[r]) need += nl + (nl >> 2) + 4;
  }
  if (need) atomicAdd(&ctl->overflow_need, need);
}

// Merge, one thread per entry: every old entry and every inserted entry
// computes its position in the merged sorted row directly.  Rows are found by
// binary search over per-row offsets, so long rows spread over all threads.
__device__ inline uint64_t row_of(const uint64_t* off, uint64_t nt, uint64_t x) {
  // largest t < nt with off[t] <= x
  uint64_t lo = 0, hi = nt;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Entry-parallel walk over rows: the entries [0, tot) of consecutive rows
// (row t owns [off[t], off[t + 1])) are cut into one contiguous range per
// block.  A block finds the row of its first entry by binary search, then
// stages kRowWin row offsets at a time in LDS; each thread finds its row in
// that window, and the next tile starts from the row of the tile's last
// entry.  Rows beyond the window (only when a tile spans more rows than the
// window holds) are found by binary search.  f(t, x) runs once per entry x.
constexpr uint32_t kRowWin = 512;

__device__ inline uint64_t row_in(const uint64_t* off, uint64_t lo, uint64_t hi, uint64_t x) {
  // largest t in [lo, hi) with off[t] <= x, given off[lo] <= x
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename F>
__device__ inline void block_rows_for_each(const uint64_t* off, uint64_t nt, uint64_t tot, F f) {
  __shared__ uint64_t woff[kRowWin];
  __shared__ uint64_t t0s, tnext;
  const uint64_t per = (tot + gridDim.x - 1) / gridDim.x;
  const uint64_t xb = (uint64_t)blockIdx.x * per, xe = min(tot, xb + per);
  if (xb >= xe) return;  // block-uniform
  if (threadIdx.x == 0) t0s = row_in(off, 0, nt, xb);
  __syncthreads();
  for (uint64_t x0 = xb; x0 < xe; x0 += kBlock) {
    const uint64_t t0 = t0s;
    const uint64_t w = min((uint64_t)kRowWin, nt - t0);
    for (uint32_t k = threadIdx.x; k < w; k += kBlock) woff[k] = off[t0 + k];
    __syncthreads();
    const uint64_t x = x0 + threadIdx.x;
    const uint64_t xl = min(x0 + kBlock, xe) - 1;
    if (x <= xl) {
      uint64_t t;
      if (w == kRowWin && x >= woff[w - 1]) {
        t = row_in(off, t0 + w - 1, nt, x);
      } else {
        uint64_t lo = 0, hi = w;
        while (hi - lo > 1) {
          const uint64_t mid = (lo + hi) >> 1;
          if (woff[mid] <= x)
            lo = mid;
          else
            hi = mid;
        }
        t = t0 + lo;
      }
      f(t, x);
      if (x == xl) tnext = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) t0s = tnext;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_old_len(uint64_t nt, const uint32_t* len, BatchBufs b) {
  GRID_STRIDE(t, nt) b.old_len[t] = len[b.touched[t]];
}

__device__ inline void merge_old_entry(uint64_t t, uint64_t x, const Rows<uint32_t>& g, const BatchBufs& b) {
  const uint32_t r = b.touched[t];
  const uint32_t p = (uint32_t)(x - b.old_off[t]);
  const uint64_t s0 = b.seg_off[t];
  const uint32_t L = (uint32_t)(b.seg_off[t + 1] - s0);
  const int64_t r0 = g.start[r];
  const uint32_t y = g.cols[r0 + p];
  uint32_t lo = 0, hi = L;  // first segment entry with dst >= y
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (b.seg_dst[s0 + mid] < y)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < L && b.seg_dst[s0 + lo] == y) return;  // deleted (insertions of present pairs were rejected)
  const uint64_t dels = b.seg_pre[s0 + lo] - b.seg_pre[s0];
  const uint64_t inss = lo - dels;
  const uint64_t pos = b.out_off[t] + p - dels + inss;
  b.mcols[pos] = y;
  b.mw[pos] = g.w[r0 + p];
}

__global__ __launch_bounds__(kBlock) void k_merge_old(uint64_t nt, const uint64_t* total_old, Rows<uint32_t> g,
                                                      BatchBufs b) {
  block_rows_for_each(b.old_off, nt, *total_old, [&](uint64_t t, uint64_t x) { merge_old_entry(t, x, g, b); });
}

__global__ __launch_bounds__(kBlock) void k_merge_ins(uint64_t ne, Rows<uint32_t> g, BatchBufs b) {
  GRID_STRIDE(q, ne) {
    if (b.seg_del[q]) continue;
    const uint32_t t = b.seg_id[q];
    const uint32_t r = b.touched[t];
    const uint64_t s0 = b.seg_off[t];
    const uint32_t y = b.seg_dst[q];
    const uint32_t lb = row_lower_bound(g.cols, g.start[r], g.len[r], y);
    const uint64_t dels = b.seg_pre[q] - b.seg_pre[s0];
    const uint64_t inss = (q - s0) - dels;
    const uint64_t pos = b.out_off[t] + lb - dels + inss;
    b.mcols[pos] = y;
    b.mw[pos] = b.seg_w[q];
  }
}

// Per touched row: destination of the merged row (in place, or a new span in
// the overflow area when it outgrew its capacity) and the new length.
__global__ __launch_bounds__(kBlock) void k_commit_rows(uint64_t nt, int64_t* start, uint32_t* len, uint32_t* cap,
                                                        BatchBufs b, unsigned long long* edge_top) {
  GRID_STRIDE(t, nt) {
    const uint32_t r = b.touched[t];
    const uint32_t nl = b.new_len[t];
    if (nl > cap[r]) {
      const uint32_t nc = nl + (nl >> 2) + 4;
      start[r] = (int64_t)atomicAdd(edge_top, (unsigned long long)nc);
      cap[r] = nc;
    }
    b.dest[t] = (uint64_t)start[r];
    len[r] = nl;
  }
}

__global__ __launch_bounds__(kBlock) void k_commit_copy(uint64_t nt, const uint64_t* total_new, uint32_t* cols,
                                                        uint32_t* w, BatchBufs b) {
  block_rows_for_each(b.out_off, nt, *total_new, [&](uint64_t t, uint64_t x) {
    const uint64_t d = b.dest[t] + (x - b.out_off[t]);
    cols[d] = b.mcols[x];
    w[d] = b.mw[x];
  });
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
  hipLaunchKernelGGL(k_sort_short, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, b);
  hipLaunchKernelGGL(k_sort_lds, dim3(grid_n(nt, 1, 1024)), dim3(kBlock), 0, s, nt, b);
  hipLaunchKernelGGL(k_sort_long, dim3(grid_n(nt, 1, 256)), dim3(kBlock), 0, s, nt, b);
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

int batch_merge(hipStream_t s, int64_t* start, uint32_t* len, uint32_t* cap, uint32_t* cols, uint32_t* w,
                uint64_t n_touched, BatchBufs& b, unsigned long long* edge_top, uint64_t edge_cap, Ctl* ctl) {
  const uint64_t nt = n_touched;
  if (nt == 0) return 0;
  hipLaunchKernelGGL(k_new_len, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, len, cap, b, ctl);
  exclusive_scan_u32(s, b.new_len, b.out_off, nt, b.total, b.scan_tmp);
  hipLaunchKernelGGL(k_old_len, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, len, b);
  exclusive_scan_u32(s, b.old_len, b.old_off, nt, b.total + 1, b.scan_tmp);
  unsigned long long* hv = (unsigned long long*)pinned_stage(32);  // need, top, merged total, old total
  if (!hv) return -100;
  (void)hipMemcpyAsync(&hv[0], &ctl->overflow_need, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(&hv[1], edge_top, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(&hv[2], b.total, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -100;
  if (hv[1] + hv[0] > edge_cap || hv[2] > b.mcap) return 1;
  Rows<uint32_t> g{start, len, cols, w};
  if (hv[3]) hipLaunchKernelGGL(k_merge_old, dim3(grid_n(hv[3])), dim3(kBlock), 0, s, nt, b.total + 1, g, b);
  const uint64_t nent = b.n_entries;
  if (nent) hipLaunchKernelGGL(k_merge_ins, dim3(grid_n(nent)), dim3(kBlock), 0, s, nent, g, b);
  hipLaunchKernelGGL(k_commit_rows, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, start, len, cap, b, edge_top);
  if (hv[2]) hipLaunchKernelGGL(k_commit_copy, dim3(grid_n(hv[2])), dim3(kBlock), 0, s, nt, b.total, cols, w, b);
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
    if (b.seg_del[q]) dS[c] = 1;
    const long long sg = S[c];
    if (ratio_exceeds((unsigned long long)dSig[c], (unsigned long long)(sg > 0 ? sg : 0), num, den)) dR[c] = 1;
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
    dC[Cprev[j]] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_ds_ins(uint64_t nt, BatchBufs b, const uint32_t* Cprev, const int64_t* K,
                                                   const int64_t* S, double inv_m, double inv_2m2, uint8_t* dV,
                                                   uint8_t* dE, uint8_t* dC) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t t = wave; t < nt; t += nwaves) {
    const uint64_t s0 = b.seg_off[t], s1 = b.seg_off[t + 1];
    const uint32_t i = b.touched[t];
    const uint32_t d = Cprev[i];
    double bdq = -INFINITY;
    uint32_t bc = kNone;
    for (uint64_t qb = s0; qb < s1; qb += kWave) {
      const uint64_t q = qb + lane;
      if (q < s1 && !b.seg_del[q]) {
        const uint32_t c = Cprev[b.seg_dst[q]];
        bool first = c != d;
        for (uint64_t p = s0; first && p < q; ++p)
          if (!b.seg_del[p] && Cprev[b.seg_dst[p]] == c) first = false;
        if (first) {
          long long h = 0;
          for (uint64_t p = s0; p < s1; ++p)
            if (!b.seg_del[p] && Cprev[b.seg_dst[p]] == c) h += b.seg_w[p];
          const double dq = delta_q(h, 0, K[i], S[c], S[d], inv_m, inv_2m2);
          if (better(dq, c, bdq, bc)) {
            bdq = dq;
            bc = c;
          }
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
