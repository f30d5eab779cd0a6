// Device slack CSR of the level-0 graph: input validation, layout with
// per-row spare capacity (so batch insertions usually land in place), and
// rebuilds when the overflow area runs out.  Plus small reductions used by
// the runtime.
#include "graph.h"

namespace lm {

static int grid_n(uint64_t n, int per_block = kBlock, int cap = 8192) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap) b = cap;
  return (int)b;
}

#define GRID_STRIDE(i, n) \
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < (uint64_t)(n); i += (uint64_t)gridDim.x * kBlock)

// Input CSR checks, one wavefront per row: IDs in range, no self-loops, w > 0,
// strictly increasing columns (sorted, no duplicates), and the reverse entry
// present with the same weight.
__global__ __launch_bounds__(kBlock) void k_csr_check(uint32_t n, const int64_t* offs, const uint32_t* cols,
                                                      const uint32_t* w, unsigned int* err) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned int e_out = 0;
  for (uint64_t i = wave; i < n; i += nwaves) {
    const int64_t a = offs[i], b = offs[i + 1];
    if (b < a) {
      e_out |= 16;
      continue;
    }
    for (int64_t e = a + lane; e < b; e += kWave) {
      const uint32_t j = cols[e];
      if (j >= n || j == (uint32_t)i || w[e] == 0) {
        e_out |= 1;
        continue;
      }
      if (e + 1 < b && cols[e + 1] <= j) e_out |= 2;
      // reverse entry (binary search in row j)
      int64_t lo = offs[j], hi = offs[j + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cols[mid] < (uint32_t)i)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo >= offs[j + 1] || cols[lo] != (uint32_t)i || w[lo] != w[e]) e_out |= 4;
    }
  }
  if (e_out) atomicOr(err, e_out);
}

__global__ __launch_bounds__(kBlock) void k_offs_check(uint32_t n, const int64_t* offs, uint64_t nnz,
                                                       unsigned int* err) {
  GRID_STRIDE(i, n) {
    if (offs[i + 1] < offs[i]) atomicOr(err, 16u);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (offs[0] != 0 || (uint64_t)offs[n] != nnz)) atomicOr(err, 16u);
}

// capacity of a row holding `len` entries (at least `reserve`)
__device__ inline uint32_t row_capacity(uint32_t len, uint32_t reserve, float slack) {
  const uint32_t base = len > reserve ? len : reserve;
  return base + (uint32_t)ceilf((float)base * slack) + 2u;
}

__global__ __launch_bounds__(kBlock) void k_caps_from_offs(uint32_t n, const int64_t* offs, float slack,
                                                           uint32_t* len, uint32_t* cap) {
  GRID_STRIDE(i, n) {
    const uint32_t L = (uint32_t)(offs[i + 1] - offs[i]);
    len[i] = L;
    cap[i] = row_capacity(L, 0, slack);
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_rows(uint32_t n, const int64_t* src_start, const uint32_t* len,
                                                      const uint32_t* src_cols, const uint32_t* src_w,
                                                      const uint64_t* off, uint32_t* dst_cols, uint32_t* dst_w) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t i = wave; i < n; i += nwaves) {
    const int64_t a = src_start[i];
    const uint64_t d = 2 * off[i];
    const uint32_t L = len[i];
    for (uint32_t e = lane; e < L; e += kWave) {
      dst_cols[d + e] = src_cols[a + e];
      dst_w[d + e] = src_w[a + e];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_start_from(uint32_t n, const uint64_t* off, const uint32_t* cap,
                                                       int64_t* start, int64_t* alt) {
  GRID_STRIDE(i, n) {
    start[i] = (int64_t)(2 * off[i]);
    alt[i] = (int64_t)(2 * off[i] + cap[i]);
  }
}

__global__ __launch_bounds__(kBlock) void k_caps_rebuild(uint32_t n, const uint32_t* len, const uint32_t* reserve,
                                                         float slack, uint32_t* cap) {
  GRID_STRIDE(i, n) cap[i] = row_capacity(len[i], reserve ? reserve[i] : 0u, slack);
}

__global__ __launch_bounds__(kBlock) void k_sum_i64(const int64_t* x, uint64_t n, unsigned long long* out) {
  __shared__ unsigned long long red[kBlock / kWave];
  unsigned long long s = 0;
  GRID_STRIDE(i, n) s += (unsigned long long)x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0 && s) atomicAdd(out, s);
}

__global__ __launch_bounds__(kBlock) void k_label_check(const uint32_t* C, const uint32_t* Cref, uint32_t n,
                                                        unsigned int* flags) {
  unsigned int f = 0;
  GRID_STRIDE(i, n) {
    if (C[i] >= n) f |= 1;
    if (Cref && C[i] != Cref[i]) f |= 2;
  }
  if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kBlock) void k_dsig_out(uint32_t n, const uint8_t* matched, const int64_t* dSig,
                                                     int64_t* out) {
  GRID_STRIDE(c, n) out[c] = matched[c] ? dSig[c] : 0;
}

__global__ __launch_bounds__(kBlock) void k_reserve_touched(uint64_t nt, const uint32_t* touched,
                                                            const uint32_t* new_len, uint32_t* reserve) {
  GRID_STRIDE(t, nt) reserve[touched[t]] = new_len[t];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
unsigned int csr_check(hipStream_t s, uint32_t n, uint64_t nnz, const int64_t* offs, const uint32_t* cols,
                       const uint32_t* w, unsigned int* err_dev) {
  unsigned int err = 0;
  (void)hipMemcpyAsync(err_dev, &err, sizeof(err), hipMemcpyHostToDevice, s);
  if (n) hipLaunchKernelGGL(k_offs_check, dim3(grid_n(n)), dim3(kBlock), 0, s, n, offs, nnz, err_dev);
  if (hipMemcpyAsync(&err, err_dev, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return 0x80000000u;
  if (err) return err;
  if (n) hipLaunchKernelGGL(k_csr_check, dim3(grid_n(n, kBlock / kWave, 16384)), dim3(kBlock), 0, s, n, offs, cols, w,
                            err_dev);
  if (hipMemcpyAsync(&err, err_dev, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return 0x80000000u;
  return err;
}

void caps_from_csr(hipStream_t s, uint32_t n, const int64_t* offs, float slack, SlackCsr& g, uint64_t* off_tmp,
                   void* scan_tmp, uint64_t* total_dev) {
  if (n) hipLaunchKernelGGL(k_caps_from_offs, dim3(grid_n(n)), dim3(kBlock), 0, s, n, offs, slack, g.len, g.cap);
  exclusive_scan_u32(s, g.cap, off_tmp, n, total_dev, scan_tmp);
}

void rebuild_caps(hipStream_t s, uint32_t n, const uint32_t* len, const uint32_t* reserve, float slack, uint32_t* cap,
                  uint64_t* off_tmp, void* scan_tmp, uint64_t* total_dev) {
  if (n) hipLaunchKernelGGL(k_caps_rebuild, dim3(grid_n(n)), dim3(kBlock), 0, s, n, len, reserve, slack, cap);
  exclusive_scan_u32(s, cap, off_tmp, n, total_dev, scan_tmp);
}

void copy_rows(hipStream_t s, uint32_t n, const int64_t* src_start, const uint32_t* len, const uint32_t* cap,
               const uint32_t* src_cols, const uint32_t* src_w, const uint64_t* off, uint32_t* dst_cols,
               uint32_t* dst_w, int64_t* new_start, int64_t* new_alt) {
  if (!n) return;
  hipLaunchKernelGGL(k_copy_rows, dim3(grid_n(n, kBlock / kWave, 16384)), dim3(kBlock), 0, s, n, src_start, len,
                     src_cols, src_w, off, dst_cols, dst_w);
  hipLaunchKernelGGL(k_start_from, dim3(grid_n(n)), dim3(kBlock), 0, s, n, off, cap, new_start, new_alt);
}

void reserve_touched(hipStream_t s, uint64_t nt, const uint32_t* touched, const uint32_t* new_len, uint32_t* reserve) {
  if (nt) hipLaunchKernelGGL(k_reserve_touched, dim3(grid_n(nt)), dim3(kBlock), 0, s, nt, touched, new_len, reserve);
}

void sum_i64(hipStream_t s, const int64_t* x, uint64_t n, unsigned long long* out_dev) {
  fill_u64(s, (uint64_t*)out_dev, 0, 1);
  if (n) hipLaunchKernelGGL(k_sum_i64, dim3(grid_n(n, kBlock, 1024)), dim3(kBlock), 0, s, x, n, out_dev);
}

void label_check(hipStream_t s, const uint32_t* C, const uint32_t* Cref, uint32_t n, unsigned int* flags_dev) {
  fill_u32(s, flags_dev, 0, 1);
  if (n) hipLaunchKernelGGL(k_label_check, dim3(grid_n(n)), dim3(kBlock), 0, s, C, Cref, n, flags_dev);
}

void dsig_out(hipStream_t s, uint32_t n, const uint8_t* matched, const int64_t* dSig, int64_t* out) {
  if (n) hipLaunchKernelGGL(k_dsig_out, dim3(grid_n(n)), dim3(kBlock), 0, s, n, matched, dSig, out);
}

}  // namespace lm
