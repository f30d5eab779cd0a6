// Modularity (Eq. 1) without any allocation: the scratch memory is one
// file-scope device array per GPU, so the call makes no hipMalloc / hipFree
// and uses no memory of the handle beyond its graph.
//
// Scratch layout (8-byte words):
//   [0, kNoAllocMaxN)                 Sigma_c, community weight sums
//   [kParts, kParts + 2 kNB)          per-block sigma and 2m partial sums
//   [kParts + 2 kNB, kParts + 4 kNB)  per-block (hi, lo) partial sums of Sigma_c^2
//   [kOut, kOut + 8)                  result: sigma, 2m, T_hi, T_lo, bad-label flag
// Every call on a GPU uses that GPU's array and leaves its contents behind;
// the call clears what must start at zero.  Calls that overlap on one GPU
// race on the array.
#include <mutex>

#include "noalloc.h"

namespace lm {

constexpr int kNB = 1024;  // blocks of the reductions
constexpr size_t kParts = kNoAllocMaxN;
constexpr size_t kOut = kParts + 4 * (size_t)kNB;
constexpr size_t kScratchWords = kOut + 8;

static __device__ __align__(256) unsigned long long scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// The array's device address on `device` (current), looked up once per device.
int scratch_of(int device, unsigned long long** out) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return -1;
    }
    g_ptr[device] = p;
  }
  *out = (unsigned long long*)g_ptr[device];
  return 0;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_na_clear(unsigned long long* ws, uint32_t n) {
  const size_t tot = (size_t)n;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < tot; i += (size_t)gridDim.x * kBlock) ws[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 8) ws[kOut + threadIdx.x] = 0;
}

// One wavefront per vertex: K_i (row sum) into Sigma_{C_i}, and the weight of
// the row's entries inside C_i; per block the sums of both.
__global__ __launch_bounds__(kBlock) void k_na_rows(Rows<uint32_t> g, uint32_t n, const uint32_t* C,
                                                    unsigned long long* ws) {
  __shared__ unsigned long long red[kBlock / kWave];
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned long long sig = 0, m2 = 0;
  for (uint64_t i = wave; i < n; i += nwaves) {
    const uint32_t c = C[i];
    if (c >= n) {
      if (lane == 0) ws[kOut + 4] = 1;
      continue;
    }
    const int64_t s0 = g.start[i];
    const uint32_t L = g.len[i];
    unsigned long long k = 0;
    for (uint32_t e = lane; e < L; e += kWave) {
      const uint32_t j = g.cols[s0 + e];
      const unsigned long long w = g.w[s0 + e];
      k += w;
      if (C[j] == c) sig += w;
    }
    k = group_sum<kWave>(k);
    if (lane == 0 && k) atomicAdd(&ws[c], k);
    if (lane == 0) m2 += k;
  }
  sig = block_sum(sig, red);
  m2 = block_sum(m2, red);
  if (threadIdx.x == 0) {
    ws[kParts + 2 * blockIdx.x] = sig;
    ws[kParts + 2 * blockIdx.x + 1] = m2;
  }
}

// Per block the 128-bit sum of Sigma_c^2.
__global__ __launch_bounds__(kBlock) void k_na_square(uint32_t n, unsigned long long* ws) {
  __shared__ unsigned long long rhi[kBlock], rlo[kBlock];
  unsigned long long hi = 0, lo = 0;
  for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += (uint64_t)gridDim.x * kBlock) {
    const unsigned long long x = ws[c];
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
    ws[kParts + 2 * kNB + 2 * blockIdx.x] = H;
    ws[kParts + 2 * kNB + 2 * blockIdx.x + 1] = L;
  }
}

__global__ void k_na_final(unsigned long long* ws) {
  if (threadIdx.x != 0) return;
  unsigned long long sig = 0, m2 = 0, H = 0, L = 0;
  for (int b = 0; b < kNB; ++b) {
    sig += ws[kParts + 2 * b];
    m2 += ws[kParts + 2 * b + 1];
    const unsigned long long lo = ws[kParts + 2 * kNB + 2 * b + 1];
    L += lo;
    H += ws[kParts + 2 * kNB + 2 * b] + (L < lo ? 1ull : 0ull);
  }
  ws[kOut + 0] = sig;
  ws[kOut + 1] = m2;
  ws[kOut + 2] = H;
  ws[kOut + 3] = L;
}

int noalloc_modularity(hipStream_t s, int device, Rows<uint32_t> g, uint32_t n, const uint32_t* C, double* q) {
  if (n > kNoAllocMaxN) return 1;
  unsigned long long* ws = nullptr;
  if (scratch_of(device, &ws) != 0) return -1;
  hipLaunchKernelGGL(k_na_clear, dim3(kNB), dim3(kBlock), 0, s, ws, n);
  if (n) {
    hipLaunchKernelGGL(k_na_rows, dim3(kNB), dim3(kBlock), 0, s, g, n, C, ws);
    hipLaunchKernelGGL(k_na_square, dim3(kNB), dim3(kBlock), 0, s, n, ws);
  }
  hipLaunchKernelGGL(k_na_final, dim3(1), dim3(64), 0, s, ws);
  unsigned long long h[5];
  if (hipMemcpyAsync(h, ws + kOut, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  if (h[4]) return 2;
  if (h[1] == 0) {
    *q = 0.0;
    return 0;
  }
  const unsigned __int128 T = ((unsigned __int128)h[2] << 64) | h[3];
  const double m2 = (double)h[1];
  const double first = (double)h[0] / m2;
  const double second = (double)T / (m2 * m2);
  *q = first - second;
  return 0;
}

}  // namespace lm
