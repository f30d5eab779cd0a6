// Level-0 slack CSR helpers of the runtime.
#pragma once

#include "kernels.h"

namespace lm {

// Row i occupies cols / w [start[i], start[i] + len[i]) inside a reserved
// span of cap[i] entries, and owns a second span of the same size at alt[i]
// that a batch merge writes the updated row into; rows that outgrow their
// spans move to a fresh pair in the overflow area above the bump pointer.
struct SlackCsr {
  int64_t* start = nullptr;
  int64_t* alt = nullptr;
  uint32_t* len = nullptr;
  uint32_t* cap = nullptr;
  uint32_t* cols = nullptr;
  uint32_t* w = nullptr;
  uint64_t edge_cap = 0;  // entries allocated in cols / w
};

unsigned int csr_check(hipStream_t s, uint32_t n, uint64_t nnz, const int64_t* offs, const uint32_t* cols,
                       const uint32_t* w, unsigned int* err_dev);
// per-row length and capacity from the input offsets; off_tmp receives the
// exclusive scan of the capacities and *total_dev their sum (each row takes
// two spans, so the layout needs twice that)
void caps_from_csr(hipStream_t s, uint32_t n, const int64_t* offs, float slack, SlackCsr& g, uint64_t* off_tmp,
                   void* scan_tmp, uint64_t* total_dev);
void rebuild_caps(hipStream_t s, uint32_t n, const uint32_t* len, const uint32_t* reserve, float slack, uint32_t* cap,
                  uint64_t* off_tmp, void* scan_tmp, uint64_t* total_dev);
// rows into the pairs of spans laid out by the capacity scan off (row i at
// 2 off[i], its spare span at 2 off[i] + cap[i])
void copy_rows(hipStream_t s, uint32_t n, const int64_t* src_start, const uint32_t* len, const uint32_t* cap,
               const uint32_t* src_cols, const uint32_t* src_w, const uint64_t* off, uint32_t* dst_cols,
               uint32_t* dst_w, int64_t* new_start, int64_t* new_alt);
void reserve_touched(hipStream_t s, uint64_t nt, const uint32_t* touched, const uint32_t* new_len, uint32_t* reserve);
void sum_i64(hipStream_t s, const int64_t* x, uint64_t n, unsigned long long* out_dev);
void label_check(hipStream_t s, const uint32_t* C, const uint32_t* Cref, uint32_t n, unsigned int* flags_dev);
void dsig_out(hipStream_t s, uint32_t n, const uint8_t* matched, const int64_t* dSig, int64_t* out);

}  // namespace lm
