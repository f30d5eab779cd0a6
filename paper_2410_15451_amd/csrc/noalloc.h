// Modularity without allocation (scratch in a file-scope device array).
#pragma once
#include "kernels.h"

namespace lm {

// Largest vertex count the scratch array holds (its Sigma_c part: 32 MiB).
constexpr uint32_t kNoAllocMaxN = 1u << 22;

// Eq. 1 of membership C (device, uint32[n]) on g, ordered on s; device is the
// current GPU.  Returns 0, 1 if n > kNoAllocMaxN, 2 if a label is >= n, -1 on
// a HIP error.
int noalloc_modularity(hipStream_t s, int device, Rows<uint32_t> g, uint32_t n, const uint32_t* C, double* q);

}  // namespace lm
