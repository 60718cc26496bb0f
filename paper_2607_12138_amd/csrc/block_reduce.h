// Deterministic per-block, per-column partial sums.
#pragma once

#include <hip/hip_runtime.h>

namespace bras {

// sh[threadIdx.x] holds this thread's contribution to column
// (blockIdx.x * blockDim.x + threadIdx.x) % R.  Writes the block's R column
// sums to out[blockIdx.x * R + c] in a fixed order.  Must be called by every
// thread of the block; blockDim.x must be a power of two.
__device__ inline void block_partials(double* sh, int R, double* out) {
  __syncthreads();
  const int bs = blockDim.x;
  if ((bs % R) == 0) {
    for (int off = bs / 2; off >= R; off >>= 1) {
      if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if ((int)threadIdx.x < R) out[(int64_t)blockIdx.x * R + threadIdx.x] = sh[threadIdx.x];
  } else if ((int)threadIdx.x < R) {
    const int64_t base = (int64_t)blockIdx.x * bs;
    double s = 0.0;
    for (int u = 0; u < bs; ++u)
      if ((int)((base + u) % R) == (int)threadIdx.x) s += sh[u];
    out[(int64_t)blockIdx.x * R + threadIdx.x] = s;
  }
}

}  // namespace bras
