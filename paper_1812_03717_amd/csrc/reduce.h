// Deterministic workgroup reductions: wavefront butterfly (shuffle-xor) then a
// fixed-order sum over the wavefronts.  Every thread receives the totals.
#pragma once

#include <hip/hip_runtime.h>

namespace sgw {

template <int NT, int M>
__device__ __forceinline__ void wg_sum(double *v, double *sh, double *out) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[m] += __shfl_xor(v[m], off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) sh[wid * M + m] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += sh[w * M + m];
    out[m] = r;
  }
  __syncthreads();
}

}  // namespace sgw
