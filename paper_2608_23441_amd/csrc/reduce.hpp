// Workgroup reductions in FP64 with a fixed summation order (results do not
// depend on timing): wavefront butterflies of cross-lane exchanges, then one
// LDS step across the wavefronts.
#pragma once
#include <hip/hip_runtime.h>

namespace ipfb {

// Sum over the 64 lanes of a wavefront: a butterfly of cross-lane exchanges.
// Each step adds the same two partials on both lanes of a pair (in swapped
// order, which IEEE addition does not distinguish), so every lane ends with
// the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a workgroup of NT threads: wavefront sums, then the NT/64 of them
// in wavefront order, so the result does not depend on timing. sh holds at
// least NT/64 doubles. Every thread returns the total.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += sh[w];
  __syncthreads();  // the caller may write sh again
  return t;
}

}  // namespace ipfb
