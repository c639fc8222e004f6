// Device helpers for the deterministic per-segment reductions (included by
// HIP sources only).  A workgroup is one tile of kFvBlock cells of one
// segment; tile sums use a fixed butterfly over the 64 lanes of a wavefront
// and a fixed order over the 4 wavefronts.
#pragma once

#include "internal.h"

namespace jfnk {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum over a 256-thread workgroup; valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* sh) {
  x = wave_sum(x);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// True (in every thread of the workgroup) for the last of a segment's n
// tiles to arrive; the partial sums the other tiles wrote before arriving
// are then visible.  The last tile resets the counter, so it is zero again
// between launches.
__device__ __forceinline__ bool last_tile_of_segment(int32_t* counter, int n) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    last = atomicAdd(counter, 1) == n - 1;
    if (last) *counter = 0;
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}


}  // namespace jfnk
