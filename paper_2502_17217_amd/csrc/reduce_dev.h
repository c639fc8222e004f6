// Device helpers for the deterministic per-segment reductions (included by
// HIP sources only).  A workgroup is one tile of kFvBlock cells of one
// segment; tile sums use a fixed reduction over the 64 lanes of a
// wavefront (wave_sum) and a fixed order over the 4 wavefronts.
#pragma once

#include "internal.h"

namespace jfnk {

// x from lane (i permuted by the DPP pattern CTRL) of the wavefront, each
// 32-bit half moved by the VALU's data-parallel-primitive path (no LDS).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(b)), CTRL, 0xF, 0xF, false));
  const unsigned hi = unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(b >> 32)), CTRL, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) { return dpp_f64<CTRL>(x); }
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) { return dpp_f32<CTRL>(x); }

// Sum over each aligned group of G lanes (G a power of two up to 64, every
// lane active), the same bits in every lane of a group: DPP exchanges inside
// rows of 16 lanes (xor 1, xor 2, the half-row mirror, the row mirror), then
// shuffles across rows.
template <int G, class T>
__device__ __forceinline__ T group_sum(T x) {
  if constexpr (G >= 2) x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) x += dpp_move<0x141>(x);  // row_half_mirror
  if constexpr (G >= 16) x += dpp_move<0x140>(x); // row_mirror
  if constexpr (G >= 32) x += __shfl_xor(x, 16, G);
  if constexpr (G >= 64) x += __shfl_xor(x, 32, G);
  return x;
}

__device__ __forceinline__ double read_lane(double x, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), lane));
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// Sum over the 64 lanes of a wavefront (every lane active), the same bits in
// every lane: within each row of 16 lanes, partners exchange by DPP (xor 1,
// xor 2, the half-row mirror, the row mirror; a + b and b + a are the same
// number, so the lanes of a row agree), then the four row sums are read into
// scalar registers and added as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0x141>(x);  // row_half_mirror
  x += dpp_f64<0x140>(x);  // row_mirror
  return (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
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
