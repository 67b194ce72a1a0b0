// Wave- and block-level scan helpers for 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vgpr {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive prefix sum over a block of NT threads (NT a multiple of 64, at
// most 1024). `smem` holds NT / 64 + 1 words. Returns the exclusive prefix and
// writes the block total to *total. Contains barriers: every thread calls it.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* smem, uint32_t* total) {
  constexpr int NW = NT / 64;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  uint32_t inc = wave_inclusive_sum(v);
  if (lane == 63) smem[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < NW; ++w) {
      uint32_t t = smem[w];
      smem[w] = run;
      run += t;
    }
    smem[NW] = run;
  }
  __syncthreads();
  uint32_t r = smem[wave] + inc - v;
  *total = smem[NW];
  __syncthreads();
  return r;
}

}  // namespace vgpr
