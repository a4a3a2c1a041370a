// Wavefront and block primitives for gfx950 (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace daic {

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// ---------------------------------------------------------------------------
// Wave and block scans (64-lane waves, blocks of 256 threads = 4 waves).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Exclusive block scan of up to three counters at once; returns the block
// totals through tot[]. Every thread of the block must call it.
template <int NV>
__device__ __forceinline__ void block_excl_scan(uint32_t (&x)[NV], uint32_t (&tot)[NV]) {
  __shared__ uint32_t s_w[4][NV];
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t incl[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    incl[i] = wave_incl_scan(x[i]);
    if (lane == 63) s_w[wave][i] = incl[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    uint32_t off = 0, t = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t c = s_w[w][i];
      off += (w < (int)wave) ? c : 0u;
      t += c;
    }
    x[i] = off + incl[i] - x[i];
    tot[i] = t;
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T block_sum256(T x) {
  __shared__ T s_w[4];
  x = wave_sum(x);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  T t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  __syncthreads();
  return t;
}

// Sum over a block of NW waves (every thread must call it).
template <int NW, typename T>
__device__ __forceinline__ T block_sum_waves(T x) {
  __shared__ T s_w[NW];
  x = wave_sum(x);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  T t = s_w[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) t += s_w[w];
  __syncthreads();
  return t;
}

}  // namespace daic
