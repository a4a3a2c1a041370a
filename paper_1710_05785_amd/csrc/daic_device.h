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

// The out-edges of rows [0, n) of a 32-bit CSR offset array, four rows to a
// wave: a group of 16 lanes per row with the row's edges strided over it
// (most rows of power-law graphs hold a few dozen edges, which a whole wave
// per row would leave mostly idle); a row of more than 1,024 edges is taken
// afterwards by the whole wave, eight edges per lane at a time with their
// loads issued together. The rows are dealt to the groups in a scrambled
// order (row = x times an odd constant modulo the next power of two above
// n, a bijection; logical indices that land at or beyond n are skipped):
// on RMAT graphs the heavy rows recur at id strides that are powers of two,
// so a plain strided deal gave one wave millions of edges of heavy rows
// (4.3 M of RMAT-24's 125 M) while most waves had none. Each edge e of row
// j is handled in two calls: load(j, e) only reads memory and returns what
// the edge needs, then use(j, e, loaded) computes, may store, and returns
// the edge's contribution; with REDUCE, done(j, sum) is called once per row
// (by one lane) with the row's sum of contributions.
template <bool REDUCE, typename Load, typename Use, typename Done>
__device__ __forceinline__ void rows_by_groups(const uint32_t* row, uint64_t n, const Load& load, const Use& use,
                                               const Done& done) {
  constexpr uint32_t kGroup = 16, kHeavy = 1024, kIlp = 8;
  constexpr uint64_t kMix = 0x9E3779B97F4A7C15ull;  // odd: x -> x kMix is a bijection modulo 2^k
  using T = decltype(load(uint64_t{0}, uint32_t{0}));
  const uint32_t lane = lane_id(), sub = lane & (kGroup - 1), grp = lane / kGroup;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t span = n <= 1 ? n : 1ull << (64 - __clzll((long long)(n - 1)));  // next power of two >= n
  for (uint64_t x0 = wave * (64 / kGroup); x0 < span; x0 += nwaves * (64 / kGroup)) {
    const uint64_t x = x0 + grp;
    const uint64_t j = (x * kMix) & (span - 1);
    const bool valid = x < span && j < n;
    uint32_t b = 0, e1 = 0;
    if (valid) {
      b = row[j];
      e1 = row[j + 1];
    }
    const bool heavy = e1 - b > kHeavy;
    double acc = 0.0;
    if (!heavy)
      for (uint32_t e = b + sub; e < e1; e += kGroup) acc += use(j, e, load(j, e));
    if constexpr (REDUCE) {
#pragma unroll
      for (uint32_t d = kGroup / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
      if (valid && !heavy && sub == 0) done(j, acc);
    }
    // heavy rows of this wave, one at a time by all 64 lanes
    uint64_t hm = __ballot(heavy && sub == 0);
    while (hm) {
      const uint32_t src = (uint32_t)__ffsll((unsigned long long)hm) - 1;
      hm &= hm - 1;
      const uint32_t hb = __shfl(b, src, 64), he = __shfl(e1, src, 64);
      const uint64_t hj = __shfl(j, src, 64);
      double h = 0.0;
      for (uint32_t e = hb + lane; e < he; e += 64 * kIlp) {
        T v[kIlp];
#pragma unroll
        for (uint32_t k = 0; k < kIlp; ++k)
          if (e + 64 * k < he) v[k] = load(hj, e + 64 * k);
#pragma unroll
        for (uint32_t k = 0; k < kIlp; ++k)
          if (e + 64 * k < he) h += use(hj, e + 64 * k, v[k]);
      }
      if constexpr (REDUCE) {
        h = wave_sum(h);
        if (lane == 0) done(hj, h);
      }
    }
  }
}

}  // namespace daic
