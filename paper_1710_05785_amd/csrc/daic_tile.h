// Device code of the tiled fused dense round (layout in daic_internal.h).
//
// Round r of Eq. sync over every pending vertex, as k_pull_fused computes it
// (pull of round r's message bases, then for every target the fold of its
// previous delta into v, the new delta kept in dv and the base of the new
// delta published for round r + 1), with the in-edges walked partition by
// partition in source order:
//   k_tile_pull  : a workgroup per tile. Each run of in-edges from one source
//                  into the partition gathers that source's base once; every
//                  in-edge adds it (times its weight) into an FP64 LDS
//                  accumulator of its target (128 KiB: one 1024-thread
//                  workgroup per CU). A partition of one tile is then
//                  finished by the same workgroup; a tile of a larger one
//                  stores its accumulators as a partial-sum slot.
//   k_tile_finish: targets of partitions with several tiles: their slots added
//                  in tile order (FP64), then finished.
//   k_tile_total : the round's residual and counters from the per-workgroup
//                  partials, in a fixed order, and the stop rule.
// The kernels only store: no fences, tickets or global atomics.
//
// The same kernels run the dense rounds of the other selection rules
// (FUSED = false): the round's claim has already folded the selected deltas
// and published their bases (0 for the others) into the first buffer, so a
// target only adds its sum into dv; the totals then also set the pending
// count and the direction of the next round, as k_pull_finish does.
#pragma once

#include "daic_device.h"
#include "daic_internal.h"
#include "daic_kernels.h"

namespace daic {

struct TileArgs {
  const uint16_t* tloc;
  const uint32_t* psrc;
  const uint32_t* segpair;
  const void* wtile;          // S[m] weights in tile order (EDGE_SCALE)
  const uint32_t* tile_part;
  const uint32_t* tile_e;
  const uint32_t* tile_slot;
  const uint32_t* tile_order;  // launch order: a workgroup takes tiles tile_order[workgroup], [workgroup + grid], ...
  const uint32_t* split_part;
  const uint32_t* split_slot;
  double* pbuf;               // [n_slots][tw] partial sums of the tiles of split partitions (SlotT<ST>)
  uint64_t m, n_tiles, n_split, n_seg;
  uint32_t tw;                // partition width (a power of two, 1,024..kTileT)
  double* tpart_r;            // per-workgroup partials of k_tile_pull: |new delta|,
  uint64_t* tpart_a;          //   vertex updates,
  uint64_t* tpart_p;          //   messages
  double* spart_r;            // the same per workgroup of k_tile_finish
  uint64_t* spart_a;
  uint64_t* spart_p;
};

// FP64 LDS atomics run at about twice the rate of FP32 ones here, so the
// accumulators are FP64 whatever the state type.
// Workgroup shapes: partitions wider than kNarrowTW take 1024 threads and
// LDS for kTileT accumulators (one workgroup per CU); narrower ones (graphs
// below about 2 M vertices) 256 threads and LDS for kNarrowTW accumulators,
// so several workgroups share a CU and hide each other's latency (kNarrowTW
// and the resident workgroups per CU are in daic_internal.h).
template <uint32_t NT>
struct TileShape {
  static constexpr uint32_t threads = NT, waves = NT / 64, cap = NT == 1024 ? kTileT : kNarrowTW;
};
constexpr uint32_t kTileU = 16;  // 64-in-edge segments a wave has in flight per step

// Finishes targets [base + i] for i = tid, tid + nthreads, ... < count with new
// deltas d(i), four targets per step with their operands loaded first.
template <int ST, int G, bool FUSED, typename D>
__device__ __forceinline__ void tile_finish_targets(const KArgs& a, typename Tr<ST>::S* mu_out, uint64_t base,
                                                    uint32_t count, uint32_t tid, uint32_t nthreads, const D& d,
                                                    double& r_part, uint64_t& act, uint64_t& pushed) {
  using S = typename Tr<ST>::S;
  if constexpr (!FUSED) {  // dv += sum; act counts the pending vertices of the new state
    S* dvw = static_cast<S*>(a.dv);
    for (uint32_t i0 = tid; i0 < count; i0 += 4 * nthreads) {
      S dvp[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) dvp[u] = dvw[base + min(i0 + u * nthreads, count - 1)];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * nthreads;
        if (i >= count) break;
        const double x = d(i);
        S nd = dvp[u];
        if (x != 0.0) {
          nd = (S)((double)dvp[u] + x);
          dvw[base + i] = nd;
        }
        r_part += fabs((double)nd);
        act += nd != (S)0 ? 1 : 0;
      }
    }
    return;
  }
  const S* dv = static_cast<const S*>(a.dv);
  const S* v = static_cast<const S*>(a.v);
  const uint32_t* row = static_cast<const uint32_t*>(a.row);
  for (uint32_t i0 = tid; i0 < count; i0 += 4 * nthreads) {
    S dvp[4], vp[4];
    float cp[4];
    uint32_t dg[4], pp[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint64_t t = base + min(i0 + u * nthreads, count - 1);
      dvp[u] = dv[t];
      vp[u] = v[t];
      cp[u] = Tr<ST>::kahan ? a.c[t] : 0.f;
      dg[u] = row[t + 1] - row[t];
      pp[u] = a.perm[t];
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t i = i0 + u * nthreads;
      if (i < count)
        FusedTarget<ST, G>::finish(a, mu_out, (uint32_t)(base + i), dvp[u], (S)d(i), vp[u], cp[u], dg[u], pp[u], r_part,
                                   act, pushed);
    }
  }
}

// Type of the partial-sum slots of split partitions: FP32 for FP32 states
// (whose messages are FP32; each slot holds an FP64 sum rounded once),
// FP64 otherwise. The slots are added in FP64.
template <int ST>
using SlotT = typename std::conditional<ST == ST_F32 || ST == ST_F32K, float, double>::type;
inline uint32_t slot_size(int st) { return st == ST_F32 || st == ST_F32K ? 4u : 8u; }

// Walks the in-edges [e0, e1) of one tile, kTileU segments of 64 in-edges
// per wave and step (every wave of the workgroup calls it): a lane loads its
// in-edge's local target; a ballot of the pair-start bits and a popcount give
// its pair (the segment's first pair plus the starts among the lanes before
// it), whose source indexes the message load msg(source, in-edge), issued for
// all kTileU segments before any is combined; add(local target, message)
// then runs for the in-edges inside the tile. With PIPE the next step's
// local targets are loaded after this step's messages, so they arrive while
// the messages do (one memory round trip of three per step hidden); the
// weighted walks, whose messages also load a weight, run without it (with it
// they would spill registers at 1,024 threads). The index arithmetic is 32-bit
// and unclamped: the tiled arrays hold kTilePadSeg segments of padding (no
// pair starts, segment pair 0), so every load of a step stays inside them and
// a padded lane's pair is a real one. Local targets are below the partition
// width, so masking the flag bit leaves an index below kTileT.
static_assert(kTileU <= kTilePadSeg, "a step's segments must stay inside the padded arrays");
template <uint32_t NT, bool PIPE, typename V, typename Msg, typename Add>
__device__ __forceinline__ void tile_walk(const TileArgs& t, uint32_t e0, uint32_t e1, const Msg& msg,
                                          const Add& add) {
  constexpr uint32_t kWaves = NT / 64;
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t s1 = (e1 + 63) >> 6, span = e1 - e0;  // segments end; in-edges of the tile
  constexpr uint32_t stride = kWaves * kTileU;
  uint32_t sg = (e0 >> 6) + wave * kTileU;
  uint32_t ploc[kTileU], psp[kTileU];  // PIPE: the coming step's local targets and segment pairs
  if (PIPE && sg < s1) {
#pragma unroll
    for (uint32_t u = 0; u < kTileU; ++u) {
      ploc[u] = t.tloc[(sg + u) * 64 + lane];
      psp[u] = t.segpair[sg + u];
    }
  }
  for (; sg < s1; sg += stride) {
    uint32_t loc[kTileU], sp[kTileU];
    bool in[kTileU];
#pragma unroll
    for (uint32_t u = 0; u < kTileU; ++u) {
      const uint32_t e = (sg + u) * 64 + lane;
      in[u] = e - e0 < span;
      if constexpr (PIPE) {
        loc[u] = ploc[u];
        sp[u] = psp[u];
      } else {
        loc[u] = t.tloc[(sg + u) * 64 + lane];
        sp[u] = t.segpair[sg + u];  // the same for the whole wave
      }
    }
    uint32_t src[kTileU];
#pragma unroll
    for (uint32_t u = 0; u < kTileU; ++u) {
      // pair starts at segment positions 1..lane (position 0 belongs to the
      // segment's pair): the starts shifted down one, counted below the lane
      const uint64_t flags = __ballot(loc[u] >= kPairStart) >> 1;
      src[u] = t.psrc[__builtin_amdgcn_mbcnt_hi((uint32_t)(flags >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)flags, sp[u]))];
    }
    V x[kTileU];
#pragma unroll
    for (uint32_t u = 0; u < kTileU; ++u) x[u] = msg(src[u], (sg + u) * 64 + lane);
    if constexpr (PIPE) {
      // the next step's offsets, in flight while this step's messages arrive
      const uint32_t ng = sg + stride;
      if (ng < s1) {
#pragma unroll
        for (uint32_t u = 0; u < kTileU; ++u) {
          ploc[u] = t.tloc[(ng + u) * 64 + lane];
          psp[u] = t.segpair[ng + u];
        }
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kTileU; ++u)
      if (in[u]) add(loc[u] & (kTileT - 1), x[u]);
  }
}

template <int ST, int G, bool FUSED, uint32_t NT>
__global__ __launch_bounds__(NT) void k_tile_pull(KArgs a, TileArgs t) {
  using S = typename Tr<ST>::S;
  constexpr uint32_t kTileThreads = NT, kTileWaves = TileShape<NT>::waves;
  if constexpr (Tr<ST>::sum) {
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || (!FUSED && !ctl->last_pull)) return;
    __shared__ double acc[TileShape<NT>::cap];
    const uint32_t tid = threadIdx.x;
    const bool odd = FUSED && ((ctl->rounds - ctl->fuse_base) & 1) != 0;
    const S* mu_in = static_cast<const S*>(odd ? a.mu_pi2 : a.mu_pi);
    S* mu_out = static_cast<S*>(odd ? a.mu_pi : a.mu_pi2);
    const S* wt = static_cast<const S*>(t.wtile);
    double r_part = 0.0;
    uint64_t act = 0, pushed = 0;
    auto msg = [&](uint32_t src, uint32_t e) -> double {
      double x = (double)mu_in[src];
      if constexpr (G == DAIC_G_EDGE_SCALE) x *= (double)wt[e];
      return x;
    };
    auto add = [&](uint32_t l, double x) { atomicAdd(&acc[l], x); };  // adding 0 leaves a sum as it is
    for (uint64_t pos = blockIdx.x; pos < t.n_tiles; pos += gridDim.x) {
      const uint32_t tile = t.tile_order[pos];
      const uint32_t part = t.tile_part[tile], e0 = t.tile_e[tile], e1 = t.tile_e[tile + 1], slot = t.tile_slot[tile];
      for (uint32_t i = tid; i < t.tw; i += kTileThreads) acc[i] = 0.0;
      __syncthreads();
      tile_walk<NT, G != DAIC_G_EDGE_SCALE, double>(t, e0, e1, msg, add);
      __syncthreads();
      const uint64_t base = (uint64_t)part * t.tw;
      const uint32_t count = (uint32_t)min((uint64_t)t.tw, a.n - base);
      if (slot == 0xFFFFFFFFu) {
        tile_finish_targets<ST, G, FUSED>(a, mu_out, base, count, tid, kTileThreads,
                                          [&](uint32_t i) { return acc[i]; }, r_part, act, pushed);
      } else {
        SlotT<ST>* dst = reinterpret_cast<SlotT<ST>*>(t.pbuf) + (uint64_t)slot * t.tw;
        for (uint32_t i = tid; i < count; i += kTileThreads) dst[i] = (SlotT<ST>)acc[i];
      }
      __syncthreads();
    }
    r_part = block_sum_waves<kTileWaves>(r_part);
    act = block_sum_waves<kTileWaves>(act);
    pushed = block_sum_waves<kTileWaves>(pushed);
    if (tid == 0) {
      t.tpart_r[blockIdx.x] = r_part;
      t.tpart_a[blockIdx.x] = act;
      t.tpart_p[blockIdx.x] = pushed;
    }
  }
}

// Targets of split partitions: a work item is 256 consecutive targets of one
// split partition; their slots are added in tile order, 16 loads in flight.
template <int ST, int G, bool FUSED>
__global__ __launch_bounds__(256) void k_tile_finish(KArgs a, TileArgs t) {
  using S = typename Tr<ST>::S;
  if constexpr (Tr<ST>::sum) {
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || (!FUSED && !ctl->last_pull)) return;
    const bool odd = FUSED && ((ctl->rounds - ctl->fuse_base) & 1) != 0;
    S* mu_out = static_cast<S*>(odd ? a.mu_pi : a.mu_pi2);
    const SlotT<ST>* pbuf = reinterpret_cast<const SlotT<ST>*>(t.pbuf);
    const uint32_t tid = threadIdx.x;
    const uint32_t kChunks = t.tw / 256;
    double r_part = 0.0;
    uint64_t act = 0, pushed = 0;
    for (uint64_t item = blockIdx.x; item < t.n_split * kChunks; item += gridDim.x) {
      const uint64_t sp = item / kChunks;
      const uint32_t chunk = (uint32_t)(item % kChunks);
      const uint32_t part = t.split_part[sp], k0 = t.split_slot[sp], k1 = t.split_slot[sp + 1];
      const uint64_t base = (uint64_t)part * t.tw + chunk * 256;
      if (base >= a.n) continue;  // uniform
      const uint32_t count = (uint32_t)min((uint64_t)256, a.n - base);
      const uint32_t i = chunk * 256 + min(tid, count - 1);
      double sum = 0.0;
      for (uint32_t k = k0; k < k1; k += 16) {
        double x[16];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) x[u] = (double)pbuf[(uint64_t)min(k + u, k1 - 1) * t.tw + i];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u)
          if (k + u < k1) sum += x[u];
      }
      tile_finish_targets<ST, G, FUSED>(a, mu_out, base, count, tid, 256, [&](uint32_t) { return sum; }, r_part, act,
                                        pushed);
    }
    r_part = block_sum256(r_part);
    act = block_sum256(act);
    pushed = block_sum256(pushed);
    if (tid == 0) {
      t.spart_r[blockIdx.x] = r_part;
      t.spart_a[blockIdx.x] = act;
      t.spart_p[blockIdx.x] = pushed;
    }
  }
}

// The round's totals (one block): partials of np k_tile_pull and nf
// k_tile_finish workgroups in a fixed order; residual, counters, round count
// and stop rule as k_fused_finish sets them (FUSED), or residual, pending
// count, round count, stop rule and next direction as k_pull_finish does.
template <int ST, bool FUSED>
__global__ __launch_bounds__(256) void k_tile_total(KArgs a, TileArgs t, uint32_t np, uint32_t nf, uint64_t k_sel,
                                                    uint64_t pull_min) {
  if constexpr (Tr<ST>::sum || !FUSED) {
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || (!FUSED && !ctl->last_pull)) return;
    double rr = 0.0;
    uint64_t aa = 0, ps = 0;
    // eight partials per thread at a time, their loads in flight together
    // and added in the same order as one at a time
    auto add_partials = [&](const double* pr, const uint64_t* pa, const uint64_t* pp, uint32_t count) {
      for (uint32_t i0 = threadIdx.x; i0 < count; i0 += 8 * 256) {
        double xr[8];
        uint64_t xa[8], xp[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
          const uint32_t i = min(i0 + u * 256, count - 1);
          xr[u] = pr[i];
          xa[u] = pa[i];
          xp[u] = pp[i];
        }
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u)
          if (i0 + u * 256 < count) {
            rr += xr[u];
            aa += xa[u];
            ps += xp[u];
          }
      }
    };
    add_partials(t.tpart_r, t.tpart_a, t.tpart_p, np);
    add_partials(t.spart_r, t.spart_a, t.spart_p, nf);
    rr = block_sum256(rr);
    aa = block_sum256(aa);
    ps = block_sum256(ps);
    if (threadIdx.x == 0) {
      ctl->r = Tr<ST>::sum ? rr : (double)aa;  // min/max: rr holds the pending vertices' out-edges
      ctl->rounds += 1;
      if constexpr (FUSED) {
        ctl->activations += aa;
        ctl->pushed += ps;
        ctl->round_act = aa;
        ctl->round_pushed = ps;
        const bool done = rr <= ctl->eps;
        ctl->done = done ? 1u : 0u;
        ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
      } else {
        const uint64_t nn = aa;  // pending vertices of the new state
        ctl->pending = nn;
        const bool done = Tr<ST>::sum ? (rr <= ctl->eps || nn == 0) : nn == 0;
        ctl->done = done ? 1u : 0u;
        ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
        ctl->pull = next_is_dense<ST>(nn, rr, k_sel, pull_min);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dense rounds of min and max problems (SSSP, connected components): the same
// walk over the tiled in-edges, with the messages combined by (+) itself.
// The round's claim has published each sender's message base (its new value
// when it improved, else the identity); an in-edge's message is g of it
// (base + weight, saturating, for EDGE_ADD; the base for COPY), combined into
// an LDS accumulator of its target with an LDS atomic min or max (integer
// bits; non-negative doubles order like their bit patterns). A target then
// takes the combined message into dv when it improves both v and dv, which
// is what the pushes of the same messages would leave (each push is filtered
// by v and dv), and counts as pending when dv improves v. Min and max are
// exact, so the result equals the push rounds' bit for bit.
// ---------------------------------------------------------------------------
template <int ST>
struct TileMM;
template <>
struct TileMM<ST_U32> {
  using L = uint32_t;
  static constexpr L ident = kInfU32;
  static __device__ __forceinline__ bool better(L a, L b) { return a < b; }
  static __device__ __forceinline__ void combine(L* p, L x) { atomicMin(p, x); }
  static __device__ __forceinline__ L enc(uint32_t s) { return s; }
  static __device__ __forceinline__ uint32_t dec(L x) { return x; }
};
template <>
struct TileMM<ST_F64MIN> {
  using L = unsigned long long;
  static constexpr L ident = 0x7FF0000000000000ull;  // +inf
  static __device__ __forceinline__ bool better(L a, L b) { return a < b; }
  static __device__ __forceinline__ void combine(L* p, L x) { atomicMin(p, x); }
  static __device__ __forceinline__ L enc(double s) { return (L)__double_as_longlong(s); }
  static __device__ __forceinline__ double dec(L x) { return __longlong_as_double((long long)x); }
};
template <>
struct TileMM<ST_I32> {
  using L = int32_t;
  static constexpr L ident = -1;
  static __device__ __forceinline__ bool better(L a, L b) { return a > b; }
  static __device__ __forceinline__ void combine(L* p, L x) { atomicMax(p, x); }
  static __device__ __forceinline__ L enc(int32_t s) { return s; }
  static __device__ __forceinline__ int32_t dec(L x) { return x; }
};

// The message an in-edge carries from base mu (weight w for EDGE_ADD), as an
// accumulator value; the identity when the source is silent.
template <int ST, int G>
__device__ __forceinline__ typename TileMM<ST>::L tile_mm_msg(typename Tr<ST>::S mu, const void* wt, uint64_t e) {
  using M = TileMM<ST>;
  if constexpr (ST == ST_U32) {
    if (mu == kInfU32) return M::ident;
    const uint64_t x = (uint64_t)mu + static_cast<const uint32_t*>(wt)[e];
    return x >= kInfU32 ? M::ident : (uint32_t)x;
  } else if constexpr (ST == ST_F64MIN) {
    if (isinf(mu)) return M::ident;
    return M::enc(mu + static_cast<const double*>(wt)[e]);
  } else {
    return mu;  // COPY; -1 (silent) is the identity
  }
}

// Takes the combined message x of target t into dv and counts t when
// pending, with its out-edges (for the next round's direction) in r_part.
template <int ST>
__device__ __forceinline__ void tile_mm_finish(const KArgs& a, uint64_t t, typename TileMM<ST>::L x,
                                               typename Tr<ST>::S vt, typename Tr<ST>::S dvt, double& r_part,
                                               uint64_t& act) {
  using M = TileMM<ST>;
  using S = typename Tr<ST>::S;
  const typename M::L lv = M::enc(vt), ld = M::enc(dvt);
  typename M::L nd = ld;
  if (M::better(x, lv) && M::better(x, ld)) {
    nd = x;
    static_cast<S*>(a.dv)[t] = (S)M::dec(x);
  }
  const bool pend = M::better(nd, lv);
  act += pend ? 1 : 0;
  if (pend) {
    const uint32_t* row = static_cast<const uint32_t*>(a.row);  // dense rounds need 32-bit offsets
    r_part += (double)(row[t + 1] - row[t]);
  }
}

template <int ST, int G, uint32_t NT>
__global__ __launch_bounds__(NT) void k_tile_pull_mm(KArgs a, TileArgs t) {
  constexpr uint32_t kTileThreads = NT, kTileWaves = TileShape<NT>::waves;
  if constexpr (!Tr<ST>::sum) {
    using S = typename Tr<ST>::S;
    using M = TileMM<ST>;
    using L = typename M::L;
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || !ctl->last_pull) return;
    __shared__ L acc[TileShape<NT>::cap];
    const uint32_t tid = threadIdx.x;
    const S* mu_in = static_cast<const S*>(a.mu_pi);
    const S* v = static_cast<const S*>(a.v);
    const S* dv = static_cast<const S*>(a.dv);
    double r_part = 0.0;
    uint64_t act = 0;
    auto msg = [&](uint32_t src, uint32_t e) -> L { return tile_mm_msg<ST, G>(mu_in[src], t.wtile, e); };
    auto add = [&](uint32_t l, L x) {
      if (x != M::ident) M::combine(&acc[l], x);
    };
    for (uint64_t pos = blockIdx.x; pos < t.n_tiles; pos += gridDim.x) {
      const uint32_t tile = t.tile_order[pos];
      const uint32_t part = t.tile_part[tile], e0 = t.tile_e[tile], e1 = t.tile_e[tile + 1], slot = t.tile_slot[tile];
      for (uint32_t i = tid; i < t.tw; i += kTileThreads) acc[i] = M::ident;
      __syncthreads();
      tile_walk<NT, G != DAIC_G_EDGE_ADD, L>(t, e0, e1, msg, add);
      __syncthreads();
      const uint64_t base = (uint64_t)part * t.tw;
      const uint32_t count = (uint32_t)min((uint64_t)t.tw, a.n - base);
      if (slot == 0xFFFFFFFFu) {
        for (uint32_t i = tid; i < count; i += kTileThreads)
          tile_mm_finish<ST>(a, base + i, acc[i], v[base + i], dv[base + i], r_part, act);
      } else {
        L* dst = reinterpret_cast<L*>(t.pbuf) + (uint64_t)slot * t.tw;
        for (uint32_t i = tid; i < count; i += kTileThreads) dst[i] = acc[i];
      }
      __syncthreads();
    }
    r_part = block_sum_waves<kTileWaves>(r_part);
    act = block_sum_waves<kTileWaves>(act);
    if (tid == 0) {
      t.tpart_r[blockIdx.x] = r_part;
      t.tpart_a[blockIdx.x] = act;
      t.tpart_p[blockIdx.x] = 0;
    }
  }
}

// Targets of split partitions: their slots combined in tile order, then
// taken into dv as above.
template <int ST, int G>
__global__ __launch_bounds__(256) void k_tile_finish_mm(KArgs a, TileArgs t) {
  if constexpr (!Tr<ST>::sum) {
    using S = typename Tr<ST>::S;
    using M = TileMM<ST>;
    using L = typename M::L;
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || !ctl->last_pull) return;
    const L* pbuf = reinterpret_cast<const L*>(t.pbuf);
    const S* v = static_cast<const S*>(a.v);
    const S* dv = static_cast<const S*>(a.dv);
    const uint32_t tid = threadIdx.x;
    const uint32_t kChunks = t.tw / 256;
    double r_part = 0.0;
    uint64_t act = 0;
    for (uint64_t item = blockIdx.x; item < t.n_split * kChunks; item += gridDim.x) {
      const uint64_t sp = item / kChunks;
      const uint32_t chunk = (uint32_t)(item % kChunks);
      const uint32_t part = t.split_part[sp], k0 = t.split_slot[sp], k1 = t.split_slot[sp + 1];
      const uint64_t base = (uint64_t)part * t.tw + chunk * 256;
      if (base >= a.n) continue;  // uniform
      const uint32_t count = (uint32_t)min((uint64_t)256, a.n - base);
      if (tid >= count) continue;
      const uint32_t i = chunk * 256 + tid;
      L x = M::ident;
      for (uint32_t k = k0; k < k1; k += 16) {
        L y[16];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) y[u] = pbuf[(uint64_t)min(k + u, k1 - 1) * t.tw + i];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u)
          if (k + u < k1 && M::better(y[u], x)) x = y[u];
      }
      tile_mm_finish<ST>(a, base + tid, x, v[base + tid], dv[base + tid], r_part, act);
    }
    r_part = block_sum256(r_part);
    act = block_sum256(act);
    if (tid == 0) {
      t.spart_r[blockIdx.x] = r_part;
      t.spart_a[blockIdx.x] = act;
      t.spart_p[blockIdx.x] = 0;
    }
  }
}

}  // namespace daic
