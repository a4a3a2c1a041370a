// Device code of one DAIC round on gfx950 (64-lane wavefronts).
//
// A round (Eq. async of the paper applied to a selected set, Sec. 3.2/3.4):
//   A2 k_sample_keys + k_sample, or k_radix_pass + k_radix_pick per digit
//                           : threshold of the priority keys (sampled or exact)
//   A3+A4 k_claim           : select, claim dv_j, fold v_j (+)= delta, compute
//                             the message base mu_j, compact into degree bins
//                             (sparse rounds) or publish mu_j (dense rounds)
//   k_bin_scan              : prefix of the per-block bin counts
//   A5 k_push               : atomic (+) of g(mu_j) into dv_k for every out-edge
//                             (small and large bins in one launch)
//      dense rounds         : every target combines its in-neighbours' bases,
//                             through the tiled in-edges (daic_tile.h: sum, min
//                             and max problems) or, without them, k_pull_stream
//                             (sum problems; then k_pull_finish: residual and
//                             stop rule)
//   A1 k_residual + k_residual_final : residual of the new state and the stop rule
// Fused dense rounds (every pending vertex, sum problems): the tiled kernels
// with FUSED = true, or k_pull_fused + k_fused_finish, per round after one
// priming claim.
// The claim happens in a kernel of its own, before any push of the round, so
// every message of the round lands in dv after the claim: it is folded in a
// later round and never lost (the receive/update split of Eq. async).
#pragma once

#include <type_traits>

#include "daic_device.h"
#include "daic_internal.h"

namespace daic {

// ---------------------------------------------------------------------------
// Element types of each state kind.
// ---------------------------------------------------------------------------
template <int ST> struct Tr;
template <> struct Tr<ST_F64> { using S = double;   using Key = uint64_t; static constexpr bool sum = true;  static constexpr bool kahan = false; };
template <> struct Tr<ST_F32> { using S = float;    using Key = uint32_t; static constexpr bool sum = true;  static constexpr bool kahan = false; };
template <> struct Tr<ST_F32K>{ using S = float;    using Key = uint32_t; static constexpr bool sum = true;  static constexpr bool kahan = true;  };
template <> struct Tr<ST_U32> { using S = uint32_t; using Key = uint32_t; static constexpr bool sum = false; static constexpr bool kahan = false; };
template <> struct Tr<ST_I32> { using S = int32_t;  using Key = uint32_t; static constexpr bool sum = false; static constexpr bool kahan = false; };
// min over non-negative doubles (SSSP with real weights); +inf = unreached
template <> struct Tr<ST_F64MIN> { using S = double; using Key = uint64_t; static constexpr bool sum = false; static constexpr bool kahan = false; };

// Kernel arguments (passed by value).
struct KArgs {
  Ctl* ctl;
  const void* row;          // RowT[n+1]
  const uint32_t* col;      // [m]
  const void* w;            // S[m] (EDGE_SCALE) or uint32[m] (EDGE_ADD)
  void* v;                  // S[n]
  void* dv;                 // S[n]
  float* c;                 // Kahan compensation [n]
  const void* alpha_pv;     // S[n] or null
  double alpha;
  uint64_t n;
  uint64_t per_block;
  uint32_t blocks;
  uint32_t* small_vid;      // [n], block b's region starts at b*per_block
  void* small_mu;           // S[n]
  uint32_t* large_vid;      // [large_cap], block b's region starts at large_off[b]
  uint32_t* large_chunk;
  void* large_mu;
  const uint64_t* large_off;  // [blocks+1]
  uint32_t* blk_small;      // per-block counts of this round
  uint32_t* blk_large;
  uint64_t* off_small;      // [blocks+1] prefix of blk_small
  uint64_t* off_large;      // [blocks+1] prefix of blk_large
  uint64_t* blk_act;        // per-block activations / pushed edges (all, large bin)
  uint64_t* blk_push;
  uint64_t* blk_push_large;
  uint32_t* blk_ties;       // exact top-k: keys equal to tau per block
  uint32_t* rhist;          // exact top-k: radix histogram (kRadixCopies x kRadixBins counters)
  uint64_t* skeys;          // sampled threshold: the round's sampled keys (kMaxSamples)
  uint64_t* off_ties;       // exclusive prefix of blk_ties
  double* part_r;           // residual partials per block
  uint64_t* part_n;         // pending-count partials per block
  uint8_t* sel_out;         // dry selection output [n]
  const float* score;       // learned scheduler: multiplier in (0,1) per vertex, or null
  uint32_t* last_upd;       // learned scheduler: 1 + round of each vertex's last update (0: none), or null
  uint64_t rr_chunk;        // round-robin: ids per block
  // dense rounds (pull over in-edges)
  const uint32_t* perm;     // renumbering of sources by out-degree
  const uint32_t* rowT;     // in-edge offsets [n+1]
  const uint32_t* srcT;     // renumbered source of each in-edge
  const void* wT;           // S[m] weights in in-edge order (EDGE_SCALE)
  void* mu_pi;              // S[n] message base of every vertex, renumbered
  uint64_t n_src;           // vertices with out-edges (renumbered positions below n_src)
  const uint32_t* sb_t;     // edge blocks of the streamed pull: first target,
  const uint32_t* sb_e;     //   first in-edge (one extra entry: m),
  const uint32_t* sb_n;     //   number of targets covered
  uint64_t sb_count;
  // fused dense rounds
  void* mu_pi2;             // S[n] second message-base buffer (rounds alternate A, B)
  const uint32_t* sb_g;     // group of a piece of a cut target, else 0xFFFFFFFF
  const uint32_t* g_np;     // pieces per group
  const uint32_t* g_first;  // first block of each group
  uint64_t n_groups;
  double* sb_part;          // partial sum of each piece (per block)
  double* fpart_r;          // per-workgroup partials of k_pull_fused: |new delta|,
  uint64_t* fpart_a;        //   vertex updates,
  uint64_t* fpart_p;        //   messages
  double* gpart_r;          // the same per block of k_fused_finish
  uint64_t* gpart_a;
  uint64_t* gpart_p;
};

__device__ __forceinline__ bool ctl_halted(const Ctl* ctl) {
  return (ctl->done | ctl->stop) != 0;
}

// SplitMix64 (Steele, Lea, Flood 2014): output number c of the generator
// seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Priority |v (+) dv - v| as an unsigned key whose integer order is the order
// of the priority (Sec. 3.5; SSSP form d - min(d, dd) of Sec. 4.2.1 with
// inf - x taken as 0xFFFFFFFF; CC form max(v, dv) - v). Key 0 = not pending.
// ---------------------------------------------------------------------------
template <int ST>
__device__ __forceinline__ typename Tr<ST>::Key prio_key(typename Tr<ST>::S v, typename Tr<ST>::S dv) {
  if constexpr (ST == ST_F64) {
    return (uint64_t)__double_as_longlong(fabs(dv));
  } else if constexpr (ST == ST_F32 || ST == ST_F32K) {
    return __float_as_uint(fabsf(dv));
  } else if constexpr (ST == ST_U32) {
    if (v == kInfU32) return dv < kInfU32 ? kInfU32 : 0u;
    return v - (dv < v ? dv : v);
  } else if constexpr (ST == ST_F64MIN) {
    // d - min(d, dd) >= 0, whose IEEE bits order like the value; a first
    // reach (d = inf, dd finite) takes the bits of +inf, above every finite
    if (isinf(v)) return isinf(dv) ? 0ull : 0x7FF0000000000000ull;
    return (uint64_t)__double_as_longlong(v - (dv < v ? dv : v));
  } else {
    int64_t mx = (int64_t)(dv > v ? dv : v);
    return (uint32_t)(mx - (int64_t)v);
  }
}

// The priority as a float (features and the learned selection key); a first
// reach of a min problem counts as 2^32, as for the integer state.
template <int ST>
__device__ __forceinline__ float prio_value(typename Tr<ST>::S v, typename Tr<ST>::S dv) {
  if constexpr (Tr<ST>::sum) {
    return (float)fabs((double)dv);
  } else if constexpr (ST == ST_F64MIN) {
    if (isinf(v)) return isinf(dv) ? 0.0f : 4294967296.0f;
    return (float)(v - (dv < v ? dv : v));
  } else {
    return (float)prio_key<ST>(v, dv);
  }
}

// Key used by the selection: the priority, or for the learned scheduler the
// priority scaled by the network's multiplier (FP32, same bit-order trick).
template <int ST>
__device__ __forceinline__ typename Tr<ST>::Key sel_key(const KArgs& a, uint64_t j, typename Tr<ST>::S v,
                                                         typename Tr<ST>::S dv) {
  using Key = typename Tr<ST>::Key;
  Key k = prio_key<ST>(v, dv);
  if (a.score != nullptr && k != 0) {
    const float p = prio_value<ST>(v, dv);
    float s = p * a.score[j];
    uint32_t b = __float_as_uint(s);
    return (Key)(b == 0 ? 1u : b);  // a pending vertex keeps a positive key
  }
  return k;
}

// sel_key with the vertex's multiplier already loaded (sc, read only when
// the learned scheduler's scores are present), so that the loads of several
// vertices can be issued before any key is formed.
template <int ST>
__device__ __forceinline__ typename Tr<ST>::Key sel_key_loaded(const KArgs& a, typename Tr<ST>::S v,
                                                                typename Tr<ST>::S dv, float sc) {
  using Key = typename Tr<ST>::Key;
  Key k = prio_key<ST>(v, dv);
  if (a.score != nullptr && k != 0) {
    const uint32_t b = __float_as_uint(prio_value<ST>(v, dv) * sc);
    return (Key)(b == 0 ? 1u : b);
  }
  return k;
}

template <typename RowT>
__device__ __forceinline__ uint64_t row_at(const void* row, uint64_t j) {
  return (uint64_t)static_cast<const RowT*>(row)[j];
}

// Index b with off[b] <= i < off[b+1] (off has nb+1 entries, off[0] = 0).
__device__ __forceinline__ uint32_t find_block(const uint64_t* off, uint32_t nb, uint64_t i) {
  uint32_t lo = 0, hi = nb;  // invariant: off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// A4: claim and fold. Returns whether j sends, and the message base mu.
// ---------------------------------------------------------------------------
template <int ST, int G>
__device__ __forceinline__ bool claim_fold(const KArgs& a, uint64_t j, uint64_t deg,
                                           typename Tr<ST>::S v_old, typename Tr<ST>::S delta,
                                           typename Tr<ST>::S& mu) {
  using S = typename Tr<ST>::S;
  S* v = static_cast<S*>(a.v);
  S* dv = static_cast<S*>(a.dv);
  if constexpr (Tr<ST>::sum) {
    dv[j] = (S)0;
    if constexpr (Tr<ST>::kahan) {
      // Compensated summation (Kahan 1965): the rounding error of each fold
      // is carried in c_j and subtracted from the next delta.
#pragma clang fp contract(off)
      float cj = a.c[j];
      float y = delta - cj;
      float t = v_old + y;
      a.c[j] = (t - v_old) - y;
      v[j] = t;
    } else {
      v[j] = v_old + delta;
    }
    double coef;
    if constexpr (G == DAIC_G_DEG_SCALE) {
      coef = a.alpha / (double)deg;
    } else {
      coef = a.alpha_pv ? (double)static_cast<const S*>(a.alpha_pv)[j] : a.alpha;
    }
    mu = (S)(coef * (double)delta);
    return delta != (S)0;
  } else if constexpr (ST == ST_U32) {
    dv[j] = kInfU32;
    if (delta < v_old) {
      v[j] = delta;
      mu = delta;
      return true;
    }
    return false;
  } else if constexpr (ST == ST_F64MIN) {
    dv[j] = __builtin_huge_val();
    if (delta < v_old) {
      v[j] = delta;
      mu = delta;
      return true;
    }
    return false;
  } else {
    dv[j] = -1;
    if (delta > v_old) {
      v[j] = delta;
      mu = delta;
      return true;
    }
    return false;
  }
}

// A5: one message along edge e into dv[k] (skipping identity messages and,
// for min/max, messages that cannot change the receiver).
template <int ST, int G>
__device__ __forceinline__ void push_edge(const KArgs& a, uint64_t e, typename Tr<ST>::S mu) {
  using S = typename Tr<ST>::S;
  const uint32_t k = a.col[e];
  S* dv = static_cast<S*>(a.dv);
  if constexpr (Tr<ST>::sum) {
    S m = mu;
    if constexpr (G == DAIC_G_EDGE_SCALE) m = mu * static_cast<const S*>(a.w)[e];
    if (m != (S)0) unsafeAtomicAdd(&dv[k], m);
  } else if constexpr (ST == ST_U32) {
    uint64_t s = (uint64_t)mu + static_cast<const uint32_t*>(a.w)[e];
    uint32_t m = s >= kInfU32 ? kInfU32 : (uint32_t)s;
    const uint32_t* v = static_cast<const uint32_t*>(a.v);
    if (m < v[k] && m < dv[k]) atomicMin(&dv[k], m);
  } else if constexpr (ST == ST_F64MIN) {
    // non-negative doubles order like their bit patterns, so the minimum is
    // an unsigned 64-bit atomic min on the bits
    const double m = mu + static_cast<const double*>(a.w)[e];
    const double* v = static_cast<const double*>(a.v);
    if (m < v[k] && m < dv[k])
      atomicMin(reinterpret_cast<unsigned long long*>(&dv[k]), (unsigned long long)__double_as_longlong(m));
  } else {
    const int32_t* v = static_cast<const int32_t*>(a.v);
    if (mu > v[k] && mu > dv[k]) atomicMax(&dv[k], mu);
  }
}

// ---------------------------------------------------------------------------
// A1: residual of the current state and the stop rule. Deterministic: every
// block of k_residual stores its partials, and k_residual_final (one block)
// sums them in a fixed order. (A last-block ticket would make all blocks
// increment one counter at the same time; those atomics serialize.)
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void k_residual(KArgs a, int skip_dense = 0) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  if (skip_dense && ctl->last_pull) return;  // a dense round's residual comes from k_pull_finish
  const uint32_t b = blockIdx.x;
  const uint64_t lo = (uint64_t)b * a.per_block;
  const uint64_t hi = min(a.n, lo + a.per_block);
  const S* v = static_cast<const S*>(a.v);
  const S* dv = static_cast<const S*>(a.dv);
  double r = 0.0;
  uint64_t cnt = 0;
  // four vertices per step, their loads in flight together (a thread walks
  // many vertices; one load at a time would leave the kernel latency-bound)
  for (uint64_t j0 = lo + threadIdx.x; j0 < hi; j0 += 1024) {
    S dj[4], vj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t j = min(j0 + 256 * u, hi - 1);
      dj[u] = dv[j];
      if constexpr (!Tr<ST>::sum) vj[u] = v[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j0 + 256 * u >= hi) break;
      if constexpr (Tr<ST>::sum) {
        double x = fabs((double)dj[u]);
        r += x;
        cnt += x > 0.0;
      } else {
        const bool pend = prio_key<ST>(vj[u], dj[u]) != 0;
        cnt += pend;
        // with dense rounds set up (32-bit row offsets): the out-edges of the
        // pending vertices, from which the next round's direction is chosen
        if (pend && a.perm != nullptr) {
          const uint32_t* row = static_cast<const uint32_t*>(a.row);
          const uint64_t j = j0 + 256 * u;
          r += (double)(row[j + 1] - row[j]);
        }
      }
    }
  }
  r = block_sum256(r);
  cnt = block_sum256(cnt);
  if (threadIdx.x == 0) {
    a.part_r[b] = r;
    a.part_n[b] = cnt;
  }
}

// The direction of the next round: a dense round (pull over in-edges) when
// the next round is expected to do enough work. Sum problems: at least
// pull_min vertices expected to update (min(pending, k_sel)). Min and max
// problems: at least pull_min messages expected, estimated from the
// out-edges of the pending vertices (pend_edges) scaled to the share of
// them the next round selects. k_sel = 0 disables dense rounds.
template <int ST>
__device__ __forceinline__ uint32_t next_is_dense(uint64_t nn, double pend_edges, uint64_t k_sel, uint64_t pull_min) {
  const uint64_t k_next = nn < k_sel ? nn : k_sel;
  if (k_sel == 0) return 0u;
  if constexpr (Tr<ST>::sum) {
    return k_next >= pull_min ? 1u : 0u;
  } else {
    const double est = nn ? pend_edges * ((double)k_next / (double)nn) : 0.0;
    return est >= (double)pull_min ? 1u : 0u;
  }
}

// Besides the residual, k_residual_final picks the direction of the next
// round (next_is_dense). One block; it returns in the cases where k_residual
// returned.
template <int ST>
__global__ __launch_bounds__(256) void k_residual_final(KArgs a, int count_round, uint64_t k_sel,
                                                        uint64_t pull_min, int skip_dense = 0) {
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  if (skip_dense && ctl->last_pull) return;
  double rr = 0.0;
  uint64_t nn = 0;
  for (uint32_t i0 = threadIdx.x; i0 < a.blocks; i0 += 1024) {
    double pr[4];
    uint64_t pn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = min(i0 + 256 * u, a.blocks - 1);
      pr[u] = a.part_r[i];
      pn[u] = a.part_n[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + 256 * u >= a.blocks) break;
      rr += pr[u];
      nn += pn[u];
    }
  }
  rr = block_sum256(rr);
  nn = block_sum256(nn);
  if (threadIdx.x == 0) {
    if constexpr (Tr<ST>::sum) ctl->r = rr; else ctl->r = (double)nn;
    ctl->pending = nn;
    ctl->rounds += (uint64_t)count_round;
    bool done = Tr<ST>::sum ? (rr <= ctl->eps || nn == 0) : (nn == 0);
    ctl->done = done ? 1u : 0u;
    ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
    ctl->pull = next_is_dense<ST>(nn, rr, k_sel, pull_min);  // rr: pending vertices' out-edges (min/max)
  }
}

// ---------------------------------------------------------------------------
// A2 (sampled): threshold = the rank-th largest of S sampled keys; a
// threshold of 0 (no positive sample) selects every pending vertex.
// k_sample_keys draws the S sampled keys (one thread each); k_sample then
// ranks them: ceil(S / 64) workgroups, each loading all S keys into LDS,
// whose four waves rank the same 64 samples against a quarter of the keys
// each (keys above, keys equal). The rank-th largest is the sample with
// above < rank <= above + equal; threads holding equal keys store the same
// threshold.
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void k_sample_keys(KArgs a, uint32_t S_n, uint64_t seed, uint64_t round_override) {
  if (a.score != nullptr && !a.ctl->use_score) a.score = nullptr;  // an exact round of a learned run
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S_n) return;
  const uint64_t round = round_override != ~0ull ? round_override : ctl->rounds;
  const uint64_t j = splitmix64_at(seed, round * (uint64_t)S_n + i) % a.n;
  const float sc = a.score != nullptr ? a.score[j] : 1.f;
  a.skeys[i] = (uint64_t)sel_key_loaded<ST>(a, static_cast<const S*>(a.v)[j], static_cast<const S*>(a.dv)[j], sc);
}

template <int ST>
__global__ __launch_bounds__(256) void k_sample(KArgs a, uint32_t S_n, uint32_t rank) {
  using Key = typename Tr<ST>::Key;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  __shared__ Key keys[kMaxSamples];
  __shared__ uint32_t s_above[4][64], s_equal[4][64];
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t PER = kMaxSamples / 256;
  Key kk[PER];
#pragma unroll
  for (uint32_t q = 0; q < PER; ++q) kk[q] = (Key)a.skeys[min(tid + 256 * q, S_n - 1)];
#pragma unroll
  for (uint32_t q = 0; q < PER; ++q)
    if (tid + 256 * q < S_n) keys[tid + 256 * q] = kk[q];
  __syncthreads();
  const uint32_t lane = tid & 63, wave = tid >> 6;
  const uint32_t mine_i = min(blockIdx.x * 64 + lane, S_n - 1);
  const Key mine = keys[mine_i];
  // this wave's quarter of the keys; every lane reads the same key (broadcast)
  const uint32_t quarter = (S_n + 3) / 4;
  const uint32_t i0 = min(S_n, wave * quarter), i1 = min(S_n, i0 + quarter);
  uint32_t above = 0, equal = 0, i = i0;
  for (; i + 8 <= i1; i += 8) {
    Key k[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) k[u] = keys[i + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      above += k[u] > mine ? 1u : 0u;
      equal += k[u] == mine ? 1u : 0u;
    }
  }
  for (; i < i1; ++i) {
    above += keys[i] > mine ? 1u : 0u;
    equal += keys[i] == mine ? 1u : 0u;
  }
  s_above[wave][lane] = above;
  s_equal[wave][lane] = equal;
  __syncthreads();
  if (wave != 0 || blockIdx.x * 64 + lane >= S_n) return;
  above = s_above[0][lane] + s_above[1][lane] + s_above[2][lane] + s_above[3][lane];
  equal = s_equal[0][lane] + s_equal[1][lane] + s_equal[2][lane] + s_equal[3][lane];
  if (above < rank && rank <= above + equal) {  // every such thread stores the same values
    __hip_atomic_store(&ctl->sel_mode, mine == 0 ? 0u : 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->tau, (uint64_t)mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Resets the control block at the start of a run.
static __global__ void k_init_ctl(Ctl* ctl, double eps, uint64_t max_rounds) {
  ctl->eps = eps;
  ctl->rounds = 0;
  ctl->max_rounds = max_rounds;
  ctl->activations = 0;
  ctl->pushed = 0;
  ctl->pushed_large = 0;
  ctl->round_act = 0;
  ctl->round_pushed = 0;
  ctl->round_pushed_large = 0;
  ctl->done = 0;
  ctl->stop = 0;
  ctl->ticket = 0;
  ctl->sel_mode = 0;
  ctl->tau = 0;
  ctl->radix_skip = 1;
  ctl->pull = 0;
  ctl->last_pull = 0;
  ctl->fuse_base = 0;
  ctl->use_score = 1;
  ctl->l_exact_left = 1;  // a learned run starts with one exact round (the judge's calibration)
  ctl->l_run = 0;
  ctl->l_r0 = 0.0;
  ctl->l_rounds0 = 0;
  ctl->l_gain = 0.0;
  ctl->l_exact_eff = 0.0;
  ctl->l_fallbacks = 0;
  ctl->l_exact_rounds = 0;
}

// Learned scheduling, before a round: remember the residual and decide
// whether the round ranks by the network (exact top-k while exact rounds
// are owed).
static __global__ void k_learned_pre(Ctl* ctl) {
  if (ctl_halted(ctl)) return;
  ctl->l_r0 = ctl->r;
  ctl->l_rounds0 = ctl->rounds;
  ctl->use_score = ctl->l_exact_left == 0 ? 1u : 0u;
}

// After the round: the judge's figure, the priority its updates realized
// (sum over the selected vertices of |v (+) dv - v|) per message, as a
// fraction of the residual at the round's start for sum problems (where the
// residual is that same priority mass), in value units for min/max problems
// (whose residual is a count). An exact round calibrates the judge; a
// learned round below 0.8 x the last exact round's figure hands the next
// kFallback rounds back to exact selection, and after kWindow learned rounds
// one exact round recalibrates.
template <bool SUM>
__global__ void k_learned_post(Ctl* ctl) {
  constexpr uint32_t kFallback = 4, kWindow = 16;
  if (ctl->rounds == ctl->l_rounds0) return;  // no round was run
  ctl->l_rounds0 = ctl->rounds;
  const double r0 = ctl->l_r0;
  double eff = ctl->l_gain / (double)(ctl->round_pushed > 1 ? ctl->round_pushed : 1);
  if (SUM) eff /= r0 > 1e-300 ? r0 : 1e-300;
  if (!ctl->use_score) {
    ctl->l_exact_eff = eff;
    ctl->l_exact_rounds += 1;
    if (ctl->l_exact_left > 0) ctl->l_exact_left -= 1;
    ctl->l_run = 0;
  } else if (eff < 0.8 * ctl->l_exact_eff) {
    ctl->l_exact_left = kFallback;
    ctl->l_fallbacks += 1;
  } else if (++ctl->l_run >= kWindow) {
    ctl->l_exact_left = 1;
  }
  ctl->use_score = 1;
}

// The stop flags are recomputed by the next residual.
static __global__ void k_clear_done(Ctl* ctl) {
  ctl->done = 0;
  ctl->stop = 0;
}

// Selection of every pending vertex (DAIC_SCHED_ALL).
static __global__ void k_select_all(Ctl* ctl) {
  ctl->sel_mode = 0;
  ctl->tau = 0;
}

// Round-robin: block (round mod nblocks) of `chunk` consecutive ids.
static __global__ void k_select_rr(Ctl* ctl, uint64_t nblocks) {
  if (ctl_halted(ctl)) return;
  ctl->sel_mode = 3;
  ctl->tau = ctl->rounds % nblocks;
}

// ---------------------------------------------------------------------------
// A2 (exact): radix select of the k-th largest key, kRadixBits bits per pass,
// most significant digit first. Ties at the k-th key go to the smaller ids;
// when every key equal to the k-th one fits in the k, the round selects
// key >= tau and needs no tie ranks.
// ---------------------------------------------------------------------------
constexpr int kRadixBits = 11;
constexpr uint32_t kRadixBins = 1u << kRadixBits;
// copies of the global histogram: workgroup b adds into copy b mod
// kRadixCopies, so each counter takes a fraction of the atomics
constexpr uint32_t kRadixCopies = 8;

template <typename Key>
constexpr int radix_passes() {
  return ((int)sizeof(Key) * 8 + kRadixBits - 1) / kRadixBits;
}

// Bits [shift, shift + width) form the digit of a pass; the bits above are
// fixed by the passes before it.
__device__ __forceinline__ void radix_digit(int key_bits, int pass, int& shift, int& width) {
  const int top = key_bits - kRadixBits * pass;
  shift = top > kRadixBits ? top - kRadixBits : 0;
  width = top - shift;
}

// One block of 256 threads: clears the histograms and starts the select.
static __global__ __launch_bounds__(256) void k_topk_init(Ctl* ctl, uint32_t* rhist, uint64_t k) {
  for (uint32_t i = threadIdx.x; i < kRadixBins * kRadixCopies; i += 256) rhist[i] = 0;
  if (threadIdx.x != 0 || ctl_halted(ctl)) return;
  if (ctl->pending <= k) {
    ctl->sel_mode = 0;
    ctl->radix_skip = 1;
  } else {
    ctl->sel_mode = 2;
    ctl->radix_skip = 0;
    ctl->k_rem = k;
    ctl->radix_prefix = 0;
  }
}

// One pass: every workgroup counts the digits of the keys that match the
// prefix in LDS and adds its counts into its copy of the global histogram;
// k_radix_pick then picks the digit.
template <int ST>
__global__ __launch_bounds__(256) void k_radix_pass(KArgs a, int pass) {
  if (a.score != nullptr && !a.ctl->use_score) a.score = nullptr;  // an exact round of a learned run
  using S = typename Tr<ST>::S;
  using Key = typename Tr<ST>::Key;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl) || ctl->radix_skip) return;
  constexpr int kBits = sizeof(Key) * 8;
  int shift, width;
  radix_digit(kBits, pass, shift, width);
  const Key hi_mask = pass == 0 ? (Key)0 : (Key)(~(Key)0 << (shift + width));
  const Key prefix = (Key)ctl->radix_prefix;
  const uint32_t nbins = 1u << width, dmask = nbins - 1;
  const uint32_t tid = threadIdx.x;
  __shared__ uint32_t h[kRadixBins];
  for (uint32_t i = tid; i < nbins; i += 256) h[i] = 0;
  __syncthreads();
  const S* v = static_cast<const S*>(a.v);
  const S* dv = static_cast<const S*>(a.dv);
  constexpr int U = 8;
  const uint64_t stride = (uint64_t)gridDim.x * 256 * U;
  // U keys per step, their loads in flight together
  for (uint64_t j0 = (uint64_t)blockIdx.x * 256 * U + tid; j0 < a.n; j0 += stride) {
    S vv[U], dd[U];
    float sc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t j = min(j0 + 256 * u, a.n - 1);
      vv[u] = v[j];
      dd[u] = dv[j];
      sc[u] = a.score != nullptr ? a.score[j] : 1.f;
    }
    Key k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = sel_key_loaded<ST>(a, vv[u], dd[u], sc[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j0 + 256 * u < a.n && k[u] != 0 && (k[u] & hi_mask) == prefix)
        atomicAdd(&h[(uint32_t)(k[u] >> shift) & dmask], 1u);
  }
  __syncthreads();
  uint32_t* hist = a.rhist + (blockIdx.x % kRadixCopies) * kRadixBins;
  for (uint32_t i = tid; i < nbins; i += 256) {
    const uint32_t c = h[i];
    if (c) atomicAdd(&hist[i], c);
  }
}

// After a pass (one block of 256 threads): the digit that holds the
// k_rem-th largest key, from the sum of the histogram copies (bins scanned
// from the top, 8 per thread); it is fixed in the prefix and the copies are
// cleared for the next pass.
template <int ST>
__global__ __launch_bounds__(256) void k_radix_pick(KArgs a, int pass) {
  using Key = typename Tr<ST>::Key;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl) || ctl->radix_skip) return;
  constexpr int kBits = sizeof(Key) * 8;
  int shift, width;
  radix_digit(kBits, pass, shift, width);
  const uint32_t nbins = 1u << width;
  const uint32_t tid = threadIdx.x;
  __shared__ uint32_t s_found;
  // bins from the top: thread t holds bins nbins-1-8t-q, q = 0..7
  uint32_t c[8];
  uint32_t sum[1] = {0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t r = tid * 8 + q;
    uint32_t x[kRadixCopies];
#pragma unroll
    for (uint32_t cp = 0; cp < kRadixCopies; ++cp)
      x[cp] = r < nbins ? a.rhist[cp * kRadixBins + nbins - 1 - r] : 0u;
    c[q] = 0;
#pragma unroll
    for (uint32_t cp = 0; cp < kRadixCopies; ++cp) c[q] += x[cp];
    sum[0] += c[q];
  }
  uint32_t tot[1];
  const uint32_t mine = sum[0];
  block_excl_scan<1>(sum, tot);  // sum[0] = keys in the bins above this thread's
  if (tid == 0) s_found = 0;
  __syncthreads();
  const uint64_t k = ctl->k_rem;
  if ((uint64_t)sum[0] < k && k <= (uint64_t)sum[0] + mine) {
    uint64_t cum = sum[0];
    int q = 0;
    for (; q < 7; ++q) {
      if (cum + c[q] >= k) break;
      cum += c[q];
    }
    const uint64_t d = nbins - 1 - (tid * 8 + q);
    const uint64_t rem = k - cum;
    ctl->k_rem = rem;
    ctl->radix_prefix |= d << shift;
    if (shift == 0) {
      ctl->tau = ctl->radix_prefix;
      ctl->ties_left = rem;
      ctl->sel_mode = c[q] == rem ? 1u : 2u;  // all equal keys fit: no tie ranks
    }
    s_found = 1;
  }
  __syncthreads();
  if (tid == 0 && !s_found) {  // fewer keys than k (not reached: pending > k)
    ctl->sel_mode = 0;
    ctl->radix_skip = 1;
  }
  for (uint32_t i = tid; i < nbins; i += 256)
#pragma unroll
    for (uint32_t cp = 0; cp < kRadixCopies; ++cp) a.rhist[cp * kRadixBins + i] = 0;
}

template <int ST>
__global__ __launch_bounds__(256) void k_tie_count(KArgs a) {
  if (a.score != nullptr && !a.ctl->use_score) a.score = nullptr;  // an exact round of a learned run
  using S = typename Tr<ST>::S;
  using Key = typename Tr<ST>::Key;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl) || ctl->sel_mode != 2) return;
  const Key tau = (Key)ctl->tau;
  const uint64_t lo = (uint64_t)blockIdx.x * a.per_block;
  const uint64_t hi = min(a.n, lo + a.per_block);
  const S* v = static_cast<const S*>(a.v);
  const S* dv = static_cast<const S*>(a.dv);
  uint32_t cnt = 0;
  // four vertices per step, their loads in flight together
  for (uint64_t j0 = lo + threadIdx.x; j0 < hi; j0 += 1024) {
    S vv[4], dd[4];
    float sc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t j = min(j0 + 256 * u, hi - 1);
      vv[u] = v[j];
      dd[u] = dv[j];
      sc[u] = a.score != nullptr ? a.score[j] : 1.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      cnt += (j0 + 256 * u < hi && sel_key_loaded<ST>(a, vv[u], dd[u], sc[u]) == tau) ? 1u : 0u;
  }
  cnt = block_sum256(cnt);
  if (threadIdx.x == 0) a.blk_ties[blockIdx.x] = cnt;
}

// Progress metric sum_j v_j of the current state (FP64; min problems skip
// infinite values; Kahan states report v - c), accumulated into *out.
template <int ST>
__global__ __launch_bounds__(256) void k_progress(KArgs a, double* out) {
  using S = typename Tr<ST>::S;
  const S* v = static_cast<const S*>(a.v);
  double s = 0.0;
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < a.n; j += (uint64_t)gridDim.x * 256) {
    if constexpr (ST == ST_U32) {
      if (v[j] != kInfU32) s += (double)v[j];
    } else if constexpr (ST == ST_F64MIN) {
      if (!isinf(v[j])) s += v[j];
    } else if constexpr (ST == ST_F32K) {
      s += (double)v[j] - (double)a.c[j];
    } else {
      s += (double)v[j];
    }
  }
  s = block_sum256(s);
  if (threadIdx.x == 0) atomicAdd(out, s);
}

// Exclusive prefix of per-block counts (one block of 1024 threads).
__device__ __forceinline__ void excl_prefix_1024(const uint32_t* in, uint64_t* out, uint32_t nb,
                                                 uint64_t* total) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nb; base += 1024) {
    uint32_t i = base + threadIdx.x;
    uint64_t x = i < nb ? in[i] : 0;
    // wave inclusive scan in 64 bits
    uint64_t s = x;
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint64_t y = __shfl_up(s, d, 64);
      if (lane >= (uint32_t)d) s += y;
    }
    if (lane == 63) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    uint64_t off = s_carry;
    for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) off += s_w[w];
    if (i < nb) out[i] = off + s - x;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = off + s;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[nb] = s_carry;
    if (total) *total = s_carry;
  }
}

static __global__ __launch_bounds__(1024) void k_tie_scan(KArgs a) {
  if (ctl_halted(a.ctl) || a.ctl->sel_mode != 2) return;
  excl_prefix_1024(a.blk_ties, a.off_ties, a.blocks, nullptr);
}

// ---------------------------------------------------------------------------
// A3+A4: select, claim, fold and compact into the two degree bins. Block b
// owns a fixed vertex range and writes its items into fixed regions, so no
// global atomics are needed and the item order is the vertex order.
// DRY = true only writes the selection (unit tests).
// ---------------------------------------------------------------------------
template <int ST, int G, typename RowT, bool DRY>
__global__ __launch_bounds__(256) void k_claim(KArgs a) {
  if (a.score != nullptr && !a.ctl->use_score) a.score = nullptr;  // an exact round of a learned run
  using S = typename Tr<ST>::S;
  using Key = typename Tr<ST>::Key;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const uint32_t b = blockIdx.x;
  const uint64_t lo = (uint64_t)b * a.per_block;
  const uint64_t hi = min(a.n, lo + a.per_block);
  const uint32_t mode = ctl->sel_mode;
  const Key tau = (Key)ctl->tau;
  const uint64_t ties_left = ctl->ties_left;
  const uint64_t tie_base = mode == 2 ? a.off_ties[b] : 0;
  const S* v = static_cast<const S*>(a.v);
  const S* dv = static_cast<const S*>(a.dv);
  S* small_mu = static_cast<S*>(a.small_mu);
  S* large_mu = static_cast<S*>(a.large_mu);
  const uint64_t large_base = DRY ? 0 : a.large_off[b];
  const bool pull = !DRY && ctl->pull != 0;
  uint64_t ties_seen = 0, n_small = 0, n_large = 0, act = 0, pushed = 0, pushed_large = 0;
  double gain = 0.0;  // learned runs (update rounds tracked): priority realized by the selected vertices
  const bool track = !DRY && a.last_upd != nullptr;

  // Dense rounds without tie counting (sum problems): no bins and no block
  // scans, so a thread takes four vertices per step with every load of the
  // four in flight together (the general loop below waits on each vertex).
  bool fast = false;
  if constexpr (!DRY && Tr<ST>::sum) {
    fast = pull && mode != 2;
    if (fast) {
      S* vw = static_cast<S*>(a.v);
      S* dw = static_cast<S*>(a.dv);
      S* mu_pi = static_cast<S*>(a.mu_pi);
      for (uint64_t base = lo; base < hi; base += 1024) {
        S vj[4], dj[4];
        float sc[4], cj[4];
        uint64_t r0[4], r1[4];
        uint32_t pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint64_t j = min(base + threadIdx.x + 256 * u, hi - 1);
          vj[u] = v[j];
          dj[u] = dv[j];
          sc[u] = a.score ? a.score[j] : 1.f;
          cj[u] = Tr<ST>::kahan ? a.c[j] : 0.f;
          r0[u] = row_at<RowT>(a.row, j);
          r1[u] = row_at<RowT>(a.row, j + 1);
          pj[u] = a.perm[j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint64_t j = base + threadIdx.x + 256 * u;
          if (j >= hi) break;
          Key key = prio_key<ST>(vj[u], dj[u]);
          if (a.score != nullptr && key != 0) {  // as sel_key
            const uint32_t bits = __float_as_uint(prio_value<ST>(vj[u], dj[u]) * sc[u]);
            key = (Key)(bits == 0 ? 1u : bits);
          }
          bool sel = false;
          if (key != 0) {
            if (mode == 0) sel = true;
            else if (mode == 1) sel = key >= tau;
            else sel = j / a.rr_chunk == tau;
          }
          const uint64_t deg = r1[u] - r0[u];
          bool send = false;
          S mu{};
          if (sel) {  // claim_fold with the operands read above
            const S delta = dj[u];
            dw[j] = (S)0;
            if constexpr (Tr<ST>::kahan) {
#pragma clang fp contract(off)
              const float y = delta - cj[u];
              const float t = vj[u] + y;
              a.c[j] = (t - vj[u]) - y;
              vw[j] = t;
            } else {
              vw[j] = vj[u] + delta;
            }
            double coef;
            if constexpr (G == DAIC_G_DEG_SCALE) coef = a.alpha / (double)deg;
            else coef = a.alpha_pv ? (double)static_cast<const S*>(a.alpha_pv)[j] : a.alpha;
            mu = (S)(coef * (double)delta);
            send = delta != (S)0 && deg > 0;
            if (track) {
              a.last_upd[j] = (uint32_t)ctl->rounds + 1u;
              gain += (double)prio_value<ST>(vj[u], dj[u]);
            }
          }
          if (pj[u] < a.n_src) mu_pi[pj[u]] = send ? mu : (S)0;  // no reader otherwise
          act += sel ? 1 : 0;
          pushed += send ? deg : 0;
          pushed_large += (send && deg > kSmallMaxDeg) ? deg : 0;
        }
      }
    }
  }

  for (uint64_t base = lo; base < hi && !fast; base += 256) {
    const uint64_t j = base + threadIdx.x;
    const bool in = j < hi;
    S vj{}, dj{};
    Key key = 0;
    if (in) {
      vj = v[j];
      dj = dv[j];
      key = sel_key<ST>(a, j, vj, dj);
    }
    const bool pend = key != 0;
    uint32_t tie[1] = {(mode == 2 && pend && key == tau) ? 1u : 0u};
    uint32_t tie_tot[1];
    if (mode == 2) block_excl_scan<1>(tie, tie_tot); else tie_tot[0] = 0;
    bool sel = false;
    if (pend) {
      if (mode == 0) sel = true;
      else if (mode == 1) sel = key >= tau;
      else if (mode == 2) sel = key > tau || (key == tau && tie_base + ties_seen + tie[0] < ties_left);
      else sel = j / a.rr_chunk == tau;
    }
    ties_seen += tie_tot[0];
    if constexpr (DRY) {
      if (in) a.sel_out[j] = sel ? 1 : 0;
      continue;
    }
    uint64_t beg = 0, deg = 0;
    bool send = false;
    S mu{};
    if (sel) {
      beg = row_at<RowT>(a.row, j);
      deg = row_at<RowT>(a.row, j + 1) - beg;
      send = claim_fold<ST, G>(a, j, deg, vj, dj, mu) && deg > 0;
      if (track) {
        a.last_upd[j] = (uint32_t)ctl->rounds + 1u;
        gain += (double)prio_value<ST>(vj, dj);
      }
    }
    if (pull) {  // dense round: every sender publishes its message base (the identity if silent)
      if (in) {
        const uint32_t pj = a.perm[j];
        if (pj < a.n_src) {  // no reader otherwise
          S silent;
          if constexpr (Tr<ST>::sum) silent = (S)0;
          else if constexpr (ST == ST_U32) silent = kInfU32;
          else if constexpr (ST == ST_F64MIN) silent = __builtin_huge_val();
          else silent = -1;
          static_cast<S*>(a.mu_pi)[pj] = send ? mu : silent;
        }
      }
      act += sel ? 1 : 0;
      pushed += send ? deg : 0;
      pushed_large += (send && deg > kSmallMaxDeg) ? deg : 0;
      continue;
    }
    uint32_t cnt[2] = {(send && deg <= kSmallMaxDeg) ? 1u : 0u,
                       (send && deg > kSmallMaxDeg) ? (uint32_t)((deg + kChunk - 1) / kChunk) : 0u};
    uint32_t tot[2];
    block_excl_scan<2>(cnt, tot);
    if (send) {
      if (deg <= kSmallMaxDeg) {
        uint64_t pos = lo + n_small + cnt[0];
        a.small_vid[pos] = (uint32_t)j;
        small_mu[pos] = mu;
      } else {
        uint32_t nch = (uint32_t)((deg + kChunk - 1) / kChunk);
        uint64_t pos = large_base + n_large + cnt[1];
        for (uint32_t c = 0; c < nch; ++c) {
          a.large_vid[pos + c] = (uint32_t)j;
          a.large_chunk[pos + c] = c;
          large_mu[pos + c] = mu;
        }
      }
    }
    n_small += tot[0];
    n_large += tot[1];
    act += sel ? 1 : 0;
    pushed += send ? deg : 0;
    pushed_large += (send && deg > kSmallMaxDeg) ? deg : 0;
  }
  if constexpr (!DRY) {
    act = block_sum256(act);
    pushed = block_sum256(pushed);
    pushed_large = block_sum256(pushed_large);
    if (track) {  // kernel-uniform; the residual's partial slots are free until the round's residual
      gain = block_sum256(gain);
      if (threadIdx.x == 0) a.part_r[b] = gain;
    }
    if (threadIdx.x == 0) {
      a.blk_small[b] = (uint32_t)n_small;
      a.blk_large[b] = (uint32_t)n_large;
      a.blk_act[b] = act;
      a.blk_push[b] = pushed;
      a.blk_push_large[b] = pushed_large;
    }
  }
}

// Prefix of the bin counts and the round's work counters (one block of 1024
// threads, two per-block entries per thread: every load is issued before any
// scan step, so the kernel pays one memory round trip).
static_assert(kMaxScanBlocks <= 2048, "k_bin_scan takes two per-block entries per thread");
static __global__ __launch_bounds__(1024) void k_bin_scan(KArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const uint32_t pull = ctl->pull;
  const uint32_t nb = a.blocks, tid = threadIdx.x, i0 = 2 * tid, i1 = 2 * tid + 1;
  const uint32_t lane = lane_id(), wave = tid >> 6;
  const bool learned = a.last_upd != nullptr;  // learned runs: the realized priority, summed in a fixed order
  uint32_t bs[2] = {0, 0}, bl[2] = {0, 0};
  uint64_t act = 0, push = 0, pl = 0;
  double g = 0.0;
#pragma unroll
  for (uint32_t u = 0; u < 2; ++u) {
    const uint32_t i = i0 + u;
    if (i < nb) {
      bs[u] = a.blk_small[i];
      bl[u] = a.blk_large[i];
      act += a.blk_act[i];
      push += a.blk_push[i];
      pl += a.blk_push_large[i];
      if (learned) g += a.part_r[i];
    }
  }
  const uint64_t xs = (uint64_t)bs[0] + bs[1], xl = (uint64_t)bl[0] + bl[1];
  uint64_t ss = xs, sl = xl;  // wave inclusive scans
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t ys = __shfl_up(ss, d, 64), yl = __shfl_up(sl, d, 64);
    if (lane >= (uint32_t)d) {
      ss += ys;
      sl += yl;
    }
  }
  act = wave_sum(act);
  push = wave_sum(push);
  pl = wave_sum(pl);
  g = wave_sum(g);
  __shared__ uint64_t w_s[16], w_l[16], w_a[16], w_p[16], w_pl[16];
  __shared__ double w_g[16];
  if (lane == 63) {
    w_s[wave] = ss;
    w_l[wave] = sl;
    w_a[wave] = act;
    w_p[wave] = push;
    w_pl[wave] = pl;
    w_g[wave] = g;
  }
  __syncthreads();
  if (!pull) {  // the bins feed the push kernels only
    uint64_t os = 0, ol = 0;
    for (uint32_t w = 0; w < wave; ++w) {
      os += w_s[w];
      ol += w_l[w];
    }
    const uint64_t es = os + ss - xs, el = ol + sl - xl;
    if (i0 < nb) {
      a.off_small[i0] = es;
      a.off_large[i0] = el;
    }
    if (i1 < nb) {
      a.off_small[i1] = es + bs[0];
      a.off_large[i1] = el + bl[0];
    }
  }
  if (tid == 0) {
    uint64_t ts = 0, tl = 0, ta = 0, tp = 0, tpl = 0;
    double tg = 0.0;
    for (int w = 0; w < 16; ++w) {
      ts += w_s[w];
      tl += w_l[w];
      ta += w_a[w];
      tp += w_p[w];
      tpl += w_pl[w];
      tg += w_g[w];
    }
    ctl->last_pull = pull;
    if (!pull) {
      a.off_small[nb] = ts;
      a.off_large[nb] = tl;
    }
    ctl->n_small = pull ? 0 : ts;
    ctl->n_large = pull ? 0 : tl;
    if (learned) ctl->l_gain = tg;
    ctl->activations += ta;
    ctl->pushed += tp;
    ctl->pushed_large += tpl;
    ctl->round_act = ta;
    ctl->round_pushed = tp;
    ctl->round_pushed_large = tpl;
  }
}

// ---------------------------------------------------------------------------
// A5, small bin (out-degree 1..32): one wave (= one block of 64) takes 64
// items and spreads their concatenated edges over its lanes, so lanes stay
// busy whatever the degree mix and column reads stay contiguous.
// ---------------------------------------------------------------------------
template <int ST, int G, typename RowT>
__device__ __forceinline__ void push_small_items(const KArgs& a, uint64_t bid, uint64_t nb) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  const uint64_t total = ctl->n_small;
  __shared__ uint8_t owner[64 * kSmallMaxDeg];
  __shared__ uint32_t s_excl[64];
  __shared__ uint64_t s_beg[64];
  __shared__ S s_mu[64];
  const uint32_t lane = threadIdx.x;
  const S* small_mu = static_cast<const S*>(a.small_mu);
  for (uint64_t g = bid; g * 64 < total; g += nb) {
    const uint64_t i = g * 64 + lane;
    uint32_t deg = 0;
    uint64_t beg = 0;
    S mu{};
    if (i < total) {
      uint32_t blk = find_block(a.off_small, a.blocks, i);
      uint64_t idx = (uint64_t)blk * a.per_block + (i - a.off_small[blk]);
      uint32_t vid = a.small_vid[idx];
      mu = small_mu[idx];
      beg = row_at<RowT>(a.row, vid);
      deg = (uint32_t)(row_at<RowT>(a.row, vid + 1) - beg);
    }
    const uint32_t incl = wave_incl_scan(deg);
    const uint32_t excl = incl - deg;
    const uint32_t E = __shfl(incl, 63, 64);
    s_excl[lane] = excl;
    s_beg[lane] = beg;
    s_mu[lane] = mu;
    for (uint32_t k = 0; k < deg; ++k) owner[excl + k] = (uint8_t)lane;
    __syncthreads();
    for (uint32_t e = lane; e < E; e += 64) {
      const uint32_t o = owner[e];
      push_edge<ST, G>(a, s_beg[o] + (e - s_excl[o]), s_mu[o]);
    }
    __syncthreads();
  }
}

// A5, large bin: one wave per item of up to kChunk consecutive out-edges.
template <int ST, int G, typename RowT>
__device__ __forceinline__ void push_large_items(const KArgs& a, uint64_t bid, uint64_t nb) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  const uint64_t total = ctl->n_large;
  const S* large_mu = static_cast<const S*>(a.large_mu);
  for (uint64_t i = bid; i < total; i += nb) {
    uint32_t blk = find_block(a.off_large, a.blocks, i);
    uint64_t idx = a.large_off[blk] + (i - a.off_large[blk]);
    uint32_t vid = a.large_vid[idx];
    uint32_t ch = a.large_chunk[idx];
    S mu = large_mu[idx];
    uint64_t rb = row_at<RowT>(a.row, vid);
    uint64_t re = row_at<RowT>(a.row, vid + 1);
    uint64_t beg = rb + (uint64_t)ch * kChunk;
    uint64_t end = min(re, beg + kChunk);
    for (uint64_t e = beg + threadIdx.x; e < end; e += 64) push_edge<ST, G>(a, e, mu);
  }
}

// A5: both bins in one launch, the first small_blocks one-wave workgroups on
// the small bin and the others on the large bin.
template <int ST, int G, typename RowT>
__global__ __launch_bounds__(64) void k_push(KArgs a, uint32_t small_blocks) {
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl) || ctl->pull) return;
  if (blockIdx.x < small_blocks) push_small_items<ST, G, RowT>(a, blockIdx.x, small_blocks);
  else push_large_items<ST, G, RowT>(a, blockIdx.x - small_blocks, gridDim.x - small_blocks);
}

// ---------------------------------------------------------------------------
// Dense rounds: the receive side of Eq. async done by the receiver. Every
// target sums the message bases of its in-neighbours (0 for silent ones) and
// adds the sum to dv. Sums are formed in FP64.
// ---------------------------------------------------------------------------
// Streamed pull: the in-edges are cut into blocks of at most kStreamEdges
// consecutive in-edges covering whole targets (a target with more in-edges
// is cut into pieces of its own). A workgroup of 256 threads reads a block's
// sources with consecutive lanes, gathers the messages into LDS, then every
// thread sums its run of kStreamEdges/256 consecutive values per target it
// meets, adding into per-target LDS accumulators (FP64). Targets wholly
// inside the block are written once; pieces of a cut target add atomically.
// msg(source, in-edge) returns the message carried by an in-edge.
// Gathers one block's messages and sums them per target. On return (after a
// barrier) acc[i] holds the FP64 sum of target t0 + i and off[0..nr] the
// block-relative in-edge offsets, clipped to [0, ne]. A block may have no
// in-edges (then every sum is 0).
// tid is the thread's index in its group of 256 (a workgroup of 1024 runs
// four groups on four blocks; every thread of the workgroup reaches both
// barriers).
template <typename V, typename Msg>
__device__ __forceinline__ void stream_sums(const uint32_t* rowT, const uint32_t* srcT, uint32_t t0, uint32_t nr,
                                            uint32_t e0, uint32_t e1, V* vals, double* acc, uint32_t* off,
                                            const Msg& msg, const uint32_t tid) {
  constexpr uint32_t PER = kStreamEdges / 256, ROFF = (kStreamRows + 256) / 256;
  const uint32_t ne = e1 - e0;
  // every independent load first, at clamped indices (no branch around
  // them, so they are in flight together): row offsets and sources
  uint32_t ro[ROFF];
#pragma unroll
  for (uint32_t k = 0; k < ROFF; ++k) ro[k] = rowT[t0 + min(tid + 256 * k, nr)];
  if (ne > 0) {  // uniform over the workgroup
    uint32_t src[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) src[j] = srcT[e0 + min(tid + 256 * j, ne - 1)];
    V val[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) val[j] = msg(src[j], e0 + min(tid + 256 * j, ne - 1));
    // lanes past the block's end store 0
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) vals[tid + 256 * j] = tid + 256 * j < ne ? val[j] : (V)0;
  }
#pragma unroll
  for (uint32_t k = 0; k < ROFF; ++k) {
    const uint32_t i = tid + 256 * k;
    if (i <= nr) off[i] = ro[k] <= e0 ? 0u : min(ro[k] - e0, ne);
    if (i < nr) acc[i] = 0.0;
  }
  __syncthreads();
  // this thread's run [q0, q1) of the block's values
  const uint32_t q0 = min(tid * PER, ne), q1 = min(q0 + PER, ne);
  if (q0 < q1) {
    uint32_t lo = 0, hi = nr - 1;  // last row i with off[i] <= q0
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= q0) lo = mid;
      else hi = mid - 1;
    }
    uint32_t i = lo, next = off[i + 1];
    double sum = 0.0;
    for (uint32_t q = q0; q < q1; ++q) {
      while (q >= next) {  // row i ends before q
        if (sum != 0.0) atomicAdd(&acc[i], sum);
        sum = 0.0;
        ++i;
        next = off[i + 1];
      }
      sum += (double)vals[q];
    }
    atomicAdd(&acc[i], sum);
  }
  __syncthreads();
}

template <typename S, typename V, typename Msg>
__device__ __forceinline__ void stream_block(const uint32_t* rowT, const uint32_t* srcT, S* dv, uint32_t t0,
                                             uint32_t nr, uint32_t e0, uint32_t e1, V* vals, double* acc,
                                             uint32_t* off, const Msg& msg) {
  constexpr uint32_t RDV = kStreamRows / 256;
  const uint32_t tid = threadIdx.x;
  // dv of this thread's targets, read early (only this workgroup writes a
  // whole target's dv)
  S dvp[RDV];
#pragma unroll
  for (uint32_t k = 0; k < RDV; ++k) dvp[k] = dv[t0 + min(tid + 256 * k, nr - 1)];
  stream_sums<V>(rowT, srcT, t0, nr, e0, e1, vals, acc, off, msg, threadIdx.x);
  // several targets: all whole; one target: whole or a piece
  const bool piece = nr == 1 && (rowT[t0] != e0 || rowT[t0 + 1] != e1);
#pragma unroll
  for (uint32_t k = 0; k < RDV; ++k) {
    const uint32_t i = tid + 256 * k;
    if (i >= nr || off[i + 1] == off[i]) continue;  // beyond the block, or no in-edges
    const uint32_t t = t0 + i;
    if (!piece) dv[t] = (S)((double)dvp[k] + acc[i]);
    else unsafeAtomicAdd(&dv[t], (S)acc[i]);
  }
  __syncthreads();
}

// Dense round by streamed blocks (Eq. sync over the in-edges): message of an
// in-edge = the source's base (times the edge weight for EDGE_SCALE). Every
// vertex is in one edge block, so each workgroup also stores the residual
// partials (sum of |dv| and pending count) of the vertices it finished;
// cut targets and the round's totals are left to k_pull_finish.
template <int ST, int G>
__global__ __launch_bounds__(256) void k_pull_stream(KArgs a) {
  using S = typename Tr<ST>::S;
  if constexpr (Tr<ST>::sum) {
    constexpr uint32_t RDV = kStreamRows / 256;
    Ctl* ctl = a.ctl;
    uint64_t b = blockIdx.x;
    if (b >= a.sb_count) {  // only with an empty block table (grid of one)
      if (threadIdx.x == 0) {
        a.fpart_r[b] = 0.0;
        a.fpart_a[b] = 0;
      }
      return;
    }
    // the first block's descriptors are read together with the control block
    uint32_t t0 = a.sb_t[b], nr = a.sb_n[b], e0 = a.sb_e[b], e1 = a.sb_e[b + 1], grp = a.sb_g[b];
    if (ctl_halted(ctl) || !ctl->pull) return;
    using V = typename std::conditional<G == DAIC_G_EDGE_SCALE, double, S>::type;
    __shared__ V vals[kStreamEdges];
    __shared__ double acc[kStreamRows];
    __shared__ uint32_t off[kStreamRows + 1];
    const uint32_t tid = threadIdx.x;
    const S* mu = static_cast<const S*>(a.mu_pi);
    const S* wT = static_cast<const S*>(a.wT);
    S* dv = static_cast<S*>(a.dv);
    auto msg = [&](uint32_t src, uint32_t p) -> V {
      V m = (V)mu[src];
      if constexpr (G == DAIC_G_EDGE_SCALE) m *= (V)wT[p];
      return m;
    };
    double r_part = 0.0;
    uint64_t pend = 0;
    for (;;) {
      S dvp[RDV];
#pragma unroll
      for (uint32_t q = 0; q < RDV; ++q) dvp[q] = dv[t0 + min(tid + 256 * q, nr - 1)];
      stream_sums<V>(a.rowT, a.srcT, t0, nr, e0, e1, vals, acc, off, msg, threadIdx.x);
      if (grp == 0xFFFFFFFFu) {  // whole targets
#pragma unroll
        for (uint32_t q = 0; q < RDV; ++q) {
          const uint32_t i = tid + 256 * q;
          if (i >= nr) continue;
          S d = dvp[q];
          if (off[i + 1] != off[i]) {  // in-edges
            d = (S)((double)dvp[q] + acc[i]);
            dv[t0 + i] = d;
          }
          r_part += fabs((double)d);
          pend += d != (S)0 ? 1 : 0;
        }
      } else if (tid == 0) {  // a piece of a cut target
        unsafeAtomicAdd(&dv[t0], (S)acc[0]);
      }
      __syncthreads();
      b += gridDim.x;
      if (b >= a.sb_count) break;
      t0 = a.sb_t[b];
      nr = a.sb_n[b];
      e0 = a.sb_e[b];
      e1 = a.sb_e[b + 1];
      grp = a.sb_g[b];
    }
    r_part = block_sum256(r_part);
    pend = block_sum256(pend);
    if (tid == 0) {
      a.fpart_r[blockIdx.x] = r_part;
      a.fpart_a[blockIdx.x] = pend;
    }
  }
}

// After a dense round's k_pull_stream (nf workgroups): the residual of the
// round's end state as k_residual computes it (sum of |dv| in FP64, pending
// count, round count, stop rule, direction of the next round), from the
// pull's partials and the cut targets' final dv; the last block to finish
// adds the per-block partials in a fixed order.
template <int ST>
__global__ __launch_bounds__(256) void k_pull_finish(KArgs a, uint32_t nf, uint64_t k_sel, uint64_t pull_min) {
  using S = typename Tr<ST>::S;
  if constexpr (Tr<ST>::sum) {
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl) || !ctl->last_pull) return;
    __shared__ uint32_t s_last;
    const uint32_t tid = threadIdx.x;
    double r = 0.0;
    uint64_t cnt = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + tid; i < nf; i += (uint64_t)gridDim.x * 256) {
      r += a.fpart_r[i];  // written by the previous kernel
      cnt += a.fpart_a[i];
    }
    const uint64_t g = (uint64_t)blockIdx.x * 256 + tid;
    if (g < a.n_groups) {
      const double x = fabs((double)static_cast<const S*>(a.dv)[a.sb_t[a.g_first[g]]]);
      r += x;
      cnt += x > 0.0 ? 1 : 0;
    }
    r = block_sum256(r);
    cnt = block_sum256(cnt);
    if (tid == 0) {
      a.gpart_r[blockIdx.x] = r;
      a.gpart_a[blockIdx.x] = cnt;
      __threadfence();
      s_last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double rr = 0.0;
    uint64_t nn = 0;
    for (uint32_t i = tid; i < gridDim.x; i += 256) {
      rr += __hip_atomic_load(&a.gpart_r[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      nn += __hip_atomic_load(&a.gpart_a[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    rr = block_sum256(rr);
    nn = block_sum256(nn);
    if (tid == 0) {
      ctl->r = rr;
      ctl->pending = nn;
      ctl->rounds += 1;
      const bool done = rr <= ctl->eps || nn == 0;
      ctl->done = done ? 1u : 0u;
      ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
      ctl->pull = (k_sel != 0 && (nn < k_sel ? nn : k_sel) >= pull_min) ? 1u : 0u;
      ctl->ticket = 0;
    }
  }
}

// Fused dense round (sum problems, every pending vertex updated each round).
// Round r of Eq. sync claims the deltas left by round r - 1 (folds them into
// v and sends their messages) and pulls those messages into new deltas. Here
// one kernel does round r's pull and, for each target right after its sum
// is known, the claim work that does not change round r's messages: it folds
// the target's previous delta into v and publishes the message base of its
// new delta into the other buffer (A and B alternate by round), to be pulled
// by round r + 1. After the round, (v, dv) is exactly the state after round
// r, and the bases in flight are those round r + 1 would send. The kernel
// only stores (no atomics, no fences): a piece of a cut target stores its
// partial sum, every workgroup stores its partial residual and counters, and
// k_fused_finish completes the cut targets and the round's totals.
template <int ST, int G>
struct FusedTarget {
  using S = typename Tr<ST>::S;
  // target t: fold its previous delta d_old into v (Kahan when the state
  // has the compensation term: the claim of Eq. sync), keep the new delta
  // d_new in dv and publish its message base into mu_out
  static __device__ __forceinline__ void finish(const KArgs& a, S* mu_out, uint32_t t, S d_old, S d_new, S vt,
                                                float ct, uint32_t deg, uint32_t pt, double& r_part, uint64_t& act,
                                                uint64_t& pushed) {
    S* v = static_cast<S*>(a.v);
    if (d_old != (S)0) {
      if constexpr (Tr<ST>::kahan) {
#pragma clang fp contract(off)
        const float y = d_old - ct;
        const float tt = vt + y;
        a.c[t] = (tt - vt) - y;
        v[t] = tt;
      } else {
        v[t] = vt + d_old;
      }
      act += 1;
      pushed += deg;
    }
    if (d_new != d_old) static_cast<S*>(a.dv)[t] = d_new;
    r_part += fabs((double)d_new);
    if (pt < a.n_src) {
      double coef;
      if constexpr (G == DAIC_G_DEG_SCALE) coef = a.alpha / (double)max(deg, 1u);
      else coef = a.alpha_pv ? (double)static_cast<const S*>(a.alpha_pv)[t] : a.alpha;
      mu_out[pt] = (d_new != (S)0 && deg > 0) ? (S)(coef * (double)d_new) : (S)0;
    }
  }
};

template <int ST, int G>
__global__ __launch_bounds__(256) void k_pull_fused(KArgs a) {
  using S = typename Tr<ST>::S;
  if constexpr (Tr<ST>::sum) {
    constexpr uint32_t RDV = kStreamRows / 256;
    Ctl* ctl = a.ctl;
    uint64_t b = blockIdx.x;  // the grid never exceeds the block count
    uint32_t t0 = a.sb_t[b], nr = a.sb_n[b], e0 = a.sb_e[b], e1 = a.sb_e[b + 1], grp = a.sb_g[b];
    if (ctl_halted(ctl)) return;
    using V = typename std::conditional<G == DAIC_G_EDGE_SCALE, double, S>::type;
    __shared__ V vals[kStreamEdges];
    __shared__ double acc[kStreamRows];
    __shared__ uint32_t off[kStreamRows + 1];
    const uint32_t tid = threadIdx.x;
    const bool odd = ((ctl->rounds - ctl->fuse_base) & 1) != 0;
    const S* mu_in = static_cast<const S*>(odd ? a.mu_pi2 : a.mu_pi);
    S* mu_out = static_cast<S*>(odd ? a.mu_pi : a.mu_pi2);
    const S* wT = static_cast<const S*>(a.wT);
    const uint32_t* row = static_cast<const uint32_t*>(a.row);
    const S* dv = static_cast<const S*>(a.dv);
    const S* v = static_cast<const S*>(a.v);
    auto msg = [&](uint32_t src, uint32_t p) -> V {
      V m = (V)mu_in[src];
      if constexpr (G == DAIC_G_EDGE_SCALE) m *= (V)wT[p];
      return m;
    };
    double r_part = 0.0;
    uint64_t act = 0, pushed = 0;
    for (;;) {
      S dvp[RDV], vp[RDV];
      float cp[RDV];
      uint32_t dg[RDV], pp[RDV];
      if (grp == 0xFFFFFFFFu) {  // uniform: whole targets; their operands are read early
#pragma unroll
        for (uint32_t k = 0; k < RDV; ++k) {
          const uint32_t t = t0 + min(tid + 256 * k, nr - 1);
          dvp[k] = dv[t];
          vp[k] = v[t];
          cp[k] = Tr<ST>::kahan ? a.c[t] : 0.f;
          dg[k] = row[t + 1] - row[t];
          pp[k] = a.perm[t];
        }
      }
      stream_sums<V>(a.rowT, a.srcT, t0, nr, e0, e1, vals, acc, off, msg, threadIdx.x);
      if (grp == 0xFFFFFFFFu) {
#pragma unroll
        for (uint32_t k = 0; k < RDV; ++k) {
          const uint32_t i = tid + 256 * k;
          if (i < nr)
            FusedTarget<ST, G>::finish(a, mu_out, t0 + i, dvp[k], (S)acc[i], vp[k], cp[k], dg[k], pp[k], r_part,
                                       act, pushed);
        }
      } else if (tid == 0) {
        a.sb_part[b] = acc[0];  // a piece of a cut target
      }
      __syncthreads();
      b += gridDim.x;
      if (b >= a.sb_count) break;
      t0 = a.sb_t[b];
      nr = a.sb_n[b];
      e0 = a.sb_e[b];
      e1 = a.sb_e[b + 1];
      grp = a.sb_g[b];
    }
    r_part = block_sum256(r_part);
    act = block_sum256(act);
    pushed = block_sum256(pushed);
    if (tid == 0) {
      a.fpart_r[blockIdx.x] = r_part;
      a.fpart_a[blockIdx.x] = act;
      a.fpart_p[blockIdx.x] = pushed;
    }
  }
}

// After k_pull_fused (nf of its workgroups): one thread per cut target sums
// the target's pieces in order and finishes it, and the blocks add up the
// partials of k_pull_fused; the last block to finish adds the per-block
// partials in a fixed order and updates the control block (residual,
// counters, round count, stop rule).
template <int ST, int G>
__global__ __launch_bounds__(256) void k_fused_finish(KArgs a, uint32_t nf) {
  using S = typename Tr<ST>::S;
  if constexpr (Tr<ST>::sum) {
    Ctl* ctl = a.ctl;
    if (ctl_halted(ctl)) return;
    __shared__ uint32_t s_last;
    const uint32_t tid = threadIdx.x;
    const bool odd = ((ctl->rounds - ctl->fuse_base) & 1) != 0;
    S* mu_out = static_cast<S*>(odd ? a.mu_pi : a.mu_pi2);
    const uint32_t* row = static_cast<const uint32_t*>(a.row);
    double r_part = 0.0;
    uint64_t act = 0, pushed = 0;
    // the partials of k_pull_fused, spread over this grid (written by the
    // previous kernel)
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + tid; i < nf; i += (uint64_t)gridDim.x * 256) {
      r_part += a.fpart_r[i];
      act += a.fpart_a[i];
      pushed += a.fpart_p[i];
    }
    const uint64_t g = (uint64_t)blockIdx.x * 256 + tid;
    if (g < a.n_groups) {
      const uint32_t b0 = a.g_first[g], np = a.g_np[g];
      // the pieces' partials in order, 32 loads in flight at a time (a hub
      // has hundreds of pieces; one load per step would make its thread the
      // kernel's critical path)
      double sum = 0.0;
      for (uint32_t k0 = 0; k0 < np; k0 += 32) {
        double x[32];
#pragma unroll
        for (uint32_t u = 0; u < 32; ++u) x[u] = a.sb_part[b0 + min(k0 + u, np - 1)];
#pragma unroll
        for (uint32_t u = 0; u < 32; ++u)
          if (k0 + u < np) sum += x[u];
      }
      const uint32_t t = a.sb_t[b0];
      FusedTarget<ST, G>::finish(a, mu_out, t, static_cast<const S*>(a.dv)[t], (S)sum, static_cast<const S*>(a.v)[t],
                                 Tr<ST>::kahan ? a.c[t] : 0.f, row[t + 1] - row[t], a.perm[t], r_part, act, pushed);
    }
    r_part = block_sum256(r_part);
    act = block_sum256(act);
    pushed = block_sum256(pushed);
    if (tid == 0) {
      a.gpart_r[blockIdx.x] = r_part;
      a.gpart_a[blockIdx.x] = act;
      a.gpart_p[blockIdx.x] = pushed;
      __threadfence();
      s_last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double rr = 0.0;
    uint64_t aa = 0, ps = 0;
    for (uint32_t i = tid; i < gridDim.x; i += 256) {
      rr += __hip_atomic_load(&a.gpart_r[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      aa += __hip_atomic_load(&a.gpart_a[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ps += __hip_atomic_load(&a.gpart_p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    rr = block_sum256(rr);
    aa = block_sum256(aa);
    ps = block_sum256(ps);
    if (tid == 0) {
      ctl->r = rr;
      ctl->rounds += 1;
      ctl->activations += aa;
      ctl->pushed += ps;
      ctl->round_act = aa;
      ctl->round_pushed = ps;
      const bool done = rr <= ctl->eps;
      ctl->done = done ? 1u : 0u;
      ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
      ctl->ticket = 0;
    }
  }
}

// Start of fused dense rounds: the bases just published went to buffer A.
static __global__ void k_fuse_begin(Ctl* ctl) { ctl->fuse_base = ctl->rounds; }

// Weights in in-edge order: wT[p] = w[eidT[p]] for p < m, 0 up to total
// (the padding of the tiled arrays).
template <typename S>
__global__ void k_gather_weights(const S* w, const uint32_t* eidT, uint64_t m, uint64_t total, S* wT) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (; i < total; i += st) wT[i] = i < m ? w[eidT[i]] : (S)0;
}

// ---------------------------------------------------------------------------
// Set-up kernels.
// ---------------------------------------------------------------------------
// Per-block capacity of the large bin: the chunks of every vertex of the
// block's range whose degree exceeds the small-bin bound.
template <typename RowT>
__global__ __launch_bounds__(256) void k_large_capacity(const void* row, uint64_t n, uint64_t per_block,
                                                        uint64_t* cap) {
  const uint64_t lo = (uint64_t)blockIdx.x * per_block;
  const uint64_t hi = min(n, lo + per_block);
  uint64_t c = 0;
  for (uint64_t j = lo + threadIdx.x; j < hi; j += 256) {
    uint64_t d = row_at<RowT>(row, j + 1) - row_at<RowT>(row, j);
    if (d > kSmallMaxDeg) c += (d + kChunk - 1) / kChunk;
  }
  c = block_sum256(c);
  if (threadIdx.x == 0) cap[blockIdx.x] = c;
}

}  // namespace daic
