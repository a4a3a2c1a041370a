// Sweep scheduling for sum problems: round-robin over blocks of ceil(q n)
// consecutive vertex ids. A round handles one block: each vertex of the block
// receives, by a pull over its in-edges, the newest message base of every
// in-neighbour, then folds the sum into its state and publishes its own
// message base. Blocks later in a sweep therefore see the updates made
// earlier in it, an asynchronous activation order (Eq. async) that Theorem 1
// allows; with a single block (q = 1) it is the synchronous round.
//
// Numbering. Message bases are stored by a sweep numbering of the sources:
// block-major (block c owns numbers [c B, c B + |block c|)) and, inside a
// block, by out-degree descending, so that a source's block follows from its
// number and the hot senders of a block share cache lines.
//
// Exactly-once delivery. Message bases live in two slots per vertex, chosen
// by the parity of the sweep that published them. When block c of sweep k
// runs, an in-neighbour numbered s < c B has published in sweep k (slot
// k mod 2) and its previous base was consumed by this target in sweep k - 1;
// an in-neighbour at s >= c B (this block included) last published in sweep
// k - 1 (slot (k - 1) mod 2), after this target's pull of sweep k - 1. Either
// way the target reads exactly the one base it has not consumed. Every
// vertex of the block writes its slot each sweep (0 when silent), so a slot
// never holds a base older than the previous sweep.
//
// Residual. After a whole sweep the messages not yet consumed are those of
// every source s to its out-neighbours in blocks up to its own, so
// sum_s |mu_s| * sum_{t in out(s), block(t) <= block(s)} |w_st| bounds the
// pending L1 mass (with equality for non-negative messages, e.g. PageRank);
// the sweep stops when that bound is <= eps. A final pass delivers the
// messages still in flight into dv, after which the exact residual is taken.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "daic_device.h"
#include "daic_problem.h"

namespace daic {

struct SweepArgs {
  Ctl* ctl;
  uint64_t n;
  uint64_t B;                 // positions per block
  uint32_t P;                 // blocks per sweep
  const uint32_t* row;        // out-edge offsets [n+1]
  const uint32_t* rowT;       // in-edge offsets [n+1]
  const uint32_t* srcT;       // sweep number of the source of each in-edge
  const uint32_t* perm;       // sweep number of each vertex
  const void* wT;             // S[m] weights in in-edge order (EDGE_SCALE)
  void* v;
  void* dv;
  float* c;                   // Kahan term or null
  const void* alpha_pv;
  double alpha;
  void* mu2;                  // S[2n]: slot 0 then slot 1, by position
  const uint32_t* voff;       // [P+1]: block c owns ids [voff[c], voff[c+1])
  const uint32_t* sb_t;       // edge blocks of the streamed pull, cut at block boundaries:
  const uint32_t* sb_e;       //   first target, first in-edge (closing entry m),
  const uint32_t* sb_n;       //   targets covered
  const uint32_t* rv;         // vertices with in-edges, grouped by block, ids ascending
  const uint32_t* roff;       // [P+1]
  const double* coef_le;      // [n] by position: sum of |w| to out-neighbours in blocks <= own
  double* part_r;             // residual partials per grid block
  uint64_t* part_n;
  uint64_t* part_a;           // claim partials per grid block: activations, messages
  uint64_t* part_m;
  uint32_t claim_blocks;      // grid of k_sweep_claim
};

struct SweepState {
  uint64_t B = 0;
  uint32_t P = 0;
  uint64_t max_block_verts = 0;
  std::vector<uint32_t> block_sb_off;  // [P+1]: edge blocks of block c
  uint64_t sb_total = 0;           // edge blocks of all blocks
  // the tiled in-edges with sources in sweep numbers (when B is a multiple of
  // a partition width of at least 256): block c's tiles and split partitions
  TileGraph tiles;
  TileArgs ta{};
  std::vector<uint32_t> tile_off, split_off;  // [P+1]
  std::vector<void*> allocs;
  SweepArgs a{};
  // targets numbered by in-degree octave within each block (the tiles'
  // numbering): the block pulls take `ar`, whose state, out-edge offsets,
  // sweep numbers (and per-vertex alpha) are in that order; the state moves
  // there for the run's sweeps and back before the final delivery
  bool numbered = false;
  SweepArgs ar{};
};

namespace {

constexpr uint32_t kResGrid = 2048;
constexpr uint32_t kSweepFinishGrid = 2048;  // workgroups of k_sweep_tile_finish (at most)

// Block c: streamed pull of the block's targets. An in-edge from a source
// at position s reads the base published in this sweep when s lies in an
// earlier block (s < c B), else the base of the previous sweep.
template <int ST, int G>
__global__ __launch_bounds__(256) void k_sweep_stream(SweepArgs a, uint32_t c, uint32_t b_begin, uint32_t b_end) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  uint64_t b = b_begin + blockIdx.x;
  if (b >= b_end) return;
  // the first edge block's descriptors are read together with the control block
  uint32_t t0 = a.sb_t[b], nr = a.sb_n[b], e0 = a.sb_e[b], e1 = a.sb_e[b + 1];
  if (ctl_halted(ctl)) return;
  using V = typename std::conditional<G == DAIC_G_EDGE_SCALE, double, S>::type;
  __shared__ V vals[kStreamEdges];
  __shared__ double acc[kStreamRows];
  __shared__ uint32_t off[kStreamRows + 1];
  const uint64_t k = ctl->rounds / a.P;
  const uint64_t cur = (k & 1) * a.n, prev = ((k + 1) & 1) * a.n, lo = (uint64_t)c * a.B;
  const S* mu2 = static_cast<const S*>(a.mu2);
  const S* wT = static_cast<const S*>(a.wT);
  auto msg = [&](uint32_t src, uint32_t p) -> V {
    V m = (V)mu2[(src < lo ? cur : prev) + src];
    if constexpr (G == DAIC_G_EDGE_SCALE) m *= (V)wT[p];
    return m;
  };
  for (;;) {
    stream_block<S, V>(a.rowT, a.srcT, static_cast<S*>(a.dv), t0, nr, e0, e1, vals, acc, off, msg);
    b += gridDim.x;
    if (b >= b_end) break;
    t0 = a.sb_t[b];
    nr = a.sb_n[b];
    e0 = a.sb_e[b];
    e1 = a.sb_e[b + 1];
  }
}

// The claim of vertex j in its block's round: d = its delta with this
// round's received sum included (dv_old is the delta before the pull). A
// nonzero delta is folded into v (Kahan for the compensated state) and its
// message base published into the slot of this sweep (0 when silent; only
// vertices with out-edges have readers).
template <int ST, int G>
__device__ __forceinline__ void sweep_claim_vertex(const SweepArgs& a, uint32_t j, typename Tr<ST>::S d,
                                                   typename Tr<ST>::S dv_old, uint64_t cur, uint64_t& act,
                                                   uint64_t& pushed) {
  using S = typename Tr<ST>::S;
  S* mu2 = static_cast<S*>(a.mu2);
  S* v = static_cast<S*>(a.v);
  S* dv = static_cast<S*>(a.dv);
  const uint32_t deg = a.row[j + 1] - a.row[j];
  S mu = (S)0;
  if (d != (S)0) {
    dv[j] = (S)0;
    const S vj = v[j];
    if constexpr (Tr<ST>::kahan) {
      // compensated fold (Kahan 1965), as in the round kernels
#pragma clang fp contract(off)
      const float cj = a.c[j];
      const float y = d - cj;
      const float t = vj + y;
      a.c[j] = (t - vj) - y;
      v[j] = t;
    } else {
      v[j] = vj + d;
    }
    double coef;
    if constexpr (G == DAIC_G_DEG_SCALE) {
      coef = deg ? a.alpha / (double)deg : 0.0;
    } else {
      coef = a.alpha_pv ? (double)static_cast<const S*>(a.alpha_pv)[j] : a.alpha;
    }
    mu = (S)(coef * (double)d);
    act += 1;
    pushed += deg;
  } else if (dv_old != (S)0) {
    dv[j] = (S)0;  // the received sum cancelled the delta
  }
  if (deg) mu2[cur + a.perm[j]] = mu;
}

// Block c: fold the received sum (dv, filled by k_sweep_stream) into the
// state and publish the message base. Vertices without in-edges receive
// nothing, so after their claim of the first sweep and the clearing of both
// slots (sweeps 1 and 2) they are skipped.
template <int ST, int G>
__global__ __launch_bounds__(256) void k_sweep_claim(SweepArgs a, uint32_t c) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const uint64_t k = ctl->rounds / a.P;
  const uint64_t cur = (k & 1) * a.n;
  const S* dv = static_cast<const S*>(a.dv);
  const bool all = k < 3;
  const uint64_t vb = all ? a.voff[c] : a.roff[c], ve = all ? a.voff[c + 1] : a.roff[c + 1];
  uint64_t act = 0, pushed = 0;
  for (uint64_t i = vb + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ve;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = all ? (uint32_t)i : a.rv[i];
    const S d = dv[j];
    sweep_claim_vertex<ST, G>(a, j, d, d, cur, act, pushed);
  }
  act = block_sum256(act);
  pushed = block_sum256(pushed);
  if (threadIdx.x == 0) {
    a.part_a[blockIdx.x] = act;
    a.part_m[blockIdx.x] = pushed;
  }
}

// Block c through the tiled in-edges (sources in sweep numbers): tiles
// [tb, te) of the block's partitions; the message of an in-edge from source
// s is the base published in this sweep when s < c B, else the previous
// sweep's (times the weight for EDGE_SCALE), summed per target in FP64 LDS
// accumulators. A workgroup then claims the targets of an unsplit partition
// with their sums included (every vertex of the block lies in one partition,
// so this is the block's claim); the tiles of split partitions store slots,
// whose targets k_sweep_tile_finish claims. The update counts go to the
// claim partials (tile workgroups first, then the finishing workgroups).
template <int ST, int G, uint32_t NT>
__global__ __launch_bounds__(NT) void k_sweep_tile(SweepArgs a, TileArgs t, uint32_t c, uint32_t tb, uint32_t te) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  uint64_t act = 0, pushed = 0;
  __shared__ double acc[TileShape<NT>::cap];
  const uint32_t tid = threadIdx.x;
  const uint64_t k = ctl->rounds / a.P;
  const uint64_t cur = (k & 1) * a.n, prev = ((k + 1) & 1) * a.n, lo = (uint64_t)c * a.B;
  const S* mu2 = static_cast<const S*>(a.mu2);
  const S* wt = static_cast<const S*>(t.wtile);
  const S* dv = static_cast<const S*>(a.dv);
  auto msg = [&](uint32_t src, uint32_t e) -> double {
    double x = (double)mu2[(src < lo ? cur : prev) + src];
    if constexpr (G == DAIC_G_EDGE_SCALE) x *= (double)wt[e];
    return x;
  };
  auto add = [&](uint32_t l, double x) { atomicAdd(&acc[l], x); };  // adding 0 leaves a sum as it is
  for (uint64_t pos = tb + blockIdx.x; pos < te; pos += gridDim.x) {
    const uint32_t tile = t.tile_order[pos];
    const uint32_t part = t.tile_part[tile], e0 = t.tile_e[tile], e1 = t.tile_e[tile + 1], slot = t.tile_slot[tile];
    for (uint32_t i = tid; i < t.tw; i += NT) acc[i] = 0.0;
    __syncthreads();
    tile_walk<NT, G != DAIC_G_EDGE_SCALE, double>(t, e0, e1, msg, add);
    __syncthreads();
    const uint64_t base = (uint64_t)part * t.tw;
    const uint32_t count = (uint32_t)min((uint64_t)t.tw, a.n - base);
    if (slot == 0xFFFFFFFFu) {
      for (uint32_t i = tid; i < count; i += NT) {
        const S old = dv[base + i];
        sweep_claim_vertex<ST, G>(a, (uint32_t)(base + i), (S)((double)old + acc[i]), old, cur, act, pushed);
      }
    } else {
      SlotT<ST>* dst = reinterpret_cast<SlotT<ST>*>(t.pbuf) + (uint64_t)slot * t.tw;
      for (uint32_t i = tid; i < count; i += NT) dst[i] = (SlotT<ST>)acc[i];
    }
    __syncthreads();
  }
  act = block_sum_waves<NT / 64>(act);
  pushed = block_sum_waves<NT / 64>(pushed);
  if (threadIdx.x == 0) {
    a.part_a[blockIdx.x] = act;
    a.part_m[blockIdx.x] = pushed;
  }
}

// Targets of block c's split partitions [sb, se): their slots added in tile
// order (FP64), then claimed with the sum included. Partials at
// part_a/part_m[poff + workgroup].
template <int ST, int G>
__global__ __launch_bounds__(256) void k_sweep_tile_finish(SweepArgs a, TileArgs t, uint32_t sb, uint32_t se,
                                                           uint32_t poff) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const S* dv = static_cast<const S*>(a.dv);
  const SlotT<ST>* pbuf = reinterpret_cast<const SlotT<ST>*>(t.pbuf);
  const uint64_t cur = ((ctl->rounds / a.P) & 1) * a.n;
  uint64_t act = 0, pushed = 0;
  const uint32_t chunks = t.tw / 256;
  for (uint64_t item = (uint64_t)sb * chunks + blockIdx.x; item < (uint64_t)se * chunks; item += gridDim.x) {
    const uint64_t sp = item / chunks;
    const uint32_t chunk = (uint32_t)(item % chunks);
    const uint32_t part = t.split_part[sp], k0 = t.split_slot[sp], k1 = t.split_slot[sp + 1];
    const uint64_t base = (uint64_t)part * t.tw + chunk * 256;
    if (base + threadIdx.x >= a.n) continue;
    const uint32_t i = chunk * 256 + threadIdx.x;
    double sum = 0.0;
    for (uint32_t q = k0; q < k1; q += 16) {
      double x[16];
#pragma unroll
      for (uint32_t u = 0; u < 16; ++u) x[u] = (double)pbuf[(uint64_t)min(q + u, k1 - 1) * t.tw + i];
#pragma unroll
      for (uint32_t u = 0; u < 16; ++u)
        if (q + u < k1) sum += x[u];
    }
    const uint32_t j = (uint32_t)(base + threadIdx.x);
    const S old = dv[j];
    sweep_claim_vertex<ST, G>(a, j, (S)((double)old + sum), old, cur, act, pushed);
  }
  act = block_sum256(act);
  pushed = block_sum256(pushed);
  if (threadIdx.x == 0) {
    a.part_a[poff + blockIdx.x] = act;
    a.part_m[poff + blockIdx.x] = pushed;
  }
}

// After each round: add the claim's per-block counts to the totals; when the
// round does not end a sweep, count it and apply the round limit (the sweep's
// last round is counted by k_sweep_residual_final).
__global__ __launch_bounds__(256) void k_sweep_step(SweepArgs a, int sweep_end, uint32_t nparts) {
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  uint64_t act = 0, msg = 0;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256) {
    act += a.part_a[i];
    msg += a.part_m[i];
  }
  act = block_sum256(act);
  msg = block_sum256(msg);
  if (threadIdx.x == 0) {
    ctl->activations += act;
    ctl->pushed += msg;
    if (!sweep_end) {
      ctl->rounds += 1;
      ctl->stop = ctl->rounds >= ctl->max_rounds ? 1u : 0u;
    }
  }
}

// End of a sweep: per-workgroup partials of the bound on the pending mass
// (k_sweep_residual_final adds them in a fixed order).
template <int ST>
__global__ __launch_bounds__(256) void k_sweep_residual(SweepArgs a) {
  using S = typename Tr<ST>::S;
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  const uint64_t k = ctl->rounds / a.P;
  const S* mu = static_cast<const S*>(a.mu2) + (k & 1) * a.n;
  double r = 0.0;
  uint64_t cnt = 0;
  // four positions per step, their loads in flight together
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s0 < a.n; s0 += 4 * stride) {
    S mv[4];
    double cf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t s = min(s0 + stride * u, a.n - 1);
      mv[u] = mu[s];
      cf[u] = a.coef_le[s];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (s0 + stride * u >= a.n) break;
      const double m = fabs((double)mv[u]);
      r += m * cf[u];
      cnt += m > 0.0 ? 1 : 0;
    }
  }
  r = block_sum256(r);
  cnt = block_sum256(cnt);
  if (threadIdx.x == 0) {
    a.part_r[blockIdx.x] = r;
    a.part_n[blockIdx.x] = cnt;
  }
}

// One block after k_sweep_residual (nparts workgroups): their partials
// summed in a fixed order, the stop rule and the round count.
__global__ __launch_bounds__(256) void k_sweep_residual_final(SweepArgs a, uint32_t nparts) {
  Ctl* ctl = a.ctl;
  if (ctl_halted(ctl)) return;
  double rr = 0.0;
  uint64_t nn = 0;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256) {
    rr += a.part_r[i];
    nn += a.part_n[i];
  }
  rr = block_sum256(rr);
  nn = block_sum256(nn);
  if (threadIdx.x == 0) {
    ctl->r = rr;
    ctl->pending = nn;
    ctl->rounds += 1;
    const bool done = rr <= ctl->eps;
    ctl->done = done ? 1u : 0u;
    ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
  }
}

// Delivery of the messages still in flight after R rounds, R = k P + cl + 1
// (blocks 0..cl of sweep k done). A source at position s last published in
// sweep k if s < L = (cl + 1) B, else in sweep k - 1. A target of block bt
// last pulled in sweep k if bt <= cl, else in sweep k - 1; a base is
// unconsumed when it was published at or after the target's pull in
// (sweep, block) order, equal blocks included.
// Every edge block (of all blocks) pulls the messages still in flight
// towards its targets, which share one block bt.
template <int ST, int G>
__global__ __launch_bounds__(256) void k_sweep_deliver_stream(SweepArgs a, uint64_t nb) {
  using S = typename Tr<ST>::S;
  const uint64_t R = a.ctl->rounds;
  if (R == 0) return;
  using V = typename std::conditional<G == DAIC_G_EDGE_SCALE, double, S>::type;
  __shared__ V vals[kStreamEdges];
  __shared__ double acc[kStreamRows];
  __shared__ uint32_t off[kStreamRows + 1];
  const uint64_t k = (R - 1) / a.P, cl = (R - 1) % a.P;
  const uint64_t L = min<uint64_t>(a.n, (cl + 1) * a.B);
  const uint64_t cur = (k & 1) * a.n, prev = ((k + 1) & 1) * a.n;
  const S* mu2 = static_cast<const S*>(a.mu2);
  const S* wT = static_cast<const S*>(a.wT);
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint32_t t0 = a.sb_t[b];
    const uint64_t bt = t0 / a.B, T0 = bt * a.B;
    auto msg = [&](uint32_t src, uint32_t p) -> V {
      bool take;
      uint64_t o;
      if (bt <= cl) {
        take = src >= T0 && src < L;
        o = cur;
      } else {
        take = src < L || src >= T0;
        o = src < L ? cur : prev;
      }
      V m = take ? (V)mu2[o + src] : (V)0;
      if constexpr (G == DAIC_G_EDGE_SCALE) m *= (V)wT[p];
      return m;
    };
    stream_block<S, V>(a.rowT, a.srcT, static_cast<S*>(a.dv), t0, a.sb_n[b], a.sb_e[b], a.sb_e[b + 1], vals, acc,
                       off, msg);
  }
}

// coef_le[perm[j]] = sum over out-edges (j, t) with block(t) <= block(j) of
// |w_jt| (1 per edge when unweighted); rows walked by lane groups.
template <typename S, bool W>
__global__ __launch_bounds__(256) void k_sweep_coef(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col,
                                                    const S* __restrict__ w, const uint32_t* __restrict__ perm,
                                                    uint64_t n, uint64_t B, double* __restrict__ coef_le) {
  struct Edge {
    uint32_t rank;  // perm of the edge's target
    double weight;
  };
  rows_by_groups<true>(
      row, n, [&](uint64_t, uint32_t e) { return Edge{perm[col[e]], W ? fabs((double)w[e]) : 1.0}; },
      [&](uint64_t j, uint32_t, const Edge& x) {
        // block(t) <= block(j) <=> t's number is below the end of j's block
        // (one 32-bit division per row once hoisted, none per edge)
        const uint64_t end = (uint64_t)(perm[j] / (uint32_t)B + 1) * B;
        return x.rank < end ? x.weight : 0.0;
      },
      [&](uint64_t j, double acc) { coef_le[perm[j]] = acc; });
}

// srcT_sweep[p] = psw[inv[srcT[p]]]: from dense-round numbers to sweep numbers.
__global__ void k_sweep_renumber(const uint32_t* srcT, const uint32_t* inv, const uint32_t* psw, uint64_t m,
                                 uint32_t* out) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (uint64_t)gridDim.x * blockDim.x)
    out[p] = psw[inv[srcT[p]]];
}

__global__ void k_sweep_reopen(Ctl* ctl) {
  ctl->done = 0;
  ctl->stop = 0;
}

uint32_t sgrid(uint64_t count, uint32_t per = 256, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((count + per - 1) / per, cap));
}

// Enqueue table per (state, g).
struct SweepOps {
  void (*round)(const SweepState&, hipStream_t, uint32_t c);
  void (*deliver)(const SweepState&, hipStream_t);
};

template <int ST, int G>
struct SweepImpl {
  static void round(const SweepState& w, hipStream_t s, uint32_t c) {
    const SweepArgs& a = w.a;
    uint32_t nparts = a.claim_blocks;
    if (w.tiles.ready) {  // the block's tiles, then its split partitions, each claiming its targets
      const uint32_t tb = w.tile_off[c], te = w.tile_off[c + 1], sb = w.split_off[c], se = w.split_off[c + 1];
      const uint32_t fg = se > sb ? sgrid((uint64_t)(se - sb) * (w.ta.tw / 256), 1, kSweepFinishGrid) : 0;
      const SweepArgs& at = w.numbered ? w.ar : w.a;
      if (te > tb) {
        if (w.ta.tw > kNarrowTW)
          hipLaunchKernelGGL((k_sweep_tile<ST, G, 1024>), dim3(te - tb), dim3(1024), 0, s, at, w.ta, c, tb, te);
        else
          hipLaunchKernelGGL((k_sweep_tile<ST, G, 256>), dim3(te - tb), dim3(256), 0, s, at, w.ta, c, tb, te);
      }
      if (fg)
        hipLaunchKernelGGL((k_sweep_tile_finish<ST, G>), dim3(fg), dim3(256), 0, s, at, w.ta, sb, se, te - tb);
      nparts = (te - tb) + fg;
    } else {
      // one workgroup per edge block of block c, at most 16384
      const uint32_t bb = w.block_sb_off[c], be = w.block_sb_off[c + 1];
      if (be > bb)
        hipLaunchKernelGGL((k_sweep_stream<ST, G>), dim3(sgrid(be - bb, 1, 16384)), dim3(256), 0, s, a, c, bb, be);
      hipLaunchKernelGGL((k_sweep_claim<ST, G>), dim3(a.claim_blocks), dim3(256), 0, s, a, c);
    }
    const bool end = c + 1 == a.P;
    hipLaunchKernelGGL(k_sweep_step, dim3(1), dim3(256), 0, s, a, end ? 1 : 0, nparts);
    if (end) {
      const uint32_t g = sgrid(a.n, 256, kResGrid);
      hipLaunchKernelGGL(k_sweep_residual<ST>, dim3(g), dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_sweep_residual_final, dim3(1), dim3(256), 0, s, a, g);
    }
  }
  static void deliver(const SweepState& w, hipStream_t s) {
    const SweepArgs& a = w.a;
    if (w.sb_total)
      hipLaunchKernelGGL((k_sweep_deliver_stream<ST, G>), dim3(sgrid(w.sb_total, 1, 16384)), dim3(256), 0, s, a,
                         w.sb_total);
  }
};

template <int ST>
bool sweep_ops_st(int gk, SweepOps* o) {
  switch (gk) {
    case DAIC_G_SRC_SCALE: *o = {SweepImpl<ST, DAIC_G_SRC_SCALE>::round, SweepImpl<ST, DAIC_G_SRC_SCALE>::deliver}; return true;
    case DAIC_G_EDGE_SCALE: *o = {SweepImpl<ST, DAIC_G_EDGE_SCALE>::round, SweepImpl<ST, DAIC_G_EDGE_SCALE>::deliver}; return true;
    case DAIC_G_DEG_SCALE: *o = {SweepImpl<ST, DAIC_G_DEG_SCALE>::round, SweepImpl<ST, DAIC_G_DEG_SCALE>::deliver}; return true;
    default: return false;
  }
}

bool sweep_ops(const daic_problem* p, SweepOps* o) {
  switch (p->st) {
    case ST_F64: return sweep_ops_st<ST_F64>(p->gk, o);
    case ST_F32: return sweep_ops_st<ST_F32>(p->gk, o);
    case ST_F32K: return sweep_ops_st<ST_F32K>(p->gk, o);
    default: return false;
  }
}

size_t sweep_state_size(int st) { return st == ST_F64 ? 8 : 4; }

// Per-problem set-up for block size B: the sweep numbering (host, from the
// dense-round renumbering), the in-edge sources in that numbering, the items
// of the large targets grouped by block, the residual coefficients and the
// two message slots.
daic_status sweep_setup(daic_problem* p, uint64_t B, hipStream_t s) {
  SweepState*& w = p->sweep;
  if (w && w->B == B) return DAIC_OK;
  sweep_release(p);
  w = new SweepState();
  const GraphDev& d = p->g->dev;
  const PullGraph& PG = p->g->pull;
  const uint64_t n = d.n;
  const uint32_t P = (uint32_t)((n + B - 1) / B);
  w->B = B;
  w->P = P;
  auto grab = [&](void** q, size_t bytes) -> daic_status {
    void* m = nullptr;
    hipError_t e = hipMalloc(&m, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(DAIC_E_OOM, "sweep set-up: hipMalloc of %zu bytes failed", bytes);
    w->allocs.push_back(m);
    *q = m;
    return DAIC_OK;
  };
  // sweep numbering: block-major, out-degree order (the dense-round
  // renumbering) inside a block
  std::vector<uint32_t> perm(n), inv(n), rt(n + 1), psw(n);
  DAIC_HIP(hipMemcpy(perm.data(), PG.perm, n * 4, hipMemcpyDeviceToHost));
  DAIC_HIP(hipMemcpy(rt.data(), PG.rowT, (n + 1) * 4, hipMemcpyDeviceToHost));
  for (uint64_t j = 0; j < n; ++j) inv[perm[j]] = (uint32_t)j;
  std::vector<uint32_t> voff(P + 1, 0);
  for (uint32_t c = 0; c <= P; ++c) voff[c] = (uint32_t)std::min<uint64_t>(n, (uint64_t)c * B);
  {
    std::vector<uint32_t> fill(voff.begin(), voff.end() - 1);
    for (uint64_t q = 0; q < n; ++q) {
      const uint32_t j = inv[q];
      psw[j] = fill[j / B]++;
    }
  }
  std::vector<uint32_t> rv, roff(P + 1, 0);
  std::vector<uint32_t> sbt, sbe, sbn, sboff(P + 1, 0);
  for (uint32_t c = 0; c < P; ++c) {
    for (uint32_t t = voff[c]; t < voff[c + 1]; ++t)
      if (rt[t + 1] > rt[t]) rv.push_back(t);
    roff[c + 1] = (uint32_t)rv.size();
    stream_blocks(rt.data(), voff[c], voff[c + 1], sbt, sbe, sbn, false);
    sboff[c + 1] = (uint32_t)sbt.size();
    w->max_block_verts = std::max<uint64_t>(w->max_block_verts, voff[c + 1] - voff[c]);
  }
  SweepArgs& a = w->a;
  void* q = nullptr;
  daic_status rc;
#define SGRAB(field, type, bytes)            \
  do {                                       \
    if ((rc = grab(&q, (bytes)))) return rc; \
    a.field = (type)q;                       \
  } while (0)
  const size_t S = sweep_state_size(p->st);
  SGRAB(mu2, void*, 2 * n * S);
  SGRAB(voff, const uint32_t*, (P + 1) * 4);
  sbe.push_back((uint32_t)d.m);
  w->sb_total = sbt.size();
  w->block_sb_off = sboff;
  SGRAB(sb_t, const uint32_t*, sbt.size() * 4);
  SGRAB(sb_e, const uint32_t*, sbe.size() * 4);
  SGRAB(sb_n, const uint32_t*, sbn.size() * 4);
  SGRAB(rv, const uint32_t*, rv.size() * 4);
  SGRAB(roff, const uint32_t*, (P + 1) * 4);
  SGRAB(coef_le, const double*, n * 8);
  SGRAB(perm, const uint32_t*, n * 4);
  SGRAB(srcT, const uint32_t*, std::max<uint64_t>(d.m, 1) * 4);
  SGRAB(part_r, double*, kResGrid * 8);
  SGRAB(part_n, uint64_t*, kResGrid * 8);
  a.claim_blocks = sgrid(w->max_block_verts, 256, 4096);
  SGRAB(part_a, uint64_t*, a.claim_blocks * 8);
  SGRAB(part_m, uint64_t*, a.claim_blocks * 8);
#undef SGRAB
  DAIC_HIP(hipMemcpy((void*)a.voff, voff.data(), (P + 1) * 4, hipMemcpyHostToDevice));
  if (!sbt.empty()) {
    DAIC_HIP(hipMemcpy((void*)a.sb_t, sbt.data(), sbt.size() * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.sb_n, sbn.data(), sbn.size() * 4, hipMemcpyHostToDevice));
  }
  DAIC_HIP(hipMemcpy((void*)a.sb_e, sbe.data(), sbe.size() * 4, hipMemcpyHostToDevice));
  if (!rv.empty()) DAIC_HIP(hipMemcpy((void*)a.rv, rv.data(), rv.size() * 4, hipMemcpyHostToDevice));
  DAIC_HIP(hipMemcpy((void*)a.roff, roff.data(), (P + 1) * 4, hipMemcpyHostToDevice));
  a.ctl = p->a.ctl;
  a.n = n;
  a.B = B;
  a.P = P;
  a.row = static_cast<const uint32_t*>(d.row);
  a.rowT = static_cast<const uint32_t*>(PG.rowT);
  DAIC_HIP(hipMemcpy((void*)a.perm, psw.data(), n * 4, hipMemcpyHostToDevice));
  {
    // sweep numbers of the in-edge sources, in the in-edge order of the
    // dense rounds (so edge weights in in-edge order stay aligned)
    uint32_t* d_inv = nullptr;
    DAIC_HIP(hipMalloc(&d_inv, n * 4));
    hipError_t e = hipMemcpy(d_inv, inv.data(), n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && d.m)
      hipLaunchKernelGGL(k_sweep_renumber, dim3(sgrid(d.m)), dim3(256), 0, s, PG.srcT, d_inv, a.perm, d.m,
                         const_cast<uint32_t*>(a.srcT));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_inv);
    if (e != hipSuccess) return fail(DAIC_E_DEVICE, "sweep set-up: %s", hipGetErrorString(e));
  }
  a.wT = p->a.wT;
  a.v = p->a.v;
  a.dv = p->a.dv;
  a.c = p->a.c;
  a.alpha_pv = p->a.alpha_pv;
  a.alpha = p->a.alpha;
  const uint32_t* row = static_cast<const uint32_t*>(d.row);
  double* cl = const_cast<double*>(a.coef_le);
  if (p->gk == DAIC_G_EDGE_SCALE) {
    if (p->st == ST_F64)
      hipLaunchKernelGGL((k_sweep_coef<double, true>), dim3(sgrid(n, 4)), dim3(256), 0, s, row, d.col,
                         static_cast<const double*>(p->a.w), a.perm, n, B, cl);
    else
      hipLaunchKernelGGL((k_sweep_coef<float, true>), dim3(sgrid(n, 4)), dim3(256), 0, s, row, d.col,
                         static_cast<const float*>(p->a.w), a.perm, n, B, cl);
  } else {
    hipLaunchKernelGGL((k_sweep_coef<float, false>), dim3(sgrid(n, 4)), dim3(256), 0, s, row, d.col,
                       (const float*)nullptr, a.perm, n, B, cl);
  }
  DAIC_HIP(hipStreamSynchronize(s));
  // the tiled in-edges in sweep numbers, when the blocks are whole
  // partitions (B a multiple of a width of at least 2^8); DAIC_NO_TILE=1
  // keeps the streamed pull
  uint32_t lb = tile_default_bits(n);
  if (const char* e = std::getenv("DAIC_SWEEP_TILE_BITS")) lb = (uint32_t)std::min(14ul, std::strtoul(e, nullptr, 10));
  while (lb >= 8 && B % (1ull << lb) != 0) --lb;
  if (lb >= 8 && !std::getenv("DAIC_NO_TILE") && d.m > 0 && tile_fits(d.m)) {
    // tiles of up to one resident workgroup's share of their own block's
    // in-edges: RMAT-24's id blocks hold very different numbers of in-edges
    // (4 blocks: 58, 18, 18 and 6 %), so one size for all either splits the
    // light blocks' partitions too little (their largest tile then outlasts
    // the rest) or the heavy block's too much (4 blocks: 81.5 ms per solve
    // against 86.8 ms with tiles of at most 196,608 for all blocks; a half
    // or 3/4 share: 84-86 ms). DAIC_SWEEP_TILE_SHARE sets the divisor,
    // DAIC_SWEEP_TILE_EDGES caps the tiles.
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint64_t max_edges = 0;
    if (const char* e = std::getenv("DAIC_SWEEP_TILE_EDGES")) max_edges = std::strtoull(e, nullptr, 10);
    uint32_t share = (uint32_t)std::max(cus, 1) * tile_wgs_per_cu(lb);
    if (const char* e = std::getenv("DAIC_SWEEP_TILE_SHARE")) share = (uint32_t)std::strtoul(e, nullptr, 10);
    // targets numbered by in-degree octave within each block, as for the
    // fused rounds; DAIC_TILE_ID_ORDER=1 keeps id order
    uint32_t *trank = nullptr, *tinv = nullptr, *rowP = nullptr, *permP = nullptr;
    if (!std::getenv("DAIC_TILE_ID_ORDER") &&
        (rc = rank_targets(p->g, a.perm, B, &trank, &tinv, &rowP, &permP, s)))
      return rc;
    rc = tile_build(d, a.perm, lb, max_edges, B >> lb, share, w->tiles, s, trank);
    if (trank) (void)hipFree(trank);
    if (rc) {
      for (void* q : {(void*)tinv, (void*)rowP, (void*)permP})
        if (q) (void)hipFree(q);
      return rc;
    }
    w->tiles.tinv = tinv;
    w->tiles.rowP = rowP;
    w->tiles.permP = permP;
    const TileGraph& T = w->tiles;
    const uint64_t TW = 1ull << T.tbits;
    std::vector<uint32_t> tp(T.n_tiles), sp(T.n_split);
    DAIC_HIP(hipMemcpy(tp.data(), T.tile_part, T.n_tiles * 4, hipMemcpyDeviceToHost));
    if (T.n_split) DAIC_HIP(hipMemcpy(sp.data(), T.split_part, T.n_split * 4, hipMemcpyDeviceToHost));
    w->tile_off.assign(P + 1, 0);
    w->split_off.assign(P + 1, 0);
    uint32_t max_tiles = 0;
    for (uint32_t c = 0; c <= P; ++c) {
      const uint64_t first_part = std::min<uint64_t>((uint64_t)c * B / TW, T.n_part);
      w->tile_off[c] = (uint32_t)(std::lower_bound(tp.begin(), tp.end(), (uint32_t)first_part) - tp.begin());
      w->split_off[c] = (uint32_t)(std::lower_bound(sp.begin(), sp.end(), (uint32_t)first_part) - sp.begin());
      if (c) max_tiles = std::max(max_tiles, w->tile_off[c] - w->tile_off[c - 1]);
    }
    // claim partials of a round: its tile workgroups, then its finishing ones
    if (max_tiles + kSweepFinishGrid > a.claim_blocks) {
      void *pa = nullptr, *pm = nullptr;
      if ((rc = grab(&pa, (max_tiles + kSweepFinishGrid) * 8)) || (rc = grab(&pm, (max_tiles + kSweepFinishGrid) * 8)))
        return rc;
      a.part_a = static_cast<uint64_t*>(pa);
      a.part_m = static_cast<uint64_t*>(pm);
    }
    TileArgs& t = w->ta;
    t.tloc = T.tloc;
    t.psrc = T.psrc;
    t.segpair = T.segpair;
    t.tile_part = T.tile_part;
    t.tile_e = T.tile_e;
    t.tile_slot = T.tile_slot;
    t.tile_order = T.tile_order;
    t.split_part = T.split_part;
    t.split_slot = T.split_slot;
    t.m = d.m;
    t.n_tiles = T.n_tiles;
    t.n_split = T.n_split;
    t.n_seg = T.n_seg;
    t.tw = (uint32_t)TW;
    void* pb = nullptr;
    if ((rc = grab(&pb, std::max<uint64_t>(T.n_slots, 1) * TW * 8))) return rc;
    t.pbuf = static_cast<double*>(pb);
    if (T.tinv) {
      SweepArgs& r = w->ar;
      r = a;
      void *vp = nullptr, *dvp = nullptr, *cp = nullptr, *ap = nullptr;
      if ((rc = grab(&vp, n * S)) || (rc = grab(&dvp, n * S))) return rc;
      if (a.c && (rc = grab(&cp, n * 4))) return rc;
      if (a.alpha_pv && (rc = grab(&ap, n * S))) return rc;
      r.v = vp;
      r.dv = dvp;
      r.c = static_cast<float*>(cp);
      r.alpha_pv = ap;
      r.row = T.rowP;
      r.perm = T.permP;
      w->numbered = true;
    }
    if (p->gk == DAIC_G_EDGE_SCALE) {  // weights in the tiles' in-edge order
      void* wt = nullptr;
      const uint64_t pe = tile_padded_edges(T);
      if ((rc = grab(&wt, pe * S))) return rc;
      if (p->st == ST_F64)
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(sgrid(pe)), dim3(256), 0, s,
                           static_cast<const double*>(p->a.w), T.eid, d.m, pe, static_cast<double*>(wt));
      else
        hipLaunchKernelGGL(k_gather_weights<float>, dim3(sgrid(pe)), dim3(256), 0, s,
                           static_cast<const float*>(p->a.w), T.eid, d.m, pe, static_cast<float*>(wt));
      t.wtile = wt;
    }
    DAIC_HIP(hipStreamSynchronize(s));
  }
  return DAIC_OK;
}

}  // namespace

void sweep_release(daic_problem* p) {
  if (!p->sweep) return;
  tile_free(p->sweep->tiles);
  for (void* q : p->sweep->allocs)
    if (q) (void)hipFree(q);
  delete p->sweep;
  p->sweep = nullptr;
}

daic_status sweep_run(daic_problem* p, const daic_run_opts* o, daic_stats* stats, hipStream_t s) {
  const bool sum = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
  if (!sum) return fail(DAIC_E_UNSUPPORTED, "SWEEP scheduling takes sum problems");
  const uint64_t n = p->g->dev.n;
  daic_status rc = dense_rounds_setup(p, o, s);
  if (rc) return rc;
  if (!p->pull_ready) return fail(DAIC_E_UNSUPPORTED, "SWEEP scheduling needs n, m < 2^31 (and DAIC_NO_PULL unset)");
  Ops ops;
  SweepOps sw;
  if (!get_ops(p, &ops) || !sweep_ops(p, &sw)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  const uint64_t B = std::max<uint64_t>(1, std::min<uint64_t>(n, (uint64_t)std::ceil(o->priority_fraction * (double)n)));
  rc = sweep_setup(p, B, s);
  if (rc) {
    sweep_release(p);  // a half-built state must not pass for a finished one on the next run
    return rc;
  }
  const SweepState& w = *p->sweep;
  const uint32_t P = w.P;
  // rounds captured per launch: whole sweeps, at least rounds_per_check rounds
  const uint32_t want = o->rounds_per_check ? o->rounds_per_check : 1;
  const uint32_t K = P * std::max<uint32_t>(1, (want + P - 1) / P);
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;

  DAIC_HIP(hipMemsetAsync(w.a.mu2, 0, 2 * n * sweep_state_size(p->st), s));
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, o->eps, max_rounds);
  ops.residual(p, s, 0);
  DAIC_HIP(hipEventRecord(p->ev0, s));
  const size_t SS = sweep_state_size(p->st);
  const uint32_t* tinv = w.tiles.tinv;
  if (w.numbered) {  // the state into the block pulls' target numbering
    perm_gather(w.a.v, w.ar.v, SS, tinv, n, s);
    perm_gather(w.a.dv, w.ar.dv, SS, tinv, n, s);
    if (w.a.c) perm_gather(w.a.c, w.ar.c, 4, tinv, n, s);
    if (w.a.alpha_pv) perm_gather(w.a.alpha_pv, const_cast<void*>(w.ar.alpha_pv), SS, tinv, n, s);
  }
  auto unnumber = [&]() {
    if (!w.numbered) return;
    perm_scatter(w.ar.v, w.a.v, SS, tinv, n, s);
    perm_scatter(w.ar.dv, w.a.dv, SS, tinv, n, s);
    if (w.a.c) perm_scatter(w.ar.c, w.a.c, 4, tinv, n, s);
  };
  const bool use_graph = std::getenv("DAIC_NO_GRAPH") == nullptr;
  GraphCacheKey key;
  key.sched = DAIC_SCHED_SWEEP;
  key.k = B;
  key.q = o->priority_fraction;
  key.K = K;
  key.stream = s;
  if (use_graph && !(p->exec && p->key == key)) {
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (uint32_t r = 0; r < K; ++r) sw.round(w, s, r % P);
    hipGraph_t graph;
    DAIC_HIP(hipStreamEndCapture(s, &graph));
    p->graph = graph;
    DAIC_HIP(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0));
    p->key = key;
  }
  uint64_t seen_rounds = ~0ull;
  for (;;) {
    DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    if (p->h_ctl->done || p->h_ctl->stop) break;
    // every launch advances the round count; fail instead of spinning if not
    if (p->h_ctl->rounds == seen_rounds) {
      unnumber();
      return fail(DAIC_E_DEVICE, "sweep run made no progress (round %llu)", (unsigned long long)seen_rounds);
    }
    seen_rounds = p->h_ctl->rounds;
    if (use_graph) {
      DAIC_HIP(hipGraphLaunch(p->exec, s));
    } else {
      for (uint32_t r = 0; r < K; ++r) sw.round(w, s, r % P);
    }
  }
  // deliver the messages in flight, then the exact residual of (v, dv)
  unnumber();
  sw.deliver(w, s);
  hipLaunchKernelGGL(k_sweep_reopen, dim3(1), dim3(1), 0, s, p->a.ctl);
  ops.residual(p, s, 0);
  DAIC_HIP(hipEventRecord(p->ev1, s));
  DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DAIC_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  DAIC_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
  const Ctl& c = *p->h_ctl;
  if (stats) {
    stats->rounds = c.rounds;
    stats->activations = c.activations;
    stats->pushed_edges = c.pushed;
    stats->final_residual = c.r;
    stats->time_ms = ms;
    stats->gteps = ms > 0 ? (double)c.pushed / (ms * 1e-3) / 1e9 : 0.0;
    stats->alg_bytes = 0.0;
  }
  return c.done ? DAIC_OK : DAIC_NOT_CONVERGED;
}

}  // namespace daic
