// Batched DAIC: many graphs of uneven size, each with many right-hand sides,
// solved together (personalized PageRank: the Rooted PageRank row of Table 1
// read with damping, g_{j,k}(x) = d x / outdeg_j, Delta v^1 = (1-d) p).
//
// The graphs are joined into one block-diagonal graph; the state is
// [vertex][64 right-hand sides] in FP32, so one message is a contiguous
// 256-byte vector. While few vertices are pending, a round is three kernels
// (claim, push with atomics, residual). Once the pending set is dense, one
// claim publishes the message bases and every later round is a fused pass
// over graph-aligned vertex ranges: pull the previous round's messages over
// in-edges (high in-degree targets are summed beforehand by a chunked
// kernel), take the residual, claim and publish the next messages into a
// second buffer. Every instance (graph, right-hand side) has its own residual
// and finish state. Lanes per vertex and grid sizes come from an autotuner
// that times the kernels on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "daic_device.h"
#include "daic_internal.h"

namespace daic {

constexpr int kR = 64;                 // right-hand sides per vertex (padded)
constexpr uint32_t kBChunk = 1024;     // in-edges per pull item
constexpr uint32_t kPushChunk = 256;   // out-edges per push item
constexpr uint32_t kResChunk = 4096;   // at most this many vertices per residual item
constexpr uint32_t kItemWork = 32768;  // and about this much work (in-edges + kVertexWork per vertex)
constexpr uint32_t kVertexWork = 4;
// sweep rounds run one block (a fraction of the items) per launch, so their
// items are smaller: the longest item bounds each launch
constexpr uint32_t kSwResChunk = 1024;
constexpr uint32_t kSwItemWork = 8192;
constexpr uint32_t kSwHubChunk = 256;
constexpr uint32_t kHubDeg = 64;       // default in-degree above which a target is a hub

// Round modes: 0 = sparse round (claim, push, residual); 1 = the claim that
// starts the dense phase (publishes message bases, delivers nothing);
// 2 = fused dense round (deliver the previous round's messages by pulling,
// then claim and publish, with the residual in the same pass); 3 = sweep
// round (the fused pass over one block of every graph, pulling the newest
// message of every in-neighbour; see k_bfused).
struct BCtl {
  uint32_t done;          // every instance finished and nothing in flight
  uint32_t stop;          // round limit reached
  uint32_t mode;          // mode of the next round
  uint32_t ticket;
  uint32_t prev_all_done; // every instance was finished after the previous round
  uint32_t dense_mode;    // mode the dense phase starts in: 1 (synchronous) or 3 (sweep)
  uint32_t sw_c;          // sweep rounds: block of the current round
  uint32_t sw_started;    // a sweep round has run since the dense phase began
  uint64_t sw_k;          // sweep rounds: sweep of the current round
  uint64_t base;          // round at which the sweep phase began
  uint64_t rounds;
  uint64_t max_rounds;
  uint64_t pending;       // vertices with a pending right-hand side
  uint64_t activations;   // (vertex, rhs) updates
  uint64_t messages;      // (edge, rhs) messages
  double eps;
};

struct BArgs {
  BCtl* ctl;
  uint64_t N;                 // vertices of the union graph
  const uint32_t* row;        // union CSR (uint32 offsets)
  const uint32_t* col;
  const uint32_t* gid;        // graph of each vertex
  float* v;                   // [N][64]
  float* dv;
  float* c;                   // Kahan term, or null
  float* mu;                  // [N][64]: by vertex (sparse) / renumbered, even rounds (dense)
  float* mu2;                 // [N][64]: renumbered, odd rounds (dense)
  const float* w;             // EDGE_SCALE: weight of each out-edge, or null (DEG_SCALE)
  const float* wT;            // the same in in-edge order
  uint8_t* active;            // [N] vertex sent this round (sparse rounds)
  uint8_t* done;              // [G][64] instance finished
  double alpha;
  // dense rounds
  const uint32_t* perm;
  const uint32_t* rowT;
  const uint32_t* srcT;
  // sparse rounds
  const uint32_t* sv;         // push items (vertex, chunk)
  const uint32_t* sc;
  uint64_t n_push;
  // residual items: (graph, first vertex, last vertex)
  const uint32_t* rg;
  const uint64_t* rlo;
  const uint64_t* rhi;
  uint32_t n_res;
  const uint32_t* g_first_item;  // [G+1] residual items of each graph
  uint32_t G;
  double* part_r;             // [n_res][64]
  uint64_t* part_p;           // [n_res] union pending
  uint64_t* part_a;           // [claim blocks] activations
  uint64_t* part_m;           // [claim blocks] messages
  uint64_t* part_fa;          // [n_res] activations / messages of fused rounds
  uint64_t* part_fm;
  double* inst_r;             // [G][64] residual per instance
  uint64_t pull_min;          // dense phase when union pending >= pull_min
  // per graph: item tickets and the sums of its retired items
  uint32_t* g_ticket;
  uint32_t* g_flag;
  uint64_t* g_pend;
  uint64_t* g_act;
  uint64_t* g_msg;
  // fused dense rounds: in-edges of hub targets (in-degree > hub_deg) are
  // summed by a chunked kernel before the fused pass
  uint32_t hub_deg;
  uint32_t hub_chunk;         // in-edges per hub item
  const uint32_t* ht;         // hub items (target, chunk)
  const uint32_t* hc;
  uint64_t n_hub;
  const uint32_t* item_order; // block -> residual item of the fused pass (~0u: none)
  // sweep rounds (the sweep copy of these arguments also points the item,
  // hub-item, source-numbering and partial fields at the sweep's own arrays)
  uint32_t sw_P;              // blocks per graph
  const uint64_t* sw_bstart;  // [P+1] first sweep number of each block
  const uint32_t* sw_items;   // items of each block (XCD-interleaved, ~0u padding)
  const uint32_t* sw_ioff;    // [P+1]
  const uint32_t* sw_hoff;    // [P+1] hub items of each block
  const double* sw_coef;      // [N] sum of |w| (1 per edge when unweighted) to out-neighbours in blocks <= own
  const uint32_t* sw_blk;     // [N] block of each vertex
  const uint32_t* vord;       // [N] vertices of each item by pulled in-degree, descending, isolated last
  const uint64_t* rha;        // [n_res] end of the item's vertices that have any edge
  uint32_t n_fused_blocks;
};

__device__ __forceinline__ bool bhalted(const BCtl* c) { return (c->done | c->stop) != 0; }


// Message-base buffer written by the claims of round t (dense phase).
__device__ __forceinline__ float* mu_of_round(const BArgs& a, uint64_t t) { return (t & 1) ? a.mu2 : a.mu; }

template <int W>
struct VecF;
template <> struct VecF<1> { using T = float; };
template <> struct VecF<2> { using T = float2; };
template <> struct VecF<4> { using T = float4; };

template <int W>
__device__ __forceinline__ void vload(const float* p, float (&x)[W]) {
  typename VecF<W>::T t = *reinterpret_cast<const typename VecF<W>::T*>(p);
  const float* f = reinterpret_cast<const float*>(&t);
#pragma unroll
  for (int i = 0; i < W; ++i) x[i] = f[i];
}

template <int W>
__device__ __forceinline__ void vstore(float* p, const float (&x)[W]) {
  typename VecF<W>::T t;
  float* f = reinterpret_cast<float*>(&t);
#pragma unroll
  for (int i = 0; i < W; ++i) f[i] = x[i];
  *reinterpret_cast<typename VecF<W>::T*>(p) = t;
}

// ---------------------------------------------------------------------------
// Claim and fold for every vertex and right-hand side; publishes the 64-wide
// message base (renumbered in dense rounds) or marks the vertex active.
// LPV lanes per vertex, each holding W = 64/LPV consecutive right-hand sides.
// ---------------------------------------------------------------------------
template <int LPV, bool KAHAN>
__global__ __launch_bounds__(256) void k_bclaim(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int VPB = 256 / LPV;
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->mode >= 2) return;
  const bool pull = ctl->mode == 1;
  float* mu_dense = mu_of_round(a, ctl->rounds);
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  uint64_t act = 0, msg = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * VPB; base < a.N; base += (uint64_t)gridDim.x * VPB) {
    const uint64_t j = base + sub;
    if (j >= a.N) continue;
    const uint32_t g = a.gid[j];
    const uint32_t deg = a.row[j + 1] - a.row[j];
    const double coef = a.w ? a.alpha : (deg ? a.alpha / (double)deg : 0.0);
    float d[W], mu[W];
    bool cl[W];
    vload<W>(a.dv + j * kR + r0, d);
    bool any = false;
    uint32_t nclaim = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      cl[i] = d[i] != 0.0f && !a.done[g * kR + r0 + i];
      mu[i] = cl[i] ? (float)(coef * (double)d[i]) : 0.0f;
      any |= cl[i];
      nclaim += cl[i] ? 1u : 0u;
    }
    if (any) {
      float vv[W], dz[W];
      vload<W>(a.v + j * kR + r0, vv);
      if constexpr (KAHAN) {
#pragma clang fp contract(off)
        float cc[W];
        vload<W>(a.c + j * kR + r0, cc);
#pragma unroll
        for (int i = 0; i < W; ++i) {
          if (cl[i]) {
            float y = d[i] - cc[i];
            float t = vv[i] + y;
            cc[i] = (t - vv[i]) - y;
            vv[i] = t;
            dz[i] = 0.0f;
          } else {
            dz[i] = d[i];
          }
        }
        vstore<W>(a.c + j * kR + r0, cc);
      } else {
#pragma unroll
        for (int i = 0; i < W; ++i) {
          if (cl[i]) {
            vv[i] += d[i];
            dz[i] = 0.0f;
          } else {
            dz[i] = d[i];
          }
        }
      }
      vstore<W>(a.v + j * kR + r0, vv);
      vstore<W>(a.dv + j * kR + r0, dz);
    }
    act += nclaim;
    msg += (uint64_t)nclaim * deg;
    if (pull) {
      vstore<W>(mu_dense + (uint64_t)a.perm[j] * kR + r0, mu);
    } else {
      // a vertex is active when any of its lanes sends; every lane of the
      // vertex writes its part of the message base
      bool vany = any && deg > 0;
#pragma unroll
      for (int o = LPV / 2; o >= 1; o >>= 1) vany |= __shfl_xor((int)vany, o, LPV) != 0;
      if (vany) vstore<W>(a.mu + j * kR + r0, mu);
      if ((threadIdx.x % LPV) == 0) a.active[j] = vany ? 1 : 0;
    }
  }
  act = block_sum256(act);
  msg = block_sum256(msg);
  if (threadIdx.x == 0) {
    a.part_a[blockIdx.x] = act;
    a.part_m[blockIdx.x] = msg;
  }
}

// Sparse round: active vertices push their 64-wide message to every out-edge.
template <int LPV>
__global__ __launch_bounds__(256) void k_bpush(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int IPB = 256 / LPV;
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->mode != 0) return;
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  for (uint64_t base = (uint64_t)blockIdx.x * IPB; base < a.n_push; base += (uint64_t)gridDim.x * IPB) {
    const uint64_t i = base + sub;
    if (i >= a.n_push) continue;
    const uint32_t j = a.sv[i];
    if (!a.active[j]) continue;
    const uint32_t beg = a.row[j] + a.sc[i] * kPushChunk;
    const uint32_t end = min(a.row[j + 1], beg + kPushChunk);
    float mu[W];
    vload<W>(a.mu + (uint64_t)j * kR + r0, mu);
    for (uint32_t e = beg; e < end; ++e) {
      float* dst = a.dv + (uint64_t)a.col[e] * kR + r0;
      const float we = a.w ? a.w[e] : 1.0f;
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (mu[k] != 0.0f) unsafeAtomicAdd(dst + k, a.w ? mu[k] * we : mu[k]);
    }
  }
}

// Retirement of a residual item. The block that retires the last item of a
// graph sums the graph's per-item partials in a fixed order and moves the
// finish state of its 64 instances; the block that retires the last graph
// updates the control block. kind 0: sparse round or initial check (all
// messages delivered); kind 1: fused dense round (the residual is that of the
// previous round's end state, whose last messages are still in flight);
// kind 2: final delivery after a stop in the dense phase.
// Finish states per instance: 0 running, 1 finished with messages in flight,
// 2 finished and delivered.
// Graph g once all its items of the pass are done: sum its items' partials,
// move its instances' finish states, and take the ticket of the graphs.
__device__ void retire_graph(const BArgs& a, uint32_t g, int kind, int count_round) {
  __shared__ uint32_t s_flag;
  __shared__ double s_r[4][kR];
  BCtl* ctl = a.ctl;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t k0 = a.g_first_item[g], k1 = a.g_first_item[g + 1];
  double r = 0.0;
  for (uint32_t k = k0 + wave; k < k1; k += 4)
    r += __hip_atomic_load(&a.part_r[(uint64_t)k * kR + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s_r[wave][lane] = r;
  uint64_t pend = 0, act = 0, msg = 0;
  for (uint32_t k = k0 + threadIdx.x; k < k1; k += 256) {
    pend += __hip_atomic_load(&a.part_p[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    act += __hip_atomic_load(&a.part_fa[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    msg += __hip_atomic_load(&a.part_fm[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  pend = block_sum256(pend);
  act = block_sum256(act);
  msg = block_sum256(msg);
  if (wave == 0) {
    const uint32_t q = g * kR + lane;
    const double sr = ((s_r[0][lane] + s_r[1][lane]) + s_r[2][lane]) + s_r[3][lane];
    const uint8_t st = a.done[q];
    uint8_t ns = st;
    bool flag;
    if (kind == 0) {
      a.inst_r[q] = sr;
      if (st == 1 || (st == 0 && sr <= ctl->eps)) ns = 2;  // state 1: delivered since
      flag = ns == 2;
    } else if (kind == 1) {
      if (st != 2) a.inst_r[q] = sr;
      if (st == 1) ns = 2;
      else if (st == 0 && sr <= ctl->eps) ns = 1;
      flag = st != 0;  // nothing was claimed for this instance in this round
    } else {
      if (st != 2) a.inst_r[q] = sr;
      if (st == 1 || (st == 0 && sr <= ctl->eps)) ns = 2;
      flag = ns == 2;
    }
    a.done[q] = ns;
    const bool all = __ballot(!flag) == 0;
    if (lane == 0) {
      a.g_flag[g] = all ? 1u : 0u;
      a.g_pend[g] = pend;
      a.g_act[g] = act;
      a.g_msg[g] = msg;
      a.g_ticket[g] = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_flag = atomicAdd(&ctl->ticket, 1u) == a.G - 1;
  }
  __syncthreads();
  if (!s_flag) return;
  __threadfence();
  uint64_t pp = 0, aa = 0, mm = 0;
  uint32_t all = 1;
  for (uint32_t h = threadIdx.x; h < a.G; h += 256) {
    pp += __hip_atomic_load(&a.g_pend[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    aa += __hip_atomic_load(&a.g_act[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mm += __hip_atomic_load(&a.g_msg[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    all &= __hip_atomic_load(&a.g_flag[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  pp = block_sum256(pp);
  aa = block_sum256(aa);
  mm = block_sum256(mm);
  all = block_sum256(all);
  if (threadIdx.x == 0) {
    ctl->ticket = 0;
    if (kind == 2) {
      ctl->mode = 0;
      return;
    }
    const bool done = all == 256;
    ctl->rounds += (uint64_t)count_round;
    ctl->activations += aa;
    ctl->messages += mm;
    ctl->done = done ? 1u : 0u;
    ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
    if (kind == 0) {
      ctl->pending = pp;
      ctl->mode = (!done && pp >= a.pull_min) ? ctl->dense_mode : 0u;
      ctl->base = ctl->rounds;
      ctl->sw_started = 0;
    }
  }
}

__device__ void retire_item(const BArgs& a, uint32_t g, int kind, int count_round) {
  __shared__ uint32_t s_last;
  __threadfence();  // this block's partials are visible before its ticket
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nit = a.g_first_item[g + 1] - a.g_first_item[g];
    s_last = atomicAdd(&a.g_ticket[g], 1u) == nit - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  retire_graph(a, g, kind, count_round);
}

// Retirement of the fused dense pass, after it (its kernel only stores
// partials: a fence per item in a kernel that keeps dirtying L2 would write
// the L2 back each time): one block per graph.
__global__ __launch_bounds__(256) void k_bretire_dense(BArgs a, int final_pass) {
  BCtl* ctl = a.ctl;
  if (!final_pass && (bhalted(ctl) || ctl->mode != 2)) return;  // as k_bfused
  retire_graph(a, blockIdx.x, final_pass ? 2 : 1, 1);
}

// Retirement of a sweep: every graph's items have all run once the last
// block of the sweep has (graphs without vertices in the last blocks
// included), so after that block's pass one block per graph retires it.
__global__ __launch_bounds__(256) void k_bretire_sweep(BArgs a) {
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->mode != 3 || ctl->sw_c != a.sw_P - 1) return;  // as k_bfused, at the sweep's end
  retire_graph(a, blockIdx.x, 1, 0);
}

// Residual of a sparse round (or of the state at the start of a run): FP64
// sums of |dv| per instance and the union pending count, one block per
// residual item. After the claim that opens the dense phase it only counts
// the round and switches to fused rounds.
__global__ __launch_bounds__(256) void k_bresidual(BArgs a, int count_round) {
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->mode >= 2) return;
  if (ctl->mode == 1) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->rounds += (uint64_t)count_round;
      ctl->mode = 2;
      ctl->stop = ctl->rounds >= ctl->max_rounds ? 1u : 0u;
    }
    return;
  }
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  __shared__ double s_w[4][kR];
  double r = 0.0;
  uint64_t pend = 0;
  const uint32_t it = blockIdx.x;
  // rows j, j + 4, j + 8, j + 12 of this wave per step, their loads in
  // flight together (the same summation order as one row per step)
  const uint64_t rlo = a.rlo[it], rhi = a.rhi[it];
  for (uint64_t j0 = rlo + wave; j0 < rhi; j0 += 16) {
    float x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = a.dv[min(j0 + 4 * u, rhi - 1) * kR + lane];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j0 + 4 * u >= rhi) break;  // uniform over the wave
      r += fabs((double)x[u]);
      pend += __ballot(x[u] != 0.0f) != 0 ? 1 : 0;
    }
  }
  s_w[wave][lane] = r;
  pend = (lane == 0) ? pend : 0;
  pend = block_sum256(pend);
  if (threadIdx.x < kR)
    a.part_r[(uint64_t)it * kR + threadIdx.x] =
        ((s_w[0][threadIdx.x] + s_w[1][threadIdx.x]) + s_w[2][threadIdx.x]) + s_w[3][threadIdx.x];
  if (threadIdx.x == 0) {
    a.part_p[it] = pend;
    a.part_fa[it] = 0;
    a.part_fm[it] = 0;
  }
  retire_item(a, a.rg[it], 0, count_round);
}

// Dense phase, hub targets (in-degree > hub_deg): one item per (target, chunk
// of kBChunk in-edges) adds the previous round's message bases into dv, for
// the instances whose messages are not yet all delivered; atomics where a
// target has several chunks.
// Sum over in-edges [beg, end) of the message-base vectors (times the edge
// weight under EDGE_SCALE), four gathers in flight per lane.
template <int W, bool WGT>
__device__ __forceinline__ void bgather(const BArgs& a, const float* mu_in, uint32_t beg, uint32_t end, uint32_t r0,
                                        float (&acc)[W]) {
  uint32_t p = beg;
  for (; p + 3 < end; p += 4) {
    const uint32_t s0 = a.srcT[p], s1 = a.srcT[p + 1], s2 = a.srcT[p + 2], s3 = a.srcT[p + 3];
    float x0[W], x1[W], x2[W], x3[W];
    vload<W>(mu_in + (uint64_t)s0 * kR + r0, x0);
    vload<W>(mu_in + (uint64_t)s1 * kR + r0, x1);
    vload<W>(mu_in + (uint64_t)s2 * kR + r0, x2);
    vload<W>(mu_in + (uint64_t)s3 * kR + r0, x3);
    if constexpr (WGT) {
      const float w0 = a.wT[p], w1 = a.wT[p + 1], w2 = a.wT[p + 2], w3 = a.wT[p + 3];
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += (x0[k] * w0 + x1[k] * w1) + (x2[k] * w2 + x3[k] * w3);
    } else {
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += (x0[k] + x1[k]) + (x2[k] + x3[k]);
    }
  }
  for (; p < end; ++p) {
    float x[W];
    vload<W>(mu_in + (uint64_t)a.srcT[p] * kR + r0, x);
    const float wp = WGT ? a.wT[p] : 1.0f;
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] += WGT ? x[k] * wp : x[k];
  }
}

// Sweep rounds: the same sum, each source read from the slot of the sweep
// that last published it: this sweep's (cur) when its sweep number is below
// lo (an earlier block), else the previous sweep's (prev), which does not
// exist in the first sweep (prev_ok false: those terms are 0).
template <int W, bool WGT>
__device__ __forceinline__ void bgather_sweep(const BArgs& a, const float* cur, const float* prev, uint32_t lo,
                                              bool prev_ok, uint32_t beg, uint32_t end, uint32_t r0,
                                              float (&acc)[W]) {
  uint32_t p = beg;
  for (; p + 3 < end; p += 4) {
    const uint32_t s0 = a.srcT[p], s1 = a.srcT[p + 1], s2 = a.srcT[p + 2], s3 = a.srcT[p + 3];
    const bool n0 = s0 < lo, n1 = s1 < lo, n2 = s2 < lo, n3 = s3 < lo;
    float x0[W], x1[W], x2[W], x3[W];
    vload<W>((n0 ? cur : prev) + (uint64_t)s0 * kR + r0, x0);
    vload<W>((n1 ? cur : prev) + (uint64_t)s1 * kR + r0, x1);
    vload<W>((n2 ? cur : prev) + (uint64_t)s2 * kR + r0, x2);
    vload<W>((n3 ? cur : prev) + (uint64_t)s3 * kR + r0, x3);
    const bool o0 = n0 || prev_ok, o1 = n1 || prev_ok, o2 = n2 || prev_ok, o3 = n3 || prev_ok;
    const float w0 = WGT ? a.wT[p] : 1.0f, w1 = WGT ? a.wT[p + 1] : 1.0f;
    const float w2 = WGT ? a.wT[p + 2] : 1.0f, w3 = WGT ? a.wT[p + 3] : 1.0f;
#pragma unroll
    for (int k = 0; k < W; ++k)
      acc[k] += ((o0 ? x0[k] * w0 : 0.0f) + (o1 ? x1[k] * w1 : 0.0f)) +
                ((o2 ? x2[k] * w2 : 0.0f) + (o3 ? x3[k] * w3 : 0.0f));
  }
  for (; p < end; ++p) {
    const uint32_t sp = a.srcT[p];
    const bool np = sp < lo;
    float x[W];
    vload<W>((np ? cur : prev) + (uint64_t)sp * kR + r0, x);
    const bool op = np || prev_ok;
    const float wp = WGT ? a.wT[p] : 1.0f;
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] += op ? x[k] * wp : 0.0f;
  }
}

// Sweep rounds: block c of sweep k runs as round base + k P + c; the block
// and sweep are set here, before the round's kernels, and the round limit
// is applied.
__global__ void k_bstep(BArgs a) {
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->mode != 3) return;
  if (ctl->rounds >= ctl->max_rounds) {
    ctl->stop = 1;
    return;
  }
  const uint64_t r = ctl->rounds - ctl->base;
  ctl->sw_c = (uint32_t)(r % a.sw_P);
  ctl->sw_k = r / a.sw_P;
  ctl->sw_started = 1;
  ctl->rounds += 1;
}

template <int LPV, bool WGT, bool SWEEP>
__global__ __launch_bounds__(256) void k_bhub(BArgs a, int final_pass) {
  constexpr int W = kR / LPV;
  constexpr int IPB = 256 / LPV;
  BCtl* ctl = a.ctl;
  const float *mu_in, *mu_prev = nullptr;
  uint64_t i0 = 0, i1 = a.n_hub;
  uint32_t lo = 0;
  bool prev_ok = true;
  if constexpr (SWEEP) {
    if (bhalted(ctl) || ctl->mode != 3) return;
    const uint32_t c = ctl->sw_c;
    const uint64_t k = ctl->sw_k;
    i0 = a.sw_hoff[c];
    i1 = a.sw_hoff[c + 1];
    mu_in = (k & 1) ? a.mu2 : a.mu;
    mu_prev = (k & 1) ? a.mu : a.mu2;
    lo = (uint32_t)a.sw_bstart[c];
    prev_ok = k > 0;
  } else {
    if (!final_pass && (bhalted(ctl) || ctl->mode != 2)) return;
    mu_in = mu_of_round(a, ctl->rounds - 1);
  }
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  for (uint64_t base = i0 + (uint64_t)blockIdx.x * IPB; base < i1; base += (uint64_t)gridDim.x * IPB) {
    const uint64_t i = base + sub;
    if (i >= i1) continue;
    const uint32_t t = a.ht[i];
    const uint8_t* st = a.done + (uint64_t)a.gid[t] * kR + r0;
    bool live[W], any = false;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      live[k] = st[k] != 2;
      any |= live[k];
    }
    if (!any) continue;
    const uint32_t beg = a.rowT[t] + a.hc[i] * a.hub_chunk;
    const uint32_t end = min(a.rowT[t + 1], beg + a.hub_chunk);
    float acc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] = 0.0f;
    if constexpr (SWEEP) bgather_sweep<W, WGT>(a, mu_in, mu_prev, lo, prev_ok, beg, end, r0, acc);
    else bgather<W, WGT>(a, mu_in, beg, end, r0, acc);
    float* dst = a.dv + (uint64_t)t * kR + r0;
    if (a.rowT[t + 1] - a.rowT[t] <= a.hub_chunk) {
      float d[W];
      vload<W>(dst, d);
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (live[k]) d[k] += acc[k];
      vstore<W>(dst, d);
    } else {
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (live[k] && acc[k] != 0.0f) unsafeAtomicAdd(dst + k, acc[k]);
    }
  }
}

// Fused dense round, one block per residual item (a vertex range inside one
// graph), LPV lanes per vertex. Per vertex and running instance: deliver the
// previous round's messages by pulling over in-edges (hubs: take dv, filled
// by k_bhub), add |d| to the item's residual, then claim: fold d into v and
// publish alpha d / outdeg as this round's message base (renumbered order,
// ping-pong buffer). Instances finished at the previous check get their last
// messages delivered into dv; instances delivered earlier are skipped.
// final_pass: delivery only, after a stop in the dense phase.
template <int LPV, bool KAHAN, bool WGT, bool SWEEP>
__global__ __launch_bounds__(256) void k_bfused(BArgs a, int final_pass) {
  constexpr int W = kR / LPV;
  constexpr int VPB = 256 / LPV;
  __shared__ double s_part[VPB][kR];
  BCtl* ctl = a.ctl;
  uint32_t it;
  const float *mu_in, *mu_prev = nullptr;
  float* mu_out;
  uint32_t lo = 0;
  bool prev_ok = true, first = false;
  if constexpr (SWEEP) {
    // block c of sweep k: earlier blocks published in this sweep (mu_out's
    // slot), later blocks and this one in the previous sweep (mu_prev)
    if (bhalted(ctl) || ctl->mode != 3) return;
    const uint32_t c = ctl->sw_c;
    const uint64_t k = ctl->sw_k;
    const uint32_t ib = a.sw_ioff[c], ie = a.sw_ioff[c + 1];
    if (blockIdx.x >= ie - ib) return;
    it = a.sw_items[ib + blockIdx.x];
    if (it == ~0u) return;
    mu_out = (k & 1) ? a.mu2 : a.mu;
    mu_in = mu_out;
    mu_prev = (k & 1) ? a.mu : a.mu2;
    lo = (uint32_t)a.sw_bstart[c];
    prev_ok = k > 0;
    first = k == 0;  // the deltas left by the sparse rounds are still in dv
  } else {
    if (!final_pass && (bhalted(ctl) || ctl->mode != 2)) return;
    it = a.item_order[blockIdx.x];
    if (it == ~0u) return;
    const uint64_t t = ctl->rounds;
    mu_in = mu_of_round(a, t - 1);
    mu_out = mu_of_round(a, t);
  }
  const uint32_t g = a.rg[it];
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  uint8_t st[W];
  bool run_any = false, one_any = false;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    st[k] = a.done[(uint64_t)g * kR + r0 + k];
    if (final_pass && st[k] == 0) st[k] = 1;  // deliver only
    run_any |= st[k] == 0;
    one_any |= st[k] == 1;
  }
  const bool mine = run_any || one_any;
  double racc[W];
#pragma unroll
  for (int k = 0; k < W; ++k) racc[k] = 0.0;
  uint64_t act = 0, msg = 0;
  if (__syncthreads_or(mine)) {
    // vertices without edges only matter in the first sweep, which folds in
    // the deltas the sparse rounds left (the synchronous phase's opening
    // claim does that for them)
    const uint64_t xend = first ? a.rhi[it] : a.rha[it];
    for (uint64_t x = a.rlo[it] + sub; x < xend; x += VPB) {
      if (!mine) continue;
      const uint64_t j = a.vord[x];
      const uint32_t b0 = a.rowT[j], b1 = a.rowT[j + 1];
      const bool hub = b1 - b0 > a.hub_deg;
      float* dvp = a.dv + j * kR + r0;
      float old[W], d[W], vv[W], cc[W];
      // the state is loaded before the gathers so that its latency overlaps
      // theirs (in dense rounds nearly every running lane claims)
      if (run_any) {
        vload<W>(a.v + j * kR + r0, vv);
        if constexpr (KAHAN) vload<W>(a.c + j * kR + r0, cc);
      }
      if (hub || one_any || first) {
        vload<W>(dvp, old);
      } else {
#pragma unroll
        for (int k = 0; k < W; ++k) old[k] = 0.0f;
      }
      if (hub) {
#pragma unroll
        for (int k = 0; k < W; ++k) d[k] = old[k];
      } else {
#pragma unroll
        for (int k = 0; k < W; ++k) d[k] = first ? old[k] : 0.0f;
        if constexpr (SWEEP) bgather_sweep<W, WGT>(a, mu_in, mu_prev, lo, prev_ok, b0, b1, r0, d);
        else bgather<W, WGT>(a, mu_in, b0, b1, r0, d);
      }
      bool cl[W], claim_any = false;
      uint32_t nclaim = 0;
      float nd[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        // sweep rounds count a running lane's residual from what it sends
        // below (its messages not yet consumed at the end of the sweep)
        if (SWEEP ? st[k] == 1 : st[k] != 2) racc[k] += fabs((double)d[k]);
        cl[k] = st[k] == 0 && d[k] != 0.0f;
        claim_any |= cl[k];
        nclaim += cl[k] ? 1u : 0u;
        nd[k] = st[k] == 2 ? old[k] : (st[k] == 1 ? d[k] : 0.0f);
      }
      if (hub || one_any) vstore<W>(dvp, nd);
      if (claim_any) {
        if constexpr (KAHAN) {
#pragma clang fp contract(off)
#pragma unroll
          for (int k = 0; k < W; ++k) {
            if (cl[k]) {
              const float y = d[k] - cc[k];
              const float s = vv[k] + y;
              cc[k] = (s - vv[k]) - y;
              vv[k] = s;
            }
          }
          vstore<W>(a.c + j * kR + r0, cc);
        } else {
#pragma unroll
          for (int k = 0; k < W; ++k)
            if (cl[k]) vv[k] += d[k];
        }
        vstore<W>(a.v + j * kR + r0, vv);
      }
      // (sweep rounds: finished instances publish zeros, which the blocks
      // after this one read in the same sweep)
      if (run_any || (SWEEP && one_any)) {
        const uint32_t deg = a.row[j + 1] - a.row[j];
        const double coef = WGT ? a.alpha : (deg ? a.alpha / (double)deg : 0.0);
        float mu[W];
#pragma unroll
        for (int k = 0; k < W; ++k) mu[k] = cl[k] ? (float)(coef * (double)d[k]) : 0.0f;
        if (deg) vstore<W>(mu_out + (uint64_t)a.perm[j] * kR + r0, mu);  // no reader otherwise
        if constexpr (SWEEP) {
          const double cf = a.sw_coef[j];
#pragma unroll
          for (int k = 0; k < W; ++k)
            if (st[k] == 0) racc[k] += fabs((double)mu[k]) * cf;
        }
        act += nclaim;
        msg += (uint64_t)nclaim * deg;
      }
    }
  }
  // per-lane residual of the item: sum over the block's vertex groups in order
#pragma unroll
  for (int k = 0; k < W; ++k) s_part[sub][r0 + k] = racc[k];
  act = block_sum256(act);
  msg = block_sum256(msg);
  if (threadIdx.x < kR) {
    double sr = 0.0;
    for (int u = 0; u < VPB; ++u) sr += s_part[u][threadIdx.x];
    a.part_r[(uint64_t)it * kR + threadIdx.x] = sr;
  }
  if (threadIdx.x == 0) {
    a.part_p[it] = 0;
    a.part_fa[it] = act;
    a.part_fm[it] = msg;
  }
  // retired after the kernel: k_bretire_dense, k_bretire_sweep
}

// Sweep rounds stopped by the round limit: deliver the messages still in
// flight into dv. After round base + k P + cl, a source numbered s last
// published in sweep k if s < L (blocks up to cl), else in sweep k - 1; a
// target of block bt last pulled in sweep k if bt <= cl, else in sweep
// k - 1; a message is in flight when published at or after the target's
// pull ((sweep, block) order, equal blocks included). Targets with in-degree
// above hub_deg are handled by k_bdeliver_hub (their dv is always current).
template <int LPV, bool WGT>
__global__ __launch_bounds__(256) void k_bdeliver(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int VPB = 256 / LPV;
  const BCtl* ctl = a.ctl;
  const uint64_t k = ctl->sw_k;
  const uint32_t cl = ctl->sw_c;
  const uint32_t L = (uint32_t)a.sw_bstart[cl + 1];
  const float* cur = (k & 1) ? a.mu2 : a.mu;
  const float* prev = (k & 1) ? a.mu : a.mu2;
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  for (uint64_t base = (uint64_t)blockIdx.x * VPB; base < a.N; base += (uint64_t)gridDim.x * VPB) {
    const uint64_t j = base + sub;
    if (j >= a.N) continue;
    const uint32_t b0 = a.rowT[j], b1 = a.rowT[j + 1];
    if (b1 - b0 > a.hub_deg) continue;
    const uint32_t bt = a.sw_blk[j];
    const uint32_t T0 = (uint32_t)a.sw_bstart[bt];
    const bool processed = bt <= cl;
    uint8_t st[W];
    bool live = false;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      st[q] = a.done[(uint64_t)a.gid[j] * kR + r0 + q];
      live |= st[q] != 2;
    }
    if (!live) continue;
    float acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0f;
    for (uint32_t p = b0; p < b1; ++p) {
      const uint32_t sp = a.srcT[p];
      const float* src = nullptr;
      if (processed) {
        if (sp >= T0 && sp < L) src = cur;
      } else {
        if (sp < L) src = cur;
        else if (sp >= T0 && k > 0) src = prev;
      }
      if (!src) continue;
      float x[W];
      vload<W>(src + (uint64_t)sp * kR + r0, x);
      const float wp = WGT ? a.wT[p] : 1.0f;
#pragma unroll
      for (int q = 0; q < W; ++q) acc[q] += x[q] * wp;
    }
    float* dvp = a.dv + j * kR + r0;
    float old[W], nd[W];
    vload<W>(dvp, old);
#pragma unroll
    for (int q = 0; q < W; ++q) {
      // what dv holds for the lane: the sparse rounds' deltas (first sweep,
      // block not reached), the delivered sum (finished lanes of processed
      // blocks), else nothing (a running lane's dv is not kept current)
      const bool keep = (k == 0 && !processed) || (st[q] == 1 && processed);
      nd[q] = st[q] == 2 ? old[q] : (keep ? old[q] : 0.0f) + acc[q];
    }
    vstore<W>(dvp, nd);
  }
}

template <int LPV, bool WGT>
__global__ __launch_bounds__(256) void k_bdeliver_hub(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int IPB = 256 / LPV;
  const BCtl* ctl = a.ctl;
  const uint64_t k = ctl->sw_k;
  const uint32_t cl = ctl->sw_c;
  const uint32_t L = (uint32_t)a.sw_bstart[cl + 1];
  const float* cur = (k & 1) ? a.mu2 : a.mu;
  const float* prev = (k & 1) ? a.mu : a.mu2;
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  for (uint64_t base = (uint64_t)blockIdx.x * IPB; base < a.n_hub; base += (uint64_t)gridDim.x * IPB) {
    const uint64_t i = base + sub;
    if (i >= a.n_hub) continue;
    const uint32_t t = a.ht[i];
    const uint32_t bt = a.sw_blk[t];
    const uint32_t T0 = (uint32_t)a.sw_bstart[bt];
    const bool processed = bt <= cl;
    const uint8_t* stp = a.done + (uint64_t)a.gid[t] * kR + r0;
    bool live[W], any = false;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      live[q] = stp[q] != 2;
      any |= live[q];
    }
    if (!any) continue;
    const uint32_t beg = a.rowT[t] + a.hc[i] * a.hub_chunk;
    const uint32_t end = min(a.rowT[t + 1], beg + a.hub_chunk);
    float acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0f;
    for (uint32_t p = beg; p < end; ++p) {
      const uint32_t sp = a.srcT[p];
      const float* src = nullptr;
      if (processed) {
        if (sp >= T0 && sp < L) src = cur;
      } else {
        if (sp < L) src = cur;
        else if (sp >= T0 && k > 0) src = prev;
      }
      if (!src) continue;
      float x[W];
      vload<W>(src + (uint64_t)sp * kR + r0, x);
      const float wp = WGT ? a.wT[p] : 1.0f;
#pragma unroll
      for (int q = 0; q < W; ++q) acc[q] += x[q] * wp;
    }
    float* dst = a.dv + (uint64_t)t * kR + r0;
#pragma unroll
    for (int q = 0; q < W; ++q)
      if (live[q] && acc[q] != 0.0f) unsafeAtomicAdd(dst + q, acc[q]);
  }
}

// After a delivery: back to a sparse state whose residual pass (count 0)
// takes every delivered instance to finished.
__global__ void k_bto_sparse(BCtl* ctl) {
  ctl->mode = 0;
  ctl->stop = 0;
  ctl->ticket = 0;
}

// Item tickets of every graph and the graph ticket back to 0. A run stopped
// between sweep rounds leaves some graphs' items of the interrupted sweep
// counted; every run and every delivery starts from here.
__global__ void k_breset_tickets(BArgs a) {
  for (uint32_t g = threadIdx.x; g < a.G; g += blockDim.x) a.g_ticket[g] = 0;
  if (threadIdx.x == 0) a.ctl->ticket = 0;
}

__global__ void k_bstats(BArgs a, uint32_t nblocks) {
  if (bhalted(a.ctl) || a.ctl->mode >= 2) return;
  uint64_t s = 0, m = 0;
  for (uint32_t i = threadIdx.x; i < nblocks; i += 256) {
    s += a.part_a[i];
    m += a.part_m[i];
  }
  s = block_sum256(s);
  m = block_sum256(m);
  if (threadIdx.x == 0) {
    a.ctl->activations += s;
    a.ctl->messages += m;
  }
}

__global__ void k_binit(BCtl* ctl, double eps, uint64_t max_rounds, uint32_t dense_mode) {
  ctl->done = 0;
  ctl->stop = 0;
  ctl->mode = 0;
  ctl->prev_all_done = 0;
  ctl->dense_mode = dense_mode;
  ctl->sw_c = 0;
  ctl->sw_started = 0;
  ctl->sw_k = 0;
  ctl->base = 0;
  ctl->ticket = 0;
  ctl->rounds = 0;
  ctl->max_rounds = max_rounds;
  ctl->pending = 0;
  ctl->activations = 0;
  ctl->messages = 0;
  ctl->eps = eps;
}

// Union graph: rows of graph g shifted by its edge offset, columns by its
// vertex offset.
__global__ void k_union_rows(const uint32_t* row, uint64_t n, uint64_t voff, uint64_t eoff, uint32_t g,
                             uint32_t* urow, uint32_t* gid) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = i; j < n; j += st) {
    urow[voff + j] = (uint32_t)(row[j] + eoff);
    gid[voff + j] = g;
  }
}

__global__ void k_union_cols(const uint32_t* col, uint64_t m, uint64_t voff, uint64_t eoff, uint32_t* ucol) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = i; e < m; e += st) ucol[eoff + e] = (uint32_t)(col[e] + voff);
}

__global__ void k_set_last(uint32_t* p, uint64_t idx, uint32_t val) { p[idx] = val; }

// Union edge weights (as float) of graph g at its edge offset.
template <typename T>
__global__ void k_union_weights(const T* w, uint64_t m, uint64_t eoff, float* uw) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = i; e < m; e += st) uw[eoff + e] = (float)w[e];
}

// Sweep numbers of the in-edge sources: out[p] = psw[inv[srcT[p]]].
__global__ void k_brenumber(const uint32_t* srcT, const uint32_t* inv, const uint32_t* psw, uint64_t m,
                            uint32_t* out) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = i; p < m; p += st) out[p] = psw[inv[srcT[p]]];
}

// coef[j] = sum over out-edges (j, t) with blk[t] <= blk[j] of |w| (1 when
// unweighted): the multiplier of j's message base in the pending mass left
// at the end of a sweep. One wave per vertex.
__global__ __launch_bounds__(256) void k_bsweep_coef(const uint32_t* row, const uint32_t* col, const float* w,
                                                     const uint32_t* blk, uint64_t n, double* coef) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t j = wave; j < n; j += nwaves) {
    const uint32_t bj = blk[j];
    double acc = 0.0;
    for (uint32_t e = row[j] + lane; e < row[j + 1]; e += 64)
      if (blk[col[e]] <= bj) acc += w ? fabs((double)w[e]) : 1.0;
    acc = wave_sum(acc);
    if (lane == 0) coef[j] = acc;
  }
}

// Weights in in-edge order: wT[p] = w[eidT[p]].
__global__ void k_bgather_weights(const float* w, const uint32_t* eidT, uint64_t m, float* wT) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = i; p < m; p += st) wT[p] = w[eidT[p]];
}

static uint32_t bgrid(uint64_t count, uint32_t block = 256) {
  uint64_t g = (count + block - 1) / block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 8192));
}

}  // namespace daic

using namespace daic;

struct BTune {
  int lpv_claim = 16, lpv_fused = 16, lpv_push = 16;
  uint32_t grid_claim = 4096, grid_hub = 2048, grid_push = 8192;
};

struct daic_batch {
  uint32_t G = 0;
  std::vector<uint64_t> voff, n_of;   // per graph vertex offset and count
  std::vector<uint32_t> rhs;          // right-hand sides used per graph
  bool kahan = false;
  daic_graph* ug = nullptr;           // union graph (owned)
  BArgs a{};
  BCtl* h_ctl = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  uint32_t exec_K = 0;
  const void* exec_stream = nullptr;
  uint32_t exec_dense = 0, exec_P = 0;
  hipGraphExec_t exec_sw = nullptr;   // sweep rounds only
  hipGraph_t graph_sw = nullptr;
  BTune tune;
  bool tuned = false;
  std::vector<void*> allocs;
  // sweep rounds (built for a block count P on first use)
  BArgs as{};
  uint32_t sw_P = 0;
  uint32_t sw_grid = 0;               // fused-pass blocks per sweep round
  std::vector<void*> sw_allocs;
  std::vector<uint32_t> xcd_of;       // XCD slot given to each graph
};

namespace daic {

template <int LPV, bool KAHAN>
static void launch_claim(daic_batch* b, hipStream_t s) {
  hipLaunchKernelGGL((k_bclaim<LPV, KAHAN>), dim3(b->tune.grid_claim), dim3(256), 0, s, b->a);
}

static void enqueue_claim(daic_batch* b, hipStream_t s) {
  const int l = b->tune.lpv_claim;
  if (b->kahan) {
    if (l == 16) launch_claim<16, true>(b, s);
    else if (l == 32) launch_claim<32, true>(b, s);
    else launch_claim<64, true>(b, s);
  } else {
    if (l == 16) launch_claim<16, false>(b, s);
    else if (l == 32) launch_claim<32, false>(b, s);
    else launch_claim<64, false>(b, s);
  }
  hipLaunchKernelGGL(k_bstats, dim3(1), dim3(256), 0, s, b->a, b->tune.grid_claim);
}

template <int LPV, bool WGT>
static void launch_dense_w(daic_batch* b, hipStream_t s, int final_pass) {
  if (b->a.n_hub)
    hipLaunchKernelGGL((k_bhub<LPV, WGT, false>), dim3(b->tune.grid_hub), dim3(256), 0, s, b->a, final_pass);
  if (b->kahan)
    hipLaunchKernelGGL((k_bfused<LPV, true, WGT, false>), dim3(b->a.n_fused_blocks), dim3(256), 0, s, b->a, final_pass);
  else
    hipLaunchKernelGGL((k_bfused<LPV, false, WGT, false>), dim3(b->a.n_fused_blocks), dim3(256), 0, s, b->a, final_pass);
  hipLaunchKernelGGL(k_bretire_dense, dim3(b->a.G), dim3(256), 0, s, b->a, final_pass);
}

// One sweep round (block and sweep from the control block): step, hub sums
// of the block's hub targets, fused pass over the block's items.
template <int LPV, bool WGT>
static void launch_sweep_w(daic_batch* b, hipStream_t s) {
  const BArgs& as = b->as;
  hipLaunchKernelGGL(k_bstep, dim3(1), dim3(1), 0, s, as);
  if (as.n_hub) hipLaunchKernelGGL((k_bhub<LPV, WGT, true>), dim3(b->tune.grid_hub), dim3(256), 0, s, as, 0);
  if (b->kahan)
    hipLaunchKernelGGL((k_bfused<LPV, true, WGT, true>), dim3(b->sw_grid), dim3(256), 0, s, as, 0);
  else
    hipLaunchKernelGGL((k_bfused<LPV, false, WGT, true>), dim3(b->sw_grid), dim3(256), 0, s, as, 0);
  hipLaunchKernelGGL(k_bretire_sweep, dim3(as.G), dim3(256), 0, s, as);
}

static void enqueue_sweep(daic_batch* b, hipStream_t s) {
  const int l = b->tune.lpv_fused;
  const bool w = b->a.w != nullptr;
  if (l == 16) w ? launch_sweep_w<16, true>(b, s) : launch_sweep_w<16, false>(b, s);
  else if (l == 32) w ? launch_sweep_w<32, true>(b, s) : launch_sweep_w<32, false>(b, s);
  else w ? launch_sweep_w<64, true>(b, s) : launch_sweep_w<64, false>(b, s);
}

// Delivery of the messages in flight when sweep rounds stop at the round
// limit, then the residual of the delivered state.
template <bool WGT>
static void launch_sweep_deliver_w(daic_batch* b, hipStream_t s) {
  const BArgs& as = b->as;
  hipLaunchKernelGGL((k_bdeliver<16, WGT>), dim3(bgrid(as.N, 16)), dim3(256), 0, s, as);
  if (as.n_hub) hipLaunchKernelGGL((k_bdeliver_hub<16, WGT>), dim3(bgrid(as.n_hub, 16)), dim3(256), 0, s, as);
  hipLaunchKernelGGL(k_bto_sparse, dim3(1), dim3(1), 0, s, as.ctl);
  hipLaunchKernelGGL(k_breset_tickets, dim3(1), dim3(256), 0, s, b->a);
  hipLaunchKernelGGL(k_bresidual, dim3(b->a.n_res), dim3(256), 0, s, b->a, 0);
}

template <int LPV>
static void launch_dense(daic_batch* b, hipStream_t s, int final_pass) {
  if (b->a.w) launch_dense_w<LPV, true>(b, s, final_pass);
  else launch_dense_w<LPV, false>(b, s, final_pass);
}

// Dense-phase round (hub sums, then the fused pass); both kernels return at
// once outside the dense phase.
static void enqueue_dense(daic_batch* b, hipStream_t s, int final_pass) {
  const int l = b->tune.lpv_fused;
  if (l == 16) launch_dense<16>(b, s, final_pass);
  else if (l == 32) launch_dense<32>(b, s, final_pass);
  else launch_dense<64>(b, s, final_pass);
}

static void enqueue_push(daic_batch* b, hipStream_t s) {
  const int l = b->tune.lpv_push;
  const uint32_t g = b->tune.grid_push;
  if (l == 16) hipLaunchKernelGGL(k_bpush<16>, dim3(g), dim3(256), 0, s, b->a);
  else hipLaunchKernelGGL(k_bpush<64>, dim3(g), dim3(256), 0, s, b->a);
}

// One round in whichever mode the control block holds: sparse (claim, push,
// residual), the claim that opens the dense phase, or a fused dense round.
// Sweep set-up for P blocks per graph: graph g's block c is its vertices
// [c B_g, (c+1) B_g), B_g = ceil(n_g / P). The sweep numbering is
// block-major over the union (out-degree order, the dense rounds'
// renumbering, inside a block), so that a source's block follows from its
// number; residual items never cross a block; each block gets its items in
// XCD-interleaved order and its hub items longest first.
static daic_status batch_sweep_setup(daic_batch* b, uint32_t P, hipStream_t s) {
  if (b->sw_P == P) return DAIC_OK;
  for (void* q : b->sw_allocs)
    if (q) (void)hipFree(q);
  b->sw_allocs.clear();
  b->sw_P = 0;
  const BArgs& a = b->a;
  const uint64_t N = a.N, M = b->ug->dev.m;
  const uint32_t G = b->G;
  auto grab = [&](void** q, size_t bytes) -> daic_status {
    void* m = nullptr;
    hipError_t e = hipMalloc(&m, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(DAIC_E_OOM, "sweep set-up: hipMalloc of %zu bytes failed", bytes);
    b->sw_allocs.push_back(m);
    *q = m;
    return DAIC_OK;
  };
  std::vector<uint32_t> perm(N), inv(N), rt(N + 1), ro(N + 1), blk(N), psw(N);
  DAIC_HIP(hipMemcpy(perm.data(), b->ug->pull.perm, N * 4, hipMemcpyDeviceToHost));
  DAIC_HIP(hipMemcpy(rt.data(), b->ug->pull.rowT, (N + 1) * 4, hipMemcpyDeviceToHost));
  DAIC_HIP(hipMemcpy(ro.data(), a.row, (N + 1) * 4, hipMemcpyDeviceToHost));
  for (uint64_t j = 0; j < N; ++j) inv[perm[j]] = (uint32_t)j;
  std::vector<uint64_t> Bg(G);
  for (uint32_t g = 0; g < G; ++g) {
    const uint64_t n = b->voff[g + 1] - b->voff[g];
    Bg[g] = std::max<uint64_t>(1, (n + P - 1) / P);
    for (uint64_t v = b->voff[g]; v < b->voff[g + 1]; ++v) blk[v] = (uint32_t)((v - b->voff[g]) / Bg[g]);
  }
  std::vector<uint64_t> bstart(P + 1, 0);
  for (uint64_t j = 0; j < N; ++j) ++bstart[blk[j] + 1];
  for (uint32_t c = 0; c < P; ++c) bstart[c + 1] += bstart[c];
  {
    std::vector<uint64_t> fill(bstart.begin(), bstart.end() - 1);
    for (uint64_t q = 0; q < N; ++q) {
      const uint32_t j = inv[q];
      psw[j] = (uint32_t)fill[blk[j]]++;
    }
  }
  // items: (graph, block) segments split at kResChunk vertices or kItemWork work
  std::vector<uint32_t> rg, gfi, iblk;
  std::vector<uint64_t> rlo, rhi, rw;
  for (uint32_t g = 0; g < G; ++g) {
    gfi.push_back((uint32_t)rg.size());
    for (uint32_t c = 0; c < P; ++c) {
      const uint64_t seg_lo = b->voff[g] + c * Bg[g];
      const uint64_t seg_hi = std::min<uint64_t>(b->voff[g + 1], seg_lo + Bg[g]);
      if (seg_lo >= seg_hi) continue;
      uint64_t lo = seg_lo, w = 0;
      for (uint64_t j = seg_lo; j < seg_hi; ++j) {
        const uint32_t deg = rt[j + 1] - rt[j];
        w += (deg > a.hub_deg ? 0 : deg) + kVertexWork;
        if (j + 1 - lo >= kSwResChunk || w >= kSwItemWork || j + 1 == seg_hi) {
          rg.push_back(g);
          rlo.push_back(lo);
          rhi.push_back(j + 1);
          rw.push_back(w);
          iblk.push_back(c);
          lo = j + 1;
          w = 0;
        }
      }
    }
    if (b->voff[g] == b->voff[g + 1]) {  // empty graph: one empty item in block 0
      rg.push_back(g);
      rlo.push_back(b->voff[g]);
      rhi.push_back(b->voff[g]);
      rw.push_back(0);
      iblk.push_back(0);
    }
  }
  gfi.push_back((uint32_t)rg.size());
  const size_t nres = rg.size();
  std::vector<uint32_t> vord(N);
  std::vector<uint64_t> rha(nres);
  for (uint64_t j = 0; j < N; ++j) vord[j] = (uint32_t)j;
  auto isolated = [&](uint32_t j) { return rt[j + 1] == rt[j] && ro[j + 1] == ro[j]; };
  auto pulled = [&](uint32_t j) { const uint32_t d = rt[j + 1] - rt[j]; return d > a.hub_deg ? 0u : d; };
  for (size_t k = 0; k < nres; ++k) {
    std::stable_sort(vord.begin() + rlo[k], vord.begin() + rhi[k], [&](uint32_t x, uint32_t y) {
      const bool ix = isolated(x), iy = isolated(y);
      if (ix != iy) return iy;
      return pulled(x) > pulled(y);
    });
    uint64_t e = rlo[k];
    while (e < rhi[k] && !isolated(vord[e])) ++e;
    rha[k] = e;
  }
  // per block: items in XCD-interleaved order (each graph keeps its XCD)
  constexpr uint32_t kXcd = 8;
  std::vector<uint32_t> items, ioff(P + 1, 0);
  uint32_t grid = 1;
  for (uint32_t c = 0; c < P; ++c) {
    std::vector<std::vector<uint32_t>> bins(kXcd);
    for (size_t k = 0; k < nres; ++k)
      if (iblk[k] == c) bins[b->xcd_of[rg[k]] % kXcd].push_back((uint32_t)k);
    for (auto& bn : bins)
      std::stable_sort(bn.begin(), bn.end(), [&](uint32_t x, uint32_t y) { return rw[x] > rw[y]; });
    size_t longest = 0;
    for (auto& bn : bins) longest = std::max(longest, bn.size());
    std::vector<uint32_t> order(longest * kXcd, ~0u);
    for (uint32_t x = 0; x < kXcd; ++x)
      for (size_t i = 0; i < bins[x].size(); ++i) order[i * kXcd + x] = bins[x][i];
    items.insert(items.end(), order.begin(), order.end());
    ioff[c + 1] = (uint32_t)items.size();
    grid = std::max<uint32_t>(grid, (uint32_t)order.size());
  }
  // hub items grouped by block, longest first
  std::vector<uint32_t> ht, hc, hoff(P + 1, 0);
  {
    std::vector<std::vector<std::pair<uint32_t, uint64_t>>> per(P);
    for (uint64_t t = 0; t < N; ++t) {
      const uint32_t deg = rt[t + 1] - rt[t];
      if (deg <= a.hub_deg) continue;
      for (uint32_t c = 0; c * kSwHubChunk < deg; ++c)
        per[blk[t]].push_back({std::min(kSwHubChunk, deg - c * kSwHubChunk), (t << 32) | c});
    }
    for (uint32_t c = 0; c < P; ++c) {
      std::stable_sort(per[c].begin(), per[c].end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      for (auto& it : per[c]) {
        ht.push_back((uint32_t)(it.second >> 32));
        hc.push_back((uint32_t)it.second);
      }
      hoff[c + 1] = (uint32_t)ht.size();
    }
  }
  BArgs as = a;
  void* q = nullptr;
  daic_status rc;
#define SWGRAB(field, type, bytes, src)                                                    \
  do {                                                                                     \
    if ((rc = grab(&q, (bytes)))) return rc;                                               \
    as.field = (type)q;                                                                    \
    if ((bytes) && (src)) DAIC_HIP(hipMemcpy(q, (src), (bytes), hipMemcpyHostToDevice));   \
  } while (0)
  SWGRAB(perm, const uint32_t*, N * 4, psw.data());
  SWGRAB(sw_blk, const uint32_t*, N * 4, blk.data());
  SWGRAB(sw_bstart, const uint64_t*, (P + 1) * 8, bstart.data());
  SWGRAB(sw_items, const uint32_t*, items.size() * 4, items.data());
  SWGRAB(sw_ioff, const uint32_t*, (P + 1) * 4, ioff.data());
  SWGRAB(sw_hoff, const uint32_t*, (P + 1) * 4, hoff.data());
  SWGRAB(ht, const uint32_t*, ht.size() * 4, ht.data());
  SWGRAB(hc, const uint32_t*, hc.size() * 4, hc.data());
  SWGRAB(rg, const uint32_t*, nres * 4, rg.data());
  SWGRAB(rlo, const uint64_t*, nres * 8, rlo.data());
  SWGRAB(rhi, const uint64_t*, nres * 8, rhi.data());
  SWGRAB(rha, const uint64_t*, nres * 8, rha.data());
  SWGRAB(g_first_item, const uint32_t*, gfi.size() * 4, gfi.data());
  SWGRAB(vord, const uint32_t*, N * 4, vord.data());
  SWGRAB(part_r, double*, nres * kR * 8, (const void*)nullptr);
  SWGRAB(part_p, uint64_t*, nres * 8, (const void*)nullptr);
  SWGRAB(part_fa, uint64_t*, nres * 8, (const void*)nullptr);
  SWGRAB(part_fm, uint64_t*, nres * 8, (const void*)nullptr);
  SWGRAB(sw_coef, const double*, N * 8, (const void*)nullptr);
  SWGRAB(srcT, const uint32_t*, M * 4, (const void*)nullptr);
#undef SWGRAB
  as.n_res = (uint32_t)nres;
  as.n_hub = ht.size();
  as.hub_chunk = kSwHubChunk;
  as.sw_P = P;
  {
    uint32_t* d_inv = nullptr;
    DAIC_HIP(hipMalloc(&d_inv, std::max<uint64_t>(N, 1) * 4));
    hipError_t e = hipMemcpy(d_inv, inv.data(), N * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && M)
      hipLaunchKernelGGL(k_brenumber, dim3(bgrid(M)), dim3(256), 0, s, a.srcT, d_inv, as.perm, M,
                         const_cast<uint32_t*>(as.srcT));
    if (e == hipSuccess && N)
      hipLaunchKernelGGL(k_bsweep_coef, dim3(bgrid(N, 4)), dim3(256), 0, s, a.row, a.col, a.w, as.sw_blk, N,
                         const_cast<double*>(as.sw_coef));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_inv);
    if (e != hipSuccess) return fail(DAIC_E_DEVICE, "sweep set-up: %s", hipGetErrorString(e));
  }
  b->as = as;
  b->sw_grid = grid;
  b->sw_P = P;
  return DAIC_OK;
}

// A sparse or synchronous-dense round; sweep rounds are a graph of their own
// (the host launches the one that matches the control block's mode).
static void enqueue_round(daic_batch* b, hipStream_t s) {
  enqueue_claim(b, s);
  enqueue_push(b, s);
  enqueue_dense(b, s, 0);
  hipLaunchKernelGGL(k_bresidual, dim3(b->a.n_res), dim3(256), 0, s, b->a, 1);
}

}  // namespace daic

extern "C" {

void daic_batch_destroy(daic_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec_sw) (void)hipGraphExecDestroy(b->exec_sw);
  if (b->graph_sw) (void)hipGraphDestroy(b->graph_sw);
  for (void* q : b->allocs)
    if (q) (void)hipFree(q);
  for (void* q : b->sw_allocs)
    if (q) (void)hipFree(q);
  if (b->ug) daic_graph_destroy(b->ug);
  if (b->h_ctl) (void)hipHostFree(b->h_ctl);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

daic_status daic_batch_create(uint32_t n_graphs, const daic_graph* const* graphs, const uint32_t* rhs_per_graph,
                              daic_op op, daic_g gk, double alpha, daic_dtype state, daic_batch** out) {
  if (!out) return fail(DAIC_E_INVALID, "out is null");
  *out = nullptr;
  if (n_graphs == 0 || !graphs || !rhs_per_graph) return fail(DAIC_E_INVALID, "no graphs");
  if (op != DAIC_SUM || (gk != DAIC_G_DEG_SCALE && gk != DAIC_G_EDGE_SCALE))
    return fail(DAIC_E_UNSUPPORTED,
                "batched runs take SUM with DEG_SCALE (personalized PageRank) or EDGE_SCALE (weighted, e.g. Adsorption)");
  if (state != DAIC_F32 && state != DAIC_F32_KAHAN)
    return fail(DAIC_E_UNSUPPORTED, "batched runs take F32 or F32_KAHAN state");
  if (!std::isfinite(alpha)) return fail(DAIC_E_INVALID, "alpha must be finite");
  uint64_t N = 0, M = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    if (!graphs[g]) return fail(DAIC_E_INVALID, "graph %u is null", g);
    if (rhs_per_graph[g] == 0 || rhs_per_graph[g] > (uint32_t)kR)
      return fail(DAIC_E_INVALID, "right-hand sides per graph must be in 1..%d", kR);
    if (!graphs[g]->dev.row32) return fail(DAIC_E_UNSUPPORTED, "graph %u has m >= 2^32", g);
    if (gk == DAIC_G_EDGE_SCALE && graphs[g]->dev.m && !graphs[g]->dev.w)
      return fail(DAIC_E_INVALID, "EDGE_SCALE needs edge weights (graph %u has none)", g);
    N += graphs[g]->dev.n;
    M += graphs[g]->dev.m;
  }
  if (N >= 0x7FFFFFFFull || M >= 0x7FFFFFFFull) return fail(DAIC_E_UNSUPPORTED, "union graph too large");
  std::unique_ptr<daic_batch> b(new daic_batch());
  b->G = n_graphs;
  b->kahan = state == DAIC_F32_KAHAN;
  b->rhs.assign(rhs_per_graph, rhs_per_graph + n_graphs);
  hipStream_t s = nullptr;
  DAIC_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  s = b->stream;
  auto grab = [&](void** p, size_t bytes) -> daic_status {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(DAIC_E_OOM, "hipMalloc of %zu bytes failed", bytes);
    b->allocs.push_back(q);
    *p = q;
    return DAIC_OK;
  };
  // union graph
  uint64_t* urow64 = nullptr;
  uint32_t* ucol = nullptr;
  uint32_t* urow = nullptr;
  uint32_t* gid = nullptr;
  daic_status rc;
  void* ptr;
  if ((rc = grab(&ptr, (N + 1) * 4))) { daic_batch_destroy(b.release()); return rc; }
  urow = (uint32_t*)ptr;
  if ((rc = grab(&ptr, M * 4))) { daic_batch_destroy(b.release()); return rc; }
  ucol = (uint32_t*)ptr;
  if ((rc = grab(&ptr, N * 4))) { daic_batch_destroy(b.release()); return rc; }
  gid = (uint32_t*)ptr;
  float* uw = nullptr;
  if (gk == DAIC_G_EDGE_SCALE) {
    if ((rc = grab(&ptr, M * 4))) { daic_batch_destroy(b.release()); return rc; }
    uw = (float*)ptr;
  }
  uint64_t voff = 0, eoff = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    const GraphDev& d = graphs[g]->dev;
    b->voff.push_back(voff);
    b->n_of.push_back(d.n);
    if (d.n) hipLaunchKernelGGL(k_union_rows, dim3(bgrid(d.n)), dim3(256), 0, s, static_cast<const uint32_t*>(d.row),
                                d.n, voff, eoff, g, urow, gid);
    if (d.m) hipLaunchKernelGGL(k_union_cols, dim3(bgrid(d.m)), dim3(256), 0, s, d.col, d.m, voff, eoff, ucol);
    if (uw && d.m) {
      if (d.w_type == DAIC_F64)
        hipLaunchKernelGGL(k_union_weights<double>, dim3(bgrid(d.m)), dim3(256), 0, s, (const double*)d.w, d.m, eoff, uw);
      else if (d.w_type == DAIC_F32)
        hipLaunchKernelGGL(k_union_weights<float>, dim3(bgrid(d.m)), dim3(256), 0, s, (const float*)d.w, d.m, eoff, uw);
      else
        hipLaunchKernelGGL(k_union_weights<uint32_t>, dim3(bgrid(d.m)), dim3(256), 0, s, (const uint32_t*)d.w, d.m, eoff, uw);
    }
    voff += d.n;
    eoff += d.m;
  }
  b->voff.push_back(voff);
  hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, urow, N, (uint32_t)M);
  // a daic_graph over the union (borrowing urow as 32-bit offsets)
  daic_graph* ug = new daic_graph();
  ug->dev.n = N;
  ug->dev.m = M;
  ug->dev.row = urow;
  ug->dev.row32 = true;
  ug->dev.col = ucol;
  ug->part.blocks = 0;
  b->ug = ug;
  DAIC_HIP(hipStreamSynchronize(s));
  rc = pull_prepare(ug, s);
  if (rc) { daic_batch_destroy(b.release()); return rc; }
  (void)urow64;

  BArgs& a = b->a;
  a.N = N;
  a.row = urow;
  a.col = ucol;
  a.gid = gid;
  a.alpha = alpha;
  a.G = n_graphs;
  const size_t SV = N * (size_t)kR * 4;
#define BGRAB(field, type, bytes)                                   \
  do {                                                              \
    if ((rc = grab(&ptr, (bytes)))) { daic_batch_destroy(b.release()); return rc; } \
    a.field = (type)ptr;                                            \
  } while (0)
  BGRAB(ctl, BCtl*, sizeof(BCtl));
  BGRAB(v, float*, SV);
  BGRAB(dv, float*, SV);
  if (b->kahan) BGRAB(c, float*, SV);
  BGRAB(mu, float*, SV);
  BGRAB(mu2, float*, SV);
  BGRAB(active, uint8_t*, N);
  BGRAB(done, uint8_t*, (size_t)n_graphs * kR);
  BGRAB(inst_r, double*, (size_t)n_graphs * kR * 8);
  std::vector<uint32_t> rt(N + 1);
  {
    // hub items: targets with in-degree > hub_deg, chunks of kBChunk
    // in-edges, longest first
    a.hub_deg = kHubDeg;
    a.hub_chunk = kBChunk;
    if (const char* e = std::getenv("DAIC_HUB_DEG")) a.hub_deg = (uint32_t)std::max(1L, std::atol(e));
    DAIC_HIP(hipMemcpy(rt.data(), ug->pull.rowT, (N + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> ht, hc;
    {
      std::vector<std::pair<uint32_t, uint64_t>> items;  // (length, target << 32 | chunk)
      for (uint64_t t = 0; t < N; ++t) {
        const uint32_t deg = rt[t + 1] - rt[t];
        if (deg <= a.hub_deg) continue;
        for (uint32_t c = 0; c * kBChunk < deg; ++c)
          items.push_back({std::min(kBChunk, deg - c * kBChunk), (t << 32) | c});
      }
      std::stable_sort(items.begin(), items.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      for (auto& it : items) {
        ht.push_back((uint32_t)(it.second >> 32));
        hc.push_back((uint32_t)it.second);
      }
    }
    a.n_hub = ht.size();
    BGRAB(ht, const uint32_t*, ht.size() * 4);
    BGRAB(hc, const uint32_t*, hc.size() * 4);
    if (!ht.empty()) {
      DAIC_HIP(hipMemcpy((void*)a.ht, ht.data(), ht.size() * 4, hipMemcpyHostToDevice));
      DAIC_HIP(hipMemcpy((void*)a.hc, hc.data(), hc.size() * 4, hipMemcpyHostToDevice));
    }
    // push items: every vertex with out-edges, chunks of kPushChunk
    std::vector<uint32_t> ro(N + 1);
    DAIC_HIP(hipMemcpy(ro.data(), urow, (N + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> sv, sc;
    for (uint64_t j = 0; j < N; ++j) {
      uint32_t deg = ro[j + 1] - ro[j];
      for (uint32_t c = 0; c * kPushChunk < deg; ++c) {
        sv.push_back((uint32_t)j);
        sc.push_back(c);
      }
    }
    a.n_push = sv.size();
    BGRAB(sv, const uint32_t*, sv.size() * 4);
    BGRAB(sc, const uint32_t*, sc.size() * 4);
    DAIC_HIP(hipMemcpy((void*)a.sv, sv.data(), sv.size() * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.sc, sc.data(), sc.size() * 4, hipMemcpyHostToDevice));
    // residual items: vertex ranges inside each graph, closed at kResChunk
    // vertices or kItemWork work (in-edges pulled in the fused pass plus a
    // per-vertex share for the claim), whichever comes first, so that the
    // in-edge-heavy low ids of an RMAT graph do not form one long item
    std::vector<uint32_t> rg, gfi;
    std::vector<uint64_t> rlo, rhi, rw;
    for (uint32_t g = 0; g < n_graphs; ++g) {
      gfi.push_back((uint32_t)rg.size());
      uint64_t lo = b->voff[g], w = 0;
      for (uint64_t j = b->voff[g]; j < b->voff[g + 1]; ++j) {
        const uint32_t deg = rt[j + 1] - rt[j];
        w += (deg > a.hub_deg ? 0 : deg) + kVertexWork;
        if (j + 1 - lo >= kResChunk || w >= kItemWork || j + 1 == b->voff[g + 1]) {
          rg.push_back(g);
          rlo.push_back(lo);
          rhi.push_back(j + 1);
          rw.push_back(w);
          lo = j + 1;
          w = 0;
        }
      }
      if (b->voff[g] == b->voff[g + 1]) {  // empty graph: one empty item keeps the layout simple
        rg.push_back(g);
        rlo.push_back(b->voff[g]);
        rhi.push_back(b->voff[g]);
        rw.push_back(0);
      }
    }
    gfi.push_back((uint32_t)rg.size());
    a.n_res = (uint32_t)rg.size();
    // fused-pass visiting order inside each item: by pulled in-degree,
    // descending, so that the vertices a wave takes together loop about
    // equally long over their in-edges; vertices without any edge last and
    // left out of the fused pass (they neither receive nor send once their
    // initial delta is claimed, which the claim kernel of the first dense
    // or sparse round does)
    {
      std::vector<uint32_t> vord(N);
      std::vector<uint64_t> rha(rlo.size());
      for (uint64_t j = 0; j < N; ++j) vord[j] = (uint32_t)j;
      auto isolated = [&](uint32_t j) { return rt[j + 1] == rt[j] && ro[j + 1] == ro[j]; };
      auto pulled = [&](uint32_t j) { const uint32_t d = rt[j + 1] - rt[j]; return d > a.hub_deg ? 0u : d; };
      for (size_t k = 0; k < rlo.size(); ++k) {
        std::stable_sort(vord.begin() + rlo[k], vord.begin() + rhi[k], [&](uint32_t x, uint32_t y) {
          const bool ix = isolated(x), iy = isolated(y);
          if (ix != iy) return iy;
          return pulled(x) > pulled(y);
        });
        uint64_t e = rlo[k];
        while (e < rhi[k] && !isolated(vord[e])) ++e;
        rha[k] = e;
      }
      BGRAB(vord, const uint32_t*, std::max<size_t>(N, 1) * 4);
      if (N) DAIC_HIP(hipMemcpy((void*)a.vord, vord.data(), N * 4, hipMemcpyHostToDevice));
      BGRAB(rha, const uint64_t*, std::max<size_t>(rha.size(), 1) * 8);
      if (!rha.empty()) DAIC_HIP(hipMemcpy((void*)a.rha, rha.data(), rha.size() * 8, hipMemcpyHostToDevice));
    }
    BGRAB(rg, const uint32_t*, rg.size() * 4);
    BGRAB(rlo, const uint64_t*, rlo.size() * 8);
    BGRAB(rhi, const uint64_t*, rhi.size() * 8);
    BGRAB(g_first_item, const uint32_t*, gfi.size() * 4);
    DAIC_HIP(hipMemcpy((void*)a.rg, rg.data(), rg.size() * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.rlo, rlo.data(), rlo.size() * 8, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.rhi, rhi.data(), rhi.size() * 8, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.g_first_item, gfi.data(), gfi.size() * 4, hipMemcpyHostToDevice));
    BGRAB(part_r, double*, (size_t)a.n_res * kR * 8);
    BGRAB(part_p, uint64_t*, (size_t)a.n_res * 8);
    BGRAB(part_fa, uint64_t*, (size_t)a.n_res * 8);
    BGRAB(part_fm, uint64_t*, (size_t)a.n_res * 8);
    // Fused-pass block order. Workgroups go to the 8 XCDs round-robin by
    // block index and each XCD has its own L2, so every graph is given to one
    // XCD (largest graphs first, to the least loaded XCD by in-edges) and its
    // items take that XCD's block slots.
    constexpr uint32_t kXcd = 8;
    std::vector<uint64_t> gw(n_graphs, 0);
    for (uint32_t g = 0; g < n_graphs; ++g) gw[g] = rt[b->voff[g + 1]] - rt[b->voff[g]] + (b->voff[g + 1] - b->voff[g]);
    std::vector<uint32_t> gorder(n_graphs);
    for (uint32_t g = 0; g < n_graphs; ++g) gorder[g] = g;
    std::stable_sort(gorder.begin(), gorder.end(), [&](uint32_t x, uint32_t y) { return gw[x] > gw[y]; });
    std::vector<std::vector<uint32_t>> bins(kXcd);
    std::vector<uint64_t> load(kXcd, 0);
    b->xcd_of.assign(n_graphs, 0);
    for (uint32_t g : gorder) {
      const uint32_t x = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
      load[x] += gw[g];
      b->xcd_of[g] = x;
      for (uint32_t k = gfi[g]; k < gfi[g + 1]; ++k) bins[x].push_back(k);
    }
    // heaviest items first within each XCD, so that the long ones start early
    for (auto& bn : bins)
      std::stable_sort(bn.begin(), bn.end(), [&](uint32_t x, uint32_t y) { return rw[x] > rw[y]; });
    size_t longest = 0;
    for (auto& bn : bins) longest = std::max(longest, bn.size());
    std::vector<uint32_t> order(longest * kXcd, ~0u);
    for (uint32_t x = 0; x < kXcd; ++x)
      for (size_t i = 0; i < bins[x].size(); ++i) order[i * kXcd + x] = bins[x][i];
    a.n_fused_blocks = (uint32_t)order.size();
    BGRAB(item_order, const uint32_t*, order.size() * 4);
    DAIC_HIP(hipMemcpy((void*)a.item_order, order.data(), order.size() * 4, hipMemcpyHostToDevice));
  }
  BGRAB(g_ticket, uint32_t*, (size_t)n_graphs * 4);
  BGRAB(g_flag, uint32_t*, (size_t)n_graphs * 4);
  BGRAB(g_pend, uint64_t*, (size_t)n_graphs * 8);
  BGRAB(g_act, uint64_t*, (size_t)n_graphs * 8);
  BGRAB(g_msg, uint64_t*, (size_t)n_graphs * 8);
  BGRAB(part_a, uint64_t*, 8192 * 8);
  BGRAB(part_m, uint64_t*, 8192 * 8);
#undef BGRAB
  a.perm = ug->pull.perm;
  a.rowT = static_cast<const uint32_t*>(ug->pull.rowT);
  a.srcT = ug->pull.srcT;
  if (uw) {
    if ((rc = grab(&ptr, M * 4))) { daic_batch_destroy(b.release()); return rc; }
    float* uwT = (float*)ptr;
    if (M) hipLaunchKernelGGL(k_bgather_weights, dim3(bgrid(M)), dim3(256), 0, s, uw, ug->pull.eidT, M, uwT);
    a.w = uw;
    a.wT = uwT;
  }
  a.pull_min = std::max<uint64_t>(1, N / 32);
  DAIC_HIP(hipMemsetAsync(a.v, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.dv, 0, SV, s));
  if (a.c) DAIC_HIP(hipMemsetAsync(a.c, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.mu, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.mu2, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.active, 0, N, s));
  DAIC_HIP(hipMemsetAsync(a.g_ticket, 0, (size_t)n_graphs * 4, s));
  DAIC_HIP(hipMemsetAsync(a.done, 0, (size_t)n_graphs * kR, s));
  hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, 0.0, ~0ull, 1u);
  DAIC_HIP(hipHostMalloc((void**)&b->h_ctl, sizeof(BCtl), hipHostMallocDefault));
  DAIC_HIP(hipEventCreate(&b->ev0));
  DAIC_HIP(hipEventCreate(&b->ev1));
  DAIC_HIP(hipStreamSynchronize(s));
  *out = b.release();
  return DAIC_OK;
}

daic_status daic_batch_set_init(daic_batch* b, uint32_t graph, const double* v0, const double* dv1) {
  if (!b || !v0 || !dv1) return fail(DAIC_E_INVALID, "null argument");
  if (graph >= b->G) return fail(DAIC_E_INVALID, "graph index out of range");
  const uint64_t n = b->n_of[graph], off = b->voff[graph];
  const uint32_t R = b->rhs[graph];
  if (n == 0) return DAIC_OK;
  std::vector<float> tv(n * kR, 0.0f), td(n * kR, 0.0f), tc(n * kR, 0.0f);
  for (uint64_t j = 0; j < n; ++j)
    for (uint32_t r = 0; r < R; ++r) {
      const double x = v0[j * R + r];
      tv[j * kR + r] = (float)x;
      tc[j * kR + r] = (float)((double)(float)x - x);
      td[j * kR + r] = (float)dv1[j * R + r];
    }
  DAIC_HIP(hipMemcpy(b->a.v + off * kR, tv.data(), n * kR * 4, hipMemcpyHostToDevice));
  DAIC_HIP(hipMemcpy(b->a.dv + off * kR, td.data(), n * kR * 4, hipMemcpyHostToDevice));
  if (b->a.c) DAIC_HIP(hipMemcpy(b->a.c + off * kR, tc.data(), n * kR * 4, hipMemcpyHostToDevice));
  // the graph's instances start unfinished
  std::vector<uint8_t> z(kR, 0);
  DAIC_HIP(hipMemcpy(b->a.done + (size_t)graph * kR, z.data(), kR, hipMemcpyHostToDevice));
  return DAIC_OK;
}

// Autotuner: times the claim kernel (sparse rounds and the claim that opens
// the dense phase) and the dense round (hub sums and fused pass) for each
// lanes-per-vertex and grid size on the current state, which it saves and
// restores, and keeps the fastest. With DAIC_TUNE_CACHE set, choices are read
// from and appended to that file, keyed by the union graph's shape.
daic_status daic_batch_tune(daic_batch* b, char* desc, size_t desc_len) {
  if (!b) return fail(DAIC_E_INVALID, "null batch");
  hipStream_t s = b->stream;
  BArgs& a = b->a;
  char key[160];
  std::snprintf(key, sizeof key, "batch-fused N=%llu M=%llu G=%u kahan=%d weighted=%d", (unsigned long long)a.N,
                (unsigned long long)b->ug->dev.m, b->G, (int)b->kahan, a.w ? 1 : 0);
  const char* cache = std::getenv("DAIC_TUNE_CACHE");
  if (cache) {
    if (FILE* f = std::fopen(cache, "r")) {
      char line[512];
      while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key, std::strlen(key)) != 0) continue;
        BTune t;
        if (std::sscanf(line + std::strlen(key), " : %d %d %d %u %u %u", &t.lpv_claim, &t.lpv_fused, &t.lpv_push,
                        &t.grid_claim, &t.grid_hub, &t.grid_push) == 6) {
          b->tune = t;
          b->tuned = true;
        }
      }
      std::fclose(f);
    }
  }
  if (!b->tuned) {
    const size_t SV = a.N * (size_t)kR * 4;
    const size_t SD = (size_t)b->G * kR;
    float *sv = nullptr, *sd = nullptr, *sc = nullptr;
    DAIC_HIP(hipMalloc(&sv, SV));
    DAIC_HIP(hipMalloc(&sd, SV));
    if (a.c) DAIC_HIP(hipMalloc(&sc, SV));
    std::vector<uint8_t> done_save(SD);
    DAIC_HIP(hipMemcpyAsync(sv, a.v, SV, hipMemcpyDeviceToDevice, s));
    DAIC_HIP(hipMemcpyAsync(sd, a.dv, SV, hipMemcpyDeviceToDevice, s));
    if (sc) DAIC_HIP(hipMemcpyAsync(sc, a.c, SV, hipMemcpyDeviceToDevice, s));
    DAIC_HIP(hipMemcpyAsync(done_save.data(), a.done, SD, hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    // control blocks for the timed kernels: the opening claim (mode 1,
    // round 0) and a fused round (mode 2, round 1, reading the bases the
    // claim published); every instance running
    BCtl c_claim{}, c_dense{};
    c_claim.max_rounds = c_dense.max_rounds = ~0ull;
    c_claim.mode = 1;
    c_dense.mode = 2;
    c_dense.rounds = 1;
    auto restore = [&](const BCtl* c) -> hipError_t {
      hipError_t e = hipMemcpyAsync(a.v, sv, SV, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(a.dv, sd, SV, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess && sc) e = hipMemcpyAsync(a.c, sc, SV, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemsetAsync(a.done, 0, SD, s);
      if (e == hipSuccess && c) e = hipMemcpyAsync(a.ctl, c, sizeof(BCtl), hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      return e;
    };
    auto time_it = [&](const BCtl* c, auto&& enqueue) -> float {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)restore(c);
        (void)hipEventRecord(b->ev0, s);
        enqueue();
        (void)hipEventRecord(b->ev1, s);
        (void)hipEventSynchronize(b->ev1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
        if (rep > 0) best = std::min(best, ms);
      }
      return best;
    };
    const int lpvs[3] = {16, 32, 64};
    const uint32_t grids[3] = {2048, 4096, 8192};
    BTune best = b->tune;
    float best_claim = 1e30f, best_dense = 1e30f;
    for (int l : lpvs)
      for (uint32_t g : grids) {
        b->tune.lpv_claim = l;
        b->tune.grid_claim = g;
        float t = time_it(&c_claim, [&] { enqueue_claim(b, s); });
        if (t < best_claim) { best_claim = t; best.lpv_claim = l; best.grid_claim = g; }
      }
    // the dense round reads the bases published by the chosen claim
    b->tune.lpv_claim = best.lpv_claim;
    b->tune.grid_claim = best.grid_claim;
    (void)restore(&c_claim);
    enqueue_claim(b, s);
    DAIC_HIP(hipStreamSynchronize(s));
    for (int l : lpvs)
      for (uint32_t g : {1024u, 4096u}) {
        b->tune.lpv_fused = l;
        b->tune.grid_hub = g;
        float t = time_it(&c_dense, [&] { enqueue_dense(b, s, 0); });
        if (t < best_dense) { best_dense = t; best.lpv_fused = l; best.grid_hub = g; }
      }
    b->tune = best;
    DAIC_HIP(restore(nullptr));
    DAIC_HIP(hipMemcpy(a.done, done_save.data(), SD, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, 0.0, ~0ull, 1u);
    DAIC_HIP(hipStreamSynchronize(s));
    (void)hipFree(sv);
    (void)hipFree(sd);
    if (sc) (void)hipFree(sc);
    b->tuned = true;
    if (cache) {
      if (FILE* f = std::fopen(cache, "a")) {
        std::fprintf(f, "%s : %d %d %d %u %u %u\n", key, best.lpv_claim, best.lpv_fused, best.lpv_push,
                     best.grid_claim, best.grid_hub, best.grid_push);
        std::fclose(f);
      }
    }
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
  }
  if (desc && desc_len) {
    std::snprintf(desc, desc_len,
                  "claim lanes/vertex %d grid %u; dense round lanes/vertex %d hub grid %u; push lanes/vertex %d grid %u",
                  b->tune.lpv_claim, b->tune.grid_claim, b->tune.lpv_fused, b->tune.grid_hub, b->tune.lpv_push,
                  b->tune.grid_push);
  }
  return DAIC_OK;
}

daic_status daic_batch_run(daic_batch* b, const daic_run_opts* o, daic_stats* stats, double* inst_residual) {
  if (!b || !o) return fail(DAIC_E_INVALID, "null argument");
  const bool sweep = o->sched == DAIC_SCHED_SWEEP;
  if (!sweep && (o->sched != DAIC_SCHED_ALL || o->priority_fraction != 1.0))
    return fail(DAIC_E_UNSUPPORTED, "batched runs take sched ALL (q = 1) or SWEEP");
  if (sweep && !(o->priority_fraction > 0.0 && o->priority_fraction <= 1.0))
    return fail(DAIC_E_INVALID, "priority_fraction must be in (0, 1]");
  if (!(o->eps >= 0.0)) return fail(DAIC_E_INVALID, "eps must be >= 0");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : b->stream;
  // rounds_per_check 0: one launch of kBatchLaunchRounds captured rounds
  // (rounds after every instance finished return at once), so a solve of up
  // to that many rounds is a single graph launch
  constexpr uint32_t kBatchLaunchRounds = 128;
  const uint32_t K = o->rounds_per_check ? o->rounds_per_check : kBatchLaunchRounds;
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;
  if (stats) std::memset(stats, 0, sizeof *stats);
  BArgs& a = b->a;
  uint32_t P = 0;
  if (sweep) {
    // blocks per graph: ceil(1 / q), at most 1024
    P = (uint32_t)std::min(1024.0, std::ceil(1.0 / o->priority_fraction - 1e-9));
    P = std::max<uint32_t>(P, 1);
    daic_status rc = batch_sweep_setup(b, P, s);
    if (rc) return rc;
  }
  const uint32_t dense = sweep ? 3u : 1u;
  hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, o->eps, max_rounds, dense);
  hipLaunchKernelGGL(k_breset_tickets, dim3(1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_bresidual, dim3(a.n_res), dim3(256), 0, s, a, 0);
  DAIC_HIP(hipEventRecord(b->ev0, s));
  const bool use_graph = std::getenv("DAIC_NO_GRAPH") == nullptr;
  if (use_graph && !(b->exec && b->exec_K == K && b->exec_stream == s && b->exec_dense == dense &&
                     b->exec_P == P)) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (b->exec_sw) { (void)hipGraphExecDestroy(b->exec_sw); b->exec_sw = nullptr; }
    if (b->graph_sw) { (void)hipGraphDestroy(b->graph_sw); b->graph_sw = nullptr; }
    b->exec_K = 0;  // no match until both captures below have succeeded
    DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (uint32_t r = 0; r < K; ++r) enqueue_round(b, s);
    hipGraph_t graph;
    DAIC_HIP(hipStreamEndCapture(s, &graph));
    b->graph = graph;
    DAIC_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    if (sweep) {
      DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (uint32_t r = 0; r < K; ++r) enqueue_sweep(b, s);
      DAIC_HIP(hipStreamEndCapture(s, &graph));
      b->graph_sw = graph;
      DAIC_HIP(hipGraphInstantiate(&b->exec_sw, graph, nullptr, nullptr, 0));
    }
    b->exec_K = K;
    b->exec_stream = s;
    b->exec_dense = dense;
    b->exec_P = P;
  }
  uint64_t seen_rounds = ~0ull;
  DAIC_HIP(hipMemcpyAsync(b->h_ctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
  DAIC_HIP(hipStreamSynchronize(s));
  for (;;) {
    const bool sweep_now = sweep && b->h_ctl->mode == 3;
    if (use_graph) {
      DAIC_HIP(hipGraphLaunch(sweep_now ? b->exec_sw : b->exec, s));
    } else {
      for (uint32_t r = 0; r < K; ++r) {
        if (sweep_now) enqueue_sweep(b, s);
        else enqueue_round(b, s);
      }
    }
    DAIC_HIP(hipMemcpyAsync(b->h_ctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    if (b->h_ctl->done || b->h_ctl->stop) break;
    // every round advances the count; a launch of K rounds that did not
    // means the control block is inconsistent: fail instead of spinning
    if (b->h_ctl->rounds == seen_rounds)
      return fail(DAIC_E_DEVICE, "batched run made no progress (round %llu)", (unsigned long long)seen_rounds);
    seen_rounds = b->h_ctl->rounds;
  }
  if (!b->h_ctl->done && b->h_ctl->mode == 2) {
    // stopped in the dense phase: deliver the last round's messages
    enqueue_dense(b, s, 1);
    DAIC_HIP(hipMemcpyAsync(b->h_ctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
  }
  if (!b->h_ctl->done && b->h_ctl->mode == 3) {
    // stopped in the sweep phase: deliver the messages in flight, then the
    // residual of the delivered state (which may finish instances)
    if (b->h_ctl->sw_started) {
      if (a.w) launch_sweep_deliver_w<true>(b, s);
      else launch_sweep_deliver_w<false>(b, s);
    } else {
      hipLaunchKernelGGL(k_bto_sparse, dim3(1), dim3(1), 0, s, a.ctl);
      hipLaunchKernelGGL(k_bresidual, dim3(a.n_res), dim3(256), 0, s, a, 0);
    }
    DAIC_HIP(hipMemcpyAsync(b->h_ctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
  }
  DAIC_HIP(hipEventRecord(b->ev1, s));
  DAIC_HIP(hipEventSynchronize(b->ev1));
  float ms = 0.f;
  DAIC_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  const BCtl& c = *b->h_ctl;
  if (inst_residual) {
    std::vector<double> r((size_t)b->G * kR);
    DAIC_HIP(hipMemcpy(r.data(), a.inst_r, r.size() * 8, hipMemcpyDeviceToHost));
    size_t k = 0;
    for (uint32_t g = 0; g < b->G; ++g)
      for (uint32_t q = 0; q < b->rhs[g]; ++q) inst_residual[k++] = r[(size_t)g * kR + q];
  }
  if (stats) {
    stats->rounds = c.rounds;
    stats->activations = c.activations;
    stats->pushed_edges = c.messages;
    double mx = 0.0;
    std::vector<double> r((size_t)b->G * kR);
    DAIC_HIP(hipMemcpy(r.data(), a.inst_r, r.size() * 8, hipMemcpyDeviceToHost));
    for (uint32_t g = 0; g < b->G; ++g)
      for (uint32_t q = 0; q < b->rhs[g]; ++q) mx = std::max(mx, r[(size_t)g * kR + q]);
    stats->final_residual = mx;
    stats->time_ms = ms;
    stats->gteps = ms > 0 ? (double)c.messages / (ms * 1e-3) / 1e9 : 0.0;
    // Compulsory bytes of the dense rounds: per vertex the state vectors (v
    // read and written, with the Kahan term c read and written) and the
    // published base vector written, 64 floats each; per in-edge its source
    // index; per sender with out-edges its base vector read once. A sweep
    // round covers 1/P of the vertices. The sparse opening rounds are not
    // counted, so bytes / time is a lower bound of the dense rounds' rate.
    const uint64_t dense_rounds = c.rounds >= c.base ? c.rounds - c.base : 0;
    const double vec = (double)kR * 4.0;
    const double per_round = (double)a.N * (b->kahan ? 5.0 : 3.0) * vec + (double)b->ug->dev.m * 4.0 +
                             (double)b->ug->pull.n_src * vec;
    stats->alg_bytes = (double)dense_rounds * per_round / (double)(sweep ? std::max<uint32_t>(P, 1) : 1);
  }
  return c.done ? DAIC_OK : DAIC_NOT_CONVERGED;
}

daic_status daic_batch_get(const daic_batch* b, uint32_t graph, double* v_out) {
  if (!b || !v_out) return fail(DAIC_E_INVALID, "null argument");
  if (graph >= b->G) return fail(DAIC_E_INVALID, "graph index out of range");
  const uint64_t n = b->n_of[graph], off = b->voff[graph];
  const uint32_t R = b->rhs[graph];
  if (n == 0) return DAIC_OK;
  DAIC_HIP(hipDeviceSynchronize());
  std::vector<float> tv(n * kR), tc(n * kR, 0.0f);
  DAIC_HIP(hipMemcpy(tv.data(), b->a.v + off * kR, n * kR * 4, hipMemcpyDeviceToHost));
  if (b->a.c) DAIC_HIP(hipMemcpy(tc.data(), b->a.c + off * kR, n * kR * 4, hipMemcpyDeviceToHost));
  for (uint64_t j = 0; j < n; ++j)
    for (uint32_t r = 0; r < R; ++r) v_out[j * R + r] = (double)tv[j * kR + r] - (double)tc[j * kR + r];
  return DAIC_OK;
}


daic_status daic_batch_get_state(const daic_batch* b, uint32_t graph, double* v_out, double* dv_out,
                                 uint8_t* done_out) {
  if (!b) return fail(DAIC_E_INVALID, "null argument");
  if (graph >= b->G) return fail(DAIC_E_INVALID, "graph index out of range");
  const uint64_t n = b->n_of[graph], off = b->voff[graph];
  const uint32_t R = b->rhs[graph];
  DAIC_HIP(hipDeviceSynchronize());
  if (v_out && n) {
    daic_status rc = daic_batch_get(b, graph, v_out);
    if (rc) return rc;
  }
  if (dv_out && n) {
    std::vector<float> td(n * kR);
    DAIC_HIP(hipMemcpy(td.data(), b->a.dv + off * kR, n * kR * 4, hipMemcpyDeviceToHost));
    for (uint64_t j = 0; j < n; ++j)
      for (uint32_t r = 0; r < R; ++r) dv_out[j * R + r] = (double)td[j * kR + r];
  }
  if (done_out) {
    uint8_t st[kR];
    DAIC_HIP(hipMemcpy(st, b->a.done + (size_t)graph * kR, kR, hipMemcpyDeviceToHost));
    std::memcpy(done_out, st, R);
  }
  return DAIC_OK;
}

// Snapshot of a batch (every instance's v, dv, Kahan term and finish state)
// for checkpoint and resume; layout in include/daic.h.
static constexpr char kBatchMagic[8] = {'D', 'A', 'I', 'C', 'B', 'A', 'T', '1'};
static constexpr uint32_t kBatchVersion = 1;

static uint64_t batch_state_bytes(const daic_batch* b) {
  const uint64_t N = b->a.N;
  return 48 + 16 * (uint64_t)b->G + N * kR * 4 * (b->kahan ? 3 : 2) + (uint64_t)b->G * kR;
}

daic_status daic_batch_save(const daic_batch* b, void* buf, size_t* len) {
  if (!b || !len) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t need = batch_state_bytes(b);
  if (!buf) {
    *len = need;
    return DAIC_OK;
  }
  if (*len < need) {
    const size_t have = *len;
    *len = need;
    return fail(DAIC_E_INVALID, "buffer of %zu bytes, %llu needed", have, (unsigned long long)need);
  }
  uint8_t* p = static_cast<uint8_t*>(buf);
  const uint32_t ver = kBatchVersion, G = b->G, kah = b->kahan ? 1u : 0u, wgt = b->a.w ? 1u : 0u;
  const uint64_t N = b->a.N, pay = need - 48 - 16 * (uint64_t)b->G;
  std::memcpy(p, kBatchMagic, 8);
  std::memcpy(p + 8, &ver, 4);
  std::memcpy(p + 12, &G, 4);
  std::memcpy(p + 16, &N, 8);
  std::memcpy(p + 24, &kah, 4);
  std::memcpy(p + 28, &wgt, 4);
  std::memcpy(p + 32, &b->a.alpha, 8);
  std::memcpy(p + 40, &pay, 8);
  uint8_t* q = p + 48;
  for (uint32_t g = 0; g < G; ++g) {
    const uint64_t ng = b->n_of[g];
    const uint32_t r = b->rhs[g], z = 0;
    std::memcpy(q, &ng, 8);
    std::memcpy(q + 8, &r, 4);
    std::memcpy(q + 12, &z, 4);
    q += 16;
  }
  DAIC_HIP(hipDeviceSynchronize());
  const size_t V = (size_t)N * kR * 4;
  if (N) {
    DAIC_HIP(hipMemcpy(q, b->a.v, V, hipMemcpyDeviceToHost));
    DAIC_HIP(hipMemcpy(q + V, b->a.dv, V, hipMemcpyDeviceToHost));
    q += 2 * V;
    if (b->kahan) {
      DAIC_HIP(hipMemcpy(q, b->a.c, V, hipMemcpyDeviceToHost));
      q += V;
    }
  }
  DAIC_HIP(hipMemcpy(q, b->a.done, (size_t)G * kR, hipMemcpyDeviceToHost));
  *len = need;
  return DAIC_OK;
}

daic_status daic_batch_load(daic_batch* b, const void* buf, size_t len) {
  if (!b || !buf) return fail(DAIC_E_INVALID, "null argument");
  const uint8_t* p = static_cast<const uint8_t*>(buf);
  if (len < 48 || std::memcmp(p, kBatchMagic, 8) != 0) return fail(DAIC_E_INVALID, "not a saved batch state");
  uint32_t ver, G, kah, wgt;
  uint64_t N, pay;
  double alpha;
  std::memcpy(&ver, p + 8, 4);
  std::memcpy(&G, p + 12, 4);
  std::memcpy(&N, p + 16, 8);
  std::memcpy(&kah, p + 24, 4);
  std::memcpy(&wgt, p + 28, 4);
  std::memcpy(&alpha, p + 32, 8);
  std::memcpy(&pay, p + 40, 8);
  if (ver != kBatchVersion) return fail(DAIC_E_INVALID, "unsupported batch state version %u", ver);
  if (G != b->G || N != b->a.N || kah != (b->kahan ? 1u : 0u) || wgt != (b->a.w ? 1u : 0u) ||
      std::memcmp(&alpha, &b->a.alpha, 8) != 0)
    return fail(DAIC_E_INVALID, "saved state belongs to another batch (graphs, state type, weights or alpha differ)");
  if (len != batch_state_bytes(b) || pay != len - 48 - 16 * (uint64_t)G)
    return fail(DAIC_E_INVALID, "batch state buffer has the wrong size");
  const uint8_t* q = p + 48;
  for (uint32_t g = 0; g < G; ++g) {
    uint64_t ng;
    uint32_t r;
    std::memcpy(&ng, q, 8);
    std::memcpy(&r, q + 8, 4);
    if (ng != b->n_of[g] || r != b->rhs[g]) return fail(DAIC_E_INVALID, "graph %u differs from the saved batch", g);
    q += 16;
  }
  DAIC_HIP(hipDeviceSynchronize());
  const size_t V = (size_t)N * kR * 4;
  if (N) {
    DAIC_HIP(hipMemcpy(b->a.v, q, V, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy(b->a.dv, q + V, V, hipMemcpyHostToDevice));
    q += 2 * V;
    if (b->kahan) {
      DAIC_HIP(hipMemcpy(b->a.c, q, V, hipMemcpyHostToDevice));
      q += V;
    }
  }
  DAIC_HIP(hipMemcpy(b->a.done, q, (size_t)G * kR, hipMemcpyHostToDevice));
  return DAIC_OK;
}

}  // extern "C"
