// Batched DAIC: many graphs of uneven size, each with many right-hand sides,
// solved together (personalized PageRank: the Rooted PageRank row of Table 1
// read with damping, g_{j,k}(x) = d x / outdeg_j, Delta v^1 = (1-d) p).
//
// The graphs are joined into one block-diagonal graph; the state is
// [vertex][64 right-hand sides] in FP32, so one message is a contiguous
// 256-byte vector. A round is three kernels over every graph at once (claim,
// propagate, residual); propagation pulls over in-edges when dense and pushes
// with atomics when sparse. Every instance (graph, right-hand side) has its
// own residual and stop flag. Lanes per vertex and grid sizes come from an
// autotuner that times the dense-round kernels on the device.
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
constexpr uint32_t kResChunk = 8192;   // vertices per residual item

struct BCtl {
  uint32_t done;          // every instance finished
  uint32_t stop;          // round limit reached
  uint32_t pull;          // next round is dense
  uint32_t ticket;
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
  float* mu;                  // [N][64]: renumbered (dense) or by vertex (sparse)
  uint8_t* active;            // [N] vertex sent this round (sparse rounds)
  uint8_t* done;              // [G][64] instance finished
  double alpha;
  // dense rounds
  const uint32_t* perm;
  const uint32_t* rowT;
  const uint32_t* srcT;
  const uint32_t* pt;         // pull items (target, chunk, nchunks)
  const uint32_t* pc;
  const uint32_t* pn;
  uint64_t n_pull;
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
  double* inst_r;             // [G][64] residual per instance
  uint64_t pull_min;          // dense round when union pending >= pull_min
};

__device__ __forceinline__ bool bhalted(const BCtl* c) { return (c->done | c->stop) != 0; }

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
  if (bhalted(ctl)) return;
  const bool pull = ctl->pull != 0;
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  uint64_t act = 0, msg = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * VPB; base < a.N; base += (uint64_t)gridDim.x * VPB) {
    const uint64_t j = base + sub;
    if (j >= a.N) continue;
    const uint32_t g = a.gid[j];
    const uint32_t deg = a.row[j + 1] - a.row[j];
    const double coef = deg ? a.alpha / (double)deg : 0.0;
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
      vstore<W>(a.mu + (uint64_t)a.perm[j] * kR + r0, mu);
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

// Dense round: every target adds the message bases of its in-neighbours.
template <int LPV>
__global__ __launch_bounds__(256) void k_bpull(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int IPB = 256 / LPV;  // items per block at a time
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || !ctl->pull) return;
  const uint32_t sub = threadIdx.x / LPV;
  const uint32_t r0 = (threadIdx.x % LPV) * W;
  for (uint64_t base = (uint64_t)blockIdx.x * IPB; base < a.n_pull; base += (uint64_t)gridDim.x * IPB) {
    const uint64_t i = base + sub;
    if (i >= a.n_pull) continue;
    const uint32_t t = a.pt[i], ch = a.pc[i], nch = a.pn[i];
    const uint32_t beg = a.rowT[t] + ch * kBChunk;
    const uint32_t end = min(a.rowT[t + 1], beg + kBChunk);
    float acc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] = 0.0f;
    uint32_t p = beg;
    for (; p + 3 < end; p += 4) {
      const uint32_t s0 = a.srcT[p], s1 = a.srcT[p + 1], s2 = a.srcT[p + 2], s3 = a.srcT[p + 3];
      float x0[W], x1[W], x2[W], x3[W];
      vload<W>(a.mu + (uint64_t)s0 * kR + r0, x0);
      vload<W>(a.mu + (uint64_t)s1 * kR + r0, x1);
      vload<W>(a.mu + (uint64_t)s2 * kR + r0, x2);
      vload<W>(a.mu + (uint64_t)s3 * kR + r0, x3);
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += (x0[k] + x1[k]) + (x2[k] + x3[k]);
    }
    for (; p < end; ++p) {
      float x[W];
      vload<W>(a.mu + (uint64_t)a.srcT[p] * kR + r0, x);
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += x[k];
    }
    float* dst = a.dv + (uint64_t)t * kR + r0;
    if (nch == 1) {
      float d[W];
      vload<W>(dst, d);
#pragma unroll
      for (int k = 0; k < W; ++k) d[k] += acc[k];
      vstore<W>(dst, d);
    } else {
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (acc[k] != 0.0f) unsafeAtomicAdd(dst + k, acc[k]);
    }
  }
}

// Sparse round: active vertices push their 64-wide message to every out-edge.
template <int LPV>
__global__ __launch_bounds__(256) void k_bpush(BArgs a) {
  constexpr int W = kR / LPV;
  constexpr int IPB = 256 / LPV;
  BCtl* ctl = a.ctl;
  if (bhalted(ctl) || ctl->pull) return;
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
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (mu[k] != 0.0f) unsafeAtomicAdd(dst + k, mu[k]);
    }
  }
}

// Residual per instance (FP64 sums of |dv| per graph and right-hand side),
// union pending count, stop flags and the direction of the next round. One
// block per residual item; the last block reduces in a fixed order.
__global__ __launch_bounds__(256) void k_bresidual(BArgs a, int count_round) {
  BCtl* ctl = a.ctl;
  if (bhalted(ctl)) return;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  __shared__ double s_r[4][kR];
  __shared__ uint32_t s_last;
  double r = 0.0;
  uint64_t pend = 0;
  const uint32_t it = blockIdx.x;
  for (uint64_t j = a.rlo[it] + wave; j < a.rhi[it]; j += 4) {
    float x = a.dv[j * kR + lane];
    r += fabs((double)x);
    pend += __ballot(x != 0.0f) != 0 ? 1 : 0;
  }
  s_r[wave][lane] = r;
  pend = (lane == 0) ? pend : 0;
  pend = block_sum256(pend);
  __syncthreads();
  if (threadIdx.x < kR)
    a.part_r[(uint64_t)it * kR + threadIdx.x] =
        s_r[0][threadIdx.x] + s_r[1][threadIdx.x] + s_r[2][threadIdx.x] + s_r[3][threadIdx.x];
  if (threadIdx.x == 0) {
    a.part_p[it] = pend;
    __threadfence();
    s_last = atomicAdd(&ctl->ticket, 1u) == a.n_res - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // per instance: sum the items of its graph in order
  uint32_t all_done = 1;
  for (uint32_t q = threadIdx.x; q < a.G * kR; q += 256) {
    const uint32_t g = q / kR, rr = q % kR;
    double s = 0.0;
    for (uint32_t k = a.g_first_item[g]; k < a.g_first_item[g + 1]; ++k)
      s += __hip_atomic_load(&a.part_r[(uint64_t)k * kR + rr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.inst_r[q] = s;
    if (!a.done[q] && s <= ctl->eps) a.done[q] = 1;
    all_done &= a.done[q];
  }
  uint64_t pp = 0;
  for (uint32_t k = threadIdx.x; k < a.n_res; k += 256)
    pp += __hip_atomic_load(&a.part_p[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  pp = block_sum256(pp);
  all_done = block_sum256(all_done);
  if (threadIdx.x == 0) {
    ctl->rounds += (uint64_t)count_round;
    ctl->pending = pp;
    const bool done = all_done == 256;
    ctl->done = done ? 1u : 0u;
    ctl->stop = (!done && ctl->rounds >= ctl->max_rounds) ? 1u : 0u;
    ctl->pull = pp >= a.pull_min ? 1u : 0u;
    ctl->ticket = 0;
  }
}

__global__ void k_bstats(BArgs a, uint32_t nblocks) {
  if (bhalted(a.ctl)) return;
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

__global__ void k_binit(BCtl* ctl, double eps, uint64_t max_rounds) {
  ctl->done = 0;
  ctl->stop = 0;
  ctl->pull = 0;
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

static uint32_t bgrid(uint64_t count, uint32_t block = 256) {
  uint64_t g = (count + block - 1) / block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 8192));
}

}  // namespace daic

using namespace daic;

struct BTune {
  int lpv_claim = 16, lpv_pull = 16, lpv_push = 16;
  uint32_t grid_claim = 4096, grid_pull = 8192, grid_push = 8192;
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
  BTune tune;
  bool tuned = false;
  std::vector<void*> allocs;
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

static void enqueue_pull(daic_batch* b, hipStream_t s) {
  const int l = b->tune.lpv_pull;
  const uint32_t g = b->tune.grid_pull;
  if (l == 16) hipLaunchKernelGGL(k_bpull<16>, dim3(g), dim3(256), 0, s, b->a);
  else if (l == 32) hipLaunchKernelGGL(k_bpull<32>, dim3(g), dim3(256), 0, s, b->a);
  else hipLaunchKernelGGL(k_bpull<64>, dim3(g), dim3(256), 0, s, b->a);
}

static void enqueue_push(daic_batch* b, hipStream_t s) {
  const int l = b->tune.lpv_push;
  const uint32_t g = b->tune.grid_push;
  if (l == 16) hipLaunchKernelGGL(k_bpush<16>, dim3(g), dim3(256), 0, s, b->a);
  else hipLaunchKernelGGL(k_bpush<64>, dim3(g), dim3(256), 0, s, b->a);
}

static void enqueue_round(daic_batch* b, hipStream_t s) {
  enqueue_claim(b, s);
  enqueue_pull(b, s);
  enqueue_push(b, s);
  hipLaunchKernelGGL(k_bresidual, dim3(b->a.n_res), dim3(256), 0, s, b->a, 1);
}

}  // namespace daic

extern "C" {

void daic_batch_destroy(daic_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* q : b->allocs)
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
  if (op != DAIC_SUM || gk != DAIC_G_DEG_SCALE)
    return fail(DAIC_E_UNSUPPORTED, "batched runs take SUM with DEG_SCALE (personalized PageRank)");
  if (state != DAIC_F32 && state != DAIC_F32_KAHAN)
    return fail(DAIC_E_UNSUPPORTED, "batched runs take F32 or F32_KAHAN state");
  if (!std::isfinite(alpha)) return fail(DAIC_E_INVALID, "alpha must be finite");
  uint64_t N = 0, M = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    if (!graphs[g]) return fail(DAIC_E_INVALID, "graph %u is null", g);
    if (rhs_per_graph[g] == 0 || rhs_per_graph[g] > (uint32_t)kR)
      return fail(DAIC_E_INVALID, "right-hand sides per graph must be in 1..%d", kR);
    if (!graphs[g]->dev.row32) return fail(DAIC_E_UNSUPPORTED, "graph %u has m >= 2^32", g);
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
  uint64_t voff = 0, eoff = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    const GraphDev& d = graphs[g]->dev;
    b->voff.push_back(voff);
    b->n_of.push_back(d.n);
    if (d.n) hipLaunchKernelGGL(k_union_rows, dim3(bgrid(d.n)), dim3(256), 0, s, static_cast<const uint32_t*>(d.row),
                                d.n, voff, eoff, g, urow, gid);
    if (d.m) hipLaunchKernelGGL(k_union_cols, dim3(bgrid(d.m)), dim3(256), 0, s, d.col, d.m, voff, eoff, ucol);
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
  BGRAB(active, uint8_t*, N);
  BGRAB(done, uint8_t*, (size_t)n_graphs * kR);
  BGRAB(inst_r, double*, (size_t)n_graphs * kR * 8);
  // pull items: every target with in-edges, chunks of kBChunk, ordered by
  // in-degree class so that the targets of a block loop about equally
  {
    std::vector<uint32_t> rt(N + 1);
    DAIC_HIP(hipMemcpy(rt.data(), ug->pull.rowT, (N + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<std::vector<uint32_t>> cls(12);
    for (uint64_t t = 0; t < N; ++t) {
      uint32_t deg = rt[t + 1] - rt[t];
      if (!deg) continue;
      uint32_t c = 0;
      while (c < 11 && (1u << c) < deg) ++c;
      cls[c].push_back((uint32_t)t);
    }
    std::vector<uint32_t> pt, pc, pn;
    for (auto& cl : cls)
      for (uint32_t t : cl) {
        uint32_t deg = rt[t + 1] - rt[t];
        uint32_t nch = (deg + kBChunk - 1) / kBChunk;
        for (uint32_t c = 0; c < nch; ++c) {
          pt.push_back(t);
          pc.push_back(c);
          pn.push_back(nch);
        }
      }
    a.n_pull = pt.size();
    BGRAB(pt, const uint32_t*, pt.size() * 4);
    BGRAB(pc, const uint32_t*, pc.size() * 4);
    BGRAB(pn, const uint32_t*, pn.size() * 4);
    DAIC_HIP(hipMemcpy((void*)a.pt, pt.data(), pt.size() * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.pc, pc.data(), pc.size() * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy((void*)a.pn, pn.data(), pn.size() * 4, hipMemcpyHostToDevice));
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
    // residual items: chunks of kResChunk vertices inside each graph
    std::vector<uint32_t> rg, gfi;
    std::vector<uint64_t> rlo, rhi;
    for (uint32_t g = 0; g < n_graphs; ++g) {
      gfi.push_back((uint32_t)rg.size());
      for (uint64_t lo = b->voff[g]; lo < b->voff[g + 1]; lo += kResChunk) {
        rg.push_back(g);
        rlo.push_back(lo);
        rhi.push_back(std::min<uint64_t>(b->voff[g + 1], lo + kResChunk));
      }
      if (b->voff[g] == b->voff[g + 1]) {  // empty graph: one empty item keeps the layout simple
        rg.push_back(g);
        rlo.push_back(b->voff[g]);
        rhi.push_back(b->voff[g]);
      }
    }
    gfi.push_back((uint32_t)rg.size());
    a.n_res = (uint32_t)rg.size();
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
  }
  BGRAB(part_a, uint64_t*, 8192 * 8);
  BGRAB(part_m, uint64_t*, 8192 * 8);
#undef BGRAB
  a.perm = ug->pull.perm;
  a.rowT = static_cast<const uint32_t*>(ug->pull.rowT);
  a.srcT = ug->pull.srcT;
  a.pull_min = std::max<uint64_t>(1, N / 32);
  DAIC_HIP(hipMemsetAsync(a.v, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.dv, 0, SV, s));
  if (a.c) DAIC_HIP(hipMemsetAsync(a.c, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.mu, 0, SV, s));
  DAIC_HIP(hipMemsetAsync(a.active, 0, N, s));
  DAIC_HIP(hipMemsetAsync(a.done, 0, (size_t)n_graphs * kR, s));
  hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, 0.0, ~0ull);
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

// Autotuner: times the dense-round kernels (claim and pull) for each lanes-per-
// vertex and grid size on the current state, which it saves and restores, and
// keeps the fastest. With DAIC_TUNE_CACHE set, choices are read from and
// appended to that file, keyed by the union graph's shape.
daic_status daic_batch_tune(daic_batch* b, char* desc, size_t desc_len) {
  if (!b) return fail(DAIC_E_INVALID, "null batch");
  hipStream_t s = b->stream;
  BArgs& a = b->a;
  char key[160];
  std::snprintf(key, sizeof key, "batch N=%llu M=%llu G=%u kahan=%d", (unsigned long long)a.N,
                (unsigned long long)b->ug->dev.m, b->G, (int)b->kahan);
  const char* cache = std::getenv("DAIC_TUNE_CACHE");
  if (cache) {
    if (FILE* f = std::fopen(cache, "r")) {
      char line[512];
      while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key, std::strlen(key)) != 0) continue;
        BTune t;
        if (std::sscanf(line + std::strlen(key), " : %d %d %d %u %u %u", &t.lpv_claim, &t.lpv_pull, &t.lpv_push,
                        &t.grid_claim, &t.grid_pull, &t.grid_push) == 6) {
          b->tune = t;
          b->tuned = true;
        }
      }
      std::fclose(f);
    }
  }
  if (!b->tuned) {
    const size_t SV = a.N * (size_t)kR * 4;
    float *sv = nullptr, *sd = nullptr, *sc = nullptr;
    DAIC_HIP(hipMalloc(&sv, SV));
    DAIC_HIP(hipMalloc(&sd, SV));
    if (a.c) DAIC_HIP(hipMalloc(&sc, SV));
    DAIC_HIP(hipMemcpyAsync(sv, a.v, SV, hipMemcpyDeviceToDevice, s));
    DAIC_HIP(hipMemcpyAsync(sd, a.dv, SV, hipMemcpyDeviceToDevice, s));
    if (sc) DAIC_HIP(hipMemcpyAsync(sc, a.c, SV, hipMemcpyDeviceToDevice, s));
    auto restore = [&]() -> hipError_t {
      hipError_t e = hipMemcpyAsync(a.v, sv, SV, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(a.dv, sd, SV, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess && sc) e = hipMemcpyAsync(a.c, sc, SV, hipMemcpyDeviceToDevice, s);
      return e;
    };
    auto time_it = [&](auto&& enqueue) -> float {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)restore();
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
    // the tuning rounds run as dense rounds on unfinished instances
    hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, 0.0, ~0ull);
    BCtl hc{};
    hc.max_rounds = ~0ull;
    hc.pull = 1;
    DAIC_HIP(hipMemcpyAsync(a.ctl, &hc, sizeof hc, hipMemcpyHostToDevice, s));
    std::vector<uint8_t> done_save((size_t)b->G * kR);
    DAIC_HIP(hipMemcpyAsync(done_save.data(), a.done, done_save.size(), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    DAIC_HIP(hipMemsetAsync(a.done, 0, done_save.size(), s));
    const int lpvs[3] = {16, 32, 64};
    const uint32_t grids[3] = {2048, 4096, 8192};
    BTune best = b->tune;
    float best_claim = 1e30f, best_pull = 1e30f;
    for (int l : lpvs)
      for (uint32_t g : grids) {
        b->tune.lpv_claim = l;
        b->tune.grid_claim = g;
        float t = time_it([&] { enqueue_claim(b, s); });
        if (t < best_claim) { best_claim = t; best.lpv_claim = l; best.grid_claim = g; }
      }
    b->tune.lpv_claim = best.lpv_claim;
    b->tune.grid_claim = best.grid_claim;
    for (int l : lpvs)
      for (uint32_t g : grids) {
        b->tune.lpv_pull = l;
        b->tune.grid_pull = g;
        float t = time_it([&] { enqueue_pull(b, s); });
        if (t < best_pull) { best_pull = t; best.lpv_pull = l; best.grid_pull = g; }
      }
    b->tune = best;
    DAIC_HIP(restore());
    DAIC_HIP(hipMemcpyAsync(a.done, done_save.data(), done_save.size(), hipMemcpyHostToDevice, s));
    DAIC_HIP(hipStreamSynchronize(s));
    (void)hipFree(sv);
    (void)hipFree(sd);
    if (sc) (void)hipFree(sc);
    b->tuned = true;
    if (cache) {
      if (FILE* f = std::fopen(cache, "a")) {
        std::fprintf(f, "%s : %d %d %d %u %u %u\n", key, best.lpv_claim, best.lpv_pull, best.lpv_push,
                     best.grid_claim, best.grid_pull, best.grid_push);
        std::fclose(f);
      }
    }
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
  }
  if (desc && desc_len) {
    std::snprintf(desc, desc_len, "claim lanes/vertex %d grid %u; pull lanes/vertex %d grid %u; push lanes/vertex %d grid %u",
                  b->tune.lpv_claim, b->tune.grid_claim, b->tune.lpv_pull, b->tune.grid_pull, b->tune.lpv_push,
                  b->tune.grid_push);
  }
  return DAIC_OK;
}

daic_status daic_batch_run(daic_batch* b, const daic_run_opts* o, daic_stats* stats, double* inst_residual) {
  if (!b || !o) return fail(DAIC_E_INVALID, "null argument");
  if (o->sched != DAIC_SCHED_ALL || o->priority_fraction != 1.0)
    return fail(DAIC_E_UNSUPPORTED, "batched runs update every pending vertex (sched ALL, q = 1)");
  if (!(o->eps >= 0.0)) return fail(DAIC_E_INVALID, "eps must be >= 0");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : b->stream;
  const uint32_t K = o->rounds_per_check ? o->rounds_per_check : 1;
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;
  if (stats) std::memset(stats, 0, sizeof *stats);
  BArgs& a = b->a;
  hipLaunchKernelGGL(k_binit, dim3(1), dim3(1), 0, s, a.ctl, o->eps, max_rounds);
  hipLaunchKernelGGL(k_bresidual, dim3(a.n_res), dim3(256), 0, s, a, 0);
  DAIC_HIP(hipEventRecord(b->ev0, s));
  const bool use_graph = std::getenv("DAIC_NO_GRAPH") == nullptr;
  if (use_graph && !(b->exec && b->exec_K == K && b->exec_stream == s)) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (uint32_t r = 0; r < K; ++r) enqueue_round(b, s);
    hipGraph_t graph;
    DAIC_HIP(hipStreamEndCapture(s, &graph));
    b->graph = graph;
    DAIC_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    b->exec_K = K;
    b->exec_stream = s;
  }
  for (;;) {
    if (use_graph) {
      DAIC_HIP(hipGraphLaunch(b->exec, s));
    } else {
      for (uint32_t r = 0; r < K; ++r) enqueue_round(b, s);
    }
    DAIC_HIP(hipMemcpyAsync(b->h_ctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    if (b->h_ctl->done || b->h_ctl->stop) break;
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
    stats->alg_bytes = 0.0;
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

}  // extern "C"
