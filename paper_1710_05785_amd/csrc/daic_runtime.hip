// Host runtime and C ABI of libdaic: graphs, problems, the round loop
// (hipGraph-captured), selection, and state transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "daic_internal.h"
#include "daic_kernels.h"
#include "daic_problem.h"

namespace daic {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

daic_status fail(daic_status s, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

static size_t state_size(int st) {
  switch (st) {
    case ST_F64:
    case ST_F64MIN: return 8;
    case ST_F32:
    case ST_F32K: return 4;
    default: return 4;
  }
}

static Partition make_partition(uint64_t n) {
  Partition p;
  if (n == 0) return p;
  uint64_t blocks = std::min<uint64_t>(kMaxScanBlocks, (n + kScanBlock - 1) / kScanBlock);
  uint64_t per = (n + blocks - 1) / blocks;
  per = (per + kScanBlock - 1) / kScanBlock * kScanBlock;
  p.per_block = per;
  p.blocks = (uint32_t)((n + per - 1) / per);
  return p;
}

// The first index i < count with bad(i) (count when none), the range split
// over the host's threads (the checks of a large host CSR take a fraction of
// a second on one core).
template <typename Bad>
static uint64_t first_index_where(uint64_t count, const Bad& bad) {
  const uint64_t nt = count < (1u << 20) ? 1 : std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<uint64_t> first(nt, count);
  auto scan = [&](uint64_t t) {
    const uint64_t lo = count * t / nt, hi = count * (t + 1) / nt;
    for (uint64_t i = lo; i < hi; ++i)
      if (bad(i)) {
        first[t] = i;
        return;
      }
  };
  std::vector<std::thread> pool;
  for (uint64_t t = 1; t < nt; ++t) pool.emplace_back(scan, t);
  scan(0);
  for (auto& th : pool) th.join();
  return *std::min_element(first.begin(), first.end());
}

template <typename T>
static daic_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(DAIC_E_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
  }
  return DAIC_OK;
}

static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

}  // namespace daic

using namespace daic;

namespace daic {

static uint32_t push_grid() { return 256 * 16; }

// Per-vertex arrays through the numbering of targets by in-degree octave:
// dst[r] = src[tinv[r]] (gather) or dst[tinv[r]] = src[r] (scatter).
template <typename T, bool GATHER>
__global__ void k_perm_copy(const T* __restrict__ src, const uint32_t* __restrict__ tinv, uint64_t n,
                            T* __restrict__ dst) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
    if constexpr (GATHER) dst[r] = src[tinv[r]];
    else dst[tinv[r]] = src[r];
  }
}

template <bool GATHER>
static void perm_copy(const void* src, void* dst, size_t elem, const uint32_t* tinv, uint64_t n, hipStream_t s) {
  const dim3 grid((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 8192)));
  if (elem == 8)
    hipLaunchKernelGGL((k_perm_copy<uint64_t, GATHER>), grid, dim3(256), 0, s, static_cast<const uint64_t*>(src),
                       tinv, n, static_cast<uint64_t*>(dst));
  else
    hipLaunchKernelGGL((k_perm_copy<uint32_t, GATHER>), grid, dim3(256), 0, s, static_cast<const uint32_t*>(src),
                       tinv, n, static_cast<uint32_t*>(dst));
}

void perm_gather(const void* src, void* dst, size_t elem, const uint32_t* tinv, uint64_t n, hipStream_t s) {
  perm_copy<true>(src, dst, elem, tinv, n, s);
}
void perm_scatter(const void* src, void* dst, size_t elem, const uint32_t* tinv, uint64_t n, hipStream_t s) {
  perm_copy<false>(src, dst, elem, tinv, n, s);
}

// Fused rounds over the ranked tiles keep v, dv and c in target-number order:
// they move there after the priming claim and back when the run ends.
static void ranked_enter(daic_problem* p, hipStream_t s) {
  const uint64_t n = p->g->dev.n;
  const uint32_t* tinv = p->g->tile_r.tinv;
  const size_t S = state_size(p->st);
  perm_copy<true>(p->a.v, p->vP, S, tinv, n, s);
  perm_copy<true>(p->a.dv, p->dvP, S, tinv, n, s);
  if (p->a.c) perm_copy<true>(p->a.c, p->cP, 4, tinv, n, s);
  if (p->a.alpha_pv) perm_copy<true>(p->a.alpha_pv, p->alphaP, S, tinv, n, s);
  p->ranked_active = true;
}

static bool ranked_on(const daic_problem* p) {
  return p->ranked_ready && p->tile_ready && (!p->a.alpha_pv || p->alphaP);
}

static void ranked_leave(daic_problem* p, hipStream_t s) {
  if (!p->ranked_active) return;
  const uint64_t n = p->g->dev.n;
  const uint32_t* tinv = p->g->tile_r.tinv;
  const size_t S = state_size(p->st);
  perm_copy<false>(p->vP, p->a.v, S, tinv, n, s);
  perm_copy<false>(p->dvP, p->a.dv, S, tinv, n, s);
  if (p->a.c) perm_copy<false>(p->cP, p->a.c, 4, tinv, n, s);
  p->ranked_active = false;
}

template <int ST, int G, typename RowT>
struct Impl {
  using Key = typename Tr<ST>::Key;

  static void residual(daic_problem* p, hipStream_t s, int count_round) {
    hipLaunchKernelGGL(k_residual<ST>, dim3(p->a.blocks), dim3(256), 0, s, p->a, 0);
    hipLaunchKernelGGL(k_residual_final<ST>, dim3(1), dim3(256), 0, s, p->a, count_round, p->k_sel, p->pull_min, 0);
  }

  // Threshold of a round (A2) for the given rule.
  static void threshold(daic_problem* p, const daic_run_opts* o, hipStream_t s, const KArgs& a,
                        uint64_t round_override, Prof* pr) {
    const uint64_t n = p->a.n;
    if (o->sched == DAIC_SCHED_ALL) {
      launch(pr, "select_all", s, [&] { hipLaunchKernelGGL(k_select_all, dim3(1), dim3(1), 0, s, a.ctl); });
    } else if (o->sched == DAIC_SCHED_ROUND_ROBIN) {
      const uint64_t nb = (n + a.rr_chunk - 1) / a.rr_chunk;
      launch(pr, "select_rr", s, [&] { hipLaunchKernelGGL(k_select_rr, dim3(1), dim3(1), 0, s, a.ctl, nb); });
    } else if (o->sched == DAIC_SCHED_TOPK_SAMPLED) {
      uint32_t S = o->n_samples ? o->n_samples : kMaxSamples;
      uint32_t rank = (uint32_t)std::max(1.0, std::ceil(o->priority_fraction * (double)S));
      launch(pr, "sample_threshold", s, [&] {
        hipLaunchKernelGGL(k_sample_keys<ST>, dim3((S + 255) / 256), dim3(256), 0, s, a, S, o->seed, round_override);
        hipLaunchKernelGGL(k_sample<ST>, dim3((S + 63) / 64), dim3(256), 0, s, a, S, rank);
      });
    } else {  // exact top-k (also the learned rule, on the learned keys)
      uint64_t k = (uint64_t)std::ceil(o->priority_fraction * (double)n);
      if (k < 1) k = 1;
      const int passes = radix_passes<Key>();
      uint32_t hgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (n + 1023) / 1024));
      launch(pr, "topk_radix", s, [&] {
        hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, a.ctl, a.rhist, k);
        for (int pass = 0; pass < passes; ++pass) {
          hipLaunchKernelGGL(k_radix_pass<ST>, dim3(hgrid), dim3(256), 0, s, a, pass);
          hipLaunchKernelGGL(k_radix_pick<ST>, dim3(1), dim3(256), 0, s, a, pass);
        }
        hipLaunchKernelGGL(k_tie_count<ST>, dim3(a.blocks), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_tie_scan, dim3(1), dim3(1024), 0, s, a);
      });
    }
  }

  static void round(daic_problem* p, const daic_run_opts* o, hipStream_t s, const float* score, Prof* pr) {
    KArgs a = p->a;
    a.score = score;
    // every pending vertex: the control block keeps mode 0 from the run's
    // start, so the rounds need no threshold kernel
    if (o->sched != DAIC_SCHED_ALL) threshold(p, o, s, a, ~0ull, pr);
    launch(pr, "claim", s, [&] {
      hipLaunchKernelGGL((k_claim<ST, G, RowT, false>), dim3(a.blocks), dim3(256), 0, s, a);
    });
    launch(pr, "bin_scan", s, [&] { hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, a); });
    launch(pr, "push_edges", s, [&] {
      hipLaunchKernelGGL((k_push<ST, G, RowT>), dim3(2 * push_grid()), dim3(64), 0, s, a, push_grid());
    });
    if (p->pull_ready && p->tile_ready && !Tr<ST>::sum) {  // dense rounds of min and max problems
      const TileArgs t = tile_args(p);
      const uint32_t np = tile_pull_grid(p), nfin = tile_finish_grid(p);
      launch(pr, "pull_tile", s, [&] {
        if (t.tw > kNarrowTW) hipLaunchKernelGGL((k_tile_pull_mm<ST, G, 1024>), dim3(np), dim3(1024), 0, s, a, t);
        else hipLaunchKernelGGL((k_tile_pull_mm<ST, G, 256>), dim3(np), dim3(256), 0, s, a, t);
      });
      launch(pr, "pull_tile_finish", s, [&] {
        hipLaunchKernelGGL((k_tile_finish_mm<ST, G>), dim3(nfin), dim3(256), 0, s, a, t);
      });
      launch(pr, "pull_tile_total", s, [&] {
        hipLaunchKernelGGL((k_tile_total<ST, false>), dim3(1), dim3(256), 0, s, a, t, np, nfin, p->k_sel, p->pull_min);
      });
    } else if (p->pull_ready && p->tile_ready) {  // dense rounds through the tiled in-edges
      const TileArgs t = tile_args(p);
      const uint32_t np = tile_pull_grid(p), nfin = tile_finish_grid(p);
      launch(pr, "pull_tile", s, [&] {
        if (t.tw > kNarrowTW) hipLaunchKernelGGL((k_tile_pull<ST, G, false, 1024>), dim3(np), dim3(1024), 0, s, a, t);
        else hipLaunchKernelGGL((k_tile_pull<ST, G, false, 256>), dim3(np), dim3(256), 0, s, a, t);
      });
      launch(pr, "pull_tile_finish", s, [&] {
        hipLaunchKernelGGL((k_tile_finish<ST, G, false>), dim3(nfin), dim3(256), 0, s, a, t);
      });
      launch(pr, "pull_tile_total", s, [&] {
        hipLaunchKernelGGL((k_tile_total<ST, false>), dim3(1), dim3(256), 0, s, a, t, np, nfin, p->k_sel, p->pull_min);
      });
    } else if (p->pull_ready) {
      const uint32_t nf = fused_grid(p);
      launch(pr, "pull_stream", s, [&] {
        hipLaunchKernelGGL((k_pull_stream<ST, G>), dim3(nf), dim3(256), 0, s, a);
      });
      launch(pr, "pull_finish", s, [&] {
        hipLaunchKernelGGL(k_pull_finish<ST>, dim3(finish_grid(p)), dim3(256), 0, s, a, nf, p->k_sel, p->pull_min);
      });
    }
    launch(pr, "residual", s, [&] {
      const int skip = p->pull_ready ? 1 : 0;
      hipLaunchKernelGGL(k_residual<ST>, dim3(a.blocks), dim3(256), 0, s, a, skip);
      hipLaunchKernelGGL(k_residual_final<ST>, dim3(1), dim3(256), 0, s, a, 1, p->k_sel, p->pull_min, skip);
    });
  }

  static void select(daic_problem* p, const daic_run_opts* o, hipStream_t s, uint64_t round_override) {
    KArgs a = p->a;
    threshold(p, o, s, a, round_override, nullptr);
    hipLaunchKernelGGL((k_claim<ST, G, RowT, true>), dim3(a.blocks), dim3(256), 0, s, a);
  }

  static uint32_t fused_grid(const daic_problem* p) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(p->a.sb_count, p->stream_grid));
  }
  // one thread per cut target and at least one per partial of k_pull_fused
  static uint32_t finish_grid(const daic_problem* p) {
    return (uint32_t)std::max<uint64_t>((p->a.n_groups + 255) / 256, (fused_grid(p) + 255) / 256);
  }

  static void fuse_prime(daic_problem* p, const daic_run_opts* o, hipStream_t s, Prof* pr) {
    if constexpr (Tr<ST>::sum) {
      KArgs a = p->a;
      threshold(p, o, s, a, ~0ull, pr);
      launch(pr, "claim", s, [&] {
        hipLaunchKernelGGL((k_claim<ST, G, RowT, false>), dim3(a.blocks), dim3(256), 0, s, a);
      });
      launch(pr, "bin_scan", s, [&] { hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, a); });
      hipLaunchKernelGGL(k_fuse_begin, dim3(1), dim3(1), 0, s, a.ctl);
      if (ranked_on(p)) ranked_enter(p, s);
    }
  }

  // ranked: the layout of fused rounds with targets numbered by in-degree octave
  static TileArgs tile_args(const daic_problem* p, bool ranked = false) {
    const TileGraph& T = ranked ? p->g->tile_r : p->g->tile;
    TileArgs t{};
    t.tloc = T.tloc;
    t.psrc = T.psrc;
    t.segpair = T.segpair;
    t.wtile = ranked ? p->tile_wr : p->tile_w;
    t.tile_part = T.tile_part;
    t.tile_e = T.tile_e;
    t.tile_slot = T.tile_slot;
    t.tile_order = T.tile_order;
    t.split_part = T.split_part;
    t.split_slot = T.split_slot;
    t.pbuf = ranked ? p->tile_pbuf_r : p->tile_pbuf;
    t.m = p->g->dev.m;
    t.n_tiles = T.n_tiles;
    t.n_split = T.n_split;
    t.n_seg = T.n_seg;
    t.tw = 1u << T.tbits;
    t.tpart_r = p->tpart_r;
    t.tpart_a = p->tpart_a;
    t.tpart_p = p->tpart_p;
    t.spart_r = p->spart_r;
    t.spart_a = p->spart_a;
    t.spart_p = p->spart_p;
    return t;
  }
  static uint32_t tile_pull_grid(const daic_problem* p, bool ranked = false) {
    const TileGraph& T = ranked ? p->g->tile_r : p->g->tile;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(T.n_tiles, p->tile_grid));
  }
  static uint32_t tile_finish_grid(const daic_problem* p, bool ranked = false) {
    const TileGraph& T = ranked ? p->g->tile_r : p->g->tile;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(T.n_split * ((1ull << T.tbits) / 256), p->tfin_grid));
  }
  // The kernel arguments of fused rounds over the ranked layout: the state,
  // out-edge offsets, source numbers (and per-vertex alpha) in target-number
  // order, so every per-target access of the finishing work stays sequential.
  static KArgs ranked_args(const daic_problem* p) {
    KArgs a = p->a;
    const TileGraph& T = p->g->tile_r;
    a.v = p->vP;
    a.dv = p->dvP;
    a.c = p->cP;
    a.row = T.rowP;
    a.perm = T.permP;
    if (a.alpha_pv) a.alpha_pv = p->alphaP;
    return a;
  }

  static void fused_round(daic_problem* p, hipStream_t s, Prof* pr) {
    if constexpr (Tr<ST>::sum) {
      if (p->tile_ready) {
        const bool rk = ranked_on(p);
        const TileArgs t = tile_args(p, rk);
        const KArgs a = rk ? ranked_args(p) : p->a;
        const uint32_t np = tile_pull_grid(p, rk), nfin = tile_finish_grid(p, rk);
        launch(pr, "tile_pull", s, [&] {
          if (t.tw > kNarrowTW)
            hipLaunchKernelGGL((k_tile_pull<ST, G, true, 1024>), dim3(np), dim3(1024), 0, s, a, t);
          else
            hipLaunchKernelGGL((k_tile_pull<ST, G, true, 256>), dim3(np), dim3(256), 0, s, a, t);
        });
        launch(pr, "tile_finish", s, [&] {
          hipLaunchKernelGGL((k_tile_finish<ST, G, true>), dim3(nfin), dim3(256), 0, s, a, t);
        });
        launch(pr, "tile_total", s, [&] {
          hipLaunchKernelGGL((k_tile_total<ST, true>), dim3(1), dim3(256), 0, s, a, t, np, nfin, 0ull, 0ull);
        });
        return;
      }
      const uint32_t nf = fused_grid(p);
      launch(pr, "pull_fused", s, [&] {
        hipLaunchKernelGGL((k_pull_fused<ST, G>), dim3(nf), dim3(256), 0, s, p->a);
      });
      launch(pr, "fused_finish", s, [&] {
        hipLaunchKernelGGL((k_fused_finish<ST, G>), dim3(finish_grid(p)), dim3(256), 0, s, p->a, nf);
      });
    }
  }

  static Ops ops() { return Ops{&residual, &round, &select, &fuse_prime, &fused_round}; }
};

template <int ST, int G>
static bool pick_row(const daic_problem* p, Ops* out) {
  if (p->g->dev.row32) *out = Impl<ST, G, uint32_t>::ops();
  else *out = Impl<ST, G, uint64_t>::ops();
  return true;
}

bool get_ops(const daic_problem* p, Ops* out) {
  switch (p->st) {
    case ST_F64:
      if (p->gk == DAIC_G_SRC_SCALE) return pick_row<ST_F64, DAIC_G_SRC_SCALE>(p, out);
      if (p->gk == DAIC_G_DEG_SCALE) return pick_row<ST_F64, DAIC_G_DEG_SCALE>(p, out);
      if (p->gk == DAIC_G_EDGE_SCALE) return pick_row<ST_F64, DAIC_G_EDGE_SCALE>(p, out);
      return false;
    case ST_F32:
      if (p->gk == DAIC_G_SRC_SCALE) return pick_row<ST_F32, DAIC_G_SRC_SCALE>(p, out);
      if (p->gk == DAIC_G_DEG_SCALE) return pick_row<ST_F32, DAIC_G_DEG_SCALE>(p, out);
      if (p->gk == DAIC_G_EDGE_SCALE) return pick_row<ST_F32, DAIC_G_EDGE_SCALE>(p, out);
      return false;
    case ST_F32K:
      if (p->gk == DAIC_G_SRC_SCALE) return pick_row<ST_F32K, DAIC_G_SRC_SCALE>(p, out);
      if (p->gk == DAIC_G_DEG_SCALE) return pick_row<ST_F32K, DAIC_G_DEG_SCALE>(p, out);
      if (p->gk == DAIC_G_EDGE_SCALE) return pick_row<ST_F32K, DAIC_G_EDGE_SCALE>(p, out);
      return false;
    case ST_U32:
      if (p->gk == DAIC_G_EDGE_ADD) return pick_row<ST_U32, DAIC_G_EDGE_ADD>(p, out);
      return false;
    case ST_F64MIN:
      if (p->gk == DAIC_G_EDGE_ADD) return pick_row<ST_F64MIN, DAIC_G_EDGE_ADD>(p, out);
      return false;
    case ST_I32:
      if (p->gk == DAIC_G_COPY) return pick_row<ST_I32, DAIC_G_COPY>(p, out);
      return false;
  }
  return false;
}

// Set-up kernels that are not per instantiation.
__global__ void k_check_nonneg(const double* w, uint64_t m, uint32_t* bad) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
    if (!(w[e] >= 0.0)) *bad = 1u;  // negative or NaN
}

template <typename From, typename To>
__global__ void k_convert(const From* in, To* out, uint64_t count) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (; i < count; i += st) out[i] = (To)in[i];
}

__global__ void k_narrow_rows(const uint64_t* in, uint32_t* out, uint64_t count) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (; i < count; i += st) out[i] = (uint32_t)in[i];
}

// Device-side CSR validation for borrowed arrays: flags[0] = bad row_ptr,
// flags[1] = column out of range.
__global__ void k_validate(const uint64_t* row, const uint32_t* col, uint64_t n, uint64_t m, uint32_t* flags) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = i; j < n; j += st)
    if (row[j + 1] < row[j]) flags[0] = 1;
  if (i == 0 && (row[0] != 0 || row[n] != m)) flags[0] = 1;
  for (uint64_t e = i; e < m; e += st)
    if (col[e] >= n) flags[1] = 1;
}

template <typename T>
__global__ void k_fill(T* p, T val, uint64_t count) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (; i < count; i += st) p[i] = val;
}

static uint32_t grid_for(uint64_t count, uint32_t block = 256) {
  uint64_t g = (count + block - 1) / block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 8192));
}

// Finish graph set-up: narrowed rows, partition and large-bin regions.
static daic_status graph_finish(daic_graph* g, hipStream_t s) {
  GraphDev& d = g->dev;
  d.row32 = d.m < 0xFFFFFFFFull;
  if (d.row32 && d.n > 0) {
    uint32_t* r32;
    daic_status st = dalloc(&r32, d.n + 1);
    if (st) return st;
    g->row32 = r32;
    hipLaunchKernelGGL(k_narrow_rows, dim3(grid_for(d.n + 1)), dim3(256), 0, s,
                       static_cast<const uint64_t*>(d.row), r32, d.n + 1);
    d.row = r32;
  }
  g->part = make_partition(d.n);
  const uint32_t nb = g->part.blocks;
  std::vector<uint64_t> cap(nb + 1, 0);
  if (nb > 0) {
    uint64_t* dcap;
    daic_status st = dalloc(&dcap, nb);
    if (st) return st;
    if (d.row32)
      hipLaunchKernelGGL(k_large_capacity<uint32_t>, dim3(nb), dim3(256), 0, s, d.row, d.n, g->part.per_block, dcap);
    else
      hipLaunchKernelGGL(k_large_capacity<uint64_t>, dim3(nb), dim3(256), 0, s, d.row, d.n, g->part.per_block, dcap);
    hipError_t e = hipMemcpyAsync(cap.data() + 1, dcap, nb * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(dcap);
    if (e != hipSuccess) return fail(DAIC_E_DEVICE, "large-bin capacity: %s", hipGetErrorString(e));
  }
  for (uint32_t b = 0; b < nb; ++b) cap[b + 1] += cap[b];
  g->large_cap = cap[nb];
  daic_status st = dalloc(&g->large_off, nb + 1);
  if (st) return st;
  DAIC_HIP(hipMemcpyAsync(g->large_off, cap.data(), (nb + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  DAIC_HIP(hipStreamSynchronize(s));
  return DAIC_OK;
}

daic_status check_opts(const daic_problem* p, const daic_run_opts* o) {
  if (!o) return fail(DAIC_E_INVALID, "opts is null");
  if (!(o->priority_fraction > 0.0 && o->priority_fraction <= 1.0))
    return fail(DAIC_E_INVALID, "priority_fraction must be in (0, 1]");
  if (!(o->eps >= 0.0)) return fail(DAIC_E_INVALID, "eps must be >= 0");
  if (o->sched < DAIC_SCHED_ALL || o->sched > DAIC_SCHED_SWEEP) return fail(DAIC_E_INVALID, "unknown sched");
  if (o->sched == DAIC_SCHED_TOPK_SAMPLED && o->n_samples > kMaxSamples)
    return fail(DAIC_E_INVALID, "n_samples must be <= %u", kMaxSamples);
  if (o->sched == DAIC_SCHED_LEARNED && !o->model) return fail(DAIC_E_INVALID, "LEARNED needs a model");
  (void)p;
  return DAIC_OK;
}

// Dense rounds (pull over in-edges) for sum problems: builds the in-edge form
// on first use and sets the direction rule of this run. DAIC_NO_PULL=1 turns
// them off; DAIC_PULL_DIV (default 32) sets the fraction n/div of updating
// vertices from which a round runs dense.
// Per-run kernel arguments that depend on the options.
void apply_run_opts(daic_problem* p, const daic_run_opts* o) {
  const uint64_t n = p->g->dev.n;
  p->a.rr_chunk = std::max<uint64_t>(1, (uint64_t)std::ceil(o->priority_fraction * (double)n));
}

daic_status dense_rounds_setup(daic_problem* p, const daic_run_opts* o, hipStream_t s) {
  p->k_sel = 0;
  p->pull_min = 0;
  const bool sum = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
  const GraphDev& d = p->g->dev;
  // min and max problems take dense rounds through the tiled in-edges only
  if ((!sum && (std::getenv("DAIC_NO_TILE") || !tile_fits(d.m))) || std::getenv("DAIC_NO_PULL") || !d.row32 ||
      d.m > 0x7FFFFFFFull || d.n > 0x7FFFFFFFull)
    return DAIC_OK;
  if (!p->pull_ready) {
    daic_graph* g = const_cast<daic_graph*>(p->g);
    daic_status rc = pull_prepare(g, s);
    if (rc) return rc;
    const size_t S = state_size(p->st);
    void* mu = nullptr;
    DAIC_HIP(hipMalloc(&mu, std::max<uint64_t>(d.n, 1) * S));
    p->allocs.push_back(mu);
    DAIC_HIP(hipMemsetAsync(mu, 0, d.n * S, s));
    KArgs& a = p->a;
    a.mu_pi = mu;
    if (p->gk == DAIC_G_EDGE_SCALE) {
      void* wt = nullptr;
      DAIC_HIP(hipMalloc(&wt, std::max<uint64_t>(d.m, 1) * S));
      p->allocs.push_back(wt);
      if (p->st == ST_F64)
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(d.m)), dim3(256), 0, s,
                           static_cast<const double*>(a.w), g->pull.eidT, d.m, d.m, static_cast<double*>(wt));
      else
        hipLaunchKernelGGL(k_gather_weights<float>, dim3(grid_for(d.m)), dim3(256), 0, s,
                           static_cast<const float*>(a.w), g->pull.eidT, d.m, d.m, static_cast<float*>(wt));
      a.wT = wt;
    }
    a.perm = g->pull.perm;
    a.rowT = static_cast<const uint32_t*>(g->pull.rowT);
    a.srcT = g->pull.srcT;
    a.n_src = g->pull.n_src;
    a.sb_t = g->pull.sb_t;
    a.sb_e = g->pull.sb_e;
    a.sb_n = g->pull.sb_n;
    a.sb_count = g->pull.sb_count;
    // fused dense rounds: the second base buffer, the piece tickets and the
    // per-workgroup partials
    {
      void* mu2 = nullptr;
      DAIC_HIP(hipMalloc(&mu2, std::max<uint64_t>(d.n, 1) * S));
      p->allocs.push_back(mu2);
      DAIC_HIP(hipMemsetAsync(mu2, 0, d.n * S, s));
      a.mu_pi2 = mu2;
      a.sb_g = g->pull.sb_g;
      a.g_np = g->pull.g_np;
      a.g_first = g->pull.g_first;
      a.n_groups = g->pull.n_groups;
      auto grab8 = [&](void** q, uint64_t count) -> daic_status {
        DAIC_HIP(hipMalloc(q, std::max<uint64_t>(count, 1) * 8));
        p->allocs.push_back(*q);
        return DAIC_OK;
      };
      const uint64_t nf = std::max<uint64_t>(p->stream_grid, 1);
      const uint64_t nfin = std::max<uint64_t>((g->pull.n_groups + 255) / 256, (nf + 255) / 256);
      void *sp, *fr, *fa, *fp, *gr, *ga, *gp;
      if ((rc = grab8(&sp, g->pull.sb_count)) || (rc = grab8(&fr, nf)) || (rc = grab8(&fa, nf)) ||
          (rc = grab8(&fp, nf)) || (rc = grab8(&gr, nfin)) || (rc = grab8(&ga, nfin)) || (rc = grab8(&gp, nfin)))
        return rc;
      a.sb_part = static_cast<double*>(sp);
      a.fpart_r = static_cast<double*>(fr);
      a.fpart_a = static_cast<uint64_t*>(fa);
      a.fpart_p = static_cast<uint64_t*>(fp);
      a.gpart_r = static_cast<double*>(gr);
      a.gpart_a = static_cast<uint64_t*>(ga);
      a.gpart_p = static_cast<uint64_t*>(gp);
    }
    DAIC_HIP(hipStreamSynchronize(s));
    p->pull_ready = true;
    if (p->exec) {  // captured rounds predate the dense-round kernels
      (void)hipGraphExecDestroy(p->exec);
      p->exec = nullptr;
    }
  }
  // the tiled in-edge form of dense rounds (fused and not); DAIC_NO_TILE=1
  // keeps the streamed form
  if (!p->tile_ready && !std::getenv("DAIC_NO_TILE") && tile_fits(d.m)) {
    daic_graph* g = const_cast<daic_graph*>(p->g);
    daic_status rc = tile_prepare(g, s);
    if (rc) return rc;
    const TileGraph& T = g->tile;
    auto grab = [&](void** q, uint64_t bytes) -> daic_status {
      DAIC_HIP(hipMalloc(q, std::max<uint64_t>(bytes, 8)));
      p->allocs.push_back(*q);
      return DAIC_OK;
    };
    // slots: 8 bytes per entry covers every slot type (min/max accumulators too)
    if ((rc = grab((void**)&p->tile_pbuf, T.n_slots * (1ull << T.tbits) * 8)) ||
        (rc = grab((void**)&p->tpart_r, (uint64_t)p->tile_grid * 8)) ||
        (rc = grab((void**)&p->tpart_a, (uint64_t)p->tile_grid * 8)) ||
        (rc = grab((void**)&p->tpart_p, (uint64_t)p->tile_grid * 8)) ||
        (rc = grab((void**)&p->spart_r, (uint64_t)p->tfin_grid * 8)) ||
        (rc = grab((void**)&p->spart_a, (uint64_t)p->tfin_grid * 8)) ||
        (rc = grab((void**)&p->spart_p, (uint64_t)p->tfin_grid * 8)))
      return rc;
    const uint64_t pe = tile_padded_edges(T);
    if (p->gk == DAIC_G_EDGE_ADD) {  // weights in tile order: uint32 (U32 state) or double
      if (p->st == ST_U32) {
        if ((rc = grab(&p->tile_w, pe * 4))) return rc;
        hipLaunchKernelGGL(k_gather_weights<uint32_t>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const uint32_t*>(p->a.w), T.eid, d.m, pe, static_cast<uint32_t*>(p->tile_w));
      } else {
        if ((rc = grab(&p->tile_w, pe * 8))) return rc;
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const double*>(p->a.w), T.eid, d.m, pe, static_cast<double*>(p->tile_w));
      }
    }
    if (p->gk == DAIC_G_EDGE_SCALE) {
      const size_t S = state_size(p->st);
      if ((rc = grab(&p->tile_w, pe * S))) return rc;
      if (p->st == ST_F64)
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const double*>(p->a.w), T.eid, d.m, pe, static_cast<double*>(p->tile_w));
      else
        hipLaunchKernelGGL(k_gather_weights<float>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const float*>(p->a.w), T.eid, d.m, pe, static_cast<float*>(p->tile_w));
    }
    DAIC_HIP(hipStreamSynchronize(s));
    p->tile_ready = true;
    if (p->exec_fused) {  // captured fused rounds predate the tiled kernels
      (void)hipGraphExecDestroy(p->exec_fused);
      p->exec_fused = nullptr;
    }
  }
  // fused rounds (every pending vertex, sum problems) walk tiles whose
  // targets are numbered by in-degree octave, with the state moved into that
  // order while they run (RMAT-24 dense round 0.667 -> 0.52 ms, solve 81.0 ->
  // 63.1 ms); DAIC_TILE_ID_ORDER=1 keeps them on the id-ordered tiles
  if (sum && p->tile_ready && !p->ranked_ready && o->sched == DAIC_SCHED_ALL && !std::getenv("DAIC_TILE_ID_ORDER")) {
    daic_graph* g = const_cast<daic_graph*>(p->g);
    daic_status rc = tile_prepare_ranked(g, s);
    if (rc) return rc;
    const TileGraph& T = g->tile_r;
    const size_t S = state_size(p->st);
    auto grab = [&](void** q, uint64_t bytes) -> daic_status {
      DAIC_HIP(hipMalloc(q, std::max<uint64_t>(bytes, 8)));
      p->allocs.push_back(*q);
      return DAIC_OK;
    };
    if ((rc = grab(&p->vP, d.n * S)) || (rc = grab(&p->dvP, d.n * S)) ||
        (rc = grab((void**)&p->tile_pbuf_r, T.n_slots * (1ull << T.tbits) * 8)))
      return rc;
    if (p->a.c && (rc = grab((void**)&p->cP, d.n * 4))) return rc;
    if (p->a.alpha_pv && (rc = grab(&p->alphaP, d.n * S))) return rc;
    if (p->gk == DAIC_G_EDGE_SCALE) {  // weights in the ranked tile order
      const uint64_t pe = tile_padded_edges(T);
      if ((rc = grab(&p->tile_wr, pe * S))) return rc;
      if (p->st == ST_F64)
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const double*>(p->a.w), T.eid, d.m, pe, static_cast<double*>(p->tile_wr));
      else
        hipLaunchKernelGGL(k_gather_weights<float>, dim3(grid_for(pe)), dim3(256), 0, s,
                           static_cast<const float*>(p->a.w), T.eid, d.m, pe, static_cast<float*>(p->tile_wr));
    }
    DAIC_HIP(hipStreamSynchronize(s));
    p->ranked_ready = true;
    if (p->exec_fused) {  // captured with the id-ordered tiles
      (void)hipGraphExecDestroy(p->exec_fused);
      p->exec_fused = nullptr;
    }
  }
  // the dense-round threshold: sum problems n / 32 vertices expected to
  // update; min and max problems m / 4 messages expected (their pushes are
  // filtered by v and dv and cheap per message, so a pull over every in-edge
  // pays only for wide frontiers)
  uint64_t div = sum ? 32 : 4;
  if (const char* e = std::getenv(sum ? "DAIC_PULL_DIV" : "DAIC_PULL_EDGE_DIV"))
    div = std::max<uint64_t>(1, std::strtoull(e, nullptr, 10));
  const uint64_t n = d.n;
  p->k_sel = o->sched == DAIC_SCHED_ALL ? n : std::max<uint64_t>(1, (uint64_t)std::ceil(o->priority_fraction * (double)n));
  p->pull_min = std::max<uint64_t>(1, ((sum ? n : d.m) + div - 1) / div);
  return DAIC_OK;
}

}  // namespace daic

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* daic_last_error(void) { return daic::g_err.c_str(); }

daic_status daic_graph_create(uint64_t n, uint64_t m, const uint64_t* row_ptr, const uint32_t* col,
                              const void* w, daic_dtype w_type, daic_graph** out) {
  if (!out) return fail(DAIC_E_INVALID, "out is null");
  *out = nullptr;
  if (!row_ptr) return fail(DAIC_E_INVALID, "row_ptr is null");
  if (m > 0 && !col) return fail(DAIC_E_INVALID, "col is null");
  if (n >= 0xFFFFFFFFull) return fail(DAIC_E_INVALID, "n must be below 2^32-1");
  if (row_ptr[0] != 0 || row_ptr[n] != m) return fail(DAIC_E_INVALID, "row_ptr[0] must be 0 and row_ptr[n] must be m");
  const uint64_t bad_row = first_index_where(n, [&](uint64_t j) { return row_ptr[j + 1] < row_ptr[j]; });
  if (bad_row < n) return fail(DAIC_E_INVALID, "row_ptr not monotone at %llu", (unsigned long long)bad_row);
  const uint64_t bad_col = first_index_where(m, [&](uint64_t e) { return col[e] >= n; });
  if (bad_col < m) return fail(DAIC_E_INVALID, "col[%llu] = %u out of range", (unsigned long long)bad_col, col[bad_col]);
  size_t wsz = 0;
  if (w) {
    if (w_type == DAIC_F64) wsz = 8;
    else if (w_type == DAIC_F32 || w_type == DAIC_U32) wsz = 4;
    else return fail(DAIC_E_INVALID, "weight type must be F64, F32 or U32");
  } else {
    w_type = DAIC_NONE;
  }
  std::unique_ptr<daic_graph> g(new daic_graph());
  g->dev.n = n;
  g->dev.m = m;
  g->dev.w_type = w_type;
  uint64_t* drow;
  uint32_t* dcol;
  daic_status st = dalloc(&drow, n + 1);
  if (st) return st;
  g->own_row = drow;
  st = dalloc(&dcol, m);
  if (st) { daic_graph_destroy(g.release()); return st; }
  g->own_col = dcol;
  DAIC_HIP(hipMemcpy(drow, row_ptr, (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
  if (m) DAIC_HIP(hipMemcpy(dcol, col, m * sizeof(uint32_t), hipMemcpyHostToDevice));
  if (w) {
    uint8_t* dw;
    st = dalloc(&dw, m * wsz);
    if (st) { daic_graph_destroy(g.release()); return st; }
    g->own_w = dw;
    if (m) DAIC_HIP(hipMemcpy(dw, w, m * wsz, hipMemcpyHostToDevice));
    g->dev.w = dw;
  }
  g->dev.row = drow;
  g->dev.col = dcol;
  st = graph_finish(g.get(), nullptr);
  if (st) { daic_graph_destroy(g.release()); return st; }
  *out = g.release();
  return DAIC_OK;
}

daic_status daic_graph_create_device(uint64_t n, uint64_t m, const uint64_t* d_row_ptr, const uint32_t* d_col,
                                     const void* d_w, daic_dtype w_type, void* hip_stream, daic_graph** out) {
  if (!out) return fail(DAIC_E_INVALID, "out is null");
  *out = nullptr;
  if (!d_row_ptr || (m > 0 && !d_col)) return fail(DAIC_E_INVALID, "null device array");
  if (n >= 0xFFFFFFFFull) return fail(DAIC_E_INVALID, "n must be below 2^32-1");
  if (d_w && !(w_type == DAIC_F64 || w_type == DAIC_F32 || w_type == DAIC_U32))
    return fail(DAIC_E_INVALID, "weight type must be F64, F32 or U32");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t* flags;
  daic_status st = dalloc(&flags, 2);
  if (st) return st;
  DAIC_HIP(hipMemsetAsync(flags, 0, 2 * sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_validate, dim3(grid_for(std::max(n, m))), dim3(256), 0, s, d_row_ptr, d_col, n, m, flags);
  uint32_t hf[2] = {0, 0};
  DAIC_HIP(hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, s));
  DAIC_HIP(hipStreamSynchronize(s));
  dfree(flags);
  if (hf[0]) return fail(DAIC_E_INVALID, "row_ptr is not a valid CSR offset array");
  if (hf[1]) return fail(DAIC_E_INVALID, "a column index is out of range");
  std::unique_ptr<daic_graph> g(new daic_graph());
  g->dev.n = n;
  g->dev.m = m;
  g->dev.row = d_row_ptr;
  g->dev.col = d_col;
  g->dev.w = d_w;
  g->dev.w_type = d_w ? w_type : DAIC_NONE;
  st = graph_finish(g.get(), s);
  if (st) { daic_graph_destroy(g.release()); return st; }
  *out = g.release();
  return DAIC_OK;
}

void daic_graph_destroy(daic_graph* g) {
  if (!g) return;
  dfree(g->own_row);
  dfree(g->own_col);
  dfree(g->own_w);
  dfree(g->row32);
  dfree(g->large_off);
  pull_release(g);
  tile_release(g);
  delete g;
}

daic_status daic_problem_create(const daic_graph* g, daic_op op, daic_g gk, double alpha_scalar,
                                const double* alpha_per_vertex, daic_dtype state, daic_problem** out) {
  if (!out) return fail(DAIC_E_INVALID, "out is null");
  *out = nullptr;
  if (!g) return fail(DAIC_E_INVALID, "graph is null");
  int st;
  if (op == DAIC_SUM) {
    if (!(gk == DAIC_G_SRC_SCALE || gk == DAIC_G_DEG_SCALE || gk == DAIC_G_EDGE_SCALE))
      return fail(DAIC_E_UNSUPPORTED, "sum takes SRC_SCALE, DEG_SCALE or EDGE_SCALE");
    if (state == DAIC_F64) st = ST_F64;
    else if (state == DAIC_F32) st = ST_F32;
    else if (state == DAIC_F32_KAHAN) st = ST_F32K;
    else return fail(DAIC_E_UNSUPPORTED, "sum takes F64, F32 or F32_KAHAN state");
    if (gk == DAIC_G_EDGE_SCALE && !g->dev.w) return fail(DAIC_E_INVALID, "EDGE_SCALE needs edge weights");
    if (gk == DAIC_G_DEG_SCALE && alpha_per_vertex)
      return fail(DAIC_E_INVALID, "DEG_SCALE takes a scalar alpha only");
  } else if (op == DAIC_MIN) {
    if (gk != DAIC_G_EDGE_ADD) return fail(DAIC_E_UNSUPPORTED, "min takes EDGE_ADD");
    if (state == DAIC_U32) {
      if (!g->dev.w || g->dev.w_type != DAIC_U32) return fail(DAIC_E_INVALID, "EDGE_ADD with U32 state needs U32 edge weights");
      st = ST_U32;
    } else if (state == DAIC_F64) {
      if (!g->dev.w) return fail(DAIC_E_INVALID, "EDGE_ADD needs edge weights");
      st = ST_F64MIN;
    } else {
      return fail(DAIC_E_UNSUPPORTED, "min takes U32 or F64 state");
    }
  } else if (op == DAIC_MAX) {
    if (gk != DAIC_G_COPY) return fail(DAIC_E_UNSUPPORTED, "max takes COPY");
    if (state != DAIC_I32) return fail(DAIC_E_UNSUPPORTED, "max takes I32 state");
    st = ST_I32;
  } else {
    return fail(DAIC_E_INVALID, "unknown op");
  }
  if (alpha_per_vertex && !(gk == DAIC_G_SRC_SCALE || gk == DAIC_G_EDGE_SCALE))
    return fail(DAIC_E_INVALID, "per-vertex alpha only for SRC_SCALE and EDGE_SCALE");
  if (!std::isfinite(alpha_scalar)) return fail(DAIC_E_INVALID, "alpha must be finite");

  std::unique_ptr<daic_problem> p(new daic_problem());
  p->g = g;
  p->op = op;
  p->gk = gk;
  p->state = state;
  p->st = st;
  p->alpha = alpha_scalar;
  const GraphDev& d = g->dev;
  const uint64_t n = d.n, m = d.m;
  const size_t S = state_size(st);
  const uint32_t nb = g->part.blocks;
  auto grab = [&](void** ptr, size_t bytes) -> daic_status {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(DAIC_E_OOM, "hipMalloc of %zu bytes failed", bytes);
    p->allocs.push_back(q);
    *ptr = q;
    return DAIC_OK;
  };
  daic_status rc;
  KArgs& a = p->a;
  void* ptr;
#define GRAB(field, type, bytes)                            \
  do {                                                      \
    rc = grab(&ptr, (bytes));                               \
    if (rc) { daic_problem_destroy(p.release()); return rc; } \
    a.field = static_cast<type>(ptr);                       \
  } while (0)
  GRAB(ctl, Ctl*, sizeof(Ctl));
  GRAB(v, void*, n * S);
  GRAB(dv, void*, n * S);
  if (st == ST_F32K) GRAB(c, float*, n * sizeof(float));
  GRAB(small_vid, uint32_t*, n * 4);
  GRAB(small_mu, void*, n * S);
  GRAB(large_vid, uint32_t*, g->large_cap * 4);
  GRAB(large_chunk, uint32_t*, g->large_cap * 4);
  GRAB(large_mu, void*, g->large_cap * S);
  GRAB(blk_small, uint32_t*, nb * 4);
  GRAB(blk_large, uint32_t*, nb * 4);
  GRAB(blk_ties, uint32_t*, nb * 4);
  GRAB(rhist, uint32_t*, kRadixBins * kRadixCopies * 4);
  GRAB(skeys, uint64_t*, kMaxSamples * 8);
  GRAB(off_small, uint64_t*, (nb + 1) * 8);
  GRAB(off_large, uint64_t*, (nb + 1) * 8);
  GRAB(off_ties, uint64_t*, (nb + 1) * 8);
  GRAB(blk_act, uint64_t*, nb * 8);
  GRAB(blk_push, uint64_t*, nb * 8);
  GRAB(blk_push_large, uint64_t*, nb * 8);
  GRAB(part_r, double*, nb * 8);
  GRAB(part_n, uint64_t*, nb * 8);
#undef GRAB
  a.row = d.row;
  a.col = d.col;
  a.alpha = alpha_scalar;
  a.n = n;
  a.per_block = g->part.per_block;
  a.blocks = nb;
  a.large_off = g->large_off;
  a.sel_out = nullptr;
  a.score = nullptr;

  hipStream_t s = nullptr;
  // weights in the element type the push needs
  if (gk == DAIC_G_EDGE_SCALE) {
    bool same = (st == ST_F64 && d.w_type == DAIC_F64) || (st != ST_F64 && d.w_type == DAIC_F32);
    if (same) {
      a.w = d.w;
    } else {
      rc = grab(&p->w_conv, m * S);
      if (rc) { daic_problem_destroy(p.release()); return rc; }
      uint32_t gr = grid_for(m);
      if (st == ST_F64) {
        if (d.w_type == DAIC_F32) hipLaunchKernelGGL((k_convert<float, double>), dim3(gr), dim3(256), 0, s, (const float*)d.w, (double*)p->w_conv, m);
        else hipLaunchKernelGGL((k_convert<uint32_t, double>), dim3(gr), dim3(256), 0, s, (const uint32_t*)d.w, (double*)p->w_conv, m);
      } else {
        if (d.w_type == DAIC_F64) hipLaunchKernelGGL((k_convert<double, float>), dim3(gr), dim3(256), 0, s, (const double*)d.w, (float*)p->w_conv, m);
        else hipLaunchKernelGGL((k_convert<uint32_t, float>), dim3(gr), dim3(256), 0, s, (const uint32_t*)d.w, (float*)p->w_conv, m);
      }
      a.w = p->w_conv;
    }
  } else if (gk == DAIC_G_EDGE_ADD && st == ST_F64MIN) {
    // real weights as doubles, which must be non-negative and not NaN (the
    // atomic min compares bit patterns, and shortest paths need w >= 0)
    if (d.w_type == DAIC_F64) {
      a.w = d.w;
    } else {
      rc = grab(&p->w_conv, m * 8);
      if (rc) { daic_problem_destroy(p.release()); return rc; }
      const uint32_t gr = grid_for(m);
      if (d.w_type == DAIC_F32) hipLaunchKernelGGL((k_convert<float, double>), dim3(gr), dim3(256), 0, s, (const float*)d.w, (double*)p->w_conv, m);
      else hipLaunchKernelGGL((k_convert<uint32_t, double>), dim3(gr), dim3(256), 0, s, (const uint32_t*)d.w, (double*)p->w_conv, m);
      a.w = p->w_conv;
    }
    uint32_t* bad = nullptr;
    DAIC_HIP(hipMalloc(&bad, 4));
    hipError_t e = hipMemset(bad, 0, 4);
    if (e == hipSuccess && m)
      hipLaunchKernelGGL(k_check_nonneg, dim3(grid_for(m)), dim3(256), 0, s, (const double*)a.w, m, bad);
    uint32_t h_bad = 0;
    if (e == hipSuccess) e = hipMemcpy(&h_bad, bad, 4, hipMemcpyDeviceToHost);
    (void)hipFree(bad);
    if (e != hipSuccess) {
      daic_problem_destroy(p.release());
      return fail(DAIC_E_DEVICE, "weight check: %s", hipGetErrorString(e));
    }
    if (h_bad) {
      daic_problem_destroy(p.release());
      return fail(DAIC_E_INVALID, "EDGE_ADD with F64 state needs non-negative weights (no NaN)");
    }
  } else if (gk == DAIC_G_EDGE_ADD) {
    a.w = d.w;
  }
  if (alpha_per_vertex) {
    rc = grab(&p->alpha_pv, n * S);
    if (rc) { daic_problem_destroy(p.release()); return rc; }
    if (st == ST_F64) {
      DAIC_HIP(hipMemcpy(p->alpha_pv, alpha_per_vertex, n * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> tmp(n);
      for (uint64_t j = 0; j < n; ++j) tmp[j] = (float)alpha_per_vertex[j];
      DAIC_HIP(hipMemcpy(p->alpha_pv, tmp.data(), n * 4, hipMemcpyHostToDevice));
    }
    a.alpha_pv = p->alpha_pv;
  }
  // identity state
  const uint32_t gr = grid_for(n);
  if (st == ST_F64) {
    hipLaunchKernelGGL(k_fill<double>, dim3(gr), dim3(256), 0, s, (double*)a.v, 0.0, n);
    hipLaunchKernelGGL(k_fill<double>, dim3(gr), dim3(256), 0, s, (double*)a.dv, 0.0, n);
  } else if (st == ST_F32 || st == ST_F32K) {
    hipLaunchKernelGGL(k_fill<float>, dim3(gr), dim3(256), 0, s, (float*)a.v, 0.0f, n);
    hipLaunchKernelGGL(k_fill<float>, dim3(gr), dim3(256), 0, s, (float*)a.dv, 0.0f, n);
    if (a.c) hipLaunchKernelGGL(k_fill<float>, dim3(gr), dim3(256), 0, s, a.c, 0.0f, n);
  } else if (st == ST_U32) {
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(gr), dim3(256), 0, s, (uint32_t*)a.v, kInfU32, n);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(gr), dim3(256), 0, s, (uint32_t*)a.dv, kInfU32, n);
  } else if (st == ST_F64MIN) {
    const double inf = std::numeric_limits<double>::infinity();
    hipLaunchKernelGGL(k_fill<double>, dim3(gr), dim3(256), 0, s, (double*)a.v, inf, n);
    hipLaunchKernelGGL(k_fill<double>, dim3(gr), dim3(256), 0, s, (double*)a.dv, inf, n);
  } else {
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(gr), dim3(256), 0, s, (int32_t*)a.v, -1, n);
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(gr), dim3(256), 0, s, (int32_t*)a.dv, -1, n);
  }
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, a.ctl, 0.0, 0ull);
  DAIC_HIP(hipHostMalloc((void**)&p->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  DAIC_HIP(hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking));
  DAIC_HIP(hipEventCreate(&p->ev0));
  DAIC_HIP(hipEventCreate(&p->ev1));
  DAIC_HIP(hipDeviceSynchronize());
  Ops ops;
  if (!get_ops(p.get(), &ops)) {
    daic_problem_destroy(p.release());
    return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  }
  *out = p.release();
  return DAIC_OK;
}

daic_status daic_problem_set_init(daic_problem* p, const void* v0, const void* dv1) {
  if (!p || !v0 || !dv1) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  if (p->st == ST_F64 || p->st == ST_U32 || p->st == ST_I32 || p->st == ST_F64MIN) {
    size_t S = state_size(p->st);
    DAIC_HIP(hipMemcpy(p->a.v, v0, n * S, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy(p->a.dv, dv1, n * S, hipMemcpyHostToDevice));
  } else {
    const double* a = static_cast<const double*>(v0);
    const double* b = static_cast<const double*>(dv1);
    std::vector<float> tv(n), td(n), tc(n, 0.0f);
    for (uint64_t j = 0; j < n; ++j) {
      tv[j] = (float)a[j];
      td[j] = (float)b[j];
      // carry the FP32 rounding of v0 in the compensation term
      tc[j] = (float)((double)tv[j] - a[j]);
    }
    DAIC_HIP(hipMemcpy(p->a.v, tv.data(), n * 4, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy(p->a.dv, td.data(), n * 4, hipMemcpyHostToDevice));
    if (p->a.c) DAIC_HIP(hipMemcpy(p->a.c, tc.data(), n * 4, hipMemcpyHostToDevice));
  }
  return DAIC_OK;
}

static double per_edge_bytes(const daic_problem* p) {
  const double S = (double)state_size(p->st);
  double b = 4.0 + 2.0 * S;  // col + RMW of dv_k
  if (p->gk == DAIC_G_EDGE_SCALE) b += S;
  if (p->gk == DAIC_G_EDGE_ADD) b += p->st == ST_F64MIN ? 8.0 : 4.0;
  return b;
}

static double per_vertex_bytes(const daic_problem* p) {
  const double S = (double)state_size(p->st);
  const double R = p->g->dev.row32 ? 4.0 : 8.0;
  double b = 2.0 * R + 2.0 * S + 2.0 * S;  // row offsets, dv claim, v fold
  if (p->st == ST_F32K) b += 8.0;           // c fold
  b += 2.0 * (4.0 + S);                     // frontier item write + read
  return b;
}

daic_status daic_run(daic_problem* p, const daic_run_opts* o, daic_stats* stats) {
  if (!p) return fail(DAIC_E_INVALID, "problem is null");
  daic_status rc = check_opts(p, o);
  if (rc) return rc;
  apply_run_opts(p, o);
  const uint64_t n = p->g->dev.n;
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : p->own_stream;
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n == 0) return DAIC_OK;
  if (std::getenv("DAIC_CHECK_INIT")) {  // debug: the starting state must meet the fourth condition
    rc = check_init(p, 0.0, nullptr, s);
    if (rc) return rc;
  }
  if (o->sched == DAIC_SCHED_SWEEP) return sweep_run(p, o, stats, s);
  Ops ops;
  if (!get_ops(p, &ops)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  const uint32_t K = o->rounds_per_check ? o->rounds_per_check : 1;
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;
  if (o->sched == DAIC_SCHED_LEARNED) {
    rc = learned_prepare(p, o->model, s);
    if (rc) return rc;
  }

  rc = dense_rounds_setup(p, o, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, o->eps, max_rounds);
  ops.residual(p, s, 0);
  DAIC_HIP(hipEventRecord(p->ev0, s));

  const bool learned = o->sched == DAIC_SCHED_LEARNED;
  const bool use_graph = std::getenv("DAIC_NO_GRAPH") == nullptr;
  // Learned rounds rank by priority x sigmoid(score). Exact top-k is the
  // fallback and the judge, decided on the device each round (k_learned_pre /
  // k_learned_post): one exact round calibrates the priority realized per
  // message, a learned round below 0.8 x that figure hands the next 4 rounds
  // back to exact selection, and every 16 learned rounds are followed by a
  // fresh calibration round. So learned rounds are captured like the others.
  const bool sum_state = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
  const float* sc = nullptr;
  if (learned) {
    rc = learned_scores_array(p, o->model, &sc);
    if (rc) return rc;
  }
  auto one_round = [&]() {
    if (learned) {
      hipLaunchKernelGGL(k_learned_pre, dim3(1), dim3(1), 0, s, p->a.ctl);
      learned_scores_enqueue(p, o->model, s);
      ops.round(p, o, s, sc, nullptr);
      if (sum_state) hipLaunchKernelGGL(k_learned_post<true>, dim3(1), dim3(1), 0, s, p->a.ctl);
      else hipLaunchKernelGGL(k_learned_post<false>, dim3(1), dim3(1), 0, s, p->a.ctl);
    } else {
      ops.round(p, o, s, nullptr, nullptr);
    }
  };
  GraphCacheKey key;
  key.sched = o->sched;
  key.k = (uint64_t)std::ceil(o->priority_fraction * (double)n);
  key.S = o->n_samples;
  key.q = o->priority_fraction;
  key.seed = o->seed;
  key.K = K;
  key.stream = s;
  key.k_sel = p->k_sel;
  key.pull_min = p->pull_min;
  key.score = sc;
  key.model = learned ? o->model : nullptr;
  key.model_version = learned ? learned_model_version(o->model) : 0;
  if (use_graph && !(p->exec && p->key == key)) {
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (uint32_t r = 0; r < K; ++r) one_round();
    hipGraph_t graph;
    DAIC_HIP(hipStreamEndCapture(s, &graph));
    p->graph = graph;
    DAIC_HIP(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0));
    p->key = key;
  }
  // Fused dense rounds (every pending vertex, sum problems, in-edge form):
  // entered when a dense round is next and at least two rounds remain.
  const bool fuse = use_graph && o->sched == DAIC_SCHED_ALL && sum_state && p->pull_ready &&
                    std::getenv("DAIC_NO_FUSE") == nullptr;
  bool fused = false;
  if (fuse) {
    DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
  }
  uint64_t seen_rounds = ~0ull;
  for (;;) {
    if (fuse && !fused) {
      const Ctl& c = *p->h_ctl;
      if (!c.done && !c.stop && c.pull && c.rounds < max_rounds) {
        ops.fuse_prime(p, o, s, nullptr);
        if (!(p->exec_fused && p->fused_K == K && p->fused_stream == s)) {
          if (p->exec_fused) { (void)hipGraphExecDestroy(p->exec_fused); p->exec_fused = nullptr; }
          if (p->graph_fused) { (void)hipGraphDestroy(p->graph_fused); p->graph_fused = nullptr; }
          DAIC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          for (uint32_t r = 0; r < K; ++r) ops.fused_round(p, s, nullptr);
          hipGraph_t graph;
          DAIC_HIP(hipStreamEndCapture(s, &graph));
          p->graph_fused = graph;
          DAIC_HIP(hipGraphInstantiate(&p->exec_fused, graph, nullptr, nullptr, 0));
          p->fused_K = K;
          p->fused_stream = s;
        }
        fused = true;
      }
    }
    if (fused) {
      DAIC_HIP(hipGraphLaunch(p->exec_fused, s));
    } else if (use_graph) {
      DAIC_HIP(hipGraphLaunch(p->exec, s));
    } else {
      for (uint32_t r = 0; r < K; ++r) one_round();
    }
    DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    if (p->h_ctl->done || p->h_ctl->stop) break;
    // every round advances the count; a launch that did not means the
    // control block is inconsistent: fail instead of spinning
    if (p->h_ctl->rounds == seen_rounds) {
      ranked_leave(p, s);
      return fail(DAIC_E_DEVICE, "run made no progress (round %llu)", (unsigned long long)seen_rounds);
    }
    seen_rounds = p->h_ctl->rounds;
  }
  ranked_leave(p, s);
  DAIC_HIP(hipEventRecord(p->ev1, s));
  DAIC_HIP(hipEventSynchronize(p->ev1));
  p->a.last_upd = nullptr;  // rounds of the other rules do not track updates
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
    stats->alg_bytes = (double)c.pushed * per_edge_bytes(p) + (double)c.activations * per_vertex_bytes(p) +
                       (double)c.rounds * (double)n * (double)state_size(p->st) * 2.0;
    stats->learned_fallbacks = learned ? c.l_fallbacks : 0;
    stats->learned_exact_rounds = learned ? c.l_exact_rounds : 0;
  }
  return c.done ? DAIC_OK : DAIC_NOT_CONVERGED;
}

daic_status daic_problem_set_init_device(daic_problem* p, const void* d_v0, const void* d_dv1, void* hip_stream) {
  if (!p || !d_v0 || !d_dv1) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : p->own_stream;
  const size_t S = state_size(p->st);
  DAIC_HIP(hipMemcpyAsync(p->a.v, d_v0, n * S, hipMemcpyDeviceToDevice, s));
  DAIC_HIP(hipMemcpyAsync(p->a.dv, d_dv1, n * S, hipMemcpyDeviceToDevice, s));
  if (p->a.c) hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(256), 0, s, p->a.c, 0.0f, n);
  if (!hip_stream) DAIC_HIP(hipStreamSynchronize(s));
  return DAIC_OK;
}

// Algorithmic bytes of one launch of a kernel class in the round just run.
static double kernel_bytes(const daic_problem* p, const char* name, const Ctl& c) {
  const double S = (double)state_size(p->st);
  const double R = p->g->dev.row32 ? 4.0 : 8.0;
  const double e = per_edge_bytes(p);
  const double n = (double)p->g->dev.n;
  const double small_edges = (double)(c.round_pushed - c.round_pushed_large);
  if (!std::strcmp(name, "push_edges"))  // per edge as per_edge_bytes; per item vid, base and row offsets (+ chunk)
    return (small_edges + (double)c.round_pushed_large) * e + (double)c.n_small * (4.0 + S + 2.0 * R) +
           (double)c.n_large * (8.0 + S + 2.0 * R);
  if (!std::strcmp(name, "claim")) {
    double kahan = p->st == ST_F32K ? 8.0 : 0.0;
    double out = c.last_pull ? n * (4.0 + S) : (double)(c.n_small + c.n_large) * (4.0 + S);
    return n * 2.0 * S + (double)c.round_act * (2.0 * R + 2.0 * S + kahan) + out;
  }
  if (!std::strcmp(name, "residual")) return n * S;
  if (!std::strcmp(name, "pull_stream")) {
    // per in-edge: source 4 + message base S (+ weight S); per edge block 16;
    // dv read of every vertex S; per target with in-edges: offsets 2R + dv
    // written S; per workgroup the two residual partials 16
    const PullGraph& P = p->g->pull;
    const double per_in_edge = 4.0 + S + (p->gk == DAIC_G_EDGE_SCALE ? S : 0.0);
    const double nf = (double)std::max<uint64_t>(1, std::min<uint64_t>(P.sb_count, p->stream_grid));
    return (double)p->g->dev.m * per_in_edge + (double)P.sb_count * 16.0 + n * S +
           (double)P.n_targets * (2.0 * R + S) + nf * 16.0;
  }
  if (!std::strcmp(name, "pull_finish")) {
    // the partials of pull_stream 16 each and the final dv of every cut
    // target (block number 4, target 4, dv S)
    const PullGraph& P = p->g->pull;
    const double nf = (double)std::max<uint64_t>(1, std::min<uint64_t>(P.sb_count, p->stream_grid));
    return nf * 16.0 + (double)P.n_groups * (8.0 + S);
  }
  if (!std::strcmp(name, "fused_finish")) {
    // the pieces' partial sums 8 each, the claim of every cut target (as in
    // pull_fused) and the per-workgroup partials of pull_fused (3 x 8 each)
    const PullGraph& P = p->g->pull;
    const double kahan = p->st == ST_F32K ? 8.0 : 0.0;
    const uint64_t pieces = P.n_pieces;
    const double nf = (double)std::max<uint64_t>(1, std::min<uint64_t>(P.sb_count, p->stream_grid));
    return (double)pieces * 8.0 + (double)P.n_groups * (4.0 + 4.0 + 4.0 * S + kahan + 2.0 * R + 4.0 + S) + nf * 24.0;
  }
  if (!std::strcmp(name, "pull_tile") || !std::strcmp(name, "pull_tile_finish")) {
    // as tile_pull / tile_finish below with a target's finish reduced to its
    // dv read and written (2S; min and max problems also read v: 3S): the
    // claim of these rounds ran before. Weights in tile order: S (EDGE_SCALE)
    // or the weight type (EDGE_ADD) per in-edge.
    const TileGraph& T = p->g->tile;
    const bool sum = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
    const double tw = (double)(1ull << T.tbits);
    const double split_targets = (double)T.n_split * tw;
    const double slots = (double)T.n_slots * tw * (sum ? (double)slot_size(p->st) : S);
    const double wb = p->gk == DAIC_G_EDGE_SCALE ? S : p->gk == DAIC_G_EDGE_ADD ? (p->st == ST_U32 ? 4.0 : 8.0) : 0.0;
    const double fin = (sum ? 2.0 : 3.0) * S;
    if (!std::strcmp(name, "pull_tile"))
      return (double)p->g->dev.m * (2.0 + wb) + (double)T.n_pairs * (4.0 + S) + (double)T.n_seg * 4.0 +
             (double)T.n_tiles * 12.0 + std::max(0.0, n - split_targets) * fin + slots;
    return slots + std::min(n, split_targets) * fin;
  }
  if (!std::strcmp(name, "tile_pull") || !std::strcmp(name, "tile_finish")) {
    // tile_pull: per in-edge its local target 2 (+ weight S), per (source,
    // partition) pair the source 4 and its base S, per 64 in-edges the
    // segment's pair 4, per tile 12, and the finish of every target of the
    // partitions of one tile as below; the tiles of split partitions store
    // their partial sums (4 per target for FP32 states, 8 for FP64 ones).
    // tile_finish: the slots read back per target and tile, and the finish of
    // those targets. The finish of a
    // target: dv read and write 2S, v read and write 2S (+ Kahan term 8),
    // out-edge offsets 2R, renumbering 4, base written S. Fused rounds walk
    // the layout with targets numbered by in-degree octave when it is built.
    const TileGraph& T = ranked_on(p) ? p->g->tile_r : p->g->tile;
    const double kahan = p->st == ST_F32K ? 8.0 : 0.0;
    const double fin = 2.0 * S + 2.0 * S + kahan + 2.0 * R + 4.0 + S;
    const double tw = (double)(1ull << T.tbits);
    const double split_targets = (double)T.n_split * tw;  // upper bound (the last partition may be short)
    const double slots = (double)T.n_slots * tw * (double)slot_size(p->st);
    if (name[5] == 'p')
      return (double)p->g->dev.m * (2.0 + (p->gk == DAIC_G_EDGE_SCALE ? S : 0.0)) + (double)T.n_pairs * (4.0 + S) +
             (double)T.n_seg * 4.0 + (double)T.n_tiles * 12.0 + std::max(0.0, n - split_targets) * fin + slots;
    return slots + std::min(n, split_targets) * fin;
  }
  if (!std::strcmp(name, "pull_fused")) {
    // the pull as above (descriptor 16 per block, in-edge offsets 2R per
    // target) and the claim of every vertex: dv read and write 2S, v read
    // and write 2S (+ Kahan term 8), out-edge offsets 2R, renumbering 4,
    // base written S
    const PullGraph& P = p->g->pull;
    const double per_in_edge = 4.0 + S + (p->gk == DAIC_G_EDGE_SCALE ? S : 0.0);
    const double kahan = p->st == ST_F32K ? 8.0 : 0.0;
    return (double)p->g->dev.m * per_in_edge + (double)P.sb_count * 16.0 +
           n * (2.0 * R + 2.0 * S + 2.0 * S + kahan + 2.0 * R + 4.0 + S);
  }
  return 0.0;
}

daic_status daic_profile(daic_problem* p, const daic_run_opts* o, uint32_t cap, daic_kernel_time* out,
                         uint32_t* n_out, daic_stats* stats) {
  if (!p || !out || !n_out) return fail(DAIC_E_INVALID, "null argument");
  daic_status rc = check_opts(p, o);
  if (rc) return rc;
  if (o->sched == DAIC_SCHED_SWEEP) return fail(DAIC_E_UNSUPPORTED, "daic_profile takes the per-round rules, not SWEEP");
  apply_run_opts(p, o);
  if (o->sched == DAIC_SCHED_LEARNED) return fail(DAIC_E_UNSUPPORTED, "profile takes the plain rules");
  *n_out = 0;
  const uint64_t n = p->g->dev.n;
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n == 0) return DAIC_OK;
  Ops ops;
  if (!get_ops(p, &ops)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : p->own_stream;
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;
  rc = dense_rounds_setup(p, o, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, o->eps, max_rounds);
  ops.residual(p, s, 0);
  DAIC_HIP(hipStreamSynchronize(s));
  std::vector<daic_kernel_time> acc;
  auto slot = [&](const char* name) -> daic_kernel_time& {
    for (auto& k : acc)
      if (!std::strcmp(k.name, name)) return k;
    daic_kernel_time k{};
    std::snprintf(k.name, sizeof k.name, "%s", name);
    acc.push_back(k);
    return acc.back();
  };
  Prof prof;
  double total_ms = 0.0;
  // the same round forms as daic_run, fused dense rounds included
  const bool sum_state = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
  const bool fuse = o->sched == DAIC_SCHED_ALL && sum_state && p->pull_ready &&
                    std::getenv("DAIC_NO_FUSE") == nullptr && std::getenv("DAIC_NO_GRAPH") == nullptr;
  bool fused = false;
  DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DAIC_HIP(hipStreamSynchronize(s));
  for (;;) {
    prof.recs.clear();
    prof.used = 0;
    if (fuse && !fused) {
      const Ctl& c0 = *p->h_ctl;
      if (!c0.done && !c0.stop && c0.pull && c0.rounds < max_rounds) {
        ops.fuse_prime(p, o, s, &prof);
        fused = true;
      }
    }
    if (fused) ops.fused_round(p, s, &prof);
    else ops.round(p, o, s, nullptr, &prof);
    DAIC_HIP(hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DAIC_HIP(hipStreamSynchronize(s));
    const Ctl c = *p->h_ctl;
    for (auto& r : prof.recs) {
      float ms = 0.f;
      DAIC_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      total_ms += ms;
      // kernels of the other direction return at once: not counted as
      // launches (after a dense round, k_pull_finish takes the residual's part)
      const bool is_push = !std::strncmp(r.name, "push_", 5), is_pull = !std::strncmp(r.name, "pull_", 5);
      const bool is_res = !std::strcmp(r.name, "residual");
      if ((is_push && c.last_pull) || (is_pull && !c.last_pull) || (is_res && c.last_pull)) continue;
      daic_kernel_time& k = slot(r.name);
      k.launches += 1;
      k.total_ms += ms;
      k.alg_bytes += kernel_bytes(p, r.name, c);
      if (!std::strcmp(r.name, "push_edges")) k.edges += (double)c.round_pushed;
      if (!std::strcmp(r.name, "pull_stream") || !std::strcmp(r.name, "pull_fused") || !std::strcmp(r.name, "tile_pull") ||
          !std::strcmp(r.name, "pull_tile"))
        k.edges += (double)p->g->dev.m;
    }
    if (c.done || c.stop) break;
  }
  ranked_leave(p, s);
  DAIC_HIP(hipStreamSynchronize(s));
  const Ctl& c = *p->h_ctl;
  for (uint32_t i = 0; i < acc.size() && i < cap; ++i) out[i] = acc[i];
  *n_out = (uint32_t)std::min<size_t>(acc.size(), cap);
  if (stats) {
    stats->rounds = c.rounds;
    stats->activations = c.activations;
    stats->pushed_edges = c.pushed;
    stats->final_residual = c.r;
    stats->time_ms = total_ms;
    stats->gteps = total_ms > 0 ? (double)c.pushed / (total_ms * 1e-3) / 1e9 : 0.0;
  }
  return c.done ? DAIC_OK : DAIC_NOT_CONVERGED;
}

daic_status daic_run_progress(daic_problem* p, const daic_run_opts* o, uint64_t max_points, uint64_t* updates,
                              double* progress, uint64_t* points, daic_stats* stats) {
  if (!p || !points || (max_points && (!updates || !progress))) return fail(DAIC_E_INVALID, "null argument");
  daic_status rc = check_opts(p, o);
  if (rc) return rc;
  if (o->sched == DAIC_SCHED_SWEEP) return fail(DAIC_E_UNSUPPORTED, "daic_run_progress takes the per-round rules, not SWEEP");
  if (o->sched == DAIC_SCHED_LEARNED) return fail(DAIC_E_UNSUPPORTED, "progress traces take the plain rules");
  apply_run_opts(p, o);
  *points = 0;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  Ops ops;
  if (!get_ops(p, &ops)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : p->own_stream;
  const uint64_t max_rounds = o->max_rounds ? o->max_rounds : ~0ull;
  rc = dense_rounds_setup(p, o, s);
  if (rc) return rc;
  double* dsum = nullptr;
  DAIC_HIP(hipMalloc(&dsum, sizeof(double)));
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, o->eps, max_rounds);
  ops.residual(p, s, 0);
  const uint32_t pg = (uint32_t)std::min<uint64_t>(2048, (n + 255) / 256);
  double sum = 0.0;
  hipError_t e = hipSuccess;
  for (;;) {
    e = hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || p->h_ctl->done || p->h_ctl->stop) break;
    ops.round(p, o, s, nullptr, nullptr);
    if (*points < max_points) {
      e = hipMemsetAsync(dsum, 0, sizeof(double), s);
      if (e != hipSuccess) break;
      switch (p->st) {
        case ST_F64: hipLaunchKernelGGL(k_progress<ST_F64>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
        case ST_F32: hipLaunchKernelGGL(k_progress<ST_F32>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
        case ST_F32K: hipLaunchKernelGGL(k_progress<ST_F32K>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
        case ST_U32: hipLaunchKernelGGL(k_progress<ST_U32>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
        case ST_F64MIN: hipLaunchKernelGGL(k_progress<ST_F64MIN>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
        default: hipLaunchKernelGGL(k_progress<ST_I32>, dim3(pg), dim3(256), 0, s, p->a, dsum); break;
      }
      e = hipMemcpyAsync(&sum, dsum, sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) break;
      updates[*points] = p->h_ctl->activations;
      progress[*points] = sum;
      ++*points;
    }
  }
  (void)hipFree(dsum);
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "progress: %s", hipGetErrorString(e));
  const Ctl& c = *p->h_ctl;
  if (stats) {
    stats->rounds = c.rounds;
    stats->activations = c.activations;
    stats->pushed_edges = c.pushed;
    stats->final_residual = c.r;
  }
  return c.done ? DAIC_OK : DAIC_NOT_CONVERGED;
}

daic_status daic_select_frontier(daic_problem* p, const daic_run_opts* o, uint64_t round, uint8_t* sel_out,
                                 double* threshold_out) {
  if (!p || !sel_out) return fail(DAIC_E_INVALID, "null argument");
  daic_status rc = check_opts(p, o);
  if (rc) return rc;
  if (o->sched == DAIC_SCHED_SWEEP) return fail(DAIC_E_UNSUPPORTED, "daic_select_frontier takes the per-round rules, not SWEEP");
  apply_run_opts(p, o);
  if (o->sched == DAIC_SCHED_LEARNED) return fail(DAIC_E_UNSUPPORTED, "select_frontier takes the plain rules");
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  Ops ops;
  if (!get_ops(p, &ops)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : p->own_stream;
  void* sel;
  DAIC_HIP(hipMalloc(&sel, n));
  p->a.sel_out = static_cast<uint8_t*>(sel);
  DAIC_HIP(hipMemsetAsync(sel, 0, n, s));
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, 0.0, ~0ull);
  ops.residual(p, s, 0);
  // the residual may declare the state finished; the selection still runs
  hipLaunchKernelGGL(k_clear_done, dim3(1), dim3(1), 0, s, p->a.ctl);
  ops.select(p, o, s, round);
  hipError_t e = hipMemcpyAsync(sel_out, sel, n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  p->a.sel_out = nullptr;
  (void)hipFree(sel);
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "select_frontier: %s", hipGetErrorString(e));
  if (threshold_out) {
    const Ctl& c = *p->h_ctl;
    uint64_t t = c.tau;
    double tv;
    if (c.sel_mode == 0) tv = 0.0;
    else if (p->st == ST_F64) { double d; std::memcpy(&d, &t, 8); tv = d; }
    else if (p->st == ST_F32 || p->st == ST_F32K) { uint32_t u = (uint32_t)t; float f; std::memcpy(&f, &u, 4); tv = f; }
    else tv = (double)t;
    *threshold_out = tv;
  }
  return DAIC_OK;
}

daic_status daic_problem_get(const daic_problem* p, void* v_out, void* dv_out) {
  if (!p || !v_out) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  DAIC_HIP(hipDeviceSynchronize());
  if (p->st == ST_F64 || p->st == ST_U32 || p->st == ST_I32 || p->st == ST_F64MIN) {
    size_t S = state_size(p->st);
    DAIC_HIP(hipMemcpy(v_out, p->a.v, n * S, hipMemcpyDeviceToHost));
    if (dv_out) DAIC_HIP(hipMemcpy(dv_out, p->a.dv, n * S, hipMemcpyDeviceToHost));
    return DAIC_OK;
  }
  std::vector<float> tv(n), tc(n, 0.0f);
  DAIC_HIP(hipMemcpy(tv.data(), p->a.v, n * 4, hipMemcpyDeviceToHost));
  if (p->a.c) DAIC_HIP(hipMemcpy(tc.data(), p->a.c, n * 4, hipMemcpyDeviceToHost));
  double* vo = static_cast<double*>(v_out);
  for (uint64_t j = 0; j < n; ++j) vo[j] = (double)tv[j] - (double)tc[j];
  if (dv_out) {
    DAIC_HIP(hipMemcpy(tv.data(), p->a.dv, n * 4, hipMemcpyDeviceToHost));
    double* d = static_cast<double*>(dv_out);
    for (uint64_t j = 0; j < n; ++j) d[j] = (double)tv[j];
  }
  return DAIC_OK;
}

void daic_problem_destroy(daic_problem* p) {
  if (!p) return;
  sweep_release(p);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->exec_fused) (void)hipGraphExecDestroy(p->exec_fused);
  if (p->graph_fused) (void)hipGraphDestroy(p->graph_fused);
  for (void* q : p->allocs) dfree(q);
  if (p->h_ctl) (void)hipHostFree(p->h_ctl);
  if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  delete p;
}

}  // extern "C"
