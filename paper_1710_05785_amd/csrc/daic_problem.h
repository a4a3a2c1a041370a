// The problem object and the per-instantiation enqueue table, shared by the
// runtime and the learned scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "daic_internal.h"
#include "daic_kernels.h"
#include "daic_tile.h"

namespace daic {
struct SweepState;  // per-problem state of SWEEP scheduling (built on first use)
}

// ---------------------------------------------------------------------------
// Problem object.
// ---------------------------------------------------------------------------
struct GraphCacheKey {
  int sched = -1;
  uint64_t k = 0;
  uint32_t S = 0;
  double q = 0.0;
  uint64_t seed = 0;
  uint32_t K = 0;
  const void* stream = nullptr;
  const float* score = nullptr;
  const void* model = nullptr;   // learned rounds: the network and its version (weights,
  uint64_t model_version = 0;    // feature scales and BF16 copies captured by the graph)
  uint64_t k_sel = 0, pull_min = 0;
  bool operator==(const GraphCacheKey& o) const {
    return sched == o.sched && k == o.k && S == o.S && q == o.q && seed == o.seed && K == o.K &&
           stream == o.stream && score == o.score && k_sel == o.k_sel && pull_min == o.pull_min &&
           model == o.model && model_version == o.model_version;
  }
};

struct daic_problem {
  const daic_graph* g = nullptr;
  daic_op op = DAIC_SUM;
  daic_g gk = DAIC_G_SRC_SCALE;
  daic_dtype state = DAIC_F64;
  int st = daic::ST_F64;
  double alpha = 0.0;
  daic::KArgs a{};
  void* alpha_pv = nullptr;
  void* w_conv = nullptr;
  daic::Ctl* h_ctl = nullptr;   // pinned mirror
  hipStream_t own_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec_fused = nullptr;  // K fused dense rounds
  hipGraph_t graph_fused = nullptr;
  uint32_t fused_K = 0;
  hipStream_t fused_stream = nullptr;
  GraphCacheKey key;
  std::vector<void*> allocs;
  bool pull_ready = false;
  uint64_t stream_grid = 16384;  // workgroups of k_pull_stream
  // tiled fused dense rounds (the graph's TileGraph plus per-problem buffers)
  bool tile_ready = false;
  double* tile_pbuf = nullptr;   // partial-sum slots of split partitions
  void* tile_w = nullptr;        // weights in tile order (EDGE_SCALE)
  double* tpart_r = nullptr;     // per-workgroup partials of k_tile_pull / k_tile_finish
  uint64_t* tpart_a = nullptr;
  uint64_t* tpart_p = nullptr;
  double* spart_r = nullptr;
  uint64_t* spart_a = nullptr;
  uint64_t* spart_p = nullptr;
  // fused dense rounds over the tiles of in-degree-numbered targets: while
  // they run (from the priming claim to the end of the run) v, dv and c live
  // in target-number order in these arrays
  bool ranked_ready = false;
  bool ranked_active = false;
  void* vP = nullptr;
  void* dvP = nullptr;
  float* cP = nullptr;
  void* alphaP = nullptr;        // per-vertex alpha in target-number order (when given)
  double* tile_pbuf_r = nullptr; // partial-sum slots of their split partitions
  void* tile_wr = nullptr;       // weights in their tile order (EDGE_SCALE)
  uint32_t tile_grid = 2048;     // workgroups of k_tile_pull (at most)
  uint32_t tfin_grid = 4096;     // workgroups of k_tile_finish (at most)
  uint64_t k_sel = 0;      // dense-round rule of the current run (see k_residual)
  uint64_t pull_min = 0;
  // learned scheduler state (allocated on first use)
  bool learned_ready = false;
  uint32_t* last_upd = nullptr;  // 1 + round of the last update of each vertex, 0 = never updated
  uint32_t* indeg = nullptr;     // in-degree of each vertex
  float* score = nullptr;        // selection multiplier of each vertex
  daic::SweepState* sweep = nullptr;
  void* cst = nullptr;           // constant c of the update function (fourth-condition check), or null
};

namespace daic {

// Per-kernel timing with HIP events recorded on the launch stream.
struct Prof {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

template <class F>
static void launch(Prof* pr, const char* name, hipStream_t s, F&& f) {
  if (!pr) {
    f();
    return;
  }
  hipEvent_t a = pr->ev(), b = pr->ev();
  (void)hipEventRecord(a, s);
  f();
  (void)hipEventRecord(b, s);
  pr->recs.push_back({name, a, b});
}

// Enqueue functions per instantiation.
struct Ops {
  void (*residual)(daic_problem*, hipStream_t, int);
  void (*round)(daic_problem*, const daic_run_opts*, hipStream_t, const float* score, Prof* pr);
  void (*select)(daic_problem*, const daic_run_opts*, hipStream_t, uint64_t round_override);
  // fused dense rounds (sum problems with the in-edge form): the claim that
  // publishes buffer A, and one fused round
  void (*fuse_prime)(daic_problem*, const daic_run_opts*, hipStream_t, Prof* pr);
  void (*fused_round)(daic_problem*, hipStream_t, Prof* pr);
};

// The enqueue table of a problem's (state, g, row width) instantiation.
bool get_ops(const daic_problem* p, Ops* out);
// Validation of run options, and the dense-round set-up of a run.
daic_status check_opts(const daic_problem* p, const daic_run_opts* o);
daic_status dense_rounds_setup(daic_problem* p, const daic_run_opts* o, hipStream_t s);
void apply_run_opts(daic_problem* p, const daic_run_opts* o);
// Fourth condition of Sec. 3.1 on the current state (needs the constant c).
daic_status check_init(daic_problem* p, double tol, uint64_t* mismatches, hipStream_t s);
// SWEEP scheduling: the run loop, and the release of its per-problem state.
daic_status sweep_run(daic_problem* p, const daic_run_opts* o, daic_stats* stats, hipStream_t s);
void sweep_release(daic_problem* p);

}  // namespace daic
