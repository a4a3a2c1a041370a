/*
 * daic.h -- C ABI of libdaic, an MI355X (gfx950) implementation of the
 * per-round delta propagation of delta-based accumulative iterative
 * computation (DAIC).
 *
 * Method: Zhang, Gao, Gao, Wang, "Maiter: An Asynchronous Graph Processing
 * Framework for Delta-based Accumulative Iterative Computation".
 *   - A problem is the tuple (g_{j,k}, (+), v^0, dv^1) of Sec. 3.1 and Table 1:
 *     an operator (+) that is commutative and associative with an identity 0
 *     (third condition; identity property in Sec. 3.2), a per-edge function g
 *     distributive over (+) (second condition), and initial values that meet
 *     the fourth condition v^0 (+) dv^1 = f(v^0).
 *   - One round applies the asynchronous update of Eq. async (Sec. 3.2) to the
 *     vertices chosen by priority |v_j (+) dv_j - v_j| (Sec. 3.5):
 *        delta = dv_j;  dv_j = 0;  v_j = v_j (+) delta;
 *        for every out-edge (j,k): dv_k = dv_k (+) g_{j,k}(delta)   [skip if = 0]
 *     The chosen set is the top portion q of the state table (Sec. 5.1,
 *     priority queue), found exactly or by sampling.
 *   - The run stops when the pending residual falls to eps (sum problems) or
 *     when no vertex is pending (min/max problems); cf. the termination check
 *     of Sec. 5.1 and Sec. 6.1.3.
 *
 * The three calls of the paper's API (Sec. 5.2) map as follows: the
 * Partitioner's input parsing is the CSR load (daic_graph_create*), the
 * IterateKernel's init/accumulate/send are set by daic_problem_create (op, g)
 * and daic_problem_set_init, and the TermChecker is the residual threshold of
 * daic_run_opts.
 *
 * Conventions
 *   - Status: 0 = success; 1 = DAIC_NOT_CONVERGED (a warning, the state is
 *     valid); negative = failure, in which case no output buffer is written.
 *     daic_last_error() returns a thread-local message for the last failure.
 *   - Ownership: host arrays passed in are copied; the caller keeps them.
 *     daic_graph_create_device borrows device pointers that must outlive the
 *     graph handle. Handles are released by the matching *_destroy call.
 *   - Threads: calls on one handle must not run concurrently; distinct handles
 *     are independent.
 *   - CSR: row_ptr[n+1] (uint64, monotone, row_ptr[0] = 0, row_ptr[n] = m),
 *     col[m] (uint32, every entry < n). Each entry is one edge: duplicates and
 *     self-loops are kept and count towards the out-degree.
 */
#ifndef DAIC_H
#define DAIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DAIC_OK = 0,
  DAIC_NOT_CONVERGED = 1, /* max_rounds reached; state valid, stats filled */
  DAIC_E_INVALID = -1,    /* bad argument (message in daic_last_error)     */
  DAIC_E_UNSUPPORTED = -2,/* (+)/g/dtype combination not offered           */
  DAIC_E_OOM = -3,        /* device allocation failed                      */
  DAIC_E_DEVICE = -4      /* HIP runtime error                             */
} daic_status;

/* The accumulation operator (+) (Sec. 3.1, third condition) and its identity
 * 0: 0 for SUM, infinity for MIN (0xFFFFFFFF in U32 state, +inf in F64
 * state), -1 for MAX. */
typedef enum { DAIC_SUM = 0, DAIC_MIN = 1, DAIC_MAX = 2 } daic_op;

/* The per-edge function g_{j,k} (Table 1). a_j is alpha_per_vertex[j] when
 * given, else alpha_scalar.
 *   SRC_SCALE : g(x) = a_j * x               Katz (beta), HITS-like rows
 *   DEG_SCALE : g(x) = alpha * x / outdeg_j  PageRank (d / |N(j)|, sender degree)
 *   EDGE_SCALE: g(x) = a_j * w_jk * x        Adsorption, weighted linear sums
 *   EDGE_ADD  : g(x) = x + w_jk              SSSP (U32: saturating at infinity)
 *   COPY      : g(x) = x                     connected components            */
typedef enum {
  DAIC_G_SRC_SCALE = 0,
  DAIC_G_EDGE_SCALE = 1,
  DAIC_G_EDGE_ADD = 2,
  DAIC_G_COPY = 3,
  DAIC_G_DEG_SCALE = 4
} daic_g;

/* Element types. F32_KAHAN keeps v in FP32 with a compensation term (Kahan
 * summation); deltas and pushes are FP32 and the residual is reduced in FP64. */
typedef enum {
  DAIC_F64 = 0,
  DAIC_F32 = 1,
  DAIC_F32_KAHAN = 2,
  DAIC_U32 = 3,
  DAIC_I32 = 4,
  DAIC_NONE = 5
} daic_dtype;

/* Selection rule of a round (Sec. 3.5 priority scheduling, Sec. 5.1 queue).
 *   ALL          : every pending vertex (a synchronous DAIC round, Eq. sync)
 *   TOPK_EXACT   : the ceil(q n) largest priorities, ties to the smaller id
 *   TOPK_SAMPLED : threshold = ceil(q S)-th largest of S sampled priorities
 *   LEARNED      : top ceil(q n) by priority x sigmoid(network score)
 *   ROUND_ROBIN  : the pending vertices of the next block of ceil(q n)
 *                  consecutive ids, blocks taken cyclically (static order,
 *                  Sec. 5.1 round-robin scheduling)
 *   SWEEP        : round-robin over blocks of ceil(q n) consecutive ids
 *                  (block c holds ids [c B, (c + 1) B)), every pending vertex
 *                  of the block updated, each block receiving by a pull over
 *                  its in-edges the latest message of every in-neighbour, so
 *                  that blocks later in a sweep already see the updates made
 *                  earlier in it (an asynchronous activation order, Eq. async;
 *                  q = 1 is the synchronous round). Sum problems on graphs with
 *                  n, m < 2^31. A round is one block; the stop rule is checked
 *                  after whole sweeps, on an upper bound of the residual (exact
 *                  for non-negative messages); the run ends by delivering the
 *                  messages still in flight, so the final state and residual
 *                  are the ordinary (v, dv) ones.                            */
typedef enum {
  DAIC_SCHED_ALL = 0,
  DAIC_SCHED_TOPK_EXACT = 1,
  DAIC_SCHED_TOPK_SAMPLED = 2,
  DAIC_SCHED_LEARNED = 3,
  DAIC_SCHED_ROUND_ROBIN = 4,
  DAIC_SCHED_SWEEP = 5
} daic_sched;

typedef struct daic_graph daic_graph;
typedef struct daic_problem daic_problem;
typedef struct daic_batch daic_batch;
typedef struct daic_trace daic_trace;
typedef struct daic_sched_model daic_sched_model;

typedef struct {
  double eps;                 /* stop when the residual <= eps (sum problems)  */
  double priority_fraction;   /* q in (0, 1]; portion of the state table      */
  daic_sched sched;           /* selection rule                                */
  uint64_t max_rounds;        /* DAIC_NOT_CONVERGED once reached               */
  uint32_t rounds_per_check;  /* rounds per host check of the residual (>= 1)  */
  uint32_t n_samples;         /* S for TOPK_SAMPLED (0 = 4096; max 4096)       */
  uint64_t seed;              /* sampling seed                                 */
  void* hip_stream;           /* hipStream_t to run on (NULL = default stream) */
  const daic_sched_model* model; /* network for DAIC_SCHED_LEARNED           */
} daic_run_opts;

typedef struct {
  uint64_t rounds;            /* rounds that did work                          */
  uint64_t activations;       /* vertex updates performed                      */
  uint64_t pushed_edges;      /* messages sent (out-edges of updated vertices) */
  double final_residual;      /* sum |dv| (sum) or pending count (min/max)     */
  double time_ms;             /* device time of the round loop                 */
  double gteps;               /* pushed_edges / time / 1e9                     */
  double alg_bytes;           /* algorithmic bytes moved by the round loop     */
  uint64_t learned_exact_rounds; /* LEARNED: rounds taken by exact top-k       */
  uint64_t learned_fallbacks; /* LEARNED: times the judge handed the next rounds
                                 back to exact selection                       */
} daic_stats;

/* ---- Graphs --------------------------------------------------------------
 * daic_graph_create: host CSR, copied to the device. w may be NULL (w_type
 * DAIC_NONE) or hold m weights of type w_type (F64, F32 or U32).
 * daic_graph_create_device: the same arrays already on the device (e.g. torch
 * tensors); they are borrowed, not copied, and validated on the device.   */
daic_status daic_graph_create(uint64_t n, uint64_t m, const uint64_t* row_ptr, const uint32_t* col,
                              const void* w, daic_dtype w_type, daic_graph** out);
daic_status daic_graph_create_device(uint64_t n, uint64_t m, const uint64_t* d_row_ptr,
                                     const uint32_t* d_col, const void* d_w, daic_dtype w_type,
                                     void* hip_stream, daic_graph** out);
void daic_graph_destroy(daic_graph* g);

/* ---- Problems ------------------------------------------------------------
 * Allowed combinations (second and third conditions):
 *   SUM x {SRC_SCALE, DEG_SCALE, EDGE_SCALE} x {F64, F32, F32_KAHAN}
 *   MIN x EDGE_ADD x U32 (weights U32)      MAX x COPY x I32
 *   MIN x EDGE_ADD x F64 (real weights, Sec. 6.1.2's log-normal SSSP; the
 *     weights, of any stored type, must be >= 0 and not NaN, else
 *     DAIC_E_INVALID)
 * alpha_per_vertex: NULL or n doubles (SRC_SCALE and EDGE_SCALE only).
 * The new problem holds v = 0 and dv = 0 (identity); call set_init.       */
daic_status daic_problem_create(const daic_graph* g, daic_op op, daic_g gk, double alpha_scalar,
                                const double* alpha_per_vertex, daic_dtype state,
                                daic_problem** out);
/* v0, dv1: n host values each, typed double for FP states, uint32 for U32,
 * int32 for I32. The fourth condition v0 (+) dv1 = f(v0) is the caller's. */
daic_status daic_problem_set_init(daic_problem* p, const void* v0, const void* dv1);
/* The same from device arrays (borrowed only for the call) in the state's
 * element type: double (F64), float (F32, F32_KAHAN; the compensation is
 * cleared), uint32 (U32), int32 (I32). Enqueued on hip_stream; with a NULL
 * stream the call returns after the copy. */
daic_status daic_problem_set_init_device(daic_problem* p, const void* d_v0, const void* d_dv1,
                                         void* hip_stream);
/* Run rounds until the stop rule holds (DAIC_OK) or max_rounds (warning).
 * A round whose messages reach most of the graph runs as a pull over the
 * in-edges (Eq. sync read per receiver; the same state as the pushes): sum
 * problems when at least n/32 vertices update (env DAIC_PULL_DIV sets 32),
 * min and max problems when the pending vertices' out-edges reach m/4
 * (DAIC_PULL_EDGE_DIV sets 4); DAIC_NO_PULL=1 always pushes. Under
 * DAIC_SCHED_ALL sum rounds fuse the next round's claim into the pull
 * (DAIC_NO_FUSE=1 keeps them apart, and so does DAIC_NO_GRAPH=1, which
 * launches every round eagerly instead of replaying captured groups). The pulls walk the in-edges in
 * partition tiles built once per graph (fused rounds and the sweep's block
 * pulls: with targets numbered by in-degree octave, highest first and ids
 * ascending within an octave, within each id block for the sweep, the state
 * moved into that order while they run and back before daic_run returns;
 * DAIC_TILE_ID_ORDER=1 keeps partitions of consecutive ids for them too;
 * DAIC_NO_TILE=1 keeps the streamed
 * pull for sum problems and pushes for min/max; DAIC_TILE_EDGES and
 * DAIC_TILE_BITS, read when a graph's tiles are built, set the in-edges per
 * tile and the partition width 2^bits; the sweep schedule's tiles take
 * DAIC_SWEEP_TILE_EDGES, DAIC_SWEEP_TILE_BITS and DAIC_SWEEP_TILE_SHARE,
 * the divisor of a block's in-edges that sizes its tiles). Every form
 * ends in the same state after the same rounds (min/max bit for bit, sums up
 * to the order of their FP additions). */
daic_status daic_run(daic_problem* p, const daic_run_opts* opts, daic_stats* stats);
/* Copy the state out: v_out (n values; double for FP states, where F32_KAHAN
 * reports v - c in FP64), dv_out nullable (same type). */
daic_status daic_problem_get(const daic_problem* p, void* v_out, void* dv_out);
void daic_problem_destroy(daic_problem* p);

/* ---- Fourth condition (Sec. 3.1) -----------------------------------------
 * The initial values must satisfy v0_j (+) dv1_j = f(v0)_j, with f the
 * update function of Eq. decompose: f(v)_j = (+)_{i->j} g_{i,j}(v_i) (+) c_j.
 * The library is given (g, (+), v0, dv1) but not c, so the check needs it:
 * daic_problem_set_const copies c (n host values: double for FP states,
 * uint32 for U32, int32 for I32). daic_problem_check_init then checks the
 * problem's current state on the device (the identity also holds at every
 * state a run leaves, since all messages are then delivered): exact for
 * min/max problems; for sum problems |lhs - rhs| <= tol x (s_j + mean_k s_k)
 * with s_j = |c_j| + sum of |g_ij(v_i)| + |v_j| + |dv_j| (the mean is a floor
 * for vertices whose terms cancel), tol 0 meaning 1e-12 (F64) or 1e-5 (FP32
 * states). It returns DAIC_E_INVALID when some vertex fails (count in
 * *mismatches, nullable; first vertex in daic_last_error) and also when no
 * constant was given. With the environment variable DAIC_CHECK_INIT set,
 * daic_run performs this check on its starting state first and returns its
 * failure without running. The check allocates device scratch per call (a
 * debug path).                                                              */
daic_status daic_problem_set_const(daic_problem* p, const void* c);
daic_status daic_problem_check_init(daic_problem* p, double tol, uint64_t* mismatches);

/* ---- Checkpoint / resume (the snapshots of the state table of Sec. 5.1) ---
 * daic_problem_save writes the problem's state (v, dv and, for F32_KAHAN,
 * the compensation term, all bit-exact) into buf; with buf NULL it writes
 * the size needed to *len, and with *len too small it fails (DAIC_E_INVALID,
 * size needed in *len). Layout, little-endian: "DAICPRB1", uint32 version 1,
 * uint32 state type, uint64 n, uint64 m, uint32 op, uint32 g kind, double
 * alpha, uint64 payload bytes, then v[n], dv[n] in the device element type
 * (8 bytes for F64 states, 4 otherwise) and c[n] (FP32, F32_KAHAN only).
 * daic_problem_load restores such a buffer into a problem of the same kind
 * (op, g, state type, alpha, n, m; anything else is DAIC_E_INVALID). A state
 * saved after daic_run (which returns with every message delivered, also at
 * max_rounds) resumes the same computation: the next daic_run continues it. */
daic_status daic_problem_save(const daic_problem* p, void* buf, size_t* len);
daic_status daic_problem_load(daic_problem* p, const void* buf, size_t len);

const char* daic_last_error(void);

/* ---- Device-side round pieces, exposed for unit tests --------------------
 * daic_select_frontier runs the selection of one round on the current state
 * without updating it and writes the 0/1 selection of every vertex to
 * sel_out (n host bytes). threshold_out (nullable) receives the threshold as
 * a double. round selects the sample stream of TOPK_SAMPLED.              */
daic_status daic_select_frontier(daic_problem* p, const daic_run_opts* opts, uint64_t round,
                                 uint8_t* sel_out, double* threshold_out);
/* daic_select_frontier for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection (opts: sched ALL, TOPK_EXACT, TOPK_SAMPLED or ROUND_ROBIN,
 * priority_fraction, n_samples <= 4096, seed; round picks the sample stream)
 * on caller device arrays d_v, d_dv (n values of the state's device element
 * type: double for F64, float for F32 and F32_KAHAN, uint32 for U32, int32
 * for I32; op and state as daic_problem_create takes them), written to
 * caller device arrays: d_sel_out (n bytes, 0/1) and d_threshold_out
 * (nullable, one double: the threshold, 0 when every pending vertex is
 * taken). Inputs are only read. It allocates nothing and does not
 * synchronize: kernels are enqueued on opts->hip_stream (NULL = default
 * stream) and the call returns. Its scratch (control block, radix
 * histograms, sampled keys, per-block partials: under 160 KiB, the same for every
 * n up to the maximum n < 2^32 - 1) is one fixed array per device that every
 * call on that device shares and overwrites, so calls that overlap on one
 * device (other streams, other threads) race and must be serialized by the
 * caller. Errors (DAIC_E_INVALID, DAIC_E_UNSUPPORTED) are returned before
 * anything is enqueued. */
daic_status daic_select_frontier_noalloc(daic_op op, daic_dtype state, uint64_t n, const void* d_v,
                                         const void* d_dv, const daic_run_opts* opts, uint64_t round,
                                         uint8_t* d_sel_out, double* d_threshold_out);

/* ---- Batched personalized PageRank --------------------------------------
 * Many graphs of uneven size, each with up to 64 right-hand sides (the
 * Rooted PageRank row of Table 1 read with damping: g(x) = alpha x / outdeg_j,
 * dv1 = (1 - alpha) p for a personalization vector p). All graphs are solved
 * together: every kernel of a round covers every graph, and K rounds are one
 * hipGraph launch. Each instance (graph, right-hand side) has its own
 * residual and stop flag; a run ends when every instance has residual <= eps.
 * op must be DAIC_SUM with DAIC_G_DEG_SCALE, or with DAIC_G_EDGE_SCALE
 * (g(x) = alpha w_jk x; every graph with edges must carry weights; e.g.
 * multi-label Adsorption with one label per right-hand side and the
 * receiver's continuation probability folded into w); state DAIC_F32 or
 * F32_KAHAN.
 * The graphs are copied into one block-diagonal graph; they may be destroyed
 * after the call. Dense rounds pull targets of in-degree above a threshold
 * (64; env DAIC_HUB_DEG, read here) in chunks of in-edges of their own.        */
daic_status daic_batch_create(uint32_t n_graphs, const daic_graph* const* graphs,
                              const uint32_t* rhs_per_graph, daic_op op, daic_g gk, double alpha,
                              daic_dtype state, daic_batch** out);
/* v0, dv1: host arrays [n_g][rhs_g] (row-major, vertex-major) in double. */
daic_status daic_batch_set_init(daic_batch* b, uint32_t graph, const double* v0, const double* dv1);
/* Autotuner: times the claim kernel and the dense round (hub sums and fused
 * pass) for each lanes-per-vertex and grid size on the current state
 * (restored afterwards, finish flags included) and keeps the fastest; with
 * DAIC_TUNE_CACHE set, results are cached in that file. desc receives a
 * description of the choice (nullable). */
daic_status daic_batch_tune(daic_batch* b, char* desc, size_t desc_len);
/* Run every instance to residual <= eps: sched ALL (q = 1; synchronous dense
 * rounds) or SWEEP (dense rounds take blocks of ceil(q n_g) vertices of
 * every graph in turn, each pulling the newest message of every
 * in-neighbour; one round is one block). inst_residual
 * (nullable) receives the final residual of every instance, graph-major.
 * stats->final_residual is the largest instance residual. Instances are
 * updated until the check after the round in which their residual fell to
 * eps, so they may end below eps; a run stopped by max_rounds returns
 * DAIC_NOT_CONVERGED with every message delivered (a later run resumes).
 * opts->rounds_per_check rounds are one graph launch between host checks;
 * 0 means 128, so that a whole solve of up to 128 rounds is one launch
 * (rounds after every instance finished return at once). */
daic_status daic_batch_run(daic_batch* b, const daic_run_opts* opts, daic_stats* stats,
                           double* inst_residual);
/* v_out: [n_g][rhs_g] doubles (FP32 state; with Kahan, v - c). */
daic_status daic_batch_get(const daic_batch* b, uint32_t graph, double* v_out);
/* The state of one graph's instances, each output nullable: v_out and dv_out
 * [n_g][rhs_g] doubles, done_out [rhs_g] finish states (0 running, 1
 * finished with its last messages in flight, 2 finished and delivered). */
daic_status daic_batch_get_state(const daic_batch* b, uint32_t graph, double* v_out, double* dv_out,
                                 uint8_t* done_out);
/* Snapshot of the whole batch for checkpoint and resume, bit-exact, with the
 * size protocol of daic_problem_save. Layout, little-endian: "DAICBAT1",
 * uint32 version 1, uint32 G, uint64 N (union vertices), uint32 Kahan flag,
 * uint32 weighted flag, double alpha, uint64 payload bytes; per graph uint64
 * n_g, uint32 rhs_g, uint32 0; then v, dv and (Kahan) c as [N][64] FP32 and
 * the finish states [G][64] uint8. daic_batch_load restores it into a batch
 * built from graphs of the same sizes with the same right-hand-side counts,
 * state type, weights flag and alpha. A batch run stopped by max_rounds ends
 * with every message delivered, so a saved state resumes with
 * daic_batch_run. */
daic_status daic_batch_save(const daic_batch* b, void* buf, size_t* len);
daic_status daic_batch_load(daic_batch* b, const void* buf, size_t len);
void daic_batch_destroy(daic_batch* b);

/* ---- Learned scheduler ----------------------------------------------------
 * A 3 -> 64 -> 64 -> 1 network (ReLU, logit output) scoring pending vertices
 * from the features [log2(priority), log2((1 + indeg) / (1 + outdeg)),
 * min(rounds since the last update, 64) / 64], standardized by the model's
 * feature mean and scale. Under DAIC_SCHED_LEARNED a round takes the top
 * ceil(q n) vertices by priority x sigmoid(score); the exact top-k round is its
 * fallback and the residual remains the stop rule. Not part of the paper: an
 * addition that changes the update order only, which Theorems 1 and 3 allow.
 * The exact rounds and the judge: a learned run starts with one exact top-k
 * round; each round's realized priority per message (the sum of
 * |v (+) dv - v| over the vertices it updated, divided by the messages it
 * sent, and for sum problems also by the residual at the round's start) is
 * compared on the device with the last exact round's; a learned round below
 * 0.8 x that figure hands the next 4 rounds back to exact selection, and
 * every 16 learned rounds are followed by one exact round. Learned rounds are captured in graphs like the others
 * (rounds_per_check rounds per launch).
 * Parameters: 4481 FP32 values, [W1 (64x3), b1 (64), W2 (64x64), b2 (64),
 * W3 (1x64), b3 (1)], row-major (output, input). The device keeps FP32
 * master weights and BF16 copies for the MFMA kernels.                     */
daic_status daic_sched_model_create(const float* params /* nullable: seeded init */, uint64_t seed,
                                    daic_sched_model** out);
daic_status daic_sched_model_get(const daic_sched_model* m, float* params /* 4481 */,
                                 float* feat_mean /* 3, nullable */, float* feat_std /* 3, nullable */);
daic_status daic_sched_model_set_features(daic_sched_model* m, const float* feat_mean,
                                          const float* feat_std);
void daic_sched_destroy(daic_sched_model* m);
/* Forward (logits) and gradient of the mean BCE-with-logits loss on host
 * inputs x [N][3] (already standardized) and labels y [N] in {0, 1}, on the
 * BF16 MFMA kernels: for checking against a reference. grad: 4481 floats. */
daic_status daic_mlp_forward(const daic_sched_model* m, const float* x, uint64_t N, float* logits);
/* The scoring kernel of a learned round, exposed for unit tests: on the
 * problem's current state at round 0 with no vertex updated yet (so every
 * vertex is one round past its last update, counted at round -1),
 * writes each vertex's selection multiplier to score_out (n host floats):
 * sigmoid(logit) of its standardized features for pending vertices, 0 for
 * the others. The problem's state is not changed.                          */
daic_status daic_sched_score(daic_problem* p, const daic_sched_model* m, float* score_out);
daic_status daic_mlp_grad(const daic_sched_model* m, const float* x, const float* y, uint64_t N,
                          float* grad, double* loss /* nullable */);

/* Trace capture: runs exact top-k rounds (opts->sched = TOPK_EXACT, the
 * priority scheduling of Sec. 3.5) from the problem's current state to its
 * stop rule (or max_rounds, at most 4096). In round t, S = samples_per_round
 * vertices are drawn before the round (sample i is output t S + i of
 * SplitMix64 seeded with opts->seed XOR 0x7A3E5C91, mod n) with their raw
 * features at that moment; a vertex never updated counts as last updated in
 * round -1. A sampled vertex that was pending and is updated by round t
 * becomes one training sample (once per draw): its features and label 1, or
 * 0 when the update was premature: at the start of one of the next `horizon`
 * rounds (the state after the last round standing for every later start) its
 * priority reached half its priority at t (sum problems) or it was pending
 * again (min/max problems). Samples of the last `horizon` rounds are dropped
 * unless the run ended converged. Samples are ordered by round, then draw.
 * The problem ends converged (or at max_rounds). samples_per_round in
 * 1..2^20, horizon in 1..64.                                                  */
daic_status daic_trace_record(daic_problem* p, const daic_run_opts* opts, uint32_t samples_per_round,
                              uint32_t horizon, daic_trace** out);
/* Copies the samples out: x [n][3] raw features, y [n]; *n = sample count.
 * x and y may be NULL to query n. */
daic_status daic_trace_get(const daic_trace* tr, float* x, float* y, uint64_t* n);
/* Vertex and round of each sample of a recorded trace (n of each; NULL to
 * query n; a trace made by daic_trace_create has none: *n = 0). */
daic_status daic_trace_samples(const daic_trace* tr, uint32_t* vid, uint32_t* round, uint64_t* n);
/* A trace from caller samples: x [n][3] raw features (finite), y [n] labels in
 * {0, 1}; both copied. For training on samples gathered elsewhere. */
daic_status daic_trace_create(const float* x, const float* y, uint64_t n, daic_trace** out);
void daic_trace_destroy(daic_trace* tr);

typedef struct {
  uint32_t epochs;   /* passes over the samples (0 = 10)      */
  uint32_t batch;    /* minibatch size (0 = 65536)            */
  float lr;          /* Adam step size (0 = 1e-3)             */
  uint64_t seed;     /* shuffle seed                          */
} daic_train_opts;
typedef struct {
  uint64_t samples;
  double positive_fraction;
  double loss_first;  /* mean loss before training  */
  double loss_final;  /* mean loss after training   */
  double time_ms;     /* device time of the epochs  */
  uint32_t epochs;
} daic_train_stats;
/* Trains m on the union of the traces on the device (BF16 MFMA gradients,
 * FP32 Adam); sets the model's feature standardization from the samples
 * (mean and population standard deviation in FP64, kept as FP32, scale at
 * least 1e-6), shuffles them with a seeded Fisher-Yates and takes minibatch
 * steps as daic_sched_step does. */
daic_status daic_sched_train(const daic_trace* const* traces, uint32_t n_traces,
                             const daic_train_opts* opts, daic_sched_model* m,
                             daic_train_stats* stats);
/* One training step of m on host samples x [N][3] (already standardized) and
 * labels y [N]: the gradient of the mean BCE-with-logits loss on the BF16
 * MFMA kernels, then one Adam step (Kingma and Ba 2015; beta1 0.9, beta2
 * 0.999, eps 1e-8, bias-corrected, FP32 moments and master weights; the step
 * count is kept in the model). grad_out (nullable, 4481 floats) receives the
 * gradient applied, loss (nullable) the mean loss before the step. Exposed
 * for checking the trainer against a reference. */
daic_status daic_sched_step(daic_sched_model* m, const float* x, const float* y, uint64_t N, float lr,
                            float* grad_out, double* loss);
/* Serialization of a model: FP32 master weights, both Adam moments, the Adam
 * step count and the feature standardization, in a versioned little-endian
 * buffer ("DAICSCH1", version 1, 53,820 bytes). daic_sched_save with buf NULL
 * writes the size to *len; with *len too small it fails (DAIC_E_INVALID) and
 * writes the size needed. daic_sched_load checks the magic, version, size and
 * that every value is finite (scales positive) and makes a new model. */
daic_status daic_sched_save(const daic_sched_model* m, void* buf, size_t* len);
daic_status daic_sched_load(const void* buf, size_t len, daic_sched_model** out);

/* Progress trace for update-count studies (Sec. 6.3): runs like daic_run,
 * one round at a time, and after every round records the cumulative number
 * of vertex updates and the progress metric sum_j v_j (sum problems: in
 * FP64; min problems: over finite values; max problems: over all values).
 * At most max_points rounds are recorded; *points receives the count. */
daic_status daic_run_progress(daic_problem* p, const daic_run_opts* opts, uint64_t max_points,
                              uint64_t* updates, double* progress, uint64_t* points,
                              daic_stats* stats);

/* daic_profile runs like daic_run but launches every kernel on its own,
 * bracketed by HIP events on the run's stream, one round at a time, and
 * reports per kernel class: launches, summed duration and the algorithmic
 * bytes those launches had to move (per-edge and per-vertex figures of the
 * round's actual work). At most cap classes are written; *n_out receives
 * the count. Slower than daic_run (one host sync per round).             */
typedef struct {
  char name[32];
  uint64_t launches;
  double total_ms;
  double alg_bytes;
  double edges;
} daic_kernel_time;
daic_status daic_profile(daic_problem* p, const daic_run_opts* opts, uint32_t cap,
                         daic_kernel_time* out, uint32_t* n_out, daic_stats* stats);

/* The tile table that dense rounds build over the partition-tiled in-edges
 * (the synchronous pull of Eq. sync, walked partition by partition), computed
 * on the host alone and exposed for unit tests of its invariants; no device
 * is touched. Input: pstart[p], the first in-edge of partition p in the
 * sorted in-edge order (n_part + 1 host entries, non-decreasing, the last
 * one the in-edge count, below 2^31), and the partition width 2^lb (lb in
 * 8..14). Every partition gets at least one tile; one with more in-edges
 * than its cap is cut into cap-sized tiles and a remainder, numbered in
 * order and given consecutive partial-sum slots. The cap is max_edges (at
 * least 1,024), or with share_div > 0 the in-edges of each group of
 * group_parts consecutive partitions (all partitions when 0) divided by
 * share_div (at least 1,024; under max_edges when both are given).
 * Outputs, host arrays of cap entries each: tile_part[t] (partition of tile
 * t), tile_e (n_tiles + 1 entries; tile t holds in-edges [tile_e[t],
 * tile_e[t + 1])), tile_slot[t] (0xFFFFFFFF for the single tile of an
 * unsplit partition) and order (the launch order: within each group the
 * tiles by work, largest first, ties in tile order; work = in-edges, plus
 * 2 * 2^lb for an unsplit partition, whose targets the tile finishes).
 * *n_tiles, *n_split (partitions with several tiles) and *n_slots are
 * written even when cap < n_tiles + 1, which returns DAIC_E_INVALID.      */
daic_status daic_tile_table(const uint32_t* pstart, uint64_t n_part, uint32_t lb, uint64_t max_edges,
                            uint64_t group_parts, uint32_t share_div, uint64_t cap, uint32_t* tile_part,
                            uint32_t* tile_e, uint32_t* tile_slot, uint32_t* order, uint64_t* n_tiles,
                            uint64_t* n_split, uint64_t* n_slots);

#ifdef __cplusplus
}
#endif
#endif /* DAIC_H */
