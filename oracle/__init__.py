"""CPU oracle for delta-based accumulative iterative computation (DAIC).

TEST INFRASTRUCTURE ONLY: plain, slow, obviously correct implementations of
what the GPU path computes, written from the paper (Zhang, Gao, Gao, Wang,
"Maiter: An Asynchronous Graph Processing Framework for Delta-based Accumulative
Iterative Computation"). Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the GPU library; only the seeded input generators (``daic_gen``) serve both.

Contents
--------
* ``jacobi_sum``     -- traditional synchronous iteration (Eq. concurrent in the
  form of Eq. decompose), FP64 pull over in-edges (C, OpenMP).
* ``sync_daic_sum``  -- synchronous DAIC, Eq. sync (C, one thread).
* ``async_run``      -- asynchronous DAIC, Eq. async, with priority (Sec. 3.5)
  or round-robin (Sec. 5.1) scheduling, for sum, min and max (C, one thread).
* ``sweep_blocks``   -- asynchronous DAIC in blocks of B consecutive ids taken
  round-robin, each block updated together (numpy).
* ``dijkstra``       -- SSSP distances, the min problem's textbook answer.
* ``dijkstra_f64``   -- the same for real non-negative weights (Python heap).
* ``maxlabel``       -- max-id reachability, the max problem's answer.
* ``priority``       -- |v (+) dv - v| per vertex (Sec. 3.5 and Table 1 rows).
* ``sampled_threshold`` / ``topk_exact`` -- the two selection rules of a round.
* ``mlp_*``          -- FP64 forward/backward of the scheduler network.
* ``adam_step``      -- one Adam update (Kingma and Ba 2015) in FP64.
* ``trace_exact_topk`` -- rounds of exact top-k scheduling with the learned
  scheduler's training samples: the features of sampled vertices and the
  label "not pending again within H rounds" (integer min/max problems) or
  "priority not back to half within H rounds" (sum problems, FP64) (numpy).

Parity status: every function here is pinned by tests under ``tests/`` except
the ones listed as "parity unpinned" in their docstrings.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)

OP_SUM, OP_MIN, OP_MAX = 0, 1, 2
G_SRC_SCALE, G_EDGE_SCALE, G_EDGE_ADD, G_COPY, G_DEG_SCALE = 0, 1, 2, 3, 4
SCHED_PRIORITY, SCHED_ROUND_ROBIN, SCHED_SWEEP = 0, 1, 2
INF_U32 = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle's C++ part with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        import subprocess

        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", os.path.join(_HERE, "oracle.cpp"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_jacobi_sum.argtypes = [ctypes.c_uint64, _u64p, _u32p, _f64p, ctypes.c_int,
                                       ctypes.c_double, _f64p, _f64p, _f64p, ctypes.c_double,
                                       ctypes.c_int64, ctypes.c_int, _f64p, _f64p]
        lib.orc_jacobi_sum.restype = ctypes.c_int64
        lib.orc_sync_daic_sum.argtypes = [ctypes.c_uint64, _u64p, _u32p, _f64p, ctypes.c_int,
                                          ctypes.c_double, _f64p, ctypes.c_double, ctypes.c_int64,
                                          _f64p, _f64p, _f64p]
        lib.orc_sync_daic_sum.restype = ctypes.c_int64
        lib.orc_async.argtypes = [ctypes.c_uint64, _u64p, _u32p, _f64p, _u32p, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_double, _f64p, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int64, _f64p, _f64p, _u32p, _u32p,
                                  _i32p, _i32p, _f64p, _f64p, ctypes.c_int64, ctypes.c_int64]
        lib.orc_async.restype = ctypes.c_int64
        lib.orc_dijkstra.argtypes = [ctypes.c_uint64, _u64p, _u32p, _u32p, ctypes.c_uint32, _u32p]
        lib.orc_dijkstra.restype = ctypes.c_int
        lib.orc_maxlabel.argtypes = [ctypes.c_uint64, _u64p, _u32p, _i32p]
        _lib = lib
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _csr(g):
    return (np.ascontiguousarray(g.row_ptr, dtype=np.uint64),
            np.ascontiguousarray(g.col, dtype=np.uint32))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Graph solvers (C).
# ---------------------------------------------------------------------------

def jacobi_sum(g, gkind, alpha, dv1, v0=None, w=None, alpha_pv=None, eps=1e-13,
               max_iter=100000, threads=0):
    """Traditional synchronous iteration of a linear (sum) DAIC problem.

    v^k_j = c_j + sum_{i->j} coef_ij v^{k-1}_i with c = v0 + dv1 - M^T v0 (the
    fourth condition, Sec. 3.1), until sum|v^k - v^{k-1}| <= eps.
    Returns (v, sweeps, last_diff).
    """
    rp, col = _csr(g)
    n = g.n
    dv1 = _f64(dv1)
    v0 = np.zeros(n) if v0 is None else _f64(v0)
    w, alpha_pv = _f64(w), _f64(alpha_pv)
    out = np.empty(n, dtype=np.float64)
    last = ctypes.c_double(0)
    it = _get().orc_jacobi_sum(n, _ptr(rp, _u64p), _ptr(col, _u32p), _ptr(w, _f64p), gkind,
                               alpha, _ptr(alpha_pv, _f64p), _ptr(v0, _f64p), _ptr(dv1, _f64p),
                               eps, max_iter, threads, _ptr(out, _f64p), ctypes.byref(last))
    return out, int(it), float(last.value)


def sync_daic_sum(g, gkind, alpha, v0, dv1, w=None, alpha_pv=None, eps=1e-13, max_rounds=100000):
    """Synchronous DAIC (Eq. sync). Returns (v, dv, rounds, residual)."""
    rp, col = _csr(g)
    v = np.array(v0, dtype=np.float64, copy=True)
    dv = np.array(dv1, dtype=np.float64, copy=True)
    w, alpha_pv = _f64(w), _f64(alpha_pv)
    r = ctypes.c_double(0)
    k = _get().orc_sync_daic_sum(g.n, _ptr(rp, _u64p), _ptr(col, _u32p), _ptr(w, _f64p), gkind,
                                 alpha, _ptr(alpha_pv, _f64p), eps, max_rounds, _ptr(v, _f64p),
                                 _ptr(dv, _f64p), ctypes.byref(r))
    return v, dv, int(k), float(r.value)


def async_run(g, op, gkind, v0, dv1, alpha=0.0, alpha_pv=None, w=None, sched=SCHED_PRIORITY,
              eps=1e-13, max_updates=2**62, trace_every=0, trace_len=0):
    """Asynchronous DAIC (Eq. async), one update at a time.

    Returns dict(v, dv, updates, residual, trace). For op=sum the state is
    FP64; for min it is uint32 (0xFFFFFFFF = infinity); for max int32.
    """
    rp, col = _csr(g)
    n = g.n
    lib = _get()
    trace = np.zeros(max(trace_len, 0), dtype=np.float64)
    r = ctypes.c_double(0)
    wf = wu = None
    if op == OP_SUM:
        v = np.array(v0, dtype=np.float64, copy=True)
        dv = np.array(dv1, dtype=np.float64, copy=True)
        wf = _f64(w)
        args = (_ptr(v, _f64p), _ptr(dv, _f64p), None, None, None, None)
    elif op == OP_MIN:
        v = np.array(v0, dtype=np.uint32, copy=True)
        dv = np.array(dv1, dtype=np.uint32, copy=True)
        wu = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
        args = (None, None, _ptr(v, _u32p), _ptr(dv, _u32p), None, None)
    else:
        v = np.array(v0, dtype=np.int32, copy=True)
        dv = np.array(dv1, dtype=np.int32, copy=True)
        args = (None, None, None, None, _ptr(v, _i32p), _ptr(dv, _i32p))
    upd = lib.orc_async(n, _ptr(rp, _u64p), _ptr(col, _u32p), _ptr(wf, _f64p), _ptr(wu, _u32p),
                        op, gkind, alpha, _ptr(_f64(alpha_pv), _f64p), sched, eps, max_updates,
                        *args, ctypes.byref(r), _ptr(trace, _f64p) if trace_len else None,
                        trace_len, trace_every)
    return dict(v=v, dv=dv, updates=int(upd), residual=float(r.value), trace=trace)


def sweep_blocks(g, gkind, alpha, v0, dv1, B, rounds, w=None, alpha_pv=None):
    """Asynchronous DAIC (Eq. async) under round-robin scheduling over blocks
    of B consecutive ids (Sec. 5.1): round r updates block r mod P, P =
    ceil(n / B). Updating a block takes every delta of the block at once
    (delta_j = dv_j, dv_j = 0, v_j += delta_j), then sends g_jk(delta_j) along
    every out-edge of the block into dv_k, so that later blocks see these
    messages in the same sweep and the block itself in the next one. g is
    alpha x / outdeg_j (DEG_SCALE), alpha_j x (SRC_SCALE) or alpha_j w_jk x
    (EDGE_SCALE), alpha_j = alpha_pv[j] when given. FP64; returns (v, dv).
    B = n is the synchronous round (Eq. sync); B = 1 updates one vertex at a
    time in id order."""
    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    deg = np.diff(rp)
    v = np.array(v0, dtype=np.float64, copy=True)
    dv = np.array(dv1, dtype=np.float64, copy=True)
    if gkind == G_DEG_SCALE:
        coef = np.where(deg > 0, alpha / np.maximum(deg, 1), 0.0)
    else:
        coef = np.full(n, float(alpha)) if alpha_pv is None else np.asarray(alpha_pv, dtype=np.float64)
    wv = None if w is None else np.asarray(w, dtype=np.float64)
    P = max(1, -(-n // B)) if n else 1
    for r in range(rounds):
        if n == 0:
            break
        c = r % P
        lo, hi = c * B, min(n, (c + 1) * B)
        delta = dv[lo:hi].copy()
        dv[lo:hi] = 0.0
        v[lo:hi] += delta
        e0, e1 = rp[lo], rp[hi]
        src = np.repeat(np.arange(lo, hi), deg[lo:hi])
        msg = coef[src] * delta[src - lo]
        if gkind == G_EDGE_SCALE:
            msg = msg * wv[e0:e1]
        np.add.at(dv, col[e0:e1], msg)
    return v, dv


def dijkstra(g, w, source):
    """SSSP distances (uint32, 0xFFFFFFFF = unreachable) by Dijkstra."""
    rp, col = _csr(g)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    out = np.empty(g.n, dtype=np.uint32)
    rc = _get().orc_dijkstra(g.n, _ptr(rp, _u64p), _ptr(col, _u32p), _ptr(w, _u32p), source,
                             _ptr(out, _u32p))
    if rc != 0:
        raise OverflowError("a shortest distance does not fit in 32 bits")
    return out


def dijkstra_f64(g, w, source):
    """SSSP distances with real non-negative weights (FP64, +inf =
    unreachable) by Dijkstra's algorithm with a binary heap; the distance of
    a vertex is d(u) + w(u, v) of its best settled predecessor, added once."""
    import heapq

    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    dist = np.full(n, np.inf)
    done = np.zeros(n, dtype=bool)
    dist[source] = 0.0
    heap = [(0.0, int(source))]
    while heap:
        du, u = heapq.heappop(heap)
        if done[u] or du > dist[u]:
            continue
        done[u] = True
        for e in range(rp[u], rp[u + 1]):
            k = col[e]
            nd = du + w[e]
            if nd < dist[k]:
                dist[k] = nd
                heapq.heappush(heap, (nd, int(k)))
    return dist


def maxlabel(g):
    """label_j = max({i : i reaches j} U {j}) (int32)."""
    rp, col = _csr(g)
    out = np.empty(g.n, dtype=np.int32)
    _get().orc_maxlabel(g.n, _ptr(rp, _u64p), _ptr(col, _u32p), _ptr(out, _i32p))
    return out


# ---------------------------------------------------------------------------
# Problem set-up helpers for the paper's algorithm table (Table 1).
# ---------------------------------------------------------------------------

def pagerank_init(n, d):
    """PageRank: v0 = 0, dv1 = 1 - d (Sec. 3.1, fourth condition)."""
    return np.zeros(n), np.full(n, 1.0 - d)


def sssp_init(n, source):
    """SSSP: v0 = inf, dv1 = 0 at the source, inf elsewhere (Table 1)."""
    v0 = np.full(n, INF_U32, dtype=np.uint32)
    dv1 = np.full(n, INF_U32, dtype=np.uint32)
    dv1[source] = 0
    return v0, dv1


def cc_init(n):
    """Connected components: v0 = -1, dv1_j = j (Table 1)."""
    return np.full(n, -1, dtype=np.int32), np.arange(n, dtype=np.int32)


def priority(op, v, dv):
    """Scheduling priority |v (+) dv - v| (Sec. 3.5); SSSP form d - min(d, dd)
    with inf - x taken as 0xFFFFFFFF (Sec. 4.2.1)."""
    if op == OP_SUM:
        return np.abs(np.asarray(dv, dtype=np.float64))
    if op == OP_MIN:
        v = np.asarray(v, dtype=np.uint64)
        dv = np.asarray(dv, dtype=np.uint64)
        mn = np.minimum(v, dv)
        p = v - mn
        first = (v == INF_U32) & (mn < INF_U32)
        p = np.where(v == INF_U32, np.where(first, INF_U32, 0), p)
        return p.astype(np.uint64)
    v = np.asarray(v, dtype=np.int64)
    dv = np.asarray(dv, dtype=np.int64)
    return (np.maximum(v, dv) - v).astype(np.int64)


def topk_exact(p, q):
    """Exact selection of a round: the k = ceil(q n) largest priorities, ties to
    the smaller id, restricted to pending vertices (p > 0) (Sec. 5.1, priority
    queue as a portion of the state table)."""
    p = np.asarray(p)
    n = p.shape[0]
    k = int(np.ceil(q * n))
    order = np.lexsort((np.arange(n), -p.astype(np.float64)))
    chosen = order[:k]
    return np.sort(chosen[p[chosen] > 0])


def splitmix64(seed, counters):
    """SplitMix64 outputs (Steele, Lea, Flood 2014): output number c of the
    generator seeded with `seed` is mix(seed + (c + 1) * 0x9E3779B97F4A7C15)."""
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counters, dtype=np.uint64) + np.uint64(1)) * g
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def sample_indices(n, n_samples, seed, round_no):
    """Indices sampled in a round: sample i of round t is output number
    t*S + i of SplitMix64(seed), reduced mod n."""
    c = np.uint64(round_no) * np.uint64(n_samples) + np.arange(n_samples, dtype=np.uint64)
    return (splitmix64(seed, c) % np.uint64(n)).astype(np.int64)


def sampled_threshold(p, q, n_samples, seed, round_no):
    """Sampled selection threshold (the PrIter-style O(N) extraction cited in
    Sec. 5.1): tau = the ceil(q S)-th largest of the S sampled priorities; when
    that is not positive, tau = the smallest positive priority (take all
    pending). A round selects p_j >= tau with p_j > 0."""
    p = np.asarray(p)
    idx = sample_indices(p.shape[0], n_samples, seed, round_no)
    s = np.sort(p[idx])[::-1]
    rank = max(1, int(np.ceil(q * n_samples)))
    tau = s[rank - 1]
    if not tau > 0:
        pos = p[p > 0]
        tau = pos.min() if pos.size else 0
    return tau


# ---------------------------------------------------------------------------
# Scheduler network: 3 -> 64 -> 64 -> 1, ReLU, BCE-with-logits, FP64.
# ---------------------------------------------------------------------------

def mlp_forward(params, x, rnd=None):
    """Returns (logits[N], cache). params = dict(W1[64,3], b1[64], W2[64,64],
    b2[64], W3[1,64], b3[1]); x = [N, 3]. rnd (optional) is applied to the
    hidden activations after each ReLU: a kernel that rounds them to a
    narrower type (BF16 between MFMA layers) is compared with this function
    given that rounding, so that both take their ReLU decisions on the same
    values; rnd = None is the plain FP64 network."""
    r = (lambda a: a) if rnd is None else rnd
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ params["W1"].T + params["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ params["W2"].T + params["b2"]
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ params["W3"].T + params["b3"]
    return z3[:, 0], (x, z1, h1, z2, h2)


def bce_with_logits(logits, y):
    """Mean binary cross-entropy of sigmoid(logits) against labels y."""
    z = np.asarray(logits, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def mlp_backward(params, cache, logits, y, rnd=None):
    """Gradients of the mean BCE-with-logits loss w.r.t. every parameter.
    rnd (optional) is applied to the back-propagated deltas where they enter
    a product (dZ2 before dH1 = dZ2 W2 and dW2 = dZ2^T H1; dZ1 before
    dW1 = dZ1^T X), as a kernel with BF16 product operands does; the bias
    gradients take the unrounded deltas."""
    r = (lambda a: a) if rnd is None else rnd
    x, z1, h1, z2, h2 = cache
    n = x.shape[0]
    y = np.asarray(y, dtype=np.float64)
    dz3 = (1.0 / (1.0 + np.exp(-logits)) - y)[:, None] / n          # [N,1]
    g = {"W3": dz3.T @ h2, "b3": dz3.sum(0)}
    dh2 = dz3 @ params["W3"]
    dz2 = dh2 * (z2 > 0)
    g["b2"] = dz2.sum(0)
    rdz2 = r(dz2)
    g["W2"] = rdz2.T @ h1
    dh1 = rdz2 @ params["W2"]
    dz1 = dh1 * (z1 > 0)
    g["b1"] = dz1.sum(0)
    g["W1"] = r(dz1).T @ x
    return g


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) in FP64 with bias correction:
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
    w <- w - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    t counts steps from 1. Returns (w, m, v) as new arrays."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


# Sample stream of traced rounds: SplitMix64 seeded with (seed XOR this value),
# a stream apart from the one of the sampled selection rule.
TRACE_SEED_XOR = 0x7A3E5C91


def _prio_f32(op, v, dv):
    """The priority as an FP32 number, as the learned features take it: the
    integer priority of ``priority`` rounded to FP32 (a first reach of a min
    problem counts as 0xFFFFFFFF, which rounds to 2^32)."""
    return priority(op, v, dv).astype(np.float32)


def trace_exact_topk(g, op, v0, dv1, q, samples_per_round, horizon, seed, w=None,
                     max_rounds=4096, gk=G_DEG_SCALE, alpha=0.0, alpha_pv=None, eps=0.0):
    """Rounds of exact top-k priority scheduling, recording the learned
    scheduler's training samples: on an integer problem (op = OP_MIN with
    g(x) = x + w_jk saturating at 0xFFFFFFFF, uint32 state; or OP_MAX with
    g(x) = x, int32 state) or on a sum problem in FP64 (op = OP_SUM with g of
    kind gk: DEG_SCALE alpha x / outdeg_j, SRC_SCALE a_j x, EDGE_SCALE
    a_j w_jk x, a_j = alpha_pv[j] or alpha; the run also stops when the
    residual sum |dv| is at most eps). Sec. 3.5 (priority scheduling), Eq.
    async (update); the trace rule itself is not in the paper.

    Round t (t = 0, 1, ...) runs while some vertex is pending and t <
    max_rounds:
      1. S = samples_per_round vertices are drawn: sample i is output
         t S + i of SplitMix64(seed XOR TRACE_SEED_XOR), mod n. For each its
         features at the start of the round are taken:
         [log2(p + 1e-30), log2((1 + indeg) / (1 + outdeg)),
          min(rounds since its last update, 64) / 64] in FP32, where p is the
         priority and a vertex never updated counts as updated in round -1.
      2. The round selects the k = ceil(q n) largest priorities among the
         pending vertices (ties to the smaller id; all pending when fewer),
         claims every selected delta (dv_j becomes the identity, v_j takes the
         delta when it improves v_j), then sends g_jk(delta) along every
         out-edge of each improved vertex, combined into dv_k with (+).
    A sample counts when its vertex was pending and selected in its round. Its
    label is 0 ("premature") when the vertex is pending at the start of any of
    the next `horizon` rounds (the state after the last round standing for
    every later start), else 1. Labels are given for every sampled round when
    the run ends with nothing pending, otherwise for rounds t < T - horizon.

    For sum problems the label is 0 when, at the start of one of the next
    `horizon` rounds (the final state standing for later starts), the
    vertex's priority in FP32 reaches half its FP32 priority when sampled.

    Returns dict(x [N,3] float32, y [N] float32, vid, round, value (the value
    the update stored in v), rounds T, v, dv)."""
    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    outdeg = np.diff(rp)
    indeg = np.bincount(col, minlength=n)
    S, H = int(samples_per_round), int(horizon)
    if op == OP_MIN:
        v = np.array(v0, dtype=np.uint32, copy=True)
        dv = np.array(dv1, dtype=np.uint32, copy=True)
        wu = np.asarray(w, dtype=np.uint64)
    elif op == OP_MAX:
        v = np.array(v0, dtype=np.int32, copy=True)
        dv = np.array(dv1, dtype=np.int32, copy=True)
    else:
        v = np.array(v0, dtype=np.float64, copy=True)
        dv = np.array(dv1, dtype=np.float64, copy=True)
        a = np.full(n, float(alpha)) if alpha_pv is None else np.asarray(alpha_pv, dtype=np.float64)
        if gk == G_DEG_SCALE:
            a = float(alpha) / np.maximum(outdeg, 1).astype(np.float64)
        wf = np.asarray(w, dtype=np.float64) if gk == G_EDGE_SCALE else None
    last = np.full(n, -1, dtype=np.int64)           # round of the last update, -1 = none
    k = int(np.ceil(q * n))
    f1 = np.log2((np.float32(1) + indeg.astype(np.float32)) /
                 (np.float32(1) + outdeg.astype(np.float32))).astype(np.float32)
    rec = []                                        # per round: vid, feat, p0, sel, value
    pend_hist = []                                  # pending mask at the start of each round
    pf_hist = []                                    # FP32 priorities at the start of each round (sum)
    t = 0
    while t < max_rounds:
        p = priority(op, v, dv)
        pending = p > 0
        if not pending.any() or (op == OP_SUM and p.sum() <= eps):
            break
        pend_hist.append(pending.copy())
        if op == OP_SUM:
            pf_hist.append(np.where(pending, _prio_f32(op, v, dv), np.float32(0)))
        # 1. samples and their features
        c = np.uint64(t) * np.uint64(S) + np.arange(S, dtype=np.uint64)
        vid = (splitmix64(seed ^ TRACE_SEED_XOR, c) % np.uint64(n)).astype(np.int64)
        pf = _prio_f32(op, v, dv)[vid]
        since = t - last[vid]
        feat = np.stack([np.log2(pf + np.float32(1e-30)), f1[vid],
                         (np.minimum(since, 64).astype(np.float32) * np.float32(1.0 / 64.0))],
                        axis=1).astype(np.float32)
        # 2. the round: select, claim, send
        sel = topk_exact(p, q) if pending.sum() > k else np.flatnonzero(pending)
        delta = dv[sel].copy()
        if op == OP_SUM:
            dv[sel] = 0.0
            v[sel] += delta
            improves = delta != 0.0
        elif op == OP_MIN:
            dv[sel] = INF_U32
            improves = delta < v[sel]
            v[sel[improves]] = delta[improves]
        else:
            dv[sel] = -1
            improves = delta > v[sel]
            v[sel[improves]] = delta[improves]
        last[sel] = t
        senders = sel[improves]
        for j, d in zip(senders, delta[improves]):
            e0, e1 = rp[j], rp[j + 1]
            if op == OP_SUM:
                m = a[j] * d * (wf[e0:e1] if wf is not None else np.ones(e1 - e0))
                np.add.at(dv, col[e0:e1], m)
            elif op == OP_MIN:
                if int(d) == INF_U32:
                    continue
                msg = np.minimum(np.uint64(d) + wu[e0:e1], np.uint64(INF_U32)).astype(np.uint32)
                np.minimum.at(dv, col[e0:e1], msg)
            else:
                np.maximum.at(dv, col[e0:e1], np.int32(d))
        chosen = np.zeros(n, dtype=bool)
        chosen[sel] = True
        rec.append((vid, feat, pending[vid], chosen[vid], v[vid].copy(), pf))
        t += 1
    T = t
    pfin = priority(op, v, dv)
    final_pending = pfin > 0
    final_pf = np.where(final_pending, _prio_f32(op, v, dv), np.float32(0)) if op == OP_SUM else None
    done = not final_pending.any() or (op == OP_SUM and pfin.sum() <= eps)
    full = T if done else max(T - H, 0)
    xs, ys, vids, rounds, vals = [], [], [], [], []
    for r in range(full):
        vid, feat, p0, chosen, val, pf0 = rec[r]
        for i in range(S):
            if not (p0[i] and chosen[i]):
                continue
            j = vid[i]
            again = False
            for s in range(r + 1, r + H + 1):
                if op == OP_SUM:
                    later = pf_hist[s][j] if s < T else final_pf[j]
                    if later >= np.float32(0.5) * pf0[i]:
                        again = True
                        break
                    continue
                mask = pend_hist[s] if s < T else final_pending
                if mask[j]:
                    again = True
                    break
            xs.append(feat[i])
            ys.append(0.0 if again else 1.0)
            vids.append(j)
            rounds.append(r)
            vals.append(val[i])
    x = np.array(xs, dtype=np.float32).reshape(-1, 3)
    return dict(x=x, y=np.array(ys, dtype=np.float32), vid=np.array(vids, dtype=np.int64),
                round=np.array(rounds, dtype=np.int64), value=np.array(vals), rounds=T, v=v,
                dv=dv)
