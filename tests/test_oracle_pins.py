"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a value
worked out by hand from the paper's equations (tests/golden), a closed form, a
library routine (LAPACK solve, scipy's Dijkstra and connected components), a
brute-force search on tiny inputs, or an invariant that holds exactly.

Which plausible oracle mistake each pin catches:
* dense-solve / golden PageRank: wrong divisor (receiver's instead of sender's
  out-degree, Table 1 typo), dropped constant c, transposed operand;
* mass conservation and the per-vertex state identity: a lost or double-counted
  delta in the update step (Eq. async);
* Dijkstra / Bellman-Ford / golden SSSP: wrong (+) or g for the min problem;
* brute-force reachability / golden CC: wrong direction of propagation;
* Katz closed form: missing l = 0 term, wrong power of beta.
"""
import itertools
import os

import numpy as np
import pytest

import daic_gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def random_graph(n, m, seed, self_loops=True):
    """Small multigraph with duplicates, self-loops and dangling vertices."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    # leave a few vertices without out-edges
    dead = rng.choice(n, max(1, n // 10), replace=False)
    keep = ~np.isin(src, dead)
    return daic_gen.from_edges(n, src[keep], dst[keep])


def dense_pagerank(g, d):
    """Solve (I - M^T) v = (1-d) 1 with M_jk = d * (#edges j->k) / outdeg_j."""
    n = g.n
    deg = g.outdeg()
    M = np.zeros((n, n))
    for j in range(n):
        for e in range(int(g.row_ptr[j]), int(g.row_ptr[j + 1])):
            M[j, g.col[e]] += d / deg[j]
    return np.linalg.solve(np.eye(n) - M.T, np.full(n, 1.0 - d))


# ---------------------------------------------------------------------------
# Sum problems (PageRank, Katz)
# ---------------------------------------------------------------------------

def test_golden_pagerank_3node():
    gd = read_golden("pagerank_3node.txt")
    e = list(map(int, gd["edges"]))
    g = daic_gen.from_edges(3, e[0::2], e[1::2])
    d = float(gd["d"][0])
    want = np.array(list(map(float, gd["fixed_point_num"]))) / float(gd["fixed_point_den"][0])
    v0, dv1 = oracle.pagerank_init(3, d)
    v, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, dv1, eps=1e-15)
    np.testing.assert_allclose(v, want, rtol=0, atol=1e-13)
    for sched in (oracle.SCHED_PRIORITY, oracle.SCHED_ROUND_ROBIN):
        r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, sched=sched,
                             eps=1e-15)
        np.testing.assert_allclose(r["v"], want, rtol=0, atol=1e-13)
    vs, _, _, _ = oracle.sync_daic_sum(g, oracle.G_DEG_SCALE, d, v0, dv1, eps=1e-15)
    np.testing.assert_allclose(vs, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pagerank_matches_dense_solve(seed):
    g = random_graph(150, 900, seed)
    d = 0.8
    want = dense_pagerank(g, d)
    v0, dv1 = oracle.pagerank_init(g.n, d)
    vj, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, dv1, eps=1e-14)
    vs, _, _, _ = oracle.sync_daic_sum(g, oracle.G_DEG_SCALE, d, v0, dv1, eps=1e-14)
    vp = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=1e-14)["v"]
    vr = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=1e-14,
                          sched=oracle.SCHED_ROUND_ROBIN)["v"]
    for v in (vj, vs, vp, vr):
        assert np.abs(v - want).sum() <= 1e-12 * g.n


def test_pagerank_normalized_linear_system():
    """(I - d W^T) x = (1-d)/n 1 is the paper's solution divided by n."""
    g = daic_gen.powerlaw(n=300, seed=11)
    d = 0.8
    n = g.n
    W = np.zeros((n, n))
    deg = g.outdeg()
    for j in range(n):
        for e in range(int(g.row_ptr[j]), int(g.row_ptr[j + 1])):
            W[j, g.col[e]] += 1.0 / deg[j]
    x = np.linalg.solve(np.eye(n) - d * W.T, np.full(n, (1 - d) / n))
    v, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, np.full(n, 1 - d), eps=1e-14)
    np.testing.assert_allclose(v / n, x, rtol=1e-11, atol=1e-15)


def test_closed_forms_pagerank():
    d = 0.8
    # directed cycle: every vertex keeps rank 1
    n = 17
    cyc = daic_gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    v, _, _ = oracle.jacobi_sum(cyc, oracle.G_DEG_SCALE, d, np.full(n, 1 - d), eps=1e-15)
    np.testing.assert_allclose(v, 1.0, atol=1e-13)
    # edgeless: only the constant remains
    empty = daic_gen.from_edges(5, [], [])
    v, _, _ = oracle.jacobi_sum(empty, oracle.G_DEG_SCALE, d, np.full(5, 1 - d))
    np.testing.assert_allclose(v, 1 - d, atol=0)
    # no dangling vertex: total rank equals n (Sec. 6.3: sum R grows from 0.2 N to N)
    g = random_graph(200, 1500, 7)
    deg = g.outdeg()
    if (deg == 0).any():  # add a self-loop to every dangling vertex
        extra = np.nonzero(deg == 0)[0]
        src = np.concatenate([np.repeat(np.arange(g.n), deg), extra])
        dst = np.concatenate([g.col, extra])
        g = daic_gen.from_edges(g.n, src, dst)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, np.zeros(g.n),
                         np.full(g.n, 1 - d), alpha=d, eps=1e-12)
    assert abs(r["v"].sum() - g.n) <= 1e-11 * g.n


def test_golden_katz_cycle():
    gd = read_golden("katz_cycle4.txt")
    e = list(map(int, gd["edges"]))
    g = daic_gen.from_edges(4, e[0::2], e[1::2])
    beta = float(gd["beta"][0])
    s = int(gd["source"][0])
    want = np.array(list(map(float, gd["fixed_point_num"]))) / float(gd["fixed_point_den"][0])
    dv1 = np.zeros(4)
    dv1[s] = 1.0
    v, _, _ = oracle.jacobi_sum(g, oracle.G_SRC_SCALE, beta, dv1, eps=1e-16)
    np.testing.assert_allclose(v, want, atol=1e-14)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_SRC_SCALE, np.zeros(4), dv1, alpha=beta,
                         eps=1e-16)
    np.testing.assert_allclose(r["v"], want, atol=1e-14)


def test_edge_scale_matches_dense_solve():
    """Adsorption-style g(x) = a_j w_jk x with per-vertex a_j and log-normal w."""
    g = random_graph(80, 500, 3)
    w = daic_gen.lognormal_f64(17, g.m, 0.4, 0.8)
    deg = g.outdeg()
    # scale so that every row sums to at most 0.9: a contraction
    rowsum = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
    rowsum = np.where(deg > 0, rowsum, 1.0)
    a = 0.9 / rowsum
    M = np.zeros((g.n, g.n))
    for j in range(g.n):
        for e in range(int(g.row_ptr[j]), int(g.row_ptr[j + 1])):
            M[j, g.col[e]] += a[j] * w[e]
    c = daic_gen.lognormal_f64(18, g.n, 0.0, 1.0)
    want = np.linalg.solve(np.eye(g.n) - M.T, c)
    v, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 0.0, c, w=w, alpha_pv=a, eps=1e-14)
    np.testing.assert_allclose(v, want, rtol=1e-11)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_EDGE_SCALE, np.zeros(g.n), c, alpha_pv=a,
                         w=w, eps=1e-14)
    np.testing.assert_allclose(r["v"], want, rtol=1e-11)


def test_nonzero_v0_uses_fourth_condition():
    """Any (v0, dv1) with v0 + dv1 = f(v0) reaches the same fixed point."""
    g = random_graph(60, 300, 5)
    d = 0.8
    want = dense_pagerank(g, d)
    rng = np.random.default_rng(0)
    v0 = rng.uniform(0, 2, g.n)
    # f(v0) = c + M^T v0, so dv1 = f(v0) - v0
    deg = g.outdeg()
    mtv = np.zeros(g.n)
    for j in range(g.n):
        for e in range(int(g.row_ptr[j]), int(g.row_ptr[j + 1])):
            mtv[g.col[e]] += d / deg[j] * v0[j]
    dv1 = (1 - d) + mtv - v0
    v, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, dv1, v0=v0, eps=1e-14)
    np.testing.assert_allclose(v, want, atol=1e-11)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=1e-14)
    np.testing.assert_allclose(r["v"], want, atol=1e-11)


@pytest.mark.parametrize("updates", [1, 37, 400, 5000])
@pytest.mark.parametrize("sched", [oracle.SCHED_PRIORITY, oracle.SCHED_ROUND_ROBIN])
def test_mass_conservation_and_state_identity(updates, sched):
    """At every point of an asynchronous run (Eq. async), exactly in reals:
    sum_j dv_j + sum_j (1 - s_j) v_j = sum_j dv1_j   (s_j = d, or 0 if dangling)
    and per vertex v + dv = c + M^T v with c = dv1 (v0 = 0)."""
    g = random_graph(120, 700, 9)
    d = 0.8
    n = g.n
    deg = g.outdeg()
    v0, dv1 = oracle.pagerank_init(n, d)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, sched=sched,
                         eps=0.0, max_updates=updates)
    v, dv = r["v"], r["dv"]
    s = np.where(deg > 0, d, 0.0)
    lhs = dv.sum() + ((1 - s) * v).sum()
    assert abs(lhs - dv1.sum()) <= 1e-12 * dv1.sum()
    mtv = np.zeros(n)
    for j in range(n):
        for e in range(int(g.row_ptr[j]), int(g.row_ptr[j + 1])):
            mtv[g.col[e]] += d / deg[j] * v[j]
    np.testing.assert_allclose(v + dv, dv1 + mtv, rtol=1e-12, atol=1e-13)


def test_progress_is_monotone_and_bounded():
    """sum_j v_j grows monotonically from 0.2 N towards its limit (Sec. 3.4, 6.3)."""
    g = daic_gen.powerlaw(n=400, seed=4)
    d = 0.8
    v0, dv1 = oracle.pagerank_init(g.n, d)
    r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=1e-12,
                         trace_every=1, trace_len=20000)
    tr = r["trace"][: min(r["updates"], 20000)]
    assert np.all(np.diff(tr) >= -1e-12)
    want = dense_pagerank(g, d)
    assert tr[-1] <= want.sum() + 1e-9


def test_residual_bound():
    """For PageRank ||v* - v||_1 <= r / (1 - d) at any state (r = sum |dv|)."""
    g = random_graph(100, 600, 12)
    d = 0.8
    want = dense_pagerank(g, d)
    v0, dv1 = oracle.pagerank_init(g.n, d)
    for upd in (10, 100, 1000):
        r = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=0.0,
                             max_updates=upd)
        err = np.abs(want - r["v"]).sum()
        assert err <= r["residual"] / (1 - d) * (1 + 1e-9) + 1e-12


def test_theorem2_async_closer_than_sync_per_vertex():
    """Same synchronous update sequence: after k subsequences the asynchronous
    state is per vertex at least as close to the fixed point (Theorem 2)."""
    g = daic_gen.powerlaw(n=300, seed=21)
    d = 0.8
    want = dense_pagerank(g, d)
    v0, dv1 = oracle.pagerank_init(g.n, d)
    for k in (1, 2, 5, 10):
        vs, _, _, _ = oracle.sync_daic_sum(g, oracle.G_DEG_SCALE, d, v0, dv1, eps=0.0,
                                           max_rounds=k)
        ra = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d,
                              sched=oracle.SCHED_SWEEP, eps=0.0, max_updates=k * g.n)
        assert np.all(np.abs(want - ra["v"]) <= np.abs(want - vs) + 1e-12)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_sweep_blocks_whole_graph_is_the_synchronous_round(k):
    """Blocks of n ids: one round is one synchronous DAIC round (Eq. sync)."""
    g = random_graph(150, 900, 41)
    d = 0.8
    v0, dv1 = oracle.pagerank_init(g.n, d)
    vs, dvs, _, _ = oracle.sync_daic_sum(g, oracle.G_DEG_SCALE, d, v0, dv1, eps=0.0, max_rounds=k)
    vb, dvb = oracle.sweep_blocks(g, oracle.G_DEG_SCALE, d, v0, dv1, g.n, k)
    np.testing.assert_allclose(vb, vs, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dvb, dvs, rtol=1e-13, atol=1e-15)
    # weighted form with per-source coefficients
    rng = np.random.default_rng(4)
    w = rng.uniform(0.1, 1.0, g.m)
    a = rng.uniform(0.1, 0.5, g.n) / np.maximum(1, g.outdeg())
    c = rng.uniform(0, 1, g.n)
    vs, dvs, _, _ = oracle.sync_daic_sum(g, oracle.G_EDGE_SCALE, 0.0, np.zeros(g.n), c, w=w, alpha_pv=a,
                                         eps=0.0, max_rounds=k)
    vb, dvb = oracle.sweep_blocks(g, oracle.G_EDGE_SCALE, 0.0, np.zeros(g.n), c, g.n, k, w=w, alpha_pv=a)
    np.testing.assert_allclose(vb, vs, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dvb, dvs, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 6])
def test_sweep_blocks_of_one_is_the_id_order_sequence(k):
    """Blocks of one id: k n rounds are k passes of the one-vertex-at-a-time
    update sequence in id order (the C oracle's sweep schedule)."""
    g = daic_gen.powerlaw(n=300, seed=22)
    d = 0.8
    v0, dv1 = oracle.pagerank_init(g.n, d)
    ra = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d,
                          sched=oracle.SCHED_SWEEP, eps=0.0, max_updates=k * g.n)
    vb, dvb = oracle.sweep_blocks(g, oracle.G_DEG_SCALE, d, v0, dv1, 1, k * g.n)
    np.testing.assert_allclose(vb, ra["v"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dvb, ra["dv"], rtol=1e-13, atol=1e-15)
    beta = 0.5 / max(1, int(g.outdeg().max()))
    ra = oracle.async_run(g, oracle.OP_SUM, oracle.G_SRC_SCALE, np.zeros(g.n), dv1, alpha=beta,
                          sched=oracle.SCHED_SWEEP, eps=0.0, max_updates=k * g.n)
    vb, dvb = oracle.sweep_blocks(g, oracle.G_SRC_SCALE, beta, np.zeros(g.n), dv1, 1, k * g.n)
    np.testing.assert_allclose(vb, ra["v"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dvb, ra["dv"], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("B", [1, 7, 33])
def test_sweep_blocks_invariants_and_fixed_point(B):
    """Any number of block rounds keeps the state identities of Eq. async
    (mass; v + dv = c + M^T v) and the rounds reach the dense solve."""
    g = random_graph(120, 700, 9)
    d = 0.8
    n = g.n
    deg = g.outdeg()
    v0, dv1 = oracle.pagerank_init(n, d)
    s = np.where(deg > 0, d, 0.0)
    src = np.repeat(np.arange(n), deg)
    for rounds in (1, 5, 40):
        v, dv = oracle.sweep_blocks(g, oracle.G_DEG_SCALE, d, v0, dv1, B, rounds)
        assert abs(dv.sum() + ((1 - s) * v).sum() - dv1.sum()) <= 1e-12 * dv1.sum()
        mtv = np.bincount(g.col.astype(np.int64), weights=d * v[src] / deg[src], minlength=n)
        np.testing.assert_allclose(v + dv, dv1 + mtv, rtol=1e-12, atol=1e-13)
    P = -(-n // B)
    v, dv = oracle.sweep_blocks(g, oracle.G_DEG_SCALE, d, v0, dv1, B, 200 * P)
    np.testing.assert_allclose(v, dense_pagerank(g, d), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_theorem4_priority_ahead_of_round_robin_in_l1(seed):
    """After the same number of updates, priority scheduling is at least as
    close to the fixed point as round-robin, in aggregate L1 (Theorem 4)."""
    g = daic_gen.powerlaw(n=500, seed=seed)
    d = 0.8
    want = dense_pagerank(g, d)
    v0, dv1 = oracle.pagerank_init(g.n, d)
    for upd in (250, 1000, 4000):
        rp = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=0.0,
                              max_updates=upd)
        rr = oracle.async_run(g, oracle.OP_SUM, oracle.G_DEG_SCALE, v0, dv1, alpha=d, eps=0.0,
                              max_updates=upd, sched=oracle.SCHED_ROUND_ROBIN)
        assert np.abs(want - rp["v"]).sum() <= np.abs(want - rr["v"]).sum()


# ---------------------------------------------------------------------------
# Min problem (SSSP)
# ---------------------------------------------------------------------------

def bellman_ford(n, src, dst, w, s):
    inf = float("inf")
    dist = [inf] * n
    dist[s] = 0
    for _ in range(n):
        changed = False
        for a, b, c in zip(src, dst, w):
            if dist[a] + c < dist[b]:
                dist[b] = dist[a] + c
                changed = True
        if not changed:
            break
    return [0xFFFFFFFF if x == inf else int(x) for x in dist]


def test_golden_sssp():
    gd = read_golden("sssp_5node.txt")
    e = list(map(int, gd["edges"]))
    src, dst, w = e[0::3], e[1::3], e[2::3]
    g = daic_gen.from_edges(5, src, dst)
    # from_edges sorts edges by (src, dst); carry the weights along
    order = np.lexsort((dst, src))
    w = np.asarray(w, dtype=np.uint32)[order]
    want = np.array(list(map(int, gd["dist"])), dtype=np.uint32)
    s = int(gd["source"][0])
    np.testing.assert_array_equal(oracle.dijkstra(g, w, s), want)
    v0, dv1 = oracle.sssp_init(5, s)
    for sched in (oracle.SCHED_PRIORITY, oracle.SCHED_ROUND_ROBIN):
        r = oracle.async_run(g, oracle.OP_MIN, oracle.G_EDGE_ADD, v0, dv1, w=w, sched=sched)
        np.testing.assert_array_equal(r["v"], want)


@pytest.mark.parametrize("seed", [0, 1])
def test_dijkstra_vs_bellman_ford_and_scipy(seed):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra

    rng = np.random.default_rng(seed)
    n, m = 60, 240
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    w = rng.integers(1, 256, m).astype(np.uint32)
    order = np.lexsort((dst, src))
    src, dst, w = src[order], dst[order], w[order]
    g = daic_gen.from_edges(n, src, dst)
    got = oracle.dijkstra(g, w, 0)
    np.testing.assert_array_equal(got, bellman_ford(n, src, dst, w, 0))
    # scipy sums duplicate entries, so keep only the lightest parallel edge
    best = {}
    for a, b, c in zip(src, dst, w):
        if a != b:
            best[(a, b)] = min(best.get((a, b), 1 << 40), int(c))
    keys = list(best)
    A = csr_matrix(([best[k] for k in keys], ([k[0] for k in keys], [k[1] for k in keys])),
                   shape=(n, n))
    ref = sp_dijkstra(A, indices=0)
    ref = np.where(np.isinf(ref), 0xFFFFFFFF, ref).astype(np.uint64)
    np.testing.assert_array_equal(got.astype(np.uint64), ref)


def test_async_min_matches_dijkstra_on_rmat():
    g = daic_gen.rmat(12, 8, seed=42)
    w = daic_gen.sssp_weights(g.m, seed=43)
    want = oracle.dijkstra(g, w, 0)
    v0, dv1 = oracle.sssp_init(g.n, 0)
    for sched in (oracle.SCHED_PRIORITY, oracle.SCHED_ROUND_ROBIN):
        r = oracle.async_run(g, oracle.OP_MIN, oracle.G_EDGE_ADD, v0, dv1, w=w, sched=sched)
        np.testing.assert_array_equal(r["v"], want)
        assert r["residual"] == 0


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_dijkstra_f64_vs_bellman_ford_and_scipy(seed):
    """Real log-normal weights (the paper's SSSP data, Sec. 6.1): the heap
    Dijkstra equals Bellman-Ford relaxation to a fixed point, and scipy's
    Dijkstra on the graph with duplicate edges reduced to the lightest."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra

    g = random_graph(200, 1500, seed)
    w = daic_gen.lognormal_f64(seed, g.m, 0.0, 1.0)
    got = oracle.dijkstra_f64(g, w, 0)
    # Bellman-Ford: relax every edge until nothing changes
    src = np.repeat(np.arange(g.n), g.outdeg())
    col = g.col.astype(np.int64)
    bf = np.full(g.n, np.inf)
    bf[0] = 0.0
    for _ in range(g.n):
        cand = bf[src] + w
        new = bf.copy()
        np.minimum.at(new, col, cand)
        if np.array_equal(new, bf):
            break
        bf = new
    np.testing.assert_array_equal(got, bf)
    best = {}
    for s_, t_, w_ in zip(src, col, w):
        if s_ == t_:
            continue  # a self-loop never shortens a path
        if (s_, t_) not in best or w_ < best[(s_, t_)]:
            best[(s_, t_)] = w_
    keys = np.array(list(best.keys()), dtype=np.int64).reshape(-1, 2)
    M = csr_matrix((np.array(list(best.values())), (keys[:, 0], keys[:, 1])), shape=(g.n, g.n))
    ref = sp_dijkstra(M, directed=True, indices=0)
    np.testing.assert_allclose(got, ref, rtol=1e-15, atol=0)
    assert np.array_equal(np.isinf(got), np.isinf(ref))


def test_dijkstra_f64_integer_weights_match_u32_oracle():
    g = daic_gen.rmat(10, 8, seed=3)
    w = daic_gen.sssp_weights(g.m, seed=4)
    got = oracle.dijkstra_f64(g, w.astype(np.float64), 0)
    ref = oracle.dijkstra(g, w, 0)
    reach = ref != 0xFFFFFFFF
    np.testing.assert_array_equal(got[reach], ref[reach].astype(np.float64))
    assert np.all(np.isinf(got[~reach]))


def test_sssp_path_graph_prefix_sums():
    n = 50
    g = daic_gen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    w = daic_gen.sssp_weights(g.m, seed=5)
    want = np.concatenate([[0], np.cumsum(w.astype(np.uint64))]).astype(np.uint32)
    np.testing.assert_array_equal(oracle.dijkstra(g, w, 0), want)


# ---------------------------------------------------------------------------
# Max problem (connected components)
# ---------------------------------------------------------------------------

def test_golden_cc():
    gd = read_golden("cc_6node.txt")
    e = list(map(int, gd["edges"]))
    g = daic_gen.from_edges(6, e[0::2], e[1::2])
    want = np.array(list(map(int, gd["directed_labels"])), dtype=np.int32)
    np.testing.assert_array_equal(oracle.maxlabel(g), want)
    v0, dv1 = oracle.cc_init(6)
    r = oracle.async_run(g, oracle.OP_MAX, oracle.G_COPY, v0, dv1)
    np.testing.assert_array_equal(r["v"], want)


def test_maxlabel_vs_bruteforce_reachability():
    rng = np.random.default_rng(3)
    n, m = 40, 70
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    g = daic_gen.from_edges(n, src, dst)
    adj = [[] for _ in range(n)]
    for a, b in zip(src, dst):
        adj[a].append(b)
    want = np.arange(n, dtype=np.int32)
    for s in range(n):
        seen, stack = {s}, [s]
        while stack:
            u = stack.pop()
            for x in adj[u]:
                if x not in seen:
                    seen.add(x)
                    stack.append(x)
        for x in seen:
            want[x] = max(want[x], s)
    np.testing.assert_array_equal(oracle.maxlabel(g), want)


def test_maxlabel_symmetric_equals_components():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    g0 = daic_gen.rmat(10, 2, seed=8)
    src = np.repeat(np.arange(g0.n), g0.outdeg())
    dst = g0.col.astype(np.int64)
    g = daic_gen.from_edges(g0.n, np.concatenate([src, dst]), np.concatenate([dst, src]))
    A = csr_matrix((np.ones(len(src)), (src, dst)), shape=(g0.n, g0.n))
    ncomp, lab = connected_components(A, directed=True, connection="weak")
    comp_max = np.full(ncomp, -1)
    np.maximum.at(comp_max, lab, np.arange(g0.n))
    want = comp_max[lab].astype(np.int32)
    np.testing.assert_array_equal(oracle.maxlabel(g), want)
    v0, dv1 = oracle.cc_init(g.n)
    r = oracle.async_run(g, oracle.OP_MAX, oracle.G_COPY, v0, dv1)
    np.testing.assert_array_equal(r["v"], want)


# ---------------------------------------------------------------------------
# Selection rules and priorities
# ---------------------------------------------------------------------------

def test_priority_rows_of_table1():
    # sum: |dv|
    np.testing.assert_array_equal(oracle.priority(oracle.OP_SUM, [1.0, 2.0], [-0.5, 0.25]),
                                  [0.5, 0.25])
    # SSSP: d - min(d, dd), first reach -> 0xFFFFFFFF, nothing pending -> 0
    inf = oracle.INF_U32
    p = oracle.priority(oracle.OP_MIN, [inf, inf, 10, 10], [inf, 7, 3, 12])
    np.testing.assert_array_equal(p, [0, inf, 7, 0])
    # CC: max(v, dv) - v
    np.testing.assert_array_equal(oracle.priority(oracle.OP_MAX, [-1, 5, 5], [3, 9, 2]),
                                  [4, 4, 0])


def test_topk_exact_bruteforce():
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = int(rng.integers(1, 60))
        p = rng.integers(0, 5, n).astype(np.float64)  # many ties and zeros
        q = float(rng.uniform(0.01, 1.0))
        k = int(np.ceil(q * n))
        ranked = sorted(range(n), key=lambda j: (-p[j], j))[:k]
        want = sorted(j for j in ranked if p[j] > 0)
        np.testing.assert_array_equal(oracle.topk_exact(p, q), want)


def test_splitmix64_reference_values():
    """First outputs of SplitMix64 seeded with 1234567, the published test
    sequence of the Rosetta Code "Pseudo-random numbers/Splitmix64" task."""
    got = oracle.splitmix64(1234567, np.arange(5))
    want = np.array([6457827717110365317, 3203168211198807973, 9817491932198370423,
                     4593380528125082431, 16408922859458223821], dtype=np.uint64)
    np.testing.assert_array_equal(got, want)


def test_sampled_threshold_properties():
    rng = np.random.default_rng(2)
    p = rng.exponential(1.0, 100000)
    p[rng.random(p.size) < 0.3] = 0.0
    # q = 1: every pending vertex is selected
    tau = oracle.sampled_threshold(p, 1.0, 4096, 9, 0)
    assert tau == p[p > 0].min()
    # q = 0.1: the selected fraction is close to q (sampling error ~ 1/sqrt(S))
    tau = oracle.sampled_threshold(p, 0.1, 4096, 9, 3)
    frac = np.mean(p >= tau)
    assert abs(frac - 0.1) < 0.02
    # no positive sample: take all pending
    p2 = np.zeros(1000)
    p2[5] = 1.0
    assert oracle.sampled_threshold(p2, 0.01, 64, 1, 0) == 1.0


def test_golden_sampled_threshold_rank():
    """The rank rule of the sampled threshold, by hand: ceil(q S)-th largest,
    ranked from 1 (floor, or a rank counted from 0, fail one of the cases)."""
    gd = read_golden("sampled_threshold_10.txt")
    n, S, seed = int(gd["n"][0]), int(gd["S"][0]), int(gd["seed"][0])
    p = np.array(list(map(float, gd["prio"])))
    for t in (0, 1):
        np.testing.assert_array_equal(oracle.sample_indices(n, S, seed, t),
                                      list(map(int, gd[f"ids_round{t}"])))
    for key, vals in gd.items():
        if key.startswith("tau_round"):
            t = int(key[len("tau_round")])
            q = float(key.split("_q")[1])
            assert oracle.sampled_threshold(p, q, S, seed, t) == float(vals[0]), key


# ---------------------------------------------------------------------------
# Scheduler network
# ---------------------------------------------------------------------------

def test_mlp_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = {"W1": rng.normal(0, 0.5, (64, 3)), "b1": rng.normal(0, 0.1, 64),
              "W2": rng.normal(0, 0.2, (64, 64)), "b2": rng.normal(0, 0.1, 64),
              "W3": rng.normal(0, 0.2, (1, 64)), "b3": rng.normal(0, 0.1, 1)}
    x = rng.normal(0, 1, (32, 3))
    y = (rng.random(32) < 0.4).astype(np.float64)
    z, cache = oracle.mlp_forward(params, x)
    grads = oracle.mlp_backward(params, cache, z, y)
    h = 1e-6
    for name, p in params.items():
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = oracle.bce_with_logits(oracle.mlp_forward(params, x)[0], y)
            flat[idx] = old - h
            lm = oracle.bce_with_logits(oracle.mlp_forward(params, x)[0], y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, an)


def test_generators_are_deterministic_and_shaped():
    a = daic_gen.rmat(10, 4, seed=3)
    b = daic_gen.rmat(10, 4, seed=3)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
    assert a.m == 4 * 1024 and a.row_ptr[-1] == a.m
    assert all(np.all(np.diff(a.col[a.row_ptr[i]:a.row_ptr[i + 1]].astype(np.int64)) >= 0)
               for i in range(a.n))
    pl = daic_gen.powerlaw(n=2000, seed=1)
    deg = pl.outdeg()
    assert deg.max() <= 500
    for j in range(pl.n):  # no self-loop, no duplicate per source
        row = pl.col[pl.row_ptr[j]:pl.row_ptr[j + 1]]
        assert j not in row and len(set(row.tolist())) == len(row)


def test_golden_adam_steps():
    """Adam by hand: a constant gradient moves w by exactly -lr g / (|g| + eps)
    per step (bias-corrected moments equal g and g^2); a sign flip gives
    w2 = -0.1 (18/19) / (1 + eps). A dropped bias correction, a swapped beta
    or a missing square fails one of them."""
    gd = read_golden("adam_steps.txt")
    w, m, v = np.array([float(gd["const_w0"][0])]), np.zeros(1), np.zeros(1)
    g = np.array([float(gd["const_g"][0])])
    for t in range(1, int(gd["const_steps"][0]) + 1):
        w, m, v = oracle.adam_step(w, g, m, v, t, float(gd["const_lr"][0]))
    np.testing.assert_allclose(w, float(gd["const_w"][0]), rtol=0, atol=1e-15)
    lr = float(gd["flip_lr"][0])
    w, m, v = oracle.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, lr)
    np.testing.assert_allclose(w, float(gd["flip_w1"][0]), rtol=0, atol=1e-15)
    w, m, v = oracle.adam_step(w, -np.ones(1), m, v, 2, lr)
    np.testing.assert_allclose(w, float(gd["flip_w2"][0]), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Trace rule of the learned scheduler (exact top-k rounds, integer problems)
# ---------------------------------------------------------------------------

def _golden_trace(name="trace_sssp_4node.txt"):
    gd = {}
    ups = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "update":
                ups.append(vals)
            else:
                gd[key] = vals
    return gd, ups


@pytest.mark.parametrize("H", [1, 4])
def test_golden_trace_sssp_4node(H):
    """Features and labels of every sampled update against the hand-worked
    4-vertex run; the emitted samples are exactly the sampled vertices that
    were selected in their round (once per draw)."""
    gd, ups = _golden_trace()
    n = int(gd["n"][0])
    e = list(map(int, gd["edges"]))
    g = daic_gen.from_edges(n, e[0::3], e[1::3])
    order = np.lexsort((e[1::3], e[0::3]))  # the CSR keeps edges sorted by source
    w = np.array(e[2::3], dtype=np.uint32)[order]
    np.testing.assert_array_equal(g.col, np.array(e[1::3])[order])
    v0, dv1 = oracle.sssp_init(n, int(gd["source"][0]))
    S, seed = 16, 5
    r = oracle.trace_exact_topk(g, oracle.OP_MIN, v0, dv1, float(gd["q"][0]), S, H, seed, w=w)
    assert r["rounds"] == int(gd["rounds"][0])
    np.testing.assert_array_equal(r["v"], list(map(int, gd["dist"])))
    want = {(int(u[0]), int(u[1])): u for u in ups}
    expect_count = 0
    for t in range(r["rounds"]):
        ids = oracle.sample_indices(n, S, seed ^ oracle.TRACE_SEED_XOR, t)
        expect_count += sum(1 for j in ids if (t, int(j)) in want)
    assert len(r["y"]) == expect_count
    for i in range(len(r["y"])):
        u = want[(int(r["round"][i]), int(r["vid"][i]))]
        np.testing.assert_allclose(r["x"][i], np.array(u[2:5], dtype=np.float64), rtol=1e-6,
                                   atol=1e-7)
        assert r["y"][i] == float(u[5] if H == 4 else u[6])
        assert r["value"][i] == int(u[7])


@pytest.mark.parametrize("H", [1, 2])
def test_golden_trace_pagerank_2cycle(H):
    """The sum-problem trace rule against the hand-worked 2-vertex run: the
    state after 4 rounds, and features, labels and stored values of every
    sampled update (labels only for rounds before T - H)."""
    gd, ups = _golden_trace("trace_pr_2cycle.txt")
    n = int(gd["n"][0])
    e = list(map(int, gd["edges"]))
    g = daic_gen.from_edges(n, e[0::2], e[1::2])
    dv1 = np.array(list(map(float, gd["dv1"])))
    S, seed = 16, 5
    r = oracle.trace_exact_topk(g, oracle.OP_SUM, np.zeros(n), dv1, float(gd["q"][0]), S, H, seed,
                                max_rounds=int(gd["rounds"][0]), gk=oracle.G_DEG_SCALE,
                                alpha=float(gd["d"][0]))
    assert r["rounds"] == int(gd["rounds"][0])
    np.testing.assert_allclose(r["v"], list(map(float, gd["v"])), rtol=1e-14)
    np.testing.assert_allclose(r["dv"], list(map(float, gd["dv"])), rtol=1e-14, atol=1e-15)
    col = 5 if H == 1 else 6
    want = {(int(u[0]), int(u[1])): u for u in ups if u[col] != "-"}
    expect_count = 0
    for t in range(r["rounds"] - H):
        ids = oracle.sample_indices(n, S, seed ^ oracle.TRACE_SEED_XOR, t)
        expect_count += sum(1 for j in ids if (t, int(j)) in want)
    assert expect_count > 0
    assert len(r["y"]) == expect_count
    for i in range(len(r["y"])):
        u = want[(int(r["round"][i]), int(r["vid"][i]))]
        np.testing.assert_allclose(r["x"][i], np.array(u[2:5], dtype=np.float64), rtol=1e-6, atol=1e-6)
        assert r["y"][i] == float(u[col])
        assert abs(r["value"][i] - float(u[7])) <= 1e-14


def test_trace_sum_rounds_reach_the_dense_solve():
    """The sum branch of the trace's exact top-k rounds, run to a tiny
    residual, reaches the fixed point of the dense solve (Theorem 1): a wrong
    claim (delta not cleared, not folded) or message (coefficient, target)
    breaks it."""
    g = random_graph(120, 700, 4)
    d = 0.8
    want = dense_pagerank(g, d)
    r = oracle.trace_exact_topk(g, oracle.OP_SUM, np.zeros(g.n), np.full(g.n, 1 - d), 0.1, 32, 3, 9,
                                gk=oracle.G_DEG_SCALE, alpha=d, eps=1e-13)
    assert np.abs(r["dv"]).sum() <= 1e-13
    assert np.abs(r["v"] - want).sum() <= 1e-11 * g.n
    assert 0.0 < r["y"].mean() < 1.0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_trace_labels_match_final_values(seed):
    """With a horizon past the run's end, an update is labelled 1 exactly when
    the value it stored is the vertex's final value: Dijkstra distances (min)
    and max-label reachability (max), both computed independently. A label
    window off by one round, or a stale pending test, breaks this."""
    rng = np.random.default_rng(seed)
    n = 60
    src, dst = rng.integers(0, n, 240), rng.integers(0, n, 240)
    g = daic_gen.from_edges(n, src, dst)
    w = rng.integers(1, 30, g.m).astype(np.uint32)
    v0, dv1 = oracle.sssp_init(n, 0)
    r = oracle.trace_exact_topk(g, oracle.OP_MIN, v0, dv1, 0.3, 64, 64, seed, w=w)
    assert r["rounds"] < 64
    dist = oracle.dijkstra(g, w, 0)
    np.testing.assert_array_equal(r["v"], dist)
    assert len(r["y"]) > 20
    np.testing.assert_array_equal(r["y"], (r["value"] == dist[r["vid"]]).astype(np.float32))
    v0, dv1 = oracle.cc_init(n)
    r = oracle.trace_exact_topk(g, oracle.OP_MAX, v0, dv1, 0.3, 64, 64, seed)
    assert r["rounds"] < 64
    lab = oracle.maxlabel(g)
    np.testing.assert_array_equal(r["v"], lab)
    np.testing.assert_array_equal(r["y"], (r["value"] == lab[r["vid"]]).astype(np.float32))


def test_mlp_rounding_hook():
    """The optional rounding of activations and deltas: with values that the
    rounding keeps (small integers and halves in BF16) it changes nothing;
    with BF16 rounding of random values it moves the logits by at most a few
    BF16 units of the absolute-value network (three rounding points)."""
    def bf16(a):
        a = np.asarray(a, dtype=np.float32)
        u = a.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)

    rng = np.random.default_rng(4)
    P = {"W1": rng.integers(-2, 3, (64, 3)).astype(float), "b1": rng.integers(-1, 2, 64) * 0.5,
         "W2": rng.integers(-1, 2, (64, 64)) * (rng.random((64, 64)) < 0.1),
         "b2": rng.integers(-1, 2, 64) * 0.5,
         "W3": rng.integers(-1, 2, (1, 64)).astype(float), "b3": np.array([0.5])}
    x = rng.integers(-1, 2, (40, 3)).astype(float)
    y = (rng.random(40) < 0.5).astype(float)
    P["W2"] = P["W2"].astype(float)
    z0, c0 = oracle.mlp_forward(P, x)
    z1, c1 = oracle.mlp_forward(P, x, rnd=bf16)
    assert np.abs(c0[4]).max() < 128 and np.any(c0[4] > 0)  # every activation exact in BF16
    np.testing.assert_array_equal(z0, z1)
    # logits are integers and halves here; the gradient's deltas are not, so
    # compare only the forward and the layer-3 terms that see no rounded delta
    g0 = oracle.mlp_backward(P, c0, z0, y)
    g1 = oracle.mlp_backward(P, c1, z1, y, rnd=bf16)
    for k in ("W3", "b3", "b2"):
        np.testing.assert_array_equal(g0[k], g1[k])
    Q = {k: rng.normal(0, 0.5, v.shape) for k, v in P.items()}
    xr = rng.normal(0, 1, (200, 3))
    za, _ = oracle.mlp_forward(Q, xr)
    zb, _ = oracle.mlp_forward(Q, xr, rnd=bf16)
    A = {k: np.abs(v) for k, v in Q.items()}
    zabs, _ = oracle.mlp_forward(A, np.abs(xr))
    assert np.all(np.abs(za - zb) <= 2.0 ** -7 * zabs)
    assert np.any(za != zb)
