"""GPU parity of SWEEP scheduling (blocks of ceil(q n) consecutive vertex ids,
each block pulling the newest message of every in-neighbour) against
the CPU oracle, with the tolerances of the other parity tests: FP64 L1 <= 1e-9
at residual 1e-10, FP32 relative L1 <= 1e-5. Runs stopped inside a sweep are
checked through the invariants that any DAIC state with every message
delivered satisfies (per-vertex v + dv = c + M^T v; PageRank mass)."""
import sys

import numpy as np
import pytest

import daic_gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def daic():
    from paper_1710_05785_amd import daic as d

    d.lib()
    return d


def pr_problem(daic, g, d=0.8, state="f64"):
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=d, state=state)
    p.set_init(*oracle.pagerank_init(g.n, d))
    return p


def mt_v(g, v, d):
    """(M^T v)_t = sum over edges s -> t of d v_s / outdeg_s."""
    deg = g.outdeg().astype(np.float64)
    src = np.repeat(np.arange(g.n), g.outdeg())
    return np.bincount(g.col.astype(np.int64), weights=d * v[src] / deg[src], minlength=g.n)


@pytest.fixture(scope="module")
def pl10k():
    return daic_gen.powerlaw(n=10000, seed=1)


@pytest.fixture(scope="module")
def pl10k_ref(pl10k):
    v, _, _ = oracle.jacobi_sum(pl10k, oracle.G_DEG_SCALE, 0.8, np.full(pl10k.n, 0.2), eps=1e-13)
    return v


@pytest.mark.parametrize("q", [1.0, 0.5, 0.125, 0.01, 2e-3])
def test_sweep_pagerank_f64(daic, pl10k, pl10k_ref, q):
    say("case sweep f64", q)
    p = pr_problem(daic, pl10k)
    res = p.run(eps=1e-10, q=q, sched="sweep", max_rounds=10**7)
    assert res.converged
    assert res.stats["final_residual"] <= 1e-10
    err = np.abs(p.get() - pl10k_ref).sum()
    assert err <= 1e-9, err


def test_sweep_single_block_is_the_synchronous_round(daic, pl10k):
    """q = 1: one block per sweep, every in-neighbour read from the previous
    sweep, i.e. the synchronous round; same round count as sched ALL (the
    residual bound is exact for non-negative messages) and the same result."""
    say("case sweep q=1 vs all")
    a = pr_problem(daic, pl10k)
    ra = a.run(eps=1e-10, q=1.0, sched="all", rounds_per_check=1)
    b = pr_problem(daic, pl10k)
    rb = b.run(eps=1e-10, q=1.0, sched="sweep", rounds_per_check=1)
    assert ra.converged and rb.converged
    assert ra.stats["rounds"] == rb.stats["rounds"]
    assert ra.stats["pushed_edges"] == rb.stats["pushed_edges"]
    np.testing.assert_allclose(b.get(), a.get(), rtol=1e-12, atol=0)


def test_sweep_needs_fewer_sweeps_than_synchronous_rounds(daic):
    """Later blocks see the updates of earlier blocks in the same sweep (the
    asynchronous order of Eq. async): fewer passes over the edges."""
    say("case sweep passes")
    g = daic_gen.rmat(14, 16, seed=31)
    a = pr_problem(daic, g)
    ra = a.run(eps=1e-8, q=1.0, sched="all")
    b = pr_problem(daic, g)
    P = 8
    rb = b.run(eps=1e-8, q=1.0 / P, sched="sweep")
    assert ra.converged and rb.converged
    sweeps = rb.stats["rounds"] / P
    say("synchronous rounds", ra.stats["rounds"], "sweeps", sweeps)
    assert sweeps <= 0.8 * ra.stats["rounds"]
    assert rb.stats["pushed_edges"] < ra.stats["pushed_edges"]


@pytest.mark.parametrize("state", ["f32_kahan", "f32"])
@pytest.mark.parametrize("q", [0.25, 0.03])
def test_sweep_pagerank_fp32_rmat(daic, state, q):
    """RMAT-15, edge factor 16: hub targets split into several 1024-edge items."""
    say("case sweep fp32 rmat", state, q)
    g = daic_gen.rmat(15, 16, seed=22)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    p = pr_problem(daic, g, state=state)
    assert p.run(eps=1e-6 * g.n / 1e4, q=q, sched="sweep").converged
    rel = np.abs(p.get() - ref).sum() / ref.sum()
    assert rel <= 1e-5, rel


@pytest.mark.parametrize("q", [1.0, 0.3, 0.05])
def test_sweep_stopped_inside_a_sweep_is_consistent(daic, q):
    """After max_rounds rounds (a round is one block, so most limits stop
    inside a sweep) the messages in flight are delivered: v + dv = c + M^T v
    per vertex, and sum dv + sum (1 - s_j) v = sum dv1 (PageRank mass)."""
    say("case sweep partial", q)
    g = daic_gen.rmat(13, 8, seed=11)
    d = 0.8
    deg = g.outdeg()
    s = np.where(deg > 0, d, 0.0)
    P = int(np.ceil(1.0 / q)) if q < 1 else 1
    for rounds in sorted({1, 2, 3, P, P + 1, 2 * P + 3}):
        p = pr_problem(daic, g)
        res = p.run(eps=0.0, q=q, sched="sweep", max_rounds=rounds, rounds_per_check=1)
        assert res.stats["rounds"] == rounds
        v, dv = p.get(with_dv=True)
        lhs = dv.sum() + ((1 - s) * v).sum()
        assert abs(lhs - 0.2 * g.n) <= 1e-12 * 0.2 * g.n, (rounds, lhs)
        np.testing.assert_allclose(v + dv, 0.2 + mt_v(g, v, d), rtol=1e-12, atol=1e-12)
        # the reported residual is the exact sum |dv| of the delivered state
        assert abs(res.stats["final_residual"] - np.abs(dv).sum()) <= 1e-12 * np.abs(dv).sum()


def test_sweep_resume_and_switch_schedule(daic, pl10k, pl10k_ref):
    say("case sweep resume")
    p = pr_problem(daic, pl10k)
    r1 = p.run(eps=1e-10, q=0.2, sched="sweep", max_rounds=7, rounds_per_check=1)
    assert r1.status == daic.NOT_CONVERGED
    r2 = p.run(eps=1e-10, q=1.0, sched="all")
    assert r2.converged
    r3 = p.run(eps=1e-11, q=0.1, sched="sweep")
    assert r3.converged
    assert np.abs(p.get() - pl10k_ref).sum() <= 1e-9


def test_sweep_katz_src_scale(daic):
    say("case sweep katz")
    g = daic_gen.rmat(12, 8, seed=41)
    beta = 0.9 / max(1, int(g.outdeg().max()))
    dv1 = np.zeros(g.n)
    dv1[5] = 1.0
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_SRC_SCALE, beta, dv1, eps=1e-15)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_SRC_SCALE, alpha=beta)
    p.set_init(np.zeros(g.n), dv1)
    assert p.run(eps=1e-13, q=0.1, sched="sweep").converged
    assert np.abs(p.get() - ref).sum() <= 1e-11


@pytest.mark.parametrize("state", ["f64", "f32_kahan"])
def test_sweep_edge_scale_weights(daic, state):
    say("case sweep edge scale", state)
    g = daic_gen.rmat(12, 8, seed=51)
    w = daic_gen.lognormal_f64(52, g.m, 0.4, 0.8)
    deg = g.outdeg()
    rs = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
    rs = np.where(deg > 0, rs, 1.0)
    a = 0.85 / rs
    c = daic_gen.lognormal_f64(53, g.n, 0.0, 1.0)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 0.0, c, w=w, alpha_pv=a, eps=1e-13)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE, alpha_pv=a, state=state)
    p.set_init(np.zeros(g.n), c)
    eps = 1e-11 if state == "f64" else 1e-3
    assert p.run(eps=eps, q=0.15, sched="sweep").converged
    rel = np.abs(p.get() - ref).sum() / np.abs(ref).sum()
    assert rel <= (1e-12 if state == "f64" else 1e-5), rel


def test_sweep_signed_jacobi_solver(daic):
    """Signed coefficients: the sweep's stop test uses an upper bound of the
    pending mass; the returned residual is the exact one after delivery."""
    say("case sweep jacobi")
    from scipy.sparse import random as sprandom

    n = 3000
    rng = np.random.default_rng(3)
    A = sprandom(n, n, density=8.0 / n, random_state=4, format="csr")
    A.data = rng.uniform(-1, 1, A.data.size)
    A.setdiag(0)
    A.eliminate_zeros()
    diag = 2.0 * np.asarray(abs(A).sum(axis=1)).ravel() + 1.0
    b = rng.normal(0, 1, n)
    want = np.linalg.solve(A.toarray() + np.diag(diag), b)
    AT = A.T.tocsr()
    AT.sort_indices()
    src = np.repeat(np.arange(n), np.diff(AT.indptr))
    dst = AT.indices
    w = -AT.data / diag[dst]
    order = np.lexsort((dst, src))
    g = daic_gen.from_edges(n, src[order], dst[order])
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w[order].astype(np.float64)), daic.SUM,
                     daic.G_EDGE_SCALE, alpha=1.0, state="f64")
    p.set_init(np.zeros(n), b / diag)
    res = p.run(eps=1e-12, q=0.07, sched="sweep")
    assert res.converged and res.stats["final_residual"] <= 1e-12
    np.testing.assert_allclose(p.get(), want, rtol=0, atol=1e-10)


def test_sweep_edge_cases(daic):
    say("case sweep edge cases")
    # one vertex, no edges; one vertex with a self-loop
    g = daic_gen.from_edges(1, [], [])
    p = pr_problem(daic, g)
    assert p.run(eps=0.0, q=0.5, sched="sweep").converged
    np.testing.assert_allclose(p.get(), [0.2])
    g = daic_gen.from_edges(1, [0], [0])
    p = pr_problem(daic, g)
    assert p.run(eps=1e-14, q=1.0, sched="sweep").converged
    np.testing.assert_allclose(p.get(), [1.0], atol=1e-13)
    # edgeless ragged graph, one vertex per block
    g = daic_gen.from_edges(777, [], [])
    p = pr_problem(daic, g)
    assert p.run(eps=0.0, q=1e-9, sched="sweep").converged
    np.testing.assert_allclose(p.get(), 0.2)
    # directed cycle of ragged length: v = 1 everywhere
    n = 1000003 % 4099 + 300
    g = daic_gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    p = pr_problem(daic, g)
    assert p.run(eps=1e-12, q=0.037, sched="sweep").converged
    np.testing.assert_allclose(p.get(), 1.0, atol=1e-12)
    # a hub with more in-edges than one 1024-edge item, and out-edges to all
    n = 5000
    src = np.zeros(n - 1, dtype=np.int64)
    dst = np.arange(1, n)
    g = daic_gen.from_edges(n, np.concatenate([src, dst]), np.concatenate([dst, np.zeros(n - 1)]))
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(n, 0.2), eps=1e-14)
    for q in (1.0, 0.5, 0.02):
        p = pr_problem(daic, g)
        assert p.run(eps=1e-12, q=q, sched="sweep").converged
        assert np.abs(p.get() - ref).sum() <= 1e-12 * ref.sum()


def test_sweep_rejects_min_problems(daic):
    say("case sweep rejects min")
    g = daic_gen.rmat(8, 4, seed=2)
    w = daic_gen.sssp_weights(g.m, seed=3)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
    p.set_init(*oracle.sssp_init(g.n, 0))
    with pytest.raises(daic.DaicError):
        p.run(q=0.5, sched="sweep")


@pytest.mark.parametrize("q", [1.0, 0.3, 0.25, 0.0625, 0.05])
def test_sweep_trajectory_matches_block_oracle(daic, q):
    """Round by round, the GPU state (messages in flight delivered) equals the
    oracle's block-sequential DAIC with the same blocks: checks the order of
    updates and that every message is delivered exactly once. Blocks of 4,096,
    1,024 and 256 ids are whole partitions of the tiled in-edges (pulled
    through the tiles), the others take the streamed pull."""
    say("case sweep trajectory", q)
    g = daic_gen.rmat(12, 16, seed=71)
    d = 0.8
    v0, dv1 = oracle.pagerank_init(g.n, d)
    B = max(1, int(np.ceil(q * g.n)))
    P = -(-g.n // B)
    for rounds in sorted({1, 2, P, P + 1, 3 * P + 2}):
        p = pr_problem(daic, g)
        p.run(eps=0.0, q=q, sched="sweep", max_rounds=rounds, rounds_per_check=1)
        v, dv = p.get(with_dv=True)
        vo, dvo = oracle.sweep_blocks(g, oracle.G_DEG_SCALE, d, v0, dv1, B, rounds)
        np.testing.assert_allclose(v, vo, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(dv, dvo, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("B", [300, 512])
def test_sweep_trajectory_edge_scale(daic, B):
    """As above with per-source coefficients and edge weights; 512-id blocks
    take the tiled pull (weights in the tiles' in-edge order)."""
    say("case sweep trajectory edge scale", B)
    g = daic_gen.rmat(11, 8, seed=72)
    w = daic_gen.lognormal_f64(73, g.m, 0.4, 0.8)
    deg = g.outdeg()
    rs = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
    a = 0.85 / np.where(deg > 0, rs, 1.0)
    c = daic_gen.lognormal_f64(74, g.n, 0.0, 1.0)
    for rounds in (3, 8, 21):
        p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE, alpha_pv=a, state="f64")
        p.set_init(np.zeros(g.n), c)
        p.run(eps=0.0, q=B / g.n, sched="sweep", max_rounds=rounds, rounds_per_check=1)
        v, dv = p.get(with_dv=True)
        vo, dvo = oracle.sweep_blocks(g, oracle.G_EDGE_SCALE, 0.0, np.zeros(g.n), c, B, rounds, w=w, alpha_pv=a)
        np.testing.assert_allclose(v, vo, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(dv, dvo, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("state", ["f32_kahan", "f64"])
def test_sweep_tiled_matches_streamed(daic, monkeypatch, state):
    """The tiled pull of sweep blocks (RMAT-16, 8 blocks of 8,192 ids) against
    the streamed pull: the same rounds, vertex updates and messages, states
    equal to rounding, and both within the tolerance of the oracle."""
    say("case sweep tiled vs streamed", state)
    g = daic_gen.rmat(16, 16, seed=75)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    eps = 1e-10 if state == "f64" else 1e-6
    out = []
    for tiled in (False, True):
        if tiled:
            monkeypatch.delenv("DAIC_NO_TILE", raising=False)
        else:
            monkeypatch.setenv("DAIC_NO_TILE", "1")
        p = pr_problem(daic, g, state=state)
        r = p.run(eps=eps, q=0.125, sched="sweep", rounds_per_check=8)
        assert r.converged
        out.append((r, p.get()))
    (ra, va), (rb, vb) = out
    for key in ("rounds", "activations", "pushed_edges"):
        assert rb.stats[key] == ra.stats[key], (key, ra.stats, rb.stats)
    tol = 1e-12 if state == "f64" else 2e-6
    assert np.abs(vb - va).sum() <= tol * np.abs(va).sum()
    bound = 1e-9 if state == "f64" else 1e-5 * ref.sum()
    assert np.abs(vb - ref).sum() <= bound


@pytest.mark.parametrize("state", ["f32_kahan", "f64"])
def test_sweep_tile_sizes_agree(daic, monkeypatch, state):
    """Tiled sweeps (RMAT-16, 4 blocks) with the default tiles (a CU's share
    of each block's in-edges), with one tile per partition (share 1: nothing
    split) and with tiles of at most 2,048 in-edges (most partitions split,
    slots added by the finishing kernel): the same rounds, vertex updates and
    messages, states equal to rounding, within the oracle's tolerance."""
    say("case sweep tile sizes", state)
    g = daic_gen.rmat(16, 16, seed=76)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    eps = 1e-10 if state == "f64" else 1e-6
    out = []
    for share, edges in ((None, None), ("1", None), (None, "2048")):
        for key, val in (("DAIC_SWEEP_TILE_SHARE", share), ("DAIC_SWEEP_TILE_EDGES", edges)):
            if val is None:
                monkeypatch.delenv(key, raising=False)
            else:
                monkeypatch.setenv(key, val)
        p = pr_problem(daic, g, state=state)  # a new problem builds its sweep tiles
        r = p.run(eps=eps, q=0.25, sched="sweep", rounds_per_check=8)
        assert r.converged
        out.append((r, p.get()))
    monkeypatch.delenv("DAIC_SWEEP_TILE_SHARE", raising=False)
    monkeypatch.delenv("DAIC_SWEEP_TILE_EDGES", raising=False)
    ra, va = out[0]
    tol = 1e-12 if state == "f64" else 2e-6
    for rb, vb in out[1:]:
        for key in ("rounds", "activations", "pushed_edges"):
            assert rb.stats[key] == ra.stats[key], (key, ra.stats, rb.stats)
        assert np.abs(vb - va).sum() <= tol * np.abs(va).sum()
    bound = 1e-9 if state == "f64" else 1e-5 * ref.sum()
    for _, v in out:
        assert np.abs(v - ref).sum() <= bound
