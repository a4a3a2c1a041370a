"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances:
* integer (+) (SSSP min, components max): bit-exact, three repeats;
* FP64 sum problems: L1 distance to the oracle's fixed point <= 1e-9, with the
  GPU stopped at residual 1e-10 (bound r/(1-d) = 5e-10 for d = 0.8) and the
  oracle at 1e-13;
* FP32 paths: relative L1 <= 1e-5 against the FP64 oracle.
Every case is seeded; sizes span many blocks of the per-vertex kernels, end on
a ragged tail, and include hubs split into several large-bin chunks.
"""
import os
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


def pr_problem(daic, g, d, state="f64"):
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=d, state=state)
    v0, dv1 = oracle.pagerank_init(g.n, d)
    p.set_init(v0, dv1)
    return p


@pytest.fixture(scope="module")
def pl10k():
    return daic_gen.powerlaw(n=10000, seed=1)


@pytest.fixture(scope="module")
def pl10k_ref(pl10k):
    v, _, _ = oracle.jacobi_sum(pl10k, oracle.G_DEG_SCALE, 0.8, np.full(pl10k.n, 0.2), eps=1e-13)
    return v


@pytest.mark.parametrize("sched,q", [("all", 1.0), ("sampled", 0.1), ("exact", 0.1),
                                     ("sampled", 0.01), ("exact", 0.5)])
def test_pagerank_f64_powerlaw10k(daic, pl10k, pl10k_ref, sched, q):
    say("case pagerank f64 powerlaw10k", sched, q)
    p = pr_problem(daic, pl10k, 0.8)
    res = p.run(eps=1e-10, q=q, sched=sched, max_rounds=100000, seed=7)
    assert res.converged
    v = p.get()
    err = np.abs(v - pl10k_ref).sum()
    assert err <= 1e-9, err
    assert err <= res.stats["final_residual"] / (1 - 0.8) + 1e-12
    assert res.stats["final_residual"] <= 1e-10


def test_pagerank_f64_timed_config_bound(daic, pl10k, pl10k_ref):
    """The timed run stops at sum|dv| < 1e-9: error within r/(1-d)."""
    say("case pagerank f64 stop 1e-9")
    p = pr_problem(daic, pl10k, 0.8)
    res = p.run(eps=1e-9, q=1.0, sched="all")
    err = np.abs(p.get() - pl10k_ref).sum()
    assert err <= res.stats["final_residual"] / 0.2 + 1e-12


@pytest.mark.parametrize("state", ["f32_kahan", "f32"])
@pytest.mark.parametrize("sched,q", [("all", 1.0), ("sampled", 0.1)])
def test_pagerank_fp32_relative_l1(daic, pl10k, pl10k_ref, state, sched, q):
    say("case pagerank", state, sched, q)
    p = pr_problem(daic, pl10k, 0.8, state=state)
    res = p.run(eps=1e-6, q=q, sched=sched, seed=3)
    assert res.converged
    v = p.get()
    rel = np.abs(v - pl10k_ref).sum() / np.abs(pl10k_ref).sum()
    assert rel <= 1e-5, rel


def test_mass_conservation_partial_runs(daic):
    """sum dv + sum (1 - s_j) v = sum dv1 after any number of rounds."""
    say("case mass conservation")
    g = daic_gen.rmat(14, 8, seed=11)
    d = 0.8
    deg = g.outdeg()
    s = np.where(deg > 0, d, 0.0)
    for sched, q in (("all", 1.0), ("sampled", 0.05), ("exact", 0.2)):
        p = pr_problem(daic, g, d)
        for rounds in (1, 2, 5):
            p.run(eps=0.0, q=q, sched=sched, max_rounds=rounds, rounds_per_check=1, seed=5)
            v, dv = p.get(with_dv=True)
            lhs = dv.sum() + ((1 - s) * v).sum()
            assert abs(lhs - 0.2 * g.n) <= 1e-12 * 0.2 * g.n, (sched, rounds, lhs)


@pytest.mark.parametrize("scale,ef,seed", [(12, 8, 21), (15, 16, 22)])
def test_pagerank_rmat_f64_and_kahan(daic, scale, ef, seed):
    say("case pagerank rmat", scale, ef)
    g = daic_gen.rmat(scale, ef, seed=seed)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    p = pr_problem(daic, g, 0.8)
    assert p.run(eps=1e-10, q=1.0, sched="all").converged
    assert np.abs(p.get() - ref).sum() <= 1e-9
    pk = pr_problem(daic, g, 0.8, state="f32_kahan")
    assert pk.run(eps=1e-6 * g.n / 1e4, q=1.0, sched="all").converged
    assert np.abs(pk.get() - ref).sum() / ref.sum() <= 1e-5


@pytest.mark.parametrize("state,gk", [("f32_kahan", "deg"), ("f64", "edge_pv"), ("f32", "edge")])
def test_ranked_tiles_match_id_tiles(daic, monkeypatch, state, gk):
    """Fused dense rounds walk tiles whose targets are numbered by in-degree
    octave (highest first, ids ascending within an octave), with v, dv (and
    the Kahan term) moved into that order while they run.
    Against the same rounds over partitions of consecutive ids: the same
    round, update and message counts and the same state to rounding, after a
    stop by the round limit (the state must be back in vertex order), after
    resuming from it, and at convergence, which the oracle's FP64 iteration
    checks. RMAT-16 with edge factor 16: its hub partition is cut into
    several tiles."""
    say("case ranked vs id tiles", state, gk)
    monkeypatch.delenv("DAIC_NO_TILE", raising=False)
    g = daic_gen.rmat(16, 16, seed=43)
    rng = np.random.default_rng(44)
    n = g.n
    outdeg = np.diff(g.row_ptr).astype(np.float64)
    src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
    w = a_pv = None
    if gk != "deg":
        w = rng.uniform(0.1, 1.0, g.m) / np.maximum(outdeg[src], 1.0)
        w = w.astype(np.float64 if state == "f64" else np.float32)
    if gk == "edge_pv":
        a_pv = rng.uniform(0.5, 0.9, n)
    alpha = 0.85
    dv1 = rng.uniform(0.0, 0.3, n)

    def make():
        G = daic.Graph(g.row_ptr, g.col, w)
        kwp = dict(alpha_pv=a_pv) if a_pv is not None else dict(alpha=alpha)
        P = daic.Problem(G, daic.SUM, daic.G_DEG_SCALE if gk == "deg" else daic.G_EDGE_SCALE, state=state, **kwp)
        P.set_init(np.zeros(n), dv1)
        return P

    eps = 1e-10 if state == "f64" else 1e-5
    kw = dict(eps=eps, q=1.0, sched="all", rounds_per_check=4)
    runs = {}
    for order in ("id", "ranked"):
        if order == "id":
            monkeypatch.setenv("DAIC_TILE_ID_ORDER", "1")
        else:
            monkeypatch.delenv("DAIC_TILE_ID_ORDER", raising=False)
        P = make()
        r1 = P.run(max_rounds=6, **kw)
        s1 = P.get(with_dv=True)
        r2 = P.run(**kw)  # resumes from the stopped state
        runs[order] = (r1, s1, r2, P.get(with_dv=True))
    (a1, sa1, a2, sa2), (b1, sb1, b2, sb2) = runs["id"], runs["ranked"]
    for x, y in ((a1, b1), (a2, b2)):
        for k in ("rounds", "activations", "pushed_edges"):
            assert x.stats[k] == y.stats[k], (k, x.stats, y.stats)
    assert not b1.converged and b2.converged
    tol = 1e-12 if state == "f64" else 2e-6
    for (va, dva), (vb, dvb) in ((sa1, sb1), (sa2, sb2)):
        scale = np.abs(va).sum()
        assert np.abs(vb - va).sum() <= tol * scale
        assert np.abs(dvb - dva).sum() <= tol * max(scale, 1.0)
    d = alpha if a_pv is None else 0.0
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE if gk != "deg" else oracle.G_DEG_SCALE, d, dv1,
                                  w=w.astype(np.float64) if w is not None else None, alpha_pv=a_pv, eps=1e-13)
    vb = sb2[0]
    assert np.abs(vb - ref).sum() <= (1e-9 if state == "f64" else 1e-5) * np.abs(ref).sum()
    # daic_profile runs the fused rounds eagerly and must hand the state back
    # in vertex order too
    P = make()
    rp, _ = P.profile(**kw)
    vp, dvp = P.get(with_dv=True)
    assert rp.stats["rounds"] == a2.stats["rounds"] + a1.stats["rounds"]
    assert np.abs(vp - vb).sum() <= tol * np.abs(vb).sum()
    assert np.abs(dvp - sb2[1]).sum() <= tol * max(np.abs(vb).sum(), 1.0)


@pytest.mark.parametrize("tiled", [True, False])
@pytest.mark.parametrize("state,gk", [("f32_kahan", "deg"), ("f64", "deg"), ("f32", "edge")])
def test_fused_dense_rounds_match_plain_rounds(daic, monkeypatch, state, gk, tiled):
    """Dense rounds with every pending vertex run as one fused kernel per
    round (pull, then the claim work of the next round). They must give the
    plain rounds' state after the same number of rounds, with the same work
    counters: to convergence and when stopped by the round limit. RMAT-16
    with edge factor 16 has targets with more than 2,048 in-edges, which the
    fused round finishes through per-group tickets. tiled: the fused round
    walks partitions of 16,384 targets in source order (one gather per
    source and partition); RMAT-16 has partitions cut into several tiles,
    whose partial sums a finishing kernel adds."""
    say("case fused vs plain", state, gk, "tiled", tiled)
    if not tiled:
        monkeypatch.setenv("DAIC_NO_TILE", "1")
    else:
        monkeypatch.delenv("DAIC_NO_TILE", raising=False)
    g = daic_gen.rmat(16, 16, seed=41)
    indeg = np.bincount(g.col, minlength=g.n)
    assert indeg.max() > 2048
    rng = np.random.default_rng(42)
    w = rng.uniform(0.1, 1.0, g.m).astype(np.float32) if gk == "edge" else None
    if w is not None:  # column-stochastic-like scaling: sum of weights per source <= 1
        outdeg = np.diff(g.row_ptr).astype(np.float64)
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr).astype(np.int64))
        w = (w / np.maximum(outdeg[src], 1.0)).astype(np.float32)

    def make():
        G = daic.Graph(g.row_ptr, g.col, w)
        P = daic.Problem(G, daic.SUM, daic.G_EDGE_SCALE if w is not None else daic.G_DEG_SCALE,
                         alpha=0.85, state=state)
        P.set_init(np.zeros(g.n), np.full(g.n, 0.15))
        return P

    for max_rounds in (7, 0):
        kw = dict(eps=1e-9 if state == "f64" else 1e-5, q=1.0, sched="all", rounds_per_check=4,
                  max_rounds=max_rounds)
        monkeypatch.setenv("DAIC_NO_FUSE", "1")
        a = make()
        ra = a.run(**kw)
        va, dva = a.get(with_dv=True)
        monkeypatch.delenv("DAIC_NO_FUSE")
        b = make()
        rb = b.run(**kw)
        vb, dvb = b.get(with_dv=True)
        assert rb.stats["rounds"] == ra.stats["rounds"], (max_rounds, rb.stats, ra.stats)
        if max_rounds:
            assert rb.stats["rounds"] == max_rounds and not rb.converged
        assert rb.stats["activations"] == ra.stats["activations"]
        assert rb.stats["pushed_edges"] == ra.stats["pushed_edges"]
        tol = 1e-12 if state == "f64" else 2e-6
        assert np.abs(vb - va).sum() <= tol * np.abs(va).sum()
        assert np.abs(dvb - dva).sum() <= tol * max(np.abs(va).sum(), 1.0)
        assert abs(rb.stats["final_residual"] - ra.stats["final_residual"]) <= tol * np.abs(va).sum()


@pytest.mark.parametrize("graph", ["rmat16", "powerlaw10k"])
@pytest.mark.parametrize("kind", ["sssp_u32", "sssp_f64", "cc_i32"])
@pytest.mark.parametrize("sched,q", [("all", 1.0), ("exact", 0.1), ("sampled", 0.1)])
def test_minmax_dense_rounds_match_push(daic, monkeypatch, graph, kind, sched, q):
    """Dense rounds of min and max problems (the tiled pull with LDS atomic
    min/max) against push-only rounds: the same rounds, vertex updates and
    messages, and the same state bit for bit (min and max are exact), and the
    oracle's answer. RMAT-16 has split partitions; the all-pending SSSP run
    takes several dense rounds in its middle. The 10,000-vertex power-law
    graph ends in a partial partition (10,000 = 9 x 1,024 + 784)."""
    say("case minmax dense vs push", graph, kind, sched, q)
    g = daic_gen.rmat(16, 16, seed=47) if graph == "rmat16" else daic_gen.powerlaw(n=10000, seed=48)
    if kind == "cc_i32":
        src = np.repeat(np.arange(g.n), g.outdeg())
        g = daic_gen.from_edges(g.n, np.concatenate([src, g.col.astype(np.int64)]),
                                np.concatenate([g.col.astype(np.int64), src]))
    w = None
    if kind == "sssp_u32":
        w = daic_gen.sssp_weights(g.m, seed=48)
        ref = oracle.dijkstra(g, w, 0)
    elif kind == "sssp_f64":
        w = daic_gen.lognormal_f64(49, g.m, 0.0, 1.0)
        ref = oracle.dijkstra_f64(g, w, 0)
    else:
        ref = oracle.maxlabel(g)

    def make():
        G = daic.Graph(g.row_ptr, g.col, w)
        if kind == "cc_i32":
            P = daic.Problem(G, daic.MAX, daic.G_COPY, state="i32")
            P.set_init(*oracle.cc_init(g.n))
        else:
            P = daic.Problem(G, daic.MIN, daic.G_EDGE_ADD, state="u32" if kind == "sssp_u32" else "f64")
            v0 = np.full(g.n, 0xFFFFFFFF if kind == "sssp_u32" else np.inf)
            dv1 = v0.copy()
            dv1[0] = 0
            P.set_init(v0.astype(np.uint32) if kind == "sssp_u32" else v0, dv1.astype(np.uint32) if kind == "sssp_u32" else dv1)
        return P

    out = []
    for push_only in (True, False):
        if push_only:
            monkeypatch.setenv("DAIC_NO_PULL", "1")
        else:
            monkeypatch.delenv("DAIC_NO_PULL", raising=False)
        P = make()
        r = P.run(q=q, sched=sched, rounds_per_check=4)
        assert r.converged
        out.append((r, P.get()))
        if not push_only:
            rp, ks = make().profile(q=q, sched=sched)
            names = {k["name"]: k for k in ks}
            say("  dense rounds", names.get("pull_tile", {}).get("launches", 0), "of", rp.stats["rounds"])
            # min and max problems take dense rounds through the tiles only
            if sched == "all" and graph == "rmat16" and not os.environ.get("DAIC_NO_TILE"):
                assert names["pull_tile"]["launches"] >= 1
    (ra, va), (rb, vb) = out
    for key in ("rounds", "activations", "pushed_edges"):
        assert rb.stats[key] == ra.stats[key], (key, ra.stats, rb.stats)
    np.testing.assert_array_equal(vb, va)
    np.testing.assert_array_equal(vb, ref)


@pytest.mark.parametrize("state,gk", [("f32_kahan", "deg"), ("f64", "deg"), ("f32", "edge")])
def test_tiled_unfused_dense_rounds_match_streamed(daic, monkeypatch, state, gk):
    """Dense rounds that are not fused (the claim folds and publishes, the
    pull adds into dv) through the tiled in-edges against the streamed pull:
    the same rounds, updates and messages, and the same state, to
    convergence and when stopped by the round limit. RMAT-16 has split
    partitions; the run also decides the direction of every next round from
    the tiled pull's pending count."""
    say("case tiled unfused", state, gk)
    monkeypatch.setenv("DAIC_NO_FUSE", "1")
    g = daic_gen.rmat(16, 16, seed=43)
    rng = np.random.default_rng(44)
    w = None
    if gk == "edge":
        outdeg = np.diff(g.row_ptr).astype(np.float64)
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr).astype(np.int64))
        w = (rng.uniform(0.1, 1.0, g.m) / np.maximum(outdeg[src], 1.0)).astype(np.float32)

    def make():
        P = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM,
                         daic.G_EDGE_SCALE if w is not None else daic.G_DEG_SCALE, alpha=0.85, state=state)
        P.set_init(np.zeros(g.n), np.full(g.n, 0.15))
        return P

    for max_rounds in (9, 0):
        kw = dict(eps=1e-9 if state == "f64" else 1e-5, q=1.0, sched="all", rounds_per_check=4,
                  max_rounds=max_rounds)
        out = []
        for tiled in (False, True):
            if tiled:
                monkeypatch.delenv("DAIC_NO_TILE", raising=False)
            else:
                monkeypatch.setenv("DAIC_NO_TILE", "1")
            P = make()
            r = P.run(**kw)
            out.append((r, *P.get(with_dv=True)))
        (ra, va, dva), (rb, vb, dvb) = out
        for key in ("rounds", "activations", "pushed_edges"):
            assert rb.stats[key] == ra.stats[key], (key, max_rounds, ra.stats, rb.stats)
        tol = 1e-12 if state == "f64" else 2e-6
        assert np.abs(vb - va).sum() <= tol * np.abs(va).sum()
        assert np.abs(dvb - dva).sum() <= tol * max(np.abs(va).sum(), 1.0)


@pytest.mark.parametrize("kind", ["pagerank_f64", "pagerank_f32_kahan", "sssp_u32", "cc_i32"])
def test_tile_sizes_agree(daic, monkeypatch, kind):
    """The tiled dense rounds with tiles of at most 2,048 in-edges (almost
    every partition split, hundreds of slots per hub partition, the launch
    order largest first), with the default size, and with one tile per
    partition (nothing split): the same rounds, updates and messages, the
    same min/max state bit for bit and the same sum state to rounding (the
    tiles change the order of the FP64 additions), and the sum states within
    the oracle's bound."""
    say("case tile sizes", kind)
    g = daic_gen.rmat(16, 16, seed=47)
    w = daic_gen.sssp_weights(g.m, seed=48) if kind == "sssp_u32" else None
    out = []
    for te in ("2048", None, "1073741824"):
        if te is None:
            monkeypatch.delenv("DAIC_TILE_EDGES", raising=False)
        else:
            monkeypatch.setenv("DAIC_TILE_EDGES", te)
        G = daic.Graph(g.row_ptr, g.col, w)  # the tiles are built per graph
        if kind.startswith("pagerank"):
            P = daic.Problem(G, daic.SUM, daic.G_DEG_SCALE, alpha=0.85, state=kind.split("_", 1)[1])
            P.set_init(np.zeros(g.n), np.full(g.n, 0.15))
            kw = dict(eps=1e-10 if kind == "pagerank_f64" else 1e-6, q=1.0, sched="all", rounds_per_check=4)
        elif kind == "sssp_u32":
            P = daic.Problem(G, daic.MIN, daic.G_EDGE_ADD, state="u32")
            v0, dv1 = oracle.sssp_init(g.n, 0)
            P.set_init(v0, dv1)
            kw = dict(q=1.0, sched="all", rounds_per_check=4)
        else:
            P = daic.Problem(G, daic.MAX, daic.G_COPY, state="i32")
            v0, dv1 = oracle.cc_init(g.n)
            P.set_init(v0, dv1)
            kw = dict(q=1.0, sched="all", rounds_per_check=4)
        r = P.run(**kw)
        assert r.converged, (te, r.stats)
        out.append((r, P.get()))
    monkeypatch.delenv("DAIC_TILE_EDGES", raising=False)
    ra, va = out[1]
    for rb, vb in (out[0], out[2]):
        for key in ("rounds", "activations", "pushed_edges"):
            assert rb.stats[key] == ra.stats[key], (kind, key, ra.stats, rb.stats)
        if kind in ("sssp_u32", "cc_i32"):
            assert np.array_equal(vb, va)
        else:
            tol = 1e-12 if kind == "pagerank_f64" else 2e-6
            assert np.abs(vb - va).sum() <= tol * np.abs(va).sum()
    if kind.startswith("pagerank"):
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.85, np.full(g.n, 0.15), eps=1e-13)
        for _, v in out:
            if kind == "pagerank_f64":
                assert np.abs(v - ref).sum() <= 1e-10 / (1 - 0.85) * 1.01
            else:
                assert np.abs(v - ref).sum() <= 1e-5 * np.abs(ref).sum()
    elif kind == "sssp_u32":
        assert np.array_equal(out[1][1], oracle.dijkstra(g, w, 0))
    else:
        assert np.array_equal(out[1][1], oracle.maxlabel(g))


@pytest.mark.parametrize("n,ef", [(5, 2), (300, 3), (3000, 6)])
def test_fused_pull_small_graphs(daic, monkeypatch, n, ef):
    """Fused dense rounds on graphs with fewer edge blocks than the grid
    would take: the same rounds and state as unfused rounds."""
    say("case fused small", n, ef)
    rng = np.random.default_rng(n)
    src, dst = rng.integers(0, n, n * ef), rng.integers(0, n, n * ef)
    g = daic_gen.from_edges(n, src, dst)
    out = []
    for fuse in (False, True):
        if fuse:
            monkeypatch.delenv("DAIC_NO_FUSE", raising=False)
        else:
            monkeypatch.setenv("DAIC_NO_FUSE", "1")
        p = pr_problem(daic, g, 0.85, state="f64")
        r = p.run(eps=1e-12, q=1.0, sched="all", rounds_per_check=4)
        assert r.converged
        out.append((r.stats["rounds"], p.get()))
    monkeypatch.delenv("DAIC_NO_FUSE", raising=False)
    assert out[0][0] == out[1][0]
    assert np.abs(out[0][1] - out[1][1]).sum() <= 1e-12 * np.abs(out[0][1]).sum()
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.85, np.full(n, 0.15), eps=1e-14)
    assert np.abs(out[1][1] - ref).sum() <= 1e-9


def test_profile_matches_run_and_accounts_the_pull(daic, monkeypatch):
    """daic_profile (the source of the benchmark's roofline) runs the same
    rounds as daic_run, to the same state, and reports every dense round's
    pull over all m in-edges: the fused kernel under all-pending scheduling,
    the streamed pull with the claim and the pull's finishing kernel (which
    takes the residual's place after a dense round) otherwise."""
    say("case profile accounting")
    g = daic_gen.rmat(14, 8, seed=51)
    for fuse in (True, False):
        if fuse:
            monkeypatch.delenv("DAIC_NO_FUSE", raising=False)
        else:
            monkeypatch.setenv("DAIC_NO_FUSE", "1")
        a = pr_problem(daic, g, 0.85, state="f32_kahan")
        ra = a.run(eps=1e-6, q=1.0, sched="all")
        b = pr_problem(daic, g, 0.85, state="f32_kahan")
        rb, ks = b.profile(eps=1e-6, q=1.0, sched="all")
        assert ra.converged and rb.converged
        assert rb.stats["rounds"] == ra.stats["rounds"]
        assert rb.stats["pushed_edges"] == ra.stats["pushed_edges"]
        va, vb = a.get(), b.get()
        assert np.abs(va - vb).sum() <= 2e-6 * np.abs(va).sum()
        names = {k["name"]: k for k in ks}
        if fuse and not os.environ.get("DAIC_NO_GRAPH"):  # eager rounds (DAIC_NO_GRAPH=1) are not fused
            pull = names["tile_pull" if "tile_pull" in names else "pull_fused"]
        else:
            pull = names["pull_tile" if "pull_tile" in names else "pull_stream"]
        assert pull["launches"] == rb.stats["rounds"]
        assert pull["edges"] == pull["launches"] * g.m
        # the streamed pull reads a source and a base per in-edge; the tiled
        # one a 2-byte target per in-edge and a source and base per pair
        per_edge = 2 if pull["name"] in ("tile_pull", "pull_tile") else 8
        assert pull["alg_bytes"] >= pull["edges"] * per_edge and pull["total_ms"] > 0
        if not fuse:
            fin = "pull_tile_total" if "pull_tile" in names else "pull_finish"
            assert {"claim", fin} <= set(names)
            assert names[fin]["launches"] == pull["launches"]
            # a residual launch is counted only after a sparse round
            assert names.get("residual", {"launches": 0})["launches"] == rb.stats["rounds"] - pull["launches"]


def sssp_case(g, wseed, source=0):
    w = daic_gen.sssp_weights(g.m, seed=wseed)
    return w, oracle.dijkstra(g, w, source)


@pytest.mark.parametrize("scale", [10, 16])
@pytest.mark.parametrize("sched,q", [("all", 1.0), ("sampled", 0.1), ("exact", 0.1)])
def test_sssp_bit_exact(daic, scale, sched, q):
    say("case sssp rmat", scale, sched, q)
    g = daic_gen.rmat(scale, 16, seed=100 + scale)
    w, ref = sssp_case(g, 3)
    gg = daic.Graph(g.row_ptr, g.col, w)
    for rep in range(3):
        p = daic.Problem(gg, daic.MIN, daic.G_EDGE_ADD, state="u32")
        v0, dv1 = oracle.sssp_init(g.n, 0)
        p.set_init(v0, dv1)
        res = p.run(q=q, sched=sched, seed=rep)
        assert res.converged
        np.testing.assert_array_equal(p.get(), ref)
        assert res.stats["final_residual"] == 0


def test_sssp_rmat20_full_config(daic):
    """The single-source shortest-path workload at full size: RMAT scale 20,
    edge factor 16, weights U{1..255}, source 0, q = 0.1 (sampled)."""
    say("case sssp rmat20 full")
    g = daic_gen.rmat(20, 16, seed=2)
    w, ref = sssp_case(g, 3)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
    v0, dv1 = oracle.sssp_init(g.n, 0)
    p.set_init(v0, dv1)
    res = p.run(q=0.1, sched="sampled", seed=1)
    assert res.converged
    np.testing.assert_array_equal(p.get(), ref)


def sssp_f64_problem(daic, g, w, source=0):
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="f64")
    v0 = np.full(g.n, np.inf)
    dv1 = np.full(g.n, np.inf)
    dv1[source] = 0.0
    p.set_init(v0, dv1)
    return p


@pytest.mark.parametrize("graph", ["rmat16", "paper_lognormal"])
@pytest.mark.parametrize("sched,q", [("all", 1.0), ("sampled", 0.1), ("exact", 0.1)])
def test_sssp_f64_lognormal_weights_bit_exact(daic, graph, sched, q):
    """SSSP with the paper's real log-normal(0, 1) edge weights (Sec. 6.1) in
    FP64: min over d(u) + w(u, v) is exact in the sense that every path sum
    is formed once, left to right, so the fixed point equals the heap
    Dijkstra's distances bit for bit."""
    say("case sssp f64", graph, sched, q)
    if graph == "rmat16":
        g = daic_gen.rmat(16, 16, seed=81)
    else:
        g = daic_gen.paper_lognormal(20000, seed=82)
    w = daic_gen.lognormal_f64(83, g.m, 0.0, 1.0)
    ref = oracle.dijkstra_f64(g, w, 0)
    for _ in range(2):
        p = sssp_f64_problem(daic, g, w)
        res = p.run(q=q, sched=sched, seed=3)
        assert res.converged
        got = p.get()
        np.testing.assert_array_equal(got, ref)
    # weights stored as float32 are widened to double first
    w32 = w.astype(np.float32)
    p = sssp_f64_problem(daic, g, w32)
    assert p.run(q=1.0, sched="all").converged
    np.testing.assert_array_equal(p.get(), oracle.dijkstra_f64(g, w32.astype(np.float64), 0))


def test_sssp_f64_rejects_negative_or_nan_weights(daic):
    say("case sssp f64 invalid weights")
    g = daic_gen.rmat(8, 4, seed=2)
    for bad in (-1.0, np.nan):
        w = np.ones(g.m)
        w[g.m // 2] = bad
        with pytest.raises(daic.DaicError):
            daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="f64")


@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("sched,q", [("all", 1.0), ("exact", 0.3)])
def test_components_max_label_bit_exact(daic, symmetric, sched, q):
    say("case cc", symmetric, sched, q)
    g0 = daic_gen.rmat(13, 4, seed=31)
    if symmetric:
        src = np.repeat(np.arange(g0.n), g0.outdeg())
        dst = g0.col.astype(np.int64)
        g = daic_gen.from_edges(g0.n, np.concatenate([src, dst]), np.concatenate([dst, src]))
    else:
        g = g0
    ref = oracle.maxlabel(g)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.MAX, daic.G_COPY, state="i32")
    v0, dv1 = oracle.cc_init(g.n)
    p.set_init(v0, dv1)
    assert p.run(q=q, sched=sched).converged
    np.testing.assert_array_equal(p.get(), ref)


def test_katz_src_scale(daic):
    say("case katz")
    g = daic_gen.rmat(12, 8, seed=41)
    beta = 0.9 / max(1, int(g.outdeg().max()))
    dv1 = np.zeros(g.n)
    dv1[5] = 1.0
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_SRC_SCALE, beta, dv1, eps=1e-15)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_SRC_SCALE, alpha=beta)
    p.set_init(np.zeros(g.n), dv1)
    assert p.run(eps=1e-13, q=1.0, sched="all").converged
    assert np.abs(p.get() - ref).sum() <= 1e-11


@pytest.mark.parametrize("state", ["f64", "f32_kahan"])
def test_edge_scale_adsorption_weights(daic, state):
    say("case edge scale", state)
    g = daic_gen.rmat(12, 8, seed=51)
    w = daic_gen.lognormal_f64(52, g.m, 0.4, 0.8)
    deg = g.outdeg()
    rs = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
    rs = np.where(deg > 0, rs, 1.0)
    a = 0.85 / rs
    c = daic_gen.lognormal_f64(53, g.n, 0.0, 1.0)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 0.0, c, w=w, alpha_pv=a, eps=1e-13)
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE, alpha_pv=a,
                     state=state)
    p.set_init(np.zeros(g.n), c)
    eps = 1e-11 if state == "f64" else 1e-3
    assert p.run(eps=eps, q=1.0, sched="all").converged
    rel = np.abs(p.get() - ref).sum() / np.abs(ref).sum()
    assert rel <= (1e-12 if state == "f64" else 1e-5), rel


def test_edge_cases(daic):
    say("case edge cases")
    # one vertex, no edges
    g = daic_gen.from_edges(1, [], [])
    p = pr_problem(daic, g, 0.8)
    assert p.run(eps=0.0, q=1.0).converged
    np.testing.assert_allclose(p.get(), [0.2])
    # self-loop only: v = 0.2 / (1 - 0.8) = 1
    g = daic_gen.from_edges(1, [0], [0])
    p = pr_problem(daic, g, 0.8)
    assert p.run(eps=1e-14, q=1.0).converged
    np.testing.assert_allclose(p.get(), [1.0], atol=1e-13)
    # edgeless ragged graph
    g = daic_gen.from_edges(777, [], [])
    p = pr_problem(daic, g, 0.8)
    assert p.run(eps=0.0, q=0.01, sched="exact").converged
    np.testing.assert_allclose(p.get(), 0.2)
    # directed cycle of ragged length: v = 1 everywhere
    n = 1000003 % 4099 + 300
    g = daic_gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    p = pr_problem(daic, g, 0.8)
    assert p.run(eps=1e-12, q=1.0).converged
    np.testing.assert_allclose(p.get(), 1.0, atol=1e-12)
    # a single hub with more edges than one large-bin chunk
    n = 5000
    src = np.zeros(n - 1, dtype=np.int64)
    dst = np.arange(1, n)
    g = daic_gen.from_edges(n, np.concatenate([src, dst]), np.concatenate([dst, np.zeros(n - 1)]))
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(n, 0.2), eps=1e-14)
    for sched, q in (("all", 1.0), ("exact", 1e-4), ("sampled", 0.001)):
        p = pr_problem(daic, g, 0.8)
        assert p.run(eps=1e-12, q=q, sched=sched).converged
        # the hub's value is a sum of ~5000 terms on both sides: FP64 rounding
        # of that order, so the bound is relative
        assert np.abs(p.get() - ref).sum() <= 1e-12 * ref.sum()


def test_not_converged_status(daic):
    say("case max rounds")
    g = daic_gen.rmat(12, 8, seed=61)
    p = pr_problem(daic, g, 0.8)
    res = p.run(eps=1e-12, q=1.0, max_rounds=3, rounds_per_check=1)
    assert res.status == daic.NOT_CONVERGED
    assert res.stats["rounds"] == 3
    # resume from the stopped state reaches the same fixed point
    res2 = p.run(eps=1e-10, q=1.0)
    assert res2.converged
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    assert np.abs(p.get() - ref).sum() <= 1e-9


# ---------------------------------------------------------------------------
# Selection kernels against the oracle's rules
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1000, 70001])
@pytest.mark.parametrize("q", [0.001, 0.1, 0.6])
@pytest.mark.parametrize("state", ["f64", "f32", "u32"])
def test_exact_topk_matches_oracle(daic, n, q, state):
    say("case exact topk", n, q, state)
    rng = np.random.default_rng(n + int(q * 1000))
    g = daic_gen.from_edges(n, [], [])
    if state == "u32":
        w = np.ones(0, dtype=np.uint32)
        gg = daic.Graph(g.row_ptr, g.col, w)
        p = daic.Problem(gg, daic.MIN, daic.G_EDGE_ADD, state="u32")
        v = rng.integers(0, 50, n).astype(np.uint32)
        v[rng.random(n) < 0.1] = oracle.INF_U32
        dv = rng.integers(0, 60, n).astype(np.uint32)
        dv[rng.random(n) < 0.3] = oracle.INF_U32
        p.set_init(v, dv)
        pr = oracle.priority(oracle.OP_MIN, v, dv)
    else:
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8,
                         state=state)
        dv = rng.integers(0, 40, n) * 0.125  # many exact ties
        dv[rng.random(n) < 0.2] = 0.0
        dv *= np.where(rng.random(n) < 0.5, -1, 1)
        p.set_init(np.zeros(n), dv)
        pr = np.abs(dv)
    sel, _ = p.select_frontier(q=q, sched="exact")
    want = oracle.topk_exact(pr, q)
    np.testing.assert_array_equal(np.nonzero(sel)[0], want)


@pytest.mark.parametrize("case", ["distinct", "ties_fit", "ties_cut"])
@pytest.mark.parametrize("state", ["f64", "f32"])
def test_exact_topk_tie_forms(daic, case, state):
    """The k-th key alone (distinct keys), its equal keys all inside the k
    (the round takes key >= tau without tie ranks), or cut by the k (ties go
    to the smaller ids), for 64- and 32-bit keys."""
    say("case exact topk ties", case, state)
    n = 100003
    rng = np.random.default_rng(7)
    zero = rng.random(n) < 0.05
    if case == "distinct":
        dv = rng.permutation(n).astype(np.float64) + 1.0
        q = 0.05
    else:
        # 4,000 keys above 10, 1,000 keys equal to 10, the other pending ones below
        dv = rng.uniform(0.5, 9.5, n)
        hi = rng.choice(n, 5000, replace=False)
        dv[hi[:4000]] = rng.uniform(11.0, 20.0, 4000)
        dv[hi[4000:]] = 10.0
        zero[hi] = False
        q = 5000 / n if case == "ties_fit" else 4500 / n
    dv[zero] = 0.0
    if state == "f32":
        dv = dv.astype(np.float32).astype(np.float64)
    g = daic_gen.from_edges(n, [], [])
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8, state=state)
    p.set_init(np.zeros(n), dv)
    sel, _ = p.select_frontier(q=q, sched="exact")
    want = oracle.topk_exact(np.abs(dv), q)
    if case != "distinct":
        assert len(want) == int(np.ceil(q * n)) and (np.abs(dv)[want] >= 10.0).all()
    np.testing.assert_array_equal(np.nonzero(sel)[0], want)


@pytest.mark.parametrize("round_no", [0, 3, 17])
@pytest.mark.parametrize("q", [0.01, 0.1, 1.0])
def test_sampled_threshold_matches_oracle(daic, round_no, q):
    say("case sampled", round_no, q)
    n = 50000
    rng = np.random.default_rng(round_no)
    g = daic_gen.from_edges(n, [], [])
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8,
                     state="f32")
    dv = rng.exponential(1.0, n).astype(np.float32).astype(np.float64)
    dv[rng.random(n) < 0.4] = 0.0
    p.set_init(np.zeros(n), dv)
    sel, tau = p.select_frontier(q=q, sched="sampled", seed=1234, round_no=round_no, n_samples=4096)
    pr = np.abs(dv).astype(np.float32)
    tau_o = oracle.sampled_threshold(pr, q, 4096, 1234, round_no)
    want = (pr >= tau_o) & (pr > 0)
    np.testing.assert_array_equal(sel, want)
    if q < 1.0:
        assert np.float32(tau) == tau_o


@pytest.mark.parametrize("n_samples", [1, 1000, 4096])
@pytest.mark.parametrize("q", [0.01, 0.37])
def test_sampled_threshold_with_ties_matches_oracle(daic, n_samples, q):
    """Sample counts that leave a ragged last workgroup of the ranking
    kernel, and integer priorities, so the threshold sample has many equal
    keys; q * S below 1 takes the largest sample."""
    say("case sampled ties", n_samples, q)
    n = 30011
    rng = np.random.default_rng(n_samples)
    g = daic_gen.from_edges(n, [], [])
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8, state="f64")
    dv = rng.integers(0, 12, n).astype(np.float64)
    p.set_init(np.zeros(n), dv)
    for round_no in (0, 5):
        sel, tau = p.select_frontier(q=q, sched="sampled", seed=99, round_no=round_no, n_samples=n_samples)
        tau_o = oracle.sampled_threshold(dv, q, n_samples, 99, round_no)
        np.testing.assert_array_equal(sel, (dv >= tau_o) & (dv > 0))
        if tau != 0:  # 0: the sample at the rank was not pending, every pending vertex is taken
            assert tau == tau_o


def test_device_graph_from_torch(daic):
    import torch

    say("case device graph")
    g = daic_gen.rmat(12, 8, seed=71)
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    col = torch.from_numpy(g.col.astype(np.int32)).cuda()
    stream = torch.cuda.current_stream()
    gd = daic.Graph.from_device(rp, col, stream=stream)
    p = daic.Problem(gd, daic.SUM, daic.G_DEG_SCALE, alpha=0.8)
    p.set_init(*oracle.pagerank_init(g.n, 0.8))
    assert p.run(eps=1e-10, stream=stream).converged
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    assert np.abs(p.get() - ref).sum() <= 1e-9
    bad = col.clone()
    bad[3] = g.n
    with pytest.raises(daic.DaicError, match="out of range"):
        daic.Graph.from_device(rp, bad, stream=stream)


@pytest.mark.parametrize("direction", ["push_only", "pull_when_dense", "pull_always"])
@pytest.mark.parametrize("state,gk", [("f64", "deg"), ("f32_kahan", "deg"), ("f64", "edge")])
def test_push_and_pull_rounds_agree(daic, monkeypatch, direction, state, gk):
    """Dense rounds (receivers pull over in-edges) and push rounds reach the
    same fixed point: both are legal update sequences of Eq. async."""
    say("case direction", direction, state, gk)
    monkeypatch.delenv("DAIC_NO_PULL", raising=False)
    monkeypatch.delenv("DAIC_PULL_DIV", raising=False)
    if direction == "push_only":
        monkeypatch.setenv("DAIC_NO_PULL", "1")
    elif direction == "pull_always":
        monkeypatch.setenv("DAIC_PULL_DIV", "1000000000")
    g = daic_gen.rmat(13, 16, seed=81)
    if gk == "deg":
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
        p = pr_problem(daic, g, 0.8, state=state)
    else:
        w = daic_gen.lognormal_f64(82, g.m, 0.4, 0.8)
        deg = g.outdeg()
        rs = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
        a = 0.8 / np.where(deg > 0, rs, 1.0)
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 0.0, np.full(g.n, 0.2), w=w,
                                      alpha_pv=a, eps=1e-13)
        p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE,
                         alpha_pv=a, state=state)
        p.set_init(np.zeros(g.n), np.full(g.n, 0.2))
    for sched, q in (("all", 1.0), ("sampled", 0.2), ("exact", 0.05)):
        p.set_init(np.zeros(g.n), np.full(g.n, 0.2))
        eps = 1e-10 if state == "f64" else 1e-5
        assert p.run(eps=eps, q=q, sched=sched, seed=2).converged
        err = np.abs(p.get() - ref).sum()
        if state == "f64":
            assert err <= 1e-9, (sched, err)
        else:
            assert err / ref.sum() <= 1e-5, (sched, err)


# ---------------------------------------------------------------------------
# Round-robin scheduling and progress traces (Sec. 5.1, Sec. 6.3)
# ---------------------------------------------------------------------------

def test_round_robin_selection_block(daic):
    say("case rr selection")
    n = 1000
    g = daic_gen.from_edges(n, [], [])
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8)
    dv = np.where(np.arange(n) % 3 == 0, 0.0, 1.0)
    p.set_init(np.zeros(n), dv)
    sel, _ = p.select_frontier(q=0.1, sched="round_robin")
    # round 0 takes block 0 = ids 0..99, pending ones only
    want = (np.arange(n) < 100) & (dv != 0)
    np.testing.assert_array_equal(sel, want)


def test_round_robin_reaches_the_fixed_point(daic, pl10k, pl10k_ref):
    say("case rr pagerank")
    p = pr_problem(daic, pl10k, 0.8)
    res = p.run(eps=1e-10, q=0.1, sched="round_robin")
    assert res.converged
    assert np.abs(p.get() - pl10k_ref).sum() <= 1e-9
    g = daic_gen.rmat(12, 16, seed=5)
    w, ref = sssp_case(g, 3)
    ps = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
    ps.set_init(*oracle.sssp_init(g.n, 0))
    assert ps.run(q=0.05, sched="round_robin").converged
    np.testing.assert_array_equal(ps.get(), ref)


def test_progress_trace_is_monotone(daic):
    """sum_j v_j grows monotonically for PageRank and falls for SSSP (Sec. 6.3);
    the last point equals the fixed point's total."""
    say("case progress")
    g = daic_gen.rmat(13, 16, seed=9)
    p = pr_problem(daic, g, 0.8)
    res, up, pr = p.run_progress(eps=1e-9, q=0.2, sched="exact")
    assert res.converged and len(pr) == res.stats["rounds"]
    assert np.all(np.diff(pr) >= -1e-9) and np.all(np.diff(up.astype(np.int64)) > 0)
    assert abs(pr[-1] - p.get().sum()) <= 1e-9 * pr[-1]
    w, ref = sssp_case(g, 4)
    ps = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
    ps.set_init(*oracle.sssp_init(g.n, 0))
    res, up, pr = ps.run_progress(q=0.2, sched="round_robin")
    assert res.converged
    finite = ref != oracle.INF_U32
    assert pr[-1] == ref[finite].astype(np.float64).sum()


# ---------------------------------------------------------------------------
# Further rows of the algorithm table (Table 1) through the same kernels
# ---------------------------------------------------------------------------

def test_jacobi_linear_solver(daic):
    """Jacobi method (Sec. 4.2.2): g_{i,j}(x) = -A_ji / A_jj x, dv1_j = b_j / A_jj,
    on a diagonally dominant sparse system; signed coefficients."""
    say("case jacobi")
    from scipy.sparse import random as sprandom

    n = 3000
    rng = np.random.default_rng(3)
    A = sprandom(n, n, density=8.0 / n, random_state=4, format="csr")
    A.data = rng.uniform(-1, 1, A.data.size)
    A.setdiag(0)
    A.eliminate_zeros()
    rowabs = np.asarray(abs(A).sum(axis=1)).ravel()
    diag = 2.0 * rowabs + 1.0
    b = rng.normal(0, 1, n)
    Ad = A.toarray() + np.diag(diag)
    want = np.linalg.solve(Ad, b)
    # edge i -> j carries -A_ji / A_jj: the transpose's rows are the senders
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
    assert p.run(eps=1e-12, q=1.0, sched="all").converged
    np.testing.assert_allclose(p.get(), want, rtol=0, atol=1e-10)


def test_hits_authority(daic):
    """HITS authority (Table 1): g(x) = d A(i,j) x with A = W^T W built first."""
    say("case hits")
    from scipy.sparse import csr_matrix

    g0 = daic_gen.rmat(10, 4, seed=12)
    n = g0.n
    src = np.repeat(np.arange(n), g0.outdeg())
    W = csr_matrix((np.ones(g0.m), (src, g0.col.astype(np.int64))), shape=(n, n))
    W.data[:] = 1.0
    A = (W.T @ W).tocsr()
    A.sort_indices()
    d = 0.5 / max(1.0, float(abs(A).sum(axis=1).max()))
    src = np.repeat(np.arange(n), np.diff(A.indptr))
    g = daic_gen.from_edges(n, src, A.indices)
    w = A.data.astype(np.float64)
    want = np.linalg.solve(np.eye(n) - d * A.toarray().T, np.ones(n))
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE, alpha=d)
    p.set_init(np.zeros(n), np.ones(n))
    assert p.run(eps=1e-12).converged
    np.testing.assert_allclose(p.get(), want, rtol=1e-10)


def test_checkpoint_resume_through_files(daic, tmp_path):
    """A round boundary is a consistent cut: (v, dv) saved to a file and loaded
    into a fresh problem reaches the same fixed point (cf. Sec. 5.1 fault
    tolerance; no in-flight messages exist between rounds)."""
    say("case checkpoint")
    g = daic_gen.rmat(13, 16, seed=21)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    p = pr_problem(daic, g, 0.8)
    res = p.run(eps=1e-12, q=0.3, sched="exact", max_rounds=5, rounds_per_check=1)
    assert res.status == daic.NOT_CONVERGED
    v, dv = p.get(with_dv=True)
    np.savez(tmp_path / "ckpt.npz", v=v, dv=dv)
    del p
    ck = np.load(tmp_path / "ckpt.npz")
    q = pr_problem(daic, g, 0.8)
    q.set_init(ck["v"], ck["dv"])
    assert q.run(eps=1e-10, q=1.0).converged
    assert np.abs(q.get() - ref).sum() <= 1e-9


def test_library_checkpoint_resume(daic, tmp_path):
    """Checkpoint through the library's own snapshot (daic_problem_save /
    load, Sec. 5.1 snapshots of the state table): runs stopped by max_rounds
    are written to files, every handle (graph included) is destroyed, the
    problems are rebuilt from the CSR and the files, and the resumed runs
    reach the oracle's fixed point. The snapshot is bit-exact: a reloaded
    state saves to the same bytes."""
    say("case library checkpoint")
    g = daic_gen.rmat(13, 16, seed=23)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    w = daic_gen.sssp_weights(g.m, seed=24)
    dist = oracle.dijkstra(g, w, 0)
    paths = {}
    for kind in ("f32_kahan", "f64", "sssp"):
        if kind == "sssp":
            p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
            p.set_init(*oracle.sssp_init(g.n, 0))
            res = p.run(q=0.1, sched="exact", max_rounds=3, rounds_per_check=1)
        else:
            p = pr_problem(daic, g, 0.8, state=kind)
            res = p.run(eps=1e-10, q=0.3, sched="exact", max_rounds=6, rounds_per_check=1)
        assert res.status == daic.NOT_CONVERGED
        paths[kind] = tmp_path / f"{kind}.state"
        p.save(paths[kind])
        blob = p.save_state()
        p.close()
        del p
        if kind == "sssp":
            q = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
        else:
            q = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8,
                             state=kind)
        q.load(paths[kind])
        assert q.save_state() == blob
        if kind == "sssp":
            assert q.run(q=0.1, sched="sampled").converged
            np.testing.assert_array_equal(q.get(), dist)
        else:
            assert q.run(eps=1e-10 if kind == "f64" else 1e-7, q=1.0).converged
            err = np.abs(q.get() - ref).sum()
            assert err <= (1e-9 if kind == "f64" else 1e-5 * ref.sum()), (kind, err)
    # a snapshot of another kind of problem, or a damaged one, is refused
    q = pr_problem(daic, g, 0.85)
    with pytest.raises(daic.DaicError):
        q.load(paths["f64"])
    bad = bytearray(open(paths["f32_kahan"], "rb").read())
    bad[3] ^= 0x20
    q2 = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8, state="f32_kahan")
    with pytest.raises(daic.DaicError):
        q2.load_state(bytes(bad))
    with pytest.raises(daic.DaicError):
        q2.load_state(open(paths["f32_kahan"], "rb").read()[:-8])


@pytest.mark.parametrize("kind", ["pagerank_f64", "pagerank_f32_kahan", "sssp", "cc", "katz"])
def test_fourth_condition_check(daic, monkeypatch, kind):
    """v0 (+) dv1 = f(v0) (fourth condition, Sec. 3.1) checked on the device:
    the paper's initial values pass, a wrong delta at one vertex is caught
    (DAIC_E_INVALID, one mismatch), with DAIC_CHECK_INIT set daic_run refuses
    the wrong start without touching the state, and a converged state still
    satisfies the identity."""
    say("case fourth condition", kind)
    g = daic_gen.rmat(11, 8, seed=31)
    n = g.n
    if kind.startswith("pagerank"):
        state = kind.split("_", 1)[1]
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8, state=state)
        v0, dv1 = oracle.pagerank_init(n, 0.8)
        c = np.full(n, 0.2)
        wrong = dv1.copy()
        wrong[77] = 0.25
        run = dict(eps=1e-9, q=1.0)
    elif kind == "katz":
        # Katz from a nonzero start: v0 random, dv1 = f(v0) - v0 with c = e_s
        beta = 0.9 / max(1, int(g.outdeg().max()))
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_SRC_SCALE, alpha=beta, state="f64")
        rng = np.random.default_rng(5)
        v0 = rng.uniform(0, 1, n)
        c = np.zeros(n)
        c[3] = 1.0
        fv = c.copy()
        np.add.at(fv, g.col, beta * np.repeat(v0, g.outdeg()))
        dv1 = fv - v0
        wrong = dv1.copy()
        wrong[1000] += 1e-6
        run = dict(eps=1e-12, q=1.0)
    elif kind == "sssp":
        w = daic_gen.sssp_weights(g.m, seed=32)
        p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
        v0, dv1 = oracle.sssp_init(n, 0)
        c = dv1.copy()
        wrong = dv1.copy()
        wrong[9] = 3
        run = dict(q=0.1, sched="sampled")
    else:
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.MAX, daic.G_COPY, state="i32")
        v0, dv1 = oracle.cc_init(n)
        c = np.arange(n, dtype=np.int32)
        wrong = dv1.copy()
        wrong[5] = 4
        run = dict(q=1.0)
    with pytest.raises(daic.DaicError):
        p.check_init()  # no constant given yet
    p.set_const(c)
    p.set_init(v0, wrong)
    with pytest.raises(daic.DaicError, match="1 mismatches"):
        p.check_init()
    monkeypatch.setenv("DAIC_CHECK_INIT", "1")
    with pytest.raises(daic.DaicError):
        p.run(**run)
    _, dv_after = p.get(with_dv=True)
    expect = wrong.astype(np.float32) if kind == "pagerank_f32_kahan" else wrong
    np.testing.assert_array_equal(dv_after, expect.astype(dv_after.dtype))
    p.set_init(v0, dv1)
    assert p.check_init() == 0
    assert p.run(**run).converged
    monkeypatch.delenv("DAIC_CHECK_INIT")
    if kind == "katz":  # a start away from 0 with deltas of both signs
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_SRC_SCALE, beta, dv1, v0=v0, eps=1e-15)
        assert np.abs(p.get() - ref).sum() <= 1e-9
    assert p.check_init(tol=1e-4 if kind == "pagerank_f32_kahan" else 0.0) == 0
