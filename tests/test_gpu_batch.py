"""GPU parity of the batched personalized PageRank path against the oracle.

Every instance (graph, right-hand side) is compared with the oracle's FP64
traditional iteration on the same graph and personalization vector: relative
L1 error <= 1e-5 (FP32 state), and every instance residual <= eps.
"""
import sys

import numpy as np
import pytest

import daic_gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ppr_inputs(g, seed, rhs_base, rhs, d, max_k=32):
    counts, seeds = daic_gen.ppr_seeds(g, seed, rhs_base, rhs, max_k)
    dv1 = np.zeros((g.n, rhs))
    for r in range(rhs):
        s = seeds[r, : counts[r]]
        dv1[s, r] = (1.0 - d) / len(s)
    return dv1


@pytest.fixture(scope="module")
def daic():
    from paper_1710_05785_amd import daic as d

    d.lib()
    return d


@pytest.mark.parametrize("state", ["f32", "f32_kahan"])
@pytest.mark.parametrize("rhs", [64, 5])
def test_batched_ppr_matches_oracle(daic, state, rhs):
    say("case batch", state, rhs)
    d = 0.85
    scales = [7, 10, 9, 12, 8, 11]
    gs = [daic_gen.rmat(s, 8, seed=1000 + i) for i, s in enumerate(scales)]
    # one graph without edges and one tiny ragged graph join the batch
    gs.append(daic_gen.from_edges(37, [], []))
    gs.append(daic_gen.from_edges(5, [0, 1, 2, 3, 4], [1, 2, 3, 4, 0]))
    dgs = [daic.Graph(g.row_ptr, g.col) for g in gs]
    b = daic.Batch(dgs, rhs, alpha=d, state=state)
    inits = []
    for i, g in enumerate(gs):
        if g.m == 0:
            dv1 = np.zeros((g.n, rhs))
            dv1[np.arange(rhs) % g.n, np.arange(rhs)] = 1 - d
        else:
            dv1 = ppr_inputs(g, 6, i * 64, rhs, d)
        inits.append(dv1)
        b.set_init(i, np.zeros((g.n, rhs)), dv1)
    desc = b.tune()
    say("tuned:", desc)
    res, inst = b.run(eps=1e-7, rounds_per_check=4)
    assert res.converged
    assert np.all(inst <= 1e-7)
    for i, g in enumerate(gs):
        v = b.get(i)
        for r in range(rhs):
            ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, inits[i][:, r], eps=1e-14)
            den = max(np.abs(ref).sum(), 1e-300)
            rel = np.abs(v[:, r] - ref).sum() / den
            assert rel <= 1e-5, (i, r, rel)


def test_batched_equals_single_solves(daic):
    """The batched run and per-instance single-problem runs agree."""
    say("case batch vs single")
    d = 0.85
    gs = [daic_gen.rmat(s, 8, seed=2000 + s) for s in (9, 11)]
    dgs = [daic.Graph(g.row_ptr, g.col) for g in gs]
    rhs = 16
    b = daic.Batch(dgs, rhs, alpha=d)
    inits = [ppr_inputs(g, 6, 100 * i, rhs, d) for i, g in enumerate(gs)]
    for i, g in enumerate(gs):
        b.set_init(i, np.zeros((g.n, rhs)), inits[i])
    assert b.run(eps=1e-7)[0].converged
    for i, g in enumerate(gs):
        vb = b.get(i)
        for r in (0, 7, 15):
            p = daic.Problem(dgs[i], daic.SUM, daic.G_DEG_SCALE, alpha=d, state="f64")
            p.set_init(np.zeros(g.n), inits[i][:, r])
            assert p.run(eps=1e-12).converged
            vs = p.get()
            assert np.abs(vb[:, r] - vs).sum() <= 1e-5 * np.abs(vs).sum()


def test_batched_max_rounds_and_resume(daic):
    say("case batch resume")
    d = 0.85
    g = daic_gen.rmat(10, 8, seed=77)
    gd = daic.Graph(g.row_ptr, g.col)
    b = daic.Batch([gd], 8, alpha=d)
    dv1 = ppr_inputs(g, 6, 0, 8, d)
    b.set_init(0, np.zeros((g.n, 8)), dv1)
    res, _ = b.run(eps=1e-8, rounds_per_check=1, max_rounds=3)
    assert res.status == daic.NOT_CONVERGED and res.stats["rounds"] == 3
    res, inst = b.run(eps=1e-8)
    assert res.converged and np.all(inst <= 1e-8)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, dv1[:, 3], eps=1e-14)
    assert np.abs(b.get(0)[:, 3] - ref).sum() <= 1e-5 * ref.sum()


def hub_graph(n=5000):
    """A ring plus three hub targets: every vertex points at 0 and 1 and every
    even vertex at 2, so in-degrees span one to five 1024-edge chunks."""
    i = np.arange(n)
    src = np.concatenate([i, i[i != 0], i[i != 1], i[(i % 2 == 0) & (i != 2)]])
    dst = np.concatenate([(i + 1) % n, np.zeros(n - 1, np.int64), np.ones(n - 1, np.int64),
                          np.full(((i % 2 == 0) & (i != 2)).sum(), 2)])
    return daic_gen.from_edges(n, src, dst)


@pytest.mark.parametrize("state", ["f32", "f32_kahan"])
def test_batched_hub_targets_match_oracle(daic, state):
    """Dense rounds with hub targets (in-degree above 1024, summed in chunks
    with atomics before the fused pass) next to an RMAT graph."""
    say("case batch hubs", state)
    d = 0.85
    gs = [hub_graph(), daic_gen.rmat(11, 8, seed=3)]
    b = daic.Batch([daic.Graph(g.row_ptr, g.col) for g in gs], 64, alpha=d, state=state)
    inits = [ppr_inputs(g, 9, 64 * i, 64, d) for i, g in enumerate(gs)]
    for i, g in enumerate(gs):
        b.set_init(i, np.zeros((g.n, 64)), inits[i])
    res, inst = b.run(eps=1e-7, rounds_per_check=8)
    assert res.converged and np.all(inst <= 1e-7)
    for i, g in enumerate(gs):
        v = b.get(i)
        for r in (0, 13, 63):
            ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, inits[i][:, r], eps=1e-14)
            assert np.abs(v[:, r] - ref).sum() <= 1e-5 * np.abs(ref).sum(), (i, r)


def test_batched_stop_in_dense_phase_delivers(daic):
    """Runs stopped by max_rounds in the dense phase (messages of the last
    claim still in flight) deliver them before returning: later runs resume
    from a consistent state and reach the oracle's fixed point."""
    say("case batch stop dense")
    d = 0.85
    g = daic_gen.rmat(12, 8, seed=41)
    b = daic.Batch([daic.Graph(g.row_ptr, g.col)], 64, alpha=d)
    dv1 = ppr_inputs(g, 4, 0, 64, d)
    b.set_init(0, np.zeros((g.n, 64)), dv1)
    for k in (2, 5):
        res, inst = b.run(eps=1e-9, rounds_per_check=1, max_rounds=k)
        assert res.status == daic.NOT_CONVERGED and res.stats["rounds"] == k
        assert np.all(np.isfinite(inst)) and np.all(inst > 0)
    res, inst = b.run(eps=1e-9, rounds_per_check=16)
    assert res.converged and np.all(inst <= 1e-9)
    v = b.get(0)
    for r in (0, 31, 63):
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, dv1[:, r], eps=1e-14)
        assert np.abs(v[:, r] - ref).sum() <= 1e-5 * ref.sum()


def adsorption_case(g, seed):
    """Adsorption (Table 1): A column-normalized from log-normal(0.4, 0.8)
    weights (the sum of a vertex's in-edge weights is 1), p_cont ~ U[0.5, 0.9]
    per vertex, p_inj = 1 - p_cont; g_{i,j}(x) = p_cont_j A(i,j) x is folded
    into one weight per edge (receiver's coefficient, reading 4)."""
    raw = daic_gen.lognormal_f64(seed, g.m, 0.4, 0.8)
    col = g.col.astype(np.int64)
    insum = np.bincount(col, weights=raw, minlength=g.n)
    A = raw / np.where(insum[col] > 0, insum[col], 1.0)
    rng = np.random.default_rng(seed)
    p_cont = rng.uniform(0.5, 0.9, g.n)
    return A * p_cont[col], 1.0 - p_cont


@pytest.mark.parametrize("state", ["f32", "f32_kahan"])
def test_batched_multilabel_adsorption_matches_oracle(daic, state):
    """Multi-label Adsorption through the batched path: one label per
    right-hand side (64 labels), dv1_{j,l} = p_inj_j I_{j,l}; every label of
    every graph against the oracle's FP64 traditional iteration."""
    say("case batch adsorption", state)
    gs = [daic_gen.rmat(11, 8, seed=301), daic_gen.paper_lognormal(3000, seed=302),
          daic_gen.from_edges(40, [], []), daic_gen.rmat(9, 16, seed=303)]
    labels = 64
    ws, inits = [], []
    dgs = []
    for i, g in enumerate(gs):
        if g.m:
            w, p_inj = adsorption_case(g, 310 + i)
            dgs.append(daic.Graph(g.row_ptr, g.col, w))
        else:
            w, p_inj = None, np.full(g.n, 0.3)
            dgs.append(daic.Graph(g.row_ptr, g.col))
        ws.append(w)
        seeds = ppr_inputs(g, 320 + i, 64 * i, labels, 0.0, max_k=8) if g.m else None
        dv1 = np.zeros((g.n, labels))
        if seeds is not None:
            dv1 = (seeds > 0) * p_inj[:, None]
        else:
            dv1[np.arange(labels) % g.n, np.arange(labels)] = p_inj[0]
        inits.append(dv1)
    b = daic.Batch(dgs, labels, alpha=1.0, state=state, g=daic.G_EDGE_SCALE)
    for i, g in enumerate(gs):
        b.set_init(i, np.zeros((g.n, labels)), inits[i])
    say("tuned:", b.tune())
    res, inst = b.run(eps=1e-7, rounds_per_check=4)
    assert res.converged and np.all(inst <= 1e-7)
    for i, g in enumerate(gs):
        v = b.get(i)
        for l in range(0, labels, 7):
            if g.m:
                ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 1.0, inits[i][:, l], w=ws[i], eps=1e-14)
            else:
                ref = inits[i][:, l]
            den = max(np.abs(ref).sum(), 1e-300)
            assert np.abs(v[:, l] - ref).sum() / den <= 1e-5, (i, l)


def test_batched_edge_scale_needs_weights(daic):
    say("case batch edge scale without weights")
    g = daic_gen.rmat(8, 4, seed=5)
    with pytest.raises(daic.DaicError):
        daic.Batch([daic.Graph(g.row_ptr, g.col)], 8, alpha=1.0, g=daic.G_EDGE_SCALE)


def ppr_batch(daic, gs, rhs, d, state, seed0=6):
    dgs = [daic.Graph(g.row_ptr, g.col) for g in gs]
    b = daic.Batch(dgs, rhs, alpha=d, state=state)
    inits = []
    for i, g in enumerate(gs):
        if g.m == 0:
            dv1 = np.zeros((g.n, rhs))
            dv1[np.arange(rhs) % g.n, np.arange(rhs)] = 1 - d
        else:
            dv1 = ppr_inputs(g, seed0, i * 64, rhs, d)
        inits.append(dv1)
        b.set_init(i, np.zeros((g.n, rhs)), dv1)
    return b, inits


def check_ppr(b, gs, inits, d, rhs, every=1, tol=1e-5):
    for i, g in enumerate(gs):
        v = b.get(i)
        for r in range(0, rhs, every):
            ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, inits[i][:, r], eps=1e-14)
            den = max(np.abs(ref).sum(), 1e-300)
            assert np.abs(v[:, r] - ref).sum() / den <= tol, (i, r)


@pytest.mark.parametrize("state", ["f32", "f32_kahan"])
@pytest.mark.parametrize("rhs,q", [(64, 0.125), (5, 0.3), (64, 1.0)])
def test_batched_sweep_matches_oracle(daic, state, rhs, q):
    """Sweep rounds over the batch (blocks of ceil(q n_g) vertices of every
    graph in turn, each pulling the newest messages): every instance at the
    oracle's fixed point and at residual <= eps."""
    say("case batch sweep", state, rhs, q)
    d = 0.85
    gs = [daic_gen.rmat(s, 8, seed=1000 + i) for i, s in enumerate([7, 10, 9, 12, 8, 11])]
    gs.append(daic_gen.from_edges(37, [], []))
    gs.append(daic_gen.from_edges(5, [0, 1, 2, 3, 4], [1, 2, 3, 4, 0]))
    gs.append(hub_graph(3000))
    b, inits = ppr_batch(daic, gs, rhs, d, state)
    res, inst = b.run(eps=1e-7, rounds_per_check=4, sched="sweep", q=q)
    assert res.converged and np.all(inst <= 1e-7)
    check_ppr(b, gs, inits, d, rhs)


def test_batched_sweep_needs_fewer_passes(daic):
    say("case batch sweep passes")
    d = 0.85
    gs = [daic_gen.rmat(s, 8, seed=2000 + s) for s in (12, 13)]
    b, inits = ppr_batch(daic, gs, 64, d, "f32")
    ra, _ = b.run(eps=1e-7, rounds_per_check=4)
    b2, _ = ppr_batch(daic, gs, 64, d, "f32")
    rs, _ = b2.run(eps=1e-7, rounds_per_check=4, sched="sweep", q=0.125)
    assert ra.converged and rs.converged
    say("synchronous rounds", ra.stats["rounds"], "sweep rounds", rs.stats["rounds"],
        "messages", ra.stats["pushed_edges"], rs.stats["pushed_edges"])
    assert rs.stats["rounds"] / 8 <= 0.8 * ra.stats["rounds"]
    assert rs.stats["pushed_edges"] < ra.stats["pushed_edges"]


def test_batched_sweep_stop_and_resume(daic):
    """Runs stopped by max_rounds inside a sweep deliver the messages in
    flight; resuming (sweep or synchronous) reaches the fixed point."""
    say("case batch sweep stop")
    d = 0.85
    gs = [daic_gen.rmat(12, 8, seed=41), hub_graph(2000), daic_gen.rmat(9, 16, seed=42)]
    for stops in ((3,), (5, 11), (9, 2, 17)):
        b, inits = ppr_batch(daic, gs, 64, d, "f32")
        for k in stops:
            res, inst = b.run(eps=1e-7, rounds_per_check=1, max_rounds=k, sched="sweep", q=0.2)
            assert res.status == daic.NOT_CONVERGED
            assert np.all(np.isfinite(inst))
        res, inst = b.run(eps=1e-7, rounds_per_check=4, sched="sweep", q=0.2)
        assert res.converged and np.all(inst <= 1e-7)
        check_ppr(b, gs, inits, d, 64, every=9)
    b, inits = ppr_batch(daic, gs, 64, d, "f32")
    b.run(eps=1e-7, rounds_per_check=1, max_rounds=6, sched="sweep", q=0.25)
    res, inst = b.run(eps=1e-7)
    assert res.converged
    check_ppr(b, gs, inits, d, 64, every=9)


def test_batched_sweep_adsorption(daic):
    say("case batch sweep adsorption")
    gs = [daic_gen.rmat(11, 8, seed=301), daic_gen.paper_lognormal(3000, seed=302)]
    labels = 64
    dgs, ws, inits = [], [], []
    for i, g in enumerate(gs):
        w, p_inj = adsorption_case(g, 310 + i)
        dgs.append(daic.Graph(g.row_ptr, g.col, w))
        ws.append(w)
        inits.append((ppr_inputs(g, 320 + i, 64 * i, labels, 0.0, max_k=8) > 0) * p_inj[:, None])
    b = daic.Batch(dgs, labels, alpha=1.0, state="f32_kahan", g=daic.G_EDGE_SCALE)
    for i, g in enumerate(gs):
        b.set_init(i, np.zeros((g.n, labels)), inits[i])
    res, inst = b.run(eps=1e-7, rounds_per_check=4, sched="sweep", q=0.125)
    assert res.converged and np.all(inst <= 1e-7)
    for i, g in enumerate(gs):
        v = b.get(i)
        for l in range(0, labels, 9):
            ref, _, _ = oracle.jacobi_sum(g, oracle.G_EDGE_SCALE, 1.0, inits[i][:, l], w=ws[i], eps=1e-14)
            assert np.abs(v[:, l] - ref).sum() / max(np.abs(ref).sum(), 1e-300) <= 1e-5, (i, l)


def test_batch_checkpoint_resume(daic, tmp_path):
    """A batched run stopped by max_rounds is saved (daic_batch_save), every
    handle destroyed, the batch rebuilt from the graphs and the file, and the
    resumed run reaches every instance's oracle fixed point. The state
    read-out returns v, dv and the finish states; a reloaded batch saves to
    the same bytes."""
    say("case batch checkpoint")
    d, rhs = 0.85, 16
    gs = [daic_gen.rmat(s, 8, seed=1300 + s) for s in (9, 11, 10)]
    inits = [ppr_inputs(g, 6, i * 64, rhs, d) for i, g in enumerate(gs)]

    def build():
        b = daic.Batch([daic.Graph(g.row_ptr, g.col) for g in gs], rhs, alpha=d, state="f32_kahan")
        return b

    b = build()
    for i, g in enumerate(gs):
        b.set_init(i, np.zeros((g.n, rhs)), inits[i])
    r, _ = b.run(eps=1e-7, max_rounds=6, rounds_per_check=2)
    assert r.status == daic.NOT_CONVERGED
    v1, dv1s, done = b.get_state(1)
    assert v1.shape == dv1s.shape == (gs[1].n, rhs) and done.shape == (rhs,)
    assert np.abs(dv1s).sum() > 0
    np.testing.assert_array_equal(v1, b.get(1))
    path = tmp_path / "batch.state"
    b.save(path)
    blob = b.save_state()
    b.close()
    del b
    b2 = build()
    b2.load(path)
    assert b2.save_state() == blob
    r, inst = b2.run(eps=1e-7)
    assert r.converged and inst.max() <= 1e-7
    for i, g in enumerate(gs):
        got = b2.get(i)
        for k in range(rhs):
            ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, d, inits[i][:, k], eps=1e-14)
            err = np.abs(got[:, k] - ref).sum() / max(ref.sum(), 1e-300)
            assert err <= 1e-5, (i, k, err)
    other = daic.Batch([daic.Graph(g.row_ptr, g.col) for g in gs[:2]], rhs, alpha=d, state="f32_kahan")
    with pytest.raises(daic.DaicError):
        other.load(path)


def test_batched_single_launch(daic):
    """rounds_per_check = 0: the solve is one launch of 128 captured rounds
    (rounds after every instance finished return at once); the same rounds
    and state as checks every 4 rounds."""
    say("case batch single launch")
    d, rhs = 0.85, 32
    gs = [daic_gen.rmat(s, 8, seed=1400 + s) for s in (10, 12, 9)]
    out = []
    for rpc in (4, 0):
        b = daic.Batch([daic.Graph(g.row_ptr, g.col) for g in gs], rhs, alpha=d, state="f32_kahan")
        inits = [ppr_inputs(g, 6, i * 64, rhs, d) for i, g in enumerate(gs)]
        for i, g in enumerate(gs):
            b.set_init(i, np.zeros((g.n, rhs)), inits[i])
        r, inst = b.run(eps=1e-7, rounds_per_check=rpc)
        assert r.converged and inst.max() <= 1e-7
        out.append((r.stats["rounds"], [b.get(i) for i in range(len(gs))]))
    assert out[0][0] == out[1][0] <= 128
    for va, vb in zip(out[0][1], out[1][1]):
        assert np.abs(va - vb).sum() <= 1e-6 * np.abs(va).sum()
