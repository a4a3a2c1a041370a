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
