"""GPU checks of the learned scheduler's network kernels (BF16 MFMA, FP32
accumulation) against the FP64 oracle on identical BF16-rounded weights and
inputs. Tolerance 2e-2 relative (BF16 carries 8 significant bits; hidden
activations and back-propagated deltas are rounded to BF16 between layers)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    """Round-to-nearest-even to BF16, returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def daic():
    from paper_1710_05785_amd import daic as d

    d.lib()
    return d


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30))


def ref_params(p):
    """The oracle's view of the model: BF16 weights, FP32 biases."""
    return {"W1": bf16_round(p["W1"]), "b1": p["b1"].astype(np.float64),
            "W2": bf16_round(p["W2"]), "b2": p["b2"].astype(np.float64),
            "W3": bf16_round(p["W3"]), "b3": p["b3"].astype(np.float64)}


@pytest.mark.parametrize("n", [16, 37, 5000])
def test_mlp_forward_matches_oracle(daic, n):
    say("case mlp forward", n)
    rng = np.random.default_rng(n)
    m = daic.SchedModel(seed=3)
    p, _, _ = m.params()
    # nonzero biases so every term is exercised
    p["b1"] = rng.normal(0, 0.3, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.3, 64).astype(np.float32)
    p["b3"] = rng.normal(0, 0.3, 1).astype(np.float32)
    m = daic.SchedModel(params=p)
    x = rng.normal(0, 1, (n, 3)).astype(np.float32)
    got = m.forward(x)
    want, _ = oracle.mlp_forward(ref_params(p), bf16_round(x))
    assert rel(got, want) <= 2e-2, rel(got, want)


@pytest.mark.parametrize("case", ["powerlaw_5000", "rmat_14"])
def test_score_kernel_matches_oracle(daic, case):
    """The scoring kernel of learned rounds (features, standardization, BF16
    network on MFMA, sigmoid) against the oracle network on the features
    computed here from the same state: vertices without a pending delta
    score exactly 0; the others' logits agree to the BF16 tolerance. Sizes
    span many 64-vertex chunks with a ragged tail (5000)."""
    import daic_gen

    say("case score kernel", case)
    g = daic_gen.powerlaw(5000, seed=31) if case == "powerlaw_5000" else daic_gen.rmat(14, 8, seed=32)
    n = g.n
    rng = np.random.default_rng(33)
    dv1 = (rng.uniform(0.5, 1.0, n) * 10.0 ** rng.uniform(-6, 0, n)).astype(np.float32)
    dv1[rng.uniform(size=n) < 0.25] = 0.0  # not pending
    v0 = rng.uniform(0, 1, n).astype(np.float32)
    P = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.85,
                     state="f32_kahan")
    P.set_init(v0.astype(np.float64), dv1.astype(np.float64))
    m0 = daic.SchedModel(seed=34)
    p, _, _ = m0.params()
    p["b1"] = rng.normal(0, 0.3, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.3, 64).astype(np.float32)
    p["b3"] = rng.normal(0, 0.3, 1).astype(np.float32)
    m = daic.SchedModel(params=p)
    mean = np.array([-8.0, 0.1, 0.2], dtype=np.float32)
    std = np.array([5.0, 1.5, 0.5], dtype=np.float32)
    m.set_features(mean, std)
    got = P.sched_score(m)
    # features in FP32 as the kernel forms them (round 0: no rounds since the last update)
    outdeg = np.diff(g.row_ptr).astype(np.float32)
    indeg = np.bincount(g.col, minlength=n).astype(np.float32)
    pend = dv1 != 0
    f = np.zeros((n, 3), dtype=np.float32)
    f[:, 0] = np.log2(np.abs(dv1) + np.float32(1e-30))
    f[:, 1] = np.log2((np.float32(1) + indeg) / (np.float32(1) + outdeg))
    x = (f - mean) * (np.float32(1) / std)
    want_logit, _ = oracle.mlp_forward(ref_params(p), bf16_round(x[pend]))
    assert np.all(got[~pend] == 0.0)
    s = got[pend].astype(np.float64)
    ok = (s > 1e-4) & (s < 1 - 1e-4)
    assert ok.mean() > 0.9
    got_logit = np.log(s[ok] / (1 - s[ok]))
    assert rel(got_logit, want_logit[ok]) <= 2e-2, rel(got_logit, want_logit[ok])


def test_mfma_lane_layout_single_units(daic):
    """Each hidden unit and input feature in isolation: catches a transposed
    or misplaced operand in the MFMA lane layout (exact up to BF16 rounding)."""
    say("case mfma layout")
    for h in (0, 5, 17, 33, 63):
        for f in range(3):
            p = {"W1": np.zeros((64, 3), np.float32), "b1": np.zeros(64, np.float32),
                 "W2": np.zeros((64, 64), np.float32), "b2": np.zeros(64, np.float32),
                 "W3": np.zeros((1, 64), np.float32), "b3": np.zeros(1, np.float32)}
            p["W1"][h, f] = 1.0
            h2 = (h * 7 + 3) % 64
            p["W2"][h2, h] = 2.0
            p["W3"][0, h2] = 0.5
            m = daic.SchedModel(params=p)
            x = np.zeros((16, 3), np.float32)
            x[:, f] = np.arange(16, dtype=np.float32) - 4.0  # negative values die in ReLU
            got = m.forward(x)
            want = np.maximum(np.arange(16) - 4.0, 0.0) * 2.0 * 0.5
            np.testing.assert_allclose(got, want, rtol=1e-2, atol=1e-6)


@pytest.mark.parametrize("n", [16, 300, 20000])
def test_mlp_gradients_match_oracle(daic, n):
    say("case mlp grad", n)
    rng = np.random.default_rng(100 + n)
    m = daic.SchedModel(seed=11)
    p, _, _ = m.params()
    p["b1"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.2, 64).astype(np.float32)
    m = daic.SchedModel(params=p)
    x = rng.normal(0, 1, (n, 3)).astype(np.float32)
    y = (rng.random(n) < 0.35).astype(np.float32)
    g, loss = m.grad(x, y)
    rp = ref_params(p)
    z, cache = oracle.mlp_forward(rp, bf16_round(x))
    want = oracle.mlp_backward(rp, cache, z, y)
    assert abs(loss - oracle.bce_with_logits(z, y)) <= 1e-2 * abs(oracle.bce_with_logits(z, y))
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel(g[k], want[k]) <= 2e-2, (k, rel(g[k], want[k]))


# ---------------------------------------------------------------------------
# Trace capture, training and learned rounds
# ---------------------------------------------------------------------------

import daic_gen  # noqa: E402


def pr_problem(daic, g, state="f32_kahan", d=0.8):
    p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=d, state=state)
    p.set_init(*oracle.pagerank_init(g.n, d))
    return p


def sssp_problem(daic, g, w):
    p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.MIN, daic.G_EDGE_ADD, state="u32")
    p.set_init(*oracle.sssp_init(g.n, 0))
    return p


@pytest.fixture(scope="module")
def trained_pr(daic):
    traces = []
    for seed in (101, 102, 103):
        g = daic_gen.rmat(14, 16, seed=seed)
        p = pr_problem(daic, g)
        traces.append(daic.Trace.record(p, samples_per_round=4096, horizon=4, q=0.1, eps=1e-6))
    m = daic.SchedModel(seed=8)
    stats = daic.sched_train(traces, m, epochs=20, batch=16384, lr=3e-3, seed=1)
    return m, stats, traces


def test_trace_samples_are_well_formed(daic, trained_pr):
    say("case trace")
    _, _, traces = trained_pr
    x, y = traces[0].get()
    assert x.shape[0] == y.shape[0] > 1000
    assert np.all(np.isfinite(x))
    assert set(np.unique(y)).issubset({0.0, 1.0})
    assert 0.0 < y.mean() < 1.0
    assert np.all((x[:, 2] >= 0) & (x[:, 2] <= 1))


def test_training_reduces_loss(daic, trained_pr):
    say("case training")
    _, stats, _ = trained_pr
    say(stats)
    assert stats["loss_final"] < stats["loss_first"]


def test_learned_pagerank_reaches_the_fixed_point(daic, trained_pr):
    """Learned scheduling changes the update order only: same fixed point
    (Theorems 1 and 3), measured against the FP64 oracle; the gain over exact
    top-k at the same q and residual is printed."""
    say("case learned pagerank")
    m, _, _ = trained_pr
    g = daic_gen.rmat(15, 16, seed=200)
    ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
    pe = pr_problem(daic, g)
    re = pe.run(eps=1e-6, q=0.1, sched="exact")
    pl = pr_problem(daic, g)
    rl = pl.run(eps=1e-6, q=0.1, sched="learned", model=m)
    assert re.converged and rl.converged
    for p in (pe, pl):
        assert np.abs(p.get() - ref).sum() / ref.sum() <= 1e-5
    say("exact pushed", re.stats["pushed_edges"], "rounds", re.stats["rounds"],
        "learned pushed", rl.stats["pushed_edges"], "rounds", rl.stats["rounds"])
    # the fallback keeps the learned form within reach of the exact one
    assert rl.stats["pushed_edges"] <= 1.5 * re.stats["pushed_edges"]


def test_learned_sssp_is_bit_exact(daic):
    say("case learned sssp")
    traces = []
    for seed in (111, 112):
        g = daic_gen.rmat(13, 16, seed=seed)
        w = daic_gen.sssp_weights(g.m, seed=seed + 1)
        traces.append(daic.Trace.record(sssp_problem(daic, g, w), q=0.1, horizon=4))
    m = daic.SchedModel(seed=9)
    daic.sched_train(traces, m, epochs=10, batch=8192, lr=3e-3)
    g = daic_gen.rmat(14, 16, seed=120)
    w = daic_gen.sssp_weights(g.m, seed=7)
    ref = oracle.dijkstra(g, w, 0)
    p = sssp_problem(daic, g, w)
    r = p.run(q=0.1, sched="learned", model=m)
    assert r.converged
    np.testing.assert_array_equal(p.get(), ref)
