"""GPU checks of the learned scheduler against the oracle.

Network kernels (BF16 MFMA, FP32 accumulation) are compared element by element
with the FP64 oracle network on identical BF16 weights and inputs, with the
activations and product deltas rounded to BF16 where the kernels round them
(so both sides take their ReLU decisions on the same values). What remains is
FP32 accumulation order and an occasional value that lands on the other side
of a BF16 rounding boundary; each entry's tolerance is 2^-7 (one BF16 unit)
of the absolute-value network at that entry, which bounds every term that
can move it.

The trace rule (sampling, features, labels) and the Adam step are compared
with the oracle's exact top-k rounds and Adam update: labels bit-exact,
features within a few FP32 units."""
import os
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


def ref_params(p):
    """The oracle's view of the model: BF16 weights, FP32 biases."""
    return {"W1": bf16_round(p["W1"]), "b1": p["b1"].astype(np.float64),
            "W2": bf16_round(p["W2"]), "b2": p["b2"].astype(np.float64),
            "W3": bf16_round(p["W3"]), "b3": p["b3"].astype(np.float64)}


def abs_forward(rp, x):
    """Logits of the absolute-value network (|W|, |b|, |x|): a bound on every
    term that enters each logit."""
    z, _ = oracle.mlp_forward({k: np.abs(v) for k, v in rp.items()}, np.abs(x))
    return z


def abs_grad(rp, x, logits, y):
    """Absolute-value bound of every gradient entry: the backward pass with
    |W|, |activations| and |deltas|, every ReLU mask taken as open."""
    A = {k: np.abs(v) for k, v in rp.items()}
    xa = np.abs(np.asarray(x, dtype=np.float64))
    h1 = xa @ A["W1"].T + A["b1"]
    h2 = h1 @ A["W2"].T + A["b2"]
    n = xa.shape[0]
    dz3 = np.abs(1.0 / (1.0 + np.exp(-logits)) - y)[:, None] / n
    g = {"W3": dz3.T @ h2, "b3": dz3.sum(0)}
    dz2 = dz3 @ A["W3"]
    g["W2"], g["b2"] = dz2.T @ h1, dz2.sum(0)
    dz1 = dz2 @ A["W2"]
    g["W1"], g["b1"] = dz1.T @ xa, dz1.sum(0)
    return g


def assert_elementwise(got, want, bound, what, units=2.0 ** -7):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    tol = units * np.asarray(bound, dtype=np.float64) + 1e-9
    err = np.abs(got - want)
    bad = err > tol
    if bad.any():
        i = np.unravel_index(np.argmax(err - tol), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} entries outside tolerance; worst "
                             f"at {i}: got {got[i]!r}, want {want[i]!r}, tol {tol[i]!r}")


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
    rp, xb = ref_params(p), bf16_round(x)
    want, _ = oracle.mlp_forward(rp, xb, rnd=bf16_round)
    assert_elementwise(got, want, abs_forward(rp, xb), "logits")


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
    # features in FP32 as the kernel forms them (round 0, no vertex updated
    # yet: one round since the last update, counted at round -1)
    outdeg = np.diff(g.row_ptr).astype(np.float32)
    indeg = np.bincount(g.col, minlength=n).astype(np.float32)
    pend = dv1 != 0
    f = np.zeros((n, 3), dtype=np.float32)
    f[:, 0] = np.log2(np.abs(dv1) + np.float32(1e-30))
    f[:, 1] = np.log2((np.float32(1) + indeg) / (np.float32(1) + outdeg))
    f[:, 2] = np.float32(1.0 / 64.0)
    x = (f - mean) * (np.float32(1) / std)
    rp, xb = ref_params(p), bf16_round(x[pend])
    want_logit, _ = oracle.mlp_forward(rp, xb, rnd=bf16_round)
    assert np.all(got[~pend] == 0.0)
    s = got[pend].astype(np.float64)
    ok = (s > 1e-4) & (s < 1 - 1e-4)  # where the logit is recoverable from the sigmoid
    assert ok.mean() > 0.9
    got_logit = np.log(s[ok] / (1 - s[ok]))
    # the sigmoid is FP32 with a fast exponential: an error of a few FP32
    # units in s moves the recovered logit by up to 2^-20 / (s (1 - s)),
    # added to the network tolerance (as a multiple of its 2^-7 units)
    bound = abs_forward(rp, xb)[ok] + 2.0 ** -13 / (s[ok] * (1 - s[ok]))
    assert_elementwise(got_logit, want_logit[ok], bound, "score logits")


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
    rp, xb = ref_params(p), bf16_round(x)
    z, cache = oracle.mlp_forward(rp, xb, rnd=bf16_round)
    want = oracle.mlp_backward(rp, cache, z, y, rnd=bf16_round)
    assert abs(loss - oracle.bce_with_logits(z, y)) <= 1e-3 * abs(oracle.bce_with_logits(z, y))
    bound = abs_grad(rp, xb, z, y)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert_elementwise(g[k], want[k], bound[k], "grad " + k)


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


def inverted_model(daic):
    """A network that ranks against the priority: logit = -10 relu(feature 0),
    feature 0 being log2 of the priority, so the learned order prefers the
    pending vertices of smallest priority."""
    prm = {k: np.zeros(shp, np.float32) for k, shp in daic._PARAM_SHAPES}
    prm["W1"][0, 0] = 1.0
    prm["W2"][0, 0] = 1.0
    prm["W3"][0, 0] = -10.0
    m = daic.SchedModel(prm)
    m.set_features(np.array([-30.0, 0.0, 0.0], np.float32), np.ones(3, np.float32))
    return m


@pytest.mark.parametrize("kind", ["pagerank", "sssp"])
def test_learned_fallback_on_a_bad_network(daic, kind):
    """The device-side judge hands rounds back to exact top-k when the
    learned order drops the residual (pending count for min problems) per
    message below 0.8 x the exact round's: with an inverted network the run
    still converges to the oracle's result, with fallbacks recorded."""
    say("case learned fallback", kind)
    m = inverted_model(daic)
    g = daic_gen.rmat(14, 16, seed=130)
    if kind == "pagerank":
        ref, _, _ = oracle.jacobi_sum(g, oracle.G_DEG_SCALE, 0.8, np.full(g.n, 0.2), eps=1e-13)
        pe, pl = pr_problem(daic, g), pr_problem(daic, g)
        re = pe.run(eps=1e-6, q=0.1, sched="exact")
        rl = pl.run(eps=1e-6, q=0.1, sched="learned", model=m)
        assert re.converged and rl.converged
        assert np.abs(pl.get() - ref).sum() / ref.sum() <= 1e-5
    else:
        w = daic_gen.sssp_weights(g.m, seed=131)
        ref = oracle.dijkstra(g, w, 0)
        pe, pl = sssp_problem(daic, g, w), sssp_problem(daic, g, w)
        re = pe.run(q=0.1, sched="exact")
        rl = pl.run(q=0.1, sched="learned", model=m)
        assert re.converged and rl.converged
        np.testing.assert_array_equal(pl.get(), ref)
    st = rl.stats
    say("exact pushed", re.stats["pushed_edges"], "rounds", re.stats["rounds"], "learned pushed",
        st["pushed_edges"], "rounds", st["rounds"], "fallbacks", st["learned_fallbacks"], "exact rounds",
        st["learned_exact_rounds"])
    assert st["learned_exact_rounds"] >= 1
    assert st["learned_fallbacks"] >= 1
    assert st["learned_exact_rounds"] < st["rounds"]


def test_learned_rounds_captured_equal_eager(daic, trained_pr, monkeypatch):
    """Learned rounds (scoring, selection, judge) captured in a graph give
    the same rounds, messages and state, bit for bit, as the same rounds
    launched one by one; a change of the network's parameters is seen by
    the next run (the captured graph is rebuilt)."""
    say("case learned captured vs eager")
    m, _, _ = trained_pr
    g = daic_gen.rmat(14, 16, seed=140)
    runs = []
    for eager in (False, True):
        if eager:
            monkeypatch.setenv("DAIC_NO_GRAPH", "1")
        p = pr_problem(daic, g)
        r = p.run(eps=1e-6, q=0.1, sched="learned", model=m, rounds_per_check=8)
        assert r.converged
        runs.append((r.stats, p.get(with_dv=True)))
    monkeypatch.delenv("DAIC_NO_GRAPH")
    (sa, (va, da)), (sb, (vb, db)) = runs
    for k in ("rounds", "pushed_edges", "activations", "learned_fallbacks", "learned_exact_rounds"):
        assert sa[k] == sb[k], k
    if os.environ.get("DAIC_NO_TILE"):
        # the streamed pull adds the pieces of cut targets with FP32 atomics,
        # so its sums vary in the last bits from run to run
        np.testing.assert_allclose(va, vb, rtol=1e-6, atol=0)
        np.testing.assert_allclose(da, db, rtol=1e-5, atol=1e-9)
    else:
        np.testing.assert_array_equal(va, vb)
        np.testing.assert_array_equal(da, db)
    # the same problem object re-run after the network changed: the result
    # must follow the new network (the inverted one), not a stale capture
    p = pr_problem(daic, g)
    r1 = p.run(eps=1e-6, q=0.1, sched="learned", model=m)
    bad = inverted_model(daic)
    p.set_init(*oracle.pagerank_init(g.n, 0.8))
    r2 = p.run(eps=1e-6, q=0.1, sched="learned", model=bad)
    q = pr_problem(daic, g)
    r3 = q.run(eps=1e-6, q=0.1, sched="learned", model=bad)
    assert r2.stats["pushed_edges"] == r3.stats["pushed_edges"]
    assert r2.stats["learned_fallbacks"] == r3.stats["learned_fallbacks"]
    # the same network object with new feature scales (every score 0.5)
    bad.set_features(np.array([100.0, 0.0, 0.0], np.float32), np.ones(3, np.float32))
    p.set_init(*oracle.pagerank_init(g.n, 0.8))
    r4 = p.run(eps=1e-6, q=0.1, sched="learned", model=bad)
    q2 = pr_problem(daic, g)
    r5 = q2.run(eps=1e-6, q=0.1, sched="learned", model=bad)
    assert r4.stats["pushed_edges"] == r5.stats["pushed_edges"]
    assert r4.stats["pushed_edges"] != r2.stats["pushed_edges"]
    say("runs", r1.stats["pushed_edges"], r2.stats["pushed_edges"], r4.stats["pushed_edges"])


# ---------------------------------------------------------------------------
# Trace rule, Adam step, trainer and model serialization against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,scale,q,S,H", [("sssp", 12, 0.1, 512, 4), ("sssp", 12, 0.3, 1000, 2),
                                              ("cc", 11, 0.2, 700, 3)])
def test_trace_matches_oracle(daic, kind, scale, q, S, H):
    """daic_trace_record against the oracle's exact top-k rounds and trace
    rule, sample by sample: the same vertices and rounds, labels bit-exact,
    features within a few FP32 units (log2 on the device). The integer
    problems make the rounds themselves deterministic."""
    say("case trace parity", kind, scale, q, S, H)
    g = daic_gen.rmat(scale, 16, seed=40 + scale)
    seed = 77
    if kind == "sssp":
        w = daic_gen.sssp_weights(g.m, seed=41)
        p = sssp_problem(daic, g, w)
        v0, dv1 = oracle.sssp_init(g.n, 0)
        want = oracle.trace_exact_topk(g, oracle.OP_MIN, v0, dv1, q, S, H, seed, w=w)
    else:
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.MAX, daic.G_COPY, state="i32")
        v0, dv1 = oracle.cc_init(g.n)
        p.set_init(v0, dv1)
        want = oracle.trace_exact_topk(g, oracle.OP_MAX, v0, dv1, q, S, H, seed)
    tr = daic.Trace.record(p, samples_per_round=S, horizon=H, q=q, seed=seed)
    x, y = tr.get()
    vid, rnd = tr.samples()
    say("rounds", want["rounds"], "samples", len(y), "positive", float(y.mean()) if len(y) else 0)
    assert len(y) == len(want["y"]) > 100
    np.testing.assert_array_equal(rnd, want["round"])
    np.testing.assert_array_equal(vid, want["vid"])
    np.testing.assert_array_equal(y, want["y"])
    assert 0.0 < y.mean() < 1.0
    np.testing.assert_allclose(x, want["x"], rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(p.get(), want["v"])


@pytest.mark.parametrize("gk,q,H", [("deg", 0.1, 4), ("edge", 0.2, 2)])
def test_trace_sum_problem_matches_oracle(daic, gk, q, H):
    """The sum-problem trace (FP64 state; label 0 when the vertex's FP32
    priority reaches half its sampled priority within H round starts)
    against the oracle's FP64 exact top-k rounds: the same samples and
    rounds, features within a few FP32 units, labels equal except where the
    later priority lies within 1e-6 (relative) of the half threshold, and
    the state after the run within rounding of the oracle's. Random initial
    deltas keep the exact top-k free of ties."""
    say("case sum trace parity", gk, q, H)
    g = daic_gen.rmat(11, 8, seed=90)
    rng = np.random.default_rng(91)
    dv1 = rng.uniform(0.1, 1.0, g.n)
    seed, S = 33, 700
    if gk == "deg":
        p = daic.Problem(daic.Graph(g.row_ptr, g.col), daic.SUM, daic.G_DEG_SCALE, alpha=0.8, state="f64")
        want = oracle.trace_exact_topk(g, oracle.OP_SUM, np.zeros(g.n), dv1, q, S, H, seed,
                                       gk=oracle.G_DEG_SCALE, alpha=0.8, eps=1e-9)
    else:
        deg = g.outdeg()
        w = daic_gen.lognormal_f64(92, g.m, 0.4, 0.8)
        rs = np.bincount(np.repeat(np.arange(g.n), deg), weights=w, minlength=g.n)
        a = 0.85 / np.where(deg > 0, rs, 1.0)
        p = daic.Problem(daic.Graph(g.row_ptr, g.col, w), daic.SUM, daic.G_EDGE_SCALE, alpha_pv=a, state="f64")
        want = oracle.trace_exact_topk(g, oracle.OP_SUM, np.zeros(g.n), dv1, q, S, H, seed, w=w,
                                       gk=oracle.G_EDGE_SCALE, alpha_pv=a, eps=1e-9)
    p.set_init(np.zeros(g.n), dv1)
    tr = daic.Trace.record(p, samples_per_round=S, horizon=H, q=q, seed=seed, eps=1e-9)
    x, y = tr.get()
    vid, rnd = tr.samples()
    say("rounds", want["rounds"], "samples", len(y), "positive", float(y.mean()) if len(y) else 0)
    assert len(y) == len(want["y"]) > 100
    np.testing.assert_array_equal(rnd, want["round"])
    np.testing.assert_array_equal(vid, want["vid"])
    np.testing.assert_allclose(x, want["x"], rtol=1e-5, atol=1e-5)
    mism = np.flatnonzero(y != want["y"])
    say("label mismatches", len(mism))
    assert len(mism) <= max(1, len(y) // 1000)
    assert 0.0 < y.mean() < 1.0
    v = p.get()
    assert np.abs(v - want["v"]).sum() <= 1e-12 * np.abs(want["v"]).sum()


def test_sched_step_matches_oracle_adam(daic):
    """Two training steps (gradient on the MFMA kernels, then Adam) against
    the oracle: each applied gradient element-wise against the oracle
    gradient, and the updated FP32 weights against the oracle's Adam update
    of the same gradient from the same moments."""
    say("case sched step")
    rng = np.random.default_rng(51)
    m = daic.SchedModel(seed=52)
    p, _, _ = m.params()
    p["b1"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b3"] = rng.normal(0, 0.2, 1).astype(np.float32)
    m = daic.SchedModel(params=p)
    N, lr = 3000, 2e-3
    x = rng.normal(0, 1, (N, 3)).astype(np.float32)
    y = (rng.random(N) < 0.4).astype(np.float32)
    w = daic.pack_params(p).astype(np.float64)
    mo = np.zeros_like(w)
    vo = np.zeros_like(w)
    for t in (1, 2):
        pc, _, _ = m.params()
        rp, xb = ref_params(pc), bf16_round(x)
        z, cache = oracle.mlp_forward(rp, xb, rnd=bf16_round)
        gw = oracle.mlp_backward(rp, cache, z, y, rnd=bf16_round)
        bound = abs_grad(rp, xb, z, y)
        g, loss = m.step(x, y, lr)
        assert abs(loss - oracle.bce_with_logits(z, y)) <= 1e-3 * oracle.bce_with_logits(z, y)
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            assert_elementwise(g[k], gw[k], bound[k], f"step {t} grad {k}")
        w, mo, vo = oracle.adam_step(w, daic.pack_params(g).astype(np.float64), mo, vo, t, lr)
        got = daic.pack_params(m.params()[0]).astype(np.float64)
        np.testing.assert_allclose(got, w, rtol=1e-6, atol=1e-7, err_msg=f"weights after step {t}")


def test_sched_train_standardizes_and_reports_loss(daic):
    """daic_sched_train on caller samples: the model's feature mean and scale
    are the samples' mean and population standard deviation (FP64, kept in
    FP32); the reported first loss is the oracle's loss of the untrained
    network on the standardized samples."""
    say("case sched train")
    rng = np.random.default_rng(61)
    N = 5000
    x = np.stack([rng.normal(-12, 4, N), rng.normal(0.5, 1.5, N), rng.uniform(0, 1, N)],
                 axis=1).astype(np.float32)
    y = (rng.random(N) < 0.3).astype(np.float32)
    m = daic.SchedModel(seed=62)
    p0, _, _ = m.params()
    st = daic.sched_train([daic.Trace.from_samples(x, y)], m, epochs=1, batch=N, lr=1e-3, seed=3)
    _, mean, sd = m.params()
    x64 = x.astype(np.float64)
    np.testing.assert_allclose(mean, x64.mean(0).astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(sd, np.maximum(1e-6, x64.std(0)).astype(np.float32), rtol=1e-6)
    xs = ((x64 - mean.astype(np.float64)) / sd.astype(np.float64)).astype(np.float32)
    z, _ = oracle.mlp_forward(ref_params(p0), bf16_round(xs), rnd=bf16_round)
    assert st["samples"] == N
    assert abs(st["positive_fraction"] - y.mean()) < 1e-12
    assert abs(st["loss_first"] - oracle.bce_with_logits(z, y)) <= 1e-3 * oracle.bce_with_logits(z, y)


def test_sched_save_load_round_trip(daic):
    """A saved model loads with the same weights, standardization and Adam
    state: forward passes agree exactly, and a further step on each gives
    the same weights. Damaged buffers are refused with an error."""
    say("case sched save/load")
    rng = np.random.default_rng(71)
    m = daic.SchedModel(seed=72)
    x = rng.normal(0, 1, (2000, 3)).astype(np.float32)
    y = (rng.random(2000) < 0.5).astype(np.float32)
    m.step(x, y, 1e-3)
    m.set_features(np.array([1.0, -2.0, 0.5], np.float32), np.array([2.0, 3.0, 0.25], np.float32))
    buf = m.save()
    assert len(buf) == 53820
    m2 = daic.SchedModel.load(buf)
    pa, ma, sa = m.params()
    pb, mb, sb = m2.params()
    for k in pa:
        np.testing.assert_array_equal(pa[k], pb[k])
    np.testing.assert_array_equal(ma, mb)
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(m.forward(x), m2.forward(x))
    m.step(x, y, 1e-3)
    m2.step(x, y, 1e-3)
    np.testing.assert_array_equal(daic.pack_params(m.params()[0]), daic.pack_params(m2.params()[0]))
    bad = bytearray(buf)
    bad[0] ^= 1
    with pytest.raises(daic.DaicError):
        daic.SchedModel.load(bytes(bad))
    with pytest.raises(daic.DaicError):
        daic.SchedModel.load(buf[:-4])
    nan = bytearray(buf)
    nan[48:52] = np.array([np.nan], np.float32).tobytes()
    with pytest.raises(daic.DaicError):
        daic.SchedModel.load(bytes(nan))
