"""The no-allocation selection entry point (daic_select_frontier_noalloc)
against daic_select_frontier on the same state: identical 0/1 selections
(bit-exact) and thresholds, for every selection rule and state type, on two
sizes in a row (the second smaller, so the shared scratch of the first call
is reused)."""
import sys

import numpy as np
import pytest

import daic_gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def daic():
    from paper_1710_05785_amd import daic as d

    d.lib()
    return d


CASES = [("all", 1.0, 0), ("exact", 0.1, 0), ("exact", 0.5, 0), ("sampled", 0.05, 0), ("sampled", 0.3, 5),
         ("round_robin", 0.25, 0)]


def states(torch, n, seed):
    """(op, state, g kind, v, dv) on the device with many equal keys and
    non-pending vertices."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    out = []
    for state, dt in (("f32_kahan", torch.float32), ("f64", torch.float64)):
        dv = (torch.randint(0, 50, (n,), generator=gen, device="cuda").to(dt) * 0.25)
        v = torch.rand(n, generator=gen, device="cuda", dtype=dt)
        out.append(("sum", state, v, dv))
    v = torch.randint(0, 1000, (n,), generator=gen, device="cuda", dtype=torch.int32)
    v[::7] = -1  # 0xFFFFFFFF: unreached
    dv = torch.randint(0, 1000, (n,), generator=gen, device="cuda", dtype=torch.int32)
    dv[::3] = -1
    out.append(("min", "u32", v, dv))
    v = torch.randint(-1, 500, (n,), generator=gen, device="cuda", dtype=torch.int32)
    dv = torch.randint(-1, 500, (n,), generator=gen, device="cuda", dtype=torch.int32)
    out.append(("max", "i32", v, dv))
    return out


def test_select_noalloc_matches_select_frontier(daic):
    import torch

    for n, seed in ((70001, 1), (5003, 2)):
        g = daic_gen.from_edges(n, np.arange(n - 1), np.arange(1, n))
        w = np.ones(g.m, dtype=np.uint32)
        for opname, state, v, dv in states(torch, n, seed):
            op = {"sum": daic.SUM, "min": daic.MIN, "max": daic.MAX}[opname]
            if opname == "sum":
                P = daic.Problem(daic.Graph(g.row_ptr, g.col), op, daic.G_DEG_SCALE, alpha=0.8, state=state)
            elif opname == "min":
                P = daic.Problem(daic.Graph(g.row_ptr, g.col, w), op, daic.G_EDGE_ADD, state=state)
            else:
                P = daic.Problem(daic.Graph(g.row_ptr, g.col), op, daic.G_COPY, state=state)
            P.set_init_device(v, dv)
            for sched, q, rnd in CASES:
                say("case noalloc", n, state, sched, q, rnd)
                want, tau_want = P.select_frontier(round_no=rnd, sched=sched, q=q, seed=7)
                sel = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
                tau = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
                daic.select_frontier_noalloc(op, state, v, dv, sel, tau, round_no=rnd, sched=sched, q=q, seed=7)
                torch.cuda.synchronize()
                got = sel.cpu().numpy()
                assert set(np.unique(got)) <= {0, 1}
                np.testing.assert_array_equal(got.astype(bool), want)
                assert tau.item() == tau_want, (tau.item(), tau_want)
                assert want.sum() > 0


def test_select_noalloc_rejects_bad_input(daic):
    import torch

    v = torch.zeros(10, dtype=torch.float32, device="cuda")
    sel = torch.zeros(10, dtype=torch.uint8, device="cuda")
    with pytest.raises(daic.DaicError):
        daic.select_frontier_noalloc(daic.SUM, "f32", v, v, sel, sched="sampled", q=0.1, n_samples=5000)
    with pytest.raises(daic.DaicError):
        daic.select_frontier_noalloc(daic.SUM, "f32", v, v, sel, sched="learned", q=0.1)
    with pytest.raises(daic.DaicError):
        daic.select_frontier_noalloc(daic.MIN, "f32", v, v, sel, sched="all")
