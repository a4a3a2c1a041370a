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
