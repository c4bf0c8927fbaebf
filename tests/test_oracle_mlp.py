"""Pins of the FP64 MLP reference (oracle/mlp.py) against values fixed by
their definitions: the published SplitMix64 outputs, BF16 round-to-nearest-
even cases, finite differences of the loss, closed forms of the softmax
cross-entropy and of Adam's first step."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))
    _, z = mlp.splitmix64(g["seed"], 3)
    assert [int(v) for v in z] == [int(h, 16) for h in g["first_outputs_hex"]]


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (1.0 + 2.0 ** -8, 1.0), (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),
    (-(1.0 + 2.0 ** -8), -1.0), (3.0, 3.0), (0.0, 0.0),
    (1.0 / 3.0, 0.333984375), (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
])
def test_bf16_round_to_nearest_even(x, want):
    assert mlp.bf16(np.array([x]))[0] == want


def test_init_he_uniform_from_the_stream():
    d, h, k = 4, 6, 5
    th = mlp.init_params(d, h, k, seed=0)
    p = mlp.unflatten(th, d, h, k)
    _, z = mlp.splitmix64(0, 1)
    u = float(z[0] >> np.uint64(11)) * 2.0 ** -53
    assert p["W1"][0, 0] == (2 * u - 1) * math.sqrt(6.0 / d)
    for name, fan in (("W1", d), ("W2", h), ("W3", h)):
        assert np.abs(p[name]).max() <= math.sqrt(6.0 / fan)
    for b in ("b1", "b2", "b3"):
        assert (p[b] == 0).all()
    assert mlp.param_count(32, 256, 4096) == 1126912
    assert (mlp.init_params(d, h, k, 7) == mlp.init_params(d, h, k, 7)).all()


def test_gradient_matches_finite_differences():
    d, h, k, B = 3, 5, 4, 6
    rng = np.random.default_rng(0)
    th = mlp.init_params(d, h, k, seed=3) + rng.normal(size=mlp.param_count(d, h, k)) * 0.05
    X = rng.normal(size=(B, d))
    y = rng.integers(0, k, size=B)
    _, g = mlp.loss_and_grad(th, X, y, d, h, k, use_bf16=False)
    eps = 1e-6
    for i in rng.choice(th.size, size=40, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        lp, _ = mlp.loss_and_grad(tp, X, y, d, h, k, use_bf16=False)
        lm, _ = mlp.loss_and_grad(tm, X, y, d, h, k, use_bf16=False)
        assert abs((lp - lm) / (2 * eps) - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_uniform_logits_closed_form():
    d, h, k, B = 3, 4, 7, 5
    th = mlp.init_params(d, h, k, seed=1)
    p = mlp.unflatten(th, d, h, k)
    p["W3"][...] = 0.0                       # logits all zero
    rng = np.random.default_rng(2)
    X = rng.normal(size=(B, d))
    y = np.array([0, 1, 1, 3, 6])
    loss, g = mlp.loss_and_grad(th, X, y, d, h, k, use_bf16=False)
    assert abs(loss - math.log(k)) < 1e-15
    G = mlp.unflatten(g, d, h, k)
    freq = np.bincount(y, minlength=k) / B
    assert np.allclose(G["b3"], 1.0 / k - freq, atol=1e-15, rtol=0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, np.zeros(50), np.zeros(50), g, t=1)
    want = th - mlp.ADAM_LR * g / (np.abs(g) + mlp.ADAM_EPS)
    assert np.allclose(new, want, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_path_close_to_exact_path():
    d, h, k, B = 8, 16, 10, 32
    rng = np.random.default_rng(5)
    th = mlp.init_params(d, h, k, seed=9)
    X = rng.normal(size=(B, d))
    y = rng.integers(0, k, size=B)
    l1, g1 = mlp.loss_and_grad(th, X, y, d, h, k, use_bf16=True)
    l0, g0 = mlp.loss_and_grad(th, X, y, d, h, k, use_bf16=False)
    assert abs(l1 - l0) < 2e-2 * abs(l0)
    assert np.linalg.norm(g1 - g0) < 5e-2 * np.linalg.norm(g0)


def test_standardize():
    X = np.array([[1.0, 5.0], [3.0, 5.0], [5.0, 5.0]])
    mean, std = mlp.standardize(X)
    assert (mean == [3.0, 5.0]).all()
    assert std[0] == math.sqrt(8.0 / 3.0) and std[1] == 1.0
