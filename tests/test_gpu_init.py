"""GPU: the seeded initial-centroid modes against their host
re-implementations (tests/init_reference.py), and the per-iteration
centroid history against the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from tests import init_reference as ir

pytestmark = pytest.mark.gpu


def _knor():
    import paper_1606_08905_amd as knor
    knor.load()
    return knor


def _dev(a, dtype):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mixture(n, d, kc, dtype, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-10, 10, size=(kc, d))
    return workloads.gaussian_mixture(rng, n, mu, np.ones(kc), np.ones(kc), dtype)


def _initial(knor, X, dtype, k, init, seed):
    C, lab, st = knor.fit(_dev(X, dtype), k, init=init, seed=seed, max_iters=1,
                          centroid_history=True)
    return st["centroid_history"][0].cpu().numpy()


@pytest.mark.parametrize("init,rule", [("forgy", ir.forgy_rows),
                                       ("shuffle_first_k", ir.shuffle_first_k_rows)])
@pytest.mark.parametrize("n,k,seed", [(5000, 10, 1234), (777, 777, 3), (100003, 64, 0)])
def test_shuffle_modes_match_host_rules(init, rule, n, k, seed):
    knor = _knor()
    X = _mixture(n, 5, 8, "f32", seed)
    print("CASE", init, n, k, seed, flush=True)
    C0 = _initial(knor, X, "f32", k, init, seed)
    rows = rule(n, k, seed)
    assert (C0 == X[rows].astype(np.float64)).all()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,d,k,seed", [(3001, 7, 20, 11), (1, 3, 1, 5), (2048, 16, 40, 2),
                                        (5000, 33, 64, 99)])
def test_kmeanspp_matches_host_rule(dtype, n, d, k, seed):
    knor = _knor()
    X = _mixture(n, d, 12, dtype, seed)
    print("CASE kmeans++", dtype, n, d, k, seed, flush=True)
    C0 = _initial(knor, X, dtype, k, "kmeans++", seed)
    X64 = workloads.to_f64(X, dtype)
    rows = ir.kmeanspp_rows(X64, k, seed)
    assert (C0 == X64[rows]).all()


def test_kmeanspp_duplicate_points_fall_back_to_uniform_draws():
    knor = _knor()
    base = np.array([[0.0, 1.0], [5.0, 5.0], [-3.0, 2.0]], np.float32)
    X = np.ascontiguousarray(np.repeat(base, 40, axis=0))      # 120 rows, 3 values
    C0 = _initial(knor, X, "f32", 6, "kmeans++", 17)
    rows = ir.kmeanspp_rows(X.astype(np.float64), 6, 17)
    assert (C0 == X[rows].astype(np.float64)).all()
    # the first three picks cover the three values; later draws are uniform
    assert len({tuple(r) for r in C0[:3]}) == 3


def test_kmeanspp_fit_equals_given_fit():
    knor = _knor()
    w = workloads.config(2, n=20000, k=40, seed=3)
    X = _dev(w.X, "f32")
    C1, l1, s1 = knor.fit(X, 40, init="kmeans++", seed=8, max_iters=30,
                          centroid_history=True)
    C0 = s1["centroid_history"][0]
    C2, l2, s2 = knor.fit(X, 40, C0=C0, max_iters=30)
    assert (C1.cpu().numpy() == C2.cpu().numpy()).all()
    assert (l1.cpu().numpy() == l2.cpu().numpy()).all()
    assert s1["iters"] == s2["iters"]


@pytest.mark.parametrize("prune,update", [(True, "canonical"), (False, "canonical"),
                                          (True, "exact")])
def test_centroid_history_follows_the_oracle(prune, update):
    knor = _knor()
    w = workloads.config(2, n=30000, k=50, seed=5)
    X64 = w.x64()
    C, lab, st = knor.fit(_dev(w.X, "f32"), w.k, C0=_dev(w.C0, "f64"), max_iters=25,
                          prune=prune, update=update, history=True, centroid_history=True)
    H = st["label_history"].cpu().numpy()
    CH = st["centroid_history"].cpu().numpy()
    assert CH.shape == (st["iters"], w.k, w.d)
    assert (CH[0] == w.C0).all()
    upd = oracle.update_exact if update == "exact" else oracle.update
    for t in range(st["iters"]):
        lab_o, _ = oracle.assign(X64, CH[t])
        assert (H[t] == lab_o).all(), t
        Cn, _ = upd(X64, H[t], CH[t])
        nxt = CH[t + 1] if t + 1 < st["iters"] else C.cpu().numpy()
        assert (nxt == Cn).all(), t
