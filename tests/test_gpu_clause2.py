"""GPU parity of the Clause-2 candidate-list tile (MTI survivors scanned
only against the centroids that Clause 2 cannot exclude, per block of 64
survivors of one cluster sorted by bound): labels at every iteration and
FP64 centroids bit-exact against the FP64 oracle, over shapes that span the
tile's row widths, ragged k, clusters with more survivors than one sorted
round holds, integer data with exact ties, the learned proposal and the
exact-mean update."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _knor():
    import paper_1606_08905_amd as knor
    knor.load()
    return knor


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(X, C0, k, iters, exact_mean=False, **kw):
    knor = _knor()
    X64 = X.astype(np.float64)
    print("CASE clause2", X.shape, k, iters, kw, flush=True)
    ref = oracle.mti_fit(X64, C0, iters, history=True, exact_mean=exact_mean)
    C, lab, st = knor.fit(_dev(X), k, C0=_dev(C0), max_iters=iters, prune=True,
                          history=True, counters=True,
                          update="exact" if exact_mean else "canonical", **kw)
    assert st["iters"] == ref.iters
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), f"iteration {t}"
    assert (C.cpu().numpy() == ref.C).all()
    assert st["counters"][:, 0].tolist() == ref.changed.tolist()
    return st


def _mixture(n, d, kc, seed, spread=10.0, sigma=(0.5, 3.0)):
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.0, spread, size=(kc, d))
    sig = rng.uniform(*sigma, size=kc)
    X = workloads.gaussian_mixture(rng, n, mu, sig, np.ones(kc), "f32")
    rows = workloads.distinct_rows(rng, n, kc)
    return X, X[rows].astype(np.float64)


def test_large_k_workload_reduced():
    """The large-k workload's recipe at n = 1e5, k = 1024 (on by default)."""
    w = workloads.config(5, n=100000, k=1024)
    st = _compare(w.X, w.C0, w.k, 25)
    ctr = st["counters"]
    # after the first iterations the survivors scan far fewer than k each
    assert ctr[5:, 7].sum() < 0.5 * (ctr[5:, 1].sum() * w.k)


@pytest.mark.parametrize("n,d,k,seed", [(20000, 7, 300, 1), (30000, 33, 100, 2),
                                        (15000, 100, 64, 3), (8000, 256, 40, 4),
                                        (40000, 16, 17, 5), (25000, 32, 2000, 6)])
def test_shapes(n, d, k, seed):
    X, C0 = _mixture(n, d, k, seed)
    _compare(X, C0, k, 15, clause2="on")


def test_clusters_larger_than_a_sorted_round():
    """k = 8 over 60000 uniform points: thousands of survivors per cluster,
    taken in several rounds of at most 2048."""
    X = workloads.uniform_cube(60000, 8, "f32", seed=11)
    _compare(X, X[:8].astype(np.float64), 8, 20, clause2="on")


def test_integer_data_with_ties():
    rng = np.random.default_rng(2)
    base = rng.integers(-4, 5, size=(300, 4)).astype(np.float32)
    Xd = base[rng.integers(0, 300, size=20000)]
    st = _compare(Xd, Xd[:40].astype(np.float64), 40, 30, clause2="on")
    print("integer ties: rechecked", st["rechecked"], flush=True)


def test_uniform_near_ties_recheck_path():
    X = workloads.uniform_cube(30000, 8, "f32", seed=3)
    st = _compare(X, X[:64].astype(np.float64), 64, 25, clause2="on")
    print("uniform: rechecked", st["rechecked"], flush=True)


def test_on_and_off_agree_and_on_computes_less():
    knor = _knor()
    w = workloads.config(5, n=200000, k=2048, seed=1)
    X, C0 = _dev(w.X), _dev(w.C0)
    outs = {}
    for c2 in ("off", "on"):
        outs[c2] = knor.fit(X, w.k, C0=C0, max_iters=20, clause2=c2, counters=True)
    (Ca, la, sa), (Cb, lb, sb) = outs["off"], outs["on"]
    assert (Ca == Cb).all() and (la == lb).all() and sa["iters"] == sb["iters"]
    assert sb["dists_computed"] < 0.6 * sa["dists_computed"]


def test_with_learned_proposal():
    w = workloads.config(5, n=60000, k=1024, seed=3)
    st = _compare(w.X, w.C0, w.k, 12, learned=True, train_iters=3)
    assert st["mlp_queries"] > 0


def test_with_exact_update():
    w = workloads.config(5, n=60000, k=1024, seed=4)
    _compare(w.X, w.C0, w.k, 20, exact_mean=True)


def test_learned_with_exact_update():
    """The certificate relabels points before the Clause-2 tile; the exact
    update's member counts must still move each relabelled point once."""
    w = workloads.config(5, n=60000, k=1024, seed=5)
    st = _compare(w.X, w.C0, w.k, 20, exact_mean=True, learned=True, train_iters=3)
    assert st["mlp_queries"] > 0
