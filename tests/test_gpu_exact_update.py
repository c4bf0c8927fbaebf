"""GPU parity of the exact update (update="exact") against the oracle's
exactly rounded mean.

Bars: centroids bit-exact (both sides round the exact member mean once, to
nearest with ties to even); counts and labels bit-exact at every iteration.
The GPU fit moves only changed points between the clusters' exact sums
when few change (delta mode) and re-sums dirty clusters from the sorted
members otherwise (full mode); both modes occur in the fits below.
"""
import numpy as np
import pytest

import oracle
import workloads

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


def _print_case(**kw):
    print("CASE", kw, flush=True)


def _delta_max(n, d):
    # changed labels up to which the library moves points one by one
    return max(256, min(1 << 22, max((1 << 20) // (4 * d), n // 128)))


# ---------------------------------------------------------------------------
# one update
# ---------------------------------------------------------------------------

UPDATE_CASES = [(1, 4, 1), (100, 3, 5), (5000, 16, 10), (70000, 32, 100),
                (20000, 64, 1000), (9000, 33, 4096), (3000, 256, 7), (4097, 65, 3)]


@pytest.mark.parametrize("n,d,k", UPDATE_CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_exact_update_parity(n, d, k, dtype):
    knor = _knor()
    _print_case(test="exact-update", n=n, d=d, k=k, dtype=dtype)
    rng = np.random.default_rng(n * 11 + k)
    X = workloads.cast(rng.normal(size=(n, d)) * 5 + 2, dtype)
    lab = (rng.zipf(1.5, size=n) % k).astype(np.int32)   # skewed, empty clusters
    Cp = rng.normal(size=(k, d))
    C_o, cnt_o = oracle.update_exact(workloads.to_f64(X, dtype), lab, Cp)
    C, cnt = knor.update(_dev(X, dtype), _dev(lab, None), _dev(Cp, "f64"), mode="exact")
    assert (cnt.cpu().numpy() == cnt_o).all()
    assert (C.cpu().numpy() == C_o).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_exact_update_wide_exponents(dtype):
    """Values from subnormal to 1e37 with both signs in one cluster, and
    cancellation: every digit of the fixed-point sum is used."""
    knor = _knor()
    rng = np.random.default_rng(3)
    n, d, k = 6000, 24, 5
    mag = 10.0 ** rng.integers(-44, 37, size=(n, d)).astype(np.float64)
    X = rng.normal(size=(n, d)) * mag
    X[::7, 3] = 1e37
    X[1::7, 3] = -1e37                               # cancels except a remainder
    X[:, 5] = 0.0
    X[::3, 6] = -0.0
    X = workloads.cast(X, dtype)
    lab = rng.integers(0, k, size=n).astype(np.int32)
    Cp = rng.normal(size=(k, d))
    C_o, cnt_o = oracle.update_exact(workloads.to_f64(X, dtype), lab, Cp)
    C, cnt = knor.update(_dev(X, dtype), _dev(lab, None), _dev(Cp, "f64"), mode="exact")
    assert (cnt.cpu().numpy() == cnt_o).all()
    assert (C.cpu().numpy() == C_o).all()


def test_exact_update_ties_round_to_even():
    """Means of FP32 members that lie exactly halfway between two doubles
    (hand-derived): (2^30 + 2^-23) / 2 = 2^29 + 2^-24 is half an ulp above
    2^29 (even) and rounds down; (2^30 + 1.5 2^-22) / 2 = 2^29 + 2^-23 +
    2^-24 is half an ulp above 2^29 + 2^-23 (odd) and rounds up to
    2^29 + 2^-22; a third member off the tie rounds to nearest."""
    knor = _knor()
    X = np.array([[2.0 ** 30], [2.0 ** -23],
                  [2.0 ** 30], [1.5 * 2.0 ** -22],
                  [2.0 ** 30], [2.0 ** -23], [2.0 ** -23]], np.float32)
    lab = np.array([0, 0, 1, 1, 2, 2, 2], np.int32)
    Cp = np.zeros((3, 1))
    C, _ = knor.update(_dev(X, "f32"), _dev(lab, None), _dev(Cp, "f64"), mode="exact")
    C = C.cpu().numpy()[:, 0]
    assert C[0] == 2.0 ** 29
    assert C[1] == 2.0 ** 29 + 2.0 ** -22
    # (2^30 + 2^-22) / 3: compared with the oracle's exact mean
    C_o, _ = oracle.update_exact(X.astype(np.float64), lab, Cp)
    assert (C == C_o[:, 0]).all()


def test_exact_update_rejects_f64():
    knor = _knor()
    import torch
    X = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    lab = torch.zeros(10, dtype=torch.int32, device="cuda")
    Cp = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(knor.KnorError) as ei:
        knor.update(X, lab, Cp, mode="exact")
    assert ei.value.code == 5                        # KNOR_ERR_UNSUPPORTED
    with pytest.raises(knor.KnorError) as ei:
        knor.fit(X, 2, C0=Cp, max_iters=3, update="exact")
    assert ei.value.code == 5


# ---------------------------------------------------------------------------
# fits: identical labels at every iteration, bit-exact centroids
# ---------------------------------------------------------------------------

def _fit_exact_compare(X, dtype, C0, k, iters, prune, tol=0.0):
    knor = _knor()
    X64 = workloads.to_f64(X, dtype)
    if prune:
        ref = oracle.mti_fit(X64, C0, iters, tol=tol, history=True, exact_mean=True)
    else:
        ref = oracle.fit_exact_mean(X64, C0, iters, tol=tol, history=True)
    C, lab, st = knor.fit(_dev(X, dtype), k, C0=_dev(C0, "f64"), max_iters=iters,
                          tol=tol, prune=prune, history=True, counters=True,
                          update="exact")
    assert st["iters"] == ref.iters
    assert bool(st["converged"]) == ref.converged
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), f"iteration {t}"
    assert (lab.cpu().numpy() == ref.labels).all()
    assert (C.cpu().numpy() == ref.C).all()
    assert st["counters"][:, 0].tolist() == ref.changed.tolist()
    return st, ref


@pytest.mark.parametrize("prune", [False, True])
def test_exact_fit_config2_modes(prune):
    """Early iterations change more labels than the delta limit (full mode),
    later ones fewer (delta mode)."""
    w = workloads.config(2, n=500000, seed=1)
    _print_case(test="exact-fit-config2", prune=prune)
    st, ref = _fit_exact_compare(w.X, w.dtype, w.C0, w.k, 60, prune)
    lim = _delta_max(*w.X.shape)
    ch = ref.changed.tolist()
    assert any(c > lim for c in ch[1:]) and any(0 < c <= lim for c in ch[1:]), ch


@pytest.mark.parametrize("n,d,k,seed", [(30000, 3, 7, 1), (20000, 33, 40, 2),
                                        (8000, 128, 20, 3), (6000, 256, 9, 4),
                                        (12000, 16, 600, 5), (5000, 70, 3000, 6)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_exact_fit_shapes(n, d, k, seed, dtype):
    rng = np.random.default_rng(seed)
    kc = max(2, min(k, 64))
    mu = rng.uniform(-10, 10, size=(kc, d))
    X = workloads.gaussian_mixture(rng, n, mu, np.ones(kc), np.ones(kc), dtype)
    rows = workloads.distinct_rows(rng, n, k)
    C0 = workloads.to_f64(X[rows], dtype).copy()
    _print_case(test="exact-fit-shapes", n=n, d=d, k=k, dtype=dtype)
    _fit_exact_compare(X, dtype, C0, k, 15, True)


@pytest.mark.parametrize("poll_every", [1, 3])
def test_exact_fit_delta_only_after_poll(poll_every):
    """The host stops launching the full pass at the first convergence poll
    that sees few changes; centroids and labels are unchanged."""
    knor = _knor()
    w = workloads.config(2, n=100000, seed=5)
    ref = oracle.mti_fit(w.x64(), w.C0, 40, history=True, exact_mean=True)
    C, lab, st = knor.fit(_dev(w.X, "f32"), w.k, C0=_dev(w.C0, "f64"), max_iters=40,
                          history=True, update="exact", poll_every=poll_every)
    assert st["iters"] == ref.iters
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), f"iteration {t}"
    assert (C.cpu().numpy() == ref.C).all()


def test_exact_fit_mixed_magnitudes():
    """Coordinates spanning 40 decades (tiny ones near FP32's subnormal
    range) move between clusters in delta mode."""
    rng = np.random.default_rng(8)
    n, d, k = 40000, 8, 12
    mu = rng.uniform(-50, 50, size=(k, d))
    X = workloads.gaussian_mixture(rng, n, mu, np.full(k, 4.0), np.ones(k), "f32")
    tiny = rng.random((n, d)) < 0.2
    X = np.where(tiny, X * np.float32(1e-36), X).astype(np.float32)
    C0 = X[workloads.distinct_rows(rng, n, k)].astype(np.float64)
    _print_case(test="exact-fit-mixed-magnitudes")
    st, ref = _fit_exact_compare(X, "f32", C0, k, 40, True)


def test_exact_fit_tol_and_empty_clusters():
    """A centroid far from every point loses all members and keeps its
    value; the fit stops on the tolerance."""
    rng = np.random.default_rng(9)
    X = rng.normal(size=(5000, 4)).astype(np.float32)
    C0 = np.vstack([X[:5].astype(np.float64), np.full((1, 4), 1e6)])
    _print_case(test="exact-fit-empty")
    st, ref = _fit_exact_compare(X, "f32", C0, 6, 50, True, tol=1e-3)
    assert ref.C[5, 0] == 1e6


def test_exact_fit_config2_full_size():
    """The benchmark workload (n = 1e6, d = 32, k = 100, MTI) with the exact
    update, against the oracle's MTI loop with the exact mean."""
    w = workloads.config(2)
    _print_case(test="exact-fit-config2-full")
    st, ref = _fit_exact_compare(w.X, w.dtype, w.C0, w.k, w.max_iters, True)
    print("exact config2 iters", st["iters"], flush=True)


@pytest.mark.parametrize("graph", [False, True])
def test_exact_fit_batched_equals_single(graph):
    knor = _knor()
    probs, singles = [], []
    for i, (n, d, k) in enumerate([(20000, 16, 30), (9000, 32, 100), (15000, 8, 7)]):
        rng = np.random.default_rng(20 + i)
        mu = rng.uniform(-10, 10, size=(k, d))
        X = workloads.gaussian_mixture(rng, n, mu, np.ones(k), np.ones(k), "f32")
        C0 = X[workloads.distinct_rows(rng, n, k)].astype(np.float64)
        probs.append({"X": _dev(X, "f32"), "k": k, "C0": C0, "max_iters": 25})
        singles.append(knor.fit(_dev(X, "f32"), k, C0=_dev(C0, "f64"), max_iters=25,
                                update="exact"))
    out = knor.fit_batched(probs, update="exact", graph=graph)
    for (C, lab, st), (C1, lab1, st1) in zip(out, singles):
        assert (C.cpu().numpy() == C1.cpu().numpy()).all()
        assert (lab.cpu().numpy() == lab1.cpu().numpy()).all()
        assert st["iters"] == st1["iters"]
