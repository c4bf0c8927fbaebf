"""GPU parity of the streamed fit (knor_fit_streamed: rows in pinned host
memory, processed in batches, with the lazily refreshed row cache of the
paper's semi-external-memory mode) against the oracle's exact-mean reading.

Bars: labels bit-exact at every iteration, centroids bit-exact, the same
iteration count; and the host-link accounting that defines the mode: a full
pass copies every row once, an MTI iteration reads exactly the rows of the
points that fail Clause 1 (from the cache or from host memory), the cache
serves nothing before its first refresh and is refilled only at the refresh
iterations I, 3I, 7I, ...
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


def _pinned(a, dtype):
    import torch
    if dtype == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a))
    return t.pin_memory()


def _dev(a, dtype):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda().view(
            torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _print_case(**kw):
    print("CASE", kw, flush=True)


def _refresh_iters(I, upto):
    out, r, gap = [], I, 2 * I
    while r < upto:
        out.append(r)
        r += gap
        gap *= 2
    return out


def _check_io(st, n, prune, cache_rows, interval, objective):
    io = st["io"]
    cnt = st["counters"]
    iters = st["iters"]
    refresh = set(_refresh_iters(interval, iters)) if (prune and cache_rows) else set()
    for t in range(iters):
        copied, gathered, cached, admitted = (int(v) for v in io[t])
        extra = n if (objective and t == iters - 1) else 0
        if not prune or t == 0:
            assert copied == n + extra, (t, io[t])
            assert gathered == cached == admitted == 0, (t, io[t])
            continue
        # every point that fails Clause 1 has its row read once, no other
        cand = n - int(cnt[t][2])
        assert copied == extra, (t, io[t])
        assert gathered + cached == cand, (t, io[t], cand)
        if not cache_rows or t <= interval:
            assert cached == 0, (t, io[t])
        if t in refresh:
            assert admitted == min(cache_rows, cand), (t, io[t], cand)
        else:
            assert admitted == 0, (t, io[t])


def _stream_compare(X, dtype, C0, k, iters, prune=True, batch_rows=8192, cache_rows=0,
                    interval=2, objective=True, tol=0.0):
    knor = _knor()
    n = X.shape[0]
    X64 = workloads.to_f64(X, dtype)
    if prune:
        ref = oracle.mti_fit(X64, C0, iters, tol=tol, history=True, exact_mean=True)
    else:
        ref = oracle.fit_exact_mean(X64, C0, iters, tol=tol, history=True)
    C, lab, st = knor.fit_streamed(_pinned(X, dtype), k, C0=C0, max_iters=iters, tol=tol,
                                   prune=prune, history=True, counters=True,
                                   batch_rows=batch_rows, cache_rows=cache_rows,
                                   cache_interval=interval, objective=objective)
    assert st["iters"] == ref.iters
    assert bool(st["converged"]) == ref.converged
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), f"iteration {t}"
    assert (lab.cpu().numpy() == ref.labels).all()
    assert (C.cpu().numpy() == ref.C).all()
    assert st["counters"][:, 0].tolist() == ref.changed.tolist()
    _check_io(st, n, prune, cache_rows, interval, objective)
    if objective:
        assert st["objective"] == oracle.objective(X64, ref.C, ref.labels)
    return st, ref


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n,d,k,batch,cache", [
    (50001, 16, 40, 8192, 6000),     # ragged tail, several batches, small cache
    (30000, 5, 12, 4096, 30000),     # rows that are not a multiple of 16 bytes
    (12289, 33, 64, 0, 2000),        # one batch (default size), odd d
    (20000, 64, 300, 16384, 0),      # no cache
])
def test_streamed_fit_matches_oracle(dtype, n, d, k, batch, cache):
    _print_case(test="streamed-fit", dtype=dtype, n=n, d=d, k=k, batch=batch, cache=cache)
    rng = np.random.default_rng(n + d + k)
    kc = max(2, min(k, 48))
    mu = rng.uniform(-10, 10, size=(kc, d))
    X = workloads.gaussian_mixture(rng, n, mu, np.full(kc, 1.5), np.ones(kc), dtype)
    C0 = workloads.to_f64(X[workloads.distinct_rows(rng, n, k)], dtype).copy()
    st, ref = _stream_compare(X, dtype, C0, k, 25, batch_rows=batch, cache_rows=cache)
    if cache and ref.iters > 4:
        assert st["io"][3:, 2].sum() > 0      # the cache served rows after its refresh


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_streamed_fit_without_pruning(dtype):
    """Every iteration is a full pass: each batch is copied whole."""
    rng = np.random.default_rng(3)
    n, d, k = 20000, 8, 10
    X = workloads.gaussian_mixture(rng, n, rng.uniform(-5, 5, (k, d)), np.ones(k),
                                   np.ones(k), dtype)
    C0 = workloads.to_f64(X[workloads.distinct_rows(rng, n, k)], dtype).copy()
    _print_case(test="streamed-no-prune", dtype=dtype)
    _stream_compare(X, dtype, C0, k, 12, prune=False, batch_rows=4096, objective=False)


def test_streamed_equals_in_memory_fit():
    """Same labels, centroids, counters and objective as knor_fit with the
    exact update on the same values (the config-2 workload, 300k points),
    with a cache smaller than the active set."""
    knor = _knor()
    w = workloads.config(2, n=300000, seed=4)
    _print_case(test="streamed-vs-fit")
    C1, l1, s1 = knor.fit(_dev(w.X, "f32"), w.k, C0=_dev(w.C0, "f64"), max_iters=30,
                          history=True, counters=True, update="exact")
    C2, l2, s2 = knor.fit_streamed(_pinned(w.X, "f32"), w.k, C0=w.C0, max_iters=30,
                                   history=True, counters=True, batch_rows=65536,
                                   cache_rows=20000, cache_interval=3)
    assert s1["iters"] == s2["iters"]
    assert (s1["label_history"].cpu() == s2["label_history"].cpu()).all()
    assert (C1.cpu() == C2.cpu()).all()
    assert (s1["counters"][:, :6] == s2["counters"][:, :6]).all()
    assert s1["objective"] == s2["objective"]
    _check_io(s2, w.X.shape[0], True, 20000, 3, True)
    io = s2["io"]
    print("streamed io per iteration (copied, gathered, cached, admitted):",
          io.tolist(), flush=True)


@pytest.mark.parametrize("init", ["forgy", "shuffle_first_k"])
def test_streamed_seeded_init(init):
    """The seeded init modes read their k rows from host memory and pick the
    same rows as knor_fit."""
    knor = _knor()
    rng = np.random.default_rng(11)
    n, d, k = 30000, 12, 20
    X = workloads.gaussian_mixture(rng, n, rng.uniform(-8, 8, (k, d)), np.ones(k),
                                   np.ones(k), "f32")
    _print_case(test="streamed-init", init=init)
    C1, l1, s1 = knor.fit(_dev(X, "f32"), k, init=init, seed=77, max_iters=15,
                          update="exact")
    C2, l2, s2 = knor.fit_streamed(_pinned(X, "f32"), k, init=init, seed=77, max_iters=15,
                                   batch_rows=8192, cache_rows=5000)
    assert s1["iters"] == s2["iters"]
    assert (l1.cpu() == l2.cpu()).all()
    assert (C1.cpu() == C2.cpu()).all()


def test_streamed_rows_at_an_offset():
    """X may start inside a pinned allocation (a row slice of a pinned
    tensor); the rows before it are never read."""
    knor = _knor()
    rng = np.random.default_rng(12)
    n, d, k = 10000, 8, 6
    X = workloads.gaussian_mixture(rng, n + 7, rng.uniform(-8, 8, (k, d)), np.ones(k),
                                   np.ones(k), "f32")
    base = _pinned(X, "f32")
    view = base[7:]
    C0 = X[7:][workloads.distinct_rows(rng, n, k)].astype(np.float64)
    _print_case(test="streamed-offset")
    ref = oracle.mti_fit(X[7:].astype(np.float64), C0, 20, history=False, exact_mean=True)
    C, lab, st = knor.fit_streamed(view, k, C0=C0, max_iters=20, batch_rows=4096)
    assert st["iters"] == ref.iters
    assert (lab.cpu().numpy() == ref.labels).all()
    assert (C.cpu().numpy() == ref.C).all()


def test_streamed_rejects_device_rows():
    import torch
    knor = _knor()
    L = knor.load()
    X = torch.zeros((100, 4), device="cuda")
    C = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    lab = torch.zeros(100, dtype=torch.int32, device="cuda")
    import ctypes
    o = knor._opts(update="exact")
    rc = L.knor_fit_streamed(X.data_ptr(), 1, 100, 4, 3, 0, C.data_ptr(), 5, 0.0,
                             ctypes.byref(o), None, C.data_ptr(), lab.data_ptr(), None)
    assert rc == knor.KNOR_ERR_INVALID_ARG


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_streamed_numeric_check(dtype):
    """A NaN in the fourth batch is caught as its rows arrive in iteration 0
    (KNOR_ERR_NUMERIC); a NaN in the initial centroids before any pass; the
    library is usable afterwards."""
    import torch
    knor = _knor()
    rng = np.random.default_rng(21)
    n, d, k = 20000, 8, 5
    X = workloads.cast(rng.normal(size=(n, d)), dtype)
    C0 = workloads.to_f64(X[:k], dtype).copy()
    bad = X.copy()
    bad[3 * 4096 + 17, 5] = workloads.cast(np.array([np.nan]), dtype)[0]
    _print_case(test="streamed-numeric", dtype=dtype)
    with pytest.raises(knor.KnorError) as e:
        knor.fit_streamed(_pinned(bad, dtype), k, C0=C0, max_iters=5, batch_rows=4096)
    assert e.value.code == knor.KNOR_ERR_NUMERIC
    C0n = C0.copy()
    C0n[2, 1] = np.nan
    with pytest.raises(knor.KnorError) as e:
        knor.fit_streamed(_pinned(X, dtype), k, C0=C0n, max_iters=5, batch_rows=4096)
    assert e.value.code == knor.KNOR_ERR_NUMERIC
    ref = oracle.mti_fit(workloads.to_f64(X, dtype), C0, 5, exact_mean=True)
    C, lab, st = knor.fit_streamed(_pinned(X, dtype), k, C0=C0, max_iters=5, batch_rows=4096)
    assert (C.cpu().numpy() == ref.C).all()


def test_streamed_split_adds_large_n():
    """n >= 2^23: every point's entry at iteration 0 and every move after it
    goes to the digits in two pieces (the split form); labels and centroids
    still equal the oracle's exact-mean reading."""
    knor = _knor()
    rng = np.random.default_rng(31)
    n, d, k = (1 << 23) + 4097, 4, 8
    mu = rng.uniform(-6, 6, size=(k, d))
    X = workloads.gaussian_mixture(rng, n, mu, np.full(k, 2.0), np.ones(k), "f32")
    C0 = X[workloads.distinct_rows(rng, n, k)].astype(np.float64)
    _print_case(test="streamed-split", n=n)
    ref = oracle.mti_fit(X.astype(np.float64), C0, 4, history=False, exact_mean=True)
    C, lab, st = knor.fit_streamed(_pinned(X, "f32"), k, C0=C0, max_iters=4,
                                   batch_rows=1 << 21, cache_rows=1 << 20, cache_interval=1)
    assert st["iters"] == ref.iters
    assert (lab.cpu().numpy() == ref.labels).all()
    assert (C.cpu().numpy() == ref.C).all()
