"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Bars: labels bit-exact (integer results); FP64 centroids bit-exact (both
sides use the same canonical summation order and correctly rounded FP64
division); the FP64 objective bit-exact (same canonical order).  Every call
goes through the C ABI via the thin binding.
"""
import math

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


def _data(n, d, k, dtype="f32", seed=0, scale=1.0, shift=0.0):
    rng = np.random.default_rng(seed)
    kc = max(2, min(k, 64))
    mu = rng.uniform(-10, 10, size=(kc, d)) * scale + shift
    X = workloads.gaussian_mixture(rng, n, mu, np.full(kc, scale), np.ones(kc), dtype)
    rows = workloads.distinct_rows(rng, n, k)
    C = workloads.to_f64(X[rows], dtype).copy()
    return X, C


def _print_case(**kw):
    print("CASE", kw, flush=True)


# ---------------------------------------------------------------------------
# assignment
# ---------------------------------------------------------------------------

ASSIGN_CASES = [
    # n, d, k   (ragged n, d not a power of two, k not a multiple of 16)
    (1, 3, 1), (100, 3, 2), (1000, 8, 7), (4097, 16, 16), (5000, 32, 100),
    (3001, 33, 17), (2500, 64, 257), (2000, 100, 50), (1500, 128, 33),
    (1000, 256, 20), (20000, 32, 1000), (777, 5, 300),
]


@pytest.mark.parametrize("n,d,k", ASSIGN_CASES)
@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_assign_parity(n, d, k, dtype):
    knor = _knor()
    _print_case(test="assign", n=n, d=d, k=k, dtype=dtype)
    X, C = _data(n, d, k, dtype, seed=n + d + k)
    lab_o, D_o = oracle.assign(workloads.to_f64(X, dtype), C)
    lab, dd = knor.assign(_dev(X, dtype), _dev(C, "f64"), dist2=True)
    assert (lab.cpu().numpy() == lab_o).all()
    assert (dd.cpu().numpy() == D_o).all()


@pytest.mark.parametrize("recheck", [1, 2])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_assign_ties_and_duplicates(recheck, dtype):
    """Integer data: many exact ties; the lowest index must win."""
    knor = _knor()
    rng = np.random.default_rng(5)
    X = workloads.cast(rng.integers(-3, 4, size=(5000, 8)).astype(np.float64), dtype)
    C = rng.integers(-3, 4, size=(40, 8)).astype(np.float64)
    C[20:] = C[:20]                       # duplicated centroids: exact ties
    lab_o, _ = oracle.assign(workloads.to_f64(X, dtype), C)
    lab = knor.assign(_dev(X, dtype), _dev(C, "f64"), recheck=recheck)
    assert (lab.cpu().numpy() == lab_o).all()


@pytest.mark.parametrize("scale,shift", [(1e-3, 0.0), (1.0, 1e4), (1e3, 0.0), (1.0, -3e5)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_assign_far_from_origin(scale, shift, dtype):
    """Large |x| relative to the cluster spread stresses the error bound."""
    knor = _knor()
    X, C = _data(6000, 32, 50, dtype, seed=3, scale=scale, shift=shift)
    lab_o, _ = oracle.assign(workloads.to_f64(X, dtype), C)
    lab = knor.assign(_dev(X, dtype), _dev(C, "f64"))
    assert (lab.cpu().numpy() == lab_o).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n,d,k", [(20000, 16, 48), (20000, 64, 48),
                                   (300000, 16, 48), (20000, 32, 1000)])
def test_assign_near_bisectors(dtype, n, d, k):
    """Points placed on and near the bisecting hyperplanes of centroid pairs
    (then rounded to the storage type): the squared-distance gaps fall
    around the tile's decision threshold, so a bound that is too small shows
    up as a label that differs from the oracle.  Nearly every point is
    undecided by the tile with a clear third centroid, so the FP32 tile
    resolves it from its two best centroids; n = 3e5 puts more such points
    into a workgroup than its list holds (the rest take the full recheck),
    k = 1000 runs the chunked schedule."""
    knor = _knor()
    _print_case(test="near_bisectors", n=n, d=d, k=k, dtype=dtype)
    rng = np.random.default_rng(40 + d + k)
    C = rng.normal(size=(k, d)) * 4.0
    a = rng.integers(0, k, size=n)
    b = (a + 1 + rng.integers(0, k - 1, size=n)) % k
    mid = 0.5 * (C[a] + C[b])
    step = (C[b] - C[a]) * rng.uniform(-1e-3, 1e-3, size=(n, 1))
    X = workloads.cast(mid + step, dtype)
    lab_o, _ = oracle.assign(workloads.to_f64(X, dtype), C)
    lab = knor.assign(_dev(X, dtype), _dev(C, "f64"))
    assert (lab.cpu().numpy() == lab_o).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_assign_near_three_way_ties(dtype):
    """Points near the circumcentre of three centroids (inside their plane):
    three squared distances fall within the tile's margin, so even the two
    best cannot be trusted and the point must take the full FP64 recheck."""
    knor = _knor()
    rng = np.random.default_rng(77)
    k, d, n = 48, 16, 20000
    C = rng.normal(size=(k, d)) * 4.0
    a = rng.integers(0, k, size=n)
    b = (a + 1 + rng.integers(0, k - 1, size=n)) % k
    c = (b + 1 + rng.integers(0, k - 2, size=n)) % k
    c = np.where(c == a, (c + 1) % k, c)
    Ca, Cb, Cc = C[a], C[b], C[c]
    u, v = Cb - Ca, Cc - Ca
    # P = Ca + s u + t v with |P - Ca| = |P - Cb| = |P - Cc|
    uu, uv, vv = (u * u).sum(1), (u * v).sum(1), (v * v).sum(1)
    r1, r2 = 0.5 * uu, 0.5 * vv
    det = uu * vv - uv * uv
    s = (r1 * vv - r2 * uv) / det
    t = (r2 * uu - r1 * uv) / det
    P = Ca + s[:, None] * u + t[:, None] * v
    P += rng.normal(size=P.shape) * 1e-4
    X = workloads.cast(P, dtype)
    lab_o, D_o = oracle.assign(workloads.to_f64(X, dtype), C)
    lab = knor.assign(_dev(X, dtype), _dev(C, "f64"))
    assert (lab.cpu().numpy() == lab_o).all()


# ---------------------------------------------------------------------------
# update
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,k", [(1, 4, 1), (100, 3, 5), (5000, 16, 10),
                                   (70000, 32, 100), (20000, 64, 1000),
                                   (9000, 33, 4096), (3000, 256, 7)])
@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_update_parity(n, d, k, dtype):
    knor = _knor()
    _print_case(test="update", n=n, d=d, k=k, dtype=dtype)
    rng = np.random.default_rng(n * 7 + k)
    X = workloads.cast(rng.normal(size=(n, d)) * 5, dtype)
    # skewed labels with empty clusters
    lab = (rng.zipf(1.5, size=n) % k).astype(np.int32)
    Cp = rng.normal(size=(k, d))
    C_o, cnt_o = oracle.update(workloads.to_f64(X, dtype), lab, Cp)
    C, cnt = knor.update(_dev(X, dtype), _dev(lab, None), _dev(Cp, "f64"))
    assert (cnt.cpu().numpy() == cnt_o).all()
    assert (C.cpu().numpy() == C_o).all()


# ---------------------------------------------------------------------------
# fit: identical labels at every iteration, bit-exact centroids
# ---------------------------------------------------------------------------

def _fit_compare(w_X, dtype, C0, k, iters, prune, recheck=1, tol=0.0,
                 oracle_fit=None):
    knor = _knor()
    X64 = workloads.to_f64(w_X, dtype)
    # the MTI oracle's labels equal plain Lloyd's at every iteration (pinned
    # in test_oracle_pins); it is used where the plain oracle is too slow
    ref = (oracle_fit or oracle.fit)(X64, C0, iters, tol=tol, history=True)
    C, lab, st = knor.fit(_dev(w_X, dtype), k, C0=_dev(C0, "f64"),
                          max_iters=iters, tol=tol, prune=prune,
                          recheck=recheck, history=True, counters=True)
    assert st["iters"] == ref.iters
    assert bool(st["converged"]) == ref.converged
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), f"iteration {t}"
    assert (lab.cpu().numpy() == ref.labels).all()
    assert (C.cpu().numpy() == ref.C).all()
    assert st["counters"][:, 0].tolist() == ref.changed.tolist()
    obj = oracle.objective(X64, ref.C, ref.labels)
    assert st["objective"] == obj
    return st, ref


@pytest.mark.parametrize("prune", [False, True])
def test_fit_config1_full(prune):
    w = workloads.config(1)
    _print_case(test="fit-config1", prune=prune)
    _fit_compare(w.X, w.dtype, w.C0, w.k, w.max_iters, prune)


@pytest.mark.parametrize("prune", [False, True])
@pytest.mark.parametrize("seed", [0, 2])
def test_fit_config2_small(prune, seed):
    w = workloads.config(2, n=40000, seed=seed)
    _print_case(test="fit-config2-small", prune=prune, seed=seed)
    st, ref = _fit_compare(w.X, w.dtype, w.C0, w.k, 60, prune)
    if prune:
        # most points are decided by the bounds after the first iterations
        assert st["pruned_a"] + st["pruned_b"] > 0.3 * 40000 * (st["iters"] - 1)


@pytest.mark.parametrize("prune", [False, True])
def test_fit_config3_small(prune):
    """The mixed-precision workload (BF16 points, d=64, k=256, 5% uniform
    outliers) at a reduced n."""
    w = workloads.config(3, n=30000)
    _print_case(test="fit-config3-small", prune=prune)
    st, ref = _fit_compare(w.X, w.dtype, w.C0, w.k, w.max_iters, prune,
                           oracle_fit=oracle.mti_fit)
    print("config3-small rechecked", st["rechecked"], "of", 30000 * st["iters"],
          flush=True)


def test_fit_bf16_shapes():
    for (n, d, k, seed) in [(5000, 3, 7, 1), (8000, 33, 40, 2), (3000, 128, 20, 3),
                            (2000, 256, 9, 4), (6000, 16, 600, 5)]:
        X, C0 = _data(n, d, k, "bf16", seed=seed)
        _print_case(test="fit-bf16", n=n, d=d, k=k)
        _fit_compare(X, "bf16", C0, k, 12, True, oracle_fit=oracle.mti_fit)


def test_fit_recheck_all_equals_oracle():
    w = workloads.config(2, n=8000, k=30, seed=4)
    _fit_compare(w.X, w.dtype, w.C0, w.k, 30, True, recheck=2)


def test_fit_tol_early_stop():
    w = workloads.config(2, n=20000, k=40, seed=5)
    _fit_compare(w.X, w.dtype, w.C0, w.k, 50, True, tol=0.01)


def test_fit_uniform_and_duplicates():
    X = workloads.uniform_cube(30000, 8, "f32", seed=3)
    _fit_compare(X, "f32", X[:64].astype(np.float64), 64, 25, True)
    rng = np.random.default_rng(2)
    base = rng.integers(-4, 5, size=(300, 4)).astype(np.float32)
    Xd = base[rng.integers(0, 300, size=20000)]
    _fit_compare(Xd, "f32", Xd[:12].astype(np.float64), 12, 30, True)


def test_fit_k_edge_cases():
    rng = np.random.default_rng(8)
    X = rng.normal(size=(300, 5)).astype(np.float32)
    _fit_compare(X, "f32", X[:1].astype(np.float64), 1, 5, True)
    _fit_compare(X, "f32", X.astype(np.float64), 300, 5, True)   # k = n


def _splitmix64(state):
    M = (1 << 64) - 1
    state = (state + 0x9E3779B97F4A7C15) & M
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return state, z ^ (z >> 31)


def _forgy_rows(n, k, seed):
    # the last k slots of a Fisher-Yates pass, i = n-1 down to n-k
    a = {}
    st = seed
    rows = []
    for r in range(k):
        i = n - 1 - r
        st, z = _splitmix64(st)
        j = z % (i + 1)
        vi, vj = a.get(i, i), a.get(j, j)
        a[i], a[j] = vj, vi
        rows.append(vj)
    return rows


def test_fit_forgy_init_matches_given():
    knor = _knor()
    w = workloads.config(1, n=5000)
    rows = _forgy_rows(5000, 10, 1234)
    C0 = w.x64()[rows]
    C1, l1, s1 = knor.fit(_dev(w.X, "f64"), 10, init="forgy", seed=1234, max_iters=20)
    C2, l2, s2 = knor.fit(_dev(w.X, "f64"), 10, C0=_dev(C0, "f64"), max_iters=20)
    assert (C1.cpu().numpy() == C2.cpu().numpy()).all()
    assert (l1.cpu().numpy() == l2.cpu().numpy()).all()


def test_fit_numeric_error_leaves_outputs():
    import torch
    knor = _knor()
    X = torch.randn(1000, 8, device="cuda")
    X[17, 3] = float("nan")
    C0 = X[:4].double().clone()
    C0[0] = 0
    C = torch.full((4, 8), 7.0, dtype=torch.float64, device="cuda")
    lab = torch.full((1000,), 3, dtype=torch.int32, device="cuda")
    with pytest.raises(knor.KnorError) as e:
        knor.fit(X, 4, C0=C0, out=(C, lab))
    assert e.value.code == knor.KNOR_ERR_NUMERIC
    assert (C == 7.0).all() and (lab == 3).all()


@pytest.mark.parametrize("dtype,prune,update", [("f32", True, "canonical"),
                                                 ("bf16", True, "exact"),
                                                 ("f64", False, "canonical"),
                                                 ("f32", False, "exact")])
def test_objective_history_matches_oracle(dtype, prune, update):
    """J_t at every iteration equals the oracle's traced objective bit for bit
    (same canonical distances, same canonical summation order), and the final
    objective too."""
    knor = _knor()
    w = workloads.config(2, n=60000, seed=3, k=30)
    X = workloads.cast(w.x64(), dtype)
    X64 = workloads.to_f64(X, dtype)
    ex = update == "exact"
    _print_case(test="objective-history", dtype=dtype, prune=prune, update=update)
    if prune:
        ref = oracle.mti_fit(X64, w.C0, 25, history=False, exact_mean=ex)
    elif ex:
        ref = oracle.fit_exact_mean(X64, w.C0, 25)
    else:
        ref = oracle.fit(X64, w.C0, 25)
    C, lab, st = knor.fit(_dev(X, dtype), w.k, C0=_dev(w.C0, "f64"), max_iters=25,
                          prune=prune, update=update, objective_history=True)
    assert st["iters"] == ref.iters
    assert st["objective_history"].tolist() == ref.objective.tolist()
    assert st["objective"] == oracle.objective(X64, ref.C, ref.labels)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("where", ["first", "middle", "last", "offset"])
def test_fit_numeric_check_positions(dtype, where):
    """The finite check sees every element: aligned vector pieces, the tail
    past the last whole 16-byte piece, and a start that is not 16-byte
    aligned (a view one row in)."""
    import torch
    knor = _knor()
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}[dtype]
    base = torch.randn(1002, 3, device="cuda").to(tdt)
    X = base[1:] if where == "offset" else base[:1001]
    X = X.contiguous() if where != "offset" else X
    flat = X.view(-1)
    pos = {"first": 0, "middle": 1500, "last": flat.numel() - 1, "offset": 7}[where]
    flat[pos] = float("inf") if where == "last" else float("nan")
    with pytest.raises(knor.KnorError) as e:
        knor.fit(X, 4, C0=torch.zeros((4, 3), dtype=torch.float64, device="cuda"))
    assert e.value.code == knor.KNOR_ERR_NUMERIC


def test_fit_workspace_cap():
    import torch
    knor = _knor()
    X = torch.randn(1000, 8, device="cuda")
    with pytest.raises(knor.KnorError) as e:
        knor.fit(X, 4, C0=X[:4].double(), workspace_cap=1024)
    assert e.value.code == knor.KNOR_ERR_OUT_OF_MEMORY


def test_profile_every_samples_iterations():
    """profile=(ms, launches, mask, every) times the masked groups only in
    iterations t with t % every == 0; the results do not change."""
    knor = _knor()
    w = workloads.config(2, n=30000, k=50, seed=1)
    Xd, C0d = _dev(w.X, "f32"), _dev(w.C0, "f64")
    ms = np.zeros(knor.NPROF)
    la = np.zeros(knor.NPROF, np.int64)
    list_g = knor.PROF_GROUPS.index("assign_list")
    C, lab, st = knor.fit(Xd, 50, C0=C0d, max_iters=25, profile=(ms, la, 1 << list_g, 2))
    sampled = [t for t in range(st["iters"]) if t >= 1 and t % 2 == 0]
    assert len(sampled) >= 1
    assert la[list_g] == len(sampled) and la.sum() == la[list_g]
    assert ms[list_g] > 0
    C2, lab2, _ = knor.fit(Xd, 50, C0=C0d, max_iters=25)
    assert (C == C2).all() and (lab == lab2).all()


def test_fit_deterministic_repeat():
    knor = _knor()
    w = workloads.config(2, n=30000, k=50, seed=1)
    Xd = _dev(w.X, "f32")
    a = knor.fit(Xd, 50, C0=_dev(w.C0, "f64"), max_iters=30)
    b = knor.fit(Xd, 50, C0=_dev(w.C0, "f64"), max_iters=30)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    assert a[2]["rechecked"] == b[2]["rechecked"]


def test_resume_equals_uninterrupted():
    """State (C, labels, t) resumes exactly: MTI is exact, so restarting from
    the centroids of iteration t reproduces the remaining iterations."""
    knor = _knor()
    w = workloads.config(2, n=20000, k=40, seed=6)
    Xd = _dev(w.X, "f32")
    Cfull, lfull, sfull = knor.fit(Xd, 40, C0=_dev(w.C0, "f64"), max_iters=25)
    Ca, la, sa = knor.fit(Xd, 40, C0=_dev(w.C0, "f64"), max_iters=10)
    Cb, lb, sb = knor.fit(Xd, 40, C0=Ca, max_iters=15)
    assert (Cb == Cfull).all() and (lb == lfull).all()


# ---------------------------------------------------------------------------
# full-size configuration 2 (the benchmark workload)
# ---------------------------------------------------------------------------

def test_fit_config2_full_size():
    w = workloads.config(2)
    _print_case(test="fit-config2-full")
    st, ref = _fit_compare(w.X, w.dtype, w.C0, w.k, w.max_iters, True,
                           oracle_fit=oracle.mti_fit)
    print("config2 iters", st["iters"], "rechecked", st["rechecked"], flush=True)


# ---------------------------------------------------------------------------
# FP32 tile schedules and the batched form
# ---------------------------------------------------------------------------

SCHEDULE_SHAPES = [(20000, 16, 50), (12000, 64, 300), (8000, 128, 40), (6000, 32, 2000)]


@pytest.mark.parametrize("n,d,k", SCHEDULE_SHAPES)
def test_tile_schedules_give_identical_results(n, d, k):
    """Every (blocks per wave, resident/chunked) schedule of the FP32 tile
    gives the oracle's labels at every iteration and its centroids."""
    knor = _knor()
    X, C0 = _data(n, d, k, "f32", seed=n + k)
    ref = oracle.mti_fit(X.astype(np.float64), C0, 8, history=True)
    ran = 0
    for res in (1, 2):
        for pb in (1, 2, 4):
            _print_case(test="schedule", n=n, d=d, k=k, pb=pb, res=res)
            try:
                C, lab, st = knor.fit(_dev(X, "f32"), k, C0=_dev(C0, "f64"),
                                      max_iters=8, history=True,
                                      tile_blocks=pb, tile_resident=res)
            except knor.KnorError as e:
                assert e.code == knor.KNOR_ERR_UNSUPPORTED
                continue
            ran += 1
            hist = st["label_history"].cpu().numpy()
            for t in range(ref.iters):
                assert (hist[t] == ref.label_hist[t]).all(), (pb, res, t)
            assert (C.cpu().numpy() == ref.C).all(), (pb, res)
    assert ran >= 2


def test_autotuned_fit_matches_default():
    knor = _knor()
    X, C0 = _data(30000, 32, 64, "f32", seed=9)
    a = knor.fit(_dev(X, "f32"), 64, C0=_dev(C0, "f64"), max_iters=15)
    b = knor.fit(_dev(X, "f32"), 64, C0=_dev(C0, "f64"), max_iters=15, autotune=True)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


@pytest.mark.parametrize("graph", [False, True])
def test_fit_batched_equals_single_fits(graph):
    """A batch mixing dtypes, shapes, given and Forgy starts: every problem's
    result equals knor_fit on it alone, and the oracle's (worker streams, or
    one graph holding every problem's iterations)."""
    knor = _knor()
    specs = [(9000, 8, 12, "f32", True), (20000, 32, 100, "f32", True),
             (5000, 3, 5, "f64", True), (7000, 64, 40, "bf16", True),
             (15000, 16, 30, "f32", False), (3000, 33, 17, "f32", True),
             (12000, 64, 256, "f32", True), (400, 5, 400, "f32", True),
             (6000, 128, 20, "bf16", False)]
    probs, data = [], []
    for i, (n, d, k, dt, given) in enumerate(specs):
        X, C0 = _data(n, d, k, dt, seed=100 + i)
        data.append((X, C0, dt))
        probs.append(dict(X=_dev(X, dt), k=k, C0=_dev(C0, "f64") if given else None,
                          max_iters=20))
    _print_case(test="batched", count=len(probs), graph=graph)
    out = knor.fit_batched(probs, seed=77, graph=graph)
    for i, ((X, C0, dt), p, (C, lab, st)) in enumerate(zip(data, probs, out)):
        single = knor.fit(p["X"], p["k"], C0=p["C0"], init="given" if p["C0"] is not None else "forgy",
                          seed=77 + i, max_iters=20)
        assert (C == single[0]).all() and (lab == single[1]).all(), i
        assert st["iters"] == single[2]["iters"], i
        if p["C0"] is not None:
            ref = oracle.mti_fit(workloads.to_f64(X, dt), C0, 20)
            assert (lab.cpu().numpy() == ref.labels).all(), i
            assert (C.cpu().numpy() == ref.C).all(), i


@pytest.mark.parametrize("graph", [False, True])
def test_fit_batched_workload_sample(graph):
    """Eight instances of the batched-restart workload (n scaled by 1/20),
    each against the FP64 oracle."""
    knor = _knor()
    ws = workloads.batched(8, n_scale=0.05)
    probs = [dict(X=_dev(w.X, "f32"), k=w.k, C0=_dev(w.C0, "f64"),
                  max_iters=w.max_iters) for w in ws]
    out = knor.fit_batched(probs, graph=graph)
    for w, (C, lab, st) in zip(ws, out):
        _print_case(test="batched-workload", n=w.n, d=w.d, k=w.k)
        ref = oracle.mti_fit(w.x64(), w.C0, w.max_iters)
        assert st["iters"] == ref.iters
        assert (lab.cpu().numpy() == ref.labels).all()
        assert (C.cpu().numpy() == ref.C).all()


def test_fit_batched_graph_repeated():
    """The graph form three times in a row, with eager fits between the calls:
    every call's results equal the worker-stream form's."""
    knor = _knor()
    ws = workloads.batched(6, n_scale=0.03)
    probs = [dict(X=_dev(w.X, "f32"), k=w.k, C0=_dev(w.C0, "f64"),
                  max_iters=w.max_iters) for w in ws]
    _print_case(test="batched-graph-repeated")
    ref = knor.fit_batched(probs)
    for rep in range(3):
        out = knor.fit_batched(probs, graph=True)
        for i, ((C, lab, st), (Cr, labr, str_)) in enumerate(zip(out, ref)):
            assert (C == Cr).all() and (lab == labr).all(), (rep, i)
            assert st["iters"] == str_["iters"], (rep, i)
        knor.fit(probs[rep]["X"], ws[rep].k, C0=probs[rep]["C0"], max_iters=5)


# ---------------------------------------------------------------------------
# learned candidate proposal
# ---------------------------------------------------------------------------

def _mlp_case(d, h, k, B, seed):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    th = mlp.init_params(d, h, k, seed) + rng.normal(size=mlp.param_count(d, h, k)) * 0.02
    th = th.astype(np.float32).astype(np.float64)
    Xs = rng.normal(size=(B, d)).astype(np.float32).astype(np.float64)
    y = rng.integers(0, k, size=B).astype(np.int32)
    return th, Xs, y


def test_mlp_init_matches_reference():
    from oracle import mlp
    knor = _knor()
    for (d, h, k, seed) in [(8, 32, 64, 5), (32, 256, 4096, 1)]:
        th = knor.mlp_init(d, h, k, seed).cpu().numpy()
        assert (th == mlp.init_params(d, h, k, seed).astype(np.float32)).all()


@pytest.mark.parametrize("d,h,k,B", [(8, 32, 64, 96), (32, 256, 4096, 512), (5, 64, 100, 130)])
def test_mlp_gradient_matches_reference(d, h, k, B):
    """Loss and gradient against the FP64 reference on the same BF16-rounded
    operands.  The GPU sums in FP32 (relative error ~K 2^-24, K <= 4096) and
    a hidden activation within that error of a BF16 rounding boundary can
    round one BF16 ulp (2^-8) the other way; both effects stay far below the
    normwise bound 2e-3 used here, while a wrong index, transpose or term
    gives errors of order one."""
    import torch
    from oracle import mlp
    knor = _knor()
    th, Xs, y = _mlp_case(d, h, k, B, seed=d + h + k)
    loss_o, g_o = mlp.loss_and_grad(th, Xs, y, d, h, k, use_bf16=True)
    P = th.size
    thd = torch.from_numpy(th.astype(np.float32)).cuda()
    grad = torch.zeros(P, dtype=torch.float32, device="cuda")
    m = torch.zeros(P, dtype=torch.float32, device="cuda")
    v = torch.zeros(P, dtype=torch.float32, device="cuda")
    loss = knor.mlp_train_step(thd, m, v, 1, d, h, k,
                               torch.from_numpy(Xs.astype(np.float32)).cuda(),
                               torch.from_numpy(y).cuda(), lr=0.0, grad=grad)
    assert abs(loss - loss_o) <= 1e-4 * abs(loss_o)
    g = grad.cpu().numpy().astype(np.float64)
    G, Go = mlp.unflatten(g, d, h, k), mlp.unflatten(g_o, d, h, k)
    for name in Go:
        err = np.linalg.norm(G[name] - Go[name]) / max(np.linalg.norm(Go[name]), 1e-30)
        assert err <= 2e-3, (name, err)
    # one Adam step, against FP64 Adam applied to the GPU's own gradient
    loss2 = knor.mlp_train_step(thd, m, v, 1, d, h, k,
                                torch.from_numpy(Xs.astype(np.float32)).cuda(),
                                torch.from_numpy(y).cuda(), lr=1e-3, grad=grad)
    assert loss2 == loss
    g = grad.cpu().numpy().astype(np.float64)
    want, m_o, v_o = mlp.adam_step(th, np.zeros(P), np.zeros(P), g, 1)
    assert np.allclose(thd.cpu().numpy(), want, rtol=2e-6, atol=1e-7)
    assert np.allclose(m.cpu().numpy(), m_o, rtol=1e-6, atol=1e-30)
    assert np.allclose(v.cpu().numpy(), v_o, rtol=1e-5, atol=1e-30)


@pytest.mark.parametrize("d,h,k,m", [(8, 32, 64, 300), (32, 256, 4096, 700), (16, 64, 100, 257),
                                     (40, 128, 1000, 513), (5, 256, 20, 64)])
def test_mlp_propose_matches_reference(d, h, k, m):
    """Candidates are the 16 largest logits (each rounded towards zero to its
    leading mantissa bits, ties by class), in decreasing order.  Against the
    FP64 reference on the same BF16 operands: every class whose reference
    logit clears the 17th largest by more than the tolerance is proposed,
    and every proposed class is within the tolerance of the 16th largest.
    The tolerance covers FP32 summation, an occasional hidden activation
    rounding one BF16 ulp the other way, and the key rounding."""
    import torch
    from oracle import mlp
    knor = _knor()
    _print_case(test="mlp-propose", d=d, h=h, k=k, m=m)
    th, Xs, _ = _mlp_case(d, h, k, m, seed=7 * d + k)
    _, _, z = mlp.forward(th, Xs, d, h, k, use_bf16=True)
    cand = knor.mlp_propose(torch.from_numpy(th.astype(np.float32)).cuda(), d, h, k,
                            torch.from_numpy(Xs.astype(np.float32)).cuda()).cpu().numpy()
    assert cand.shape == (m, 16)
    nreal = min(16, k)
    assert (cand[:, nreal:] == -1).all()
    c = cand[:, :nreal]
    assert ((c >= 0) & (c < k)).all()
    assert all(len(set(row)) == nreal for row in c)
    zs = -np.sort(-z, axis=1)
    z16 = zs[:, nreal - 1]
    z17 = zs[:, nreal] if k > nreal else np.full(m, -np.inf)
    tol = 4e-3 * (np.abs(z16) + 1.0)
    zc = np.take_along_axis(z, c, axis=1)
    assert (zc >= (z16 - tol)[:, None]).all()
    must = z > (z17 + tol)[:, None]
    for r in range(m):
        assert set(np.nonzero(must[r])[0]) <= set(c[r].tolist()), r
    # decreasing order (up to the tolerance)
    assert (np.diff(zc, axis=1) <= tol[:, None]).all()
    # the check is not vacuous: most of the top 16 clear the tolerance
    assert must.sum() >= 0.5 * nreal * m


@pytest.mark.parametrize("k", [128, 100])
def test_learned_fit_exact_and_certifies(k):
    """The learned proposal never changes a label: identical label history and
    centroids to the oracle; and it does decide some survivors."""
    w = workloads.config(5, n=60000, k=k)
    _print_case(test="learned-fit", k=k)
    knor = _knor()
    ref = oracle.mti_fit(w.x64(), w.C0, 20, history=True)
    C, lab, st = knor.fit(_dev(w.X, "f32"), k, C0=_dev(w.C0, "f64"), max_iters=20,
                          history=True, counters=True, learned=True, train_iters=3,
                          train_batches=4)
    assert st["iters"] == ref.iters
    hist = st["label_history"].cpu().numpy()
    for t in range(ref.iters):
        assert (hist[t] == ref.label_hist[t]).all(), t
    assert (C.cpu().numpy() == ref.C).all()
    if ref.iters > 4:
        assert st["mlp_queries"] > 0
        assert st["certified"] > 0
    # a point's candidates are computed once: the network sees each point at
    # most once per fit, and a later iteration's new rows are only survivors
    # that never survived before
    ctr = st["counters"]
    assert st["mlp_forward_rows"] == int(ctr[:, 8].sum()) <= w.n
    assert (ctr[:, 8] <= ctr[:, 6]).all()
    assert st["mlp_queries"] == int(ctr[:, 6].sum())
    print("learned-fit k", k, "queries", st["mlp_queries"], "forward rows",
          st["mlp_forward_rows"], "certified", st["certified"], flush=True)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_largest_k():
    """k = 16384 (the limit): assignment and a short fit against the oracle."""
    knor = _knor()
    rng = np.random.default_rng(11)
    X = rng.normal(size=(40000, 8)).astype(np.float32)
    C0 = X[:16384].astype(np.float64)
    lab_o, D_o = oracle.assign(X.astype(np.float64), C0)
    lab, dd = knor.assign(_dev(X, "f32"), _dev(C0, "f64"), dist2=True)
    assert (lab.cpu().numpy() == lab_o).all() and (dd.cpu().numpy() == D_o).all()
    _fit_compare(X, "f32", C0, 16384, 3, True, oracle_fit=oracle.mti_fit)


def test_empty_inputs():
    import torch
    knor = _knor()
    for dt in ("f32", "f64", "bf16"):
        X = _dev(workloads.cast(np.zeros((0, 5)), dt), dt)
        C = torch.ones((3, 5), dtype=torch.float64, device="cuda")
        lab = knor.assign(X, C)
        assert lab.shape == (0,)
        Cn, cnt = knor.update(X, torch.zeros((0,), dtype=torch.int32, device="cuda"), C)
        assert (Cn == C).all() and (cnt == 0).all()


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_degenerate_data(dtype):
    """All points identical (every distance ties), all-zero points, and k=1:
    labels, centroids and the stopping iteration match the oracle."""
    rng = np.random.default_rng(12)
    same = workloads.cast(np.tile(rng.normal(size=(1, 6)), (3000, 1)), dtype)
    C0 = np.tile(workloads.to_f64(same[:1], dtype), (5, 1))
    C0[2:] += rng.normal(size=(3, 6))
    _fit_compare(same, dtype, C0, 5, 10, True, oracle_fit=oracle.mti_fit)
    zero = workloads.cast(np.zeros((2000, 9)), dtype)
    _fit_compare(zero, dtype, rng.normal(size=(4, 9)), 4, 10, True, oracle_fit=oracle.mti_fit)
    X = workloads.cast(rng.normal(size=(5000, 40)) * 3, dtype)
    _fit_compare(X, dtype, workloads.to_f64(X[:1], dtype), 1, 5, True, oracle_fit=oracle.mti_fit)
