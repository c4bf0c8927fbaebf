"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each compares it with a
hand-derived value (tests/golden), a brute-force optimum, a closed form, an
exact invariance, a third-party library, or a bound.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# hand-derived fixtures
# --------------------------------------------------------------------------

def test_golden_2d_integer_assign_update_fit(orc):
    g = _gold("lloyd_2d_integer.json")
    X = np.array(g["X"], float)
    C0 = np.array(g["C0"], float)
    for p, row in enumerate(g["iter0_dist2_to_each"]):
        for j, v in enumerate(row):
            assert orc.dist2(X[p], C0[j]) == v
    lab, D = orc.assign(X, C0)
    assert lab.tolist() == g["iter0_labels"]
    assert D.tolist() == g["iter0_best_dist2"]
    C1, cnt = orc.update(X, lab, C0)
    assert C1.tolist() == g["iter1_centroids"]
    assert cnt.tolist() == [3, 2]
    for fn in (orc.fit, orc.mti_fit):
        r = fn(X, C0, max_iters=10)
        assert r.labels.tolist() == g["final_labels"]
        assert r.C.tolist() == g["final_centroids"]
        assert r.iters == g["iters"] and r.converged
        assert r.changed.tolist() == g["changed"]
        assert r.objective.tolist() == g["objective"]


def test_objective_golden_2d_integer(orc):
    """The objective J = sum_p D(x_p, c_label(p)) on the hand-derived fixture:
    16 at (C0, iteration-0 labels), 9 at the converged state, and 106 when
    every point is charged to centroid 1 (the second column of the
    fixture's iteration-0 distance table)."""
    g = _gold("lloyd_2d_integer.json")
    X = np.array(g["X"], float)
    C0 = np.array(g["C0"], float)
    assert orc.objective(X, C0, np.array(g["iter0_labels"])) == g["objective"][0] == 16
    Cf = np.array(g["final_centroids"], float)
    assert orc.objective(X, Cf, np.array(g["final_labels"])) == g["objective"][-1] == 9
    col1 = sum(row[1] for row in g["iter0_dist2_to_each"])
    assert col1 == 106
    assert orc.objective(X, C0, np.ones(5, np.int32)) == col1


def test_objective_summation_order_golden(orc):
    """The objective sums its n terms in the fixed canonical order: the
    193-term fixture (2^53 at member 0, 1 at members 128 and 192) gives
    2^53 + 2, where a left-to-right sum would give 2^53.  The terms are
    realised as squared distances of integer points to the origin."""
    g = _gold("canonical_order_sum.json")
    m = g["m"]
    X = np.zeros((m, 2))
    X[0] = (2.0 ** 26, 2.0 ** 26)                 # D = 2^52 + 2^52 = 2^53
    X[128] = (1.0, 0.0)
    X[192] = (0.0, 1.0)
    C = np.array([[0.0, 0.0], [7.0, 7.0]])
    lab = np.zeros(m, np.int32)
    assert orc.objective(X, C, lab) == g["canonical_sum"] != g["sequential_sum"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_objective_bruteforce_integer(orc, seed):
    """Integer points, centroids and arbitrary labels: every FP64 step is
    exact, so the objective equals the exact integer sum, computed here in
    Python integers term by term."""
    rng = np.random.default_rng(100 + seed)
    n, d, k = 301, 3, 5
    X = rng.integers(-40, 41, size=(n, d))
    C = rng.integers(-40, 41, size=(k, d))
    lab = rng.integers(0, k, size=n).astype(np.int32)
    exact = 0
    for p in range(n):
        for i in range(d):
            t = int(X[p, i]) - int(C[lab[p], i])
            exact += t * t
    assert orc.objective(X.astype(float), C.astype(float), lab) == float(exact)


def test_golden_1d_threshold(orc):
    g = _gold("lloyd_1d_threshold.json")
    X = np.array(g["X"], float)
    C0 = np.array(g["C0"], float)
    lab, _ = orc.assign(X, C0)
    assert lab.tolist() == g["iter0_labels"]
    r = orc.fit(X, C0, max_iters=10)
    assert r.labels.tolist() == g["final_labels"]
    assert r.C.tolist() == g["final_centroids"]
    assert r.iters == g["iters"]
    assert r.changed.tolist() == g["changed"]


def test_golden_canonical_order(orc):
    g = _gold("canonical_order_sum.json")
    m = g["m"]
    v = np.zeros(m)
    for i, val in g["nonzero"].items():
        v[int(i)] = val
    X = v[:, None]
    C, cnt = orc.update(X, np.zeros(m, np.int32), np.zeros((1, 1)))
    assert cnt[0] == m
    assert C[0, 0] == g["canonical_sum"] / m
    assert orc.canonical_sum(v) == g["canonical_sum"]
    # the plain left-to-right sum differs, so the order is really exercised
    s = 0.0
    for x in v:
        s += x
    assert s == g["sequential_sum"] != g["canonical_sum"]


# --------------------------------------------------------------------------
# distance and tie-breaking on exact inputs
# --------------------------------------------------------------------------

def test_dist2_integer_exact(orc):
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = int(rng.integers(1, 40))
        x = rng.integers(-1000, 1000, d).astype(float)
        c = rng.integers(-1000, 1000, d).astype(float)
        exact = sum(int(a - b) ** 2 for a, b in zip(x, c))   # integer arithmetic
        assert orc.dist2(x, c) == float(exact)


def test_tie_lowest_index(orc):
    # x on the bisector of several equal-distance integer centroids
    X = np.array([[0.0, 0.0], [1.0, 1.0]])
    C = np.array([[3.0, 4.0], [5.0, 0.0], [-4.0, 3.0], [0.0, -5.0], [9.0, 9.0]])
    lab, D = orc.assign(X, C)
    assert lab[0] == 0 and D[0] == 25.0
    # x = (1,1): distances 13, 17, 29, 37, 128 -> index 0
    assert lab[1] == 0
    # reversed order: the lowest index among the equal ones wins
    lab2, _ = orc.assign(X[:1], C[[4, 3, 2, 1, 0]])
    assert lab2[0] == 1


# --------------------------------------------------------------------------
# brute force on tiny inputs
# --------------------------------------------------------------------------

def _labeling_cost(X, lab, k):
    cost = 0.0
    for j in range(k):
        M = X[lab == j]
        if len(M):
            mu = M.mean(axis=0)
            cost += float(((M - mu) ** 2).sum())
    return cost


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_fixed_point_and_optimum(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 8))
    k = int(rng.integers(2, min(3, n) + 1))
    d = int(rng.integers(1, 3))
    X = rng.integers(-6, 7, (n, d)).astype(float)
    X[: n // 2] += 20.0 * rng.integers(0, 2)
    best_cost, best_labs = math.inf, []
    for lab in itertools.product(range(k), repeat=n):
        lab = np.array(lab)
        if len(set(lab.tolist())) < k:
            continue
        c = _labeling_cost(X, lab, k)
        if c < best_cost - 1e-9:
            best_cost, best_labs = c, [lab]
        elif abs(c - best_cost) <= 1e-9:
            best_labs.append(lab)
    C0 = X[rng.choice(n, k, replace=False)]
    r = orc.fit(X, C0, max_iters=100)
    assert r.converged
    # a converged Lloyd state can never beat the global optimum
    assert r.objective[-1] >= best_cost - 1e-9
    # converged = fixed point: labels are the argmin for the returned centroids
    lab, _ = orc.assign(X, r.C)
    assert (lab == r.labels).all()
    # started at an optimal partition's means, Lloyd's stays at an optimum
    opt = best_labs[0]
    Copt = np.stack([X[opt == j].mean(axis=0) for j in range(k)])
    r2 = orc.fit(X, Copt, max_iters=100)
    assert abs(r2.objective[-1] - best_cost) <= 1e-9 * max(1.0, best_cost)


def test_k_equals_one_is_global_mean(orc):
    rng = np.random.default_rng(7)
    X = rng.normal(size=(1000, 5)) * 3 + 1
    r = orc.fit(X, X[:1], max_iters=5)
    assert r.iters == 2 and r.converged
    for i in range(5):
        ref = math.fsum(X[:, i]) / 1000
        assert abs(r.C[0, i] - ref) <= 4e-16 * max(1.0, abs(ref)) * 1000


def test_k_equals_n_zero_objective(orc):
    rng = np.random.default_rng(8)
    X = rng.normal(size=(40, 3))
    r = orc.fit(X, X.copy(), max_iters=5)
    assert (r.labels == np.arange(40)).all()
    assert r.objective[0] == 0.0
    assert (r.C == X).all()


def test_empty_cluster_keeps_previous(orc):
    X = np.array([[0.0], [1.0], [2.0]])
    C0 = np.array([[1.0], [100.0], [-50.0]])
    r = orc.fit(X, C0, max_iters=5)
    assert r.labels.tolist() == [0, 0, 0]
    assert r.C[1, 0] == 100.0 and r.C[2, 0] == -50.0
    assert r.C[0, 0] == 1.0


# --------------------------------------------------------------------------
# invariants on random inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [-3, 5, 20])
def test_power_of_two_scaling_exact(orc, p):
    w = workloads.config(1, n=1500, seed=4)
    X = w.x64()
    r1 = orc.fit(X, w.C0, max_iters=15)
    r2 = orc.fit(X * 2.0 ** p, w.C0 * 2.0 ** p, max_iters=15)
    assert (r1.labels == r2.labels).all()
    assert (r2.C == r1.C * 2.0 ** p).all()
    assert (r2.objective == r1.objective * 4.0 ** p).all()


@pytest.mark.parametrize("seed", range(4))
def test_objective_nonincreasing_and_means(orc, seed):
    w = workloads.config(2, n=3000, k=12, seed=seed)
    X = w.x64()
    r = orc.fit(X, w.C0, max_iters=60)
    J = r.objective
    assert (np.diff(J) <= 1e-12 * J[:-1]).all()
    # converged centroids are the means of their members (canonical order:
    # recomputing the update from the returned labels reproduces them bit
    # for bit), and agree with compensated-sum means to FP64 accuracy
    C2, cnt = orc.update(X, r.labels, r.C)
    assert (C2 == r.C).all()
    for j in range(12):
        M = X[r.labels == j]
        if len(M):
            ref = np.array([math.fsum(M[:, i]) / len(M) for i in range(X.shape[1])])
            assert np.all(np.abs(r.C[j] - ref) <= 1e-14 * np.maximum(1, np.abs(ref)))


def _bottom_up_pairs(leaves):
    # independent iterative form of the tree: combine adjacent pairs level by
    # level, carrying an odd last element upward unchanged
    cur = list(leaves)
    while len(cur) > 1:
        nxt = [cur[i] + cur[i + 1] for i in range(0, len(cur) - 1, 2)]
        if len(cur) % 2:
            nxt.append(cur[-1])
        cur = nxt
    return cur[0]


@pytest.mark.parametrize("m", [1, 2, 63, 64, 65, 127, 128, 129, 300, 1000, 4097])
def test_canonical_sum_bottom_up(orc, m):
    rng = np.random.default_rng(m)
    v = rng.normal(size=m) * np.exp(rng.uniform(-30, 30, size=m))
    leaves = []
    for L in range(0, m, 64):
        s = v[L]
        for x in v[L + 1: L + 64]:
            s = s + x
        leaves.append(s)
    assert orc.canonical_sum(v) == _bottom_up_pairs(leaves)


def test_sklearn_lloyd_agrees(orc):
    from sklearn.cluster import KMeans
    w = workloads.config(1, n=4000, seed=11)
    X = w.x64()
    r = orc.fit(X, w.C0, max_iters=50)
    km = KMeans(n_clusters=w.k, init=w.C0, n_init=1, algorithm="lloyd",
                max_iter=50, tol=0.0).fit(X)
    assert (km.labels_ == r.labels).all()
    assert np.allclose(km.cluster_centers_, r.C, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# MTI: identical labels to plain Lloyd's at every iteration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["cfg1", "cfg2", "uniform", "dups"])
def test_mti_equals_plain_every_iteration(orc, case):
    if case == "cfg1":
        w = workloads.config(1, n=3000, seed=2)
        X, C0, it = w.x64(), w.C0, 30
    elif case == "cfg2":
        w = workloads.config(2, n=5000, k=20, seed=3)
        X, C0, it = w.x64(), w.C0, 40
    elif case == "uniform":
        X = workloads.to_f64(workloads.uniform_cube(3000, 4, seed=5), "f32")
        C0 = X[:9].copy()
        it = 40
    else:
        rng = np.random.default_rng(9)
        base = rng.integers(-3, 4, (50, 2)).astype(float)
        X = base[rng.integers(0, 50, 2000)]
        C0 = X[:6].copy()
        it = 30
    a = orc.fit(X, C0, max_iters=it, history=True)
    b = orc.mti_fit(X, C0, max_iters=it, history=True)
    assert a.iters == b.iters
    assert (a.label_hist == b.label_hist).all()
    assert (a.C == b.C).all()
    assert b.bound_violations == 0
    if case in ("cfg1", "cfg2"):
        # pruning actually happens on clustered data
        frac = {"cfg1": 0.5, "cfg2": 0.8}[case]
        assert b.ndist[1:].sum() < frac * a.ndist[1:].sum()


def test_mti_prunes_more_on_clusters_than_uniform(orc):
    # the paper reports MTI pruning well on clustered data and poorly on
    # uniformly random data (Section "Experimental Evaluation")
    n = 20000
    w = workloads.config(2, n=n, seed=1)
    Xc = w.x64()
    Xu = workloads.to_f64(workloads.uniform_cube(n, 32, seed=1), "f32")
    rc = orc.mti_fit(Xc, w.C0, max_iters=15)
    ru = orc.mti_fit(Xu, Xu[:100].copy(), max_iters=15)
    fc = rc.ndist[1:].sum() / (n * 100 * (rc.iters - 1))
    fu = ru.ndist[1:].sum() / (n * 100 * (ru.iters - 1))
    assert fc < 0.2 and fu > 0.8
    assert rc.pruned1[1:].sum() > 0.3 * n * (rc.iters - 1)


def test_cc_bounds_bruteforce(orc):
    rng = np.random.default_rng(0)
    C = rng.integers(-5, 6, (7, 3)).astype(float)
    s = orc.cc_bounds(C)
    for i in range(7):
        m = min(math.sqrt(sum((C[i] - C[j]) ** 2)) for j in range(7) if j != i)
        assert s[i] == 0.5 * m


def test_thread_count_independent(orc):
    import subprocess, sys
    code = ("import sys; sys.path.insert(0, %r); import numpy as np, oracle, workloads;"
            "w = workloads.config(2, n=4000, k=16, seed=1);"
            "r = oracle.mti_fit(w.x64(), w.C0, 20);"
            "print(r.C.tobytes().hex()[:4000], r.labels.sum(), r.iters)") % os.path.dirname(GOLD)[:-len("/tests")]
    outs = []
    for th in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=th)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env))
    assert outs[0] == outs[1]
