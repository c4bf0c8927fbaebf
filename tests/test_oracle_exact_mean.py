"""Pins for the oracle's second update reading: the exactly rounded mean.

The reference values come from Python's exact rational arithmetic
(fractions.Fraction, whose conversion to float is correctly rounded, ties to
even, subnormals included) and from hand-derived ties; none re-types the
oracle's fixed-point accumulator or its long division.
"""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import workloads

TINY = 2.0 ** -1074          # smallest subnormal
ULP1 = 2.0 ** -52            # spacing of doubles in [1, 2)


def _exact(v):
    return float(sum((Fraction(x) for x in v), Fraction(0)) / len(v))


def _bits(x):
    return struct.unpack("<q", struct.pack("<d", x))[0]


def _same(a, b):
    # bit-identical, so that -0.0 and +0.0 are told apart
    return _bits(a) == _bits(b)


def _cases(seed):
    rng = np.random.default_rng(seed)
    yield rng.normal(size=rng.integers(1, 200))
    yield rng.normal(size=50) * 10.0 ** rng.integers(-300, 300, size=50)
    yield rng.integers(-8, 9, size=rng.integers(1, 40)) * TINY * rng.integers(1, 5)
    yield rng.normal(size=1000).astype(np.float32).astype(np.float64)
    yield np.concatenate([rng.normal(size=20), -rng.normal(size=20)])
    v = rng.normal(size=30) * 1e200
    yield np.concatenate([v, [rng.normal()], -v])         # cancellation
    yield np.full(rng.integers(1, 50), rng.normal())      # constant


@pytest.mark.parametrize("seed", range(40))
def test_exact_mean_is_correctly_rounded(orc, seed):
    for v in _cases(seed):
        got = orc.exact_mean(v)
        ref = _exact(v)
        assert _same(got, ref) or (got == 0.0 and ref == 0.0), (v, got, ref)


def test_exact_mean_ties_to_even(orc):
    # 1 + 2^-53 lies halfway between 1 (even) and 1 + 2^-52 (odd)
    assert orc.exact_mean([1.0, 1.0 + ULP1]) == 1.0
    # 1 + 1.5 * 2^-52 lies halfway between 1 + 2^-52 (odd) and 1 + 2^-51 (even)
    assert orc.exact_mean([1.0 + ULP1, 1.0 + 2 * ULP1]) == 1.0 + 2 * ULP1
    # the same two ties mirrored to negative values
    assert orc.exact_mean([-1.0, -1.0 - ULP1]) == -1.0
    assert orc.exact_mean([-1.0 - ULP1, -1.0 - 2 * ULP1]) == -1.0 - 2 * ULP1
    # off a tie: the nearer neighbour wins
    v = [1.0, 1.0 + ULP1, 1.0 + ULP1, 1.0 + ULP1]           # mean 1 + 0.75 ulp
    assert orc.exact_mean(v) == 1.0 + ULP1
    v = [1.0, 1.0, 1.0, 1.0 + ULP1]                          # mean 1 + 0.25 ulp
    assert orc.exact_mean(v) == 1.0


def test_exact_mean_subnormal_and_extreme(orc):
    assert orc.exact_mean([TINY, 0.0]) == 0.0                # 2^-1075: tie to 0
    assert orc.exact_mean([TINY, TINY, TINY, 0.0]) == TINY   # 0.75 tiny
    assert orc.exact_mean([3 * TINY, 0.0]) == 2 * TINY       # 1.5 tiny: tie to even
    assert orc.exact_mean([TINY, TINY, 0.0]) == TINY         # 2/3 tiny
    assert orc.exact_mean([TINY, 0.0, 0.0]) == 0.0           # 1/3 tiny
    big = np.finfo(np.float64).max
    assert orc.exact_mean([big, big]) == big                 # no overflow
    assert orc.exact_mean([big, -big, 3.0]) == 1.0
    assert orc.exact_mean([1e300, 1.0, -1e300]) == 1.0 / 3.0
    assert orc.exact_mean([2.0 ** 1023, 2.0 ** 1023, -TINY]) == 2.0 ** 1023 / 3 * 2
    assert orc.exact_mean([5.0]) == 5.0 and orc.exact_mean([-TINY]) == -TINY


def test_exact_mean_sign_symmetry_and_zero(orc):
    rng = np.random.default_rng(11)
    v = rng.normal(size=101)
    assert orc.exact_mean(-v) == -orc.exact_mean(v)
    assert orc.exact_mean(np.concatenate([v, -v])) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_exact_mean_order_independent(orc, seed):
    rng = np.random.default_rng(100 + seed)
    v = rng.normal(size=777) * 10.0 ** rng.integers(-20, 20, size=777)
    ref = orc.exact_mean(v)
    for _ in range(5):
        assert orc.exact_mean(rng.permutation(v)) == ref


def test_exact_mean_many_terms_carry(orc):
    # 100000 equal terms near the top of each 64-bit word: the sum carries
    # through several words of the accumulator; the mean is the term itself
    for x in (1.0 - 2.0 ** -53, 2.0 ** 511 * 1.999, 3 * TINY):
        assert orc.exact_mean(np.full(100000, x)) == x


def _update_ref(X, labels, C_prev):
    k, d = C_prev.shape
    C = C_prev.copy()
    cnt = np.bincount(labels, minlength=k)
    for j in range(k):
        rows = X[labels == j]
        if len(rows):
            C[j] = [_exact(rows[:, i]) for i in range(d)]
    return C, cnt


@pytest.mark.parametrize("seed", range(3))
def test_update_exact_against_rationals(orc, seed):
    rng = np.random.default_rng(seed)
    n, d, k = 300, 5, 9
    X = rng.normal(size=(n, d)) * 10.0 ** rng.integers(-5, 5, size=(n, 1))
    labels = rng.integers(0, k - 2, size=n).astype(np.int32)   # clusters k-2, k-1 empty
    C_prev = rng.normal(size=(k, d))
    C, cnt = orc.update_exact(X, labels, C_prev)
    Cr, cntr = _update_ref(X, labels, C_prev)
    assert (cnt == cntr).all()
    assert (C == Cr).all()
    assert (C[k - 2:] == C_prev[k - 2:]).all()


def test_update_exact_equals_canonical_when_sums_are_exact(orc):
    # small integers: every canonical partial sum is exact, so both readings
    # round the same exact quotient once
    rng = np.random.default_rng(5)
    X = rng.integers(-1000, 1000, size=(500, 4)).astype(np.float64)
    labels = rng.integers(0, 7, size=500).astype(np.int32)
    C_prev = np.zeros((7, 4))
    Ce, ce = orc.update_exact(X, labels, C_prev)
    Cc, cc = orc.update(X, labels, C_prev)
    assert (Ce == Cc).all() and (ce == cc).all()


def test_update_exact_rejects_bad_labels(orc):
    X = np.zeros((3, 2))
    with pytest.raises(ValueError):
        orc.update_exact(X, np.array([0, 2, 0], np.int32), np.zeros((2, 2)))


def test_fit_exact_mean_k1_is_rational_mean(orc):
    rng = np.random.default_rng(9)
    X = rng.normal(size=(400, 3)) * 1e3 + 7
    r = orc.fit_exact_mean(X, X[:1], max_iters=5)
    assert r.converged and r.iters == 2
    for i in range(3):
        assert r.C[0, i] == _exact(X[:, i])


@pytest.mark.parametrize("case", ["cfg", "uniform", "dups"])
def test_exact_mean_mti_equals_plain(orc, case):
    if case == "cfg":
        w = workloads.config(1, n=2000, seed=2)
        X, C0 = w.x64(), w.C0
    elif case == "uniform":
        rng = np.random.default_rng(3)
        X = rng.random((1500, 6))
        C0 = X[rng.choice(1500, 12, replace=False)]
    else:
        rng = np.random.default_rng(4)
        base = rng.integers(0, 4, size=(60, 3)).astype(np.float64)
        X = base[rng.integers(0, 60, size=900)]
        C0 = base[:8]
    a = orc.fit_exact_mean(X, C0, max_iters=30, history=True)
    b = orc.mti_fit(X, C0, max_iters=30, history=True, exact_mean=True)
    assert a.iters == b.iters and a.converged == b.converged
    assert (a.label_hist == b.label_hist).all()
    assert (a.C == b.C).all()
    assert b.bound_violations == 0
    # the converged centroids are the exact member means
    Cr, _ = _update_ref(X, a.labels, C0)
    if a.converged:
        assert (a.C == Cr).all()


def test_exact_mean_fit_objective_nonincreasing(orc):
    w = workloads.config(1, n=3000, seed=6)
    r = orc.fit_exact_mean(w.x64(), w.C0, max_iters=40)
    ob = r.objective
    assert all(ob[t + 1] <= ob[t] * (1 + 1e-12) for t in range(len(ob) - 1))
    assert math.isfinite(ob[-1])
