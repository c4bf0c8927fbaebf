"""The exactness bound the exact update's full pass relies on, checked on the
host against exact rational sums.

Every FP32 (or BF16) value is m 2^(sh - 149) with m < 2^24.  With L the
lowest set bit and M = max(sh) + 24 over a set of values (in units of
2^-149), every value is a multiple of 2^L and every partial sum is below
count 2^M; when M - L + ceil(log2 count) <= 53, a left-to-right FP64 sum of
the values is exact.  Here: the claim is checked on random sets, with the
bound computed from the FP32 bit patterns as the kernel does, and the cases
where it fails are shown to be the ones that can round.
"""
import math
from fractions import Fraction

import numpy as np


def _bound_parts(v32):
    u = v32.view(np.uint32).astype(np.int64)
    ef = (u >> 23) & 255
    m = (u & 0x7FFFFF) | np.where(ef > 0, 0x800000, 0)
    sh = np.where(ef > 0, ef - 1, 0)
    nz = m != 0
    ctz = np.array([(int(x) & -int(x)).bit_length() - 1 if x else 0 for x in m])
    L = int((sh + ctz)[nz].min()) if nz.any() else 1 << 30
    M = int((sh + 24)[nz].max()) if nz.any() else -1
    return L, M, int(nz.sum())


def _fp64_sum(v32):
    s = 0.0
    for x in v32.astype(np.float64):
        s += float(x)
    return s


def test_fp64_sum_exact_when_bound_holds():
    rng = np.random.default_rng(12)
    held = failed_bound = 0
    for trial in range(400):
        cnt = int(rng.integers(1, 257))
        spread = float(rng.uniform(0, 30))
        mag = 2.0 ** rng.uniform(-spread, 0, size=cnt) * 10.0 ** rng.integers(-30, 30)
        v = (rng.normal(size=cnt) * mag).astype(np.float32)
        if trial % 3 == 0:                           # BF16 values
            v = (v.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
        L, M, c = _bound_parts(v)
        if c == 0:
            continue
        lg = max(0, math.ceil(math.log2(c)))
        exact = sum((Fraction(float(x)) for x in v), Fraction(0))
        if M - L + lg <= 53:
            held += 1
            assert Fraction(_fp64_sum(v)) == exact, (trial, L, M, c)
        else:
            failed_bound += 1
    assert held > 100 and failed_bound > 10        # both sides are exercised


def test_bound_is_needed():
    # a set outside the bound whose FP64 sum does round: 1 + 2^-60 (FP32
    # values 1 and 2^-60; the exact sum needs 61 bits)
    v = np.array([1.0, 2.0 ** -60], np.float32)
    L, M, c = _bound_parts(v)
    assert M - L + 1 > 53
    assert Fraction(_fp64_sum(v)) != sum(Fraction(float(x)) for x in v)
