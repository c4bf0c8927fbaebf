"""A host model of the exact update's digit arithmetic, checked against exact
integers: an FP32 (or BF16) value as one add to a 16-bit-weighted digit
(m 2^(sh mod 16) on digit sh div 16, in units of 2^-149), and the split form
that puts the add in two pieces below 2^32 on digits idx and idx + 2 (the
form taken when an iteration may move 2^23 points or more).  Digits are
64-bit two's-complement registers; the model wraps every add to 64 bits and
asserts that the true signed value never leaves that range, then
normalises the digits (the finalize's model) and compares the result with
the exact sum of the values.  It exercises the split path at move counts no
GPU test reaches in full and at every exponent, subnormals included.
"""
import random
import struct
from fractions import Fraction

import pytest

from tests.test_exact_quotient_model import KXD, normalise

UNIT = Fraction(1, 2 ** 149)
MASK64 = (1 << 64) - 1


def fixed_of(u):
    """The kernel's decomposition of the FP32 bit pattern u: (digit index,
    signed amount) with value = amount 2^(16 idx) units of 2^-149."""
    ef = (u >> 23) & 255
    m = (u & 0x7FFFFF) | (0x800000 if ef else 0)
    sh = ef - 1 if ef else 0
    v = m << (sh & 15)
    return sh >> 4, (-v if u >> 31 else v)


def exact_units(u):
    """The value of bit pattern u in units of 2^-149 (an integer)."""
    f = struct.unpack("<f", struct.pack("<I", u))[0]
    q = Fraction(f) / UNIT
    assert q.denominator == 1
    return q.numerator


class Digits:
    def __init__(self):
        self.reg = [0] * KXD          # 64-bit registers (two's complement)
        self.true = [0] * KXD         # the signed values they should hold

    def add(self, idx, w):
        assert 0 <= idx < KXD
        self.true[idx] += w
        assert -(1 << 63) <= self.true[idx] < (1 << 63), "digit overflow"
        self.reg[idx] = (self.reg[idx] + w) & MASK64

    def add_split(self, idx, w):
        if w == 0:
            return
        neg = w < 0
        m = -w if neg else w
        for t, pc in enumerate((m & 0xFFFFFFFF, m >> 32)):
            if pc and idx + 2 * t < KXD:
                self.add(idx + 2 * t, -pc if neg else pc)

    def value(self):
        signed = [r - (1 << 64) if r >> 63 else r for r in self.reg]
        assert signed == self.true
        dig, top = normalise(signed)
        v = top << (32 * len(dig))
        for s, x in enumerate(dig):
            v += x << (32 * s)
        return v


def _random_bits(rng, n, subnormal_frac=0.1):
    out = []
    for _ in range(n):
        sign = rng.getrandbits(1) << 31
        if rng.random() < subnormal_frac:
            out.append(sign | rng.getrandbits(23))
        else:
            out.append(sign | (rng.randint(1, 254) << 23) | rng.getrandbits(23))
    return out


@pytest.mark.parametrize("split", [False, True])
def test_digits_sum_every_exponent(split):
    rng = random.Random(5 + split)
    vals = _random_bits(rng, 40000)
    dg = Digits()
    for u in vals:
        idx, v = fixed_of(u)
        (dg.add_split if split else dg.add)(idx, v)
    assert dg.value() == sum(exact_units(u) for u in vals)


def test_split_moves_in_and_out():
    """Points enter one cluster and leave it again (the delta update's -x for
    the old cluster): the digits equal the exact sum of the members left."""
    rng = random.Random(11)
    vals = _random_bits(rng, 30000)
    dg = Digits()
    for u in vals:
        dg.add_split(*fixed_of(u))
    gone = rng.sample(range(len(vals)), 12000)
    for i in gone:
        idx, v = fixed_of(vals[i])
        dg.add_split(idx, -v)
    keep = set(range(len(vals))) - set(gone)
    assert dg.value() == sum(exact_units(vals[i]) for i in keep)


def test_extreme_values():
    """The largest finite values, the smallest subnormal, and cancellation
    between them."""
    big = [0x7F7FFFFF, 0xFF7FFFFF, 0x7F7FFFFF]
    tiny = [0x00000001, 0x80000001, 0x00000001]
    for split in (False, True):
        dg = Digits()
        for u in big + tiny:
            idx, v = fixed_of(u)
            (dg.add_split if split else dg.add)(idx, v)
        assert dg.value() == sum(exact_units(u) for u in big + tiny)


def test_digit_headroom():
    """The bounds the two forms rely on: one add is below 2^39, so fewer than
    2^23 adds keep a digit below 2^62; a split piece is below 2^32, so any
    n < 2^31 points keep it below 2^63."""
    worst = 0
    for u in (0x7F7FFFFF, 0x7F7FFFF0, 0x0F7FFFFF, 0x00FFFFFF, 0x007FFFFF):
        idx, v = fixed_of(u)
        worst = max(worst, abs(v))
        m = abs(v)
        assert max(m & 0xFFFFFFFF, m >> 32) < 2 ** 32
    assert worst < 2 ** 39
    assert (2 ** 23 - 1) * worst < 2 ** 62
    assert (2 ** 31 - 1) * (2 ** 32 - 1) < 2 ** 63
    # many split adds of the largest pieces to one digit stay exact
    dg = Digits()
    idx, v = fixed_of(0x7F7FFFFF)
    for _ in range(5000):
        dg.add_split(idx, v)
    assert dg.value() == 5000 * exact_units(0x7F7FFFFF)
