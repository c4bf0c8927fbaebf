"""A host model of the exact update's finalize arithmetic, checked against
exact rationals: carry-save digits of 16 bits normalised and paired into
32-bit digits, the long division whose quotient digits come from an FP64
reciprocal estimate fixed by at most one from the remainder, and rounding
to nearest with ties to even.  It pins the claims the kernel relies on (the
estimate is off by at most one, three guard digits and a sticky bit give
the correctly rounded mean) at sizes the GPU tests do not reach: counts up
to 2^31 - 1, sums near 2^308 units, negative sums and exact ties.
"""
import math
import struct
from fractions import Fraction

import numpy as np

KXD, KQ, G = 20, 10, 3
UNIT = Fraction(1, 2 ** 149)


def normalise(slots):
    """Carry-save digits (signed ints, weight 2^16s) -> 9 x 32-bit digits
    and a signed top of weight 2^288, as the kernel pairs them."""
    carry = 0
    h = []
    for s in range(KXD - 1):
        v = slots[s] + carry
        h.append(v & 0xFFFF)
        carry = v >> 16                      # floor, like the arithmetic shift
    t16 = slots[KXD - 1] + carry
    dig = [h[2 * t] | (h[2 * t + 1] << 16) for t in range(KQ - 1)]
    top = t16 * 65536 + h[KXD - 2]
    return dig, top


def quotient(dig, top, cnt):
    neg = top < 0
    W = KQ + G
    a = [0] * G
    borrow = 1 if neg else 0
    for s in range(KQ - 1):
        x = (~dig[s] & 0xFFFFFFFF) if neg else dig[s]
        v = x + borrow
        a.append(v & 0xFFFFFFFF)
        borrow = v >> 32
    tmag = ((~top) + borrow) if neg else top
    a.append(tmag & 0xFFFFFFFF)
    rn = 1.0 / float(cnt)
    rem = 0
    q = [0] * W
    for s in range(W - 1, -1, -1):
        cur = (rem << 32) | a[s]
        qd = int(float(cur) * rn)            # truncation, as the kernel's cast
        r = cur - qd * cnt
        assert -cnt <= r < 2 * cnt, "estimate off by more than one"
        if r < 0:
            qd, r = qd - 1, r + cnt
        elif r >= cnt:
            qd, r = qd + 1, r - cnt
        q[s], rem = qd, r
    t = W - 1
    while t > 0 and q[t] == 0:
        t -= 1
    if q[t] == 0:
        return 0.0
    lz = 32 - q[t].bit_length()
    hi64 = (q[t] << 32) | q[t - 1]
    lo32 = q[t - 2]
    w = ((hi64 << lz) | (lo32 >> (32 - lz))) & (2 ** 64 - 1) if lz else hi64
    mant = w >> 11
    rbit = (w >> 10) & 1
    sticky = (w & 0x3FF) != 0 or rem != 0 or (((lo32 << lz) & 0xFFFFFFFF) if lz else lo32) != 0
    sticky = sticky or any(q[s] for s in range(t - 2))
    if rbit and (sticky or (mant & 1)):
        mant += 1
    b = 32 * t + 31 - lz
    r = math.ldexp(float(mant), b - 52 - 149 - 32 * G)
    return -r if neg else r


def _exact(total_units, cnt):
    return float(Fraction(total_units, 1) * UNIT / cnt)


def _carry_save(total_units, rng):
    """A carry-save representation of total_units: its base-2^16 digits
    (signed top), then random transfers r 2^16 from digit s to digit s + 1
    that keep the value (digits end up negative or above 16 bits)."""
    slots = [(total_units >> (16 * s)) & 0xFFFF for s in range(KXD - 1)]
    slots.append(total_units >> (16 * (KXD - 1)))
    for s in range(KXD - 1):
        r = int(rng.integers(-2 ** 30, 2 ** 30))
        slots[s] -= r << 16
        slots[s + 1] += r
    assert sum(v << (16 * s) for s, v in enumerate(slots)) == total_units
    return slots


def _bits(x):
    return struct.unpack("<q", struct.pack("<d", x))[0]


def test_quotient_matches_rationals():
    rng = np.random.default_rng(21)
    for _ in range(3000):
        cnt = int(rng.choice([1, 2, 3, 7, 1000, 65537, 2 ** 24 + 1, 2 ** 31 - 1,
                              int(rng.integers(1, 2 ** 31))]))
        bits = int(rng.integers(1, 300))
        total = int(rng.integers(1, 2 ** 62)) << max(0, bits - 62)
        total = total % (2 ** 307)
        if total == 0:
            continue
        if rng.random() < 0.5:
            total = -total
        dig, top = normalise(_carry_save(total, rng))
        got = quotient(dig, top, cnt)
        assert _bits(got) == _bits(_exact(total, cnt)), (total, cnt)


def test_quotient_ties_to_even():
    # (2^53 + 1) / 2 and (2^53 + 3) / 2 units scaled to the double grid:
    # halfway cases between two doubles
    rng = np.random.default_rng(3)
    for odd in (1, 3, 5, 7):
        for scale in (0, 40, 200):
            total = ((2 ** 53 + odd) << scale)
            for sign in (1, -1):
                dig, top = normalise(_carry_save(sign * total, rng))
                got = quotient(dig, top, 2)
                assert got == _exact(sign * total, 2)


def test_zero_and_extremes():
    rng = np.random.default_rng(4)
    dig, top = normalise(_carry_save(0, rng))
    assert quotient(dig, top, 5) == 0.0
    big = 2 ** 307 - 1                        # near the largest sum
    dig, top = normalise(_carry_save(big, rng))
    assert quotient(dig, top, 2 ** 31 - 1) == _exact(big, 2 ** 31 - 1)
    dig, top = normalise(_carry_save(1, rng))  # the smallest nonzero sum
    assert quotient(dig, top, 2 ** 31 - 1) == _exact(1, 2 ** 31 - 1)
