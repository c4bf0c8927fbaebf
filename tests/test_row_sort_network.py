"""CPU model of the neighbour-row sort network (the bitonic network in its
direction-free form, laid out as one wave of 64 lanes with KPL keys each):
the same stages in the same order as the kernel, checked against np.sort.

A merge of size s first compares i with i xor (s - 1), then runs
half-cleaners with strides s/4 ... 1, the smaller key going to the lower
index.  Merges of up to KPL keys stay within a lane; larger ones take the
partner key from lane l xor (s/KPL - 1) (at register KPL - 1 - r) or from
lane l xor (stride/KPL) (same register)."""
import numpy as np
import pytest


def _wave_sort(v):
    """v: (64, KPL) uint32, lane-major (key index l*KPL + r)."""
    v = v.copy()
    kpl = v.shape[1]
    lanes = np.arange(64)

    def cmpx(r, q):
        lo, hi = np.minimum(v[:, r], v[:, q]), np.maximum(v[:, r], v[:, q])
        v[:, r], v[:, q] = lo, hi

    size = 2
    while size <= kpl:
        for r in range(kpl):
            if r & (size >> 1) == 0:
                cmpx(r, r ^ (size - 1))
        st = size >> 2
        while st > 0:
            for r in range(kpl):
                if r & st == 0:
                    cmpx(r, r + st)
            st >>= 1
        size <<= 1
    lsz = 2
    while lsz <= 64:
        low = (lanes & (lsz >> 1)) == 0
        partner = v[lanes ^ (lsz - 1)][:, ::-1]        # register KPL - 1 - r of the partner lane
        v = np.where(low[:, None], np.minimum(v, partner), np.maximum(v, partner))
        ls = lsz >> 2
        while ls > 0:
            lo = (lanes & ls) == 0
            p = v[lanes ^ ls]
            v = np.where(lo[:, None], np.minimum(v, p), np.maximum(v, p))
            ls >>= 1
        st = kpl >> 1
        while st > 0:
            for r in range(kpl):
                if r & st == 0:
                    cmpx(r, r + st)
            st >>= 1
        lsz <<= 1
    return v


@pytest.mark.parametrize("kpl", [4, 8, 16, 32, 64])
def test_network_sorts(kpl):
    rng = np.random.default_rng(kpl)
    kp2 = 64 * kpl
    for k in (kp2, kp2 - 1, kp2 // 2 + 1):
        ib = int(np.ceil(np.log2(k)))
        j = np.arange(kp2, dtype=np.uint32)
        # keys: a non-negative float's bits with the low ib bits replaced by j
        # (several equal distances: ties broken by the index), +inf padding
        val = rng.integers(0, 0x7F7FF000, size=kp2, dtype=np.uint32) & np.uint32(0x7F7F0000)
        keys = (val & ~np.uint32((1 << ib) - 1)) | j
        keys[k:] = np.uint32(0x7F800000)
        out = _wave_sort(keys.reshape(64, kpl)).reshape(-1)
        assert (out == np.sort(keys)).all()
        # integer order is float order for these keys
        assert (np.argsort(out.view(np.float32), kind="stable") == np.arange(kp2)).all()
