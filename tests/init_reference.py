"""Host re-implementations of the library's seeded initial-centroid rules
(include/knor.h, knor_init), written from their documented definitions for
the GPU tests to compare against.  The paper fixes no initialisation; these
are the library's own definitions, not part of the method."""
import math

import numpy as np

M64 = (1 << 64) - 1


def splitmix64_stream(seed, count):
    """The first `count` outputs of SplitMix64 seeded with `seed`."""
    out = []
    st = seed & M64
    for _ in range(count):
        st = (st + 0x9E3779B97F4A7C15) & M64
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def forgy_rows(n, k, seed):
    """Fisher-Yates over slots i = n-1 down to n-k, j = next() % (i + 1);
    centroid r is the row landing in slot n-1-r."""
    a = {}
    rows = []
    for r, z in enumerate(splitmix64_stream(seed, k)):
        i = n - 1 - r
        j = z % (i + 1)
        vi, vj = a.get(i, i), a.get(j, j)
        a[i], a[j] = vj, vi
        rows.append(vj)
    return rows


def shuffle_first_k_rows(n, k, seed):
    """Front-to-back Fisher-Yates: for i = 0..k-1, j = i + next() % (n - i),
    swap slots i and j; centroid i is the row in slot i."""
    a = {}
    rows = []
    for i, z in enumerate(splitmix64_stream(seed, k)):
        j = i + z % (n - i)
        vi, vj = a.get(i, i), a.get(j, j)
        a[i], a[j] = vj, vi
        rows.append(vj)
    return rows


def _dist2_rows(X64, c):
    """Squared distances of every row to c, summed in index order, one
    rounding per operation (NumPy does not contract to FMA)."""
    acc = np.zeros(X64.shape[0])
    for i in range(X64.shape[1]):
        t = X64[:, i] - c[i]
        acc = acc + t * t
    return acc


def kmeanspp_rows(X64, k, seed):
    """k-means++ with integer weights: w(p) = floor(D(p) 2^(B - e)),
    M = max D < 2^e, B = 63 - ceil(log2 n); target floor(r W / 2^64); the
    point whose weight interval holds the target; W = 0 -> floor(r n / 2^64).
    The first centroid is row floor(r_0 n / 2^64)."""
    n = X64.shape[0]
    rs = splitmix64_stream(seed, k)
    lg = 0
    while (1 << lg) < n:
        lg += 1
    B = 63 - lg
    rows = [(rs[0] * n) >> 64]
    D = None
    for t in range(1, k):
        acc = _dist2_rows(X64, X64[rows[-1]])
        D = acc if D is None else np.where(acc < D, acc, D)
        M = float(D.max())
        if M == 0.0:
            rows.append((rs[t] * n) >> 64)
            continue
        e = math.frexp(M)[1]                 # M < 2^e
        w = np.floor(np.ldexp(D, B - e)).astype(np.uint64)
        cs = np.cumsum(w, dtype=np.uint64)
        W = int(cs[-1])
        q = (rs[t] * W) >> 64
        rows.append(int(np.searchsorted(cs, np.uint64(q), side="right")))
    return rows
