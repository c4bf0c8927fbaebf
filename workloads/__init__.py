"""Seeded synthetic inputs for the k-means hot path.

This module only *draws* data: Gaussian-mixture points, their storage-dtype
cast, and initial centroids.  It contains none of the Lloyd iteration's
arithmetic (no assignment, no update, no pruning), so that the FP64 oracle
and the GPU path can both be fed from it without sharing method code.

The paper evaluates on the Friendster eigenvector matrices and on synthetic
RM/RU matrices (Table 2).  Those data are not available here; the
configurations below are synthetic stand-ins with the paper's shapes
(d = 16 as RM856M, d = 32 with k in the tens-to-hundreds as Friendster-32,
d = 64 as RU2B).  The paper is silent on initialisation; each configuration
fixes its own seeding rule, and every parity run passes the resulting C0
explicitly.

Every array is a deterministic function of (configuration, seed, n):
  rng = numpy.random.default_rng(seed)      (PCG64)
  component z ~ Categorical(w),  x = mu_z + sigma_z * N(0, I_d)  in FP64,
  then cast to the storage dtype (BF16 by round-to-nearest-even from FP64);
  the cast array *is* the dataset.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Row chunk for drawing the Gaussian noise; part of the definition of the
# stream of draws (changing it changes the data).
_CHUNK = 1 << 20

DTYPES = ("f64", "f32", "bf16")


@dataclasses.dataclass
class Workload:
    """One synthetic clustering problem.

    X      : (n, d) array in the storage dtype.  f64 -> float64, f32 -> float32,
             bf16 -> uint16 holding the BF16 bit patterns.
    C0     : (k, d) float64 initial centroids (rows of X, upcast exactly).
    dtype  : "f64" | "f32" | "bf16".
    meta   : dict describing the recipe (sizes, seeds, init rule, stop rule).
    """

    X: np.ndarray
    C0: np.ndarray
    k: int
    dtype: str
    max_iters: int
    tol: float
    meta: dict

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    def x64(self) -> np.ndarray:
        """The dataset upcast to float64 (exact for every storage dtype)."""
        return to_f64(self.X, self.dtype)


# ---------------------------------------------------------------------------
# storage-dtype casts (representation only)
# ---------------------------------------------------------------------------

def bf16_from_f64(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to BF16 (round to nearest, ties to even), returned as
    uint16 bit patterns.  Computed from the FP64 value in one rounding (no
    intermediate FP32 rounding).  Inputs must be finite."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    bits = x.view(np.uint64)
    sign = (bits >> np.uint64(63)).astype(np.uint16)
    ax = np.abs(x)
    # BF16 has an 8-bit significand (7 stored bits).  For a normal FP64 value
    # ax = m * 2^e with 1 <= m < 2, the BF16 grid spacing is 2^(e-7); the
    # smallest normal BF16 exponent is -126 and below it the spacing is 2^-133.
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0))).astype(np.int64)
    # guard log2 rounding at powers of two
    m = np.ldexp(ax, -e)
    e = np.where(m >= 2.0, e + 1, e)
    e = np.where((m < 1.0) & (ax > 0), e - 1, e)
    e = np.maximum(e, -126)
    q = np.ldexp(ax, -(e - 7))           # exact: scaling by a power of two
    r = np.rint(q)                        # round half to even
    y = np.ldexp(r, e - 7)                # exact
    y32 = y.astype(np.float32)            # exact: y has <= 8 significant bits
    out = (y32.view(np.uint32) >> np.uint32(16)).astype(np.uint16)
    out = np.where(ax == 0, np.uint16(0), out) | (sign << np.uint16(15))
    return out.astype(np.uint16)


def bf16_to_f64(b: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (uint16) -> float64, exactly."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def to_f64(X: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "bf16":
        return bf16_to_f64(X)
    return np.ascontiguousarray(X, dtype=np.float64)


def cast(x64: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f64":
        return np.ascontiguousarray(x64, dtype=np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(x64.astype(np.float32))
    if dtype == "bf16":
        return bf16_from_f64(x64)
    raise ValueError(f"unknown dtype {dtype!r}")


# ---------------------------------------------------------------------------
# draws
# ---------------------------------------------------------------------------

def gaussian_mixture(rng, n, means, sigmas, weights, dtype, out=None):
    """n points from sum_c w_c N(mu_c, sigma_c^2 I), drawn in FP64 and cast.

    Component labels for all n points are drawn first, then the N(0, I) noise
    in row chunks of a fixed size, so the stream of draws is fixed."""
    means = np.asarray(means, dtype=np.float64)
    sigmas = np.asarray(sigmas, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    kc, d = means.shape
    z = rng.choice(kc, size=n, p=weights / weights.sum())
    if out is None:
        out = np.empty((n, d), dtype=_np_store(dtype))
    for r0 in range(0, n, _CHUNK):
        r1 = min(n, r0 + _CHUNK)
        zz = z[r0:r1]
        x = means[zz] + sigmas[zz, None] * rng.standard_normal((r1 - r0, d))
        out[r0:r1] = cast(x, dtype)
    return out


def _np_store(dtype):
    return {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[dtype]


def distinct_rows(rng, n, k):
    """k distinct row indices drawn without replacement."""
    return rng.choice(n, size=k, replace=False)


def kmeanspp_rows(X64, k, rng):
    """Plain k-means++ seeding (Arthur & Vassilvitskii 2007): first row
    uniform, then each next row drawn with probability proportional to its
    squared distance to the nearest row already chosen; one candidate per
    step, FP64 on the host.  Returns the k chosen row indices.

    This is input generation (the paper is silent on initialisation); its
    squared distances are a sampling weight, not the method's assignment."""
    n = X64.shape[0]
    idx = np.empty(k, dtype=np.int64)
    idx[0] = rng.integers(n)
    diff = X64 - X64[idx[0]]
    w = np.einsum("ij,ij->i", diff, diff)
    for i in range(1, k):
        cw = np.cumsum(w)
        r = rng.random() * cw[-1]
        j = int(np.searchsorted(cw, r, side="right"))
        j = min(j, n - 1)
        idx[i] = j
        diff = X64 - X64[j]
        np.minimum(w, np.einsum("ij,ij->i", diff, diff), out=w)
    return idx


# ---------------------------------------------------------------------------
# the five configurations
# ---------------------------------------------------------------------------

FULL_N = {1: 10_000, 2: 1_000_000, 3: 20_000_000, 5: 10_000_000}


def config(i: int, n: int | None = None, seed: int = 0, init_seed: int = 1,
           k: int | None = None) -> Workload:
    """Configuration i in {1, 2, 3, 5}; n (and k) may be reduced for tests.

    1: plain Lloyd's, f64, d=16, k=10, 10 components, mu~U[-10,10]^d, sigma=1,
       equal weights; C0 = first k rows of a seeded shuffle; 50 iters, tol 0.
    2: MTI, f32, d=32, k=100, 100 components, mu~U[-20,20]^d,
       sigma_c~U[0.5,2], Dirichlet(1) weights; k-means++ seeding; 100 iters.
    3: mixed precision, bf16, d=64, k=256; 95% from 256 components
       mu~N(0,25 I), sigma=1.5, equal weights, 5% uniform on [-50,50]^d,
       shuffled; C0 = k distinct random rows; 30 iters.
    5: learned proposal, f32, d=32, k=4096, 4096 components mu~N(0,100 I),
       sigma_c~U[0.5,3], equal weights; C0 = k distinct random rows; 40 iters.
    """
    rng = np.random.default_rng(seed)
    rinit = np.random.default_rng(init_seed)
    if i == 1:
        n = n or FULL_N[1]
        d, kk = 16, (k or 10)
        kc = 10
        mu = rng.uniform(-10, 10, size=(kc, d))
        X = gaussian_mixture(rng, n, mu, np.ones(kc), np.ones(kc), "f64")
        perm = rinit.permutation(n)
        rows = perm[:kk]
        dtype, iters, init = "f64", 50, "shuffle-first-k"
    elif i == 2:
        n = n or FULL_N[2]
        d, kk = 32, (k or 100)
        kc = 100
        mu = rng.uniform(-20, 20, size=(kc, d))
        sig = rng.uniform(0.5, 2.0, size=kc)
        w = rng.dirichlet(np.ones(kc))
        X = gaussian_mixture(rng, n, mu, sig, w, "f32")
        rows = kmeanspp_rows(to_f64(X, "f32"), kk, rinit)
        dtype, iters, init = "f32", 100, "k-means++"
    elif i == 3:
        n = n or FULL_N[3]
        d, kk = 64, (k or 256)
        kc = 256
        n_out = int(round(0.05 * n))
        n_mix = n - n_out
        mu = rng.normal(0.0, 5.0, size=(kc, d))
        X = np.empty((n, d), dtype=np.uint16)
        gaussian_mixture(rng, n_mix, mu, np.full(kc, 1.5), np.ones(kc), "bf16",
                         out=X[:n_mix])
        for r0 in range(n_mix, n, _CHUNK):
            r1 = min(n, r0 + _CHUNK)
            X[r0:r1] = cast(rng.uniform(-50, 50, size=(r1 - r0, d)), "bf16")
        perm = rng.permutation(n)
        X = X[perm]
        rows = distinct_rows(rinit, n, kk)
        dtype, iters, init = "bf16", 30, "random-rows"
    elif i == 5:
        n = n or FULL_N[5]
        d, kk = 32, (k or 4096)
        kc = 4096 if k is None else max(k, 2)
        mu = rng.normal(0.0, 10.0, size=(kc, d))
        sig = rng.uniform(0.5, 3.0, size=kc)
        X = gaussian_mixture(rng, n, mu, sig, np.ones(kc), "f32")
        rows = distinct_rows(rinit, n, kk)
        dtype, iters, init = "f32", 40, "random-rows"
    else:
        raise ValueError("config must be one of 1, 2, 3, 5 (4 is batched())")
    C0 = to_f64(X[rows], dtype).copy()
    meta = dict(config=i, n=n, d=d, k=kk, dtype=dtype, seed=seed,
                init_seed=init_seed, init=init, max_iters=iters, tol=0.0)
    return Workload(X=np.ascontiguousarray(X), C0=C0, k=kk, dtype=dtype,
                    max_iters=iters, tol=0.0, meta=meta)


def batched_instance(s: int, n_scale: float = 1.0) -> Workload:
    """Instance s (0..63) of the batched-restart workload.

    rng = default_rng(s); n = round(exp(U[ln 1e4, ln 2e6])) (scaled by
    n_scale for tests, at least 2k); d ~ U{8,16,32,64}; k ~ U{8..512};
    k components mu~U[-10,10]^d, sigma=1, equal weights; C0 = k distinct
    random rows from the same rng; f32; 50 iterations."""
    rng = np.random.default_rng(s)
    n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6)))))
    d = int(rng.choice([8, 16, 32, 64]))
    k = int(rng.integers(8, 513))
    n = max(int(round(n * n_scale)), 2 * k)
    mu = rng.uniform(-10, 10, size=(k, d))
    X = gaussian_mixture(rng, n, mu, np.ones(k), np.ones(k), "f32")
    rows = distinct_rows(rng, n, k)
    C0 = to_f64(X[rows], "f32").copy()
    meta = dict(config=4, instance=s, n=n, d=d, k=k, dtype="f32",
                init="random-rows", max_iters=50, tol=0.0)
    return Workload(X=X, C0=C0, k=k, dtype="f32", max_iters=50, tol=0.0,
                    meta=meta)


def batched(count: int = 64, n_scale: float = 1.0):
    return [batched_instance(s, n_scale) for s in range(count)]


def uniform_cube(n, d, dtype="f32", seed=0, lo=-1.0, hi=1.0):
    """Unclustered control data: U[lo, hi]^d."""
    rng = np.random.default_rng(seed)
    return cast(rng.uniform(lo, hi, size=(n, d)), dtype)
