"""GPU: the assignment tiles' rounding bound E(x) holds.

For every (point, centroid) pair the tile's FP32 value y~ of
y = |c|^2 - 2 x.c must satisfy |y~ - y| <= E(x), the bound its decisions
use (a point is trusted only when its two smallest values differ by more
than 2E plus the FP64 evaluation error).  The values come from the
library's own accumulation code (knor_tile_values); y is evaluated in FP64
on the GPU (its own error is below 2^-40 of E here).  Random pairs (over
10^8 per tile type) and adversarial ones: large |x| against small |c|,
cancellation (x close to c, both far from the origin), exact duplicates,
dimensions at and around the tiles' padding edges, mixed magnitudes across
dimensions, and tiny values."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MAX_RATIO = {}


def _knor():
    import paper_1606_08905_amd as knor
    knor.load()
    return knor


def _ratio(X, C, dtype):
    """max over pairs of |y~ - y| / E(x), and the number of pairs."""
    import torch
    knor = _knor()
    if dtype == "bf16":
        Xd = torch.from_numpy(X.view(np.int16)).cuda().view(torch.bfloat16)
        X64 = torch.from_numpy(workloads.bf16_to_f64(X)).cuda()
    else:
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        X64 = Xd.double()
    Cd = torch.from_numpy(np.ascontiguousarray(C)).cuda()
    Y, E = knor.tile_values(Xd, Cd)
    cn = (Cd * Cd).sum(1)
    worst = 0.0
    n = X.shape[0]
    for r0 in range(0, n, 8192):
        y = cn[None, :] - 2.0 * (X64[r0:r0 + 8192] @ Cd.T)
        r = ((Y[r0:r0 + 8192].double() - y).abs() / E[r0:r0 + 8192, None]).max().item()
        worst = max(worst, r)
    assert torch.isfinite(E).all() and (E > 0).all()
    return worst, n * C.shape[0]


def _check(name, X, C, dtype):
    r, pairs = _ratio(X, C, dtype)
    MAX_RATIO[(name, dtype)] = (r, pairs)
    print(f"BOUND {dtype} {name}: max |y~ - y| / E = {r:.3e} over {pairs} pairs", flush=True)
    assert r <= 1.0, (name, r)


@pytest.mark.parametrize("dtype,n,d,k", [("f32", 100_000, 32, 1024),
                                         ("bf16", 50_000, 64, 2048)])
def test_bound_random_pairs(dtype, n, d, k):
    rng = np.random.default_rng(1)
    X = workloads.cast(rng.normal(size=(n, d)) * rng.uniform(0.1, 30, size=(n, 1)), dtype)
    C = rng.normal(size=(k, d)) * rng.uniform(0.1, 30, size=(k, 1))
    _check("random", X, C, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bound_adversarial(dtype):
    rng = np.random.default_rng(2)
    n, k = 4000, 300
    cases = []
    # large |x| against small |c|
    cases.append(("large-x", 1e4 + rng.normal(size=(n, 32)), rng.normal(size=(k, 32))))
    # cancellation: points next to centroids far from the origin
    C = 1e3 + rng.normal(size=(k, 32)) * 1e-2
    cases.append(("cancellation", C[rng.integers(0, k, n)] + rng.normal(size=(n, 32)) * 1e-3, C))
    # exact duplicates (rows of X as centroids)
    Xdup = rng.normal(size=(n, 24)) * 50
    cases.append(("duplicates", Xdup, workloads.to_f64(workloads.cast(Xdup[:k], dtype), dtype)))
    # mixed magnitudes across dimensions
    sc = 10.0 ** rng.uniform(-3, 3, size=40)
    cases.append(("mixed-scale", rng.normal(size=(n, 40)) * sc, rng.normal(size=(k, 40)) * sc))
    # tiny values (products far below the normal range of FP32 for BF16/FP32)
    cases.append(("tiny", rng.normal(size=(n, 16)) * 1e-20, rng.normal(size=(k, 16)) * 1e-19))
    for name, X, C in cases:
        _check(name, workloads.cast(X, dtype), C, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bound_dimensions_at_tile_edges(dtype):
    rng = np.random.default_rng(3)
    for d in (1, 3, 4, 7, 8, 9, 16, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256):
        X = workloads.cast(rng.normal(size=(3000, d)) * 20, dtype)
        C = rng.normal(size=(257, d)) * 20
        _check(f"d={d}", X, C, dtype)
