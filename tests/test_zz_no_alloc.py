"""GPU: the allocation-free assignment (knor_assign_noalloc, through the C
ABI) equals knor_assign on the same inputs, on two calls in a row -- the
second smaller, so stale scratch from the first would show -- and a request
larger than its fixed scratch is refused before any device work."""
import ctypes

import numpy as np
import pytest

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


def _case(n, d, k, dtype, seed):
    rng = np.random.default_rng(seed)
    kc = max(2, min(k, 64))
    mu = rng.uniform(-10, 10, size=(kc, d))
    X = workloads.gaussian_mixture(rng, n, mu, np.ones(kc), np.ones(kc), dtype)
    rows = workloads.distinct_rows(rng, n, k)
    return X, workloads.to_f64(X[rows], dtype).copy()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_noalloc_equals_assign_on_two_calls(dtype):
    import torch
    knor = _knor()
    for (n, d, k, seed) in [(200000, 32, 300, 1), (5003, 17, 40, 2)]:
        print("CASE noalloc", dtype, n, d, k, flush=True)
        X, C = _case(n, d, k, dtype, seed)
        Xd, Cd = _dev(X, dtype), _dev(C, "f64")
        lab_ref, d2_ref = knor.assign(Xd, Cd, dist2=True)
        lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        d2 = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        knor.assign_noalloc(Xd, Cd, lab, d2)
        torch.cuda.synchronize()
        assert (lab == lab_ref).all()
        assert (d2 == d2_ref).all()


def test_noalloc_refuses_a_request_over_its_scratch():
    import torch
    knor = _knor()
    n, d, k = 9_000_000, 32, 64             # about 36 MB of flags alone
    X = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    C = torch.zeros((k, d), dtype=torch.float64, device="cuda")
    lab = torch.full((n,), 5, dtype=torch.int32, device="cuda")
    L = knor.load()
    o = knor._opts()
    rc = L.knor_assign_noalloc(X.data_ptr(), 1, n, d, C.data_ptr(), k, ctypes.byref(o),
                               lab.data_ptr(), None)
    assert rc == knor.KNOR_ERR_SCRATCH
    torch.cuda.synchronize()
    assert (lab == 5).all()                  # outputs untouched
