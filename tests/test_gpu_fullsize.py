"""GPU parity at the full sizes of the extended forms' workloads, on sampled
outputs the FP64 oracle can compute one by one, and on properties that hold
at any size:

  at every iteration t of a whole fit, the labels of 20000 random rows ==
  the oracle's assignment of those rows under the centroids C_t iteration t
  used (from the fit's centroid history), and C_{t+1} == the oracle's
  canonical update of every row from (labels_t, C_t), bit for bit;
  the returned centroids are the means of the returned labels (the oracle's
  update reproduces them bit for bit);
  a converged fit's labels are a fixed point of the oracle's assignment.
"""
import numpy as np
import pytest

import oracle
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


def _sample(n, m, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))


def _check_whole_fit(knor, w, Xd, C0d, rows, **kw):
    """Every iteration t of one fit: the labels of `rows` equal the oracle's
    assignment under the centroids C_t the iteration used, and C_{t+1} equals
    the oracle's canonical update of all rows from (labels_t, C_t), bit for
    bit (C_t from the fit's centroid history)."""
    C, lab, st = knor.fit(Xd, w.k, C0=C0d, max_iters=w.max_iters, history=True,
                          centroid_history=True, **kw)
    iters = st["iters"]
    H = st["label_history"]
    CH = st["centroid_history"].cpu().numpy()
    assert (CH[0] == w.C0).all()
    X64 = w.x64()
    X64s = X64[rows]
    Cfin = C.cpu().numpy()
    for t in range(iters):
        Ht = H[t].cpu().numpy()
        lab_o, _ = oracle.assign(X64s, CH[t])
        assert (Ht[rows] == lab_o).all(), t
        Cn, _ = oracle.update(X64, Ht, CH[t])
        nxt = CH[t + 1] if t + 1 < iters else Cfin
        assert (nxt == Cn).all(), t
    assert (lab.cpu().numpy() == H[iters - 1].cpu().numpy()).all()
    return C, lab, st


def test_mixed_precision_full_size():
    """BF16, n=2e7, d=64, k=256, MTI: all 30 iterations."""
    knor = _knor()
    w = workloads.config(3)
    print("CASE mixed full", w.n, flush=True)
    rows = _sample(w.n, 20000, 3)
    _, _, st = _check_whole_fit(knor, w, _dev(w.X, "bf16"), _dev(w.C0, "f64"), rows)
    assert st["iters"] == w.max_iters or st["converged"]


def test_learned_full_size():
    """FP32, n=1e7, d=32, k=4096, MTI + learned proposal (trained on
    iterations 1-5, proposing from iteration 6): all 40 iterations; the
    whole fit equals the one without the proposal."""
    knor = _knor()
    w = workloads.config(5)
    print("CASE learned full", w.n, flush=True)
    Xd, C0d = _dev(w.X, "f32"), _dev(w.C0, "f64")
    rows = _sample(w.n, 20000, 5)
    C, lab, st = _check_whole_fit(knor, w, Xd, C0d, rows, learned=True)
    assert st["mlp_queries"] > 0 and st["certified"] > 0
    Cm, labm, _ = knor.fit(Xd, w.k, C0=C0d, max_iters=w.max_iters)
    assert (C == Cm).all() and (lab == labm).all()


def test_batched_full_size():
    """The 64-problem batch at full size: every problem equals its single
    fit; returned centroids are the oracle's means of the returned labels;
    converged problems' labels are fixed points of the oracle's assignment
    (sampled rows)."""
    knor = _knor()
    ws = workloads.batched(64)
    print("CASE batched full", sum(w.n for w in ws), flush=True)
    probs = [dict(X=_dev(w.X, "f32"), k=w.k, C0=_dev(w.C0, "f64"), max_iters=w.max_iters)
             for w in ws]
    out = knor.fit_batched(probs)
    for i, (w, p, (C, lab, st)) in enumerate(zip(ws, probs, out)):
        Cs, labs, sts = knor.fit(p["X"], w.k, C0=p["C0"], max_iters=w.max_iters)
        assert (C == Cs).all() and (lab == labs).all() and st["iters"] == sts["iters"], i
        Ch, labh = C.cpu().numpy(), lab.cpu().numpy()
        X64 = w.X.astype(np.float64)
        Cu, _ = oracle.update(X64, labh, Ch)
        assert (Cu == Ch).all(), i
        if st["converged"]:
            rows = _sample(w.n, min(w.n, 4000), i)
            lab_o, _ = oracle.assign(X64[rows], Ch)
            assert (labh[rows] == lab_o).all(), i
