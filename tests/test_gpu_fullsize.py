"""GPU parity at the full sizes of the extended forms' workloads, on sampled
outputs the FP64 oracle can compute one by one, and on properties that hold
at any size:

  labels of iteration t on random rows == the oracle's assignment of those
  rows at the centroids iteration t used (C_t from fits stopped after t
  iterations; labels do not depend on where a fit stops);
  the centroids after iteration 0 == the oracle's canonical update of the
  full data (exact FP64 means, every row);
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


def _check_iterations(knor, w, Xd, C0d, iters, rows, **kw):
    """Labels of iterations 0..iters-1 on `rows` against the oracle, and the
    first update against the oracle's full canonical update."""
    _, _, st = knor.fit(Xd, w.k, C0=C0d, max_iters=iters, history=True, **kw)
    hist = st["label_history"].cpu().numpy()
    X64s = workloads.to_f64(w.X[rows], w.dtype)
    C_t = w.C0
    for t in range(min(iters, st["iters"])):
        lab_o, _ = oracle.assign(X64s, C_t)
        assert (hist[t][rows] == lab_o).all(), t
        if t + 1 < iters:
            C_t = knor.fit(Xd, w.k, C0=C0d, max_iters=t + 1, **kw)[0].cpu().numpy()
            if t == 0:
                C1_o, _ = oracle.update(w.x64(), hist[0], w.C0)
                assert (C_t == C1_o).all()
    return st


def test_mixed_precision_full_size():
    """BF16, n=2e7, d=64, k=256, MTI: three iterations sampled."""
    knor = _knor()
    w = workloads.config(3)
    print("CASE mixed full", w.n, flush=True)
    rows = _sample(w.n, 20000, 3)
    _check_iterations(knor, w, _dev(w.X, "bf16"), _dev(w.C0, "f64"), 3, rows)


def test_learned_full_size():
    """FP32, n=1e7, d=32, k=4096, MTI + learned proposal (trained on
    iterations 1-5, proposing from iteration 6): iterations 0, 1, 6 sampled;
    the whole fit equals the one without the proposal."""
    knor = _knor()
    w = workloads.config(5)
    print("CASE learned full", w.n, flush=True)
    Xd, C0d = _dev(w.X, "f32"), _dev(w.C0, "f64")
    rows = _sample(w.n, 8000, 5)
    X64s = w.X[rows].astype(np.float64)
    C, lab, st = knor.fit(Xd, w.k, C0=C0d, max_iters=7, history=True, learned=True)
    hist = st["label_history"].cpu().numpy()
    for t in (0, 1, 6):
        C_t = w.C0 if t == 0 else knor.fit(Xd, w.k, C0=C0d, max_iters=t,
                                           learned=True)[0].cpu().numpy()
        lab_o, _ = oracle.assign(X64s, C_t)
        assert (hist[t][rows] == lab_o).all(), t
    C1_o, _ = oracle.update(w.x64(), hist[0], w.C0)
    assert (knor.fit(Xd, w.k, C0=C0d, max_iters=1)[0].cpu().numpy() == C1_o).all()
    Cm, labm, _ = knor.fit(Xd, w.k, C0=C0d, max_iters=7)
    assert (C == Cm).all() and (lab == labm).all()
    assert st["mlp_queries"] > 0


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
