"""Python binding of the MI355X k-means library (libknor.so, C ABI in
include/knor.h).

Argument marshalling only: tensors must already live on the GPU; every step
of the Lloyd iteration runs in the library's HIP kernels.  There is no CPU
fallback -- importing works without a GPU, but every call needs the built
library and a visible GPU, and fails loudly otherwise.

    C, labels, stats = fit(X, k, C0=C0, max_iters=100, tol=0.0, prune=True)
    labels = assign(X, C)
    C_new, counts = update(X, labels, C_prev)

X: (n, d) CUDA tensor of float64, float32 or bfloat16, row-major contiguous.
C, C0, C_prev: (k, d) CUDA float64.  labels: (n,) CUDA int32.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["fit", "fit_batched", "assign", "assign_noalloc", "update", "load", "KnorError",
           "COUNTERS", "library_path", "mlp_param_count", "mlp_init",
           "mlp_train_step", "mlp_propose"]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_PKG, "libknor.so")

KNOR_OK, KNOR_ERR_INVALID_ARG, KNOR_ERR_OUT_OF_MEMORY, KNOR_ERR_HIP, \
    KNOR_ERR_NUMERIC, KNOR_ERR_UNSUPPORTED, KNOR_ERR_SCRATCH = range(7)
INIT_GIVEN, INIT_FORGY, INIT_SHUFFLE_FIRSTK, INIT_KMEANSPP = 0, 1, 2, 3
INITS = {"given": INIT_GIVEN, "forgy": INIT_FORGY,
         "shuffle_first_k": INIT_SHUFFLE_FIRSTK, "kmeans++": INIT_KMEANSPP}
NCOUNTERS = 9
COUNTERS = ("changed", "scanned", "pruned_a", "pruned_b", "rechecked",
            "certified", "queried", "dists", "forward")
CLAUSE2 = {"auto": 0, "off": 1, "on": 2}


class KnorError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"knor error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("prune", ctypes.c_int32),
                ("recheck", ctypes.c_int32), ("check_numeric", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p),
                ("workspace_cap", ctypes.c_size_t),
                ("label_history", ctypes.c_void_p),
                ("iter_counters", ctypes.c_void_p),
                ("poll_every", ctypes.c_int32),
                ("profile_ms", ctypes.c_void_p),
                ("profile_launches", ctypes.c_void_p),
                ("profile_mask", ctypes.c_int32),
                ("tile_blocks", ctypes.c_int32),
                ("tile_resident", ctypes.c_int32),
                ("autotune", ctypes.c_int32),
                ("learned", ctypes.c_int32),
                ("train_iters", ctypes.c_int32),
                ("train_batches", ctypes.c_int32),
                ("profile_every", ctypes.c_int32),
                ("update", ctypes.c_int32),
                ("centroid_history", ctypes.c_void_p),
                ("clause2", ctypes.c_int32),
                ("batch_graph", ctypes.c_int32),
                ("objective_history", ctypes.c_void_p)]


NPROF = 10
PROF_GROUPS = ("assign_dense", "assign_list", "recheck", "filter", "sort",
               "leaf", "tree", "cc", "learned", "certify")


class Problem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("dt", ctypes.c_int),
                ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("k", ctypes.c_int32), ("C_init", ctypes.c_void_p),
                ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("C_out", ctypes.c_void_p), ("labels_out", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("changed_last", ctypes.c_int64),
                ("dists_computed", ctypes.c_int64),
                ("scanned", ctypes.c_int64), ("pruned_a", ctypes.c_int64),
                ("pruned_b", ctypes.c_int64), ("rechecked", ctypes.c_int64),
                ("objective", ctypes.c_double), ("seconds", ctypes.c_double),
                ("certified", ctypes.c_int64), ("mlp_queries", ctypes.c_int64),
                ("mlp_forward_rows", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


class StreamOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("batch_rows", ctypes.c_int64),
                ("cache_rows", ctypes.c_int64), ("cache_interval", ctypes.c_int32),
                ("skip_objective", ctypes.c_int32), ("io_counters", ctypes.c_void_p)]


# columns of the streamed fit's per-iteration I/O counters (KNOR_IO_*)
IO_COUNTERS = ["copied", "gathered", "cached", "admitted"]
NIO = len(IO_COUNTERS)


def library_path() -> str:
    return _LIB


def load():
    """Load libknor.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise RuntimeError(
            f"{_LIB} is missing: build it first (python -m "
            "paper_1606_08905_amd._build); there is no CPU fallback")
    L = ctypes.CDLL(_LIB)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.knor_fit.argtypes = [P, ctypes.c_int, i64, i32, i32, ctypes.c_int, P, i32,
                           f64, ctypes.POINTER(Opts), P, P, ctypes.POINTER(Stats)]
    L.knor_fit.restype = ctypes.c_int
    L.knor_assign.argtypes = [P, ctypes.c_int, i64, i32, P, i32,
                              ctypes.POINTER(Opts), P, P]
    L.knor_assign.restype = ctypes.c_int
    L.knor_assign_noalloc.argtypes = [P, ctypes.c_int, i64, i32, P, i32,
                                      ctypes.POINTER(Opts), P, P]
    L.knor_assign_noalloc.restype = ctypes.c_int
    L.knor_tile_values.argtypes = [P, ctypes.c_int, i64, i32, P, i32,
                                   ctypes.POINTER(Opts), P, P]
    L.knor_tile_values.restype = ctypes.c_int
    L.knor_update.argtypes = [P, ctypes.c_int, i64, i32, P, i32, P,
                              ctypes.POINTER(Opts), P, P]
    L.knor_update.restype = ctypes.c_int
    L.knor_fit_streamed.argtypes = [P, ctypes.c_int, i64, i32, i32, ctypes.c_int, P, i32,
                                    f64, ctypes.POINTER(Opts), ctypes.POINTER(StreamOpts),
                                    P, P, ctypes.POINTER(Stats)]
    L.knor_fit_streamed.restype = ctypes.c_int
    L.knor_fit_batched.argtypes = [ctypes.POINTER(Problem), i32,
                                   ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
    L.knor_fit_batched.restype = ctypes.c_int
    L.knor_mlp_param_count.argtypes = [i32, i32, i32]
    L.knor_mlp_param_count.restype = i64
    L.knor_mlp_init.argtypes = [P, i32, i32, i32, ctypes.c_uint64, ctypes.POINTER(Opts)]
    L.knor_mlp_init.restype = ctypes.c_int
    L.knor_mlp_train_step.argtypes = [P, P, P, i64, i32, i32, i32, P, P, i32,
                                      ctypes.c_float, P, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(Opts)]
    L.knor_mlp_train_step.restype = ctypes.c_int
    L.knor_mlp_propose.argtypes = [P, i32, i32, i32, P, i64, P, ctypes.POINTER(Opts)]
    L.knor_mlp_propose.restype = ctypes.c_int
    L.knor_status_string.argtypes = [ctypes.c_int]
    L.knor_status_string.restype = ctypes.c_char_p
    L.knor_version.restype = ctypes.c_int32
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    m = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
    if t.dtype not in m:
        raise TypeError(f"unsupported point dtype {t.dtype}")
    return m[t.dtype]


def _check_dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (no CPU path exists)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _raise(rc):
    if rc != KNOR_OK:
        raise KnorError(rc, load().knor_status_string(rc).decode())


def _opts(prune=True, recheck=1, check_numeric=True, seed=0, stream=None,
          workspace_cap=0, label_history=None, iter_counters=None,
          poll_every=0, profile=None, tile_blocks=0, tile_resident=0,
          autotune=False, learned=False, train_iters=0, train_batches=0,
          update="canonical", centroid_history=None, clause2="auto",
          objective_history=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    o = Opts()
    o.struct_size = ctypes.sizeof(Opts)
    o.prune = 1 if prune else 0
    o.recheck = int(recheck)
    o.check_numeric = 1 if check_numeric else 0
    o.seed = int(seed)
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    o.workspace_cap = int(workspace_cap)
    o.label_history = label_history.data_ptr() if label_history is not None else None
    o.iter_counters = iter_counters.ctypes.data if iter_counters is not None else None
    o.poll_every = int(poll_every)
    if profile is not None:
        ms, launches = profile[0], profile[1]
        o.profile_ms = ms.ctypes.data
        o.profile_launches = launches.ctypes.data
        o.profile_mask = int(profile[2]) if len(profile) > 2 else 0
        o.profile_every = int(profile[3]) if len(profile) > 3 else 0
    o.tile_blocks = int(tile_blocks)
    o.tile_resident = int(tile_resident)
    o.autotune = 1 if autotune else 0
    o.learned = 1 if learned else 0
    o.train_iters = int(train_iters)
    o.train_batches = int(train_batches)
    o.update = _update_code(update)
    o.centroid_history = (centroid_history.data_ptr()
                          if centroid_history is not None else None)
    if clause2 not in CLAUSE2:
        raise ValueError(f"clause2 must be one of {sorted(CLAUSE2)}")
    o.clause2 = CLAUSE2[clause2]
    o.objective_history = (objective_history.ctypes.data
                           if objective_history is not None else None)
    return o


UPDATES = {"canonical": 0, "exact": 1}


def _update_code(update):
    if update not in UPDATES:
        raise ValueError(f"update must be one of {sorted(UPDATES)}")
    return UPDATES[update]


def fit(X, k, C0=None, init="given", max_iters=100, tol=0.0, prune=True,
        recheck=1, seed=0, history=False, counters=False, out=None,
        check_numeric=True, workspace_cap=0, poll_every=0, profile=None,
        tile_blocks=0, tile_resident=0, autotune=False, learned=False,
        train_iters=0, train_batches=0, update="canonical",
        centroid_history=False, clause2="auto", objective_history=False):
    """Lloyd's k-means on the GPU.  Returns (C, labels, stats dict).

    init: "given" (C0), "forgy", "shuffle_first_k" or "kmeans++" (the last
    three are deterministic functions of seed and X; see include/knor.h).

    history=True adds stats["label_history"]: (iters, n) int32 CUDA tensor of
    the labels each iteration's assignment produced; centroid_history=True
    adds stats["centroid_history"]: (iters, k, d) float64 CUDA tensor of the
    centroids each iteration's assignment used.  counters=True adds
    stats["counters"]: (iters, 9) int64 numpy array (KNOR_CNT_* columns).
    objective_history=True adds stats["objective_history"]: (iters,) float64
    numpy array of J_t (the canonical-order sum of each point's FP64 distance
    to its iteration-t centroid, under the centroids iteration t used).
    out=(C, labels) reuses preallocated output tensors.  profile=(ms, launches
    [, mask]) (float64 and int64 numpy arrays of NPROF entries, optional bit
    mask of groups) accumulates per-group GPU time measured with HIP events
    on the launch stream.  tile_blocks / tile_resident force an FP32 tile
    schedule (1, 2 or 4 blocks of 16 points per wave; 1 resident, 2
    chunked); autotune=True times the schedules of this (d, k) class once
    per process.  No schedule changes the results.  learned=True adds the
    certified MLP candidate proposal on MTI survivors (train_iters /
    train_batches: 0 = library defaults); it never changes the results.
    clause2="auto" | "off" | "on": MTI Clause 2 per block of survivors (see
    include/knor.h; "auto" uses it for FP32 points with 1024 <= k <= 8192).
    update="exact" takes each centroid as the exact member mean rounded once
    (FP32 / BF16 points), moving only changed points between sums when few
    change; "canonical" (default) sums in the canonical order."""
    torch = _torch()
    import numpy as np
    L = load()
    _check_dev(X, "X")
    n, d = X.shape
    dev = X.device
    if out is None:
        C = torch.empty((k, d), dtype=torch.float64, device=dev)
        lab = torch.empty((n,), dtype=torch.int32, device=dev)
    else:
        C, lab = out
    if init not in INITS:
        raise ValueError(f"init must be one of {sorted(INITS)}")
    init_code = INITS[init]
    if init_code == INIT_GIVEN:
        if C0 is None:
            raise ValueError("init='given' needs C0")
        C0 = torch.as_tensor(C0, dtype=torch.float64, device=dev).contiguous()
        c0p = C0.data_ptr()
    else:
        c0p = None
    hist = torch.empty((max_iters, n), dtype=torch.int32, device=dev) if history else None
    chist = (torch.empty((max_iters, k, d), dtype=torch.float64, device=dev)
             if centroid_history else None)
    cnt = np.zeros((max_iters, NCOUNTERS), np.int64) if counters else None
    objh = np.zeros(max_iters, np.float64) if objective_history else None
    o = _opts(prune, recheck, check_numeric, seed, None, workspace_cap, hist,
              cnt, poll_every, profile, tile_blocks, tile_resident, autotune,
              learned, train_iters, train_batches, update, chist, clause2, objh)
    st = Stats()
    rc = L.knor_fit(X.data_ptr(), _dtype_code(X), n, d, k, init_code, c0p,
                    max_iters, float(tol), ctypes.byref(o), C.data_ptr(),
                    lab.data_ptr(), ctypes.byref(st))
    _raise(rc)
    s = st.as_dict()
    if history:
        s["label_history"] = hist[: st.iters]
    if counters:
        s["counters"] = cnt[: st.iters]
    if centroid_history:
        s["centroid_history"] = chist[: st.iters]
    if objective_history:
        s["objective_history"] = objh[: st.iters]
    return C, lab, s


def fit_streamed(X, k, C0=None, init="given", max_iters=100, tol=0.0, prune=True,
                 recheck=1, seed=0, history=False, counters=False, check_numeric=True,
                 workspace_cap=0, tile_blocks=0, tile_resident=0, batch_rows=0,
                 cache_rows=0, cache_interval=0, objective=True, centroid_history=False,
                 device=None):
    """Lloyd's k-means with the rows in host memory (knor_fit_streamed).

    X: a CPU tensor in pinned memory (torch.Tensor.pin_memory()), float32
    or bfloat16.  The outputs live on `device` (default: the current CUDA
    device).  Same results as fit(..., update="exact") on the same values.
    batch_rows / cache_rows / cache_interval: 0 = library defaults (2^22
    rows per batch, no row cache, refresh interval 5).  objective=False
    skips the final pass that computes stats["objective"].  Returns (C,
    labels, stats dict) with stats["io"]: (iters, 4) int64 numpy array of
    rows copied whole, gathered one by one, served by the row cache, and
    admitted to it (IO_COUNTERS), plus the options of fit()."""
    torch = _torch()
    import numpy as np
    L = load()
    if X.is_cuda or not X.is_pinned():
        raise ValueError("X must be a pinned CPU tensor (X.pin_memory())")
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    n, d = X.shape
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    C = torch.empty((k, d), dtype=torch.float64, device=dev)
    lab = torch.empty((n,), dtype=torch.int32, device=dev)
    if init not in INITS:
        raise ValueError(f"init must be one of {sorted(INITS)}")
    init_code = INITS[init]
    if init_code == INIT_GIVEN:
        if C0 is None:
            raise ValueError("init='given' needs C0")
        C0 = torch.as_tensor(C0, dtype=torch.float64, device=dev).contiguous()
        c0p = C0.data_ptr()
    else:
        c0p = None
    hist = torch.empty((max_iters, n), dtype=torch.int32, device=dev) if history else None
    chist = (torch.empty((max_iters, k, d), dtype=torch.float64, device=dev)
             if centroid_history else None)
    cnt = np.zeros((max_iters, NCOUNTERS), np.int64) if counters else None
    io = np.zeros((max_iters, NIO), np.int64)
    o = _opts(prune, recheck, check_numeric, seed, None, workspace_cap, hist, cnt, 0,
              None, tile_blocks, tile_resident, False, False, 0, 0, "exact", chist, "auto")
    so = StreamOpts()
    so.struct_size = ctypes.sizeof(StreamOpts)
    so.batch_rows = int(batch_rows)
    so.cache_rows = int(cache_rows)
    so.cache_interval = int(cache_interval)
    so.skip_objective = 0 if objective else 1
    so.io_counters = io.ctypes.data
    st = Stats()
    with torch.cuda.device(dev):
        rc = L.knor_fit_streamed(X.data_ptr(), _dtype_code(X), n, d, k, init_code, c0p,
                                 max_iters, float(tol), ctypes.byref(o), ctypes.byref(so),
                                 C.data_ptr(), lab.data_ptr(), ctypes.byref(st))
    _raise(rc)
    s = st.as_dict()
    s["io"] = io[: st.iters]
    if history:
        s["label_history"] = hist[: st.iters]
    if counters:
        s["counters"] = cnt[: st.iters]
    if centroid_history:
        s["centroid_history"] = chist[: st.iters]
    return C, lab, s


def fit_batched(problems, prune=True, recheck=1, seed=0, check_numeric=True,
                workspace_cap=0, tile_blocks=0, tile_resident=0, update="canonical",
                clause2="auto", graph=False):
    """knor_fit on each problem of a batch, run concurrently.  problems: list
    of dicts with keys X, k and optionally C0 (None: Forgy from seed + index),
    max_iters (default 100), tol (default 0).  graph=True records every
    problem's iterations into one HIP graph launched once (knor_opts.
    batch_graph).  Returns a list of (C, labels, stats dict), each equal to
    what fit() gives on its own."""
    torch = _torch()
    L = load()
    arr = (Problem * max(1, len(problems)))()
    keep, outs = [], []
    for i, p in enumerate(problems):
        X = p["X"]
        _check_dev(X, "X")
        n, d = X.shape
        k = int(p["k"])
        C = torch.empty((k, d), dtype=torch.float64, device=X.device)
        lab = torch.empty((n,), dtype=torch.int32, device=X.device)
        C0 = p.get("C0")
        if C0 is not None:
            C0 = torch.as_tensor(C0, dtype=torch.float64, device=X.device).contiguous()
            keep.append(C0)
        a = arr[i]
        a.X = X.data_ptr(); a.dt = _dtype_code(X); a.n = n; a.d = d; a.k = k
        a.C_init = C0.data_ptr() if C0 is not None else None
        a.max_iters = int(p.get("max_iters", 100)); a.tol = float(p.get("tol", 0.0))
        a.C_out = C.data_ptr(); a.labels_out = lab.data_ptr()
        outs.append((C, lab))
    o = _opts(prune, recheck, check_numeric, seed, None, workspace_cap,
              tile_blocks=tile_blocks, tile_resident=tile_resident, update=update,
              clause2=clause2)
    o.batch_graph = 1 if graph else 0
    sts = (Stats * max(1, len(problems)))()
    rc = L.knor_fit_batched(arr, len(problems), ctypes.byref(o), sts)
    _raise(rc)
    return [(C, lab, sts[i].as_dict()) for i, (C, lab) in enumerate(outs)]


def assign(X, C, recheck=1, dist2=False):
    """Nearest centroid of every row of X (and, with dist2=True, the FP64
    squared distance to it).  Asynchronous on the current stream."""
    torch = _torch()
    L = load()
    _check_dev(X, "X")
    _check_dev(C, "C")
    if C.dtype != torch.float64:
        raise TypeError("C must be float64")
    n, d = X.shape
    k = C.shape[0]
    lab = torch.empty((n,), dtype=torch.int32, device=X.device)
    dd = torch.empty((n,), dtype=torch.float64, device=X.device) if dist2 else None
    o = _opts(recheck=recheck)
    rc = L.knor_assign(X.data_ptr(), _dtype_code(X), n, d, C.data_ptr(), k,
                       ctypes.byref(o), lab.data_ptr(),
                       dd.data_ptr() if dd is not None else None)
    _raise(rc)
    return (lab, dd) if dist2 else lab


def assign_noalloc(X, C, labels, dist2=None, recheck=1):
    """knor_assign_noalloc: the assignment into caller-provided outputs
    (labels: (n,) int32, dist2: (n,) float64 or None) with no device
    allocation in the library (its fixed per-GPU scratch).  Asynchronous on
    the current stream; calls that overlap on one GPU race."""
    torch = _torch()
    L = load()
    _check_dev(X, "X")
    _check_dev(C, "C")
    _check_dev(labels, "labels")
    if C.dtype != torch.float64 or labels.dtype != torch.int32:
        raise TypeError("C must be float64 and labels int32")
    n, d = X.shape
    k = C.shape[0]
    o = _opts(recheck=recheck)
    rc = L.knor_assign_noalloc(X.data_ptr(), _dtype_code(X), n, d, C.data_ptr(), k,
                               ctypes.byref(o), labels.data_ptr(),
                               dist2.data_ptr() if dist2 is not None else None)
    _raise(rc)
    return labels


def tile_values(X, C):
    """(Y, E): the assignment tile's FP32 values Y[p][j] of |c_j|^2 - 2 x_p.c_j
    and the rounding bound E[p] its decisions use (FP32 / BF16 points)."""
    torch = _torch()
    L = load()
    _check_dev(X, "X")
    _check_dev(C, "C")
    n, d = X.shape
    k = C.shape[0]
    Y = torch.empty((n, k), dtype=torch.float32, device=X.device)
    E = torch.empty((n,), dtype=torch.float64, device=X.device)
    o = _opts()
    _raise(L.knor_tile_values(X.data_ptr(), _dtype_code(X), n, d, C.data_ptr(), k,
                              ctypes.byref(o), Y.data_ptr(), E.data_ptr()))
    return Y, E


def update(X, labels, C_prev, mode="canonical"):
    """Centroids as member means (empty clusters keep C_prev) and counts.
    mode="exact": the exact mean rounded once (FP32 / BF16 points)."""
    torch = _torch()
    L = load()
    _check_dev(X, "X")
    _check_dev(labels, "labels")
    _check_dev(C_prev, "C_prev")
    if labels.dtype != torch.int32 or C_prev.dtype != torch.float64:
        raise TypeError("labels must be int32 and C_prev float64")
    n, d = X.shape
    k = C_prev.shape[0]
    C = torch.empty_like(C_prev)
    cnt = torch.empty((k,), dtype=torch.int64, device=X.device)
    o = _opts(update=mode)
    rc = L.knor_update(X.data_ptr(), _dtype_code(X), n, d, labels.data_ptr(), k,
                       C_prev.data_ptr(), ctypes.byref(o), C.data_ptr(),
                       cnt.data_ptr())
    _raise(rc)
    return C, cnt


# ---------------------------------------------------------------------------
# the proposal MLP on its own
# ---------------------------------------------------------------------------

def mlp_param_count(d, h, k):
    return int(load().knor_mlp_param_count(d, h, k))


def mlp_init(d, h, k, seed, device="cuda"):
    """FP32 parameter vector (CUDA tensor) with the library's initialisation."""
    torch = _torch()
    L = load()
    P = mlp_param_count(d, h, k)
    if P < 0:
        raise ValueError("MLP sizes out of range")
    th = torch.empty((P,), dtype=torch.float32, device=device)
    _raise(L.knor_mlp_init(th.data_ptr(), d, h, k, int(seed), ctypes.byref(_opts())))
    return th


def mlp_train_step(params, m, v, step, d, h, k, Xs, y, lr=1e-3, grad=None):
    """One training step; returns the minibatch loss (params, m, v updated in
    place when lr > 0; grad, if given, receives the gradient)."""
    torch = _torch()
    L = load()
    for t, nm in ((params, "params"), (Xs, "Xs"), (y, "y")):
        _check_dev(t, nm)
    loss = ctypes.c_double(0.0)
    rc = L.knor_mlp_train_step(params.data_ptr(), m.data_ptr() if m is not None else None,
                               v.data_ptr() if v is not None else None, int(step), d, h, k,
                               Xs.data_ptr(), y.data_ptr(), int(Xs.shape[0]), float(lr),
                               grad.data_ptr() if grad is not None else None,
                               ctypes.byref(loss), ctypes.byref(_opts()))
    _raise(rc)
    return loss.value


def mlp_propose(params, d, h, k, Xs):
    """(m, 16) int32 CUDA tensor of candidate classes."""
    torch = _torch()
    L = load()
    _check_dev(Xs, "Xs")
    m = int(Xs.shape[0])
    cand = torch.empty((m, 16), dtype=torch.int32, device=Xs.device)
    _raise(L.knor_mlp_propose(params.data_ptr(), d, h, k, Xs.data_ptr(), m,
                              cand.data_ptr(), ctypes.byref(_opts())))
    return cand
