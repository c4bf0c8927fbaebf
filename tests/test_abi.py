"""Host-only checks of the C ABI: the library loads, exports every function
that include/knor.h declares, and rejects invalid arguments before touching
any device memory (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1606_08905_amd as knor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "knor.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knor_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(knor.library_path()):
        pytest.skip("libknor.so not built")
    return knor.load()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert {"knor_fit", "knor_assign", "knor_update", "knor_status_string",
            "knor_version"} <= set(names)
    for nm in names:
        assert hasattr(L, nm), nm


def test_status_strings(L):
    for code in range(6):
        assert L.knor_status_string(code)
    assert L.knor_version() >= 400


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _fit(L, **kw):
    a = dict(X=FAKE, dt=1, n=100, d=8, k=4, init=0, C=FAKE, it=10, tol=0.0,
             opts=None, Cout=FAKE, lab=FAKE, st=None)
    a.update(kw)
    return L.knor_fit(a["X"], a["dt"], a["n"], a["d"], a["k"], a["init"], a["C"],
                      a["it"], a["tol"], a["opts"], a["Cout"], a["lab"], a["st"])


@pytest.mark.parametrize("kw", [
    dict(X=None), dict(dt=9), dict(n=0), dict(d=0), dict(d=257), dict(k=0),
    dict(k=101), dict(k=20000, n=30000), dict(it=0), dict(tol=1.0),
    dict(tol=-0.1), dict(tol=float("nan")), dict(init=0, C=None), dict(init=4),
    dict(init=-1),
    dict(Cout=None), dict(lab=None), dict(n=1 << 31),
])
def test_fit_rejects_invalid(L, kw):
    assert _fit(L, **kw) == knor.KNOR_ERR_INVALID_ARG


def test_fit_rejects_bad_opts(L):
    o = knor.Opts()
    o.struct_size = 3
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.batch_graph = 2
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 7
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    o.recheck = 1
    o.profile_every = -1
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG


def test_assign_update_reject_invalid(L):
    P = FAKE
    assert L.knor_assign(None, 1, 10, 4, P, 2, None, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_assign(P, 1, 10, 0, P, 2, None, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_assign(P, 1, 10, 4, P, 0, None, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_update(P, 1, 10, 4, None, 2, P, None, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_update(P, 1, -1, 4, P, 2, P, None, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_update(P, 3, 10, 4, P, 2, P, None, P, None) == knor.KNOR_ERR_INVALID_ARG


def test_binding_refuses_cpu_tensors():
    import torch
    X = torch.zeros((10, 4))
    with pytest.raises((ValueError, RuntimeError)):
        knor.fit(X, 2, C0=torch.zeros((2, 4), dtype=torch.float64))


def _problem(**kw):
    p = knor.Problem()
    p.X = 0x1000; p.dt = 1; p.n = 100; p.d = 8; p.k = 4; p.C_init = 0x1000
    p.max_iters = 10; p.tol = 0.0; p.C_out = 0x1000; p.labels_out = 0x1000
    for key, v in kw.items():
        setattr(p, key, v)
    return p


@pytest.mark.parametrize("kw", [
    dict(X=None), dict(dt=7), dict(n=0), dict(d=300), dict(k=0), dict(k=200),
    dict(max_iters=0), dict(tol=1.5), dict(C_out=None), dict(labels_out=None),
])
def test_fit_batched_rejects_invalid(L, kw):
    arr = (knor.Problem * 3)(_problem(), _problem(**kw), _problem())
    assert L.knor_fit_batched(arr, 3, None, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_fit_batched(None, 2, None, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_fit_batched(arr, -1, None, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_fit_batched(None, 0, None, None) == knor.KNOR_OK


@pytest.mark.parametrize("field,value", [("tile_blocks", 3), ("tile_resident", 3),
                                         ("autotune", 2)])
def test_tile_options_validated(L, field, value):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    setattr(o, field, value)
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    arr = (knor.Problem * 1)(_problem())
    assert L.knor_fit_batched(arr, 1, ctypes.byref(o), None) == knor.KNOR_ERR_INVALID_ARG


def test_fit_batched_rejects_per_call_arrays(L):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    o.label_history = 0x1000
    arr = (knor.Problem * 1)(_problem())
    assert L.knor_fit_batched(arr, 1, ctypes.byref(o), None) == knor.KNOR_ERR_INVALID_ARG


def test_mlp_entry_points_validate(L):
    P = ctypes.c_void_p(0x1000)
    assert L.knor_mlp_param_count(32, 256, 4096) == 1126912
    for bad in [(0, 256, 10), (300, 256, 10), (8, 100, 10), (8, 32, 0), (8, 32, 20000)]:
        assert L.knor_mlp_param_count(*bad) == -1
        assert L.knor_mlp_init(P, *bad, 0, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_init(None, 8, 32, 10, 0, None) == knor.KNOR_ERR_INVALID_ARG
    # train step: missing arrays, batch 0, negative lr, Adam without state
    assert L.knor_mlp_train_step(P, P, P, 1, 8, 32, 10, None, P, 4, 1e-3, None, None,
                                 None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_train_step(P, P, P, 1, 8, 32, 10, P, P, 0, 1e-3, None, None,
                                 None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_train_step(P, P, P, 1, 8, 32, 10, P, P, 4, -1.0, None, None,
                                 None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_train_step(P, None, P, 1, 8, 32, 10, P, P, 4, 1e-3, None, None,
                                 None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_train_step(P, P, P, 0, 8, 32, 10, P, P, 4, 1e-3, None, None,
                                 None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_propose(P, 8, 32, 10, P, -1, P, None) == knor.KNOR_ERR_INVALID_ARG
    assert L.knor_mlp_propose(P, 8, 32, 10, P, 0, P, None) == knor.KNOR_OK
    assert L.knor_mlp_propose(None, 8, 32, 10, P, 5, P, None) == knor.KNOR_ERR_INVALID_ARG


def test_learned_needs_valid_options(L):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    for field, value in (("learned", 2), ("train_iters", -1), ("train_batches", -3)):
        setattr(o, field, value)
        assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
        setattr(o, field, 0)


def _opts_update(v):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    o.update = v
    return o


@pytest.mark.parametrize("v", [-1, 2])
def test_update_option_validated(L, v):
    o = _opts_update(v)
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    P = FAKE
    assert L.knor_update(P, 1, 10, 4, P, 2, P, ctypes.byref(o), P, None) == \
        knor.KNOR_ERR_INVALID_ARG
    arr = (knor.Problem * 1)(_problem())
    assert L.knor_fit_batched(arr, 1, ctypes.byref(o), None) == knor.KNOR_ERR_INVALID_ARG


def test_exact_update_rejects_f64_points(L):
    # the exact mean covers FP32 and BF16 points; FP64 is refused before any
    # device work (the pointers are never dereferenced)
    o = _opts_update(1)
    assert _fit(L, dt=0, opts=ctypes.byref(o)) == knor.KNOR_ERR_UNSUPPORTED
    P = FAKE
    assert L.knor_update(P, 0, 10, 4, P, 2, P, ctypes.byref(o), P, None) == \
        knor.KNOR_ERR_UNSUPPORTED
    arr = (knor.Problem * 2)(_problem(), _problem(dt=0))
    assert L.knor_fit_batched(arr, 2, ctypes.byref(o), None) == knor.KNOR_ERR_UNSUPPORTED


def test_binding_update_names():
    with pytest.raises(ValueError):
        knor._update_code("sorted")
    assert knor._update_code("canonical") == 0 and knor._update_code("exact") == 1


@pytest.mark.parametrize("field", ["centroid_history", "objective_history"])
def test_fit_batched_rejects_histories(L, field):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    setattr(o, field, 0x1000)
    arr = (knor.Problem * 1)(_problem())
    assert L.knor_fit_batched(arr, 1, ctypes.byref(o), None) == knor.KNOR_ERR_INVALID_ARG


def test_binding_init_names():
    assert knor.INITS == {"given": 0, "forgy": 1, "shuffle_first_k": 2, "kmeans++": 3}


def test_clause2_option_validated(L):
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    o.clause2 = 3
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG
    o.clause2 = 2                      # FP64 points: not served by the tile
    assert _fit(L, dt=0, opts=ctypes.byref(o)) == knor.KNOR_ERR_UNSUPPORTED
    o.prune = 0                        # needs MTI
    assert _fit(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_UNSUPPORTED
    o.prune = 1
    assert _fit(L, k=9000, n=20000, opts=ctypes.byref(o)) == knor.KNOR_ERR_UNSUPPORTED
    arr = (knor.Problem * 1)(_problem(dt=2))
    assert L.knor_fit_batched(arr, 1, ctypes.byref(o), None) == knor.KNOR_ERR_UNSUPPORTED


def _fit_streamed(L, opts=None, sopts=None, **kw):
    a = dict(X=FAKE, dt=1, n=100, d=8, k=4, init=0, C=FAKE, it=10, tol=0.0,
             Cout=FAKE, lab=FAKE, st=None)
    a.update(kw)
    return L.knor_fit_streamed(a["X"], a["dt"], a["n"], a["d"], a["k"], a["init"], a["C"],
                               a["it"], a["tol"], opts, sopts, a["Cout"], a["lab"], a["st"])


def _exact_opts():
    o = knor.Opts()
    o.struct_size = ctypes.sizeof(knor.Opts)
    o.prune = 1
    o.recheck = 1
    o.check_numeric = 1
    o.update = 1
    return o


@pytest.mark.parametrize("kw", [
    dict(X=None), dict(dt=0), dict(dt=9), dict(n=0), dict(d=0), dict(d=257), dict(k=0),
    dict(k=101), dict(it=0), dict(tol=1.0), dict(init=0, C=None), dict(init=4),
    dict(Cout=None), dict(lab=None), dict(n=1 << 31),
])
def test_fit_streamed_rejects_invalid(L, kw):
    o = _exact_opts()
    assert _fit_streamed(L, opts=ctypes.byref(o), **kw) == knor.KNOR_ERR_INVALID_ARG


def test_fit_streamed_rejects_bad_stream_opts(L):
    o = _exact_opts()
    for field, v in [("struct_size", 5), ("batch_rows", -1), ("cache_rows", -2),
                     ("cache_interval", -1), ("skip_objective", 2)]:
        so = knor.StreamOpts()
        so.struct_size = ctypes.sizeof(knor.StreamOpts)
        setattr(so, field, v)
        assert _fit_streamed(L, opts=ctypes.byref(o), sopts=ctypes.byref(so)) == \
            knor.KNOR_ERR_INVALID_ARG, field


def test_fit_streamed_unsupported_options(L):
    # the canonical update (the default), the learned proposal, forced
    # Clause 2, autotuning and k-means++ are not offered for host rows
    assert _fit_streamed(L) == knor.KNOR_ERR_UNSUPPORTED
    for field, v in [("update", 0), ("learned", 1), ("clause2", 2), ("autotune", 1),
                     ("objective_history", 0x1000)]:
        o = _exact_opts()
        setattr(o, field, v)
        assert _fit_streamed(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_UNSUPPORTED, field
    o = _exact_opts()
    assert _fit_streamed(L, opts=ctypes.byref(o), init=3, C=None) == knor.KNOR_ERR_UNSUPPORTED


def test_fit_streamed_needs_pinned_host_rows(L):
    # a pointer that is not page-locked host memory is refused
    o = _exact_opts()
    assert _fit_streamed(L, opts=ctypes.byref(o)) == knor.KNOR_ERR_INVALID_ARG


def test_binding_streamed_refuses_unpinned():
    import torch
    with pytest.raises(ValueError):
        knor.fit_streamed(torch.zeros((10, 4)), 2, C0=torch.zeros((2, 4), dtype=torch.float64))
