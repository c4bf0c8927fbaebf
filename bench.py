#!/usr/bin/env python3
"""Benchmark of the k-means hot path on one MI355X: one JSON line.

One step = one complete fit (every Lloyd iteration until no label changes or
max_iters) of the selected workload, inputs resident in HBM.  value = Lloyd
iterations per second over the timed steps.

Workloads (--config, seeded synthetic Gaussian mixtures, see workloads/):
  5 (default, the largest single-GPU configuration): learned candidate
    proposal, n=1e7, d=32, k=4096, FP32, 40 iterations, MTI + MLP
    32-256-256-4096 trained on the labels of MTI iterations 1-5, top-16
    candidates, certificate, MTI scan for the rest;
  1: plain Lloyd's, FP64, n=1e4, d=16, k=10, 50 iterations;
  2: MTI, FP32, n=1e6, d=32, k=100, k-means++ seeding, 100 iterations;
  3: mixed precision, BF16 points, n=2e7, d=64, k=256, 30 iterations;
  4: 64 batched restarts (uneven n, d, k), FP32, 50 iterations each.

--streamed (configs 2, 3, 5): the same workload with its points in pinned host
memory (knor_fit_streamed, exact update); the line adds the host-link
accounting (rows copied whole, gathered one by one, served by the row cache,
admitted to it, bytes, rates) and the in-HBM exact fit's rate.

Every line also reports, measured in the same run:
  baselines     the same workload on this GPU without the form (plain FP32
                Lloyd's; for 3 and 5 also FP32 + MTI; for 4 sequential fits
                with the same options), with the speedups
  roofline      for the kernel group with the largest GPU time, from HIP
                events on the launch stream over the timed steps
  exact         labels of a row sample at every iteration equal the FP64
                oracle's assignment under that iteration's centroids, and the
                centroids of the first and last update equal the oracle's
                update of all rows (per-iteration centroids come from the
                fit's centroid history)
  cpu_baseline  the FP64 oracle timed on this host (whole fit for 1 and 2,
                else one iteration's assignment of a row sample, scaled)
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12      # MI355X dense FP32 matrix, FLOP/s
PEAK_BF16_MFMA = 2516.6e12
PEAK_HBM = 8.0e12              # bytes/s
PEAK_FP64_VALU = 78.6e12

# HBM bytes per launch of a kernel group on one workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs (medians over launches), each scaled by what
# the counter reads for a 2 GiB device copy (fetch x2.0, write x1.0).  A
# figure is reported only for its workload and only while the kernel sources
# it was measured on are unchanged.
MEASURED_TRAFFIC = {
    # the Clause-2 group: grouping (count, column scan, tasks, scatter), sort
    # pass and persistent tile (medians over 78 launches; fetch 26872.5 + 2121.0 + 11.1 +
    # 35890.5 + 232409.2 + 269945.2 KiB, x2 by the copy
    # calibration; write 4096.0 + 4112.0 + 36.0 + 73699.1 + 15057.8 +
    # 117503.2 KiB)
    (5, "assign_list"): {
        "bytes": (2 * (26872.5 + 2121.0 + 11.1 + 35890.5 + 232409.2 + 269945.2) +
                  (4096.0 + 4112.0 + 36.0 + 73699.1 + 15057.8 + 117503.2)) * 1024,
        "sources": {
            "tile_cand.hip": "33134145ac7c2e98d78b6d23ac50b7ea8e845985d1619ff55ecf8185b92ac963",
            "tile_f32.h": "4d4931263f7e8e9204b2ce22f0239481b0adcf71b0ce66e01e2e60c1020c482d",
            "tile_common.h": "66c8fecd8cd91705c6d3c0012eff17d6a12ef5dd3a53a3b8a7c82ec76ec33cca",
            "common.h": "1ea23988c276bf76d5a82e60bfdc7ba13bc26b76aeece46aaeb95bd9033c67a1",
        },
    },
    # the survivor tile (median over 200 launches; fetch 23664.3 KiB x2,
    # write 7153.4 KiB)
    (2, "assign_list"): {
        "bytes": (2 * 23664.3 + 7153.4) * 1024,
        "sources": {
            "tile_f32.hip": "5fac685a160eca932c038b1b3a5e9a2cddee25145289a5578c06fd29f7e6e20b",
            "tile_f32.h": "4d4931263f7e8e9204b2ce22f0239481b0adcf71b0ce66e01e2e60c1020c482d",
            "tile_common.h": "66c8fecd8cd91705c6d3c0012eff17d6a12ef5dd3a53a3b8a7c82ec76ec33cca",
            "recheck.h": "cdd421f2b40c729a29f70a8c818d95f62f97c9fad5a0e4854d07f66baacaf0ad",
            "common.h": "1ea23988c276bf76d5a82e60bfdc7ba13bc26b76aeece46aaeb95bd9033c67a1",
        },
    },
}

# iterations whose dominant-group launches are timed inside the timed region:
# every 10th where launches take tens of microseconds (the events stay out of
# the way), every one on the large-k workload, whose launches take
# milliseconds (the mean then covers the same launches as a kernel trace)
PROFILE_EVERY = 10
PROFILE_EVERY_BY_CONFIG = {5: 1}

METRIC = ("Lloyd iters/s and point·centroid dists/s (% MFMA peak) "
          "at exact assignments")

WORKLOAD_NAMES = {
    1: "plain Lloyd's: n=1e4 d=16 k=10 f64 Gaussian mixture (10 comps), first k of a "
       "seeded shuffle, 50 iters, tol=0",
    2: "MTI: n=1e6 d=32 k=100 f32 Gaussian mixture (100 comps, Dirichlet weights), "
       "k-means++ seeding, 100 iters, tol=0",
    3: "mixed precision: n=2e7 d=64 k=256 bf16 points, 95% mixture (256 comps) + 5% "
       "uniform outliers, k random rows, 30 iters, MTI, BF16 MFMA + FP64 recheck",
    4: "batched restarts: 64 instances, n log-uniform in [1e4, 2e6], d in {8,16,32,64}, "
       "k in 8..512, f32, k random rows, 50 iters each, MTI, tuned tile schedules",
    5: "learned proposal: n=1e7 d=32 k=4096 f32 Gaussian mixture (4096 comps, "
       "mu~N(0,100I), sigma~U[0.5,3]), k random rows, 40 iters, MTI + MLP "
       "32-256-256-4096 (BF16 operands, FP32 sums) trained on the labels of MTI "
       "iterations 1-5, top-16 candidates, certificate, MTI scan otherwise",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--update", default=None, choices=["canonical", "exact"],
                    help="centroid update of the measured fits and their baselines: the exact "
                         "member mean, moving only changed points (default for FP32 and BF16 "
                         "points), or the canonical leaf(64) + pairwise tree sums (default, and "
                         "the only rule, for FP64 points: --config 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the oracle comparison (profiling runs)")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the comparison fits (profiling runs)")
    ap.add_argument("--exact-rows", type=int, default=20000,
                    help="rows whose labels are compared with the oracle per iteration")
    ap.add_argument("--streamed", action="store_true",
                    help="the points stay in pinned host memory (knor_fit_streamed, "
                         "exact update); configs 2, 3 and 5")
    ap.add_argument("--batch-rows", type=int, default=0,
                    help="streamed: rows per batch (0 = library default, 2^22)")
    ap.add_argument("--cache-rows", type=int, default=1 << 22,
                    help="streamed: row cache capacity in rows")
    ap.add_argument("--cache-interval", type=int, default=5,
                    help="streamed: first refresh iteration of the row cache")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB "
                         "before the timed region (a known-size kernel for "
                         "scaling HBM byte counters)")
    a = ap.parse_args()
    if a.update is None:
        a.update = "canonical" if a.config == 1 else "exact"
    return a


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic work of the kernel groups
# ---------------------------------------------------------------------------

MLP_H = 256
MLP_BATCH = 4096


def group_work(g, w, sx, ctr, iters, its, train_iters=5, train_batches=16):
    """Algorithmic work of kernel group g summed over the iterations `its` of
    one fit, and the group's launches among them: (amount, launches, unit,
    bound, peak).  ctr: per-iteration counters (iters x 9)."""
    n, d, k = w.n, w.d, w.k
    its = [t for t in its if t < iters]
    after0 = [t for t in its if t >= 1]
    mfma_peak = PEAK_BF16_MFMA if w.dtype == "bf16" else PEAK_FP32_MFMA
    if g == 0:     # dense tile: 2 d flops per point-centroid pair
        at0 = [t for t in its if t == 0]
        return (2.0 * d * k * sum(int(ctr[t, 1]) for t in at0), len(at0),
                "TFLOP/s", "mfma", mfma_peak)
    if g == 1:     # survivor tile: all k per survivor, or with Clause 2 per block
        # (FP32, 1024 <= k <= 8192) the survivor-candidate pairs it evaluated
        # (the dists counter less the Clause-3 tightening distances)
        if w.dtype == "f32" and 1024 <= k <= 8192:
            pairs = sum(int(ctr[t, 7]) - (n - int(ctr[t, 2])) for t in after0)
            return 2.0 * d * pairs, len(after0), "TFLOP/s", "mfma", mfma_peak
        return (2.0 * d * k * sum(int(ctr[t, 1]) for t in after0), len(after0),
                "TFLOP/s", "mfma", mfma_peak)
    if g == 2:     # FP64 recheck: subtract, multiply, add per (point, centroid, dim)
        rech = sum(int(ctr[t, 4]) for t in its)
        return 3.0 * d * k * rech, len(its), "TFLOP/s", "alu", PEAK_FP64_VALU
    if g == 3:     # filter: label, bound in/out, survivor index; rows tightened
        tot = 0.0
        for t in after0:
            pa = int(ctr[t, 2])
            tot += 12.0 * n + (n - pa) * (d * sx) + 4.0 * int(ctr[t, 1])
        return tot, len(after0), "GB/s", "hbm", PEAK_HBM
    if g == 4:     # sort: labels read twice, perm written, block counts
        return (12.0 * n) * len(its), len(its), "GB/s", "hbm", PEAK_HBM
    if g == 5:     # leaf sums: every row gathered once + perm + leaf sums out
        per_iter = n * d * sx + 4.0 * n + (n / 64.0 + k) * d * 8.0
        return per_iter * len(its), len(its), "GB/s", "hbm", PEAK_HBM
    if g == 8:     # MLP on the BF16 matrix cores: forward of every row that went
        # through the network (a point's candidates are computed once per fit),
        # and training (forward + two backward products ~ 3x forward per row)
        fwd = 2.0 * (d * MLP_H + MLP_H * MLP_H + MLP_H * k)
        tot, launches = 0.0, 0
        for t in its:
            q = int(ctr[t, 8])
            tot += fwd * q
            if 1 <= t <= train_iters:
                tot += 3.0 * fwd * MLP_BATCH * train_batches
            if q or 1 <= t <= train_iters:
                launches += 1
        return tot, launches, "TFLOP/s", "mfma", PEAK_BF16_MFMA
    return None


def roofline(knor, g, ms, la, work, traffic, fits=1):
    """Roofline entry of group g: its algorithmic work over the GPU time the
    HIP events measured (ms, la: summed over `fits` fits, each timed over the
    iterations `work` covers), i.e. work per launch / mean launch time."""
    if work is None or not la[g] or ms[g] <= 0.0:
        return None
    amount, launches, unit, bound, peak = work
    ach = amount * fits / (ms[g] / 1e3)
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    return {"kernel": knor.PROF_GROUPS[g], "bound": bound,
            "achieved": round(ach / scale, 3), "peak": round(peak / scale, 1),
            "unit": unit, "frac": round(ach / peak, 4),
            "traffic": traffic, "us_per_launch": round(ms[g] / la[g] * 1e3, 3),
            "work_per_launch": amount * fits / la[g]}


def measured_traffic(cfg, group):
    import hashlib
    m = MEASURED_TRAFFIC.get((cfg, group))
    if m is None:
        return None
    csrc = os.path.join(ROOT, "paper_1606_08905_amd", "csrc")
    for fname, digest in m["sources"].items():
        with open(os.path.join(csrc, fname), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return m["bytes"]


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------

def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return outs, (time.perf_counter() - t) / steps


def measure(knor, fit, steps, warmup, every=PROFILE_EVERY):
    """Warm-up fits, one untimed calibration fit with every kernel group under
    HIP events (the breakdown, and which group dominates), then `steps` timed
    fits in which the dominant group's launches of every `every`-th iteration
    are bracketed by events."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fit()
    torch.cuda.synchronize()
    cal_ms = np.zeros(knor.NPROF)
    cal_n = np.zeros(knor.NPROF, np.int64)
    fit(profile=(cal_ms, cal_n))
    g = int(np.argmax(cal_ms))
    ms = np.zeros(knor.NPROF)
    la = np.zeros(knor.NPROF, np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [fit(profile=(ms, la, 1 << g, every)) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(o[2]["iters"] for o in outs)
    log(f"timed {steps} fits in {dt:.3f}s ({iters} iterations)")
    return dict(outs=outs, sec=dt, iters=iters, value=iters / dt, g=g, ms=ms, la=la,
                cal_ms=cal_ms, cal_n=cal_n)


def kernels_table(knor, m):
    out = {}
    for i, nm in enumerate(knor.PROF_GROUPS):
        if m["cal_n"][i]:
            out[nm] = {"ms_per_fit": round(float(m["cal_ms"][i]), 4),
                       "launches": int(m["cal_n"][i]),
                       "us_per_launch": round(1e3 * m["cal_ms"][i] / m["cal_n"][i], 3)}
    return out


def rate(fit, steps, warmup):
    outs, dt = timed(fit, steps, warmup)
    return outs[-1], outs[-1][2]["iters"] / dt


# ---------------------------------------------------------------------------
# exactness and the CPU baseline
# ---------------------------------------------------------------------------

def check_exact(oracle, workloads, w, fit, nrows, update="canonical", seed=0):
    """One more fit with label and centroid histories: at every iteration the
    labels of `nrows` random rows equal the oracle's assignment under that
    iteration's centroids; the first and the last update equal the oracle's
    update of all rows."""
    import numpy as np
    C, lab, st = fit(history=True, centroid_history=True)
    iters = st["iters"]
    H = st["label_history"]
    CH = st["centroid_history"].cpu().numpy()
    rng = np.random.default_rng(seed)
    m = min(nrows, w.n)
    rows = np.sort(rng.choice(w.n, size=m, replace=False))
    import torch
    Hs = H[:, torch.from_numpy(rows).to(H.device)].cpu().numpy()
    Xs = workloads.to_f64(w.X[rows], w.dtype)
    t0 = time.perf_counter()
    labels_ok = True
    for t in range(iters):
        lo, _ = oracle.assign(Xs, CH[t])
        if not (lo == Hs[t]).all():
            labels_ok = False
            log(f"exact: labels differ at iteration {t}")
            break
    upd = oracle.update_exact if update == "exact" else oracle.update
    X64 = w.x64()
    upd_ok = True
    for t in sorted({0, iters - 1}):
        Ht = H[t].cpu().numpy()
        Co, _ = upd(X64, Ht, CH[t])
        nxt = CH[t + 1] if t + 1 < iters else C.cpu().numpy()
        if not (Co == nxt).all():
            upd_ok = False
            log(f"exact: centroids differ after iteration {t}")
    del X64
    log(f"exactness check in {time.perf_counter() - t0:.1f}s")
    return {"exact": bool(labels_ok and upd_ok),
            "exact_check": f"labels of {m} random rows at each of {iters} iterations vs the "
                           f"FP64 oracle's assignment under that iteration's centroids; "
                           f"centroids of updates {sorted({0, iters - 1})} vs the oracle's "
                           f"update of all {w.n} rows"}


def host_info():
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            key, _, val = line.partition(":")
            key = key.strip()
            if key in ("Model name", "Socket(s)", "Core(s) per socket",
                       "Thread(s) per core", "CPU(s)"):
                info[key] = val.strip()
    except Exception:
        pass
    info["affinity"] = len(os.sched_getaffinity(0))
    info["OMP_NUM_THREADS"] = os.environ.get("OMP_NUM_THREADS")
    return info


def cpu_whole_fit(oracle, w, mti, update="canonical"):
    """The oracle's whole fit on the same workload and C0 (all threads, then
    one thread): iterations per second each."""
    X64 = w.x64()

    def run():
        t = time.perf_counter()
        if mti:
            r = oracle.mti_fit(X64, w.C0, w.max_iters, tol=w.tol, history=False,
                               objective=False, exact_mean=update == "exact")
        else:
            r = oracle.fit(X64, w.C0, w.max_iters, tol=w.tol, history=False, objective=False)
        return r.iters / (time.perf_counter() - t), r.iters

    nt = oracle.num_threads()
    v, iters = run()
    oracle.set_threads(1)
    v1, _ = run()
    oracle.set_threads(nt)
    return {"value": round(v, 4), "unit": "iters/s", "cores": nt, "kind": "oracle",
            "sample": f"FP64 {'MTI ' if mti else ''}oracle, same workload and C0, "
                      f"{iters} iterations (whole fit)",
            "one_thread": {"value": round(v1, 4), "unit": "iters/s", "cores": 1},
            "host": host_info()}


def cpu_sample(oracle, workloads, w, C0, rows_frac, seed=0):
    """The oracle's assignment of a random row sample at C0 (one iteration's
    dominant work), timed and scaled to n."""
    import numpy as np
    rng = np.random.default_rng(seed)
    m = max(1000, int(rows_frac * w.n))
    rows = np.sort(rng.choice(w.n, size=m, replace=False))
    Xs = workloads.to_f64(w.X[rows], w.dtype)
    t = time.perf_counter()
    oracle.assign(Xs, C0)
    dt = time.perf_counter() - t
    return {"value": round(m / (dt * w.n), 5), "unit": "iters/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle assignment of {m} random rows at C0 (one iteration's "
                      f"assignment, {dt:.1f}s), scaled to n={w.n}",
            "host": host_info()}


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def device_points(w):
    import numpy as np
    import torch
    if w.dtype == "bf16":
        return torch.from_numpy(w.X.view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(w.X).cuda()


def single_config(a, knor, oracle, workloads):
    import torch
    cfg = a.config
    t_gen = time.perf_counter()
    w = workloads.config(cfg)
    log(f"data n={w.n} d={w.d} k={w.k} {w.dtype} generated in "
        f"{time.perf_counter() - t_gen:.1f}s")
    X = device_points(w)
    C0 = torch.from_numpy(w.C0).cuda()
    torch.cuda.synchronize()
    form = {1: {"prune": False}, 2: {"prune": True}, 3: {"prune": True},
            5: {"prune": True, "learned": True}}[cfg]

    def fit(Xt=X, **kw):
        opts = dict(form)
        opts.update(kw)
        return knor.fit(Xt, w.k, C0=C0, max_iters=w.max_iters, tol=w.tol, counters=True,
                        update=a.update, **opts)

    every = PROFILE_EVERY_BY_CONFIG.get(cfg, PROFILE_EVERY)
    m = measure(knor, fit, a.steps, a.warmup, every)
    st = m["outs"][-1][2]
    ctr, iters = st["counters"], st["iters"]
    sx = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    sampled = [t for t in range(iters) if t % every == 0]
    g = m["g"]
    work = group_work(g, w, sx, ctr, iters, sampled)
    out = {
        "metric": METRIC, "value": round(m["value"], 3), "unit": "iters/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * m["sec"] / a.steps, 3),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": w.dtype, "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[cfg] +
                   (", update=exact" if a.update == "exact" else ""),
                   "n": w.n, "d": w.d, "k": w.k, "iters_per_fit": iters},
        "eff_dists_per_s": m["iters"] * w.n * w.k / m["sec"],
        "computed_dists_per_s": sum(o[2]["dists_computed"] for o in m["outs"]) / m["sec"],
        "roofline": roofline(knor, g, m["ms"], m["la"], work,
                             measured_traffic(cfg, knor.PROF_GROUPS[g]), a.steps),
        "kernels": kernels_table(knor, m),
        "rechecked_per_fit": st["rechecked"],
    }
    if cfg == 5:
        out["certified_per_fit"] = st["certified"]
        out["mlp_queries_per_fit"] = st["mlp_queries"]
        out["mlp_forward_rows_per_fit"] = st["mlp_forward_rows"]
    if m["cal_n"][0] and cfg != 1:
        fl = group_work(0, w, sx, ctr, iters, [0])[0]
        sec = m["cal_ms"][0] / m["cal_n"][0] / 1e3
        peak = PEAK_BF16_MFMA if w.dtype == "bf16" else PEAK_FP32_MFMA
        out["dense_tile"] = {"tflops": round(fl / sec / 1e12, 2),
                             "frac_mfma_peak": round(fl / sec / peak, 4),
                             "us": round(sec * 1e6, 2)}
    # the same workload on this GPU without the form
    if not a.no_baselines and cfg != 1:
        base = {}
        (Cb, lb, sb), v = rate(lambda: fit(X if w.dtype != "bf16" else X.float(), prune=False,
                                           learned=False), max(1, a.steps - 1), 1)
        base["fp32_plain"] = {"value": round(v, 3), "unit": "iters/s",
                              "iters_per_fit": sb["iters"]}
        C, lab = m["outs"][-1][0], m["outs"][-1][1]
        same = bool((C == Cb).all() and (lab == lb).all())
        if cfg in (3, 5):
            Xf = X.float() if w.dtype == "bf16" else X
            (Cm, lm, sm), vm = rate(lambda: fit(Xf, prune=True, learned=False),
                                    max(1, a.steps - 1), 1)
            base["fp32_mti"] = {"value": round(vm, 3), "unit": "iters/s",
                                "iters_per_fit": sm["iters"]}
            same = same and bool((C == Cm).all() and (lab == lm).all())
        for key in base:
            base[key]["speedup"] = round(m["value"] / base[key]["value"], 3)
        out["baselines"] = base
        out["same_results_as_baselines"] = same
    if not a.no_exact:
        out.update(check_exact(oracle, workloads, w, fit, a.exact_rows, a.update))
    if not a.no_cpu_baseline:
        if cfg in (1, 2):
            out["cpu_baseline"] = cpu_whole_fit(oracle, w, mti=cfg == 2, update=a.update)
        else:
            out["cpu_baseline"] = cpu_sample(oracle, workloads, w, w.C0,
                                             {3: 0.1, 5: 0.3}[cfg])
    return out


# PCIe 5.0 x16, one direction (the MI355X host link)
PEAK_LINK = 64.0e9


def pinned_points(w):
    import numpy as np
    import torch
    if w.dtype == "bf16":
        t = torch.from_numpy(w.X.view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(w.X)
    return t.pin_memory()


def dma_rate(Xh):
    """Host-to-device copy rate of one whole pinned array (torch's copy, HIP
    events on its stream): the practical ceiling of the whole-batch copies."""
    import torch
    dst = torch.empty(Xh.shape, dtype=Xh.dtype, device="cuda")
    dst.copy_(Xh, non_blocking=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    dst.copy_(Xh, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    nbytes = Xh.numel() * Xh.element_size()
    del dst
    return nbytes / (a.elapsed_time(b) / 1e3)


def streamed_config(a, knor, oracle, workloads):
    """The same workload with the points in pinned host memory: a fit reads
    whole batches in its full passes and, afterwards, only the rows of the
    points that fail MTI Clause 1 (row cache first, then the host link)."""
    import numpy as np
    import torch
    cfg = a.config
    if cfg not in (2, 3, 5):
        raise SystemExit("--streamed takes --config 2, 3 or 5")
    t_gen = time.perf_counter()
    w = workloads.config(cfg)
    log(f"data n={w.n} d={w.d} k={w.k} {w.dtype} generated in "
        f"{time.perf_counter() - t_gen:.1f}s")
    Xh = pinned_points(w)
    C0 = torch.from_numpy(w.C0).cuda()
    sx = {"f32": 4, "bf16": 2}[w.dtype]
    rb = w.d * sx

    def fit(**kw):
        return knor.fit_streamed(Xh, w.k, C0=C0, max_iters=w.max_iters, tol=w.tol,
                                 counters=True, batch_rows=a.batch_rows,
                                 cache_rows=a.cache_rows, cache_interval=a.cache_interval,
                                 **kw)

    outs, dt = timed(fit, a.steps, a.warmup)
    C, lab, st = outs[-1]
    iters = st["iters"]
    io = st["io"]
    rows_moved = int(io[:, 0].sum() + io[:, 1].sum())
    link = {
        "rows_copied_per_fit": int(io[:, 0].sum()),
        "rows_gathered_per_fit": int(io[:, 1].sum()),
        "rows_cached_per_fit": int(io[:, 2].sum()),
        "rows_admitted_per_fit": int(io[:, 3].sum()),
        "bytes_per_fit": rows_moved * rb,
        "bytes_if_every_row_every_iteration": (iters + 1) * w.n * rb,
        "achieved_GBps": round(rows_moved * rb / dt / 1e9, 3),
        "dma_GBps": round(dma_rate(Xh) / 1e9, 3),
        "peak_GBps": PEAK_LINK / 1e9,
        "io_per_iteration": io.tolist(),
    }
    out = {
        "metric": METRIC, "value": round(iters / dt, 3), "unit": "iters/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": w.dtype, "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[cfg] + "; streamed: points in pinned host "
                   f"memory, batches of {a.batch_rows or 1 << 22} rows, row cache "
                   f"{a.cache_rows} rows, first refresh at iteration {a.cache_interval}, "
                   "update=exact", "n": w.n, "d": w.d, "k": w.k, "iters_per_fit": iters},
        "link": link,
    }
    # the same fit with the points resident in HBM
    if not a.no_baselines:
        X = device_points(w)
        (Cm, lm, sm), vm = rate(lambda: knor.fit(X, w.k, C0=C0, max_iters=w.max_iters,
                                                 tol=w.tol, update="exact", prune=True),
                                max(1, a.steps - 1), 1)
        out["in_hbm"] = {"value": round(vm, 3), "unit": "iters/s",
                         "ratio": round((iters / dt) / vm, 3)}
        out["same_results_as_in_hbm"] = bool((C == Cm).all() and (lab == lm).all()
                                             and sm["iters"] == iters)
        del X
    if not a.no_exact:
        out.update(check_exact(oracle, workloads, w, fit, a.exact_rows, "exact"))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_sample(oracle, workloads, w, w.C0,
                                         {2: 1.0, 3: 0.1, 5: 0.3}[cfg])
    return out


def batched_config(a, knor, oracle, workloads):
    import numpy as np
    import torch
    t_gen = time.perf_counter()
    ws = workloads.batched(64)
    log(f"64 instances, sum n={sum(w.n for w in ws)}, generated in "
        f"{time.perf_counter() - t_gen:.1f}s")
    probs = [dict(X=torch.from_numpy(w.X).cuda(), k=w.k, C0=torch.from_numpy(w.C0).cuda(),
                  max_iters=w.max_iters, tol=w.tol) for w in ws]
    res, dt = timed(lambda: knor.fit_batched(probs, update=a.update), a.steps, a.warmup)
    res = res[-1]
    iters = sum(r[2]["iters"] for r in res)
    out = {
        "metric": METRIC, "value": round(iters / dt, 3), "unit": "iters/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[4], "instances": 64,
                   "sum_n": int(sum(w.n for w in ws)), "iters_per_batch": iters},
        "eff_dists_per_s": sum(r[2]["iters"] * w.n * w.k for r, w in zip(res, ws)) / dt,
    }
    # the same batch recorded into one graph (knor_opts.batch_graph)
    resg, dtg = timed(lambda: knor.fit_batched(probs, update=a.update, graph=True),
                      a.steps, a.warmup)
    resg = resg[-1]
    out["graph"] = {"value": round(sum(r[2]["iters"] for r in resg) / dtg, 3),
                    "unit": "iters/s", "ms_per_batch": round(dtg * 1e3, 3),
                    "vs_worker_streams": round(dt / dtg, 3),
                    "same_results": all(bool((r[0] == q[0]).all() and (r[1] == q[1]).all())
                                        for r, q in zip(res, resg))}
    if not a.no_baselines:
        def seq(prune):
            return [knor.fit(p["X"], p["k"], C0=p["C0"], max_iters=p["max_iters"],
                             prune=prune, update=a.update) for p in probs]
        sm, dsm = timed(lambda: seq(True), 1, 0)
        sp, dsp = timed(lambda: seq(False), 1, 0)
        sm, sp = sm[-1], sp[-1]
        out["baselines"] = {
            "sequential_mti": {"value": round(iters / dsm, 3), "unit": "iters/s",
                               "speedup": round(dsm / dt, 3)},
            "sequential_fp32_plain": {"value": round(iters / dsp, 3), "unit": "iters/s",
                                      "speedup": round(dsp / dt, 3)}}
        out["same_results_as_baselines"] = all(
            bool((r[0] == q[0]).all() and (r[1] == q[1]).all() and (r[0] == u[0]).all())
            for r, q, u in zip(res, sm, sp))
    # roofline: the largest instance's dominant kernel group, under events
    il = max(range(len(ws)), key=lambda i: ws[i].n * ws[i].k * ws[i].d)
    wl = ws[il]
    ms = np.zeros(knor.NPROF)
    la = np.zeros(knor.NPROF, np.int64)
    _, _, stl = knor.fit(probs[il]["X"], wl.k, C0=probs[il]["C0"], max_iters=wl.max_iters,
                         counters=True, profile=(ms, la), update=a.update)
    g = int(np.argmax(ms))
    rl = roofline(knor, g, ms, la, group_work(g, wl, 4, stl["counters"], stl["iters"],
                                               range(stl["iters"])), None)
    if rl is not None:
        rl["instance"] = {"n": wl.n, "d": wl.d, "k": wl.k}
    out["roofline"] = rl
    if not a.no_exact:
        p = probs[il]
        fit = lambda **kw: knor.fit(p["X"], wl.k, C0=p["C0"], max_iters=wl.max_iters,
                                    update=a.update, **kw)
        ex = check_exact(oracle, workloads, wl, fit, a.exact_rows, a.update)
        ex["exact_check"] += " (largest instance)"
        out.update(ex)
    if not a.no_cpu_baseline:
        cb = cpu_sample(oracle, workloads, wl, wl.C0, 0.25)
        cb["sample"] += " (largest instance)"
        out["cpu_baseline"] = cb
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the sharding "
                                   "design is described in DESIGN.md",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import torch

    import oracle
    import paper_1606_08905_amd as knor
    import workloads

    knor.load()
    if a.copy_calibration_mib > 0:
        nel = a.copy_calibration_mib << 18            # float32 elements
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.streamed:
        out = streamed_config(a, knor, oracle, workloads)
    elif a.config == 4:
        out = batched_config(a, knor, oracle, workloads)
    else:
        out = single_config(a, knor, oracle, workloads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
