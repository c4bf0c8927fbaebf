"""Compile the HIP sources of the library into libknor.so for gfx950.

Each source is compiled to an object of its own (in parallel), then the
objects are linked into one shared library.  The library's translation units
share no device functions, so separate compilation gives the same code as
one hipcc call over every source."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libknor.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # one rounding per operation in every FP64 step (no FMA contraction)
    "-ffp-contract=off",
    # never form packed FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


# per-source flags: keep the matrix-core accumulators in VGPRs (the
# epilogue reads every accumulator; from AGPRs each read is one more VALU
# instruction)
SOURCE_FLAGS = {
    "tile_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _jobs():
    n = os.cpu_count() or 4
    return max(1, min(8, n))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        extra = SOURCE_FLAGS.get(os.path.basename(src), [])
        cmd = [HIPCC, *FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, r

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, zip(srcs, objs)))
    failed = [(s, r) for s, r in results if r.returncode != 0]
    for s, r in results:
        msg = "\n".join(ln for ln in (r.stderr or "").splitlines()
                        if "packed-fp32-ops" not in ln)
        if msg.strip() and (verbose or r.returncode != 0):
            print(msg, flush=True)
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(os.path.basename(s)
                                                          for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
