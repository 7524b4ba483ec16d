"""Build the gfx950 HIP library libvp.so in-tree with hipcc.

Each source is compiled to an object of its own (in parallel, objects under
_build/), then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvp.so")
OBJ = os.path.join(ROOT, "_build", "vp")

ARCH = "--offload-arch=gfx950:xnack-"
HIPCC_FLAGS = [
    ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off (the compiler would form them from float2 code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(hipcc, src, verbose):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(hipcc, s, verbose), sources()))
    failed = False
    for src, obj, r in results:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if msg.strip():
            print(msg, flush=True)
        if r.returncode != 0:
            print(f"build failed: {src}", flush=True)
            failed = True
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, ARCH, "-shared", "-fPIC", "-o", tmp] + [obj for _, obj, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
