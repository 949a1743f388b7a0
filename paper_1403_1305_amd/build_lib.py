"""Compile libac.so in-tree for gfx950 with hipcc (host builder with g++).

    python -m paper_1403_1305_amd.build_lib
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libac.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # no packed-FP32 instructions anywhere in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", f"-I{ROOT}/include"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", f"-I{ROOT}/include"]

HIP_SOURCES = ["dfa_place_hot.hip", "dfa_place_hot_k2.hip", "dfa_place_hot_k3.hip", "dfa_place_hot_k4.hip",
               "dfa_batch_hot_k2.hip", "dfa_batch_hot_k3.hip", "dfa_batch_hot_k4.hip", "dfa_place_hot_pair.hip", "dfa_place_full.hip", "dfa_place_global.hip", "dfa_batch_hot.hip",
               "dfa_batch_global.hip", "dfa.hip", "batch.hip", "serve.hip",
               "scan.hip", "gate.hip", "qgate.hip", "measure.hip", "api.hip"]
CXX_SOURCES = ["machine.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def _stale(src: str, out: str) -> bool:
    """True unless `out` is newer than `src` and every header it may include."""
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "ac.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (only the stale ones with `incremental`) and link."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        out = os.path.join(OBJ, src + ".o")
        jobs.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", out], out, src))
    for src in CXX_SOURCES:
        out = os.path.join(OBJ, src + ".o")
        jobs.append((["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", out], out, src))
    todo = [j for j in jobs if not incremental or _stale(os.path.join(CSRC, j[2]), j[1])]
    with cf.ThreadPoolExecutor(max_workers=max(1, len(todo))) as ex:
        logs = list(ex.map(lambda j: _run(j[0]), todo))
    if verbose:
        for log in logs:
            if log.strip():
                print(log, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
          *[o for _, o, _ in jobs]])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
