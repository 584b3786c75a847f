"""Compile libdqmc.so (HIP, gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled to an object file in parallel (the sweep kernels
sit in units of their own), then the objects are linked into paper_2106_00712_amd/libdqmc.so.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libdqmc.so")
OBJ_DIR = os.path.join(HERE, "_build")
HEADERS = [os.path.join(ROOT, "include", "dqmc.h"), os.path.join(ROOT, "include", "ising.h")]

# -packed-fp32-ops: keep the compiler from forming packed FP32 arithmetic (v_pk_*_f32).
HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.stderr


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source into paper_2106_00712_amd/libdqmc.so and return its path."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJ_DIR, os.path.basename(s)[:-4] + ".o") for s in srcs]
    inc = "-I" + os.path.join(ROOT, "include")
    cmds = [[hipcc(), *HIPCC_FLAGS, inc, "-c", "-o", o, s] for s, o in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        logs = list(ex.map(_run, cmds))
    tmp = LIB_PATH + ".tmp"
    logs.append(_run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]))
    if verbose:
        print("".join(logs))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
