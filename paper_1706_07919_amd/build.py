"""Build the HIP library ``libbem.so`` in-tree for gfx950.

    python -m paper_1706_07919_amd.build          # or build() from Python

Device code is compiled with packed-FP32 instruction selection disabled.  The
host-only geometry code is compiled without floating-point contraction so that
the mesh builder is reproducible bit for bit.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libbem.so")
OBJ = os.path.join(HERE, "_build")

HIP_SOURCES = ["operator.hip", "lu.hip", "ir.hip", "field.hip", "synth.hip", "mlp.hip", "quad.hip",
               "chief.hip", "api.cpp"]
HOST_SOURCES = ["mesh.cpp", "pulse.cpp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    dev_flags = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={arch}",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Wno-unused-result"]
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(OBJ, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        jobs.append([hipcc, *dev_flags, *inc, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HOST_SOURCES:
        obj = os.path.join(OBJ, src + ".o")
        jobs.append(["g++", "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", *inc, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [os.path.join(OBJ, s + ".o") for s in HIP_SOURCES + HOST_SOURCES]
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={arch}", *objs, "-L/opt/rocm/lib",
          "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
