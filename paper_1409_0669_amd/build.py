"""Build ``libbwla.so``: the gfx950 HIP kernels and the C ABI, compiled in-tree
with hipcc (cross-compiles without a GPU).

Each kernel source is compiled once per storage type (f64, f32, bf16) so the
objects build in parallel; the API layer is compiled once; everything is linked
into one shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbwla.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

KERNEL_SOURCES = ("stream.hip", "reduce.hip", "gemv.hip", "ger.hip", "batched.hip", "strided.hip")
TYPES = {"f64": "double", "f32": "float", "bf16": "__bf16"}

COMMON_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # bitwise reproducible elementwise results need the rounding sequence as
    # written: no contraction of a*b+c into an fma behind the source's back
    "-ffp-contract=off",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (p.returncode, " ".join(cmd), out))
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    tasks = []
    for src in KERNEL_SOURCES:
        for tname, ctype in TYPES.items():
            obj = os.path.join(OBJDIR, f"{src[:-4]}_{tname}.o")
            cmd = [HIPCC, *COMMON_FLAGS, f"-DBWLA_T={ctype}",
                   f"-DBWLA_T_IS_F64={1 if tname == 'f64' else 0}",
                   "-c", os.path.join(CSRC, src), "-o", obj]
            tasks.append((obj, cmd))
    api_obj = os.path.join(OBJDIR, "api.o")
    tasks.append((api_obj, [HIPCC, *COMMON_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, "api.cpp"),
                            "-o", api_obj]))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(lambda t: _run(t[1]), tasks))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[t[0] for t in tasks]])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
