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


# Host AddressSanitizer + UndefinedBehaviorSanitizer on the API layer (argument
# validation, workspace sizing, configuration tables, plan building): each
# sanitizer flag goes to the host pass only, the kernels are the ordinary
# objects.  The library leaves the sanitizer runtime's symbols undefined; a
# process loads it with that runtime preloaded (SANITIZER_RUNTIME).
ROCM_ROOT = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
SANITIZER_RUNTIME = os.path.join(ROCM_ROOT, "llvm", "lib", "clang")


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that hipcc's host pass
    targets (it carries the UndefinedBehaviorSanitizer handlers too)."""
    for ver in sorted(os.listdir(SANITIZER_RUNTIME), reverse=True):
        p = os.path.join(SANITIZER_RUNTIME, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("no libclang_rt.asan-x86_64.so under " + SANITIZER_RUNTIME)


def build_sanitized(out_path: str) -> str:
    """Builds a copy of the library whose API layer carries host ASan/UBSan
    checks at ``out_path``; the kernel objects are those of build()."""
    objs = [os.path.join(OBJDIR, f"{src[:-4]}_{t}.o") for src in KERNEL_SOURCES for t in TYPES]
    if not all(os.path.exists(o) for o in objs):
        build()
    api_obj = out_path + ".api.o"
    _run([HIPCC, *COMMON_FLAGS, "-O1", "-g",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
          "-x", "hip", "-c", os.path.join(CSRC, "api.cpp"), "-o", api_obj])
    rocm_lib = os.path.join(ROCM_ROOT, "lib")
    _run([os.path.join(ROCM_ROOT, "llvm", "bin", "clang++"), "-shared", "-fPIC", "-o", out_path, api_obj, *objs,
          "-L" + rocm_lib, "-lamdhip64", "-Wl,-rpath," + rocm_lib])
    return out_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
