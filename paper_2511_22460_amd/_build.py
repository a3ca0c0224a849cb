"""Build libebr.so (the C-ABI library) in-tree with hipcc for gfx950.

Every source is compiled to an object of its own, in parallel (the fused scoring kernel is
compiled once per embedding width), then linked. Importable without torch; used by
__graft_entry__.build() and by the binding when no built library is present.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libebr.so")
OBJ = os.path.join(PKG, "_build")
WIDTHS = (16, 32, 48, 64, 80, 96, 112, 128)
SOURCES = ["api.cpp", "codec.cpp", "quant.cpp", "server.cpp", "kernels.hip", "noalloc.hip", "build.hip"] + \
          [f"score_d{d}.hip" for d in WIDTHS]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(extra=()) -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC,
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *extra]


def compile_cmd(src: str, obj: str, extra=()) -> list:
    return [hipcc(), *flags(extra), "-c", os.path.join(CSRC, src), "-o", obj]


def link_cmd(objs, out: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out]


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    tag = "%d" % os.getpid()

    def one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + f".{tag}.o")
        r = subprocess.run(compile_cmd(src, obj), capture_output=True, text=True)
        return src, obj, r

    objs = []
    # the slowest units first
    order = sorted(SOURCES, key=lambda s: (not s.endswith(".hip"), s))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(one, order))
    errs = [(s, r) for s, _, r in results if r.returncode != 0]
    if errs:
        raise RuntimeError("libebr build failed:\n" +
                           "\n".join(f"--- {s}\n{r.stdout}{r.stderr}" for s, r in errs))
    for s, obj, r in results:
        objs.append(obj)
        if verbose and r.stderr:
            print(f"--- {s}\n{r.stderr}")
    tmp = LIB + ".tmp" + tag
    r = subprocess.run(link_cmd(objs, tmp), capture_output=True, text=True)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    if r.returncode != 0:
        raise RuntimeError("libebr link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
