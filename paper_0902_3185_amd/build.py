"""Builds libdmrg.so in-tree with hipcc for gfx950.

    python -m paper_0902_3185_amd.build

Every HIP and C++ source under csrc/ is compiled (in parallel) to an object
file under csrc/_build/ and linked into paper_0902_3185_amd/libdmrg.so.
The library links the HIP runtime that PyTorch ships (same soname as ROCm's),
so a process that imports torch and loads the library has one HIP runtime.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmrg.so")

SOURCES = ["api.cpp", "plan.cpp", "macro_plan.cpp", "eigen.cpp", "hpsi.hip", "macro.hip", "vec.hip",
           "noalloc.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (hardware notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + os.path.join(ROOT, "include"),
]


def _torch_lib_dir():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return None


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops" not in l)   # host pass does not know the feature
    return p.returncode, out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        # host C++ (the eigen-solvers, plan and API) for the AVX2/FMA level
        # of the EPYC hosts MI355X boards sit in
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-Xarch_host", "-march=x86-64-v3"]
        cmds.append(([HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj], src))
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
        results = list(ex.map(lambda c: (c[1],) + _run(c[0]), cmds))
    for src, rc, out in results:
        if verbose and out.strip():
            print(f"[{src}]\n{out}")
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    tl = _torch_lib_dir()
    if tl:
        link += [f"-Wl,-rpath,{tl}", f"-L{tl}"]
    link += ["-Wl,-rpath,/opt/rocm/lib"]
    rc, out = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed:\n{out}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
