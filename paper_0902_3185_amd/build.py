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


# Host-side address and undefined-behaviour sanitizers (each flag after
# -Xarch_host: they do not reach the device code).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
BUILD_SAN = os.path.join(CSRC, "_build_san")
LIB_SAN = os.path.join(HERE, "libdmrg_san.so")


def asan_runtime():
    """The compiler's shared address-sanitizer runtime (to preload into a
    process that loads the sanitized library)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_sanitized(verbose=False):
    """libdmrg_san.so: the host code (plan, API, eigen-solvers, launchers)
    built with the sanitizers above (the device code as usual), for host-only tests
    run with asan_runtime() preloaded.  Rebuilt only when a source changed."""
    import hashlib
    h = hashlib.sha256()
    for src in SOURCES + ["plan.h", "macro.h", "kernels.h", "eigen.h"]:
        path = os.path.join(CSRC, src)
        if os.path.exists(path):
            with open(path, "rb") as f:
                h.update(f.read())
    with open(os.path.join(ROOT, "include", "dmrg.h"), "rb") as f:
        h.update(f.read())
    with open(os.path.abspath(__file__), "rb") as f:   # the build recipe itself
        h.update(f.read())
    stamp = os.path.join(BUILD_SAN, "stamp")
    if os.path.exists(LIB_SAN) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
        return LIB_SAN
    os.makedirs(BUILD_SAN, exist_ok=True)
    base = ["-O1", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
            "-Wno-unused-variable", "-I" + os.path.join(ROOT, "include")]
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_SAN, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-Xarch_host", "-march=x86-64-v3"]
        cmds.append(([HIPCC] + base + SANITIZE + lang + ["-c", os.path.join(CSRC, src), "-o", obj], src))
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
        results = list(ex.map(lambda c: (c[1],) + _run(c[0]), cmds))
    for src, rc, out in results:
        if verbose and out.strip():
            print(f"[{src}]\n{out}")
        if rc != 0:
            raise RuntimeError(f"hipcc (sanitized) failed on {src}:\n{out}")
    link = [HIPCC, "-shared", "-fPIC", "-o", LIB_SAN + ".tmp"] + objs
    tl = _torch_lib_dir()
    if tl:
        link += [f"-Wl,-rpath,{tl}", f"-L{tl}"]
    link += ["-Wl,-rpath,/opt/rocm/lib"]
    rc, out = _run(link)
    if rc != 0:
        raise RuntimeError(f"link (sanitized) failed:\n{out}")
    os.replace(LIB_SAN + ".tmp", LIB_SAN)
    with open(stamp, "w") as f:
        f.write(h.hexdigest())
    return LIB_SAN


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
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
