"""Build libsph.so (HIP kernels for gfx950 + the C ABI) in-tree.

    python -m paper_2302_08381_amd.build        (or: python paper_2302_08381_amd/build.py)

Compiles the kernel translation units and the C-ABI host code with hipcc in
parallel, then links paper_2302_08381_amd/libsph.so.  Every call rebuilds
the objects whose sources or headers changed (timestamps), and always
relinks.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsph.so")

ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")
SOURCES = [
    "sph_kernels_values_f32_n0.hip",
    "sph_kernels_derivs_f32_n0_m0.hip",
    "sph_kernels_derivs_f32_n0_m1.hip",
    "sph_kernels_derivs_f32_n0_m2.hip",
    "sph_kernels_values_f32_n1.hip",
    "sph_kernels_derivs_f32_n1_m0.hip",
    "sph_kernels_derivs_f32_n1_m1.hip",
    "sph_kernels_derivs_f32_n1_m2.hip",
    "sph_kernels_bwd_f32.hip",
    "sph_kernels_values_f64_n0.hip",
    "sph_kernels_derivs_f64_n0_m0.hip",
    "sph_kernels_derivs_f64_n0_m1.hip",
    "sph_kernels_derivs_f64_n0_m2.hip",
    "sph_kernels_values_f64_n1.hip",
    "sph_kernels_derivs_f64_n1_m0.hip",
    "sph_kernels_derivs_f64_n1_m1.hip",
    "sph_kernels_derivs_f64_n1_m2.hip",
    "sph_kernels_bwd_f64.hip",
    "sph_kernels_expand_f32.hip",
    "sph_kernels_expand_f64.hip",
    "sph_kernels_hess_f32.hip",
    "sph_kernels_hess_f64.hip",
    "sph_kernels_e3nn.hip",
    "sph_api.cpp",
]
COMMON = [
    "-O3", "-std=c++20", "-fPIC", "-Wall",
    # packed FP32 instructions stay off (plain float code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libsph)")


def _deps_mtime() -> float:
    t = 0.0
    for d in (CSRC, INCLUDE):
        for f in os.listdir(d):
            if f.endswith((".hpp", ".h", ".inl")):
                t = max(t, os.path.getmtime(os.path.join(d, f)))
    return t


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    path = os.path.join(CSRC, src)
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(path), _deps_mtime())):
        return obj
    cmd = [hipcc(), f"--offload-arch={ARCH}", *COMMON, "-c", path, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stderr[-8000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4, 16)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libsph.so failed:\n{' '.join(cmd)}\n{r.stderr[-8000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
