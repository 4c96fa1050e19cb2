"""Builds libjx.so in-tree: HIP kernels for gfx950 plus the host runtime.

    python -m paper_2605_19926_amd.build        (or build() from Python)

Every HIP source is compiled with packed-FP32 instruction selection disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libjx.so")
DEMO = os.path.join(PKG, "jx_demo")  # a C++ caller of the C-ABI (no Python)
STORE_CEILING = os.path.join(PKG, "jx_store_ceiling")  # HBM store-pattern calibration
ARCH = os.environ.get("JX_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_SOURCES = ["jx_kernels.hip"]
HOST_SOURCES = ["jx_abi.cpp", "jx_host.cpp", "jx_layout.cpp", "jx_server.cpp"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-fno-gpu-rdc"]
HOST_FLAGS = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-Wno-unused-result", "-Wno-unused-value"]


def _obj_dir() -> str:
    d = os.path.join(PKG, "_build")
    os.makedirs(d, exist_ok=True)
    return d


def _compile(src: str, device: bool) -> str:
    obj = os.path.join(_obj_dir(), os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + (DEVICE_FLAGS if device else HOST_FLAGS) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    jobs = [(s, True) for s in DEVICE_SOURCES] + [(s, False) for s in HOST_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    # the C++ demo links the library found next to it
    tmp = DEMO + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", f"-I{INCLUDE}"] + HOST_FLAGS + [os.path.join(CSRC, "jx_demo.cpp"),
           "-x", "none", "-o", tmp, f"-L{PKG}", "-ljx", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"demo build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, DEMO)
    # store-pattern calibration program (bench.py reports its figures)
    tmp = STORE_CEILING + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", "-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", os.path.join(CSRC, "jx_store_ceiling.cpp"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"store ceiling build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, STORE_CEILING)
    if verbose:
        print("built", OUT, "and", DEMO)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
