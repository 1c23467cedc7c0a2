"""Build libturboreg.so (HIP, gfx950) in-tree with hipcc.

Every source in csrc/ is compiled to an object in parallel, then linked into
paper_2507_01439_amd/libturboreg.so. Floating-point contraction is off so the
decision arithmetic of Eq. 1 and Eq. 9 is exactly the fused multiply-adds the
sources spell out; packed FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libturboreg.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("TURBOREG_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the TurboReg HIP library cannot be built")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *FLAGS, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host AddressSanitizer build (tests only): the same sources with the host side of every
# translation unit instrumented (-Xarch_host puts the sanitizer on the host pass alone; the GPU
# code is built as for the library), linked with the host-code driver into one executable.
ASAN_DIR = os.path.join(HERE, "_build_asan")
ASAN_DRIVER = os.path.join(os.path.dirname(HERE), "tests", "asan", "host_driver.cpp")
ASAN_EXE = os.path.join(ASAN_DIR, "host_driver")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build_asan(verbose: bool = False) -> str:
    os.makedirs(ASAN_DIR, exist_ok=True)

    def one(src):
        obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc(), *FLAGS, *ASAN_FLAGS, "-x", "hip", "-c", src, "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (host ASan) failed on {src}:\n{r.stderr}")
        return obj

    srcs = sources() + [ASAN_DRIVER]
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(one, srcs))
    tmp = ASAN_EXE + ".tmp"
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (host ASan) failed:\n{r.stderr}")
    os.replace(tmp, ASAN_EXE)
    if verbose:
        print(f"built {ASAN_EXE}")
    return ASAN_EXE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
