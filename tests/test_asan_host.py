"""Host AddressSanitizer runs (host code only; no GPU sanitizer is used).

The oracle: every entry point on small and degenerate inputs, built with gcc's address and
undefined-behaviour sanitizers, in the plain and the OpenMP build. The library: its host code
(argument checking, workspace layout, launch sequences, graph cache, tuning, scorer blobs,
inspection) built with -fsanitize=address on the host pass only, driven by
tests/asan/host_driver.cpp; without a GPU it checks the paths that need no device, on the GPU
it calls every entry point once.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_asan_ubsan(tmp_path, openmp):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    cmd = [gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
           "-ffp-contract=off", "-Wno-unknown-pragmas", "-o", exe, os.path.join(HERE, "asan", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "turboreg_oracle.c"), "-lm"] + (["-fopenmp"] if openmp else [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(ENV, OMP_NUM_THREADS="4"))
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]


def host_driver():
    from paper_2507_01439_amd import build as B
    if not os.path.exists(B.ASAN_EXE):
        B.build_asan()
    return B.ASAN_EXE


def test_library_host_code_under_asan_without_device():
    r = subprocess.run([host_driver()], capture_output=True, text=True, timeout=300,
                       env=dict(ENV, HIP_VISIBLE_DEVICES="-1"))
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]


@pytest.mark.gpu
def test_library_host_code_under_asan_on_gpu():
    from paper_2507_01439_amd import build as B
    assert os.path.exists(B.ASAN_EXE), "the host ASan driver is built by the package's build step"
    r = subprocess.run([B.ASAN_EXE], capture_output=True, text=True, timeout=240, env=ENV)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")
