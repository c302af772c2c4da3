"""AddressSanitizer and UndefinedBehaviorSanitizer on the host code (CPU
only): the oracle (gcc) driven over small ragged runs of every kind, and the
library's host side (clean_api.hip compiled with host-only sanitizers and
linked with the built kernel objects) driven through every entry point's
argument checks and the workspace size arithmetic.  Any sanitizer report
fails the run (no recovery)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2501_01461_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2501_01461_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-ffp-contract=off", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    out = run([exe], env=dict(ENV, OMP_NUM_THREADS="2"))
    assert "all checks passed" in out.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    objs = [os.path.join(BUILD, f) for f in ("clean_kernels.o", "clean_restore.o", "clean_probe.o")]
    if not os.path.exists(HIPCC) or not all(map(os.path.exists, objs)):
        pytest.skip("hipcc or the built kernel objects (run the build first) not found")
    san = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    api = str(tmp_path / "clean_api_san.o")
    run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off", *san.split(), *inc,
         "-c", os.path.join(CSRC, "clean_api.hip"), "-o", api])
    drv = str(tmp_path / "abi_driver.o")
    run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *san.split(), *inc,
         "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    run([HIPCC, "--offload-arch=gfx950", *san.split(), drv, api, *objs, "-o", exe])   # objects only
    out = run([exe], env=ENV)
    assert "all checks passed" in out.stdout
