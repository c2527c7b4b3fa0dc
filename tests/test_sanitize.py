"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer, with
-fno-sanitize-recover=all so that any report fails the run:

* the oracle (gcc): a plain C driver calls every oracle entry point on small
  valid and invalid inputs, each buffer sized exactly, so an out-of-bounds
  access, a use of freed memory, a leak or undefined behaviour aborts it;
* the host side of the HIP library: the API translation units are compiled
  with the sanitizers on their host pass only (the device code is unchanged)
  and linked with the kernel units of the regular build; a C driver makes
  every device-facing call with an argument that validation must reject and
  runs the host-only routines (error strings, the sorting-network self-test,
  the events-per-thread tables, the VEGAS grid refinement, the run-time
  compilation of a user intensity) on real data."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ORACLE_SRC = os.path.join(ROOT, "oracle", "phsp_oracle.c")
CSRC = os.path.join(ROOT, "paper_1711_05683_amd", "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
API_UNITS = ("phsp_api", "phsp_batch_api", "phsp_serve", "phsp_unweight_api", "phsp_model_api",
             "phsp_vegas_api", "phsp_probe", "phsp_user_model")
LLVM = "/opt/rocm/llvm/bin"

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
          os.path.join(SAN, "oracle_driver.c"), ORACLE_SRC, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "sanitized oracle ok" in r.stdout


def _kernel_objects():
    objs = sorted(glob.glob(os.path.join(BUILD_DIR, "*_inst_n*.o")) +
                  glob.glob(os.path.join(BUILD_DIR, "phsp_batch_mixed_n*.o")))
    if len(objs) < 38:
        from paper_1711_05683_amd import build
        build.build()
        objs = sorted(glob.glob(os.path.join(BUILD_DIR, "*_inst_n*.o")) +
                      glob.glob(os.path.join(BUILD_DIR, "phsp_batch_mixed_n*.o")))
    return objs


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(f"{LLVM}/clang++"),
                    reason="hipcc / ROCm clang not available")
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    kernels = _kernel_objects()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off",
             "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Wno-unused-command-line-argument",
             f"-I{ROOT}/include", f"-I{CSRC}", f"-I{os.path.join(BUILD_DIR, 'gen')}"]

    def compile_unit(name):
        obj = str(tmp_path / f"{name}.o")
        _run(["hipcc", *flags, "-c", os.path.join(CSRC, f"{name}.hip"), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(7, os.cpu_count() or 1)) as ex:
        api = list(ex.map(compile_unit, API_UNITS))
    drv = str(tmp_path / "driver.o")
    _run([f"{LLVM}/clang", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", f"-I{ROOT}/include", "-c", os.path.join(SAN, "abi_host_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_sanitized")
    _run([f"{LLVM}/clang++", "-fsanitize=address,undefined", "-o", exe, drv, *api, *kernels,
          "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    r = _run([exe], env=ENV, timeout=300)
    assert "sanitized abi ok" in r.stdout
