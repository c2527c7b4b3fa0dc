"""Build the HIP library ``libhydra_phsp.so`` for gfx950 (in-tree).

Every translation unit under ``csrc/`` is compiled with hipcc for gfx950 only;
the per-daughter-count kernel unit ``phsp_inst.hip`` is compiled once per
N = 2..10 so that the instantiations build in parallel.  Objects go to
``_build/`` at the repository root; the shared library lands next to this file.

Usage: ``python -m paper_1711_05683_amd.build`` (or ``build()`` from Python).
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
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_NAME = "libhydra_phsp.so"
LIB_PATH = os.path.join(PKG, LIB_NAME)

ARCH = "gfx950"
NS = range(2, 11)
BATCH_MIXED = (8, 10)

# Packed FP32 instructions are disabled for every HIP unit; the host pass warns
# that it does not know the feature, which is harmless.  Floating-point
# contraction is off: every multiply-add that should fuse is written as an
# explicit fma, so an event's arithmetic does not depend on the kernel it is
# inlined into (single-channel, batched and every events-per-thread variant give
# bit-identical events).
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


# ROCTx (the markers rocprofv3 --marker-trace records around each ABI call) and
# hiprtc (run-time compilation of user model intensities)
ROCM_LIB = "/opt/rocm/lib"
LINK_LIBS = [f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", "-lhiprtc", f"-Wl,-rpath,{ROCM_LIB}"]

# The kernel headers a user model is compiled against at run time, embedded in
# the library as strings (written to _build/gen before the units compile).
GEN_DIR = os.path.join(BUILD_DIR, "gen")
RTC_HEADERS = ("phsp_sortnet.hpp", "phsp_device.hpp", "phsp_reduce.hpp", "phsp_stage.hpp", "phsp_kernels.hpp",
               "phsp_model.hpp", "phsp_unweight.hpp", "phsp_vegas.hpp")
RTC_DELIM = "HPHSPSRC"


def _write_rtc_sources() -> None:
    """_build/gen/phsp_rtc_sources.inc: the names and texts of RTC_HEADERS as
    raw string literals, for the user-model compiler in phsp_user_model.hip."""
    os.makedirs(GEN_DIR, exist_ok=True)
    lines = ["// written by paper_1711_05683_amd/build.py from the csrc headers; not edited by hand",
             f"static const int kRtcHeaders = {len(RTC_HEADERS)};",
             "static const char* const kRtcHeaderNames[] = {" + ", ".join(f'"{h}"' for h in RTC_HEADERS) + "};",
             "static const char* const kRtcHeaderSources[] = {"]
    for h in RTC_HEADERS:
        with open(os.path.join(CSRC, h)) as f:
            text = f.read()
        if f"){RTC_DELIM}\"" in text:
            raise RuntimeError(f"{h} contains the raw-string delimiter")
        lines.append(f'R"{RTC_DELIM}({text}){RTC_DELIM}",')
    lines.append("};")
    out = os.path.join(GEN_DIR, "phsp_rtc_sources.inc")
    new = "\n".join(lines) + "\n"
    if not os.path.exists(out) or open(out).read() != new:
        with open(out, "w") as f:
            f.write(new)


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def _units():
    """(source, object, extra flags) for every translation unit."""
    units = []
    for n in NS:
        units.append((os.path.join(CSRC, "phsp_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_inst_n{n}.o"), [f"-DPHSP_N={n}"]))
    for n in NS:
        units.append((os.path.join(CSRC, "phsp_batch_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_batch_inst_n{n}.o"), [f"-DBATCH_N={n}"]))
    for n in NS:
        units.append((os.path.join(CSRC, "phsp_unweight_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_unweight_inst_n{n}.o"), [f"-DUNW_N={n}"]))
    for n in NS:
        units.append((os.path.join(CSRC, "phsp_model_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_model_inst_n{n}.o"), [f"-DMODEL_N={n}"]))
    for n in NS:
        units.append((os.path.join(CSRC, "phsp_chain_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_chain_inst_n{n}.o"), [f"-DCHAIN_N1={n}"]))
    for nmax in BATCH_MIXED:
        units.append((os.path.join(CSRC, "phsp_batch_inst.hip"),
                      os.path.join(BUILD_DIR, f"phsp_batch_mixed_n{nmax}.o"), [f"-DBATCH_MIXED={nmax}"]))
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") and not name.endswith("_inst.hip"):
            units.append((os.path.join(CSRC, name),
                          os.path.join(BUILD_DIR, name[:-4] + ".o"),
                          [f"-I{GEN_DIR}"] if name == "phsp_user_model.hip" else []))
        elif name.endswith(".cpp"):
            units.append((os.path.join(CSRC, name),
                          os.path.join(BUILD_DIR, name[:-4] + ".o"), []))
    return units


def _compile(hipcc, src, obj, extra):
    cmd = [hipcc, *HIP_FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every unit and link the shared library; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    _write_rtc_sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _units()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, hipcc, s, o, x) for s, o, x in units]
        objs = [f.result() for f in futs]
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *LINK_LIBS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH} from {len(objs)} units")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
