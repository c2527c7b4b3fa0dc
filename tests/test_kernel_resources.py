"""Register budgets of the built gfx950 kernels, read from the code-object
metadata of the library's own objects (the kernel descriptors the compiler
emits: VGPR count, private segment size, spill counts).

* No kernel spills vector registers to scratch memory, including the mixed-N
  kernels (one launch for tiles of any N), whose budget a waves-per-SIMD hint
  holds at 128 VGPRs.  (Scalar registers that spill go to lanes of vector
  registers, not to memory.)
* The mixed-N kernels fit in 128 VGPRs (4 waves per SIMD).
"""
from __future__ import annotations

import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD_DIR = os.path.join(ROOT, "_build")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _kernels(obj, tmp):
    """[(name, vgprs, private segment bytes, vgpr spills, sgpr spills)] of one object."""
    base = os.path.join(tmp, os.path.basename(obj))
    fb, co = base + ".fatbin", base + ".co"
    r = subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fb}", obj, base + ".host"],
                       capture_output=True, text=True)
    if r.returncode != 0 or not os.path.exists(fb):
        return []
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fb}",
                    f"--targets={TARGET}", f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", co], check=True, capture_output=True,
                           text=True).stdout
    out = []
    for blk in re.split(r"\n\s+- \.agpr_count:", notes)[1:]:
        def field(key):
            return re.search(rf"\.{key}:\s+(\S+)", blk).group(1)
        out.append((field("name"), int(field("vgpr_count")), int(field("private_segment_fixed_size")),
                    int(field("vgpr_spill_count")), int(field("sgpr_spill_count"))))
    return out


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not all(os.path.exists(f"{LLVM}/{t}") for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")):
        pytest.skip("ROCm LLVM tools not available")
    objs = sorted(glob.glob(os.path.join(BUILD_DIR, "*.o")))
    if len(objs) < 45:
        if shutil.which("hipcc") is None:
            pytest.skip("library not built and hipcc not available")
        from paper_1711_05683_amd import build
        build.build()
        objs = sorted(glob.glob(os.path.join(BUILD_DIR, "*.o")))
    tmp = str(tmp_path_factory.mktemp("co"))
    ks = {}
    for o in objs:
        for k in _kernels(o, tmp):
            ks[k[0]] = k[1:]
    assert len(ks) > 300, len(ks)
    return ks


def test_no_kernel_spills(kernels):
    spilling = sorted(n for n, v in kernels.items() if v[1] or v[2])
    assert not spilling, spilling


def test_mixed_n_kernels_fit_four_waves(kernels):
    mixed = [n for n in kernels if "k_phsp_batched_mixed" in n]
    # bounds 8 and 10, each at one event per thread and at the per-N defaults
    assert len(mixed) == 4 and all(kernels[n][0] <= 128 for n in mixed), [(n, kernels[n]) for n in mixed]
