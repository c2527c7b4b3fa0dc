"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the device."""
from __future__ import annotations

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1711_05683_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1711_05683_amd import build
        build.build()
    return P


def _declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(hydra_phsp_[a-z0-9_]+)\s*\(", text):
            names.append(m.group(1))
    return sorted(set(names))


def test_every_declared_symbol_is_exported(P):
    names = _declared_functions()
    assert "hydra_phsp_generate" in names and "hydra_phsp_integrate" in names
    lib = P.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_sortnet(P):
    assert P.lib().hydra_phsp_abi_version() == 1
    assert P.selftest_sortnet()


def test_strerror(P):
    for code in (P.OK, P.EINVAL, P.EKINEMATICS, P.ENOMEM, P.EDEVICE, P.EAGAIN, P.ENOTFOUND):
        assert P.lib().hydra_phsp_strerror(code)


def _gen_status(P, M, masses, nevents=10, ld=None, out=1, w=1, parent_host=None, parent_dev=None,
                ldp=0):
    m, n = P._masses(masses)
    ph = None if parent_host is None else (ctypes.c_double * 4)(*parent_host)
    return P.lib().hydra_phsp_generate(M, m, n, ph, parent_dev, ldp, nevents, 1, 0, 0,
                                       ctypes.c_void_p(out) if out else None,
                                       nevents if ld is None else ld,
                                       ctypes.c_void_p(w) if w else None, None, None)


def test_validation_before_any_device_work(P):
    # Fake non-NULL pointers: every case must fail in validation, before launch.
    assert _gen_status(P, 5.0, [1.0]) == P.EINVAL
    assert _gen_status(P, 50.0, [0.1] * 11) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, -0.1]) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, float("nan")]) == P.EINVAL
    assert _gen_status(P, float("inf"), [1.0, 1.0]) == P.EINVAL
    assert _gen_status(P, -5.0, [1.0, 1.0]) == P.EINVAL
    assert _gen_status(P, 5.0, [3.0, 2.0]) == P.EKINEMATICS
    assert _gen_status(P, 5.0, [3.0, 2.5]) == P.EKINEMATICS
    assert _gen_status(P, 5.0, [1.0, 1.0], ld=5) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, 1.0], out=0) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, 1.0], w=0) == P.EINVAL
    # parent four-vector whose mass is not M
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_host=[5.0, 1.0, 0.0, 0.0]) == P.EINVAL
    # both parent forms at once
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_host=[5.0, 0.0, 0.0, 0.0],
                       parent_dev=ctypes.c_void_p(8), ldp=10) == P.EINVAL
    # per-event parents with a too-short leading dimension
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_dev=ctypes.c_void_p(8), ldp=3) == P.EINVAL
    assert "ld_parent" in P.lib().hydra_phsp_last_error().decode()


def test_integrate_validation(P):
    m, n = P._masses([1.0, 1.0])
    mean, sigma = ctypes.c_double(), ctypes.c_double()
    assert P.lib().hydra_phsp_integrate(5.0, m, n, 1, 1, 0, 0, ctypes.byref(mean),
                                        ctypes.byref(sigma), None) == P.EINVAL
    assert P.lib().hydra_phsp_integrate(5.0, m, n, 10, 1, 0, 0, None, ctypes.byref(sigma),
                                        None) == P.EINVAL
    assert P.lib().hydra_phsp_integrate_async(5.0, m, n, 10, 1, 0, 0, None, None) == P.EINVAL
    m3, n3 = P._masses([3.0, 3.0])
    assert P.lib().hydra_phsp_integrate_async(5.0, m3, n3, 10, 1, 0, 0, ctypes.c_void_p(8),
                                              None) == P.EKINEMATICS


def test_product_path_does_not_import_oracle():
    # The product package must never route through the CPU oracle.
    pkg = os.path.join(ROOT, "paper_1711_05683_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
            text = open(path).read()
            assert "import oracle" not in text and "from oracle" not in text, path
            assert "phsp_oracle" not in text and "_liboracle" not in text, path
