"""CPU tests of user intensities compiled at run time (hiprtc needs no GPU):
compilation, the compiler's log for a bad source, and the validation of every
argument before any device work."""
from __future__ import annotations

import ctypes

import pytest

BW_SOURCE = """
// relativistic Breit-Wigner intensity in the (1, 2) pair mass: par = (mass, width)
__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py,
                                            const double* pz, const double* par) {
    const double se = e[1] + e[2], sx = px[1] + px[2], sy = py[1] + py[2], sz = pz[1] + pz[2];
    const double s = se * se - sx * sx - sy * sy - sz * sz;
    const double d = par[0] * par[0] - s;
    const double mg = par[0] * par[1];
    return 1.0 / (d * d + mg * mg);
}
"""


@pytest.fixture(scope="module")
def P():
    import paper_1711_05683_amd as P
    try:
        P.lib()
    except RuntimeError as e:
        pytest.skip(str(e))
    return P


def _create(P, src, n):
    h = ctypes.c_void_p()
    st = P.lib().hydra_phsp_user_model_create(None if src is None else src.encode(), n, ctypes.byref(h))
    return st, h


def test_user_model_compiles_without_gpu(P):
    st, h = _create(P, BW_SOURCE, 3)
    assert st == P.OK and h.value
    assert P.lib().hydra_phsp_user_model_daughters(h) == 3
    assert P.lib().hydra_phsp_user_model_destroy(h) == P.OK


@pytest.mark.parametrize("src", [
    "this is not C++",
    "__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py, "
    "const double* pz, const double* par) { return undefined_symbol; }",
    "__device__ double another_name(const double* e) { return e[0]; }",
])
def test_user_model_bad_source_is_rejected_with_the_log(P, src):
    st, h = _create(P, src, 3)
    assert st == P.EINVAL and not h.value
    msg = P.lib().hydra_phsp_last_error().decode()
    assert "user model does not compile" in msg and "error" in msg


def test_user_model_create_validation(P):
    for src, n in ((None, 3), (BW_SOURCE, 1), (BW_SOURCE, 11)):
        st, h = _create(P, src, n)
        assert st == P.EINVAL and not h.value, (src is None, n)
    assert P.lib().hydra_phsp_user_model_create(BW_SOURCE.encode(), 3, None) == P.EINVAL
    assert P.lib().hydra_phsp_user_model_destroy(None) == P.EINVAL
    assert P.lib().hydra_phsp_user_model_daughters(None) == P.EINVAL


def test_user_model_integrate_validation(P):
    """Every bad argument is rejected before the code object is loaded or any
    device memory is touched (fake device pointers are never dereferenced)."""
    st, h = _create(P, BW_SOURCE, 3)
    assert st == P.OK
    f = P.lib().hydra_phsp_integrate_user_model
    m = (ctypes.c_double * 3)(3.097, 0.4937, 0.13957)
    par = (ctypes.c_double * 2)(0.8955, 0.0473)
    stats = ctypes.c_void_p(256)
    try:
        assert f(None, 5.279, m, par, 2, 100, 1, 0, 0, None, stats, None) == P.EINVAL
        assert f(h, 5.279, m, par, 17, 100, 1, 0, 0, None, stats, None) == P.EINVAL
        assert f(h, 5.279, m, par, -1, 100, 1, 0, 0, None, stats, None) == P.EINVAL
        assert f(h, 5.279, m, None, 2, 100, 1, 0, 0, None, stats, None) == P.EINVAL
        assert f(h, 5.279, m, par, 2, 100, 1, 0, 0, None, None, None) == P.EINVAL
        assert f(h, 5.279, m, par, 2, 100, 1, 0, 0, ctypes.c_void_p(4), stats, None) == P.EINVAL
        assert f(h, 3.5, m, par, 2, 100, 1, 0, 0, None, stats, None) == P.EKINEMATICS
        assert f(h, 5.279, None, par, 2, 100, 1, 0, 0, None, stats, None) == P.EINVAL
    finally:
        assert P.lib().hydra_phsp_user_model_destroy(h) == P.OK


def test_user_model_unweighted_validation(P):
    """The unweighted sample of a user model checks its arguments before any
    device work, as the weight-only sample does."""
    st, h = _create(P, BW_SOURCE, 3)
    assert st == P.OK
    f = P.lib().hydra_phsp_generate_unweighted_user_model
    m = (ctypes.c_double * 3)(3.097, 0.4937, 0.13957)
    par = (ctypes.c_double * 2)(0.8955, 0.0473)
    out, cnt = ctypes.c_void_p(1024), ctypes.c_void_p(256)

    def call(model=h, M=5.279, mm=m, pp=par, k=2, w_max=0.0, o=out, ld=128, counts=cnt):
        return f(model, M, mm, pp, k, 100, 1, 0, 0, w_max, o, ld, None, counts, None, None)

    try:
        assert call(model=None) == P.EINVAL
        assert "model" in P.lib().hydra_phsp_last_error().decode()
        assert call(k=17) == P.EINVAL
        assert call(k=-1) == P.EINVAL
        assert call(pp=None) == P.EINVAL
        assert call(counts=None) == P.EINVAL
        assert call(w_max=-1.0) == P.EINVAL
        assert call(w_max=float("nan")) == P.EINVAL
        assert call(ld=0) == P.EINVAL
        assert call(o=ctypes.c_void_p(1028)) == P.EINVAL
        assert call(M=3.5) == P.EKINEMATICS
        assert call(mm=None) == P.EINVAL
    finally:
        assert P.lib().hydra_phsp_user_model_destroy(h) == P.OK


def test_user_model_binding_checks_daughter_count(P):
    model = P.UserModel(BW_SOURCE, 3)
    try:
        with pytest.raises(ValueError):
            model.integrate(5.279, [3.097, 0.4937], 100, [0.8955, 0.0473])
        with pytest.raises(ValueError):
            model.integrate(5.279, [3.097, 0.4937, 0.13957], 100, [0.0] * 17)
        with pytest.raises(ValueError):
            model.generate_unweighted(5.279, [3.097, 0.4937], 100, [0.8955, 0.0473])
        with pytest.raises(ValueError):
            model.generate_unweighted(5.279, [3.097, 0.4937, 0.13957], 100, [0.0] * 17)
    finally:
        model.destroy()
    with pytest.raises(P.PhspError):
        P.UserModel("not a function", 3)


# --------------------------------------------------------------------------
# VEGAS integrands compiled at run time

INTEGRAND = """
__device__ double hydra_phsp_user_integrand(const double* x, const double* par) {
    return x[0] * x[1] * x[1] * exp(x[2]) * (1.0 + par[0] * x[HYDRA_PHSP_DIM - 1]);
}
"""


def test_user_integrand_compiles_without_gpu(P):
    h = ctypes.c_void_p()
    assert P.lib().hydra_phsp_user_integrand_create(INTEGRAND.encode(), 4, ctypes.byref(h)) == P.OK and h.value
    assert P.lib().hydra_phsp_user_integrand_destroy(h) == P.OK


def test_user_integrand_create_validation(P):
    f = P.lib().hydra_phsp_user_integrand_create
    h = ctypes.c_void_p()
    assert f(None, 4, ctypes.byref(h)) == P.EINVAL
    for dim in (0, 17):
        assert f(INTEGRAND.encode(), dim, ctypes.byref(h)) == P.EINVAL and not h.value
    assert f(INTEGRAND.encode(), 4, None) == P.EINVAL
    assert f(b"double hydra_phsp_user_integrand(", 4, ctypes.byref(h)) == P.EINVAL and not h.value
    assert "user integrand does not compile" in P.lib().hydra_phsp_last_error().decode()
    assert P.lib().hydra_phsp_user_integrand_destroy(None) == P.EINVAL
    with pytest.raises(P.PhspError):
        P.UserIntegrand("not C++", 2)


def test_user_integrand_vegas_validation(P):
    """Bad boxes, parameters, bins and buffers are rejected before any device work."""
    h = ctypes.c_void_p()
    assert P.lib().hydra_phsp_user_integrand_create(INTEGRAND.encode(), 4, ctypes.byref(h)) == P.OK
    D = ctypes.c_double
    lo, hi, bad_hi = (D * 4)(0, 0, 0, -1), (D * 4)(1, 1, 1, 1), (D * 4)(1, 1, 0, 1)
    par = (D * 1)(0.5)
    it, run = P.lib().hydra_phsp_vegas_user_iteration, P.lib().hydra_phsp_vegas_user
    grid, stats = ctypes.c_void_p(256), ctypes.c_void_p(512)
    r, e, c = D(), D(), D()
    try:
        assert it(None, lo, hi, par, 1, 10, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, None, hi, par, 1, 10, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, bad_hi, par, 1, 10, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, par, 17, 10, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, None, 1, 10, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, par, 1, 1, grid, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, par, 1, 10, None, 100, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, par, 1, 10, grid, 1, 1, 0, stats, None, None, None) == P.EINVAL
        assert it(h, lo, hi, par, 1, 10, grid, 100, 1, 0, ctypes.c_void_p(4), None, None, None) == P.EINVAL
        assert run(h, lo, bad_hi, par, 1, 10, 100, 0, 1, 1.5, 1, None, ctypes.byref(r), ctypes.byref(e),
                   ctypes.byref(c), None) == P.EINVAL
        assert run(h, lo, hi, par, 1, 10, 100, 0, 0, 1.5, 1, None, ctypes.byref(r), ctypes.byref(e),
                   ctypes.byref(c), None) == P.EINVAL
        assert run(h, lo, hi, par, 1, 10, 100, 0, 1, -1.0, 1, None, ctypes.byref(r), ctypes.byref(e),
                   ctypes.byref(c), None) == P.EINVAL
    finally:
        assert P.lib().hydra_phsp_user_integrand_destroy(h) == P.OK
