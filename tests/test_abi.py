"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, validates its arguments, and carries its own Gauss rules.
No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2307_06471_amd import crkdg as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "crkdg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(crkdg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = K.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # and the binding covers them with the same names
    for n in names:
        assert n in K.EXPORTS, n


@pytest.mark.parametrize("n", range(1, 7))
def test_library_gauss_rules(n):
    x, w = K.crkdg_gauss_rule(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.abs(x - xr).max() < 1e-15 and np.abs(w - wr).max() < 1e-15
    for p in range(2 * n):  # exact for polynomials of degree <= 2n - 1
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs((w * x**p).sum() - exact) < 3e-16


def _create(**kw):
    args = dict(dim=2, nx=8, ny=8, equation=K.EQ_EULER)
    k = kw.pop("k", 2)
    flux = kw.pop("flux", K.FLUX_LLF)
    stages = kw.pop("stages", 3)
    args.update(kw)
    m = K.make_mesh(**args)
    h = C.c_void_p()
    return K.lib().crkdg_create(C.byref(m), k, flux, stages, C.byref(h)), h


@pytest.mark.parametrize("kw,code", [
    (dict(k=4), K.CRKDG_EINVAL),
    (dict(k=-1), K.CRKDG_EINVAL),
    (dict(nx=0), K.CRKDG_EINVAL),
    (dict(stages=5), K.CRKDG_EINVAL),
    (dict(stages=0), K.CRKDG_EINVAL),
    (dict(flux=K.FLUX_UPWIND), K.CRKDG_EUNSUPPORTED),
    (dict(dim=1, ny=1), K.CRKDG_EUNSUPPORTED),
    (dict(gamma=1.0), K.CRKDG_EINVAL),
    (dict(x1=0.0), K.CRKDG_EINVAL),
    (dict(bc=(7, 0, 0, 0)), K.CRKDG_EINVAL),
    (dict(precision=3), K.CRKDG_EINVAL),
    (dict(precision=K.FP32_INNER, equation=K.EQ_ADVECTION), K.CRKDG_EUNSUPPORTED),
    (dict(precision=K.FP32_INNER, k=0), K.CRKDG_EUNSUPPORTED),
    (dict(precision=K.FP32_MIXED, k=0), K.CRKDG_EUNSUPPORTED),
    (dict(nx=1 << 15, ny=1 << 14), K.CRKDG_EINVAL),  # a component slab would reach 4 GiB
])
def test_create_rejects_bad_arguments(kw, code):
    rc, _ = _create(**kw)
    assert rc == code


def test_create_sizes_and_unbound_errors():
    rc, h = _create()
    assert rc == 0
    L = K.lib()
    assert L.crkdg_state_bytes(h) == 4 * 9 * 64 * 8
    assert L.crkdg_workspace_bytes(h) >= 7 * L.crkdg_state_bytes(h)
    assert L.crkdg_step(h, 0.1) == K.CRKDG_EUNBOUND
    assert L.crkdg_limit(h, 50.0, None, None) == K.CRKDG_EUNBOUND
    assert L.crkdg_current_dofs(h) is None
    assert L.crkdg_bind(h, C.c_void_p(0x1001), C.c_void_p(0x2000), None) == K.CRKDG_EINVAL
    L.crkdg_destroy(h)


def test_state_sizes_of_the_precision_forms():
    L = K.lib()
    for prec, nbytes in ((K.FP64, 4 * 9 * 64 * 8), (K.FP32_INNER, 4 * 9 * 64 * 8),
                         (K.FP32_MIXED, 4 * 64 * 8 + 4 * 8 * 64 * 4)):
        rc, h = _create(precision=prec)
        assert rc == 0
        assert L.crkdg_state_bytes(h) == nbytes
        L.crkdg_destroy(h)


def test_set_tableau_validation():
    rc, h = _create()
    L = K.lib()
    dp = lambda a: np.ascontiguousarray(a, float).ctypes.data_as(C.POINTER(C.c_double))
    A_ok = np.array([[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]], float)
    b, c = np.array([1 / 6, 1 / 6, 2 / 3]), np.array([0, 1, 0.5])
    assert L.crkdg_set_tableau(h, 3, dp(c), dp(A_ok), dp(b)) == 0
    A_bad = A_ok.copy()
    A_bad[1, 1] = 0.5  # diagonal entry: implicit
    assert L.crkdg_set_tableau(h, 3, dp(c), dp(A_bad), dp(b)) == K.CRKDG_EINVAL
    A_nan = A_ok.copy()
    A_nan[2, 0] = np.nan
    assert L.crkdg_set_tableau(h, 3, dp(c), dp(A_nan), dp(b)) == K.CRKDG_EINVAL
    assert L.crkdg_set_tableau(h, 5, dp(c), dp(A_ok), dp(b)) == K.CRKDG_EINVAL
    L.crkdg_destroy(h)


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5):
        assert len(K.strerror(code)) >= 2


def test_rkdg_step_argument_checks():
    """the original-RKDG entry point rejects its arguments before touching
    device memory (the bound pointers below are never dereferenced)"""
    L = K.lib()
    assert L.crkdg_step_rkdg(None, 3, 50.0, 0.1, None) == K.CRKDG_EINVAL
    rc, h = _create()
    assert L.crkdg_step_rkdg(h, 3, 50.0, 0.1, None) == K.CRKDG_EUNBOUND
    assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
    for order, M, dt in ((1, 50.0, 0.1), (4, 50.0, 0.1), (3, float("nan"), 0.1),
                         (3, 50.0, 0.0), (2, -1.0, float("inf")), (3, 50.0, -1.0)):
        assert L.crkdg_step_rkdg(h, order, M, dt, None) == K.CRKDG_EINVAL, (order, M, dt)
    L.crkdg_destroy(h)
    for prec in (K.FP32_MIXED, K.FP32_INNER):
        rc, h = _create(precision=prec)
        assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
        assert L.crkdg_step_rkdg(h, 3, 50.0, 0.1, None) == K.CRKDG_EUNSUPPORTED
        L.crkdg_destroy(h)


def test_double_mach_reflection_mesh_checks():
    """CRKDG_IC_DMR boundary data need 2D Euler with inflow/outflow/Dirichlet
    sides; the learned indicator is rejected there (no such ghost rules)"""
    L = K.lib()
    dmr = dict(x1=4.0, bc=(2, 1, 2, 2), bc_exact=K.IC_DMR)
    rc, h = _create(**dmr)
    assert rc == 0
    assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
    fake = C.c_void_p(0x300000)
    assert L.crkdg_limit_mlp(h, 50.0, fake, 0.2, 0.9, None, None) == K.CRKDG_EUNSUPPORTED
    assert L.crkdg_mlp_features(h, 50.0, fake) == K.CRKDG_EUNSUPPORTED
    assert L.crkdg_limit_dt(h, 50.0, fake, 0.2, 0.9, None, 0.1, fake) == K.CRKDG_EUNSUPPORTED
    assert L.crkdg_project(h, K.IC_DMR, (C.c_double * 1)(1.0), 1, None) == K.CRKDG_EINVAL
    L.crkdg_destroy(h)
    for bad in (dict(bc=(2, 2, 2, 2)), dict(bc=(0, 1, 2, 2)), dict(equation=K.EQ_ADVECTION)):
        rc, _ = _create(**{**dmr, **bad})
        assert rc == K.CRKDG_EUNSUPPORTED, bad
