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


def _gauss_50_digits(n):
    """nodes and weights by Newton's method on P_n in 50-digit decimal
    arithmetic, started from numpy's rule"""
    from decimal import Decimal, getcontext
    getcontext().prec = 50

    def leg(m, z):
        p0, p1 = Decimal(1), z
        if m == 0:
            return p0
        for j in range(1, m):
            p0, p1 = p1, ((2 * j + 1) * z * p1 - j * p0) / (j + 1)
        return p1

    def dleg(z):  # (1 - z^2) P_n' = n (P_{n-1} - z P_n)
        return n * (leg(n - 1, z) - z * leg(n, z)) / (1 - z * z)

    xs, ws = [], []
    for x0 in np.polynomial.legendre.leggauss(n)[0]:
        z = Decimal(repr(float(x0)))
        for _ in range(8):
            if n > 1:
                z -= leg(n, z) / dleg(z)
        d = dleg(z) if n > 1 else Decimal(1)
        xs.append(z)
        ws.append(2 / ((1 - z * z) * d * d))
    return xs, ws


@pytest.mark.parametrize("n", range(1, 9))
def test_library_gauss_rules(n):
    """n <= 6 are closed forms and tables, n = 7, 8 roots of P_n found at
    compile time: nodes within 2e-16, weights within 5e-15 relative of a
    50-digit reference, and exact on polynomials of degree <= 2n - 1"""
    x, w = K.crkdg_gauss_rule(n)
    xs, ws = _gauss_50_digits(n)
    from decimal import Decimal
    for a in range(n):
        assert abs(Decimal(repr(float(x[a]))) - xs[a]) < Decimal("2e-16"), a
        assert abs(Decimal(repr(float(w[a]))) - ws[a]) < Decimal("5e-15") * ws[a], a
    for p in range(2 * n):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs((w * x**p).sum() - exact) < 1e-15


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
    (dict(k=5), K.CRKDG_EINVAL),
    (dict(k=4), K.CRKDG_EUNSUPPORTED),  # k = 4 is built for the scalar equations
    (dict(k=-1), K.CRKDG_EINVAL),
    (dict(nx=0), K.CRKDG_EINVAL),
    (dict(stages=6), K.CRKDG_EINVAL),
    (dict(stages=0), K.CRKDG_EINVAL),
    (dict(flux=K.FLUX_UPWIND), K.CRKDG_EUNSUPPORTED),
    (dict(flux=K.FLUX_GODUNOV), K.CRKDG_EUNSUPPORTED),
    (dict(flux=3), K.CRKDG_EINVAL),
    (dict(equation=K.EQ_ADVECTION, flux=K.FLUX_GODUNOV), K.CRKDG_EUNSUPPORTED),
    (dict(equation=K.EQ_BURGERS, flux=K.FLUX_GODUNOV), K.CRKDG_EUNSUPPORTED),  # 2D
    (dict(equation=K.EQ_BURGERS, dim=1, ny=1, flux=K.FLUX_LLF), K.CRKDG_EUNSUPPORTED),
    (dict(equation=K.EQ_BURGERS, dim=1, ny=1, flux=K.FLUX_GODUNOV, bc=(2, 1, 0, 0),
          bc_exact=K.IC_ADV_SIN), K.CRKDG_EUNSUPPORTED),
    (dict(equation=3), K.CRKDG_EINVAL),
    (dict(dim=1, ny=1), K.CRKDG_EUNSUPPORTED),
    (dict(gamma=1.0), K.CRKDG_EINVAL),
    (dict(x1=0.0), K.CRKDG_EINVAL),
    (dict(bc=(7, 0, 0, 0)), K.CRKDG_EINVAL),
    (dict(precision=4), K.CRKDG_EINVAL),
    (dict(precision=K.FP32_INCREMENTS, k=0), K.CRKDG_EUNSUPPORTED),
    (dict(precision=K.FP32_INCREMENTS, k=4), K.CRKDG_EUNSUPPORTED),
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
                         (K.FP32_INCREMENTS, 4 * 9 * 64 * 8),
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
    A7, b7, c7 = np.zeros((7, 7)), np.full(7, 1 / 7), np.zeros(7)
    assert L.crkdg_set_tableau(h, 7, dp(c7), dp(A7), dp(b7)) == K.CRKDG_EINVAL  # > 6 stages
    L.crkdg_destroy(h)


def test_six_stage_tableaus_size_the_workspace():
    """the workspace holds max(4, s) stages: a six-stage tableau set before
    binding enlarges it (4 more state slots), one set after binding a
    four-stage workspace is refused; rk_stages = 5 (Fehlberg) sizes it at
    creation"""
    L = K.lib()
    dp = lambda a: np.ascontiguousarray(a, float).ctypes.data_as(C.POINTER(C.c_double))
    A6, b6, c6 = np.zeros((6, 6)), np.full(6, 1 / 6), np.zeros(6)
    for i in range(1, 6):
        A6[i, i - 1] = 0.5
    rc, h = _create()
    w4 = L.crkdg_workspace_bytes(h)
    S = L.crkdg_state_bytes(h)
    assert L.crkdg_set_tableau(h, 6, dp(c6), dp(A6), dp(b6)) == 0
    assert L.crkdg_workspace_bytes(h) == w4 + 4 * S
    L.crkdg_destroy(h)
    rc, h = _create(stages=5)
    assert rc == 0 and L.crkdg_workspace_bytes(h) == w4 + 4 * S
    L.crkdg_destroy(h)
    rc, h = _create()
    assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
    assert L.crkdg_set_tableau(h, 6, dp(c6), dp(A6), dp(b6)) == K.CRKDG_EINVAL
    assert L.crkdg_set_tableau(h, 4, dp(c6[:4]), dp(A6[:4, :4]), dp(b6[:4])) == 0
    L.crkdg_destroy(h)


def test_burgers_and_degree_four_are_accepted():
    for kw in (dict(equation=K.EQ_BURGERS, dim=1, ny=1, flux=K.FLUX_GODUNOV, k=4, stages=5),
               dict(equation=K.EQ_ADVECTION, dim=2, flux=K.FLUX_UPWIND, k=4, stages=5),
               dict(equation=K.EQ_ADVECTION, dim=1, ny=1, flux=K.FLUX_UPWIND, k=4, stages=4)):
        rc, h = _create(**kw)
        assert rc == 0, kw
        K.lib().crkdg_destroy(h)


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
                         (3, 50.0, 0.0), (2, -1.0, float("inf")), (3, 50.0, -1.0),
                         (0, 50.0, 0.1), (0, 0.0, 0.1), (0, -1.0, 0.0), (-1, -1.0, 0.1)):
        assert L.crkdg_step_rkdg(h, order, M, dt, None) == K.CRKDG_EINVAL, (order, M, dt)
    L.crkdg_destroy(h)
    for prec in (K.FP32_MIXED, K.FP32_INNER, K.FP32_INCREMENTS):
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


def test_burgers_initial_data_needs_burgers():
    """checked before any device work (the bound pointers are never used)"""
    L = K.lib()
    rc, h = _create(equation=K.EQ_ADVECTION, dim=1, ny=1, flux=K.FLUX_UPWIND)
    assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
    assert L.crkdg_project(h, K.IC_BURGERS_SIN, None, 0, None) == K.CRKDG_EINVAL
    out = (C.c_double * 3)()
    assert L.crkdg_error(h, K.IC_BURGERS_SIN, None, 0, 0.0, 0, out) == K.CRKDG_EINVAL
    assert L.crkdg_project(h, 8, None, 0, None) == K.CRKDG_EINVAL
    L.crkdg_destroy(h)


def test_combine_argument_checks():
    """at most six arrays (the largest tableau); checked before device work"""
    L = K.lib()
    rc, h = _create()
    assert L.crkdg_bind(h, C.c_void_p(0x100000), C.c_void_p(0x200000), None) == 0
    coef = (C.c_double * 7)(*([0.5] * 7))
    X = (C.c_void_p * 7)(*([0x300000] * 7))
    assert L.crkdg_combine(h, C.c_void_p(0x400000), None, 7, coef, X) == K.CRKDG_EINVAL
    assert L.crkdg_combine(h, C.c_void_p(0x400000), None, -1, coef, X) == K.CRKDG_EINVAL
    assert L.crkdg_combine(h, None, None, 1, coef, X) == K.CRKDG_EINVAL
    L.crkdg_destroy(h)


def test_noalloc_gradient_argument_checks():
    """crkdg_mlp_grad_noalloc refuses batches beyond its fixed buffer and bad
    arguments before any device work (no GPU needed)"""
    L = K.lib()
    fake = C.c_void_p(0x1000)
    assert K.MLP_NOALLOC_MAX_B == 16384
    big = K.MLP_NOALLOC_MAX_B + 1
    assert L.crkdg_mlp_grad_noalloc(fake, fake, fake, big, 1.0, fake, None, None) == K.CRKDG_EINVAL
    assert L.crkdg_mlp_grad_noalloc(fake, fake, fake, 0, 1.0, fake, None, None) == K.CRKDG_EINVAL
    assert L.crkdg_mlp_grad_noalloc(fake, fake, fake, 64, 0.0, fake, None, None) == K.CRKDG_EINVAL
    assert L.crkdg_mlp_grad_noalloc(None, fake, fake, 64, 1.0, fake, None, None) == K.CRKDG_EINVAL


def test_schedule_selection_is_host_logic():
    """the fused schedule is accepted only where the fused kernel applies
    (2D Euler, FP32-bulk or FP64, k = 1 or 2, constant boundary data, weights
    on the first and last stage only); no GPU needed"""
    L = K.lib()

    def handle(k=2, stages=3, precision=K.FP32_MIXED, bc=(1, 1, 1, 1), bc_exact=0, dim=2):
        m = K.make_mesh(dim, 70, 9 if dim == 2 else 1, bc=bc, bc_exact=bc_exact,
                        equation=K.EQ_EULER, precision=precision)
        return K.crkdg_create(m, k, K.FLUX_LLF, stages)

    h = handle()
    assert L.crkdg_get_schedule(h) == K.SCHED_FUSED            # the default where it applies
    assert L.crkdg_set_schedule(h, K.SCHED_SPLIT) == K.CRKDG_OK
    assert L.crkdg_get_schedule(h) == K.SCHED_SPLIT
    assert L.crkdg_set_schedule(h, 7) == K.CRKDG_EINVAL
    assert L.crkdg_set_schedule(h, K.SCHED_FUSED) == K.CRKDG_OK
    assert L.crkdg_get_schedule(h) == K.SCHED_FUSED
    L.crkdg_destroy(h)
    for kw in (dict(k=3), dict(stages=4), dict(precision=K.FP32_INNER),
               dict(precision=K.FP32_INCREMENTS), dict(bc=(2, 1, 2, 2), bc_exact=K.IC_DMR)):
        h = handle(**kw)
        assert L.crkdg_get_schedule(h) == K.SCHED_SPLIT, kw      # falls back by itself
        assert L.crkdg_set_schedule(h, K.SCHED_FUSED) == K.CRKDG_EUNSUPPORTED, kw
        assert L.crkdg_get_schedule(h) == K.SCHED_SPLIT
        L.crkdg_destroy(h)
    for kw in (dict(k=1, stages=2), dict(stages=1), dict(bc=(0, 0, 0, 0)), dict(bc=(2, 2, 2, 2)),
               dict(precision=K.FP64), dict(precision=K.FP64, k=1, stages=2)):
        h = handle(**kw)
        assert L.crkdg_set_schedule(h, K.SCHED_FUSED) == K.CRKDG_OK, kw
        L.crkdg_destroy(h)
