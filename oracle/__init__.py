"""ctypes wrapper of the serial FP64 CPU oracle (oracle/crkdg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path (paper_2307_06471_amd) never
imports this package.

Arrays use the exchange layout u[comp][mode][cell] (cell = j*nx + i, mode
m + (k+1) n), float64, C-contiguous.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

EQ_ADVECTION, EQ_EULER, EQ_BURGERS = 0, 1, 2
FLUX_UPWIND, FLUX_LLF, FLUX_GODUNOV = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE, BC_DIRICHLET = 0, 1, 2
OP_LOC, OP_DG = 0, 1
IC_CONST, IC_ADV_SIN, IC_EULER_WAVE, IC_VORTEX, IC_QUADRANT, IC_SHOCK = 0, 1, 2, 3, 4, 5
IC_DMR = 7  # double Mach reflection (Section 4)
IC_BURGERS_SIN = 8  # 1D Burgers, u(x, 0) = sin x (Section 4.1.1)

N_MLP_PARAMS = 12 * 32 + 32 + 32 * 32 + 32 + 32 + 1


class _Mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc", C.c_int * 4), ("bc_state", (C.c_double * 4) * 4), ("bc_exact", C.c_int),
        ("equation", C.c_int), ("adv", C.c_double * 2), ("gamma", C.c_double),
        ("flux", C.c_int), ("ic_params", C.POINTER(C.c_double)),
    ]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        mp = C.POINTER(_Mesh)
        u8 = C.POINTER(C.c_uint8)
        sig = {
            "or_gauss": (C.c_int, [C.c_int, dp, dp]),
            "or_legendre": (C.c_double, [C.c_int, C.c_double]),
            "or_dlegendre": (C.c_double, [C.c_int, C.c_double]),
            "or_ncomp": (C.c_int, [mp]),
            "or_nmodes": (C.c_int, [mp, C.c_int]),
            "or_project": (C.c_int, [mp, C.c_int, C.c_int, dp, dp, C.c_double, dp]),
            "or_apply": (C.c_int, [mp, C.c_int, C.c_int, C.c_double, dp, dp]),
            "or_step_crkdg": (C.c_int, [mp, C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp]),
            "or_step_rkdg": (C.c_int, [mp, C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp]),
            "or_step_rkdg_ssp": (C.c_int, [mp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp]),
            "or_step_wrong_ssp": (C.c_int, [mp, C.c_int, C.c_int, C.c_double, C.c_double, dp]),
            "or_crkdg_stages": (C.c_int, [mp, C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp, dp]),
            "or_limit_tvb": (C.c_int64, [mp, C.c_int, C.c_double, dp, u8]),
            "or_tvb_flags": (C.c_int64, [mp, C.c_int, C.c_double, dp, u8, dp]),
            "or_limit_tvb_at": (C.c_int64, [mp, C.c_int, C.c_double, C.c_double, dp, u8]),
            "or_tvb_flags_at": (C.c_int64, [mp, C.c_int, C.c_double, C.c_double, dp, u8, dp]),
            "or_dmr_states": (None, [C.c_double, dp, dp, dp]),
            "or_euler_eig": (C.c_int, [mp, dp, C.c_int, dp, dp]),
            "or_max_wavespeed": (C.c_double, [mp, C.c_int, dp]),
            "or_errors": (C.c_int, [mp, C.c_int, dp, C.c_int, dp, dp, C.c_double, C.c_int, dp]),
            "or_errors_vs_avg": (C.c_int, [mp, C.c_int, dp, dp, C.c_int, dp]),
            "or_total_mass": (C.c_double, [mp, C.c_int, dp, C.c_int]),
            "or_mlp_features": (C.c_int, [mp, C.c_int, C.c_double, dp, dp]),
            "or_mlp_forward": (C.c_int, [dp, dp, C.c_int, dp]),
            "or_mlp_loss_grad": (C.c_double, [dp, dp, u8, C.c_int, C.c_double, dp]),
            "or_adam": (C.c_int, [dp, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


class Mesh:
    """Oracle-side description of the mesh, equation, flux and boundary data."""

    def __init__(self, dim, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=(0, 0, 0, 0),
                 bc_state=None, bc_exact=0, ic_params=None, equation=EQ_EULER,
                 adv=(1.0, 0.0), gamma=1.4, flux=FLUX_LLF):
        m = _Mesh()
        m.dim, m.nx, m.ny = dim, nx, (ny if dim == 2 else 1)
        m.x0, m.x1, m.y0, m.y1 = x0, x1, y0, y1
        for i in range(4):
            m.bc[i] = bc[i]
        if bc_state is not None:
            for s in range(4):
                for c in range(len(bc_state[s])):
                    m.bc_state[s][c] = bc_state[s][c]
        m.bc_exact = bc_exact
        self._icp = None
        if ic_params is not None:
            self._icp = np.ascontiguousarray(ic_params, dtype=np.float64)
            m.ic_params = _d(self._icp)
        m.equation, m.gamma, m.flux = equation, gamma, flux
        m.adv[0], m.adv[1] = adv
        self.m = m
        self.dim, self.nx, self.ny = dim, nx, m.ny
        self.equation = equation

    @property
    def ref(self):
        return C.byref(self.m)

    @property
    def ncells(self):
        return self.nx * self.ny

    def ncomp(self):
        return lib().or_ncomp(self.ref)

    def nmodes(self, k):
        return lib().or_nmodes(self.ref, k)

    def shape(self, k):
        return (self.ncomp(), self.nmodes(k), self.ncells)

    def zeros(self, k):
        return np.zeros(self.shape(k), dtype=np.float64)


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    assert lib().or_gauss(n, _d(x), _d(w)) == 0
    return x, w


def legendre(m, x):
    return lib().or_legendre(m, float(x))


def dlegendre(m, x):
    return lib().or_dlegendre(m, float(x))


NPARAM = 24  # initial-condition parameters; unused trailing ones are zero


def _params(params):
    p = np.zeros(NPARAM)
    v = np.asarray(params, dtype=np.float64).ravel()
    assert v.size <= NPARAM
    p[:v.size] = v
    return p


def project(mesh, k, ic, params=None, aux=None, t=0.0):
    u = mesh.zeros(k)
    p = None if params is None else _params(params)
    a = None if aux is None else np.ascontiguousarray(aux, dtype=np.float64)
    assert lib().or_project(mesh.ref, k, ic, _d(p), _d(a), t, _d(u)) == 0
    return u


def apply(mesh, k, op, u, t_bc=0.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    rc = lib().or_apply(mesh.ref, k, op, t_bc, _d(u), _d(out))
    if rc:
        raise ValueError(f"or_apply failed: {rc}")
    return out


def _tab(A, b, c):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return A, b, c, len(b)


def step_crkdg(mesh, k, tableau, t, dt, u):
    A, b, c, s = _tab(*tableau)
    u = np.array(u, dtype=np.float64, order="C")
    rc = lib().or_step_crkdg(mesh.ref, k, s, _d(A), _d(b), _d(c), t, dt, _d(u))
    if rc:
        raise ValueError(f"or_step_crkdg failed: {rc}")
    return u


def crkdg_stages(mesh, k, tableau, t, dt, u):
    A, b, c, s = _tab(*tableau)
    u = np.ascontiguousarray(u, dtype=np.float64)
    st = np.zeros((s,) + u.shape)
    rc = lib().or_crkdg_stages(mesh.ref, k, s, _d(A), _d(b), _d(c), t, dt, _d(u), _d(st))
    if rc:
        raise ValueError(rc)
    return st


def step_rkdg(mesh, k, tableau, t, dt, u):
    A, b, c, s = _tab(*tableau)
    u = np.array(u, dtype=np.float64, order="C")
    rc = lib().or_step_rkdg(mesh.ref, k, s, _d(A), _d(b), _d(c), t, dt, _d(u))
    if rc:
        raise ValueError(rc)
    return u


def step_rkdg_ssp(mesh, k, order, t, dt, u, M=-1.0):
    u = np.array(u, dtype=np.float64, order="C")
    rc = lib().or_step_rkdg_ssp(mesh.ref, k, order, t, dt, M, _d(u))
    if rc:
        raise ValueError(rc)
    return u


def step_wrong_ssp(mesh, k, order, t, dt, u):
    u = np.array(u, dtype=np.float64, order="C")
    rc = lib().or_step_wrong_ssp(mesh.ref, k, order, t, dt, _d(u))
    if rc:
        raise ValueError(rc)
    return u


def limit_tvb(mesh, k, M, u, t=0.0):
    """t: time of time-dependent ghost data (double Mach reflection)"""
    u = np.array(u, dtype=np.float64, order="C")
    flags = np.zeros(mesh.ncells, dtype=np.uint8)
    n = lib().or_limit_tvb_at(mesh.ref, k, M, t, _d(u), _u8(flags))
    return u, flags, n


def tvb_flags(mesh, k, M, u, t=0.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    flags = np.zeros(mesh.ncells, dtype=np.uint8)
    margin = np.zeros(mesh.ncells)
    n = lib().or_tvb_flags_at(mesh.ref, k, M, t, _d(u), _u8(flags), _d(margin))
    return flags, margin, n


def dmr_states(gamma=1.4):
    """double Mach reflection: (pre-shock, post-shock) conserved states and
    the shock speed"""
    pre, post, S = np.zeros(4), np.zeros(4), np.zeros(1)
    lib().or_dmr_states(gamma, _d(pre), _d(post), _d(S))
    return pre, post, float(S[0])


def euler_eig(mesh, q, d):
    nc = mesh.ncomp()
    q = np.ascontiguousarray(q, dtype=np.float64)
    L = np.zeros(nc * nc)
    R = np.zeros(nc * nc)
    lib().or_euler_eig(mesh.ref, _d(q), d, _d(L), _d(R))
    return L.reshape(nc, nc), R.reshape(nc, nc)


def max_wavespeed(mesh, k, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().or_max_wavespeed(mesh.ref, k, _d(u))


def errors(mesh, k, u, ic, params=None, aux=None, t=0.0, comp=0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(3)
    p = None if params is None else _params(params)
    a = None if aux is None else np.ascontiguousarray(aux, dtype=np.float64)
    lib().or_errors(mesh.ref, k, _d(u), ic, _d(p), _d(a), t, comp, _d(out))
    return out


def errors_vs_avg(mesh, k, u, ref_avg, comp=0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    r = np.ascontiguousarray(ref_avg, dtype=np.float64)
    out = np.zeros(3)
    lib().or_errors_vs_avg(mesh.ref, k, _d(u), _d(r), comp, _d(out))
    return out


def total_mass(mesh, k, u, comp=0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().or_total_mass(mesh.ref, k, _d(u), comp)


def mlp_features(mesh, k, M, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    X = np.zeros((mesh.ncells, 12))
    assert lib().or_mlp_features(mesh.ref, k, M, _d(u), _d(X)) == 0
    return X


def mlp_forward(params, X):
    params = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros(X.shape[0])
    lib().or_mlp_forward(_d(params), _d(X), X.shape[0], _d(out))
    return out


def mlp_loss_grad(params, X, y, pos_weight=1.0):
    params = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    g = np.zeros(N_MLP_PARAMS)
    loss = lib().or_mlp_loss_grad(_d(params), _d(X), _u8(y), X.shape[0], pos_weight, _d(g))
    return loss, g


def adam(params, m1, m2, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    for a in (params, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    lib().or_adam(_d(params), _d(m1), _d(m2), _d(grad), params.size, step, lr, b1, b2, eps)
