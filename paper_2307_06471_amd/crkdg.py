"""Thin ctypes binding of libcrkdg.so (include/crkdg.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  The functions
keep the C names; `Solver` is a small convenience wrapper that owns the
torch buffers of one handle.

The library must have been built (paper_2307_06471_amd/build.py); there is
no fallback: a missing library or a call without a HIP device raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libcrkdg.so")

CRKDG_OK, CRKDG_EINVAL, CRKDG_EUNSUPPORTED, CRKDG_ENONPHYSICAL, CRKDG_EHIP, CRKDG_EUNBOUND = \
    0, -1, -2, -3, -4, -5
EQ_ADVECTION, EQ_EULER, EQ_BURGERS = 0, 1, 2
FLUX_UPWIND, FLUX_LLF, FLUX_GODUNOV = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE, BC_DIRICHLET = 0, 1, 2
FP64, FP32_MIXED, FP32_INNER, FP32_INCREMENTS = 0, 1, 2, 3
SCHED_SPLIT, SCHED_FUSED = 0, 1
OP_LOC, OP_DG = 0, 1
IC_CONST, IC_ADV_SIN, IC_EULER_WAVE, IC_VORTEX, IC_QUADRANT, IC_SHOCK = 0, 1, 2, 3, 4, 5
IC_DMR = 6  # double Mach reflection
IC_BURGERS_SIN = 7  # 1D Burgers, u(x, 0) = sin x
RK_FEHLBERG5 = 5  # rk_stages value of the six-stage fifth-order Runge--Kutta--Fehlberg method


class crkdg_mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc", C.c_int * 4), ("bc_state", (C.c_double * 4) * 4), ("bc_exact", C.c_int),
        ("equation", C.c_int), ("adv", C.c_double * 2), ("gamma", C.c_double),
        ("precision", C.c_int),
    ]


class CrkdgError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_LIB = None
EXPORTS = {}


def _sig():
    vp, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.c_size_t
    return {
        "crkdg_create": (C.c_int, [C.POINTER(crkdg_mesh), C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
        "crkdg_set_tableau": (C.c_int, [vp, C.c_int, dp, dp, dp]),
        "crkdg_state_bytes": (sz, [vp]),
        "crkdg_workspace_bytes": (sz, [vp]),
        "crkdg_bind": (C.c_int, [vp, vp, vp, vp]),
        "crkdg_current_dofs": (vp, [vp]),
        "crkdg_set_state": (C.c_int, [vp, dp]),
        "crkdg_get_state": (C.c_int, [vp, dp]),
        "crkdg_set_time": (C.c_int, [vp, C.c_double]),
        "crkdg_get_time": (C.c_double, [vp]),
        "crkdg_project": (C.c_int, [vp, C.c_int, dp, C.c_int, vp]),
        "crkdg_step": (C.c_int, [vp, C.c_double]),
        "crkdg_step_dev": (C.c_int, [vp, vp]),
        "crkdg_set_schedule": (C.c_int, [vp, C.c_int]),
        "crkdg_get_schedule": (C.c_int, [vp]),
        "crkdg_step_rkdg": (C.c_int, [vp, C.c_int, C.c_double, C.c_double, vp]),
        "crkdg_compute_dt": (C.c_int, [vp, C.c_double, vp]),
        "crkdg_max_wavespeed": (C.c_int, [vp, dp]),
        "crkdg_limit": (C.c_int, [vp, C.c_double, vp, C.POINTER(C.c_int64)]),
        "crkdg_limit_dt": (C.c_int, [vp, C.c_double, vp, C.c_float, C.c_float, vp, C.c_double,
                                     vp]),
        "crkdg_error": (C.c_int, [vp, C.c_int, dp, C.c_int, C.c_double, C.c_int, dp]),
        "crkdg_error_ref": (C.c_int, [vp, vp, C.c_int, dp]),
        "crkdg_total": (C.c_int, [vp, C.c_int, dp]),
        "crkdg_apply_op": (C.c_int, [vp, C.c_int, vp, vp, C.c_double]),
        "crkdg_combine": (C.c_int, [vp, vp, vp, C.c_int, dp, C.POINTER(vp)]),
        "crkdg_gauss_rule": (C.c_int, [C.c_int, dp, dp]),
        "crkdg_limit_mlp": (C.c_int, [vp, C.c_double, vp, C.c_float, C.c_float, vp,
                                      C.POINTER(C.c_int64)]),
        "crkdg_mlp_features": (C.c_int, [vp, C.c_double, vp]),
        "crkdg_mlp_work_bytes": (sz, [C.c_int]),
        "crkdg_mlp_forward": (C.c_int, [vp, vp, C.c_int, vp, vp]),
        "crkdg_mlp_grad": (C.c_int, [vp, vp, vp, C.c_int, C.c_float, vp, vp, vp, sz, vp]),
        "crkdg_mlp_grad_noalloc": (C.c_int, [vp, vp, vp, C.c_int, C.c_float, vp, vp, vp]),
        "crkdg_mlp_adam": (C.c_int, [vp, vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float,
                                     C.c_float, vp]),
        "crkdg_profile_begin": (C.c_int, [vp, C.c_int]),
        "crkdg_profile_end": (C.c_int, [vp, dp, C.POINTER(C.c_int64)]),
        "crkdg_destroy": (None, [vp]),
        "crkdg_strerror": (C.c_char_p, [C.c_int]),
    }


def lib():
    """Load libcrkdg.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run paper_2307_06471_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _sig().items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
            EXPORTS[name] = f
        _LIB = L
    return _LIB


def strerror(code):
    return lib().crkdg_strerror(code).decode()


def _check(rc, what):
    if rc != CRKDG_OK:
        raise CrkdgError(rc, what)
    return rc


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def crkdg_gauss_rule(n):
    x, w = np.zeros(n), np.zeros(n)
    _check(lib().crkdg_gauss_rule(n, _dp(x), _dp(w)), "crkdg_gauss_rule")
    return x, w


def make_mesh(dim, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=(0, 0, 0, 0), bc_state=None,
              bc_exact=0, equation=EQ_EULER, adv=(1.0, 0.0), gamma=1.4, precision=FP64):
    m = crkdg_mesh()
    m.dim, m.nx, m.ny = dim, nx, (ny if dim == 2 else 1)
    m.x0, m.x1, m.y0, m.y1 = x0, x1, y0, y1
    for i in range(4):
        m.bc[i] = bc[i]
    if bc_state is not None:
        for s in range(4):
            for c in range(len(bc_state[s])):
                m.bc_state[s][c] = bc_state[s][c]
    m.bc_exact = bc_exact
    m.equation, m.gamma, m.precision = equation, gamma, precision
    m.adv[0], m.adv[1] = adv
    return m


def crkdg_create(mesh, k, flux, rk_stages):
    h = C.c_void_p()
    _check(lib().crkdg_create(C.byref(mesh), k, flux, rk_stages, C.byref(h)), "crkdg_create")
    return h


class Solver:
    """One cRKDG handle with its torch-owned device buffers."""

    def __init__(self, mesh, k, flux, rk_stages, device="cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the cRKDG library needs a HIP device")
        self.torch = torch
        self.mesh = mesh
        self.k = k
        self.dim = mesh.dim
        self.ncomp = 1 if mesh.equation != EQ_EULER else (4 if mesh.dim == 2 else 3)
        self.nmodes = (k + 1) ** 2 if mesh.dim == 2 else k + 1
        self.ncells = mesh.nx * (mesh.ny if mesh.dim == 2 else 1)
        self.h = crkdg_create(mesh, k, flux, rk_stages)
        L = lib()
        self.state_bytes = L.crkdg_state_bytes(self.h)
        self.work_bytes = L.crkdg_workspace_bytes(self.h)
        self.dofs = torch.empty(self.state_bytes + 256, dtype=torch.uint8, device=device)
        self.work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        _check(L.crkdg_bind(self.h, self._aligned(self.dofs), self._aligned(self.work),
                            C.c_void_p(self.stream.cuda_stream)), "crkdg_bind")

    @staticmethod
    def _aligned(t):
        p = t.data_ptr()
        return C.c_void_p((p + 255) // 256 * 256)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().crkdg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def shape(self):
        return (self.ncomp, self.nmodes, self.ncells)

    # -- the C entry points ---------------------------------------------
    def crkdg_set_tableau(self, A, b, c):
        """explicit Butcher tableau (A strictly lower triangular).  The
        Solver binds its workspace at construction for max(4, stages)
        stages, so a five- or six-stage tableau needs a Solver created with
        rk_stages = RK_FEHLBERG5 (CRKDG_EINVAL otherwise)"""
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        _check(lib().crkdg_set_tableau(self.h, len(b), _dp(c), _dp(A), _dp(b)), "crkdg_set_tableau")

    def crkdg_set_state(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.size != self.ncomp * self.nmodes * self.ncells:
            raise ValueError(f"state of shape {u.shape}, expected {self.shape}")
        _check(lib().crkdg_set_state(self.h, _dp(u)), "crkdg_set_state")

    def crkdg_get_state(self):
        u = np.zeros(self.shape)
        _check(lib().crkdg_get_state(self.h, _dp(u)), "crkdg_get_state")
        return u

    def crkdg_current_dofs(self):
        return lib().crkdg_current_dofs(self.h)

    def crkdg_set_time(self, t):
        _check(lib().crkdg_set_time(self.h, t), "crkdg_set_time")

    def crkdg_get_time(self):
        return lib().crkdg_get_time(self.h)

    def crkdg_project(self, ic, params=(), aux=None):
        P = np.ascontiguousarray(params, dtype=np.float64) if len(params) else None
        a = None if aux is None else C.c_void_p(aux.data_ptr())
        _check(lib().crkdg_project(self.h, ic, _dp(P), 0 if P is None else P.size, a),
               "crkdg_project")

    def crkdg_step(self, dt):
        _check(lib().crkdg_step(self.h, float(dt)), "crkdg_step")

    def crkdg_set_schedule(self, sched):
        _check(lib().crkdg_set_schedule(self.h, int(sched)), "crkdg_set_schedule")

    def crkdg_get_schedule(self):
        return lib().crkdg_get_schedule(self.h)

    def crkdg_step_dev(self, dt_tensor):
        _check(lib().crkdg_step_dev(self.h, C.c_void_p(dt_tensor.data_ptr())), "crkdg_step_dev")

    def crkdg_compute_dt(self, cfl, dt_tensor):
        _check(lib().crkdg_compute_dt(self.h, float(cfl), C.c_void_p(dt_tensor.data_ptr())),
               "crkdg_compute_dt")

    def crkdg_max_wavespeed(self):
        s = C.c_double()
        _check(lib().crkdg_max_wavespeed(self.h, C.byref(s)), "crkdg_max_wavespeed")
        return s.value

    def crkdg_step_rkdg(self, order, dt, M=-1.0, dt_tensor=None):
        """one original-RKDG step (SSP order 2 or 3, limiter every stage if
        M >= 0; order 0: Butcher form with the handle's tableau, M < 0);
        dt_tensor: device double that overrides dt"""
        p = None if dt_tensor is None else C.c_void_p(dt_tensor.data_ptr())
        _check(lib().crkdg_step_rkdg(self.h, int(order), float(M), float(dt), p),
               "crkdg_step_rkdg")

    def crkdg_limit(self, M, flags=None, count=True):
        n = C.c_int64(-1)
        f = None if flags is None else C.c_void_p(flags.data_ptr())
        rc = lib().crkdg_limit(self.h, float(M), f, C.byref(n) if count else None)
        _check(rc, "crkdg_limit")
        return n.value if count else None

    def crkdg_limit_dt(self, M, cfl, dt_tensor, flags=None, params=None, tau_lo=0.0, tau_hi=0.0):
        """limiter (TVB, or the learned indicator when params is given) and
        the next step's dt into dt_tensor (1 device double)"""
        f = None if flags is None else C.c_void_p(flags.data_ptr())
        pp = None if params is None else C.c_void_p(params.data_ptr())
        _check(lib().crkdg_limit_dt(self.h, float(M), pp, float(tau_lo), float(tau_hi), f,
                                    float(cfl), C.c_void_p(dt_tensor.data_ptr())),
               "crkdg_limit_dt")

    def crkdg_limit_mlp(self, M, params, tau_lo, tau_hi, flags=None, count=True):
        cnt = (C.c_int64 * 2)(-1, -1)
        f = None if flags is None else C.c_void_p(flags.data_ptr())
        _check(lib().crkdg_limit_mlp(self.h, float(M), C.c_void_p(params.data_ptr()),
                                     float(tau_lo), float(tau_hi), f, cnt if count else None),
               "crkdg_limit_mlp")
        return (cnt[0], cnt[1]) if count else None

    def crkdg_mlp_features(self, M, X=None):
        if X is None:
            X = self.torch.empty((self.ncells, 12), dtype=self.torch.float32, device="cuda")
        _check(lib().crkdg_mlp_features(self.h, float(M), C.c_void_p(X.data_ptr())),
               "crkdg_mlp_features")
        return X

    def crkdg_error(self, ic, params=(), t=0.0, comp=0):
        P = np.ascontiguousarray(params, dtype=np.float64) if len(params) else None
        out = np.zeros(3)
        _check(lib().crkdg_error(self.h, ic, _dp(P), 0 if P is None else P.size, float(t), comp,
                                 _dp(out)), "crkdg_error")
        return out

    def crkdg_error_ref(self, ref, comp=0):
        """errors of this state's cell averages against the finer Solver `ref`
        restricted to this mesh: (L1, L2, Linf)"""
        out = np.zeros(3)
        _check(lib().crkdg_error_ref(self.h, ref.h, comp, _dp(out)), "crkdg_error_ref")
        return out

    def crkdg_total(self, comp=0):
        s = C.c_double()
        _check(lib().crkdg_total(self.h, comp, C.byref(s)), "crkdg_total")
        return s.value

    def crkdg_apply_op(self, op, x, t_bc=0.0):
        """x: torch float64 device tensor of the state's size; returns op(x)"""
        out = self.torch.empty_like(x)
        _check(lib().crkdg_apply_op(self.h, op, C.c_void_p(x.data_ptr()),
                                    C.c_void_p(out.data_ptr()), float(t_bc)), "crkdg_apply_op")
        return out

    def crkdg_combine(self, base, coefs, arrays):
        out = self.torch.empty_like(arrays[0] if base is None else base)
        n = len(arrays)
        cf = np.ascontiguousarray(coefs, dtype=np.float64)
        ptrs = (C.c_void_p * max(n, 1))(*[C.c_void_p(a.data_ptr()) for a in arrays])
        _check(lib().crkdg_combine(self.h, C.c_void_p(out.data_ptr()),
                                   None if base is None else C.c_void_p(base.data_ptr()), n,
                                   _dp(cf), ptrs), "crkdg_combine")
        return out

    KERNEL_CLASSES = ("inner", "final", "loc", "combine", "dt", "limit", "other", "fused")

    def crkdg_profile_begin(self, max_launches):
        _check(lib().crkdg_profile_begin(self.h, int(max_launches)), "crkdg_profile_begin")

    def crkdg_profile_end(self):
        ms = np.zeros(8)
        cnt = np.zeros(8, dtype=np.int64)
        _check(lib().crkdg_profile_end(self.h, _dp(ms),
                                       cnt.ctypes.data_as(C.POINTER(C.c_int64))),
               "crkdg_profile_end")
        return {n: (float(ms[i]), int(cnt[i])) for i, n in enumerate(self.KERNEL_CLASSES)
                if cnt[i]}

    # -- helpers -------------------------------------------------------
    def current_view(self):
        """torch float64 view (ncomp, nmodes, ncells) of the current state"""
        ptr = self.crkdg_current_dofs()
        for buf in (self.dofs, self.work):
            base = buf.data_ptr()
            if base <= ptr < base + buf.numel():
                off = ptr - base
                n = self.ncomp * self.nmodes * self.ncells
                return buf[off:off + 8 * n].view(self.torch.float64).view(self.shape)
        raise RuntimeError("current state pointer outside the bound buffers")


# --- MLP kernels (no mesh) -------------------------------------------------

def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def crkdg_mlp_forward(params, X, stream=None):
    import torch
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib().crkdg_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(out), _stream(stream)),
           "crkdg_mlp_forward")
    return out


def crkdg_mlp_grad(params, X, y, pos_weight, grad=None, loss=None, work=None, stream=None):
    import torch
    B = X.shape[0]
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    nb = lib().crkdg_mlp_work_bytes(B)
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=X.device)
    _check(lib().crkdg_mlp_grad(_ptr(params), _ptr(X), _ptr(y), B, float(pos_weight), _ptr(grad),
                                _ptr(loss), _ptr(work), nb, _stream(stream)), "crkdg_mlp_grad")
    return grad, loss


MLP_NOALLOC_MAX_B = 16384  # CRKDG_MLP_NOALLOC_MAX_B


def crkdg_mlp_grad_noalloc(params, X, y, pos_weight, grad, loss, stream=None):
    """crkdg_mlp_grad with the library's own per-GPU partials buffer (no work
    memory); grad (1505 floats) and loss (1 float) are caller-owned"""
    _check(lib().crkdg_mlp_grad_noalloc(_ptr(params), _ptr(X), _ptr(y), X.shape[0],
                                        float(pos_weight), _ptr(grad), _ptr(loss),
                                        _stream(stream)), "crkdg_mlp_grad_noalloc")
    return grad, loss


def crkdg_mlp_adam(params, m1, m2, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   stream=None):
    _check(lib().crkdg_mlp_adam(_ptr(params), _ptr(m1), _ptr(m2), _ptr(grad), int(step),
                                float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
           "crkdg_mlp_adam")
