"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke entry and the CPU
baseline leg of the benchmark. The GPU library never imports this module.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

SYNC, STALE, AT, LEARNED, FLUX_STALE, FLUX_AT = 0, 1, 2, 3, 4, 5
FIXED, UNIFORM, CAA = 0, 1, 2
VORTEX, DENSITY_WAVE, CONSTANT = 0, 1, 2
LLF, RUSANOV = 0, 1
SSPRK3, LSERK22, LSERK33, SSPRK2 = 0, 1, 2, 3
PERIODIC, DIRICHLET = 0, 1


class OrcCfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("p", C.c_int32), ("nq", C.c_int32),
        ("cells", C.c_int32 * 3), ("parts", C.c_int32 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("gamma", C.c_double), ("flux", C.c_int32), ("ghost", C.c_int32),
        ("delay_kind", C.c_int32), ("L", C.c_int32), ("levels", C.c_int32),
        ("seed", C.c_uint64), ("learned_tol", C.c_double), ("integrator", C.c_int32),
        ("bc", C.c_int32), ("bc_problem", C.c_int32), ("bc_prm_set", C.c_int32),
        ("bc_prm", C.c_double * 5), ("learned_judge", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.orc_gauss.argtypes = [C.c_int, dp, dp]
        L.orc_gll.argtypes = [C.c_int, dp, dp]
        L.orc_lagrange.argtypes = [C.c_int, dp, C.c_double, dp, dp]
        L.orc_at_weights.argtypes = [C.c_int, C.c_double, dp]
        L.orc_splitmix64_draw.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix64_draw.restype = C.c_uint64
        L.orc_create.argtypes = [C.POINTER(OrcCfg)]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_ndof.argtypes = [vp]
        L.orc_ndof.restype = C.c_int64
        L.orc_nface_sides.argtypes = [vp]
        L.orc_nface_sides.restype = C.c_int64
        L.orc_set_state.argtypes = [vp, dp]
        L.orc_get_state.argtypes = [vp, dp]
        L.orc_init_problem.argtypes = [vp, C.c_int, dp]
        L.orc_step.argtypes = [vp, C.c_int64, C.c_double]
        L.orc_time.argtypes = [vp, C.POINTER(C.c_int64), dp]
        L.orc_rhs.argtypes = [vp, dp, dp]
        L.orc_stage_elements.argtypes = [vp, C.c_int, C.c_double, dp, dp, C.c_int64,
                                         C.POINTER(C.c_int64), dp]
        L.orc_error_norms.argtypes = [vp, C.c_int, dp, C.c_double, dp]
        L.orc_integrals.argtypes = [vp, dp]
        L.orc_delay.argtypes = [vp, C.c_int64, C.c_int64, C.c_int]
        L.orc_subdomain.argtypes = [vp, C.c_int64]
        L.orc_subdomain.restype = C.c_int64
        L.orc_stable_dt.argtypes = [vp, C.c_double]
        L.orc_stable_dt.restype = C.c_double
        L.orc_mlp_nparams.argtypes = [C.c_int] * 3
        L.orc_mlp_forward.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int64, dp, dp]
        L.orc_mlp_forward_bf16.argtypes = [C.POINTER(C.c_float), C.c_int, C.c_int, C.c_int, C.c_int64, dp, dp]
        L.orc_mlp_loss_grad.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int64, dp, dp, dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_adam.argtypes = [dp, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_int64]
        L.orc_set_predictor.argtypes = [vp, C.POINTER(C.c_float)]
        L.orc_learned_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_learned_features.argtypes = [vp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_numerical_flux.argtypes = [vp, dp, dp, C.c_int, C.c_double, dp]
        L.orc_record_pairs.argtypes = [vp, dp, C.c_int64]
        L.orc_recorded_pairs.argtypes = [vp]
        L.orc_recorded_pairs.restype = C.c_int64
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def gauss(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gauss(n, _dp(x), _dp(w))
    return x, w


def gll(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gll(n, _dp(x), _dp(w))
    return x, w


def lagrange(nodes, x):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    n = len(nodes)
    phi = np.zeros(n); dphi = np.zeros(n)
    lib().orc_lagrange(n, _dp(nodes), float(x), _dp(phi), _dp(dphi))
    return phi, dphi


def at_weights(nlev, tau):
    c = np.zeros(nlev)
    rc = lib().orc_at_weights(nlev, float(tau), _dp(c))
    assert rc == 0
    return c


def splitmix64_draw(seed, index):
    return int(lib().orc_splitmix64_draw(seed, index))


def set_threads(n):
    """Limit OpenMP threads of the oracle (for the timed CPU baseline)."""
    os.environ["OMP_NUM_THREADS"] = str(n)


class Oracle:
    """FP64 CPU ADG solver. `cfg` keys mirror the GPU library's config."""

    def __init__(self, dim=2, p=2, nq=0, cells=(16, 16, 1), parts=(1, 1, 1), lo=(0, 0, 0),
                 hi=(10, 10, 1), gamma=1.4, flux=LLF, ghost=SYNC, delay_kind=FIXED, L=0, levels=3,
                 seed=0, learned_tol=1e-6, integrator=0, bc=0, bc_problem=0, bc_params=None, learned_judge=1):
        c = OrcCfg()
        c.dim, c.p, c.nq = dim, p, nq
        for k in range(3):
            c.cells[k] = int(cells[k]) if k < len(cells) else 1
            c.parts[k] = int(parts[k]) if k < len(parts) else 1
            c.lo[k] = float(lo[k]) if k < len(lo) else 0.0
            c.hi[k] = float(hi[k]) if k < len(hi) else 1.0
        c.gamma, c.flux, c.ghost, c.delay_kind = gamma, flux, ghost, delay_kind
        c.L, c.levels, c.seed, c.learned_tol = L, levels, seed, learned_tol
        c.integrator = integrator
        # bc = 1: Dirichlet box, the exterior state of each boundary face is
        # the exact solution of bc_problem (bc_params, or its defaults)
        c.bc, c.bc_problem = bc, bc_problem
        c.bc_prm_set = 0 if bc_params is None else 1
        c.learned_judge = learned_judge
        if bc_params is not None:
            for i in range(5):
                c.bc_prm[i] = float(bc_params[i])
        self.cfg = c
        self.dim, self.p = dim, p
        self.P = p + 1
        self.V = dim + 2
        self.ptr = lib().orc_create(C.byref(c))
        if not self.ptr:
            raise ValueError("invalid oracle configuration")
        self.ndof = lib().orc_ndof(self.ptr)
        self.E = self.ndof // (self.V * self.P ** dim)

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_destroy(self.ptr)
            self.ptr = None

    def state(self):
        u = np.zeros(self.ndof)
        lib().orc_get_state(self.ptr, _dp(u))
        return u

    def set_state(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.size == self.ndof
        lib().orc_set_state(self.ptr, _dp(u))

    def init_problem(self, problem, params=None):
        if params is None:
            lib().orc_init_problem(self.ptr, problem, None)
        else:
            pr = np.ascontiguousarray(params, dtype=np.float64)
            lib().orc_init_problem(self.ptr, problem, _dp(pr))

    def step(self, n, dt):
        return lib().orc_step(self.ptr, int(n), float(dt))

    def time(self):
        n = C.c_int64(); t = C.c_double()
        lib().orc_time(self.ptr, C.byref(n), C.byref(t))
        return n.value, t.value

    def rhs(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(self.ndof)
        lib().orc_rhs(self.ptr, _dp(u), _dp(out))
        return out

    def stage_elements(self, stage, dt, u_in, u_n, elems):
        u_in = np.ascontiguousarray(u_in, dtype=np.float64)
        u_n = np.ascontiguousarray(u_n, dtype=np.float64)
        el = np.ascontiguousarray(elems, dtype=np.int64)
        out = np.zeros(len(el) * self.V * self.P ** self.dim)
        lib().orc_stage_elements(self.ptr, stage, float(dt), _dp(u_in), _dp(u_n), len(el),
                                 el.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
        return out

    def error_norms(self, problem, t, params=None):
        out = np.zeros(3)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        lib().orc_error_norms(self.ptr, problem, None if pr is None else _dp(pr), float(t), _dp(out))
        return out

    def integrals(self):
        out = np.zeros(self.V)
        lib().orc_integrals(self.ptr, _dp(out))
        return out

    def delay(self, n, sub, d):
        return lib().orc_delay(self.ptr, n, sub, d)

    def subdomain(self, e):
        return lib().orc_subdomain(self.ptr, e)

    def n_face_sides(self):
        return lib().orc_nface_sides(self.ptr)

    def stable_dt(self, cfl):
        return lib().orc_stable_dt(self.ptr, cfl)

    def set_predictor(self, w):
        if w is None:
            lib().orc_set_predictor(self.ptr, None)
        else:
            w = np.ascontiguousarray(w, dtype=np.float32)
            lib().orc_set_predictor(self.ptr, w.ctypes.data_as(C.POINTER(C.c_float)))

    def learned_stats(self):
        a = C.c_int64(); r = C.c_int64()
        lib().orc_learned_stats(self.ptr, C.byref(a), C.byref(r))
        return a.value, r.value

    def numerical_flux(self, wm, wp, a, sigma):
        """n.F^ for n = sigma e_a seen from the side holding wm, with this
        solver's gamma and flux kind"""
        wm = np.ascontiguousarray(wm, dtype=np.float64)
        wp = np.ascontiguousarray(wp, dtype=np.float64)
        assert wm.size == self.V and wp.size == self.V
        out = np.zeros(self.V)
        lib().orc_numerical_flux(self.ptr, _dp(wm), _dp(wp), int(a), float(sigma), _dp(out))
        return out

    def record_pairs(self, cap):
        """start recording the learned mode's training pairs (cap records)"""
        self._rec = np.zeros((cap, 6 + 2 * self.V + 2 + self.V))
        lib().orc_record_pairs(self.ptr, _dp(self._rec), int(cap))

    def recorded_pairs(self):
        """stop recording; rows (step, stage, element, face, node, k,
        features..., (live - AT) / S ...) in thread order"""
        n = min(lib().orc_recorded_pairs(self.ptr), len(self._rec))
        lib().orc_record_pairs(self.ptr, None, 0)
        out, self._rec = self._rec[:n].copy(), None
        return out

    def learned_features(self, T, tau, cm):
        T = np.ascontiguousarray(T, dtype=np.float64)
        x = np.zeros(2 * self.V + 2); s2 = C.c_double()
        lib().orc_learned_features(self.ptr, _dp(T), float(tau), float(cm), _dp(x), C.byref(s2))
        return x, s2.value


def mlp_nparams(nin, nh, nout):
    return lib().orc_mlp_nparams(nin, nh, nout)


def mlp_forward(w, nin, nh, nout, x):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.size // nin
    y = np.zeros(n * nout)
    lib().orc_mlp_forward(_dp(w), nin, nh, nout, n, _dp(x), _dp(y))
    return y.reshape(n, nout)


def mlp_forward_bf16(w32, nin, nh, nout, x):
    """forward pass in the precision of the GPU inference (bf16 operands)"""
    w32 = np.ascontiguousarray(w32, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.size // nin
    y = np.zeros(n * nout)
    lib().orc_mlp_forward_bf16(w32.ctypes.data_as(C.POINTER(C.c_float)), nin, nh, nout, n, _dp(x), _dp(y))
    return y.reshape(n, nout)


def mlp_loss_grad(w, nin, nh, nout, x, y):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.size // nin
    g = np.zeros_like(w)
    loss = lib().orc_mlp_loss_grad(_dp(w), nin, nh, nout, n, _dp(x), _dp(y), _dp(g))
    return loss, g


def adam(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam(_dp(w), _dp(m), _dp(v), _dp(g), w.size, lr, b1, b2, eps, t)
