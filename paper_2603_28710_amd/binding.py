"""ctypes binding of libadg.so (include/adg.h), same names as the C ABI.

Argument marshalling only: every step of the solver runs in the library's HIP
kernels. PyTorch provides the device buffers (tensors) and the stream. If the
library has not been built this module raises at import: there is no CPU
fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadg.so")

ADG_OK = 0
ADG_ERR_INVALID, ADG_ERR_UNBOUND, ADG_ERR_HIP = -1, -2, -3
ADG_ERR_NONFINITE, ADG_ERR_NONPHYSICAL, ADG_ERR_STATE = -4, -5, -6
ADG_FLUX_LLF, ADG_FLUX_RUSANOV = 0, 1
ADG_SSPRK3, ADG_LSERK22, ADG_LSERK33, ADG_SSPRK2 = 0, 1, 2, 3
ADG_FP64, ADG_FP32_CONTRACT = 0, 1
ADG_GHOST_SYNC, ADG_GHOST_STALE, ADG_GHOST_AT, ADG_GHOST_LEARNED = 0, 1, 2, 3
ADG_GHOST_FLUX_STALE, ADG_GHOST_FLUX_AT = 4, 5
ADG_DELAY_FIXED, ADG_DELAY_UNIFORM, ADG_DELAY_CAA = 0, 1, 2
ADG_VORTEX, ADG_DENSITY_WAVE, ADG_CONSTANT = 0, 1, 2
ADG_BC_PERIODIC, ADG_BC_DIRICHLET = 0, 1


class adg_config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("n_q", C.c_int32),
                ("cells", C.c_int32 * 3), ("parts", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("gamma", C.c_double),
                ("flux", C.c_int32), ("integrator", C.c_int32), ("precision", C.c_int32),
                ("check_every", C.c_int32), ("boundary", C.c_int32)]


class adg_async(C.Structure):
    _fields_ = [("ghost", C.c_int32), ("delay_kind", C.c_int32), ("L", C.c_int32),
                ("levels", C.c_int32), ("seed", C.c_uint64), ("learned_tol", C.c_double),
                ("learned_judge", C.c_int32)]


class AdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adg error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_28710_amd/build.py "
                      "(there is no CPU fallback)")

lib = C.CDLL(LIB_PATH)
_vp, _dp, _fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float)
_sz = C.POINTER(C.c_size_t)
_SIGS = {
    "adg_create": [C.POINTER(adg_config), C.POINTER(adg_async), _vp, C.POINTER(_vp)],
    "adg_sizes": [_vp, _sz, _sz, _sz, _sz],
    "adg_bind": [_vp, _vp, _vp, _vp, _vp, _vp],
    "adg_upload": [_vp, _dp, C.c_size_t],
    "adg_download": [_vp, _dp, C.c_size_t],
    "adg_init_problem": [_vp, C.c_int32, _dp],
    "adg_set_boundary": [_vp, C.c_int32, _dp],
    "adg_set_async": [_vp, C.POINTER(adg_async)],
    "adg_step": [_vp, C.c_int64, C.c_double],
    "adg_time": [_vp, C.POINTER(C.c_int64), _dp],
    "adg_delay": [_vp, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
    "adg_stable_dt": [_vp, C.c_double, _dp],
    "adg_basis": [_vp, _dp, _dp, _dp, _dp],
    "adg_profile": [_vp, C.c_int32],
    "adg_profile_read": [_vp, C.c_int32, _dp, C.POINTER(C.c_int64)],
    "adg_error_norms": [_vp, C.c_int32, _dp, _dp],
    "adg_diff_norm": [_vp, _dp, _dp],
    "adg_integrals": [_vp, _dp],
    "adg_integrals_noalloc": [_vp, _dp],
    "adg_save": [_vp, _vp, _sz],
    "adg_load": [_vp, _vp, C.c_size_t],
    "adg_predictor_nparams": [_vp, C.POINTER(C.c_int32)],
    "adg_predictor_pair_bytes": [_vp, _sz],
    "adg_predictor_bind": [_vp, _vp, C.c_int64],
    "adg_predictor_load_pairs": [_vp, _fp, C.c_int64],
    "adg_predictor_init": [_vp, C.c_uint64],
    "adg_predictor_grad": [_vp, C.c_int64, C.c_int64, _fp, _fp],
    "adg_predictor_infer": [_vp, C.c_int64, C.c_int64, _fp],
    "adg_predictor_collect": [_vp, C.c_int64, C.c_double, C.POINTER(C.c_int64)],
    "adg_predictor_train": [_vp, C.c_int32, C.c_int32, C.c_float, C.c_uint64, _fp],
    "adg_predictor_get": [_vp, _fp],
    "adg_predictor_set": [_vp, _fp],
    "adg_predictor_stats": [_vp, _dp, C.POINTER(C.c_int64), _dp, _dp],
    "adg_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int32
lib.adg_last_error.argtypes = []
lib.adg_last_error.restype = C.c_char_p


def check(code):
    if code != ADG_OK:
        raise AdgError(code, lib.adg_last_error().decode())
    return code


def _call(name, *args):
    return check(getattr(lib, name)(*args))


# thin wrappers with the C names ------------------------------------------------

def adg_create(cfg, asy, stream=None):
    h = _vp()
    _call("adg_create", C.byref(cfg), C.byref(asy), _vp(stream or 0), C.byref(h))
    return h


def adg_sizes(h):
    a, b, c, d = C.c_size_t(), C.c_size_t(), C.c_size_t(), C.c_size_t()
    _call("adg_sizes", h, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
    return a.value, b.value, c.value, d.value


def adg_bind(h, u_n, u_a, u_b, ring, scratch):
    _call("adg_bind", h, _vp(u_n), _vp(u_a), _vp(u_b), _vp(ring or 0), _vp(scratch))


def adg_upload(h, host_ptr, n):
    _call("adg_upload", h, C.cast(host_ptr, _dp), n)


def adg_download(h, host_ptr, n):
    _call("adg_download", h, C.cast(host_ptr, _dp), n)


def adg_init_problem(h, problem, params_ptr=None):
    _call("adg_init_problem", h, problem, C.cast(params_ptr, _dp) if params_ptr else None)


def adg_set_boundary(h, problem, params_ptr=None):
    _call("adg_set_boundary", h, problem, C.cast(params_ptr, _dp) if params_ptr else None)


def adg_set_async(h, asy):
    _call("adg_set_async", h, C.byref(asy))


def adg_step(h, n_steps, dt):
    return getattr(lib, "adg_step")(h, int(n_steps), float(dt))


def adg_time(h):
    n, t = C.c_int64(), C.c_double()
    _call("adg_time", h, C.byref(n), C.byref(t))
    return n.value, t.value


def adg_delay(h, n, sub, d):
    k, nfs = C.c_int32(), C.c_int64()
    _call("adg_delay", h, int(n), int(sub), int(d), C.byref(k), C.byref(nfs))
    return k.value, nfs.value


def adg_basis(h, P, Q):
    xl, wl, xg, wg = (C.c_double * P)(), (C.c_double * P)(), (C.c_double * Q)(), (C.c_double * Q)()
    _call("adg_basis", h, xl, wl, xg, wg)
    return list(xl), list(wl), list(xg), list(wg)


ADG_KERNEL_RHS, ADG_KERNEL_GHOST = 0, 1


def adg_profile(h, enable):
    _call("adg_profile", h, int(enable))


def adg_profile_read(h, kernel):
    ms, n = C.c_double(), C.c_int64()
    _call("adg_profile_read", h, int(kernel), C.byref(ms), C.byref(n))
    return ms.value, n.value


def adg_stable_dt(h, cfl):
    dt = C.c_double()
    _call("adg_stable_dt", h, float(cfl), C.byref(dt))
    return dt.value


def adg_error_norms(h, problem, params_ptr=None):
    out = (C.c_double * 3)()
    _call("adg_error_norms", h, problem, C.cast(params_ptr, _dp) if params_ptr else None, out)
    return list(out)


def adg_diff_norm(h, host_ref_ptr):
    out = (C.c_double * 3)()
    _call("adg_diff_norm", h, C.cast(host_ref_ptr, _dp), out)
    return list(out)


def adg_integrals(h, V):
    out = (C.c_double * V)()
    _call("adg_integrals", h, out)
    return list(out)


def adg_integrals_noalloc(h, V):
    out = (C.c_double * V)()
    _call("adg_integrals_noalloc", h, out)
    return list(out)


def adg_save(h):
    n = C.c_size_t()
    _call("adg_save", h, None, C.byref(n))
    buf = C.create_string_buffer(n.value)
    _call("adg_save", h, buf, C.byref(n))
    return buf.raw[: n.value]


def adg_load(h, blob):
    buf = C.create_string_buffer(blob, len(blob))
    _call("adg_load", h, buf, len(blob))


def adg_predictor_nparams(h):
    n = C.c_int32()
    _call("adg_predictor_nparams", h, C.byref(n))
    return n.value


def adg_predictor_pair_bytes(h):
    n = C.c_size_t()
    _call("adg_predictor_pair_bytes", h, C.byref(n))
    return n.value


def adg_predictor_bind(h, pairs_ptr, max_pairs):
    _call("adg_predictor_bind", h, _vp(pairs_ptr or 0), int(max_pairs))


def adg_predictor_load_pairs(h, host_ptr, n):
    _call("adg_predictor_load_pairs", h, C.cast(host_ptr, _fp), int(n))


def adg_predictor_init(h, seed):
    _call("adg_predictor_init", h, int(seed))


def adg_predictor_grad(h, first, count, grad_ptr):
    loss = C.c_float()
    _call("adg_predictor_grad", h, int(first), int(count), C.cast(grad_ptr, _fp), C.byref(loss))
    return loss.value


def adg_predictor_infer(h, first, count, y_ptr):
    _call("adg_predictor_infer", h, int(first), int(count), C.cast(y_ptr, _fp))


def adg_predictor_collect(h, n_steps, dt):
    n = C.c_int64()
    _call("adg_predictor_collect", h, int(n_steps), float(dt), C.byref(n))
    return n.value


def adg_predictor_train(h, epochs, batch, lr, seed):
    loss = C.c_float()
    _call("adg_predictor_train", h, int(epochs), int(batch), float(lr), int(seed), C.byref(loss))
    return loss.value


def adg_predictor_get(h, w_ptr):
    _call("adg_predictor_get", h, C.cast(w_ptr, _fp))


def adg_predictor_set(h, w_ptr):
    _call("adg_predictor_set", h, C.cast(w_ptr, _fp))


def adg_predictor_stats(h, trace_errors=False):
    """(accept rate, faces judged), and with trace_errors=True also the mean
    trace error of the ghosts used and of AT against the live values"""
    r, n, te, ta = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    _call("adg_predictor_stats", h, C.byref(r), C.byref(n), C.byref(te), C.byref(ta))
    if trace_errors:
        return r.value, n.value, te.value, ta.value
    return r.value, n.value


def adg_destroy(h):
    _call("adg_destroy", h)


def adg_last_error():
    return lib.adg_last_error().decode()


def make_config(dim=2, degree=2, cells=(16, 16, 1), parts=(1, 1, 1), lo=(0, 0, 0), hi=(10, 10, 1),
                gamma=1.4, flux=ADG_FLUX_LLF, precision=ADG_FP64, check_every=0, n_q=0, integrator=ADG_SSPRK3,
                boundary=ADG_BC_PERIODIC):
    c = adg_config()
    c.dim, c.degree, c.n_q = dim, degree, n_q
    for k in range(3):
        c.cells[k] = int(cells[k]) if k < len(cells) else 1
        c.parts[k] = int(parts[k]) if k < len(parts) else 1
        c.lo[k] = float(lo[k]) if k < len(lo) else 0.0
        c.hi[k] = float(hi[k]) if k < len(hi) else 1.0
    c.gamma, c.flux, c.integrator, c.precision, c.check_every = gamma, flux, integrator, precision, check_every
    c.boundary = boundary
    return c


def make_async(ghost=ADG_GHOST_SYNC, delay_kind=ADG_DELAY_FIXED, L=0, levels=3, seed=0, learned_tol=1e-6,
               learned_judge=1):
    """asynchrony settings; the learned judge defaults to 1: a face's
    correction must stay within the accept bound and within AT's own error
    estimate on the face"""
    a = adg_async()
    a.ghost, a.delay_kind, a.L, a.levels, a.seed, a.learned_tol = ghost, delay_kind, L, levels, seed, learned_tol
    a.learned_judge = learned_judge
    return a
