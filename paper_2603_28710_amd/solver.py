"""Solver: a context of libadg.so with its device buffers held as torch tensors.

torch supplies device memory and the stream; the library does all the work.
"""
import ctypes as C

import numpy as np
import torch

from . import binding as B


def _aligned_empty(nbytes, device):
    """A uint8 device tensor of at least nbytes, 256-byte aligned data pointer."""
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


class Solver:
    def __init__(self, device="cuda:0", stream=None, **cfg):
        asy = {k: cfg.pop(k) for k in ("ghost", "delay_kind", "L", "levels", "seed", "learned_tol", "learned_judge")
               if k in cfg}
        self.cfg = B.make_config(**cfg)
        self.asy = B.make_async(**asy)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = B.adg_create(self.cfg, self.asy, self.stream.cuda_stream)
        self.ndof, sb, rb, scb = B.adg_sizes(self.h)
        self.V = self.cfg.dim + 2
        self.P = self.cfg.degree + 1
        self.E = self.ndof // (self.V * self.P ** self.cfg.dim)
        self.u = [torch.empty(self.ndof, dtype=torch.float64, device=self.device) for _ in range(3)]
        self.ring, ring_ptr = (None, 0)
        if rb:
            self.ring, ring_ptr = _aligned_empty(rb, self.device)
        self.scratch, scr_ptr = _aligned_empty(scb, self.device)
        for t in self.u:
            assert t.data_ptr() % 256 == 0
        B.adg_bind(self.h, self.u[0].data_ptr(), self.u[1].data_ptr(), self.u[2].data_ptr(), ring_ptr, scr_ptr)
        self.ring_bytes, self.scratch_bytes = rb, scb
        self.pairs = None

    def close(self):
        if getattr(self, "h", None):
            B.adg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def state_tensor(self):
        """u_n as a device tensor (public layout)."""
        return self.u[0]

    def upload(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        B.adg_upload(self.h, u.ctypes.data, u.size)

    def download(self):
        u = np.empty(self.ndof, dtype=np.float64)
        B.adg_download(self.h, u.ctypes.data, u.size)
        return u

    def init_problem(self, problem, params=None):
        if params is None:
            B.adg_init_problem(self.h, problem)
        else:
            p = np.ascontiguousarray(params, dtype=np.float64)
            B.adg_init_problem(self.h, problem, p.ctypes.data)

    def set_boundary(self, problem, params=None):
        if params is None:
            B.adg_set_boundary(self.h, problem)
        else:
            p = np.ascontiguousarray(params, dtype=np.float64)
            B.adg_set_boundary(self.h, problem, p.ctypes.data)

    def step(self, n, dt):
        return B.check(B.adg_step(self.h, n, dt))

    def step_status(self, n, dt):
        return B.adg_step(self.h, n, dt)

    def time(self):
        return B.adg_time(self.h)

    def n_face_sides(self):
        """PE-boundary face-sides of the partition (host-only query)"""
        return B.adg_delay(self.h, self.time()[0], 0, 0)[1]

    def stable_dt(self, cfl):
        return B.adg_stable_dt(self.h, cfl)

    def error_norms(self, problem, params=None):
        if params is None:
            return B.adg_error_norms(self.h, problem)
        p = np.ascontiguousarray(params, dtype=np.float64)
        return B.adg_error_norms(self.h, problem, p.ctypes.data)

    def diff_norm(self, ref):
        ref = np.ascontiguousarray(ref, dtype=np.float64)
        return B.adg_diff_norm(self.h, ref.ctypes.data)

    def integrals(self):
        return B.adg_integrals(self.h, self.V)

    def set_async(self, **asy):
        self.asy = B.make_async(**asy)
        B.adg_set_async(self.h, self.asy)

    def save(self):
        return B.adg_save(self.h)

    def load(self, blob):
        B.adg_load(self.h, blob)

    # learned predictor
    def predictor_nparams(self):
        return B.adg_predictor_nparams(self.h)

    def predictor_bind(self, max_pairs):
        pb = B.adg_predictor_pair_bytes(self.h)
        self.pairs = None  # release the previous buffer first
        self.pairs, ptr = _aligned_empty(pb * max_pairs, self.device)
        B.adg_predictor_bind(self.h, ptr, max_pairs)

    def predictor_load_pairs(self, pairs):
        pairs = np.ascontiguousarray(pairs, dtype=np.float32)
        B.adg_predictor_load_pairs(self.h, pairs.ctypes.data, pairs.shape[0])

    def predictor_init(self, seed):
        B.adg_predictor_init(self.h, seed)

    def predictor_grad(self, first, count):
        g = np.zeros(self.predictor_nparams(), dtype=np.float32)
        loss = B.adg_predictor_grad(self.h, first, count, g.ctypes.data)
        return loss, g

    def predictor_infer(self, first, count):
        y = np.zeros(count * self.V, dtype=np.float32)
        B.adg_predictor_infer(self.h, first, count, y.ctypes.data)
        return y.reshape(count, self.V)

    def predictor_collect(self, n_steps, dt):
        return B.adg_predictor_collect(self.h, n_steps, dt)

    def predictor_train(self, epochs, batch, lr, seed):
        return B.adg_predictor_train(self.h, epochs, batch, lr, seed)

    def predictor_get(self):
        w = np.zeros(self.predictor_nparams(), dtype=np.float32)
        B.adg_predictor_get(self.h, w.ctypes.data)
        return w

    def predictor_set(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        B.adg_predictor_set(self.h, w.ctypes.data)

    def predictor_stats(self, trace_errors=False):
        return B.adg_predictor_stats(self.h, trace_errors)
