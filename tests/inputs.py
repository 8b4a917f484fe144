"""Seeded synthetic inputs shared by the oracle and GPU tests.

Holds no arithmetic of the method: only configurations (sizes mirroring the
paper's and the benchmark's workloads) and seeded random perturbations.
"""
import numpy as np

# Workload configurations (mesh, degree, decomposition, asynchrony).
# vortex: periodic [0,10]^2 isentropic vortex with mean flow (1,1);
# density wave: periodic unit cube, rho = 1 + 0.2 sin(2 pi (x+y+z-3t)).
VORTEX_2D_SMALL = dict(dim=2, p=2, cells=(16, 16, 1), parts=(1, 1, 1), lo=(0, 0, 0), hi=(10, 10, 1))
VORTEX_2D_ASYNC = dict(dim=2, p=3, cells=(256, 256, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1))
WAVE_3D = dict(dim=3, p=3, cells=(64, 64, 64), parts=(4, 4, 4), lo=(0, 0, 0), hi=(1, 1, 1))
VORTEX_2D_MIXED = dict(dim=2, p=4, cells=(1024, 1024, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1))
WAVE_3D_LEARNED = dict(dim=3, p=2, cells=(128, 128, 128), parts=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1))


def perturbation(ndof, seed, scale=1e-3):
    """Seeded uniform noise in [-scale, scale] for every degree of freedom."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=ndof)


def mlp_batch(n, nin, nout, seed):
    """Seeded (x, y) pairs for gradient checks of the predictor."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, nin))
    y = rng.standard_normal((n, nout))
    return x, y


def mlp_weights(nparams, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(nparams) * scale
