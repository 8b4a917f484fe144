"""adg_integrals_noalloc, the allocation-free variant of adg_integrals (its
partial sums in the library's static per-GPU array), through the C ABI:
the same values as adg_integrals, bit for bit, on two calls in a row, the
second on a smaller mesh (fewer partial blocks than the array kept from the
first call)."""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("order", ["large_then_small"])
def test_integrals_noalloc_matches_integrals(oracle_mod, order):
    from paper_2603_28710_amd import binding as B
    from paper_2603_28710_amd.solver import Solver
    O = oracle_mod
    cases = [
        # 4096 elements: the norm kernels use their maximum of 2048 blocks
        ("density wave 16^3 p=2", dict(dim=3, degree=2, cells=(16, 16, 16), parts=(2, 2, 2), hi=(1, 1, 1)),
         O.DENSITY_WAVE),
        # 48 elements: 48 blocks, the rest of the array holds the first call's
        ("vortex 8x6 p=3", dict(dim=2, degree=3, cells=(8, 6, 1), parts=(2, 2, 1), hi=(10, 10, 1)), O.VORTEX),
    ]
    for name, cfg, prob in cases:
        say(f"case: adg_integrals_noalloc vs adg_integrals, {name}")
        s = Solver(**cfg)
        s.init_problem(prob)
        u = s.download() + inputs.perturbation(s.ndof, 41, 1e-3)
        s.upload(u)
        a = np.array(B.adg_integrals(s.h, s.V))
        b = np.array(B.adg_integrals_noalloc(s.h, s.V))
        b2 = np.array(B.adg_integrals_noalloc(s.h, s.V))
        say("  integrals", a, " noalloc", b)
        assert np.array_equal(a, b) and np.array_equal(b, b2)
        assert np.all(np.isfinite(b)) and b[0] > 0
        s.close()


def test_integrals_noalloc_needs_bound_buffers():
    from paper_2603_28710_amd import binding as B
    cfg = B.make_config(dim=2, degree=2, cells=(4, 4, 1))
    asy = B.make_async()
    h = B.adg_create(cfg, asy, None)
    out = (B.C.c_double * 4)()
    assert B.lib.adg_integrals_noalloc(h, out) == B.ADG_ERR_UNBOUND
    assert B.lib.adg_integrals_noalloc(None, out) == B.ADG_ERR_INVALID
    B.adg_destroy(h)
