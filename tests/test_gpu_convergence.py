"""The paper's accuracy result on the GPU solver: at the paper's own setting
(Dirichlet box, CAA schedules, LSERK), and at the 256^2 vortex
settings (8x8 virtual subdomains, degree 3, uniform random delays up to L=3):
delayed traces with the standard flux lose the order of accuracy, AT
extrapolation over three past levels recovers the synchronous errors and
order p + 1 (Sec. 5.3, the convergence figures). Errors are against the
exact vortex; the time step scales as h^(4/3) so that SSP-RK3's time error
stays below the spatial one at degree 3.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_at_recovers_order_p_plus_1_stale_does_not():
    from paper_2603_28710_amd import convergence as C

    say("case: vortex p=3, parts 8x8, n = 32, 64, 128, t_end 1, sync / stale / AT3, uniform L=3")
    res = C.sweep(["sync", "stale_uniform", "at3_uniform"], [32, 64, 128], degree=3, L=3, parts=8, t_end=1.0,
                  emit=say)
    e_sync, s_sync = (np.array(x) for x in res["sync"])
    e_st, s_st = (np.array(x) for x in res["stale_uniform"])
    e_at, s_at = (np.array(x) for x in res["at3_uniform"])
    assert np.all(s_sync[-1] > 3.7)               # order p + 1 = 4
    assert np.all(s_at[-1] > 3.7)                 # recovered by AT
    np.testing.assert_allclose(e_at, e_sync, rtol=0.01)   # the curves overlap
    assert np.all(s_st[-1] < 1.6)                 # standard flux on delayed traces: order lost
    assert np.all(e_st[-1] > 100 * e_sync[-1])


@pytest.mark.parametrize("degree", [1, 2])
def test_paper_setting_caa_at_matches_sync_caa_std_first_order(degree):
    # the paper's own runs (the convergence figures of Sec. 5.3): vortex with
    # mean flow (1,0) in the Dirichlet box [0,10] x [-5,5] to t = 4, 16x16
    # subdomains, CAA schedules with L = 4, LSERK(p+1,p+1), AT over p+1
    # levels; CFL 0.05 (sync, AT) and 0.03 (standard flux)
    from paper_2603_28710_amd import convergence as C

    say(f"case: paper vortex p={degree}, n = 32, 64, 128, sync / caa_std / caa_at, L=4, t=4")
    res = C.paper_sweep(["sync", "caa_std", "caa_at"], [32, 64, 128], degree=degree, emit=say)
    e_sync, s_sync = (np.array(x) for x in res["sync"])
    e_std, s_std = (np.array(x) for x in res["caa_std"])
    e_at, s_at = (np.array(x) for x in res["caa_at"])
    assert np.all(s_sync[-1] > degree + 1 - 0.25)   # order p + 1
    assert np.all(s_at[-1] > degree + 1 - 0.25)     # kept by AT
    np.testing.assert_allclose(e_at, e_sync, rtol=0.05)
    assert np.all(s_std[-1] < 1.2)                  # first order with the standard flux
    assert np.all(e_std[-1] > 5 * e_sync[-1])


def test_wave3d_at_recovers_order_stale_does_not():
    # the hexahedron kernels: density wave on the unit cube, p = 2, 4^3
    # subdomains, uniform delays up to L = 2, t = 0.25
    from paper_2603_28710_amd import convergence as C

    say("case: density wave 3D p=2, n = 8, 16, 32, sync / stale / AT3, uniform L=2")
    res = C.sweep(["sync", "stale_uniform", "at3_uniform"], [8, 16, 32], degree=2, L=2, parts=4, t_end=0.25,
                  emit=say, dim=3)
    e_sync, s_sync = (np.array(x) for x in res["sync"])
    e_st, s_st = (np.array(x) for x in res["stale_uniform"])
    e_at, s_at = (np.array(x) for x in res["at3_uniform"])
    assert np.all(s_sync[-1] > 2.8)
    assert np.all(s_at[-1] > 2.8)
    np.testing.assert_allclose(e_at, e_sync, rtol=0.01)
    assert np.all(s_st[-1] < 1.2)
