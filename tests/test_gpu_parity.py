"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs. Tolerance for FP64: relative L2 per variable group
(density, momentum, energy) <= 1e-11 after the stated steps; bit-exact for
the integer schedule (tested on the CPU in test_host_abi.py).
"""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-11


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    from paper_2603_28710_amd.solver import Solver
    return Solver


@pytest.fixture(scope="module")
def B():
    from paper_2603_28710_amd import binding
    return binding


def rel_l2(a, b, dim, p=None, s=None):
    """max over the groups (density, momentum, energy) of ||a-b|| / ||b||,
    nodal values of the public layout [E][V][P^d]"""
    V = dim + 2
    Pd = (s.P ** dim) if s is not None else (p + 1) ** dim
    a = a.reshape(-1, V, Pd)
    b = b.reshape(-1, V, Pd)
    out = []
    for sl in (slice(0, 1), slice(1, V - 1), slice(V - 1, V)):
        num = np.linalg.norm(a[:, sl] - b[:, sl])
        den = np.linalg.norm(b[:, sl])
        out.append(num / den if den > 0 else num)
    return max(out)


def _pair(O, S, problem=None, perturb=0.0, seed=0, **cfg):
    """oracle and GPU solver on the same configuration and initial state"""
    O_ = O
    problem = O_.VORTEX if problem is None else problem
    ocfg = dict(cfg)
    gcfg = dict(cfg)
    gcfg["degree"] = gcfg.pop("p")
    o = O_.Oracle(**ocfg)
    o.init_problem(problem)
    if perturb:
        o.set_state(o.state() + inputs.perturbation(o.ndof, seed, perturb))
    s = S(**gcfg)
    s.upload(o.state())
    return o, s


# ------------------------------------------------------------------ sync

def test_vortex_16x16_p2_sync_100_steps(oracle_mod, S):
    O = oracle_mod
    cfg = dict(dim=2, p=2, cells=(16, 16, 1), hi=(10, 10, 1))
    say("case: vortex 16x16 p=2 sync, projection + 100 steps")
    o = O.Oracle(**cfg)
    o.init_problem(O.VORTEX)
    s = S(dim=2, degree=2, cells=(16, 16, 1), hi=(10, 10, 1))
    s.init_problem(O.VORTEX)
    assert rel_l2(s.download(), o.state(), 2, s=s) < 1e-13
    dt = o.stable_dt(0.1)
    assert abs(s.stable_dt(0.1) - dt) <= 1e-14 * dt
    s.upload(o.state())
    assert o.step(100, dt) == 0
    s.step(100, dt)
    r = rel_l2(s.download(), o.state(), 2, s=s)
    say("  rel L2", r)
    assert r <= TOL
    np.testing.assert_allclose(s.error_norms(O.VORTEX), o.error_norms(O.VORTEX, 100 * dt), rtol=1e-9)
    assert s.time()[0] == 100


@pytest.mark.parametrize("dim,p,cells", [
    (2, 1, (13, 11, 1)), (2, 2, (13, 11, 1)), (2, 3, (13, 11, 1)), (2, 4, (13, 11, 1)),
    (3, 1, (5, 4, 3)), (3, 2, (5, 4, 3)), (3, 3, (5, 4, 3)), (3, 4, (3, 3, 2)),
])
def test_sync_every_degree_ragged_tiles(oracle_mod, S, dim, p, cells):
    O = oracle_mod
    say(f"case: density wave dim={dim} p={p} cells={cells} sync, perturbed, 10 steps")
    o, s = _pair(O, S, problem=O.DENSITY_WAVE, perturb=1e-3, seed=p, dim=dim, p=p, cells=cells,
                 hi=(1, 1, 1))
    dt = 0.5 * o.stable_dt(0.1)
    o.step(10, dt)
    s.step(10, dt)
    r = rel_l2(s.download(), o.state(), dim, s=s)
    say("  rel L2", r)
    assert r <= TOL


@pytest.mark.parametrize("flux", [0, 1])
def test_single_rhs_stage_matches_oracle_elements(oracle_mod, S, flux):
    # stage 0 output (u_a register) against the oracle's per-element stage
    O = oracle_mod
    say(f"case: one stage, flux={flux}")
    o, s = _pair(O, S, perturb=1e-2, seed=3, dim=2, p=3, cells=(12, 10, 1), parts=(3, 2, 1),
                 hi=(10, 10, 1), flux=flux)
    u0 = o.state()
    dt = o.stable_dt(0.1)
    s.step(1, dt)
    ua = s.u[1].cpu().numpy()
    ref = o.stage_elements(0, dt, u0, u0, np.arange(o.E))
    assert rel_l2(ua, ref, 2, s=s) <= 1e-13


# ----------------------------------------------------------------- async

ASYNC_MODES = [
    ("stale_fixed2", 1, 0, 2, 1), ("stale_uniform3", 1, 1, 3, 1), ("stale_caa4", 1, 2, 4, 1),
    ("at3_fixed1", 2, 0, 1, 3), ("at3_uniform3", 2, 1, 3, 3), ("at3_caa3", 2, 2, 3, 3),
    ("at2_uniform2", 2, 1, 2, 2), ("at4_uniform2", 2, 1, 2, 4),
    ("flux_stale_caa3", 4, 2, 3, 1), ("flux_at3_caa3", 5, 2, 3, 3), ("flux_at2_caa4", 5, 2, 4, 2),
]


@pytest.mark.parametrize("name,ghost,kind,L,levels", ASYNC_MODES)
def test_async_modes_vortex_2d(oracle_mod, S, name, ghost, kind, L, levels):
    O = oracle_mod
    say(f"case: vortex 2D p=3 36x20 parts 4x2 {name}, 30 steps")
    o, s = _pair(O, S, dim=2, p=3, cells=(36, 20, 1), parts=(4, 2, 1), hi=(10, 10, 1), ghost=ghost,
                 delay_kind=kind, L=L, levels=levels, seed=7)
    dt = 0.5 * o.stable_dt(0.1)
    o.step(30, dt)
    s.step(30, dt)
    r = rel_l2(s.download(), o.state(), 2, s=s)
    say("  rel L2", r)
    assert r <= TOL


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_async_at_uniform_3d(oracle_mod, S, seed):
    O = oracle_mod
    say(f"case: density wave 3D p=2 8^3 parts 2^3 AT uniform L=2 seed={seed}, 12 steps")
    o, s = _pair(O, S, problem=O.DENSITY_WAVE, dim=3, p=2, cells=(8, 8, 8), parts=(2, 2, 2), hi=(1, 1, 1),
                 ghost=2, delay_kind=1, L=2, levels=3, seed=seed)
    dt = o.stable_dt(0.1)
    o.step(12, dt)
    s.step(12, dt)
    r = rel_l2(s.download(), o.state(), 3, s=s)
    say("  rel L2", r)
    assert r <= TOL


# The degree <= 2 hexahedron kernel cuts each x row into ranges of 12
# elements (the last one shorter) and orders them in bands of 16 z layers
# (the last band thinner): rows of 14 and 26 elements, 18 and 35 layers, PE
# faces inside a range and at a range's end, and the shared x pass's
# fallback (more than four outside x face-sides: subdomains 3 elements wide).
@pytest.mark.parametrize("p,cells,parts,ghost,kind,L,levels", [
    (2, (14, 3, 18), (2, 1, 3), 2, 1, 3, 3),
    (1, (14, 3, 18), (2, 1, 3), 2, 1, 3, 2),
    (2, (26, 2, 35), (2, 2, 5), 5, 2, 3, 3),
    (2, (24, 2, 17), (8, 1, 1), 2, 1, 2, 3),
    (2, (14, 3, 18), (1, 1, 1), 0, 0, 0, 3),
])
def test_hexahedron_wavefront_ranges(oracle_mod, S, p, cells, parts, ghost, kind, L, levels):
    O = oracle_mod
    say(f"case: density wave 3D p={p} {cells} parts {parts} ghost={ghost} kind={kind} L={L} levels={levels}, "
        f"10 steps")
    o, s = _pair(O, S, problem=O.DENSITY_WAVE, perturb=1e-3, seed=11, dim=3, p=p, cells=cells, parts=parts,
                 hi=(1, 1, 1), ghost=ghost, delay_kind=kind, L=L, levels=levels)
    dt = 0.5 * o.stable_dt(0.1)
    o.step(10, dt)
    s.step(10, dt)
    r = rel_l2(s.download(), o.state(), 3, s=s)
    say("  rel L2", r)
    assert r <= TOL


@pytest.mark.parametrize("p,cells,ghost,kind,L,levels,precision", [
    (3, (8, 8, 8), 2, 0, 2, 3, 0),   # the 64^3 density-wave settings: AT3, fixed L=2
    (3, (8, 8, 8), 2, 1, 2, 3, 0),
    (3, (8, 8, 8), 1, 1, 2, 1, 0),
    (3, (8, 8, 8), 5, 2, 3, 3, 0),
    (3, (8, 8, 8), 2, 1, 2, 3, 1),   # FP32 contractions: within 1e-6
    (4, (4, 4, 4), 2, 1, 2, 3, 0),
    (4, (4, 4, 4), 4, 2, 3, 1, 0),
])
def test_async_3d_high_degree(oracle_mod, S, p, cells, ghost, kind, L, levels, precision):
    O = oracle_mod
    say(f"case: density wave 3D p={p} {cells} parts 2^3 ghost={ghost} kind={kind} L={L} levels={levels} "
        f"precision={precision}, 8 steps")
    cfg = dict(dim=3, cells=cells, parts=(2, 2, 2), hi=(1, 1, 1), ghost=ghost, delay_kind=kind, L=L,
               levels=levels, seed=3)
    o = O.Oracle(p=p, **cfg)
    o.init_problem(O.DENSITY_WAVE)
    o.set_state(o.state() + inputs.perturbation(o.ndof, 5, 1e-3))
    s = S(degree=p, precision=precision, **cfg)
    s.upload(o.state())
    dt = o.stable_dt(0.1)
    o.step(8, dt)
    s.step(8, dt)
    r = rel_l2(s.download(), o.state(), 3, s=s)
    say("  rel L2", r)
    assert r <= (TOL if precision == 0 else 1e-6)


@pytest.mark.parametrize("ghost,precision", [(4, 0), (5, 0), (5, 1)])
def test_flux_history_3d(oracle_mod, S, ghost, precision):
    # Alg. caa-std / caa-at with stored fluxes on hexahedra: FP64 against the
    # oracle; the FP32-contraction variant within 1e-6 of it
    O = oracle_mod
    say(f"case: density wave 3D p=2 8^3 parts 2^3 flux-history ghost={ghost} precision={precision}, 14 steps")
    cfg = dict(dim=3, cells=(8, 8, 8), parts=(2, 2, 2), hi=(1, 1, 1), ghost=ghost, delay_kind=2, L=3, levels=3)
    o = O.Oracle(p=2, **cfg)
    o.init_problem(O.DENSITY_WAVE)
    s = S(degree=2, precision=precision, **cfg)
    s.upload(o.state())
    dt = o.stable_dt(0.1)
    o.step(14, dt)
    s.step(14, dt)
    r = rel_l2(s.download(), o.state(), 3, s=s)
    say("  rel L2", r)
    assert r <= (TOL if precision == 0 else 1e-6)


@pytest.mark.parametrize("dim", [2, 3])
def test_flux_history_conserves_on_gpu(oracle_mod, S, dim):
    # both sides of a PE face use one stored flux: the integrals stay put to
    # round-off through silent steps
    O = oracle_mod
    say(f"case: flux-history AT conservation {dim}D")
    cells = (32, 32, 1) if dim == 2 else (8, 8, 8)
    parts = (4, 4, 1) if dim == 2 else (2, 2, 2)
    s = S(dim=dim, degree=3 if dim == 2 else 2, cells=cells, parts=parts, hi=(10, 10, 1) if dim == 2 else (1, 1, 1),
          ghost=5, delay_kind=2, L=3, levels=3)
    s.init_problem(O.VORTEX if dim == 2 else O.DENSITY_WAVE)
    I0 = np.array(s.integrals())
    s.step(40, 0.5 * s.stable_dt(0.1))
    I1 = np.array(s.integrals())
    say("  max drift", np.abs(I1 - I0).max() / np.abs(I0).max())
    assert np.all(np.abs(I1 - I0) <= 1e-13 * np.abs(I0).max())


def test_zero_delay_bitwise_equals_sync(oracle_mod, S):
    O = oracle_mod
    say("case: AT with L=0 vs sync, bitwise")
    base = dict(dim=2, degree=3, cells=(32, 32, 1), parts=(4, 4, 1), hi=(10, 10, 1))
    a = S(**base)
    a.init_problem(O.VORTEX)
    b = S(ghost=2, delay_kind=0, L=0, levels=3, **base)
    b.init_problem(O.VORTEX)
    dt = a.stable_dt(0.1)
    a.step(20, dt)
    b.step(20, dt)
    np.testing.assert_array_equal(a.download(), b.download())


def test_deterministic_repeat(oracle_mod, S):
    O = oracle_mod
    say("case: two AT uniform runs, bitwise")
    cfg = dict(dim=2, degree=3, cells=(64, 64, 1), parts=(8, 8, 1), hi=(10, 10, 1), ghost=2, delay_kind=1,
               L=3, levels=3, seed=1)
    outs = []
    for _ in range(2):
        s = S(**cfg)
        s.init_problem(O.VORTEX)
        s.step(25, 0.002)
        outs.append(s.download())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_checkpoint_resume_bitwise(oracle_mod, S):
    O = oracle_mod
    say("case: save after 7 steps, resume, bitwise")
    cfg = dict(dim=2, degree=2, cells=(24, 24, 1), parts=(4, 4, 1), hi=(10, 10, 1), ghost=2, delay_kind=1,
               L=3, levels=3, seed=4)
    s = S(**cfg)
    s.init_problem(O.VORTEX)
    s.step(7, 0.003)
    blob = s.save()
    s.step(9, 0.003)
    a = s.download()
    t = S(**cfg)
    t.load(blob)
    assert t.time()[0] == 7
    t.step(9, 0.003)
    np.testing.assert_array_equal(t.download(), a)


def test_profile_samples_every_kth_step(oracle_mod, S, B):
    # events around the stage launches of steps n % k == 0 only
    O = oracle_mod
    say("case: event profiling of every 4th step, 20 steps")
    s = S(dim=2, degree=2, cells=(32, 32, 1), parts=(2, 2, 1), hi=(10, 10, 1), ghost=2, delay_kind=1, L=2,
          levels=3)
    s.init_problem(O.VORTEX)
    B.adg_profile(s.h, 4)
    s.step(20, 1e-3)
    ms, n = B.adg_profile_read(s.h, B.ADG_KERNEL_RHS)
    B.adg_profile(s.h, 1)
    s.step(2, 1e-3)
    ms1, n1 = B.adg_profile_read(s.h, B.ADG_KERNEL_RHS)
    B.adg_profile(s.h, 0)
    assert n == 5 * 3 and ms > 0
    assert n1 == 2 * 3 and ms1 > 0


def test_checkpoint_resume_dirichlet_box(oracle_mod, S):
    # the blob carries the boundary problem: the resumed context needs no
    # adg_set_boundary and continues bitwise
    O = oracle_mod
    say("case: Dirichlet box, save after 5 steps, resume in a new context, bitwise")
    prm = (5.0, 0.0, 5.0, 1.0, 0.0)
    cfg = dict(dim=2, degree=2, cells=(24, 24, 1), parts=(4, 4, 1), lo=(0, -5, 0), hi=(10, 5, 1), ghost=5,
               delay_kind=2, L=3, levels=3, seed=1, boundary=1, integrator=2)
    s = S(**cfg)
    s.init_problem(O.VORTEX, prm)
    s.step(5, 0.01)
    blob = s.save()
    s.step(8, 0.01)
    a = s.download()
    t = S(**cfg)
    t.load(blob)
    assert t.time()[0] == 5
    t.step(8, 0.01)
    np.testing.assert_array_equal(t.download(), a)


@pytest.mark.parametrize("ghost,kind,L", [(0, 0, 0), (1, 1, 3), (2, 1, 3), (2, 2, 2)])
def test_free_stream_every_mode(oracle_mod, S, ghost, kind, L):
    O = oracle_mod
    say(f"case: free stream 3D ghost={ghost} kind={kind}")
    s = S(dim=3, degree=3, cells=(8, 8, 8), parts=(2, 2, 2), hi=(1, 1, 1), ghost=ghost, delay_kind=kind, L=L,
          levels=3)
    s.init_problem(O.CONSTANT)
    u0 = s.download()
    s.step(10, 1e-3)
    np.testing.assert_allclose(s.download(), u0, rtol=0, atol=1e-13)


def test_sync_conservation(oracle_mod, S):
    O = oracle_mod
    say("case: sync conservation 2D p=3 with subdomains")
    s = S(dim=2, degree=3, cells=(32, 32, 1), parts=(4, 4, 1), hi=(10, 10, 1))
    s.init_problem(O.VORTEX)
    I0 = np.array(s.integrals())
    s.step(50, s.stable_dt(0.1))
    I1 = np.array(s.integrals())
    assert np.all(np.abs(I1 - I0) <= 1e-13 * np.abs(I0).max())


def test_nonfinite_state_reported(oracle_mod, S, B):
    O = oracle_mod
    say("case: NaN in the state is reported by the periodic check")
    s = S(dim=2, degree=2, cells=(8, 8, 1), hi=(10, 10, 1), check_every=1)
    s.init_problem(O.VORTEX)
    u = s.download()
    u[5] = np.nan
    s.upload(u)
    assert s.step_status(1, 1e-3) == B.ADG_ERR_NONFINITE
    s2 = S(dim=2, degree=2, cells=(8, 8, 1), hi=(10, 10, 1), check_every=1)
    s2.init_problem(O.VORTEX)
    u = s2.download()
    u[0:9] = -1.0  # negative density at every node of element 0
    s2.upload(u)
    assert s2.step_status(1, 1e-5) in (B.ADG_ERR_NONPHYSICAL, B.ADG_ERR_NONFINITE)


def test_fp32_contraction_within_1e6_of_fp64(oracle_mod, S):
    # the mixed-precision workload at reduced size: vortex 128^2, degree 4,
    # 8x8 subdomains, AT3 with uniform delays in {0..3}; FP32 contractions,
    # FP64 state. Error against the FP64 path and the oracle every 50 steps.
    O = oracle_mod
    say("case: FP32 contractions vs FP64, vortex 128^2 p=4 AT3 uniform L=3, 100 steps")
    cfg = dict(dim=2, cells=(128, 128, 1), parts=(8, 8, 1), hi=(10, 10, 1), ghost=2, delay_kind=1, L=3, levels=3,
               seed=0)
    o = O.Oracle(p=4, **cfg)
    o.init_problem(O.VORTEX)
    s64 = S(degree=4, precision=0, **cfg)
    s32 = S(degree=4, precision=1, **cfg)
    s64.upload(o.state())
    s32.upload(o.state())
    dt = o.stable_dt(0.1)
    for chunk in range(2):
        o.step(50, dt)
        s64.step(50, dt)
        s32.step(50, dt)
        ref = o.state()
        r64 = rel_l2(s64.download(), ref, 2, s=s64)
        r32 = rel_l2(s32.download(), ref, 2, s=s32)
        r3264 = rel_l2(s32.download(), s64.download(), 2, s=s32)
        say(f"  after {50 * (chunk + 1)} steps: fp64 vs oracle {r64:.2e}, fp32 vs oracle {r32:.2e}, "
            f"fp32 vs fp64 {r3264:.2e}")
        assert r64 <= TOL
        assert r32 <= 1e-6 and r3264 <= 1e-6


# --------------------------------------------------------------- LSERK (Sec. 2.3)

@pytest.mark.parametrize("dim,p,integ,ghost,kind,L,levels,precision", [
    (2, 3, 1, 0, 0, 0, 3, 0),
    (2, 3, 2, 0, 0, 0, 3, 0),
    (2, 3, 2, 2, 1, 3, 3, 0),
    (2, 3, 1, 1, 0, 2, 1, 0),
    (2, 3, 2, 5, 2, 3, 3, 0),
    (2, 4, 2, 2, 1, 2, 3, 1),   # FP32 contractions: within 1e-6
    (3, 2, 2, 2, 1, 2, 3, 0),
    (3, 3, 2, 2, 0, 2, 3, 0),
    (3, 4, 1, 2, 1, 2, 3, 0),
    (2, 3, 3, 0, 0, 0, 3, 0),   # SSP-RK2
    (2, 3, 3, 2, 1, 3, 2, 0),
    (3, 3, 3, 5, 2, 3, 3, 0),
])
def test_integrators_against_oracle(oracle_mod, S, dim, p, integ, ghost, kind, L, levels, precision):
    # the two-register schemes move the state through all three registers
    # (the second LSERK(3,3) stage writes its next input over the accumulator
    # it reads) and end every step in u_n; SSP-RK2 writes its second stage in
    # place over u_n
    O = oracle_mod
    say(f"case: integrator={integ} dim={dim} p={p} ghost={ghost} kind={kind} L={L} levels={levels} "
        f"precision={precision}, 10 steps")
    if dim == 2:
        cfg = dict(dim=2, cells=(36, 20, 1), parts=(4, 2, 1), hi=(10, 10, 1))
        prob = O.VORTEX
    else:
        n = {2: 8, 3: 8, 4: 4}[p]
        cfg = dict(dim=3, cells=(n, n, n), parts=(2, 2, 2), hi=(1, 1, 1))
        prob = O.DENSITY_WAVE
    cfg.update(ghost=ghost, delay_kind=kind, L=L, levels=levels, seed=5, integrator=integ)
    o = O.Oracle(p=p, **cfg)
    o.init_problem(prob)
    o.set_state(o.state() + inputs.perturbation(o.ndof, 9, 1e-3))
    s = S(degree=p, precision=precision, **cfg)
    s.upload(o.state())
    dt = 0.5 * o.stable_dt(0.1)
    o.step(10, dt)
    s.step(10, dt)
    r = rel_l2(s.download(), o.state(), dim, s=s)
    say("  rel L2", r)
    assert r <= (TOL if precision == 0 else 1e-6)


# ------------------------------------------- Dirichlet box (Sec. 5.1 vortex)

PAPER_VORTEX = (5.0, 0.0, 5.0, 1.0, 0.0)
WAVE_IN = (0.2, 1.0, 1.0, 0.0, 1.0)  # density wave entering through x = 0 and y = 0


@pytest.mark.parametrize("p,problem,ghost,kind,L,levels,integ,precision", [
    (1, "wave", 0, 0, 0, 3, 0, 0), (2, "wave", 0, 0, 0, 3, 0, 0), (3, "wave", 0, 0, 0, 3, 0, 0),
    (4, "wave", 0, 0, 0, 3, 0, 0), (3, "vortex", 0, 0, 0, 3, 0, 0),
    (3, "wave", 1, 2, 4, 1, 0, 0), (3, "vortex", 2, 2, 4, 3, 0, 0), (1, "vortex", 2, 2, 4, 2, 0, 0),
    (2, "wave", 2, 1, 3, 3, 0, 0), (3, "wave", 4, 2, 3, 1, 0, 0), (3, "wave", 5, 2, 4, 3, 0, 0),
    (2, "wave", 2, 2, 4, 3, 2, 0), (3, "vortex", 0, 0, 0, 3, 1, 0), (4, "wave", 2, 1, 3, 3, 0, 1),
])
def test_dirichlet_box_against_oracle(oracle_mod, S, p, problem, ghost, kind, L, levels, integ, precision):
    # every side carries the exact solution at the stage time; the density
    # wave enters through two sides, so the boundary data vary along the
    # faces and in time; 36 x 20 elements leave a ragged last wavefront
    O = oracle_mod
    say(f"case: Dirichlet box {problem} p={p} ghost={ghost} kind={kind} L={L} levels={levels} "
        f"integrator={integ} precision={precision}, 20 steps")
    if problem == "wave":
        prob, prm, lo, hi = O.DENSITY_WAVE, WAVE_IN, (0, 0, 0), (1, 1, 1)
    else:
        prob, prm, lo, hi = O.VORTEX, PAPER_VORTEX, (0, -5, 0), (10, 5, 1)
    cfg = dict(dim=2, cells=(36, 20, 1), parts=(4, 2, 1), lo=lo, hi=hi, ghost=ghost, delay_kind=kind, L=L,
               levels=levels, seed=4, integrator=integ)
    o = O.Oracle(p=p, bc=O.DIRICHLET, bc_problem=prob, bc_params=prm, **cfg)
    o.init_problem(prob, prm)
    o.set_state(o.state() + inputs.perturbation(o.ndof, 21, 1e-3))
    s = S(degree=p, precision=precision, boundary=1, **cfg)
    s.upload(o.state())
    s.set_boundary(prob, prm)
    dt = 0.5 * o.stable_dt(0.1)
    o.step(20, dt)
    s.step(20, dt)
    r = rel_l2(s.download(), o.state(), 2, s=s)
    say("  rel L2", r)
    assert r <= (TOL if precision == 0 else 1e-6)


def test_dirichlet_paper_vortex_norms_and_projection(oracle_mod, S):
    # the paper's vortex in its Dirichlet box: the GPU projection, and the
    # error norms against the unwrapped exact solution late in the run, when
    # the vortex has moved towards the x = 10 side (a periodic image would
    # reappear near x = 0)
    O = oracle_mod
    say("case: paper vortex 40x40 p=2, projection and error norms at t = 3.9")
    cfg = dict(dim=2, cells=(40, 40, 1), lo=(0, -5, 0), hi=(10, 5, 1))
    o = O.Oracle(p=2, bc=O.DIRICHLET, bc_problem=O.VORTEX, bc_params=PAPER_VORTEX, **cfg)
    o.init_problem(O.VORTEX, PAPER_VORTEX)
    s = S(degree=2, boundary=1, **cfg)
    s.init_problem(O.VORTEX, PAPER_VORTEX)
    assert rel_l2(s.download(), o.state(), 2, s=s) < 1e-13
    s.upload(o.state())
    s.set_boundary(O.VORTEX, PAPER_VORTEX)
    dt = 3.9 / 800  # sigma ~ 0.12 in the CFL reading
    o.step(800, dt)
    s.step(800, dt)
    assert rel_l2(s.download(), o.state(), 2, s=s) <= TOL
    eo = np.array(o.error_norms(O.VORTEX, 3.9, PAPER_VORTEX))
    es = np.array(s.error_norms(O.VORTEX, PAPER_VORTEX))
    say("  error norms oracle", eo, "gpu", es)
    np.testing.assert_allclose(es, eo, rtol=1e-9)
    assert eo.max() < 0.05


def test_dirichlet_needs_a_boundary_problem(oracle_mod, S, B):
    O = oracle_mod
    s = S(dim=2, degree=2, cells=(8, 8, 1), boundary=1)
    s.upload(np.ones(s.ndof))
    assert s.step_status(1, 1e-3) == B.ADG_ERR_STATE
    s.set_boundary(O.CONSTANT, (1.0, 1.0, 0.0, 0.0, 1.0))
    o = O.Oracle(dim=2, p=2, cells=(8, 8, 1), bc=O.DIRICHLET, bc_problem=O.CONSTANT,
                 bc_params=(1.0, 1.0, 0.0, 0.0, 1.0))
    o.init_problem(O.CONSTANT, (1.0, 1.0, 0.0, 0.0, 1.0))
    s.upload(o.state())
    s.step(5, 1e-3)
    np.testing.assert_allclose(s.download(), o.state(), rtol=0, atol=1e-13)


# ------------------------------------------------------------ edge cases

def test_zero_steps_leave_the_state(oracle_mod, S):
    O = oracle_mod
    s = S(dim=2, degree=3, cells=(8, 8, 1), parts=(2, 2, 1), hi=(10, 10, 1), ghost=2, delay_kind=1, L=2, levels=3)
    s.init_problem(O.VORTEX)
    u0 = s.download()
    s.step(0, 1e-3)
    assert s.time() == (0, 0.0)
    np.testing.assert_array_equal(s.download(), u0)


@pytest.mark.parametrize("dim,p,cells,parts,ghost,kind,L", [
    (2, 2, (1, 1, 1), (1, 1, 1), 0, 0, 0),   # one element, its own neighbour on every face
    (2, 3, (2, 1, 1), (2, 1, 1), 2, 1, 2),   # both x faces PE faces to the same element
    (2, 3, (3, 2, 1), (3, 2, 1), 2, 1, 2),   # one element per subdomain: every face a PE face
    (2, 4, (1, 3, 1), (1, 3, 1), 1, 2, 3),
    (3, 2, (1, 1, 1), (1, 1, 1), 0, 0, 0),
    (3, 2, (2, 2, 2), (2, 2, 2), 2, 1, 2),
    (3, 3, (2, 1, 1), (2, 1, 1), 2, 0, 1),   # lane-pair kernel
    (3, 4, (1, 1, 2), (1, 1, 2), 5, 2, 3),   # LDS kernel, flux history
])
def test_degenerate_meshes(oracle_mod, S, dim, p, cells, parts, ghost, kind, L):
    O = oracle_mod
    say(f"case: degenerate mesh dim={dim} p={p} cells={cells} parts={parts} ghost={ghost} kind={kind} L={L}")
    hi = (1, 1, 1)
    prob = O.DENSITY_WAVE
    o = O.Oracle(dim=dim, p=p, cells=cells, parts=parts, hi=hi, ghost=ghost, delay_kind=kind, L=L, levels=3,
                 seed=3)
    o.init_problem(prob)
    o.set_state(o.state() + inputs.perturbation(o.ndof, 31, 1e-3))
    s = S(dim=dim, degree=p, cells=cells, parts=parts, hi=hi, ghost=ghost, delay_kind=kind, L=L, levels=3, seed=3)
    s.upload(o.state())
    dt = 0.5 * o.stable_dt(0.1)
    o.step(12, dt)
    s.step(12, dt)
    r = rel_l2(s.download(), o.state(), dim, s=s)
    say("  rel L2", r)
    assert r <= TOL
