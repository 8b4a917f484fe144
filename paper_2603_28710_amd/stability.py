"""Largest stable CFL number of the asynchronous schemes, by bisection.

The paper observes that delays shrink the stable time step and that AT
fluxes relax that limit again (Sec. 5.3, the stability remark beside the
convergence study). This tool measures it on the GPU solver: a run at CFL sigma
is stable if `adg_step`, with the state checked every `check` steps, reports
no non-finite or non-physical state up to t_end. The returned sigma is the
largest stable value found by bisection between lo and hi.

    python -m paper_2603_28710_amd.stability [--setting paper] [--t-end 4] [--cells 64] [--degree 2]

prints one JSON line per (mode, L) with the bracket [stable, unstable]. The
learned mode trains its network first (pairs from the same mesh and
schedule at CFL 0.1), then runs with an accept bound of LEARNED_TOL.
Settings: "periodic" (default) is the vortex of mean flow (1,1) on the
periodic box [0,10]^2 with SSP-RK3; "paper" is the paper's own: mean flow
(1,0) in the Dirichlet box [0,10] x [-5,5], LSERK(p+1,p+1).
"""
import argparse
import json
import math

MODES = {
    "stale_caa": dict(ghost=1, delay_kind=2),
    "at_caa": dict(ghost=2, delay_kind=2),
    "flux_stale_caa": dict(ghost=4, delay_kind=2),
    "flux_at_caa": dict(ghost=5, delay_kind=2),
    "at_uniform": dict(ghost=2, delay_kind=1),
    # the learned predictor over AT, trained first on the same mesh and
    # schedule (see train_predictor); its accept bound is LEARNED_TOL
    "learned_caa": dict(ghost=3, delay_kind=2, learned_judge=0),
    # the same with the second judge: corrections within AT's own error
    # estimate only
    "learned_judged_caa": dict(ghost=3, delay_kind=2, learned_judge=1),
}
LEARNED_TOL = 1e-4
PAPER_VORTEX = (5.0, 0.0, 5.0, 1.0, 0.0)


def train_predictor(make, cfl, steps=400, every=40, epochs=8):
    """network weights trained on pairs the solver built by make() collects
    at CFL cfl: `every` steps, then 4 collected steps, up to `steps` steps"""
    s = make()
    dt = s.stable_dt(cfl)
    s.predictor_bind(4_000_000)
    done = 0
    while done + every + 4 <= steps:
        s.step(every, dt)
        s.predictor_collect(4, dt)
        done += every + 4
    s.predictor_train(epochs=epochs, batch=1024, lr=1e-3, seed=1)
    w = s.predictor_get()
    s.close()
    return w


def runs_stably(make, sigma, t_end):
    """True if the solver built by make() reaches t_end at CFL sigma: the
    step is sigma's (reading Z3, from the initial state) rounded so that an
    integer number of steps ends at t_end"""
    from paper_2603_28710_amd import binding as B

    s = make()
    dt0 = s.stable_dt(sigma)
    n = int(math.ceil(t_end / dt0))
    st = s.step_status(n, t_end / n)
    s.close()
    if st in (B.ADG_ERR_NONFINITE, B.ADG_ERR_NONPHYSICAL):
        return False
    if st != B.ADG_OK:
        raise RuntimeError(B.adg_last_error())
    return True


def max_stable_cfl(stable, lo=0.005, hi=1.0, iters=8):
    """bisection (geometric) on sigma with the predicate stable(sigma);
    assumes stability at lo (checked) and returns the bracket (largest
    stable, smallest unstable) found"""
    if not stable(lo):
        return 0.0, lo
    if stable(hi):
        return hi, float("inf")
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo, hi


def solver_factory(setting, cells, parts, degree, levels, mode, L, check, weights=None):
    """a function building the library's solver for one run of the sweep:
    the 2D vortex of the setting ("periodic": mean flow (1,1) on the periodic
    [0,10]^2, SSP-RK3; "paper": mean flow (1,0) in the Dirichlet box
    [0,10] x [-5,5], LSERK(p+1,p+1)), cells^2 elements in parts^2
    subdomains, the asynchrony of MODES[mode] with maximum delay L"""
    from paper_2603_28710_amd.solver import Solver

    if setting == "paper":
        box = dict(lo=(0, -5, 0), hi=(10, 5, 1), boundary=1, integrator=1 if degree == 1 else 2)
        params = PAPER_VORTEX
    else:
        box = dict(lo=(0, 0, 0), hi=(10, 10, 1))
        params = None

    def make():
        extra = dict(learned_tol=LEARNED_TOL) if MODES[mode]["ghost"] == 3 else {}
        s = Solver(dim=2, degree=degree, cells=(cells, cells, 1), parts=(parts, parts, 1), check_every=check,
                   levels=levels, L=L, seed=0, **box, **MODES[mode], **extra)
        if weights is not None:
            s.predictor_set(weights)
        s.init_problem(0, params)
        return s
    return make


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--setting", choices=["periodic", "paper"], default="periodic")
    ap.add_argument("--t-end", type=float, default=4.0)
    ap.add_argument("--cells", type=int, default=64)
    ap.add_argument("--parts", type=int, default=16)
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--L", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--modes", nargs="+", default=list(MODES))
    ap.add_argument("--check", type=int, default=50)
    a = ap.parse_args()

    def maker(mode, L, weights=None):
        return solver_factory(a.setting, a.cells, a.parts, a.degree, a.levels, mode, L, a.check, weights)

    def bracket(make):
        return max_stable_cfl(lambda sigma: runs_stably(make, sigma, a.t_end))

    sync_lo, sync_hi = bracket(maker("at_caa", 0))
    print(json.dumps({"mode": "sync", "L": 0, "stable": sync_lo, "unstable": sync_hi}), flush=True)
    for mode in a.modes:
        for L in a.L:
            if L == 0 and mode in ("stale_caa", "flux_stale_caa"):
                continue
            w = train_predictor(maker(mode, L), 0.1) if MODES[mode]["ghost"] == 3 else None
            lo, hi = bracket(maker(mode, L, w))
            print(json.dumps({"setting": a.setting, "mode": mode, "L": L, "stable": lo, "unstable": hi,
                              "cells": a.cells, "degree": a.degree, "t_end": a.t_end}), flush=True)


if __name__ == "__main__":
    main()
