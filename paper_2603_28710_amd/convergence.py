"""Convergence of the asynchronous schemes on the GPU solver.

The paper's accuracy study (Sec. 5.3, the convergence figures of the
isentropic vortex) shows that delayed neighbour data with the standard flux
degrade the scheme to first order, while AT extrapolation over past levels
recovers the synchronous curve and its order p + 1. Three settings:

* "periodic" (default): the vortex on the periodic box [0,10]^2 with mean
  flow (1,1), 8x8 virtual subdomains, uniform random delays, SSP-RK3, to
  t_end with a time step proportional to h^r (r = (p+1)/3 keeps SSP-RK3's
  time error below the spatial one at degree 3).
* "wave3d": the density wave on the periodic unit cube (the 3D workloads'
  stand-in for the paper's cylinder), 4x4x4 subdomains, uniform delays up
  to L, SSP-RK3 with dt ~ h^((p+1)/3), on the hexahedron kernels.
* "paper": the paper's own runs: the vortex of mean flow (1,0) in the
  Dirichlet box [0,10] x [-5,5], t_end = 4, 16x16 subdomains (256 PEs), the
  communication-avoiding schedules with L = 4, DG(1) with LSERK(2,2) and AT2
  or DG(2) with LSERK(3,3) and AT3, CFL 0.05 for the synchronous and AT
  schemes and 0.03 for the standard flux. Both readings of what is delayed
  run: neighbour traces ("caa_std", "caa_at") and the stored fluxes of the
  algorithms themselves ("flux_caa_std", "flux_caa_at"); "learned_caa" adds
  the learned predictor over AT, trained on each mesh first.

    python -m paper_2603_28710_amd.convergence [--setting paper|wave3d] [--ns 32 64 128 256] [--degree 2]

prints one JSON line per (mode, n) and one per mode with its slopes.
"""
import argparse
import json
import math

MODES = {
    "sync": dict(ghost=0, delay_kind=0, L=0),
    "stale_uniform": dict(ghost=1, delay_kind=1),
    "at3_uniform": dict(ghost=2, delay_kind=1),
}

PAPER_VORTEX = (5.0, 0.0, 5.0, 1.0, 0.0)  # x0, y0, beta, mean flow (1, 0)
PAPER_MODES = {
    "sync": dict(ghost=0, delay_kind=0, L=0, cfl=0.05),
    "caa_std": dict(ghost=1, delay_kind=2, cfl=0.03),
    "caa_at": dict(ghost=2, delay_kind=2, cfl=0.05),
    "flux_caa_std": dict(ghost=4, delay_kind=2, cfl=0.03),
    "flux_caa_at": dict(ghost=5, delay_kind=2, cfl=0.05),
    # the learned predictor over AT (caa-at schedule), its network trained on
    # the same mesh first (stability.train_predictor), accept bound 1e-4
    "learned_caa": dict(ghost=3, delay_kind=2, cfl=0.05, learned_tol=1e-4, learned_judge=0),
    # the same with the second judge (corrections within AT's own error estimate)
    "learned_judged_caa": dict(ghost=3, delay_kind=2, cfl=0.05, learned_tol=1e-4, learned_judge=1),
}


def _make(n, degree, asy, box, seed=0, weights=None):
    from paper_2603_28710_amd.solver import Solver

    dim = box.get("dim", 2)
    s = Solver(dim=dim, degree=degree, cells=(n, n, n if dim == 3 else 1), seed=seed, **box["cfg"], **asy)
    if weights is not None:
        s.predictor_set(weights)
    s.init_problem(box["problem"], box["params"])
    return s


def _run(n, degree, asy, box, t_end, dt_of, seed=0, weights=None):
    """L2 errors (density, momentum, energy) at t_end on the n^d mesh with
    the time step dt_of(n), and the number of steps"""
    s = _make(n, degree, asy, box, seed, weights)
    dt = dt_of(n)
    nst = int(math.ceil(t_end / dt))
    s.step(nst, t_end / nst)
    err = s.error_norms(box["problem"], box["params"])
    s.close()
    return err, nst


def _stable_dt(n, degree, box, cfl):
    from paper_2603_28710_amd.solver import Solver

    dim = box.get("dim", 2)
    s = Solver(dim=dim, degree=degree, cells=(n, n, n if dim == 3 else 1), **box["cfg"])
    s.init_problem(box["problem"], box["params"])
    dt = s.stable_dt(cfl)
    s.close()
    return dt


def slopes(errs):
    return [[math.log2(a / b) for a, b in zip(e0, e1)] for e0, e1 in zip(errs[:-1], errs[1:])]


def sweep(modes, ns, degree=3, L=3, parts=8, t_end=1.0, cfl=0.1, r=None, emit=print, dim=2):
    """the periodic settings: the 2D vortex, or (dim = 3) the density wave"""
    r = (degree + 1) / 3.0 if r is None else r
    if dim == 3:
        box = dict(dim=3, cfg=dict(parts=(parts, parts, parts), lo=(0, 0, 0), hi=(1, 1, 1)), problem=1,
                   params=None)
    else:
        box = dict(cfg=dict(parts=(parts, parts, 1), lo=(0, 0, 0), hi=(10, 10, 1)), problem=0, params=None)
    dt_ref = _stable_dt(ns[0], degree, box, cfl)
    out = {}
    for mode in modes:
        asy = dict(MODES[mode])
        asy.setdefault("L", L)
        asy["levels"] = 1 if asy["ghost"] == 1 else 3
        errs = []
        for n in ns:
            err, nst = _run(n, degree, asy, box, t_end, lambda m: dt_ref * (ns[0] / m) ** r)
            errs.append(list(err))
            emit(json.dumps({"dim": dim, "mode": mode, "n": n, "degree": degree, "L": L, "steps": nst,
                             "l2": list(err)}))
        out[mode] = (errs, slopes(errs))
        emit(json.dumps({"dim": dim, "mode": mode, "slopes": out[mode][1]}))
    return out


def paper_sweep(modes, ns, degree=2, L=4, parts=16, t_end=4.0, emit=print):
    """the paper's setting: Dirichlet box, CAA schedules, LSERK(p+1, p+1),
    AT over p + 1 levels, time step from the CFL number on each mesh"""
    box = dict(cfg=dict(parts=(parts, parts, 1), lo=(0, -5, 0), hi=(10, 5, 1), boundary=1,
                        integrator=1 if degree == 1 else 2),
               problem=0, params=PAPER_VORTEX)
    out = {}
    for mode in modes:
        m = dict(PAPER_MODES[mode])
        cfl = m.pop("cfl")
        m.setdefault("L", L)
        m["levels"] = 1 if m["ghost"] in (1, 4) else degree + 1
        errs = []
        for n in ns:
            w = None
            if m["ghost"] == 3:
                from paper_2603_28710_amd.stability import train_predictor

                w = train_predictor(lambda: _make(n, degree, m, box), cfl)
            err, nst = _run(n, degree, m, box, t_end, lambda k: _stable_dt(k, degree, box, cfl), weights=w)
            errs.append(list(err))
            emit(json.dumps({"setting": "paper", "mode": mode, "n": n, "degree": degree, "L": m["L"], "cfl": cfl,
                             "steps": nst, "l2": list(err)}))
        out[mode] = (errs, slopes(errs))
        emit(json.dumps({"setting": "paper", "mode": mode, "degree": degree, "slopes": out[mode][1]}))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--setting", choices=["periodic", "wave3d", "paper"], default="periodic")
    ap.add_argument("--ns", type=int, nargs="+", default=[32, 64, 128, 256])
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--parts", type=int, default=None)
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--cfl", type=float, default=0.1)
    ap.add_argument("--r", type=float, default=None)
    ap.add_argument("--modes", nargs="+", default=None)
    a = ap.parse_args()
    emit = lambda s: print(s, flush=True)  # noqa: E731
    if a.setting == "paper":
        paper_sweep(a.modes or list(PAPER_MODES), a.ns, a.degree or 2, a.L or 4, a.parts or 16, a.t_end or 4.0,
                    emit=emit)
    elif a.setting == "wave3d":
        sweep(a.modes or list(MODES), a.ns, a.degree or 2, a.L or 2, a.parts or 4, a.t_end or 0.25, a.cfl, a.r,
              emit=emit, dim=3)
    else:
        sweep(a.modes or list(MODES), a.ns, a.degree or 3, a.L or 3, a.parts or 8, a.t_end or 1.0, a.cfl, a.r,
              emit=emit)


if __name__ == "__main__":
    main()
