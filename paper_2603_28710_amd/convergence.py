"""Convergence of the asynchronous schemes on the GPU solver.

The paper's accuracy study (Sec. 5.1, the convergence figures of the
isentropic vortex) shows that delayed neighbour data with the standard flux
degrades the scheme to first order, while AT extrapolation over past levels
recovers the synchronous curve and its order p + 1. This tool repeats that
sweep with the GPU solver: the vortex on [0,10]^2 with 8x8 virtual
subdomains, n x n elements, degree p, run to t_end with a time step
proportional to h^r (r = (p+1)/3 keeps SSP-RK3's time error below the
spatial one at degree 3), and reports the L2 errors against the exact
solution and the slopes between consecutive meshes.

    python -m paper_2603_28710_amd.convergence [--ns 32 64 128 256] [--degree 3]

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


def run(mode, n, degree, L, parts, t_end, cfl, r, n_ref, seed=0, problem=0):
    """L2 errors (density, momentum, energy) at t_end on the n x n mesh; the
    step is the CFL step of the n_ref mesh scaled by (n_ref / n)^r"""
    from paper_2603_28710_amd.solver import Solver

    asy = dict(MODES[mode])
    asy.setdefault("L", L)
    levels = 1 if asy["ghost"] == 1 else 3

    def make(m):
        s = Solver(dim=2, degree=degree, cells=(m, m, 1), parts=(parts, parts, 1), lo=(0, 0, 0),
                   hi=(10, 10, 1), levels=levels, seed=seed, **asy)
        s.init_problem(problem)
        return s

    ref = make(n_ref)
    dt_ref = ref.stable_dt(cfl)
    ref.close()
    dt = dt_ref * (n_ref / n) ** r
    nst = int(math.ceil(t_end / dt))
    s = make(n)
    s.step(nst, t_end / nst)
    err = s.error_norms(problem)
    s.close()
    return err, nst


def slopes(errs):
    return [[math.log2(a / b) for a, b in zip(e0, e1)] for e0, e1 in zip(errs[:-1], errs[1:])]


def sweep(modes, ns, degree=3, L=3, parts=8, t_end=1.0, cfl=0.1, r=None, emit=print):
    r = (degree + 1) / 3.0 if r is None else r
    out = {}
    for mode in modes:
        errs = []
        for n in ns:
            err, nst = run(mode, n, degree, L, parts, t_end, cfl, r, ns[0])
            errs.append(list(err))
            emit(json.dumps({"mode": mode, "n": n, "degree": degree, "L": L, "steps": nst, "l2": list(err)}))
        out[mode] = (errs, slopes(errs))
        emit(json.dumps({"mode": mode, "slopes": out[mode][1]}))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ns", type=int, nargs="+", default=[32, 64, 128, 256])
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--L", type=int, default=3)
    ap.add_argument("--parts", type=int, default=8)
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--cfl", type=float, default=0.1)
    ap.add_argument("--r", type=float, default=None)
    ap.add_argument("--modes", nargs="+", default=list(MODES))
    a = ap.parse_args()
    sweep(a.modes, a.ns, a.degree, a.L, a.parts, a.t_end, a.cfl, a.r, emit=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
