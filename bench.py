#!/usr/bin/env python3
"""Throughput of the asynchronous DG solver with AT neighbour traces on one
MI355X: DOF-updates per second per SSP-RK3 stage.

A step is one full SSP-RK3 step over the whole mesh: 3 launches of the fused
stage kernel, which also publishes the ring traces (stage 0) and builds the
delayed / AT neighbour traces at the PE-boundary faces. Inputs are synthetic and resident in HBM before the timed region.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2603_28710_amd import profile_traffic  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

# Workloads (synthetic, analytic initial states). The default is the 2D
# isentropic vortex on the periodic [0,10]^2 box, 256x256 quads, degree 3,
# 8x8 virtual subdomains, AT extrapolation over 3 past levels, delays drawn
# uniformly in {0..3} per step, subdomain and face direction.
WORKLOADS = {
    "vortex256_p3_at3_uniformL3": dict(
        cfg=dict(dim=2, degree=3, cells=(256, 256, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=2, delay_kind=1, L=3, levels=3, seed=0), problem=0, precision=0),
    # synchronous references of the 256^2 vortex and the 64^3 density wave
    # (no ring, no delays): the cost of the asynchronous machinery on one GPU
    "vortex256_p3_sync": dict(
        cfg=dict(dim=2, degree=3, cells=(256, 256, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=0, delay_kind=0, L=0, levels=3, seed=0), problem=0, precision=0),
    "wave64_p3_sync": dict(
        cfg=dict(dim=3, degree=3, cells=(64, 64, 64), parts=(4, 4, 4), lo=(0, 0, 0), hi=(1, 1, 1)),
        asy=dict(ghost=0, delay_kind=0, L=0, levels=3, seed=0), problem=1, precision=0),
    "vortex16_p2_sync": dict(
        cfg=dict(dim=2, degree=2, cells=(16, 16, 1), parts=(1, 1, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=0, delay_kind=0, L=0, levels=3, seed=0), problem=0, precision=0),
    "wave64_p3_at3_fixedL2": dict(
        cfg=dict(dim=3, degree=3, cells=(64, 64, 64), parts=(4, 4, 4), lo=(0, 0, 0), hi=(1, 1, 1)),
        asy=dict(ghost=2, delay_kind=0, L=2, levels=3, seed=0), problem=1, precision=0),
    "vortex1024_p4_at3_uniformL3_fp32": dict(
        cfg=dict(dim=2, degree=4, cells=(1024, 1024, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=2, delay_kind=1, L=3, levels=3, seed=0), problem=0, precision=1,
        reference="vortex1024_p4_at3_uniformL3_fp64"),
    "vortex1024_p4_at3_uniformL3_fp64": dict(
        cfg=dict(dim=2, degree=4, cells=(1024, 1024, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=2, delay_kind=1, L=3, levels=3, seed=0), problem=0, precision=0),
    # uniform delays up to 4 need CFL 0.05 to stay stable over long runs
    "wave128_p2_at3_uniformL4": dict(
        cfg=dict(dim=3, degree=2, cells=(128, 128, 128), parts=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1)),
        asy=dict(ghost=2, delay_kind=1, L=4, levels=3, seed=0), problem=1, precision=0, cfl=0.05),
    # the learned ghost predictor (untrained, Glorot-initialised network from
    # a fixed seed: inference and the per-face judge cost the same whatever
    # the weights; a face whose correction exceeds the bound keeps AT)
    "wave128_p2_learned_uniformL4": dict(
        cfg=dict(dim=3, degree=2, cells=(128, 128, 128), parts=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1)),
        asy=dict(ghost=3, delay_kind=1, L=4, levels=3, seed=0, learned_tol=1e-6), problem=1, precision=0,
        cfl=0.05, net_seed=1, reference="wave128_p2_at3_uniformL4"),
    # the paper's low-storage LSERK(3,3) instead of SSP-RK3 (same stage kernel)
    "vortex256_p3_at3_uniformL3_lserk33": dict(
        cfg=dict(dim=2, degree=3, cells=(256, 256, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1),
                 integrator=2),
        asy=dict(ghost=2, delay_kind=1, L=3, levels=3, seed=0), problem=0, precision=0),
    # the paper's own communication-avoiding algorithm with AT fluxes
    "vortex256_p3_fluxat3_caaL3": dict(
        cfg=dict(dim=2, degree=3, cells=(256, 256, 1), parts=(8, 8, 1), lo=(0, 0, 0), hi=(10, 10, 1)),
        asy=dict(ghost=5, delay_kind=2, L=3, levels=3, seed=0), problem=0, precision=0),
    # the paper's own accuracy run at its finest mesh: the vortex of mean flow
    # (1,0) in the Dirichlet box [0,10] x [-5,5], degree 2, 16x16 subdomains,
    # Alg. caa-at with L = 4, AT3, LSERK(3,3), CFL 0.05
    "paper_vortex256_p2_at3_caaL4_lserk33": dict(
        cfg=dict(dim=2, degree=2, cells=(256, 256, 1), parts=(16, 16, 1), lo=(0, -5, 0), hi=(10, 5, 1),
                 integrator=2, boundary=1),
        asy=dict(ghost=2, delay_kind=2, L=4, levels=3, seed=0), problem=0, params=(5.0, 0.0, 5.0, 1.0, 0.0),
        precision=0, cfl=0.05),
}
DEFAULT = "vortex256_p3_at3_uniformL3"
PROFILE_EVERY = 8


def algorithmic_bytes_per_launch(ndof, nfs_nodes_vars, ghost, levels, integrator=0, bnd_values=0):
    """Minimum HBM bytes of one fused stage launch, averaged over the stages
    of a step: for SSP-RK3 the stage input read once, u^n read on stages 2
    and 3, the output written (8 B each per DoF: 64/3 B per DoF); for
    LSERK(2,2) / (3,3) the input, the accumulator w (except at the first
    stage, where it is the input) and two outputs (one at the last stage):
    24 and 80/3 B per DoF; for SSP-RK2 the input read, u^n read at the
    second stage, the output written: 20 B per DoF; at PE-boundary faces
    the ring levels read (one for stale traces, `levels` for AT, the
    predictor's ghost buffer for learned traces) and, at stage 0, one level
    written (nfs_nodes_vars values per level). The flux-history modes are
    counted by their state traffic only (their flux ring traffic depends on
    the schedule), so their figure is a lower bound. In a Dirichlet box the
    stage also reads the boundary data (bnd_values values)."""
    ring = 0.0
    if ghost in (1, 2, 3) and nfs_nodes_vars > 0:
        ring = 8.0 * nfs_nodes_vars * ((levels if ghost == 2 else 1) + 1.0 / 3.0)
    per_dof = {0: 64.0 / 3.0, 1: 24.0, 2: 80.0 / 3.0, 3: 20.0}[integrator]
    return ndof * per_dof + ring + 8.0 * bnd_values


def algorithmic_flops_per_element(dim, P, Q):
    """Flops of one element-stage of the sum-factorised operator (FMA = 2):
    d interpolation sweeps nodes->Gauss points, the Euler flux at every Gauss
    point, d collocation-derivative sweeps, d transposed interpolation sweeps,
    the face fluxes on 2d faces (trace interpolation of both sides, LLF flux,
    lift) and d inverse-mass sweeps, plus the RK combine."""
    V = dim + 2
    if dim == 2:
        interp = V * (P * P * Q + Q * P * Q)
        Fq, Fn = Q, P
    else:
        interp = V * (P * P * P * Q + Q * P * P * Q + Q * Q * P * Q)
        Fq, Fn = Q * Q, P * P
    Qd, Pd, nf = Q ** dim, P ** dim, 2 * dim
    deriv = dim * V * Qd * Q                 # FMAs
    test = interp                            # FMAs (transposed sweeps)
    traces = 2 * nf * Fq * V * Fn            # FMAs, both sides at each face Gauss point
    lift = nf * V * Fn * Fq                  # FMAs
    minv = dim * V * Pd * P                  # FMAs
    flux_qp = 12 + dim * (2 * V + 3)         # pressure, 1/rho, d scaled flux columns
    llf = 60 + 2 * V                         # two normal fluxes, wave speeds, scaling
    combine = 4 * V * Pd
    return 2 * (interp + deriv + test + traces + lift + minv) + Qd * flux_qp + nf * Fq * llf + combine


def load_traffic(workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"rhs_stage_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256_16") != profile_traffic.source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, target_s=15.0, cells=None):
    """The FP64 CPU oracle, untuned, on a bounded sample of the same workload:
    the full mesh (or `cells` elements per direction, same subdomain count),
    a few steps (as many as fit in about target_s seconds). The thread count
    is OMP_NUM_THREADS, else the usable cores up to 16."""
    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if threads <= 0:
        threads = min(len(os.sched_getaffinity(0)), 16)
        os.environ["OMP_NUM_THREADS"] = str(threads)
    c, a = w["cfg"], w["asy"]
    integ = c.get("integrator", 0)
    mesh = c["cells"] if cells is None else tuple(cells if k < c["dim"] else 1 for k in range(3))
    o = O.Oracle(dim=c["dim"], p=c["degree"], cells=mesh, parts=c["parts"], lo=c["lo"], hi=c["hi"],
                 ghost=a["ghost"], delay_kind=a["delay_kind"], L=a["L"], levels=a["levels"], seed=a["seed"],
                 integrator=integ, bc=c.get("boundary", 0), bc_problem=w["problem"], bc_params=w.get("params"))
    o.init_problem(w["problem"], w.get("params"))
    dt = o.stable_dt(w.get("cfl", 0.1))
    t0 = time.perf_counter()
    o.step(1, dt)
    t1 = time.perf_counter()
    n = max(1, min(2000, int(target_s / max(t1 - t0, 1e-3)) - 1))
    t2 = time.perf_counter()
    o.step(n, dt)
    t3 = time.perf_counter()
    return {"value": o.ndof * (2 if integ in (1, 3) else 3) * n / (t3 - t2), "unit": "DOF-updates/s per RK stage",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{'full mesh' if cells is None else 'mesh %d^%d' % (cells, c['dim'])}, {n} "
                      f"{['SSP-RK3', 'LSERK(2,2)', 'LSERK(3,3)', 'SSP-RK2'][integ]} steps after 1 warm-up "
                      f"step ({t3 - t2:.1f} s)"}


def run_steps(w, steps, warmup):
    """a solver of workload w stepped warmup + steps times at the workload's
    CFL; returns (solver, dt, wall seconds of the timed steps)"""
    import torch

    from paper_2603_28710_amd import binding as B
    from paper_2603_28710_amd.solver import Solver

    c, a = w["cfg"], w["asy"]
    s = Solver(device="cuda:0", precision=w["precision"], **c, **a)
    s.init_problem(w["problem"], w.get("params"))
    if a["ghost"] == B.ADG_GHOST_LEARNED:
        s.predictor_init(w["net_seed"])
    dt = s.stable_dt(w.get("cfl", 0.1))
    s.step(warmup, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step_status(steps, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if st != 0:
        raise RuntimeError(B.adg_last_error())
    return s, dt, t1 - t0


def matched_error(s, sec, ref_name, steps, warmup):
    """the workload's FP64 reference (same mesh, initial state, dt and step
    count) run after the timed region: relative L2 difference of the states
    (density, momentum, energy) and the reference's time over this one's"""
    r, _, rsec = run_steps(WORKLOADS[ref_name], steps, warmup)
    diff = s.diff_norm(r.download())
    r.close()
    return {"reference": ref_name, "rel_l2_vs_reference": list(diff), "speedup_vs_reference": rsec / sec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-only", action="store_true",
                    help="print only the cpu_baseline object of the workload (no GPU)")
    ap.add_argument("--cpu-cells", type=int, default=None,
                    help="with --cpu-only: elements per direction of a reduced mesh")
    args = ap.parse_args()
    if args.cpu_only:
        out = cpu_baseline(WORKLOADS[args.workload], cells=args.cpu_cells)
        out["workload"] = args.workload
        print(json.dumps(out), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_28710_amd import binding as B
    from paper_2603_28710_amd.solver import Solver

    w = WORKLOADS[args.workload]
    c, a = w["cfg"], w["asy"]
    s = Solver(device="cuda:0", precision=w["precision"], **c, **a)
    s.init_problem(w["problem"], w.get("params"))
    if a["ghost"] == B.ADG_GHOST_LEARNED:
        s.predictor_init(w["net_seed"])
    cfl = w.get("cfl", 0.1)
    dt = s.stable_dt(cfl)
    s.step(args.warmup, dt)
    torch.cuda.synchronize()

    # HIP events around the stage launches of every PROFILE_EVERY-th step:
    # the average launch duration of the roofline, without putting the
    # events' own cost (a few microseconds per pair) into every step
    B.adg_profile(s.h, PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step_status(args.steps, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if st != 0:
        raise RuntimeError(B.adg_last_error())
    rhs_ms, rhs_n = B.adg_profile_read(s.h, B.ADG_KERNEL_RHS)
    gh_ms, gh_n = B.adg_profile_read(s.h, B.ADG_KERNEL_GHOST)
    B.adg_profile(s.h, 0)

    sec = t1 - t0
    stages = (2 if c.get("integrator", 0) in (B.ADG_LSERK22, B.ADG_SSPRK2) else 3) * args.steps
    value = s.ndof * stages / sec
    nfs = B.adg_delay(s.h, s.time()[0], 0, 0)[1]
    Fn = (c["degree"] + 1) ** (c["dim"] - 1)
    # in a Dirichlet box (2D) the boundary faces keep unused slots in the
    # face-side enumeration: count only the PE face-sides, 2 (parts_a - 1)
    # interface lines of cells_b faces per axis a
    if c.get("boundary", 0):
        px, py = c["parts"][0], c["parts"][1]
        nfs = 2 * (px - 1) * c["cells"][1] * (px > 1) + 2 * (py - 1) * c["cells"][0] * (py > 1)
    bnd_values = 2 * (c["cells"][0] + c["cells"][1]) * s.V * (c["degree"] + 1) if c.get("boundary", 0) else 0
    bytes_launch = algorithmic_bytes_per_launch(s.ndof, nfs * s.V * Fn, a["ghost"], a["levels"],
                                                c.get("integrator", 0), bnd_values)
    avg_s = rhs_ms / max(rhs_n, 1) / 1e3
    achieved = bytes_launch / avg_s / 1e9
    P, Q = c["degree"] + 1, c["degree"] + 2
    flops_launch = algorithmic_flops_per_element(c["dim"], P, Q) * s.E
    fpeak = FP32_PEAK_TFLOPS if w["precision"] else FP64_PEAK_TFLOPS
    traffic = load_traffic(args.workload)
    err = s.error_norms(w["problem"], w.get("params")) if w["problem"] in (0, 1) else None

    out = {
        "metric": "DOF-updates/s per RK stage",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-contract/f64-state" if w["precision"] else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": c["dim"], "degree": c["degree"],
                   "cells": list(c["cells"][: c["dim"]]), "parts": list(c["parts"][: c["dim"]]),
                   "ghost": ["sync", "stale", "at", "learned", "flux_stale", "flux_at"][a["ghost"]],
                   "levels": a["levels"],
                   "delay": ["fixed", "uniform", "caa"][a["delay_kind"]], "L": a["L"], "seed": a["seed"],
                   "dofs": s.ndof, "elements": s.E, "dt": dt, "cfl": cfl,
                   "integrator": ["ssprk3", "lserk22", "lserk33", "ssprk2"][c.get("integrator", 0)],
                   "boundary": ["periodic", "dirichlet"][c.get("boundary", 0)]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "rhs_stage", "avg_launch_us": avg_s * 1e6, "launches": rhs_n,
                     "event_sampling": f"stage launches of every {PROFILE_EVERY}th step",
                     "algorithmic_bytes_per_launch": bytes_launch},
        "alu": {"achieved_tflops": flops_launch / avg_s / 1e12, "peak_tflops": fpeak,
                "frac": flops_launch / avg_s / 1e12 / fpeak, "flops_per_launch": flops_launch},
        "ghost_kernel": {"avg_launch_us": gh_ms / max(gh_n, 1) * 1e3, "launches": gh_n},
        "l2_error_vs_exact": err,
    }
    if a["ghost"] == B.ADG_GHOST_LEARNED:
        rate, judged = s.predictor_stats()
        out["ghost_kernel"].update({"faces_judged": judged, "accept_rate": rate})
    if "reference" in w:
        out["matched_error"] = matched_error(s, sec, w["reference"], args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
