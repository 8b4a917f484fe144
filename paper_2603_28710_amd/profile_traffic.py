"""HBM traffic and kernel timings of the fused stage kernel from rocprofv3.

run:        executes a benchmark workload for a few steps, then a plain
            elementwise copy of known size (the calibration kernel). Meant to
            be run under `rocprofv3 --pmc FETCH_SIZE` and, separately,
            `rocprofv3 --pmc WRITE_SIZE`.
summarize:  reads the two counter CSVs, scales the stage kernel's per-dispatch
            FETCH_SIZE / WRITE_SIZE by what the same counters read for the copy
            (known bytes / counter reading), and writes the JSON summary that
            bench.py picks up (it is ignored once the kernel source changes).
kstats:     turns the kernel_stats.csv of `rocprofv3 --kernel-trace --stats`
            into a short text table, headed by the command that produced it.
sqstats:    per-wavefront averages of the SQ counter passes (instruction
            mix, issue and wait cycles) of the stage kernel.
"""
import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_DOUBLES = 32 * 1024 * 1024  # 256 MiB read + 256 MiB written per copy


KERNEL_SOURCES = ("adg_rhs.hip", "adg_rhs2d.hip", "adg_rhs3d.hip", "adg_rhs3d_split.hip", "adg_device.h",
                  "adg_internal.h", "adg_tables.h")
SHARED_HEADERS = ("adg_device.h", "adg_internal.h", "adg_tables.h")
# each stage kernel and its launcher live in one translation unit of their
# own, with the shared device headers; the learned predictor's kernel lives
# with the network's code and headers
KERNEL_FILES = {"rhs_stage2d_kernel": ("adg_rhs2d.hip",) + SHARED_HEADERS,
                "rhs_stage3d_kernel": ("adg_rhs3d.hip",) + SHARED_HEADERS,
                "rhs_stage3d_split_kernel": ("adg_rhs3d_split.hip",) + SHARED_HEADERS,
                "rhs_stage_kernel": ("adg_rhs.hip",) + SHARED_HEADERS,
                "ghost_learned_kernel": ("adg_mlp.hip", "adg_mlp.h", "adg_ctx.h", "adg_internal.h")}


def kernel_base(name):
    """'void adg::rhs_stage3d_kernel<double, 3>' -> 'rhs_stage3d_kernel'"""
    return _short(name).replace("void ", "").split("<")[0].split("::")[-1].strip()


def source_hash(kernel=None):
    """first 16 hex digits of the SHA-256 of a kernel's sources: its own
    translation unit and the headers it includes (every stage kernel's
    sources when kernel is None)"""
    files = KERNEL_SOURCES if kernel is None else KERNEL_FILES[kernel_base(kernel)]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2603_28710_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run(workload, steps):
    sys.path.insert(0, ROOT)
    import torch

    import bench
    from paper_2603_28710_amd.solver import Solver

    w = bench.WORKLOADS[workload]
    s = Solver(device="cuda:0", precision=w["precision"], **w["cfg"], **w["asy"])
    s.init_problem(w["problem"], w.get("params"))
    if w["asy"]["ghost"] == 3:
        # the ghost kernel's traffic and work do not depend on the weights
        s.predictor_init(w.get("train", {}).get("seed", 1))
    dt = s.stable_dt(w.get("cfl", 0.1))
    s.step(steps, dt)
    torch.cuda.synchronize()
    src = torch.ones(COPY_DOUBLES, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"ran {workload} for {steps} steps and 3 copies of {COPY_DOUBLES * 8} bytes", flush=True)


def _short(name):
    """kernel name without the anonymous-namespace tag and argument list"""
    return name.replace("(anonymous namespace)::", "").split("(")[0]


def _per_dispatch(path, counter):
    """kernel name -> list of per-dispatch counter values (summed over
    dimensions/instances of one dispatch)"""
    per = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row.get("Kernel_Name"))
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (_, name), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def summarize(fetch_csv, write_csv, workload, out):
    fe = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wr = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, needle):
        ks = [k for k in d if needle in k]
        if not ks:
            raise SystemExit(f"no kernel matching {needle}")
        vals = sum((d[k] for k in ks), [])
        return sum(vals) / len(vals), len(vals), _short(ks[0])

    # the elementwise multiply (reads and writes COPY_DOUBLES doubles); not
    # the fill kernel that created its input
    copy_name = [k for k in fe if "elementwise" in k and "Fill" not in k]
    if not copy_name:
        raise SystemExit("calibration copy kernel not found")
    cf = sum(fe[copy_name[0]]) / len(fe[copy_name[0]])
    cw = sum(wr[copy_name[0]]) / len(wr[copy_name[0]])
    f_scale = COPY_DOUBLES * 8 / (cf * 1024.0)
    w_scale = COPY_DOUBLES * 8 / (cw * 1024.0)
    rf, nf, kname = pick(fe, "rhs_stage")
    rw, nw, _ = pick(wr, "rhs_stage")
    cmd = ("rocprofv3 --pmc {c} --output-format csv -d <dir> -o p -- python3 "
           "paper_2603_28710_amd/profile_traffic.py run --steps 2 --workload " + workload)
    res = {
        "kernel": kname, "workload": workload, "source_sha256_16": source_hash(kname),
        "fetch_command": cmd.format(c="FETCH_SIZE"), "write_command": cmd.format(c="WRITE_SIZE"),
        "summary_command": "python3 paper_2603_28710_amd/profile_traffic.py summarize --fetch <fetch csv> "
                           "--write <write csv> --workload " + workload + " --out <this file>",
        "fetch_kib_per_dispatch": rf, "write_kib_per_dispatch": rw, "dispatches": [nf, nw],
        "copy_kernel": copy_name[0][:80], "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_bytes_per_launch": rf * 1024.0 * f_scale + rw * 1024.0 * w_scale,
    }
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def first_dispatches(trace_csv, match, n):
    """(count, average us) of the first n dispatches, in launch order, of the
    kernel whose name contains match, from a rocprofv3 kernel-trace CSV"""
    d = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            if match in r["Kernel_Name"]:
                d.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    d.sort()
    d = d[:n]
    return len(d), (sum(x[1] for x in d) / len(d) / 1e3 if d else 0.0)


def kstats(stats_csv, command, out, trace_csv=None, match=None, first=None):
    rows = []
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            rows.append((_short(r["Name"])[:72], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                         float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    # the stage kernel that takes the most time names the sources hashed
    stage = next((r[0] for r in rows if "rhs_stage" in r[0]), None)
    lines = [f"# rocprofv3 kernel statistics ({kernel_base(stage) + ' ' if stage else ''}kernel sources "
             f"sha256/16 {source_hash(stage)})",
             f"# command: {command}", "",
             f"{'kernel':72s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for n, c, t, a, lo, hi, pct in rows:
        lines.append(f"{n:72s} {c:6d} {t:11.1f} {a:9.2f} {lo:9.2f} {hi:9.2f} {pct:6.2f}")
    if trace_csv and match and first:
        # the command's own timed run launches first: its launches alone,
        # apart from those of the comparison runs that follow
        cnt, avg = first_dispatches(trace_csv, match, first)
        lines += ["", f"# first {cnt} dispatches of {match} (the command's first, timed run; from the kernel "
                      f"trace): avg_us {avg:.2f}"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_PASSES = {
    "A": "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM SQ_INSTS_VALU_FMA_F64 "
         "SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64",
    "B": "SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU "
         "SQ_ACTIVE_INST_SCA SQ_ACTIVE_INST_LDS",
    "C": "SQ_WAVES SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT",
}


def sqstats(csvs, workload, out, match="rhs_stage"):
    """per-wavefront averages of the SQ counters of the kernel whose name
    contains match (the stage kernel by default), from one counter CSV per
    pass (rocprofv3 collects each pass in its own run)"""
    per = {}
    kname = None
    for path in csvs:
        disp = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if match not in row["Kernel_Name"]:
                    continue
                kname = kname or _short(row["Kernel_Name"])
                d = disp.setdefault(row["Dispatch_Id"], {})
                d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
        for d in disp.values():
            w = d.get("SQ_WAVES", 0.0)
            for c, val in d.items():
                if c != "SQ_WAVES" and w > 0:
                    per.setdefault(c, []).append(val / w)
    cmd = ("rocprofv3 --pmc {counters} --output-format csv -d <dir> -o p -- python3 "
           "paper_2603_28710_amd/profile_traffic.py run --steps 2 --workload " + workload)
    lines = [f"# rocprofv3 SQ counters of {kname}, per wavefront (kernel sources sha256/16 "
             f"{source_hash(kname if kname and kernel_base(kname) in KERNEL_FILES else None)})",
             f"# workload {workload}; one run per pass:"]
    lines += [f"#   pass {k}: " + cmd.format(counters=v) for k, v in SQ_PASSES.items()]
    lines += ["# (the cycle counters SQ_WAVE_CYCLES, SQ_WAIT_* and SQ_ACTIVE_* tick once per 4 clocks)", ""]
    for c in sorted(per):
        v = per[c]
        lines.append(f"{c:28s} {sum(v) / len(v):12.1f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="vortex256_p3_at3_uniformL3")
    r.add_argument("--steps", type=int, default=3)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--workload", default="vortex256_p3_at3_uniformL3")
    s.add_argument("--out", required=True)
    k = sub.add_parser("kstats")
    k.add_argument("--stats", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--trace", default=None, help="kernel-trace CSV of the same run")
    k.add_argument("--match", default=None, help="kernel name substring for --first")
    k.add_argument("--first", type=int, default=None, help="average the first N such dispatches")
    q = sub.add_parser("sqstats")
    q.add_argument("--csv", nargs="+", required=True)
    q.add_argument("--workload", default="vortex256_p3_at3_uniformL3")
    q.add_argument("--out", required=True)
    q.add_argument("--match", default="rhs_stage", help="kernel name substring")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.steps)
    elif a.cmd == "summarize":
        summarize(a.fetch, a.write, a.workload, a.out)
    elif a.cmd == "sqstats":
        sqstats(a.csv, a.workload, a.out, a.match)
    else:
        kstats(a.stats, a.command, a.out, a.trace, a.match, a.first)


if __name__ == "__main__":
    main()
