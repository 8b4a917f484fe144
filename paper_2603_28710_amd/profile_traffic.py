"""HBM traffic of the fused stage kernel from rocprofv3 counters.

run:        executes a benchmark workload for a few steps, then a plain
            elementwise copy of known size (the calibration kernel). Meant to
            be run under `rocprofv3 --pmc FETCH_SIZE` and, separately,
            `rocprofv3 --pmc WRITE_SIZE`.
summarize:  reads the two counter CSVs, scales the stage kernel's per-dispatch
            FETCH_SIZE / WRITE_SIZE by what the same counters read for the copy
            (known bytes / counter reading), and writes the JSON summary that
            bench.py picks up (it is ignored once the kernel source changes).
"""
import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_DOUBLES = 32 * 1024 * 1024  # 256 MiB read + 256 MiB written per copy


KERNEL_SOURCES = ("adg_rhs.hip", "adg_rhs2d.hip", "adg_internal.h", "adg_tables.h")


def source_hash():
    """first 16 hex digits of the SHA-256 of the stage kernel's sources"""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
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
    s.init_problem(w["problem"])
    dt = s.stable_dt(0.1)
    s.step(steps, dt)
    torch.cuda.synchronize()
    src = torch.ones(COPY_DOUBLES, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"ran {workload} for {steps} steps and 3 copies of {COPY_DOUBLES * 8} bytes", flush=True)


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
        return sum(vals) / len(vals), len(vals), ks[0].split("(")[0]

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
    res = {
        "kernel": kname, "workload": workload, "source_sha256_16": source_hash(),
        "fetch_kib_per_dispatch": rf, "write_kib_per_dispatch": rw, "dispatches": [nf, nw],
        "copy_kernel": copy_name[0][:80], "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_bytes_per_launch": rf * 1024.0 * f_scale + rw * 1024.0 * w_scale,
    }
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


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
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.steps)
    else:
        summarize(a.fetch, a.write, a.workload, a.out)


if __name__ == "__main__":
    main()
