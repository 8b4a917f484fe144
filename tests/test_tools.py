"""Host-side logic of the measurement tools (no GPU): the algorithmic byte
and flop counts bench.py divides by, and the rocprofv3 CSV summaries of
profile_traffic.py on small synthetic inputs."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2603_28710_amd import profile_traffic as PT  # noqa: E402


def test_algorithmic_bytes_state_and_ring():
    # 64/3 B per DoF (input, u_n on two of three stages, output), plus the AT
    # ring: `levels` levels read and a third of a level written per launch
    nd = 4194304
    assert bench.algorithmic_bytes_per_launch(nd, 0, 2, 3) == pytest.approx(nd * 64 / 3)
    vals = 8192 * 4 * 4  # 256^2 vortex, 8x8 subdomains, p=3: face-sides x V x P
    at = bench.algorithmic_bytes_per_launch(nd, vals, 2, 3)
    assert at - nd * 64 / 3 == pytest.approx(8 * vals * (3 + 1 / 3))
    stale = bench.algorithmic_bytes_per_launch(nd, vals, 1, 3)
    assert stale - nd * 64 / 3 == pytest.approx(8 * vals * (1 + 1 / 3))
    assert bench.algorithmic_bytes_per_launch(nd, vals, 0, 3) == pytest.approx(nd * 64 / 3)


def test_algorithmic_flops_grow_with_degree():
    f = [bench.algorithmic_flops_per_element(2, p + 1, p + 2) for p in (1, 2, 3, 4)]
    assert all(a < b for a, b in zip(f, f[1:]))
    # per DoF the 2D p=3 count is of the order the sum-factorised estimate gives
    per_dof = f[2] / (4 * 16)
    assert 100 < per_dof < 250


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_traffic_summary_scales_by_the_copy(tmp_path):
    copy = "void at::native::vectorized_elementwise_kernel<4, MulFunctor>"
    stage = "void adg::(anonymous namespace)::rhs_stage2d_kernel<double, 4>(adg::Mesh)"
    n = PT.COPY_DOUBLES * 8 / 1024.0  # KiB moved each way by the copy
    fetch = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="FETCH_SIZE", Counter_Value=n / 2),
             dict(Dispatch_Id=2, Kernel_Name=stage, Counter_Name="FETCH_SIZE", Counter_Value=1000.0),
             dict(Dispatch_Id=3, Kernel_Name=stage, Counter_Name="FETCH_SIZE", Counter_Value=3000.0)]
    write = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="WRITE_SIZE", Counter_Value=n),
             dict(Dispatch_Id=2, Kernel_Name=stage, Counter_Name="WRITE_SIZE", Counter_Value=500.0),
             dict(Dispatch_Id=3, Kernel_Name=stage, Counter_Name="WRITE_SIZE", Counter_Value=500.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "s.json"
    _write_csv(fp, fetch)
    _write_csv(wp, write)
    PT.summarize(str(fp), str(wp), "x", str(out))
    d = json.loads(out.read_text())
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    # mean fetch 2000 KiB counted (x2 true), write 500 KiB
    assert d["hbm_bytes_per_launch"] == pytest.approx((2000 * 2 + 500) * 1024.0)
    assert d["kernel"] == "void adg::rhs_stage2d_kernel<double, 4>"
    assert d["source_sha256_16"] == PT.source_hash(d["kernel"])


def test_source_hash_per_stage_kernel():
    # a profile stays valid while its own kernel's translation unit and the
    # shared device headers are unchanged; the other kernels' files do not count
    import hashlib
    import os
    d = os.path.join(PT.ROOT, "paper_2603_28710_amd", "csrc")
    h = hashlib.sha256()
    for f in ("adg_rhs2d.hip", "adg_device.h", "adg_internal.h", "adg_tables.h"):
        h.update(open(os.path.join(d, f), "rb").read())
    assert PT.source_hash("void adg::rhs_stage2d_kernel<float, 5>") == h.hexdigest()[:16]
    assert PT.kernel_base("void adg::rhs_stage3d_split_kernel<double, 4>(adg::Mesh, int)") == \
        "rhs_stage3d_split_kernel"
    hashes = {PT.source_hash(k) for k in PT.KERNEL_FILES}
    assert len(hashes) == len(PT.KERNEL_FILES) and PT.source_hash() not in hashes


def test_sq_summary_is_per_wavefront(tmp_path):
    stage = "void adg::rhs_stage3d_kernel<double, 3>(adg::Mesh)"
    rows = []
    for disp, waves in ((1, 100.0), (2, 300.0)):
        rows += [dict(Dispatch_Id=disp, Kernel_Name=stage, Counter_Name="SQ_WAVES", Counter_Value=waves),
                 dict(Dispatch_Id=disp, Kernel_Name=stage, Counter_Name="SQ_INSTS_VALU", Counter_Value=10 * waves),
                 dict(Dispatch_Id=disp, Kernel_Name="other", Counter_Name="SQ_INSTS_VALU", Counter_Value=1e9)]
    p, out = tmp_path / "a.csv", tmp_path / "sq.txt"
    _write_csv(p, rows)
    PT.sqstats([str(p)], "x", str(out))
    line = [ln for ln in out.read_text().splitlines() if ln.startswith("SQ_INSTS_VALU")][0]
    assert float(line.split()[1]) == pytest.approx(10.0)


def test_algorithmic_bytes_lserk():
    # LSERK: input, accumulator (not at the first stage) and two outputs (one
    # at the last stage): (2,2) (24 + 24) / 2, (3,3) (24 + 32 + 24) / 3 B per DoF
    nd = 1000
    assert bench.algorithmic_bytes_per_launch(nd, 0, 0, 3, integrator=1) == pytest.approx(nd * 24.0)
    assert bench.algorithmic_bytes_per_launch(nd, 0, 0, 3, integrator=2) == pytest.approx(nd * 80.0 / 3.0)
