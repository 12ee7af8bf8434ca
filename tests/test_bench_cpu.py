"""The measurement tooling of bench.py, on the CPU: the one-GPU guard, the
algorithmic byte counts the rooflines divide by, both roofline forms, and
the rocprofv3 summarizer (kernel trace, and HBM counters scaled by the
copy calibration) on synthetic CSV files written to a temporary root."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import sdpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_banded_pass_bytes():
    """The passes over B = L^-1 A stream m x |E_l| FP64 entries plus their
    vectors; nothing else of size m^2 (the triangular passes are folded)."""
    inst = sdpgen.workload_banded()
    m, nnz = inst.m, inst.nnz
    assert (m, nnz) == (1000, 31880)
    model = bench.stage_bytes_flops([inst], "fp32", 1.0)
    assert model["A_v"]["bytes"] == 8 * m * nnz + 8 * nnz + 16 * m
    assert model["AT_y"]["bytes"] == 8 * m * nnz + 8 * m + 24 * nnz
    assert "Linv_r" not in model and "LinvT_y" not in model
    sizes = inst.clique_sizes().astype(np.int64)
    assert model["projection"]["flops"] == int(np.sum(10 * sizes ** 3))   # the method's work


def test_roofline_hbm_and_alu_forms():
    inst = sdpgen.workload_banded()
    r = bench.roofline_of([inst], {"A_v": 0.040, "AT_y": 0.038, "projection": 0.016,
                                   "scatter": 0.004}, 1.0, "primal", {}, "no_such_workload")
    assert r["kernel"] == "A_v" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(r["algorithmic_bytes_per_launch"] / 40e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    assert r["traffic"] is None                       # no committed profile of that name
    # a projection-bound instance: 40 cliques of 128 occupy 40 of the 256 units
    big = sdpgen.workload_large_cliques()
    r = bench.roofline_of([big], {"projection": 0.150, "A_v": 0.035}, 0.0, "primal", {},
                          "no_such_workload")
    assert r["kernel"] == "projection" and r["bound"] == "alu"
    assert r["workgroups"] == 40
    assert r["frac_of_occupied_units"] == pytest.approx(r["frac"] * 256 / 40)


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarizer_trace_only_and_counters(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_1707_05058_amd" / "csrc")
    for f in set(bench.STAGE_SOURCE.values()):
        (tmp_path / "paper_1707_05058_amd" / "csrc" / f).write_text("// source " + f)
    trace = tmp_path / "trace"
    _write_csv(str(trace / "run" / "t_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void k_coldot<0, false>(AffineArgs)", 10, 380000, 38000, 60.0],
                ["void k_project<float, 16, 64, 0, false>(ProjArgs, int const*)", 10, 160000,
                 16000, 40.0]])
    # trace only: every kernel listed, no traffic file
    bench.summarize_rocprof("banded", str(trace), "-", "-", ["cmd one"])
    md = (tmp_path / "profiles" / "kernel_trace_banded.md").read_text()
    assert "`k_coldot<0, false>` | 10 | 380.0 | 38.000 |" in md
    assert "`k_project<float, 16, 64, 0, false>`" in md and "cmd one" in md
    assert not (tmp_path / "profiles" / "traffic_banded.json").exists()
    # with counters: a 512 MiB copy reads as 256 MiB fetched (x2) and 512 MiB written (x1)
    kib = bench.COPY_CAL_BYTES / 1024
    hdr = ["Kernel_Name", "Counter_Value"]
    _write_csv(str(tmp_path / "fetch" / "f_counter_collection.csv"), hdr,
               [["__amd_rocclr_copyBuffer", kib / 2],
                ["void k_coldot<0, false>(AffineArgs)", 2900.0],
                ["void k_coldot<0, false>(AffineArgs)", 1000.0],   # instances finished
                ["void k_coldot<0, false>(AffineArgs)", 3000.0]])
    _write_csv(str(tmp_path / "write" / "w_counter_collection.csv"), hdr,
               [["__amd_rocclr_copyBuffer", kib],
                ["void k_coldot<0, false>(AffineArgs)", 29.0],
                ["void k_coldot<0, false>(AffineArgs)", 10.0],
                ["void k_coldot<0, false>(AffineArgs)", 30.0]])
    bench.summarize_rocprof("banded", str(trace), str(tmp_path / "fetch"),
                            str(tmp_path / "write"), ["cmd two"])
    t = json.loads((tmp_path / "profiles" / "traffic_banded.json").read_text())
    assert t["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert t["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    st = t["stages"]["AT_y"]
    # the mean over the full launches (within 10% of the largest dispatch)
    assert st["launches"] == 2
    assert st["fetch_bytes_per_launch"] == pytest.approx(2950.0 * 2 * 1024)
    assert st["write_bytes_per_launch"] == pytest.approx(29.5 * 1024)
    # the stage is tied to its source: the traffic goes stale when it changes
    assert bench.load_traffic("banded", "AT_y") == pytest.approx(st["hbm_bytes_per_launch"])
    (tmp_path / "paper_1707_05058_amd" / "csrc" / bench.STAGE_SOURCE["AT_y"]).write_text("// new")
    assert bench.load_traffic("banded", "AT_y") is None


def test_projection_roofline_and_counter_summary(tmp_path, monkeypatch):
    """The projection block of the bench line: 10 s^3 per clique over the
    stage time; the counter summary turns MFMA and vector counts into FLOPs
    per launch, and the bench line takes the executed work of the dominant
    projection kernel only while its source is unchanged."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_1707_05058_amd" / "csrc")
    for f in ("k_project.hip", "k_affine.hip", "k_adjoint.hip"):
        (tmp_path / "paper_1707_05058_amd" / "csrc" / f).write_text("// source " + f)
    inst = sdpgen.workload_banded()
    r = bench.projection_roofline([inst], {"projection": 0.010}, "banded")
    model = 10.0 * 1985 * 16 ** 3
    assert r["model_flops_per_launch"] == pytest.approx(model)
    assert r["model_tflops"] == pytest.approx(model / 10e-6 / 1e12)
    assert r["counters"] is None
    trace = tmp_path / "trace"
    _write_csv(str(trace / "t_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void k_admm_sign<float, 1>(ProjArgs, int const*, int, int)", 4, 40000, 10000, 50.0],
                ["void k_coldot<0, false>(AffineArgs)", 4, 40000, 10000, 50.0]])
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    kname = "void k_admm_sign<float, 1>(ProjArgs, int const*, int, int)"
    _write_csv(str(tmp_path / "p1" / "a_counter_collection.csv"), hdr,
               [[kname, "SQ_INSTS_VALU_MFMA_MOPS_F32", 1000.0],
                [kname, "SQ_INSTS_VALU_MFMA_MOPS_F32", 3000.0],
                [kname, "SQ_INSTS_VALU_FMA_F32", 10.0],
                [kname, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 2.4e9 * 10e-6 * 0.25]])
    _write_csv(str(tmp_path / "p2" / "b_counter_collection.csv"), hdr,
               [[kname, "SQ_INSTS_VALU_FMA_F64", 5.0]])
    out = bench.summarize_counters("banded", str(trace), [str(tmp_path / "p1"), str(tmp_path / "p2")],
                                   ["cmd"])
    k = out["kernels"]["k_admm_sign<float, 1>"]
    assert k["mfma_flops_per_launch"] == pytest.approx(512 * 2000.0)
    assert k["valu_f32_flops_per_launch"] == pytest.approx(64 * 2 * 10.0)
    assert k["valu_f64_flops_per_launch"] == pytest.approx(64 * 2 * 5.0)
    assert k["mfma_busy"] == pytest.approx(0.25)
    r = bench.projection_roofline([inst], {"projection": 0.010}, "banded")
    ex = 512 * 2000.0 + 64 * 2 * 10.0 + 64 * 2 * 5.0
    assert r["counters"]["executed_flops_per_launch"] == pytest.approx(ex)
    assert r["counters"]["executed_tflops"] == pytest.approx(ex / 10e-6 / 1e12)
    (tmp_path / "paper_1707_05058_amd" / "csrc" / "k_project.hip").write_text("// changed")
    assert bench.projection_roofline([inst], {"projection": 0.010}, "banded")["counters"] is None
