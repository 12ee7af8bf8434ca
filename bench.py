#!/usr/bin/env python3
"""ADMM iter/s + PSD clique projections/s at 1e-4 residual, FP32-eig vs FP64.

One "step" is one iteration of Algorithm 1 (scatter, affine projection with
the cached factor, all clique PSD projections, multiplier update, residuals)
over the whole instance.  The default workload is the banded SDP: n = 2000,
half-bandwidth 15 (1985 overlapping cliques of 16), m = 1000 dense-on-pattern
N(0,1) constraints, b_i = tr A_i, C = I + sum y0_i A_i, seed 0.  Inputs are
synthetic (seeded), resident in HBM before timing starts.

Timed region: W untimed warm-up iterations, then exactly K iterations in the
FP32-eig form (eigensolves in FP32, affine step / multipliers / residuals in
FP64) between HIP events on the solver's stream.  The same is done for the
plain FP64 form, and both forms are also solved to max(eps_c, eps_lambda) <=
1e-4 from a cold start (iterations and time to solution reported).  Per-stage
times come from HIP events around back-to-back launches of each kernel stage
(sdp_time_stages); the dominant stage is reported against its roofline.  The CPU oracle is timed on
a bounded sample of the same workload on the host cores.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_TFLOPS = 157.3
FP64_VECTOR_TFLOPS = 78.6

WORKLOADS = {
    "banded": "banded n=2000, half-bandwidth 15 (1985 cliques of 16), m=1000 dense N(0,1) "
              "constraints, seed 0",
    "small": "block-arrow l=10 d=10 h=5 (n=105, 10 cliques of 15), m=100, seed 0",
    "large": "block-arrow l=40 d=120 h=8 (n=4808, 40 cliques of 128), m=4000, 0.5% dense A, "
             "seed 0",
    "batched": "512 independent block-arrow SDPs, l~U[5,50], d~U[8,40], h~U[2,10], m=n//2, "
               "seeds 0..511, solved together",
    "adjoint": "64 block-arrow SDPs l=50 d=16 h=8 (n=808, 50 cliques of 24), m=400, seeds 0..63: "
               "200 unrolled iterations checkpointed every 20, forward + reverse sweep",
    "large_m": "banded n=20000, half-bandwidth 15 (19985 cliques of 16), m=40000 sparse "
               "constraints of 64 N(0,1) coordinates each, seed 0; affine step by Jacobi-"
               "preconditioned conjugate gradients, 3 steps per iteration (no m x m factor)",
    "nonchordal": "45 x 45 grid graph pattern (n=2025, nonchordal), m=200 sparse (5%) N(0,1) "
                  "constraints, seed 0, solved on its chordal extension (minimum-degree "
                  "elimination fill: 1540 maximal cliques of 3..76 vertices)",
    "projection": "standalone batched PSD projection (sdp_psd_project_batched): 4096 GOE blocks "
                  "(symmetric N(0,1), about half the eigenvalues negative) per size "
                  "s in {15, 16, 24, 32, 50, 64, 96, 128}, seed = s",
}
# solver options of workloads that need more than the defaults
EXTRA_OPTIONS = {"large_m": dict(cg_max_iter=3, cg_tol=0.0)}
# precision forms each workload is timed in
FORMS = {"banded": ("fp32", "fp64"), "small": ("fp32", "fp64"), "large": ("fp32", "fp64"),
         "batched": ("fp32", "fp64"), "nonchordal": ("fp32", "fp64"), "large_m": ("fp32", "fp64"),
         "adjoint": ("fp32", "fp64"), "projection": ("fp32", "fp64")}


def make_instances(name, batch_count):
    import sdpgen
    if name == "banded":
        return [sdpgen.workload_banded()]
    if name == "small":
        return [sdpgen.workload_small_blockarrow()]
    if name == "large":
        return [sdpgen.workload_large_cliques()]
    if name == "batched":
        return sdpgen.workload_batched(range(batch_count))
    if name == "adjoint":
        return sdpgen.workload_adjoint(range(min(batch_count, 64)))
    if name == "nonchordal":
        return [sdpgen.workload_nonchordal()]
    if name == "large_m":
        return [sdpgen.workload_large_m()]
    raise SystemExit(f"unknown workload {name}")


def stage_bytes_flops(insts, precision, sweeps, algorithm="primal", cg_steps=0):
    """Algorithmic HBM bytes (or FLOPs) per launch of each stage, summed over
    the instances of the batch.  Dense A is streamed as B = L^-1 A (same size)
    and needs no triangular passes; sparse A is streamed as CSR (12 bytes per
    nonzero) plus the two triangular factors.  The projection's figure is the
    method's work, 10 s^3 per clique of s (9 s^3 for a symmetric
    eigendecomposition with vectors, s^3 for the rebuild), whatever the
    kernel executes (Jacobi sweeps, warm-start and Newton-Schulz products, or
    the sign iteration's products; the compute counters give that); `sweeps`
    is kept for the callers and no longer enters it.
    With the conjugate-gradient affine step (cg_steps per iteration) A is
    streamed as itself; each step is one column pass (A^T p, written as
    W D^-1 A^T p), one row pass (A v) and the per-instance row-vector update
    (11 row vectors of 8 bytes); the start reads r and diag and writes z, p."""
    import numpy as np
    tot = {k: 0 for k in ("scatter", "A_v", "Linv_r", "LinvT_y", "AT_y", "residual", "proj",
                          "cg_solve")}
    for inst in insts:
        m, nnz = inst.m, inst.nnz
        sizes = inst.clique_sizes().astype(np.int64)
        npk = int(np.sum(sizes * (sizes + 1) // 2))
        tot["scatter"] += 8 * 2 * npk + 4 * npk + 8 * 5 * nnz
        tot["residual"] += 8 * 6 * inst.p
        tot["proj"] += int(np.sum(10 * sizes ** 3))
        if cg_steps > 0:
            abytes = 12 * int(inst.a_rowptr[-1]) if inst.a_format == 1 else 8 * m * nnz
            tot["scatter"] += 8 * nnz                      # A^T y of the last solve
            tot["A_v"] += abytes + 8 * nnz + 16 * m
            tot["cg_solve"] += 32 * m + cg_steps * (2 * abytes + 32 * nnz + 104 * m)
            tot["AT_y"] += abytes + 8 * m + 32 * nnz
        elif inst.a_format == 1 or algorithm == "hsde":
            # sparse A, or the embedding (which keeps A and both triangular passes)
            abytes = 12 * int(inst.a_rowptr[-1]) if inst.a_format == 1 else 8 * m * nnz
            tri = 8 * m * (m + 1) // 2
            tot["A_v"] += abytes + 8 * nnz + 16 * m
            tot["Linv_r"] += tri + 16 * m
            tot["LinvT_y"] += tri + 16 * m
            tot["AT_y"] += abytes + 8 * m + 24 * nnz
        else:
            bbytes = 8 * m * nnz
            tot["A_v"] += bbytes + 8 * nnz + 16 * m
            tot["AT_y"] += bbytes + 8 * m + 24 * nnz
    d = {k: dict(bound="hbm", bytes=v) for k, v in tot.items() if k != "proj" and v > 0}
    d["projection"] = dict(bound="alu", flops=tot["proj"],
                           peak_tflops=FP32_VECTOR_TFLOPS if precision == "fp32"
                           else FP64_VECTOR_TFLOPS)
    return d


# source file of each stage's kernels (a summary is stale once that file changes)
STAGE_SOURCE = {"scatter": "k_affine.hip", "A_v": "k_affine.hip", "Linv_r": "k_affine.hip",
                "cg_solve": "k_affine.hip",
                "LinvT_y": "k_affine.hip", "AT_y": "k_affine.hip", "residual": "k_affine.hip",
                "projection": "k_project.hip"}


def source_hash(fname):
    with open(os.path.join(ROOT, "paper_1707_05058_amd", "csrc", fname), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def load_traffic(workload, stage):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current source of the stage's kernel."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get("stages", {}).get(stage)
    if ent is None or ent.get("source_hash") != source_hash(STAGE_SOURCE[stage]):
        return None
    return ent.get("hbm_bytes_per_launch")


# kernels of each stage as rocprofv3 names them, (prefix, suffix) pairs; the
# projection is the FP32-eig form's ADMM-mode kernel (template mode 0, or 3 with the
# positive/negative decoupling compiled in)
STAGE_KERNELS = {"scatter": (("k_scatter", ""),), "A_v": (("k_rowdot<", ""), ("k_csr_rowdot", "")),
                 "Linv_r": (("k_trmv_wave<0>", ""),), "LinvT_y": (("k_trmv_wave<1>", ""),),
                 "AT_y": (("k_coldot<0,", ""), ("k_csc_coldot<0>", "")),
                 "projection": (("k_project<float", ", 0, false>"), ("k_project<float", ", 0, true>"),
                                ("k_project<float", ", 3, false>"), ("k_admm_sign<float", "")),
                 "residual": (("k_residual_reduce", ""),)}
COPY_CAL_BYTES = 512 << 20
COMPUTE_UNITS = 256


def _short_kernel(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0] if not name.startswith("__") else name


def _csv_rows(root, suffix):
    import csv
    import glob
    files = glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {root}")
    return list(csv.DictReader(open(files[0])))


def summarize_rocprof(workload, trace_dir, fetch_dir, write_dir, commands):
    """Turns rocprofv3 CSV output (one --kernel-trace --stats run, one --pmc
    FETCH_SIZE run, one --pmc WRITE_SIZE run of this script) into
    profiles/kernel_trace_<workload>.md and profiles/traffic_<workload>.json.
    The HBM counters are scaled by what they read for a plain copy of
    COPY_CAL_BYTES (the --copy-calibration run), per launch of each stage.
    With "-" for both counter directories it writes the kernel trace only."""
    stats = _csv_rows(trace_dir, "kernel_stats.csv")
    trace_only = fetch_dir == "-" and write_dir == "-"
    lines = [f"# Kernel trace{'' if trace_only else ' and HBM traffic'}, {workload} workload "
             f"({WORKLOADS[workload]})", "",
             "Commands (repository root, one MI355X; each rocprofv3 run in its own process):", "",
             "```"] + commands + ["```", "",
             "| kernel | calls | total (us) | average (us) | % |", "|---|---:|---:|---:|---:|"]
    for r in (stats if trace_only else stats[:25]):
        lines.append(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['AverageNs']) / 1e3:.3f} | "
                     f"{float(r['Percentage']):.1f} |")
    if trace_only:
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", f"kernel_trace_{workload}.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return

    def per_kernel(rows):
        acc = {}
        for r in rows:
            name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
            val = float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
            acc.setdefault(name, []).append(val)
        return acc

    fetch = per_kernel(_csv_rows(fetch_dir, "counter_collection.csv"))
    write = per_kernel(_csv_rows(write_dir, "counter_collection.csv"))

    def copy_kib(acc):
        vals = [v for n, vs in acc.items() if "copyBuffer" in n for v in vs]
        return max(vals) if vals else None

    cf, cw = copy_kib(fetch), copy_kib(write)
    if not cf or not cw:
        raise SystemExit("no copy-calibration dispatch found (run with --copy-calibration)")
    kib = COPY_CAL_BYTES / 1024.0
    sf, sw = kib / cf, kib / cw
    out = {"workload": workload,
           "copy_calibration": {"bytes": COPY_CAL_BYTES, "fetch_kib": cf, "write_kib": cw,
                                "fetch_scale": sf, "write_scale": sw},
           "stages": {}}
    lines += ["", f"HBM counters per launch (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, mean over "
              f"the launches within 10% of the largest, "
              f"scaled by a {COPY_CAL_BYTES >> 20} MiB copy: fetch x{sf:.3f}, write x{sw:.3f}):", "",
              "| stage | kernels | full launches | fetch (MB) | write (MB) | HBM bytes per launch |",
              "|---|---|---:|---:|---:|---:|"]
    for stage, pats in STAGE_KERNELS.items():
        f_names = [n for n in fetch
                   if any(_short_kernel(n).startswith(p) and _short_kernel(n).endswith(q)
                          for p, q in pats)]
        if not f_names:
            continue
        fv = [v for n in f_names for v in fetch[n]]
        wv = [v for n in f_names for v in write.get(n, [])]
        if not fv or not wv:
            continue
        # launches with every instance active: in a batch solved to
        # tolerance, finished instances skip their work, so the launches of
        # the late iterations move fewer bytes; those within 10% of the
        # largest dispatch are the full ones
        fv = [v for v in fv if v >= 0.9 * max(fv)]
        wv = [v for v in wv if v >= 0.9 * max(wv)]
        fb = sum(fv) / len(fv) * sf * 1024.0
        wb = sum(wv) / len(wv) * sw * 1024.0
        out["stages"][stage] = {"kernels": sorted({_short_kernel(n) for n in f_names}),
                                "source": STAGE_SOURCE[stage],
                                "source_hash": source_hash(STAGE_SOURCE[stage]),
                                "launches": len(fv), "fetch_bytes_per_launch": fb,
                                "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb}
        lines.append(f"| {stage} | {', '.join('`%s`' % k for k in out['stages'][stage]['kernels'])} | "
                     f"{len(fv)} | {fb / 1e6:.2f} | {wb / 1e6:.2f} | {fb + wb:.4g} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"kernel_trace_{workload}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


# compute counters of the --summarize-counters passes (rocprofv3 --pmc, one
# pass per group; at most 8 SQ and 2 GRBM counters in one pass)
COUNTER_PASSES = (
    ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES",
     "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU",
     "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"),
    ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
     "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_LDS", "SQ_WAVES",
     "SQ_INSTS_SALU"),
)
FP32_MATRIX_TFLOPS = 157.3      # dense FP32 MFMA peak
FP64_MATRIX_TFLOPS = 78.6
SIMDS = 4 * COMPUTE_UNITS
CLOCK_GHZ = 2.4
KERNEL_SOURCES = (("k_project", "k_project.hip"), ("k_admm_sign", "k_project.hip"),
                  ("k_adj_proj", "k_adjoint.hip"), ("k_", "k_affine.hip"))


def kernel_source(short):
    for prefix, src in KERNEL_SOURCES:
        if short.startswith(prefix):
            return src
    return None


def summarize_counters(workload, trace_dir, pass_dirs, commands, kernels_prefix=("k_",)):
    """Executed work of each kernel from rocprofv3 --pmc passes (COUNTER_PASSES)
    and its mean duration from a --kernel-trace --stats run of the same
    command: matrix-core FLOPs (SQ_INSTS_VALU_MFMA_MOPS_* x 512), vector FP
    FLOPs (64 lanes x (ADD + MUL + 2 FMA) instructions; transcendental and
    other instructions are counted, not converted to flops), MFMA busy
    fraction (SQ_VALU_MFMA_BUSY_CYCLES over all SIMDs at 2.4 GHz for the
    kernel's duration).  Writes profiles/counters_<workload>.md and .json."""
    stats = {_short_kernel(r["Name"]): float(r["AverageNs"]) for r in
             _csv_rows(trace_dir, "kernel_stats.csv")}
    vals = {}
    for d in pass_dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            name = _short_kernel(r.get("Kernel_Name") or r.get("Kernel-Name") or "")
            cn = r.get("Counter_Name") or r.get("Counter-Name") or ""
            v = float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
            vals.setdefault(name, {}).setdefault(cn, []).append(v)
    out = {"workload": workload, "clock_ghz": CLOCK_GHZ, "simds": SIMDS, "kernels": {}}
    lines = [f"# Compute counters, {workload} workload ({WORKLOADS[workload]})", "",
             "Commands (repository root, one MI355X; each rocprofv3 run in its own process):", "",
             "```"] + commands + ["```", "",
             "Per launch: matrix-core FLOPs = 512 x SQ_INSTS_VALU_MFMA_MOPS_{F32,F64}; vector "
             "FLOPs = 64 x (ADD + MUL + 2 FMA) wave instructions; MFMA busy = "
             "SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x 2.4 GHz x mean duration).", "",
             "| kernel | launches | mean (us) | MFMA GFLOP | VALU F32 GFLOP | VALU F64 GFLOP | "
             "executed TFLOP/s | % FP32 matrix peak | MFMA busy | VALU instr. | LDS instr. |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name in sorted(vals, key=lambda n: -stats.get(n, 0.0)):
        if not name.startswith(tuple(kernels_prefix)) or name not in stats:
            continue
        c = {k: sum(v) / len(v) for k, v in vals[name].items()}
        launches = max(len(v) for v in vals[name].values())
        t = stats[name] * 1e-9
        mf = 512.0 * (c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) + c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0))
        v32 = 64.0 * (c.get("SQ_INSTS_VALU_ADD_F32", 0.0) + c.get("SQ_INSTS_VALU_MUL_F32", 0.0)
                      + 2.0 * c.get("SQ_INSTS_VALU_FMA_F32", 0.0))
        v64 = 64.0 * (c.get("SQ_INSTS_VALU_ADD_F64", 0.0) + c.get("SQ_INSTS_VALU_MUL_F64", 0.0)
                      + 2.0 * c.get("SQ_INSTS_VALU_FMA_F64", 0.0))
        tf = (mf + v32 + v64) / t / 1e12 if t > 0 else 0.0
        busy = (c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (SIMDS * CLOCK_GHZ * 1e9 * t)
                if t > 0 else 0.0)
        src = kernel_source(name)
        ent = {"launches": launches, "mean_us": t * 1e6, "mfma_flops_per_launch": mf,
               "valu_f32_flops_per_launch": v32, "valu_f64_flops_per_launch": v64,
               "executed_tflops": tf, "frac_fp32_matrix_peak": tf / FP32_MATRIX_TFLOPS,
               "mfma_busy": busy, "counters": c, "source": src,
               "source_hash": source_hash(src) if src else None}
        out["kernels"][name] = ent
        lines.append(f"| `{name}` | {launches} | {t * 1e6:.2f} | {mf / 1e9:.4f} | {v32 / 1e9:.4f} | "
                     f"{v64 / 1e9:.4f} | {tf:.2f} | {100 * tf / FP32_MATRIX_TFLOPS:.1f} | "
                     f"{100 * busy:.1f}% | {c.get('SQ_INSTS_VALU', 0.0):.4g} | "
                     f"{c.get('SQ_INSTS_LDS', 0.0):.4g} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"counters_{workload}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", f"counters_{workload}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))
    return out


def load_counters(workload, kernel):
    """Counter record of one kernel from profiles/counters_<workload>.json, if
    it was taken on the kernel's current source."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path))["kernels"].get(kernel)
    except Exception:
        return None
    if not ent or not ent.get("source") or ent.get("source_hash") != source_hash(ent["source"]):
        return None
    return ent


def copy_calibration(torch):
    """A plain device-to-device copy of COPY_CAL_BYTES, for scaling the HBM
    counters (rocprofv3 --pmc) of the same run."""
    src = torch.ones(COPY_CAL_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def graph_chunk_for(steps, warmup, cap=50):
    """Iterations per captured graph for the timed run: the largest divisor of
    gcd(K, W) up to `cap` (of K alone without warm-up), so that W warm-up
    iterations build the graph and K timed ones are whole graph launches."""
    g = math.gcd(steps, warmup) if warmup > 0 else steps
    return max(d for d in range(1, min(g, cap) + 1) if g % d == 0)


def timed_steps(S, torch, stream, steps, warmup):
    """W untimed iterations, then exactly K between HIP events on the solver's
    stream; returns (milliseconds, stats before, stats after)."""
    with torch.cuda.stream(stream):
        S.step(warmup, results=False)
        torch.cuda.synchronize()
        st0 = S.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.step(steps, results=False)
        e1.record(stream)
        e1.synchronize()
        torch.cuda.synchronize()
    return e0.elapsed_time(e1), st0, S.stats()


def time_form(sdp, torch, insts, precision, steps, warmup, stage_iters, stream, repeat_solve=True,
              algorithm="primal", extra=None, eager=True):
    out = {}
    extra = dict(extra or {})
    p_total = sum(i.p for i in insts)
    # --- solve to the 1e-4 residual from a cold start (second solve timed) ---
    t0 = time.perf_counter()
    S = sdp.Solver(insts, tol=1e-4, max_iter=20000, precision=precision,
                   stream=stream.cuda_stream, algorithm=algorithm, **extra)
    torch.cuda.synchronize()
    out["setup_s"] = time.perf_counter() - t0
    with torch.cuda.stream(stream):
        if repeat_solve:
            S.solve()
            S.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rs = S.solve()
        e1.record(stream)
        e1.synchronize()
    t_sol = e0.elapsed_time(e1) / 1e3
    its = [r["iters"] for r in rs]
    out["solve"] = dict(iters_to_tol=max(its), iters_mean=sum(its) / len(its),
                        converged=sum(r["status"] == 0 for r in rs), instances=len(rs),
                        time_to_tol_s=t_sol, iter_per_s=max(its) / t_sol,
                        instance_iter_per_s=sum(its) / t_sol,
                        objective=rs[0]["objective"], eps_c=max(r["eps_c"] for r in rs),
                        eps_lambda=max(r["eps_lambda"] for r in rs))
    out["objectives"] = [r["objective"] for r in rs]
    out["jacobi_sweeps_per_projection"] = (S.stats()["jacobi_sweeps"] /
                                           max(S.stats()["projections"], 1))
    two = [sdp.projection_variant_two_level(sdp.DTYPE_FP32 if precision == "fp32" else sdp.DTYPE_FP64, v)
           for v in S.projection_plan_variants()]
    out["projection_plan"] = [dict(N=n, threads=t, cliques=c, two_level=tl)
                              for (n, t, c), tl in zip(S.projection_plan(), two)]
    if extra.get("cg_max_iter"):
        out["solve"]["cg_steps_per_iteration"] = S.cg_steps() / max(sum(its), 1)
    S.close()
    # --- the contract: W warm-up + exactly K timed iterations, through the
    # captured-graph path a solve takes: the graph holds a number of iterations
    # that divides both W and K, so the warm-up captures and instantiates it
    # and the timed K iterations are graph launches only ---
    chunk = graph_chunk_for(steps, warmup)
    out["graph_chunk"] = chunk
    S = sdp.Solver(insts, tol=0.0, max_iter=10 ** 8, precision=precision,
                   stream=stream.cuda_stream, algorithm=algorithm, graph_chunk=chunk, **extra)
    ms, st0, st1 = timed_steps(S, torch, stream, steps, warmup)
    out["ms_per_step"] = ms / steps
    out["iter_per_s"] = steps / (ms / 1e3)
    out["projections_per_s"] = out["iter_per_s"] * p_total
    out["instance_iter_per_s"] = out["iter_per_s"] * len(insts)
    out["timed_sweeps_per_projection"] = ((st1["jacobi_sweeps"] - st0["jacobi_sweeps"]) /
                                          max(st1["projections"] - st0["projections"], 1))
    if eager:
        # the same W + K with plain launches (no graph), for comparison
        E = sdp.Solver(insts, tol=0.0, max_iter=10 ** 8, precision=precision,
                       stream=stream.cuda_stream, algorithm=algorithm, graph_chunk=0, **extra)
        ms_e, _, _ = timed_steps(E, torch, stream, steps, warmup)
        E.close()
        out["eager_ms_per_step"] = ms_e / steps
        out["eager_iter_per_s"] = steps / (ms_e / 1e3)
    stages = S.time_stages(stage_iters)
    if extra.get("cg_max_iter"):
        # the solve sits in the slot of the first substitution; there is no second
        stages = {("cg_solve" if k == "Linv_r" else k): v for k, v in stages.items()
                  if k != "LinvT_y"}
    out["stages_ms"] = stages
    S.close()
    return out


def batched_leg(args, sdp, torch, stream):
    """The batched half of the metric beside the headline: the 512-instance
    workload in one handle, FP32-eig and FP64 (W warm-up + at most 100 timed
    iterations each through captured graphs, and a solve of every instance to
    1e-4 from a cold start), against a loop of per-instance FP64 solves."""
    insts = make_instances("batched", args.batch_count)
    steps = min(args.steps, 100)
    out = {"workload": WORKLOADS["batched"], "steps": steps, "warmup": args.warmup}
    keep = ("setup_s", "graph_chunk", "ms_per_step", "iter_per_s", "instance_iter_per_s",
            "projections_per_s", "stages_ms", "solve")
    for precision in ("fp32", "fp64"):
        print(f"[bench] batched {precision}: timing", file=sys.stderr, flush=True)
        f = time_form(sdp, torch, insts, precision, steps, args.warmup, args.stage_iters, stream,
                      repeat_solve=False, eager=False, extra=solver_options(args))
        out["fp32_eig" if precision == "fp32" else "fp64"] = {k: f[k] for k in keep if k in f}
        if precision == "fp32":
            # the longest stage of the batched FP32 iteration, with the counter
            # traffic of profiles/traffic_batched.json when it is current
            out["roofline"] = roofline_of(insts, f["stages_ms"], f["timed_sweeps_per_projection"],
                                          "primal", solver_options(args), "batched")
        print(f"[bench] batched {precision}: {f['iter_per_s']:.1f} batched iter/s",
              file=sys.stderr, flush=True)
    print("[bench] batched: loop of per-instance FP64 solves", file=sys.stderr, flush=True)
    loop = time_loop(sdp, torch, insts[:32], "fp64", min(steps, 100), 10, stream, len(insts))
    out["loop_fp64"] = loop
    f32, f64 = out["fp32_eig"], out["fp64"]
    out["speedup_fp32_vs_fp64_iter_per_s"] = f32["iter_per_s"] / f64["iter_per_s"]
    out["speedup_fp32_vs_fp64_time_to_tol"] = (f64["solve"]["time_to_tol_s"] /
                                               f32["solve"]["time_to_tol_s"])
    out["speedup_batched_fp32_vs_loop_fp64"] = (f32["instance_iter_per_s"] /
                                                loop["instance_iter_per_s"])
    return out


def time_loop(sdp, torch, insts, precision, steps, warmup, stream, total):
    """The batch as a loop of per-instance solves: one handle per instance
    (each with its own captured graph), stepped one after another on the same
    stream.  `insts` is a sample of the batch; the time of one iteration of
    every sampled instance is extrapolated linearly to `total` instances."""
    handles = [sdp.Solver([i], tol=0.0, max_iter=10 ** 8, precision=precision,
                          stream=stream.cuda_stream) for i in insts]
    try:
        with torch.cuda.stream(stream):
            for S in handles:
                S.step(warmup, results=False)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for S in handles:
                S.step(steps, results=False)
            e1.record(stream)
            e1.synchronize()
        ms_round = e0.elapsed_time(e1) / steps          # one iteration of each sampled instance
    finally:
        for S in handles:
            S.close()
    ms_all = ms_round * total / len(insts)
    return dict(precision=precision, instances_timed=len(insts), steps=steps,
                ms_per_iteration_of_all=ms_all, instance_iter_per_s=total / (ms_all / 1e3),
                sample=f"instances 0..{len(insts) - 1} of {total}, each its own handle, "
                       f"{steps} iterations each; extrapolated linearly to {total}")


def time_adjoint(sdp, torch, insts, precision, T, ckpt, stream):
    """Unrolled forward (T iterations, checkpoints every ckpt) and the reverse
    sweep of <C, X_T>, timed with HIP events on the solver's stream."""
    out = {}
    dev = torch.device("cuda:0")
    S = sdp.Solver(insts, tol=0.0, max_iter=10 ** 7, precision=precision,
                   stream=stream.cuda_stream)
    u = torch.zeros(S.total_nnz, dtype=torch.float64, device=dev)
    import numpy as np
    ubar = torch.from_numpy(np.concatenate([i.c for i in insts])).to(dev)
    cb = torch.zeros_like(u)
    bb = torch.zeros(S.total_m, dtype=torch.float64, device=dev)
    with torch.cuda.stream(stream):
        S.unrolled_forward(2, 1, u)            # warm-up (allocations, code paths)
        S.vjp(ubar, cb, bb)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        S.unrolled_forward(T, ckpt, u)
        ev[1].record(stream)
        S.vjp(ubar, cb, bb)
        ev[2].record(stream)
        ev[2].synchronize()
    tf, tb = ev[0].elapsed_time(ev[1]) / 1e3, ev[1].elapsed_time(ev[2]) / 1e3
    S.close()
    p_total = sum(i.p for i in insts)
    out.update(T=T, ckpt_every=ckpt, forward_s=tf, backward_s=tb,
               iter_per_s=T / tf, ms_per_step=1e3 * tf / T,
               projections_per_s=T * p_total / tf,
               backward_iter_per_s=T / tb, backward_over_forward=tb / tf,
               grad_norm_c=float(cb.norm()), grad_norm_b=float(bb.norm()))
    return out, cb.cpu().numpy(), bb.cpu().numpy()


def roofline_of(insts, stages_ms, sweeps, algorithm, extra, workload):
    """Roofline of the longest stage: algorithmic bytes (or flops) per launch
    over its mean launch time, with the counter traffic of the workload's
    profile when one is committed for the current kernel source."""
    model = stage_bytes_flops(insts, "fp32", sweeps, algorithm,
                              cg_steps=extra.get("cg_max_iter", 0))
    stages = {k: v for k, v in stages_ms.items() if k in model}
    dom = max(stages, key=lambda k: stages[k])
    t_launch = stages[dom] / 1e3
    info = model[dom]
    if info["bound"] == "hbm":
        achieved = info["bytes"] / t_launch / 1e9
        return dict(kernel=dom, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=load_traffic(workload, dom),
                    algorithmic_bytes_per_launch=info["bytes"], launch_ms=stages[dom])
    achieved = info["flops"] / t_launch / 1e12
    # one workgroup per clique: a launch of fewer cliques than compute units
    # leaves the rest idle, so the fraction of the occupied units is given too
    wgs = sum(len(inst.clique_sizes()) for inst in insts)
    occupied = min(wgs, COMPUTE_UNITS) / COMPUTE_UNITS
    return dict(kernel=dom, bound="alu", achieved=achieved, peak=info["peak_tflops"],
                unit="TFLOP/s", frac=achieved / info["peak_tflops"],
                traffic=load_traffic(workload, dom),
                model_flops_per_launch=info["flops"], launch_ms=stages[dom],
                workgroups=wgs, frac_of_occupied_units=achieved / (info["peak_tflops"] * occupied))


def projection_roofline(insts, stages_ms, workload, precision="fp32"):
    """The projection stage against the FP32 (or FP64) matrix peak: the
    method's work (10 s^3 per clique) per launch over the stage's mean launch
    time, and, from the workload's committed compute-counter profile when it
    was taken on the current kernel source, the work the dominant projection
    kernel executed per launch (matrix-core plus vector FLOPs) over the same
    time, with its MFMA busy fraction."""
    import numpy as np
    sizes = np.concatenate([i.clique_sizes().astype(np.int64) for i in insts])
    model = float(np.sum(10 * sizes ** 3))
    t = stages_ms["projection"] / 1e3
    peak = FP32_MATRIX_TFLOPS if precision == "fp32" else FP64_MATRIX_TFLOPS
    out = dict(stage="projection", model="10 s^3 per clique", model_flops_per_launch=model,
               launch_ms=stages_ms["projection"], model_tflops=model / t / 1e12,
               peak_tflops=peak, model_frac=model / t / 1e12 / peak, counters=None)
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if os.path.exists(path):
        try:
            ks = json.load(open(path))["kernels"]
        except Exception:
            ks = {}
        tag = "<float" if precision == "fp32" else "<double"
        cand = [n for n in ks if (n.startswith("k_admm_sign" + tag) or n.startswith("k_project" + tag))]
        if cand:
            name = max(cand, key=lambda n: ks[n]["mean_us"] * ks[n]["launches"])
            ent = load_counters(workload, name)
            if ent is not None:
                ex = (ent["mfma_flops_per_launch"] + ent["valu_f32_flops_per_launch"]
                      + ent["valu_f64_flops_per_launch"])
                out["counters"] = dict(kernel=name, executed_flops_per_launch=ex,
                                       executed_tflops=ex / t / 1e12,
                                       executed_frac=ex / t / 1e12 / peak,
                                       mfma_busy=ent["mfma_busy"],
                                       profile_mean_us=ent["mean_us"])
    return out


def solver_options(args):
    """Per-workload solver options plus the command line's."""
    extra = dict(EXTRA_OPTIONS.get(args.workload, {}))
    if args.decouple is not None:
        extra["decouple"] = args.decouple
    if args.projection_method is not None:
        extra["projection_method"] = args.projection_method
    if args.autotune is not None:
        extra["autotune"] = args.autotune
    return extra


def cpu_baseline(insts, seconds, algorithm="primal", extra=None):
    """The oracle on a bounded sample: the first instances of the workload,
    a few iterations each; the per-iteration time of the whole batch is the
    sum over instances, extrapolated from the sampled ones."""
    import oracle
    per_inst = seconds / min(len(insts), 4)
    times, sampled, total_it = [], [], 0
    cg = (extra or {}).get("cg_max_iter", 0)
    for inst in insts[:4]:
        P = oracle.Problem(inst, factor=not cg)
        if cg:
            P.set_affine_cg(cg, (extra or {}).get("cg_tol", 0.0))
        if algorithm == "hsde":
            P.hsde_setup()
            step = P.run_hsde
        else:
            step = P.run_dual if algorithm == "dual" else P.run
        done, t0 = 0, time.perf_counter()
        while True:
            step(2, tol=0.0)
            done += 2
            el = time.perf_counter() - t0
            if el >= per_inst:
                break
        times.append(el / done)
        total_it += done
        sampled.append(inst.name)
    t_iter = sum(times) / len(times) * len(insts)
    what = (f"first {total_it} iterations of Algorithm "
            f"{dict(primal=1, dual=2, hsde=3)[algorithm]} from a "
            f"zero state on "
            f"{len(sampled)} of {len(insts)} instance(s), FP64, setup excluded")
    if cg:
        what += f"; affine step by {cg} conjugate-gradient steps per iteration, as on the GPU"
    if len(insts) > len(sampled):
        what += "; batch time per iteration extrapolated as mean x instance count"
    return dict(value=1.0 / t_iter, unit="iter/s", cores=oracle.max_threads(), kind="oracle",
                sample=what)


def extend_instances(sdp, raw):
    """The library's chordal extension (host) of each nonchordal instance,
    timed; the solver then runs on the extended instances."""
    import numpy as np
    import sdpgen
    out, t_ms, fill = [], [], 0
    for inst in raw:
        t0 = time.perf_counter()
        ext = sdp.extend_instance(inst)
        t_ms.append((time.perf_counter() - t0) * 1e3)
        fill += ext.nnz - inst.nnz
        out.append(sdpgen.Instance(n=ext.n, m=ext.m, pat_row=ext.pat_row, pat_col=ext.pat_col,
                                   clique_ptr=ext.clique_ptr, clique_vert=ext.clique_vert,
                                   a_format=ext.a_format, a_val=ext.a_val, b=ext.b, c=ext.c,
                                   a_rowptr=ext.a_rowptr, a_col=ext.a_col, name=ext.name))
    sizes = np.concatenate([np.diff(i.clique_ptr) for i in out])
    info = dict(chordal_extension_ms=sum(t_ms), fill_entries=int(fill),
                cliques=int(sizes.shape[0]), clique_size_min=int(sizes.min()),
                clique_size_max=int(sizes.max()), clique_size_mean=float(sizes.mean()),
                note="host C++ (sdp_pattern_create + index map + data remap), outside the "
                     "timed iterations")
    print(f"[bench] chordal extension {info}", file=sys.stderr, flush=True)
    return out, info


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="banded", choices=sorted(WORKLOADS))
    ap.add_argument("--stage-iters", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="instances of the batched workload")
    ap.add_argument("--algorithm", default="primal", choices=("primal", "dual", "hsde"),
                    help="Algorithm 1 (domain-space primal ADMM), Algorithm 2 (range-space "
                         "dual ADMM) or Algorithm 3 (ADMM on the homogeneous self-dual embedding)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="start with a plain 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--summarize-rocprof", nargs=3, metavar=("TRACE", "FETCH", "WRITE"),
                    help="write profiles/ summaries from rocprofv3 CSV output directories")
    ap.add_argument("--commands-file", help="text file with the rocprofv3 commands (summaries)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="TRACE PASS1 [PASS2 ...]: write profiles/counters_<workload>.{md,json} "
                         "from a kernel-trace run and rocprofv3 --pmc runs of COUNTER_PASSES")
    ap.add_argument("--decouple", type=int, choices=(0, 1), default=None,
                    help="positive/negative decoupling of warm-started projections "
                         "(default: the library's default)")
    ap.add_argument("--autotune", type=int, choices=(0, 1), default=None,
                    help="time the kernel variants at setup (default: the library's, on)")
    ap.add_argument("--no-batched", action="store_true",
                    help="leave the batched workload out of the banded (default) line")
    ap.add_argument("--projection-method", default=None,
                    choices=("auto", "scalar", "two_level", "sign"),
                    help="eigensolver of the clique projections (default: the library's)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        cmds = open(args.commands_file).read().strip().splitlines() if args.commands_file else []
        summarize_rocprof(args.workload, *args.summarize_rocprof, cmds)
        return
    if args.summarize_counters:
        cmds = open(args.commands_file).read().strip().splitlines() if args.commands_file else []
        summarize_counters(args.workload, args.summarize_counters[0], args.summarize_counters[1:],
                           cmds)
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent instances would shard across GPUs with no communication; "
              "nothing here drives a second GPU)", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import paper_1707_05058_amd as sdp

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
    if args.workload == "projection":
        run_projection(args, sdp, torch, torch.cuda.Stream())
        return
    t0 = time.perf_counter()
    insts = make_instances(args.workload, args.batch_count)
    print(f"[bench] generated {len(insts)} instance(s) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    preprocess = None
    if args.workload == "nonchordal":
        insts, preprocess = extend_instances(sdp, insts)
    stream = torch.cuda.Stream()
    if args.workload == "adjoint":
        run_adjoint(args, sdp, torch, insts, stream)
        return
    forms = {}
    for precision in FORMS[args.workload]:
        print(f"[bench] {args.workload} {precision}: timing", file=sys.stderr, flush=True)
        forms[precision] = time_form(sdp, torch, insts, precision, args.steps, args.warmup,
                                     args.stage_iters, stream,
                                     repeat_solve=args.workload not in ("batched", "large"),
                                     algorithm=args.algorithm,
                                     extra=solver_options(args))
        print(f"[bench] {args.workload} {precision}: {forms[precision]['iter_per_s']:.1f} iter/s",
              file=sys.stderr, flush=True)
    head = forms["fp32"]
    extra = solver_options(args)
    roof = roofline_of(insts, head["stages_ms"], head["timed_sweeps_per_projection"],
                       args.algorithm, extra, args.workload)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(insts, args.cpu_seconds, args.algorithm, extra)

    f32, f64 = forms["fp32"], forms.get("fp64")
    n_cl = sum(i.p for i in insts)
    line = {
        "metric": "ADMM iter/s + PSD clique projections/s at 1e-4 residual, FP32/batched vs FP64",
        "value": head["iter_per_s"],
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-eig/fp64-affine",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "precision": "fp32-eig/fp64-affine",
                   "algorithm": {"primal": "Algorithm 1 (domain-space primal ADMM)",
                                 "dual": "Algorithm 2 (range-space dual ADMM)",
                                 "hsde": "Algorithm 3 (ADMM on the homogeneous self-dual "
                                         "embedding)"}[args.algorithm],
                   "tol": 1e-4, "rho": 1.0, "adaptive_rho": False, "instances": len(insts),
                   "affine_step": (f"PCG, {extra['cg_max_iter']} steps per iteration"
                                   if extra.get("cg_max_iter") else "cached Cholesky factor"),
                   "n": [i.n for i in insts[:4]], "m": [i.m for i in insts[:4]],
                   "cliques": n_cl, "pattern_nnz": sum(i.nnz for i in insts),
                   "projection_decoupling": bool(extra.get("decouple", 1))},
        "projections_per_s": head["projections_per_s"],
        "fp32_eig": {k: v for k, v in f32.items() if k != "objectives"},
        "fp64": None if f64 is None else {k: v for k, v in f64.items() if k != "objectives"},
        "roofline": roof,
        "projection_roofline": projection_roofline(insts, head["stages_ms"], args.workload),
        "cpu_baseline": cpu,
    }
    if preprocess is not None:
        line["preprocess"] = preprocess
    if f64 is not None:
        import numpy as np
        o32, o64 = np.array(f32["objectives"]), np.array(f64["objectives"])
        line["speedup_fp32_vs_fp64_iter_per_s"] = f32["iter_per_s"] / f64["iter_per_s"]
        line["speedup_fp32_vs_fp64_time_to_tol"] = (f64["solve"]["time_to_tol_s"] /
                                                    f32["solve"]["time_to_tol_s"])
        line["objective_rel_diff_fp32_vs_fp64"] = float(np.max(np.abs(o32 - o64) / np.abs(o64)))
    if args.workload == "banded" and not args.no_batched:
        line["batched"] = batched_leg(args, sdp, torch, stream)
    if args.workload == "batched":
        # the batched handle against a loop of per-instance plain FP64 solves
        print("[bench] batched: loop of per-instance FP64 solves", file=sys.stderr, flush=True)
        loop = time_loop(sdp, torch, insts[:32], "fp64", min(args.steps, 100), 10, stream,
                         len(insts))
        line["loop_fp64"] = loop
        line["speedup_batched_fp32_vs_loop_fp64"] = (f32["instance_iter_per_s"] /
                                                     loop["instance_iter_per_s"])
        if f64 is not None:
            line["speedup_batched_fp64_vs_loop_fp64"] = (f64["instance_iter_per_s"] /
                                                         loop["instance_iter_per_s"])
    print(json.dumps(line), flush=True)


PROJ_SIZES = (15, 16, 24, 32, 50, 64, 96, 128)


def sign_products(sdp, prec, N, threads):
    """Matrix-core flops of one sign-function projection of a padded N x N
    block: the library's schedule (sdp.sign_schedule) of k1 fast steps of
    three products, k2 Newton-Schulz steps of two, one final product, at
    2 N 16^2 flops per 16 x 16 tile; the LDS kernels form the TN (TN + 1) / 2
    tiles on or below the diagonal, the one-wave register kernels for N = 32
    all TN^2 (each off-diagonal tile is the other's operand)."""
    tol = 1e-6 if prec == "fp32" else 1e-14
    k1, k2 = sdp.sign_schedule(tol, N)
    tn = N // 16
    tiles = tn * tn if (N == 32 and threads == 64) else tn * (tn + 1) // 2
    return (3 * k1 + 2 * k2 + 1) * tiles * 2 * N * 16 * 16


def run_projection(args, sdp, torch, stream):
    """Kernel-only rate of the batched projection: `count` blocks of one size
    per launch, every kernel variant that fits (the default and the fastest
    reported), timed with HIP events over `steps` launches after `warmup`."""
    import numpy as np
    import sdpgen
    count = 4096
    steps, warmup = max(3, min(args.steps, 20)), max(1, min(args.warmup, 3))
    res = {}
    for prec, npdt, tdt, dtc in (("fp32", np.float32, torch.float32, sdp.DTYPE_FP32),
                                 ("fp64", np.float64, torch.float64, sdp.DTYPE_FP64)):
        variants = sdp.projection_variants(dtc)
        nmax = max(n for n, _ in variants)
        peak = FP32_VECTOR_TFLOPS if prec == "fp32" else FP64_VECTOR_TFLOPS
        for s in PROJ_SIZES:
            if s > nmax:
                continue
            blocks = np.stack(sdpgen.goe_blocks([s] * count, seed=s, dtype=npdt))
            dev = torch.device("cuda:0")
            t_in = torch.from_numpy(blocks.reshape(-1)).to(dev)
            t_out = torch.empty_like(t_in)
            sizes = torch.full((count,), s, dtype=torch.int32, device=dev)
            offs = torch.arange(count, dtype=torch.int64, device=dev) * (s * s)
            n_fit = min(n for n, _ in variants if n >= s + (s & 1))
            kinds = [sdp.projection_variant_kind(dtc, v) for v in range(len(variants))]
            times = {}
            for v, (N, NT) in enumerate(variants):
                if N < s + (s & 1) or N > 2 * n_fit:
                    continue
                with torch.cuda.stream(stream):
                    for _ in range(warmup):
                        sdp.psd_project_batched(sizes, offs, t_in, t_out, s, stream=stream.cuda_stream,
                                                variant=v)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(steps):
                        sdp.psd_project_batched(sizes, offs, t_in, t_out, s, stream=stream.cuda_stream,
                                                variant=v)
                    e1.record(stream)
                    e1.synchronize()
                times[v] = e0.elapsed_time(e1) / steps
            kind_name = {0: "jacobi", 1: "two-level", 2: "sign"}

            def vname(v):
                return f"{variants[v][0]}x{variants[v][1]}-{kind_name[kinds[v]]}"
            bv, bms = min(times.items(), key=lambda kv: kv[1])
            # the variant the library runs without an explicit choice
            dv = sdp.projection_default_variant(dtc, s)
            model = 10.0 * s ** 3 * count
            executed = None
            if kinds[bv] == 2:
                executed = sign_products(sdp, prec, variants[bv][0], variants[bv][1]) * count / (bms / 1e3) / 1e12
            res[f"{prec}_s{s}"] = dict(
                s=s, blocks=count,
                best_variant=dict(N=variants[bv][0], threads=variants[bv][1],
                                  method=kind_name[kinds[bv]]),
                ms_per_launch=bms, projections_per_s=count / (bms / 1e3),
                model_tflops=model / (bms / 1e3) / 1e12,
                model_frac_of_peak=model / (bms / 1e3) / 1e12 / peak,
                default_variant=dict(N=variants[dv][0], threads=variants[dv][1],
                                     method=kind_name[kinds[dv]]),
                default_ms=times[dv],
                executed_matrix_tflops=executed,
                executed_frac_of_peak=None if executed is None else executed / peak,
                all_variants_ms={vname(v): t for v, t in sorted(times.items())})
            print(f"[bench] projection {prec} s={s}: {count / (bms / 1e3):.3e} proj/s "
                  f"({vname(bv)}, {bms:.3f} ms)", file=sys.stderr, flush=True)
            del t_in, t_out
    head = res["fp32_s16"]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        blocks = sdpgen.goe_blocks([16] * 256, seed=16)
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.cpu_seconds and done < len(blocks):
            oracle.psd_project(blocks[done])
            done += 1
        el = time.perf_counter() - t0
        cpu = dict(value=done / el, unit="projections/s", cores=1, kind="oracle",
                   sample=f"{done} GOE blocks of 16 projected one after another (FP64 cyclic "
                          f"Jacobi) in {el:.1f} s")
    line = {
        "metric": "PSD clique projections/s (standalone batched kernel)",
        "value": head["projections_per_s"], "unit": "projections/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": head["ms_per_launch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["projection"], "headline": "FP32, s = 16"},
        "sizes": res,
        "roofline": {"kernel": (("k_project_sign16" if head["best_variant"]["N"] == 16
                                 else "k_project_sign")
                                if head["best_variant"]["method"] == "sign"
                                else "k_project") + f" (N = {head['best_variant']['N']}, "
                               f"{head['best_variant']['threads']} threads, standalone)",
                     "bound": "mfma" if head["best_variant"]["method"] == "sign" else "alu",
                     "achieved": head["model_tflops"], "peak": FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": head["model_frac_of_peak"], "traffic": None,
                     "model": "10 s^3 per block (symmetric eigensolve with vectors 9 s^3, "
                              "rebuild s^3)",
                     "executed": head["executed_matrix_tflops"],
                     "executed_frac": head["executed_frac_of_peak"],
                     "executed_model": "sign method: (3 k1 + 2 k2 + 1) products of the padded "
                                       "N x N block, 2 N 16^2 flops per 16 x 16 tile; the LDS "
                                       "kernels form the TN (TN + 1) / 2 tiles on or below the "
                                       "diagonal (TN = N / 16), the one-wave register kernel "
                                       "for N = 32 all TN^2; FP32 matrix peak"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def run_adjoint(args, sdp, torch, insts, stream):
    import numpy as np
    res, grads = {}, {}
    for precision in FORMS["adjoint"]:
        print(f"[bench] adjoint {precision}", file=sys.stderr, flush=True)
        res[precision], cb, bb = time_adjoint(sdp, torch, insts, precision, 200, 20, stream)
        grads[precision] = (cb, bb)
    (c32, b32), (c64, b64) = grads["fp32"], grads["fp64"]
    head = res["fp32"]
    # the forward iterations are the solver's: stage timing of a handle over
    # the same instances (FP32-eig, fixed penalty, warm-started)
    with torch.cuda.stream(stream):
        S = sdp.Solver(insts, tol=0.0, max_iter=10 ** 8, precision="fp32",
                       stream=stream.cuda_stream)
        S.step(20, results=False)
        st0 = S.stats()
        S.step(20, results=False)
        st1 = S.stats()
        sweeps = ((st1["jacobi_sweeps"] - st0["jacobi_sweeps"]) /
                  max(st1["projections"] - st0["projections"], 1))
        stages = S.time_stages(20)
        S.close()
    roof = roofline_of(insts, stages, sweeps, "primal", {}, "adjoint")
    roof["note"] = "longest stage of the forward iteration (the reverse sweep reuses the same passes)"
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.Problem(insts[0])
        t0 = time.perf_counter()
        P.unrolled_vjp(200, 1.0, insts[0].c)
        el = time.perf_counter() - t0
        cpu = dict(value=200.0 / (el * len(insts)), unit="iter/s", cores=oracle.max_threads(),
                   kind="oracle",
                   sample=f"instance 0 only: 200 unrolled iterations + reverse sweep in {el:.1f} s, "
                          f"FP64; batch rate extrapolated as 1 / (time x {len(insts)})")
    line = {
        "metric": "ADMM iter/s + PSD clique projections/s at 1e-4 residual, FP32/batched vs FP64",
        "value": head["iter_per_s"], "unit": "iter/s", "n_gpus": 1, "steps": 200, "warmup": 2,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32-eig/fp64-affine", "data": "synthetic",
        "config": {"workload": WORKLOADS["adjoint"], "instances": len(insts)},
        "projections_per_s": head["projections_per_s"],
        "fp32_eig": res["fp32"], "fp64": res["fp64"],
        "grad_rel_diff_fp32_vs_fp64": {
            "c": float(np.abs(c32 - c64).max() / np.abs(c64).max()),
            "b": float(np.abs(b32 - b64).max() / np.abs(b64).max())},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
