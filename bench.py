#!/usr/bin/env python3
"""Benchmark of the CBFM + Calderon-preconditioned PMCHWT hot path on one
MI355X.

One step = the whole path for one scatterer and its batch of incidences:
primary CBFs with dual orthogonalisation (cbfm_build_cbf), the PMCHWT fill
fused with the projection Z_r = (C^JM)^H Z C^MJ (cbfm_project) and the
right-preconditioned GMRES solve of every incidence to its monostatic RCS
(cbfm_solve).  The mesh is loaded and resident on the device before the
timed region.

Workload (default): dielectric cylinder r 1, h 6 wavelengths, eps_r 3,
19,968 triangles (29,952 RWGs, 59,904 unknowns), 96 cells, 32 monostatic
incidences, CBFs from the 144 Table-I plane waves, delta_SVD 1e-3, regular
pairs filled in FP32 (near pairs, CBF build, projection and solve in FP64),
block GMRES: the 32 incidences share one Krylov space (--block 0: one space
per incidence, in s-step cycles of blocks of 8 iterations, --sstep 0 plain
cycles; the other workloads default to one space per incidence).
The FP64 form of the same step runs beside it, the same step with one
Krylov space per incidence, then the precision forms, the IPCBF leg (the
paper's cylinder conditions), the batching and serving legs and the CPU
oracle baseline (see --help for the switches).

value = logical triangle pair-evaluations (N_tri^2 per step) per second of
the whole step.  After the timed steps one more step runs with the library's
event timers on, the projection and the solve timed separately; the roofline
entry is for the kernel family with the most GPU time in that step
(algorithmic work per launch over the average launch duration) and
roofline_kernels lists every timed family.  HBM traffic per launch comes
from the committed counter summary when the kernel's source is unchanged
since it was measured, else it is null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PMCHWT fill+projection pair-evals/s; solves/s with p50/p99 latency"

# Algorithmic flops of one regular triangle pair in the fill kernel, the
# same count in FP64 and FP32 (FMA = 2 flops; square roots, reciprocals,
# sines/cosines and exponentials not counted):
#   49 point pairs x 73 (distance 12, Green's functions of both media 24,
#   inner accumulations 40 -- less 3 for the folded weight products)
#   + 7 outer points x 190 (T moments 84, K moments 106)
#   + 9 local pairs x 110 (K 38, two media X_i 36, two output operators 36)
FLOP_PER_PAIR = 49 * 73 + 7 * 190 + 9 * 110
PEAK_FP64_VALU = 78.6e12
PEAK_FP32_VALU = 157.3e12       # published vector FP32 (packed FP32 issue)
PEAK_FP32_VALU_UNPACKED = 78.6e12  # one FP32 FMA per lane per clock (packed forms not used here)
PEAK_FP64_MFMA = 78.6e12
PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12

WORKLOADS = ["cylinder19968", "cube1728", "sphere320", "sphere5120", "sphere_array4x4x2", "sphere_array8x16x2",
             "cube_array8x2x2"]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")


# timer family -> (kernel, bound, peak, unit, scale of the timer's work unit)
FAMILIES = {
    "fill_regular": ("fill_regular_kernel<double>", "alu", PEAK_FP64_VALU, "TFLOP/s", FLOP_PER_PAIR),
    "fill_regular_f32": ("fill_regular_kernel<float>", "alu", PEAK_FP32_VALU, "TFLOP/s", FLOP_PER_PAIR),
    "gemm": ("zgemm_batched_kernel", "mfma", PEAK_FP64_MFMA, "TFLOP/s", 1.0),
    "xgemm": ("xgemm_batched_kernel", "mfma", PEAK_FP32_MFMA, "TFLOP/s", 1.0),
    # the "gemm" launches that ran on the row-block kernel (names the kernel
    # of the "gemm" row; not a row of its own)
    "gemm_panel": ("zgemm_panel_kernel", "mfma", PEAK_FP64_MFMA, "TFLOP/s", 1.0),
    "gmres_dots": ("dots2_kernel", "hbm", PEAK_HBM, "GB/s", 1.0),
    "gmres_update": ("dcgs_update_kernel", "hbm", PEAK_HBM, "GB/s", 1.0),
}
# timer family -> (substring of the kernel symbol, source file), for the
# counter summaries
FAMILY_SOURCES = {
    "fill_regular": ("fill_regular_kernel<double", "paper_2111_11058_amd/csrc/fill.hip"),
    "fill_regular_f32": ("fill_regular_kernel<float", "paper_2111_11058_amd/csrc/fill.hip"),
    "gemm": ("zgemm_batched_kernel", "paper_2111_11058_amd/csrc/gemm.hip"),
    "gmres_dots": ("dots2_kernel", "paper_2111_11058_amd/csrc/solve.hip"),
    "gmres_update": ("dcgs_update_kernel", "paper_2111_11058_amd/csrc/solve.hip"),
    # s-step cycles (blocks of 8): the block Gram-Schmidt passes
    # (the dot pass runs on the row-block GEMM kernel with 16-column tiles)
    "gmres_block_dots": ("zgemm_panel_kernel<1>", "paper_2111_11058_amd/csrc/gemm.hip"),
    "gmres_block_update": ("block_update_kernel<8>", "paper_2111_11058_amd/csrc/solve.hip"),
    # the GMRES matrix-vector product: the row-block kernel's launch shape
    # with the most dispatches
    "gmres_matvec": ("zgemm_panel_kernel<2>", "paper_2111_11058_amd/csrc/gemm.hip"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from synth import configs
    if name == "cube1728":
        return configs.cube_c2()
    if name == "sphere320":
        return configs.sphere_c1()
    if name == "sphere5120":
        return configs.sphere_c3()
    if name == "cylinder19968":
        return configs.cylinder_c5()
    if name == "sphere_array4x4x2":
        return configs.sphere_array()
    if name == "sphere_array8x16x2":
        return configs.sphere_array(8, 16, 2)
    if name == "cube_array8x2x2":
        return configs.cube_array(6)
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload_name):
    """Per-kernel HBM bytes per launch from the committed counter summary,
    kept only where the kernel's source file still has the hash recorded
    with the measurement."""
    out = {}
    path = traffic_file(workload_name)
    if not os.path.exists(path):
        return out
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        src = os.path.join(ROOT, f["source"])
        if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == f["sha256"]:
            out[f["kernel"]] = float(f["bytes_per_dispatch"])
    return out


def write_traffic(workload_name, fetch_dir, write_dir, cfetch_dir, cwrite_dir, cmd):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of this
    benchmark, then of the 1 GiB copy) into the traffic summary: per kernel
    family the mean KiB per dispatch, scaled so that the copy reads and
    writes exactly 1 GiB, with the hash of the kernel's source."""
    import csv
    from collections import defaultdict

    def per_dispatch(d, sub, most_frequent_grid=False):
        acc, grid = defaultdict(float), {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if sub in r["Kernel_Name"]:
                acc[r["Dispatch_Id"]] += float(r["Counter_Value"])
                grid[r["Dispatch_Id"]] = (r["Kernel_Name"], r.get("Grid_Size", ""))
        if most_frequent_grid and grid:
            counts = defaultdict(int)
            for g in grid.values():
                counts[g] += 1
            top = max(counts, key=counts.get)
            return [v for k, v in acc.items() if grid[k] == top]
        return list(acc.values())

    gib_kib = float(1 << 20)
    fs = gib_kib / np.mean(per_dispatch(cfetch_dir, "__amd_rocclr_copyBuffer"))
    ws = gib_kib / np.mean(per_dispatch(cwrite_dir, "__amd_rocclr_copyBuffer"))
    lines = [f"# HBM traffic per dispatch, {workload_name} bench step, from rocprofv3 --pmc",
             f"# command: {cmd}",
             f"# calibration: a 1 GiB device copy reads {1 / fs:.4f} GiB by FETCH_SIZE and writes "
             f"{1 / ws:.4f} GiB by WRITE_SIZE; scales fetch x{fs:.4f}, write x{ws:.4f}"]
    for fam, (sub, src) in FAMILY_SOURCES.items():
        top = fam == "gmres_matvec"
        f, w = per_dispatch(fetch_dir, sub, top), per_dispatch(write_dir, sub, top)
        if not f or not w:
            continue
        sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        fk, wk = float(np.mean(f)), float(np.mean(w))
        b = (fk * fs + wk * ws) * 1024.0
        lines.append(f"kernel={fam} symbol={sub.split('<')[0]} source={src} sha256={sha} dispatches={len(f)} "
                     f"fetch_kib={fk:.1f} write_kib={wk:.1f} bytes_per_dispatch={b:.0f}")
    with open(traffic_file(workload_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# counter passes (one rocprofv3 --pmc run each; at most 8 SQ and 2 GRBM)
COUNTER_PASSES = {
    "valu_a": ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64",
               "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_TRANS_F32"],
    "valu_b": ["SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64",
               "SQ_INSTS_VALU_CVT", "SQ_INSTS_SALU", "SQ_WAVES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"],
    "mfma": ["SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_XF32",
             "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_VALU_MFMA_F64", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"],
}
COUNTER_KERNELS = {  # label -> (symbol substring, source)
    "fill_regular_fp64": ("fill_regular_kernel<double, false>", "paper_2111_11058_amd/csrc/fill.hip"),
    "fill_regular_f32": ("fill_regular_kernel<float, false>", "paper_2111_11058_amd/csrc/fill.hip"),
    "zgemm": ("zgemm_batched_kernel", "paper_2111_11058_amd/csrc/gemm.hip"),
    "zgemm_panel": ("zgemm_panel_kernel", "paper_2111_11058_amd/csrc/gemm.hip"),
    "xgemm": ("xgemm_batched_kernel", "paper_2111_11058_amd/csrc/gemm.hip"),
}
N_SIMD = 256 * 4
N_XCD = 8


def write_counters(workload_name, stats_dir, dirs, cmd):
    """Per-dispatch VALU and MFMA counters of the fill and GEMM kernels from
    the rocprofv3 --pmc passes in COUNTER_PASSES (folders ``dirs``, in that
    order) and the kernel durations of a --kernel-trace --stats run of the
    same command (``stats_dir``): issued FP64/FP32 VALU flops per dispatch
    (64 lanes x (2 FMA + ADD + MUL) instructions; full wavefronts),
    VALU-issue and MFMA-busy fractions, written to
    profiles/valu_mfma_counters_<workload>.txt."""
    import csv
    from collections import defaultdict

    def groups(d):
        """(kernel label, grid size) -> {counter: [per-dispatch values]}"""
        per = defaultdict(lambda: defaultdict(float))
        key = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            for lab, (sub, _) in COUNTER_KERNELS.items():
                if sub in r["Kernel_Name"]:
                    did = r["Dispatch_Id"]
                    key[did] = (lab, int(r["Grid_Size"]))
                    per[did][r["Counter_Name"]] += float(r["Counter_Value"])
        out = defaultdict(lambda: defaultdict(list))
        for did, vals in per.items():
            for c, v in vals.items():
                out[key[did]][c].append(v)
        return out

    def durations(d):
        """(kernel label, grid size) -> mean duration in ns (kernel trace)"""
        acc = defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, "run_kernel_trace.csv"))):
            for lab, (sub, _) in COUNTER_KERNELS.items():
                if sub in r["Kernel_Name"]:
                    g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                    acc[(lab, g)].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
        return {k: float(np.mean(v)) for k, v in acc.items()}

    merged = defaultdict(dict)
    for d in dirs:
        for k, cs in groups(d).items():
            for c, v in cs.items():
                merged[k][c] = float(np.mean(v))
                merged[k]["dispatches"] = len(v)
    dur = durations(stats_dir)
    lines = [f"# VALU and MFMA counters per dispatch, {workload_name} bench step, from rocprofv3 --pmc",
             f"# command: {cmd}",
             "# passes: " + "; ".join(f"{p}: {' '.join(c)}" for p, c in COUNTER_PASSES.items()),
             "# issued_fp64_tflops = 64 (2 FMA_F64 + ADD_F64 + MUL_F64) / duration (likewise FP32);"
             " valu_issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs);"
             " mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs);"
             " mfma_f64_tflops = 512 MOPS_F64 / duration; clock_ghz = GRBM_GUI_ACTIVE / 8 / duration;"
             " durations from the kernel trace of the same command; sums over the dispatches of each role"]
    for src in sorted({src for _, src in COUNTER_KERNELS.values()}):
        lines.append(f"# source {src} sha256={hashlib.sha256(open(os.path.join(ROOT, src), 'rb').read()).hexdigest()}")
    # launch shapes grouped by role, counters and durations summed over the
    # dispatches of the role: each fill kernel over its panels; the GEMMs
    # as the GMRES matvec (many dispatches of one shape), the projection
    # (launches of 1 ms or more) and the rest
    roles = defaultdict(lambda: defaultdict(float))
    for (lab, grid), c in sorted(merged.items()):
        ns, nd = dur.get((lab, grid), 0.0), c.get("dispatches", 0)
        if lab.startswith("fill"):
            role = lab
        elif nd >= 100:
            # many dispatches of one shape: the GMRES matrix-vector product
            # (row-block kernel); with block GMRES the tiled kernel's are the
            # block Gram-Schmidt update passes (one shape for every basis size)
            role = f"{lab}_gmres_matvec" if lab == "zgemm_panel" else f"{lab}_gmres_repeated"
        elif ns >= 1e6:
            role = f"{lab}_projection"
        else:
            role = f"{lab}_other"
        acc = roles[role]
        acc["dispatches"] += nd
        acc["shapes"] += 1
        acc["ns"] += ns * nd
        for key, v in c.items():
            if key != "dispatches":
                acc[key] += v * nd
    for role, c in sorted(roles.items()):
        nd, ns = c["dispatches"], c["ns"]
        f64 = 64.0 * (2 * c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"])
        f32 = 64.0 * (2 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"])
        parts = [f"kernel={role} dispatches={int(nd)} shapes={int(c['shapes'])}"]
        if ns:
            parts.append(f"duration_us_per_dispatch={ns / nd / 1e3:.1f}")
        if f64 or f32:
            parts.append(f"fp64_valu_flop_per_dispatch={f64 / nd:.4g} fp32_valu_flop_per_dispatch={f32 / nd:.4g}")
            if ns:
                parts.append(f"issued_fp64_tflops={f64 / ns / 1e3:.2f} issued_fp32_tflops={f32 / ns / 1e3:.2f}")
            parts.append(f"trans_f64_per_dispatch={c['SQ_INSTS_VALU_TRANS_F64'] / nd:.4g} "
                         f"trans_f32_per_dispatch={c['SQ_INSTS_VALU_TRANS_F32'] / nd:.4g}")
        gui = c["GRBM_GUI_ACTIVE"] / N_XCD  # the counter is summed over the XCDs; each runs for the whole dispatch
        if c["SQ_INSTS_VALU"] and gui:
            parts.append(f"valu_issue={4 * c['SQ_INSTS_VALU'] / (N_SIMD * gui):.3f} "
                         f"cvt_share={c['SQ_INSTS_VALU_CVT'] / c['SQ_INSTS_VALU']:.3f} "
                         f"clock_ghz={gui / ns if ns else 0:.2f}")
        if c["SQ_VALU_MFMA_BUSY_CYCLES"] and gui:
            m64 = 512.0 * c["SQ_INSTS_VALU_MFMA_MOPS_F64"]
            parts.append(f"mfma_busy={c['SQ_VALU_MFMA_BUSY_CYCLES'] / (N_SIMD * gui):.3f} "
                         f"mfma_f64_flop_per_dispatch={m64 / nd:.4g}")
            if ns:
                parts.append(f"mfma_f64_tflops={m64 / ns / 1e3:.2f}")
        lines.append(" ".join(parts))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"valu_mfma_counters_{workload_name}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# kernels and traffic entries of the solve's families under s-step cycles
SSTEP_KERNELS = {"gmres_dots": ("zgemm_panel_kernel<1>", "gmres_block_dots"),
                 "gmres_update": ("block_update_kernel", "gmres_block_update")}


def read_families(cbfm, traffic, phase, sstep=0, block=0):
    """Achieved rate of every timed family since the last timer_enable."""
    rows = {}
    for fam, (kernel, bound, peak, unit, scale) in FAMILIES.items():
        n, ms, work = cbfm.timer_read(fam, with_work=True)
        if n == 0 or ms <= 0:
            continue
        tkey = fam
        if phase == "solve" and fam == "gemm":
            tkey = "gmres_matvec"
        if sstep and fam in SSTEP_KERNELS:
            kernel, tkey = SSTEP_KERNELS[fam]
        per_launch = work * scale / n
        avg_s = ms * 1e-3 / n
        ach = per_launch / avg_s
        div = 1e12 if unit == "TFLOP/s" else 1e9
        row = {"bound": bound, "achieved": ach / div, "peak": peak / div, "unit": unit, "frac": ach / peak,
               "traffic": traffic.get(tkey), "kernel": kernel, "phase": phase, "launches": n,
               "avg_launch_ms": ms / n, "total_ms": ms, "work_per_launch": per_launch}
        if fam == "fill_regular_f32":
            row["frac_of_unpacked_fp32"] = ach / PEAK_FP32_VALU_UNPACKED
        rows[fam] = row
    panel = rows.pop("gemm_panel", None)
    if block and phase == "solve":
        # block GMRES: the matrix-vector products run on the row-block kernel
        # (its timer family); "gemm" also holds the block Gram-Schmidt updates,
        # the operator's formation and the residuals
        if "gemm" in rows:
            rows["gemm_all"] = dict(rows.pop("gemm"), kernel="zgemm_batched_kernel and zgemm_panel_kernel",
                                    traffic=None)
        if panel:
            rows["gemm"] = dict(panel, kernel="zgemm_panel_kernel<2>", traffic=traffic.get("gmres_matvec"))
        if "gmres_dots" in rows:
            rows["gmres_dots"].update(kernel="zgemm_panel_kernel<2> (block Gram-Schmidt dot pass)", traffic=None)
        if "gmres_update" in rows:
            rows["gmres_update"].update(kernel="zgemm_batched_kernel (block Gram-Schmidt update pass)",
                                        traffic=None)
        return rows
    if panel and "gemm" in rows:
        g = rows["gemm"]
        g["kernel"] = ("zgemm_panel_kernel" if panel["launches"] == g["launches"] else
                       f"zgemm_batched_kernel and zgemm_panel_kernel ({panel['launches']} of {g['launches']} launches)")
    return rows


def rooflines(cbfm, run_phases, traffic, prefix="", sstep=0, block=0):
    """One step with the timers on, the projection and the solve timed
    apart (run_phases calls project() and solve() in turn, each given a
    callback that switches the timers on for that phase)."""
    rows = {}
    names = {"project": {"fill_regular": "fill_regular_fp64", "fill_regular_f32": "fill_regular_f32",
                         "gemm": "projection_gemm_fp64", "xgemm": "projection_gemm_xf32"},
             "solve": {"gemm": "gmres_matvec_gemm", "xgemm": "gmres_matvec_xgemm", "gmres_dots": "gmres_dots",
                       "gmres_update": "gmres_update", "gemm_all": "solve_gemm_all"}}

    def timed(phase):
        cbfm.timer_enable(list(cbfm.TIMERS))

        def done():
            for fam, row in read_families(cbfm, traffic, phase, sstep, block).items():
                if fam in names[phase]:
                    rows[prefix + names[phase][fam]] = row
            cbfm.timer_enable(None)
        return done

    run_phases(timed)
    dom = max((k for k in rows if k != prefix + "solve_gemm_all"), key=lambda k: rows[k]["total_ms"])
    return dict(rows[dom], family=dom), rows


def serve(cbfm, n_requests, slots, budget, seed=2113, rate=200.0, tol=1e-6):
    """Replay the seeded mixed-size request stream (Poisson arrivals at
    `rate`/s) into a request server; latency = finish - submission on the
    server's clock."""
    from synth import configs
    stream = configs.serving_stream(n_requests, seed=seed, rate=rate)
    reqs = []
    for r in stream:
        w = r.work
        med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
        reqs.append(cbfm.make_request(w.V, w.T, w.edge_block, w.nblocks, med, w.gen, w.delta_svd, w.inc, tol=tol))
    srv = cbfm.Server(slots=slots, budget_bytes=budget)
    try:
        tickets = []
        t0 = time.perf_counter()
        for r, (req, _) in zip(stream, reqs):
            lag = r.t_arrival - (time.perf_counter() - t0)
            if lag > 0:
                time.sleep(lag)
            tickets.append(srv.submit(req))
        outs = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    lat = np.array([o["t_end"] - o["t_submit"] for o in outs])
    queue = np.array([o["t_start"] - o["t_submit"] for o in outs])
    nsolve = int(sum(len(o["rcs"]) for o in outs))
    ok = sum(o["status"] == "OK" for o in outs)
    status = {}
    for o in outs:
        status[o["status"]] = status.get(o["status"], 0) + 1
    its = np.concatenate([o["iters"] for o in outs])
    return {"requests": n_requests, "slots": slots, "budget_bytes": int(budget), "arrival_rate_per_s": rate,
            "wall_s": wall, "requests_per_s": n_requests / wall, "solves_per_s": nsolve / wall,
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                           "mean": float(lat.mean() * 1e3)},
            "queue_wait_ms": {"p50": float(np.percentile(queue, 50) * 1e3), "p99": float(np.percentile(queue, 99) * 1e3)},
            "status_ok": int(ok), "status": status, "gmres_iterations": {"mean": float(its.mean()), "max": int(its.max())},
            "max_running": st["max_running"], "peak_admitted_bytes": st["peak_bytes"],
            "peak_within_budget": bool(st["peak_bytes"] <= budget),
            "unknowns": {"min": int(min(r.unknowns for r in stream)), "max": int(max(r.unknowns for r in stream))}}


def batching_leg(cbfm, torch, n=16, reps=3):
    """The batching form on the mixed serving stream (its first n seeded
    scatterers, 960 to 8,000 unknowns, each with its own medium and 1-16
    incidences): (1) every scatterer projected one by one (cbfm_project)
    against all of them in one call (cbfm_project_batch: one persistent
    fill launch, batched GEMMs), FP64, CBFs built beforehand; (2) the
    reduced solves eager against HIP-graph-replayed Arnoldi chunks.  Best
    of `reps` after one warm-up."""
    from synth import configs
    stream = configs.serving_stream(n)
    items = []
    for r in stream:
        w = r.work
        mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
        med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
        cb = cbfm.build_cbf(mesh, med, w.gen, w.delta_svd)
        Zr = torch.empty((cb.n_cbf, cb.n_cbf), dtype=torch.complex128, device="cuda")
        items.append((mesh, med, cb, Zr, w))
    pairs = float(sum(it[4].nt ** 2 for it in items))

    def one_by_one():
        for mesh, med, cb, Zr, _ in items:
            cbfm.project(mesh, med, cb, Zr, cbfm.FP64)

    def batched():
        cbfm.project_batch([it[:4] for it in items], cbfm.FP64)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best

    t_one = timed(one_by_one)
    ref = [it[3].clone() for it in items]
    t_batch = timed(batched)
    dz = max(float((it[3] - r).abs().max() / r.abs().max()) for it, r in zip(items, ref))

    def solves(graph):
        out = []
        for mesh, med, cb, Zr, w in items:
            out.append(cbfm.solve(mesh, med, cb, Zr, w.inc, tol=1e-6, max_iter=3000,
                                  restart=full_restart(cb.n_cbf, len(w.inc)), use_graph=graph))
        return out

    res = {}
    for graph in (False, True):
        solves(graph)
        torch.cuda.synchronize()
        best, outs = 1e30, None
        for _ in range(reps):
            t = time.perf_counter()
            outs = solves(graph)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        res[graph] = (best, outs)
    nsolve = sum(len(it[4].inc) for it in items)
    drcs = max(float(np.max(np.abs(a["rcs"] - b["rcs"]) / np.abs(b["rcs"])))
               for a, b in zip(res[True][1], res[False][1]))
    return {"scatterers": n, "unknowns": {"min": int(min(3 * it[4].nt for it in items)),
                                         "max": int(max(3 * it[4].nt for it in items))},
            "incidences": nsolve,
            "projection_one_by_one_ms": t_one * 1e3, "projection_batched_ms": t_batch * 1e3,
            "projection_batched_pair_evals_per_s": pairs / t_batch,
            "projection_one_by_one_pair_evals_per_s": pairs / t_one,
            "batched_vs_one_by_one_max_rel_diff": dz,
            "solve_eager_ms": res[False][0] * 1e3, "solve_graph_ms": res[True][0] * 1e3,
            "solves_per_s_eager": nsolve / res[False][0], "solves_per_s_graph": nsolve / res[True][0],
            "graph_vs_eager_rcs_max_rel_diff": drcs}


def serving_legs(cbfm, torch, n, slots):
    """The serving leg under a generous budget (half the free device memory)
    and a tight one (twice the largest request's estimated footprint)."""
    from synth import configs
    free, _ = torch.cuda.mem_get_info()
    big = 0
    for r in configs.serving_stream(n):
        w = r.work
        med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
        req, keep = cbfm.make_request(w.V, w.T, w.edge_block, w.nblocks, med, w.gen, w.delta_svd, w.inc)
        big = max(big, cbfm.request_footprint(req))
    legs = {}
    for name, budget in (("generous", free // 2), ("tight", min(free // 2, 2 * big))):
        log(f"serving {name}: {n} requests, budget {budget / 2**30:.1f} GiB")
        legs[name] = serve(cbfm, n, slots, budget)
        log(f"serving {name}: {legs[name]}")
    return legs


# ----------------------------------------------------------------- CPU oracle
def _oracle_fill_chunk(args):
    """Oracle FP64 fill of a list of (P, Q) pairs (worker of the pool)."""
    name, P, Q, near = args
    from oracle import fill, mesh as om
    w = workload(name)
    m = om.build(w.V, w.T)
    k, _ = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    t0 = time.perf_counter()
    for s in range(0, len(P), 4096):
        fill.regular_local(m, k, P[s:s + 4096], Q[s:s + 4096])
    for p, q in near:
        fill.near_local(m, k, int(p), int(q))
    return time.perf_counter() - t0


def cpu_baseline(name, sample, cores, seed=5):
    """The oracle timed on the host cores: its FP64 fill on bounded seeded
    samples of the workload's triangle pairs (regular and near pairs in the
    workload's proportion), on one core and on `cores` worker processes,
    and its end-to-end CBFM path (fill, CBF build, projection, G^CBF,
    LU solve, RCS) on the 320-triangle sphere.  Never touches the GPU."""
    import multiprocessing as mp
    from oracle import fill, mesh as om
    w = workload(name)
    m = om.build(w.V, w.T)
    log("cpu baseline: near pairs")
    near = om.near_pairs(m)
    frac = len(near) / m.nt ** 2
    rng = np.random.default_rng(seed)

    def draw(n):
        n_near = max(1, int(round(n * frac)))
        n_reg = n - n_near
        isn = set(map(tuple, near.tolist()))
        P = rng.integers(0, m.nt, n_reg * 2)
        Q = rng.integers(0, m.nt, n_reg * 2)
        keep = np.array([(p, q) not in isn for p, q in zip(P.tolist(), Q.tolist())])
        return P[keep][:n_reg], Q[keep][:n_reg], near[rng.choice(len(near), n_near, replace=False)]

    P, Q, nr = draw(sample)
    log(f"cpu baseline: one core, {sample} pairs")
    t1 = _oracle_fill_chunk((name, P, Q, nr))
    one = {"value": sample / t1, "unit": "pair-evals/s", "cores": 1, "seconds": t1, "pairs": sample}
    # all cores: `cores` workers, each a sample of the same size
    chunks = [draw(sample) for _ in range(cores)]
    log(f"cpu baseline: {cores} workers x {sample} pairs")
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_fill_chunk, [(name, a, b, c) for a, b, c in chunks])
    tall = time.perf_counter() - t0
    allc = {"value": cores * sample / tall, "unit": "pair-evals/s", "cores": cores, "seconds": tall,
            "pairs": cores * sample}
    # end to end on the 320-triangle sphere (the oracle's whole CBFM path)
    from oracle import cbf, excitation, reduced
    ws = workload("sphere320")
    log("cpu baseline: oracle end to end, sphere320")
    t0 = time.perf_counter()
    ms = om.build(ws.V, ws.T)
    k, eta = fill.media(ws.k0, ws.eta0, ws.eps_r, ws.mu_r)
    Kc, TE, TH = fill.combine(*fill.fill_ops(ms, k), eta)
    cb = cbf.build(ms, Kc, TE, TH, ws.edge_block, ws.gen, ws.k0, ws.eta0, ws.delta_svd)
    CJM, CMJ = reduced.cbf_matrices(cb, ms.ne)
    Zr = reduced.project(fill.assemble_Z(Kc, TE, TH), CJM, CMJ)
    Gc = reduced.gram_cbf(cbf.rwg_gram(ms), CJM, CMJ)
    vr = CJM.conj().T @ excitation.rhs(ms, ws.inc, ws.k0, ws.eta0)
    jc = np.linalg.solve(Gc, np.linalg.solve(Zr @ np.linalg.inv(Gc), vr))
    excitation.monostatic_rcs(ms, CMJ @ jc, ws.inc, ws.k0, ws.eta0)
    te = time.perf_counter() - t0
    e2e = {"workload": "sphere320 (320 triangles, 960 unknowns, 8 cells, 1 incidence, 144 generating waves)",
           "seconds": te, "solves_per_s": len(ws.inc) / te, "pair_evals_per_s": ms.nt ** 2 / te}
    return {"value": allc["value"], "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle FP64 fill of seeded samples of the {name} triangle pairs (regular and near pairs "
                      f"in the workload's proportion): {cores} worker processes x {sample} pairs in {tall:.1f} s; "
                      f"one core: {sample} pairs in {t1:.1f} s; the end-to-end oracle CBFM path on sphere320 in "
                      f"{te:.1f} s (single process)",
            "one_core": one, "all_cores": allc, "end_to_end": e2e,
            "host": {"cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}}


def rmse_db(sig_c, sig_m):
    """RMSE of the CBFM RCS against the MoM RCS over the observation angles
    (linear sigma; 10 log10 of the rms difference over the MoM range)."""
    sig_c, sig_m = np.asarray(sig_c, float), np.asarray(sig_m, float)
    return float(10.0 * np.log10(np.sqrt(np.mean((sig_c - sig_m) ** 2)) / (sig_m.max() - sig_m.min())))


def full_restart(n, nrhs, budget=48 << 30, cap=3000):
    """GMRES restart length: the longest cycle, up to min(n, 3000), whose
    solver memory fits the budget (48 GiB of the 288 GB): the Krylov basis
    (m + 1) nrhs n and the Hessenberg and triangular factors
    2 nrhs (m + 1) m complex doubles.  On the cylinder (n = 4,224, 32 RHS)
    the unrestarted solve needs 1,263 iterations where cycles of 1,000 need
    1,975 (811 against 1,047 ms)."""
    m = min(n, cap)
    while m > 100 and ((m + 1) * nrhs * n + 2 * nrhs * (m + 1) * m) * 16 > budget:
        m = int(m * 0.9)
    return int(m)


def plane_incidences(theta_deg):
    """Monostatic theta-polarised incidences from the directions theta
    (degrees), phi = 0: arrival direction r(theta, 0), k = -r, p = theta-hat."""
    from synth import configs
    th = np.deg2rad(np.asarray(theta_deg, float))
    r, t, _ = configs.sph_dir(th, np.zeros_like(th))
    return np.concatenate([-r, t], axis=1)


def ipcbf_leg(cbfm, torch, w, mesh, med, prec, primary_rcs, primary_its, primary_ms, solver, delta_r=1e-2,
              gen=None):
    """IPCBF (the GMRES version of Sec. III-A) on the bench workload, with the
    paper's cylinder conditions: s = 10 theta-polarised generating waves in
    the phi = 0 plane (theta_s = 0, 5 degree steps), delta_svd 1e-3; then
    the same projection and CMP solve of the bench incidences (all in that
    plane).  Step time = FP32 operator fill + IPCBF GMRES + orthogonalisation
    + projection + solve.  RCS against an FP64 MoM solve (the stored FP64
    operator, GMRES to 1e-6) as RMSE (Sec. IV-A) beside the primary CBFs'."""
    gen = plane_incidences(np.arange(10) * 5.0) if gen is None else gen
    cbfm.MomOperator(mesh, med, cbfm.FP32).close()  # warm-up (first allocations), untimed as the bench's warm-up steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = cbfm.MomOperator(mesh, med, cbfm.FP32)
    t1 = time.perf_counter()
    cb, its, res = cbfm.build_ipcbf(op, gen, delta_r=delta_r, delta_svd=1e-3, max_iter=1000)
    t2 = time.perf_counter()
    op.close()
    n = cb.n_cbf
    Zr = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    cbfm.project(mesh, med, cb, Zr, prec)
    torch.cuda.current_stream().synchronize()
    t3 = time.perf_counter()
    out = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=3000, restart=full_restart(n, len(w.inc)),
                     **solver)
    t4 = time.perf_counter()
    leg = {"generating_waves": len(gen), "delta_r": delta_r, "delta_svd": 1e-3, "n_cbf": int(n),
           "ipcbf_gmres_iterations": [int(i) for i in its], "ipcbf_residual_max": float(res.max()),
           "gmres_iterations": {"mean": float(out["iters"].mean()), "max": int(out["iters"].max())},
           "status": out["status"], "ms": {"operator_fill_fp32": (t1 - t0) * 1e3, "ipcbf_gmres_and_svd": (t2 - t1) * 1e3,
                                           "projection": (t3 - t2) * 1e3, "solve": (t4 - t3) * 1e3,
                                           "step": (t4 - t0) * 1e3},
           "primary_cbfs": {"gmres_iterations_max": int(primary_its), "ms_per_step": primary_ms}}
    del Zr
    # MoM reference (FP64 operator; block GMRES: the incidences share one
    # Krylov space, so the count is of block iterations)
    t5 = time.perf_counter()
    op64 = cbfm.MomOperator(mesh, med, cbfm.FP64)
    mom = cbfm.mom_solve(op64, w.inc, tol=1e-6, max_iter=3000, restart=1000, block=True)
    t6 = time.perf_counter()
    op64.close()
    leg["mom_fp64"] = {"gmres": "block", "gmres_iterations_max": int(mom["iters"].max()), "status": mom["status"],
                       "ms": (t6 - t5) * 1e3}
    leg["rmse_db_vs_mom"] = {"ipcbf": rmse_db(out["rcs"], mom["rcs"]), "primary": rmse_db(primary_rcs, mom["rcs"])}
    # the same step with the IPCBF waves in block GMRES (one Krylov space for
    # the ten waves; its iterates meet the same allowance delta_r)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    op = cbfm.MomOperator(mesh, med, cbfm.FP32)
    b1 = time.perf_counter()
    cb, bits, bres = cbfm.build_ipcbf(op, gen, delta_r=delta_r, delta_svd=1e-3, max_iter=1000, block=True)
    b2 = time.perf_counter()
    op.close()
    nb = cb.n_cbf
    Zr = torch.empty((nb, nb), dtype=torch.complex128, device="cuda")
    cbfm.project(mesh, med, cb, Zr, prec)
    torch.cuda.current_stream().synchronize()
    b3 = time.perf_counter()
    outb = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=3000, restart=full_restart(nb, len(w.inc)),
                      **solver)
    b4 = time.perf_counter()
    del Zr
    leg["ipcbf_block_gmres"] = {
        "n_cbf": int(nb), "block_iterations": int(bits.max()), "ipcbf_residual_max": float(bres.max()),
        "status": outb["status"], "rmse_db_vs_mom": rmse_db(outb["rcs"], mom["rcs"]),
        "ms": {"operator_fill_fp32": (b1 - b0) * 1e3, "ipcbf_gmres_and_svd": (b2 - b1) * 1e3,
               "projection": (b3 - b2) * 1e3, "solve": (b4 - b3) * 1e3, "step": (b4 - b0) * 1e3}}
    return leg


# the paper's IPCBF conditions for the cylinder (Table III): (delta_r, delta_SVD)
IPCBF_CONDITIONS = ((1e-3, 1e-3), (1e-2, 1e-3), (1e-1, 1e-3), (1e-3, 1e-7))


def ipcbf_conditions_leg(cbfm, torch, w, med, cells=(96, 32)):
    """The paper's four IPCBF conditions on the cylinder (Sec. IV-C): for
    each cell division (the bench's 96 cells and 32, the paper's count),
    the IPCBFs of the 10 in-plane waves, the projection (FP32 fill) and the
    CMP solve of the bench incidences to 1e-6; N_CBF, mean and max
    iterations, and the RMSE of the RCS against the FP64 MoM solve."""
    from synth.blocks import rcb_blocks
    gen = plane_incidences(np.arange(10) * 5.0)
    base = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    op64 = cbfm.MomOperator(base, med, cbfm.FP64)
    t0 = time.perf_counter()
    mom = cbfm.mom_solve(op64, w.inc, tol=1e-6, max_iter=3000, restart=1500, block=True)
    t_mom = time.perf_counter() - t0
    op64.close()
    out = {"mom_fp64": {"gmres": "block", "iterations_max": int(mom["iters"].max()), "status": mom["status"],
                        "ms": t_mom * 1e3},
           "incidences": len(w.inc), "cells": {}}
    for nc in cells:
        eb = w.edge_block if nc == w.nblocks else rcb_blocks(w.V, w.T, nc)
        mesh = cbfm.Mesh(w.V, w.T, eb, nc)
        op = cbfm.MomOperator(mesh, med, cbfm.FP32)
        rows = []
        for dr, ds in IPCBF_CONDITIONS:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cb, its, res = cbfm.build_ipcbf(op, gen, delta_r=dr, delta_svd=ds, max_iter=1000)
            t1 = time.perf_counter()
            n = cb.n_cbf
            Zr = torch.empty((n, n), dtype=torch.complex128, device="cuda")
            cbfm.project(mesh, med, cb, Zr, cbfm.FP32)
            torch.cuda.current_stream().synchronize()
            t2 = time.perf_counter()
            o = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, tol=1e-6, max_iter=3000,
                           restart=full_restart(n, len(w.inc)))
            t3 = time.perf_counter()
            rows.append({"delta_r": dr, "delta_svd": ds, "n_cbf": int(n), "generation_iterations_max": int(its.max()),
                         "iterations_mean": float(o["iters"].mean()), "iterations_max": int(o["iters"].max()),
                         "status": o["status"], "rmse_db": rmse_db(o["rcs"], mom["rcs"]),
                         "ms": {"generation": (t1 - t0) * 1e3, "projection": (t2 - t1) * 1e3,
                                "solve": (t3 - t2) * 1e3}})
            log(f"ipcbf cells {nc} {rows[-1]}")
            del Zr
        op.close()
        out["cells"][str(nc)] = rows
    return out


def mom_leg(cbfm, torch, w, mesh, med, cb, Zr, solver):
    """The paper's comparison on its arrays (Sec. IV-A, IV-B): iterations to
    1e-6 of the MoM (its arrangement with the diagonal preconditioner, on the
    stored FP64 operator), the K-diagonal CBFM without the CMP, the
    T-diagonal CBFM and the CBFM with the CMP, for the theta-polarised wave
    along -z; and the RMSE of the CBFM RCS against the MoM RCS over
    0 <= theta <= 30 degrees, 1 degree steps, phi = 0 (both to 1e-4)."""
    op = cbfm.MomOperator(mesh, med, cbfm.FP64)
    inc = w.inc
    n = cb.n_cbf
    t0 = time.perf_counter()
    mom = cbfm.mom_solve(op, inc, tol=1e-6, max_iter=1000, restart=1000)
    t1 = time.perf_counter()
    legs = {"mom": {"iterations": int(mom["iters"].max()), "status": mom["status"],
                    "relres": float(mom["relres"].max()), "ms": (t1 - t0) * 1e3}}
    for name, uc in (("cbfm_cmp", 1), ("cbfm_k_diagonal_no_cmp", 0), ("cbfm_t_diagonal", 2)):
        o = cbfm.solve(mesh, med, cb, Zr, inc, tol=1e-6, max_iter=1000, restart=1000, use_cmp=uc)
        legs[name] = {"iterations": int(o["iters"].max()), "status": o["status"], "relres": float(o["relres"].max())}
    incs = plane_incidences(np.arange(31) * 1.0)
    a = cbfm.mom_solve(op, incs, tol=1e-4, max_iter=2000, restart=1000)
    b = cbfm.solve(mesh, med, cb, Zr, incs, tol=1e-4, max_iter=2000, restart=full_restart(n, len(incs)), use_cmp=True)
    op.close()
    legs["rmse_db"] = rmse_db(b["rcs"], a["rcs"])
    legs["rcs_directions"] = "0..30 deg, 1 deg, phi 0, theta-hat, monostatic, both solves to 1e-4"
    return legs


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cylinder19968", choices=WORKLOADS)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="fill precision of the timed step (default: fp32 for cylinder19968, else fp64)")
    ap.add_argument("--sstep", type=int, default=None, choices=[0, 4, 8],
                    help="GMRES of the main step and the FP64 leg: s-step cycles of blocks of this many "
                         "iterations, or 0 for plain cycles (DCGS2); default 8 for cylinder19968 and cube1728 "
                         "(long solves of many incidences, where it measured faster), else 0")
    ap.add_argument("--block", type=int, default=None,
                    help="block GMRES (1: groups of up to 32 right-hand sides sharing one Krylov space; 0: off; "
                         "default 1 for cylinder19968, 0 otherwise)")
    ap.add_argument("--basis-fp32", action="store_true",
                    help="time the compressed-basis form (double arithmetic, Krylov basis stored in float) as the "
                         "main step")
    ap.add_argument("--cpu-sample", type=int, default=300000)
    ap.add_argument("--cpu-cores", type=int, default=0, help="oracle worker processes (0: the host's, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-fp32", action="store_true", help="skip the precision-form legs")
    ap.add_argument("--fp64-steps", type=int, default=0, help="steps of the FP64 leg (0: half of --steps, at least 1)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only measure what PyTorch's streaming sum and copy reach on this device")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for the HBM byte counters)")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the traffic summary from four rocprofv3 --pmc output folders (no GPU use)")
    ap.add_argument("--traffic-command", default="", help="command line recorded in the traffic summary")
    ap.add_argument("--write-counters", nargs=4, metavar=("STATS", "VALU_A", "VALU_B", "MFMA"),
                    help="write the VALU/MFMA counter summary from a --kernel-trace --stats folder and three "
                         "rocprofv3 --pmc folders (no GPU use)")
    ap.add_argument("--serve", type=int, default=32,
                    help="requests of the serving leg (mixed-size stream, Poisson arrivals); 0 skips it")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg (both budgets)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-per-rhs", action="store_true", help="skip the per-incidence leg beside the block step")
    ap.add_argument("--no-batching", action="store_true", help="skip the batching leg (mixed-stream projection batch, graphs)")
    ap.add_argument("--no-ipcbf", action="store_true", help="skip the IPCBF leg of the cylinder workload")
    ap.add_argument("--ipcbf", action="store_true",
                    help="other workloads: the IPCBF leg with the Table-I generating waves")
    ap.add_argument("--mom", action="store_true", help="array workloads: the MoM, K-/T-diagonal and RMSE leg")
    ap.add_argument("--ipcbf-conditions", action="store_true",
                    help="cylinder: the paper's four IPCBF conditions with 96 and 32 cells, RMSE against the MoM")
    args = ap.parse_args()
    cores = args.cpu_cores or min(16, len(os.sched_getaffinity(0)))
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.workload, args.cpu_sample, cores)), flush=True)
        return
    if args.write_traffic:
        write_traffic(args.workload, *args.write_traffic, args.traffic_command)
        return
    if args.write_counters:
        write_counters(args.workload, args.write_counters[0], args.write_counters[1:], args.traffic_command)
        return
    if args.hbm_probe:
        # what plain streaming code reaches on this device: PyTorch's sum over
        # 8 GiB (read) and a 2 GiB device copy (read + write), best of 5
        import torch
        x = torch.ones(1 << 30, dtype=torch.float64, device="cuda")
        y = torch.empty(1 << 28, dtype=torch.float64, device="cuda")

        def best(fn):
            fn()
            torch.cuda.synchronize()
            b = 1e30
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                b = min(b, e0.elapsed_time(e1) * 1e-3)
            return b
        print(json.dumps({"sum_read_GBps": x.numel() * 8 / best(lambda: x.sum()) / 1e9,
                          "copy_read_write_GBps": 2 * y.numel() * 8 / best(lambda: y.copy_(x[: 1 << 28])) / 1e9,
                          "peak_GBps": PEAK_HBM / 1e9}))
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2111_11058_amd import cbfm
    if not torch.cuda.is_available():
        raise SystemExit("no HIP device visible")
    if args.serve_only:
        print(json.dumps(serving_legs(cbfm, torch, args.serve or 512, args.serve_slots)), flush=True)
        return
    w = workload(args.workload)
    prec_name = args.precision or ("fp32" if args.workload == "cylinder19968" else "fp64")
    PREC = cbfm.FP32 if prec_name == "fp32" else cbfm.FP64
    log(f"bench: {w.name} nt={w.nt} cells={w.nblocks} nrhs={len(w.inc)} fill {prec_name}")
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    solver = dict(tol=1e-6)
    state = {}
    traffic = measured_traffic(args.workload)

    def step(precision, inner_fp32=False, timed=None, basis_fp32=False, sstep=0, block=False):
        cb = cbfm.build_cbf(mesh, med, w.gen, w.delta_svd, max_L=w.extra.get("max_L", 0))
        n = cb.n_cbf
        Zr = state.get(n)
        if Zr is None:
            Zr = state[n] = torch.empty((n, n), dtype=torch.complex128, device="cuda")
        done = timed("project") if timed else None
        t0 = time.perf_counter()
        cbfm.project(mesh, med, cb, Zr, precision)
        # (the caller's stream only: the CMP inverse that the CBF build left
        # on the library's side stream may still run beside the projection)
        torch.cuda.current_stream().synchronize()
        t1 = time.perf_counter()
        if done:
            done()
        m = full_restart(n, len(w.inc))
        done = timed("solve") if timed else None
        t2 = time.perf_counter()
        restarts = inner_fp32 or basis_fp32 or sstep > 0
        if block:
            # block iterations: a cycle holds the whole space the library allows
            out = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=3 * n, restart=n, block=True,
                             **solver)
        else:
            out = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=(3 if restarts else 1) * max(n, 3000),
                             restart=m, inner_fp32=inner_fp32, basis_fp32=basis_fp32, sstep=sstep, **solver)
        t3 = time.perf_counter()
        if done:
            done()
        return cb, out, t1 - t0, t3 - t2

    B32 = args.basis_fp32
    BLK = 0 if B32 else (args.block if args.block is not None else (1 if args.workload == "cylinder19968" else 0))
    sst_default = 8 if args.workload in ("cylinder19968", "cube1728") else 0
    # (the compressed basis and block GMRES: no s-step cycles)
    SST = 0 if B32 or BLK else (sst_default if args.sstep is None else args.sstep)
    for i in range(args.warmup):
        log(f"warmup {i}")
        step(PREC, basis_fp32=B32, sstep=SST, block=BLK)
    torch.cuda.synchronize()
    proj_t, solve_t, iters = [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        cb, out, tp, ts = step(PREC, basis_fp32=B32, sstep=SST, block=BLK)
        proj_t.append(tp)
        solve_t.append(ts)
        iters.append(out["iters"])
        log(f"step {i}: project {tp * 1e3:.1f} ms, solve {ts * 1e3:.1f} ms, N_CBF={cb.n_cbf}, "
            f"iters max {out['iters'].max()} status {out['status']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    nt = w.nt
    roof, roofs = rooflines(cbfm, lambda timed: step(PREC, timed=timed, basis_fp32=B32, sstep=SST, block=BLK),
                            traffic, sstep=SST, block=BLK)
    nrhs = len(w.inc)
    lat = np.array(solve_t)
    result = {
        "metric": METRIC,
        "value": nt * nt * args.steps / total,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32-fill/f64" if PREC == cbfm.FP32 else "f64") + ("/f32-basis-storage" if B32 else ""),
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {nt} triangles, {3 * nt // 2} RWGs, {3 * nt} unknowns, "
                               f"{w.nblocks} cells, {nrhs} incidences, {len(w.gen)} generating waves",
                   "fill_precision": prec_name, "krylov_basis": "fp32" if B32 else "fp64",
                   "gmres": ("block (groups of up to 32 right-hand sides, one Krylov space each)" if BLK else
                             f"s-step, blocks of {SST}" if SST else "plain (DCGS2)"),
                   "n_cbf": int(cb.n_cbf), "solver": solver},
        "fill_projection_pair_evals_per_s": nt * nt / float(np.median(proj_t)),
        "solves_per_s": nrhs * args.steps / float(lat.sum()),
        "solves_per_s_end_to_end": nrhs * args.steps / total,
        "solve_batch_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                   "p99": float(np.percentile(lat, 99) * 1e3)},
        "gmres_iterations": {"mean": float(np.mean(iters)), "max": int(np.max(iters)),
                             "counts": "block iterations" if BLK else "iterations"},
        "gmres_relres_max": float(out["relres"].max()),
        "roofline": roof,
        "roofline_kernels": roofs,
        "flop_per_pair": FLOP_PER_PAIR,
    }
    rcs_ref = out["rcs"]
    if PREC != cbfm.FP64 or args.fp64_steps:
        # the plain FP64 form of the same step beside the timed one
        k = args.fp64_steps or max(1, args.steps // 2)
        step(cbfm.FP64, sstep=SST, block=BLK)
        tp_l, ts_l = [], []
        torch.cuda.synchronize()
        tt = time.perf_counter()
        for _ in range(k):
            _, o64, tp, ts = step(cbfm.FP64, sstep=SST, block=BLK)
            tp_l.append(tp)
            ts_l.append(ts)
        torch.cuda.synchronize()
        tt = time.perf_counter() - tt
        _, r64 = rooflines(cbfm, lambda timed: step(cbfm.FP64, timed=timed, sstep=SST, block=BLK), traffic,
                           sstep=SST, block=BLK)
        rcs_ref = o64["rcs"]
        result["fp64_leg"] = {"steps": k, "value": nt * nt * k / tt, "ms_per_step": tt / k * 1e3,
                              "fill_projection_pair_evals_per_s": nt * nt / float(np.median(tp_l)),
                              "solves_per_s": nrhs * k / float(np.sum(ts_l)),
                              "gmres_iterations_max": int(o64["iters"].max()), "status": o64["status"],
                              "rcs_max_rel_err_of_timed_step": float(np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref)),
                              "roofline_kernels": r64}
        log(f"fp64 leg: {result['fp64_leg']}")
    if BLK and not args.no_per_rhs:
        # the same step with every right-hand side in its own Krylov space
        # (s-step cycles of 8, the form the block solve replaces)
        step(PREC, sstep=8)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        _, o1, tp, ts = step(PREC, sstep=8)
        torch.cuda.synchronize()
        tt = time.perf_counter() - tt
        result["per_rhs_leg"] = {"gmres": "s-step, blocks of 8, one Krylov space per right-hand side",
                                 "ms_per_step": tt * 1e3, "solve_ms": ts * 1e3, "value": nt * nt / tt,
                                 "gmres_iterations_max": int(o1["iters"].max()), "status": o1["status"],
                                 "rcs_max_rel_diff_vs_block": float(np.max(np.abs(o1["rcs"] - out["rcs"]) / o1["rcs"]))}
        log(f"per-rhs leg: {result['per_rhs_leg']}")
    if (args.workload == "cylinder19968" and not args.no_ipcbf) or args.ipcbf:
        # the cylinder: the paper's in-plane generating waves (its incidences
        # lie in that plane); otherwise the Table-I waves of the primary CBFs
        log("ipcbf leg")
        result["ipcbf"] = ipcbf_leg(cbfm, torch, w, mesh, med, PREC, out["rcs"], int(out["iters"].max()),
                                    result["ms_per_step"], solver,
                                    gen=None if args.workload == "cylinder19968" else w.gen)
        log(f"ipcbf: {result['ipcbf']}")
    if w.extra.get("max_L") and args.mom:
        log("mom leg")
        result["mom_comparison"] = mom_leg(cbfm, torch, w, mesh, med, cb, state[cb.n_cbf], solver)
        log(f"mom: {result['mom_comparison']}")
    if w.extra.get("max_L"):
        # the paper's comparison on its array: the same CBFs solved without
        # the CMP (the K-diagonal CBFM without G^CBF), full GMRES up to 1000
        # iterations
        nc = state[cb.n_cbf]
        o = cbfm.solve(mesh, med, cb, nc, w.inc, use_cmp=False, max_iter=1000, restart=1000, **solver)
        result["without_cmp"] = {"gmres_iterations_max": int(o["iters"].max()), "status": o["status"],
                                 "relres_max": float(o["relres"].max())}
        log(f"without CMP: {result['without_cmp']}")
        sweep = {}
        for er in ((1.0, 2.0, 3.0, 4.0, 5.0, 6.0) if args.workload == "sphere_array4x4x2" else ()):
            med_e = cbfm.Medium.make(w.k0, w.eta0, er + 0j, w.mu_r)
            cb_e = cbfm.build_cbf(mesh, med_e, w.gen, w.delta_svd, max_L=w.extra["max_L"])
            cbfm.project(mesh, med_e, cb_e, nc, cbfm.FP64)
            a = cbfm.solve(mesh, med_e, cb_e, nc, w.inc, tol=1e-4, max_iter=3000, restart=3000, use_cmp=True)
            b = cbfm.solve(mesh, med_e, cb_e, nc, w.inc, tol=1e-4, max_iter=3000, restart=3000, use_cmp=False)
            sweep[f"{er:g}"] = {"with_cmp": int(a["iters"].max()), "without_cmp": int(b["iters"].max())}
        if sweep:
            result["eps_r_sweep_tol_1e-4"] = sweep
            log(f"eps_r sweep: {sweep}")
    if not args.no_fp32:
        # the precision forms on the same workload: the compressed-basis
        # form (the timed step with its Krylov basis stored in float, double
        # arithmetic, cycles restarted from the double residual), the mixed
        # forms (FP32 fill, FP32 or split-BF16 matrix-core projection, float
        # GMRES cycles refined against the double residual), and the FP32
        # fill alone when the timed step is FP64.  CBF build, near pairs, the
        # SVD and the refinement residual stay FP64.  RCS error against the
        # FP64 step.
        forms = {}
        legs = [("compressed_basis", PREC, dict(basis_fp32=True)),
                ("mixed_fp32", cbfm.MIXED_FP32, dict(inner_fp32=True)),
                ("mixed_bf16x3", cbfm.MIXED_BF16X3, dict(inner_fp32=True))][1 if B32 else 0:]
        if PREC == cbfm.FP64:
            legs.insert(0, ("fp32_fill", cbfm.FP32, {}))
        for name, prec, kw in legs:
            step(prec, **kw)
            tp_l, ts_l, tt = [], [], time.perf_counter()
            k = max(1, args.steps // 4)
            for _ in range(k):
                _, o, tp, ts = step(prec, **kw)
                tp_l.append(tp)
                ts_l.append(ts)
            torch.cuda.synchronize()
            tt = time.perf_counter() - tt
            forms[name] = {"steps": k, "value": nt * nt * k / tt, "ms_per_step": tt / k * 1e3,
                           "fill_projection_pair_evals_per_s": nt * nt / float(np.median(tp_l)),
                           "solves_per_s": nrhs * k / float(np.sum(ts_l)),
                           "gmres_iterations_max": int(o["iters"].max()), "status": o["status"],
                           "rcs_max_rel_err_vs_fp64": float(np.max(np.abs(o["rcs"] - rcs_ref) / rcs_ref))}
            log(f"{name}: {forms[name]}")
        result["precision_forms"] = forms
    if args.ipcbf_conditions:
        log("ipcbf conditions")
        result["ipcbf_conditions"] = ipcbf_conditions_leg(cbfm, torch, w, med)
    if not args.no_batching:
        log("batching")
        result["batching"] = batching_leg(cbfm, torch)
        log(f"batching: {result['batching']}")
    if args.serve > 0:
        log("serving")
        result["serving"] = serving_legs(cbfm, torch, args.serve, args.serve_slots)
    if not args.no_cpu_baseline:
        # in a child process that never touches the GPU (its worker pool forks)
        log("cpu baseline (oracle)")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--workload",
                            args.workload, "--cpu-sample", str(args.cpu_sample), "--cpu-cores", str(cores)],
                           capture_output=True, text=True)
        sys.stderr.write(r.stderr)
        if r.returncode == 0:
            result["cpu_baseline"] = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
