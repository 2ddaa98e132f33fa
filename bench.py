#!/usr/bin/env python3
"""Benchmark of the CBFM + Calderon-preconditioned PMCHWT hot path on one
MI355X.

One step = the whole path for one scatterer and its batch of incidences:
primary CBFs with dual orthogonalisation (cbfm_build_cbf), the PMCHWT fill
fused with the projection Z_r = (C^JM)^H Z C^MJ (cbfm_project) and the
right-preconditioned GMRES solve of every incidence to its monostatic RCS
(cbfm_solve).  The mesh is loaded and resident on the device before the
timed region.

Workload (default): dielectric cube, edge 1 wavelength, eps_r 2.5, 12 x 12
squares per face (1,728 triangles, 2,592 RWGs, 5,184 unknowns), 27 cells,
64 seeded incidences, CBFs from the 144 Table-I plane waves, delta_SVD 1e-3.

value = logical triangle pair-evaluations (N_tri^2 per step) per second of
the whole step.  After the timed steps one more step runs with the library's
event timers on; the roofline entry is for the kernel family with the most
GPU time in it (algorithmic work per launch over the average launch
duration), and roofline_kernels lists every timed family.  HBM traffic per
launch comes from the committed counter summary when the kernel's source is
unchanged since it was measured, else it is null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PMCHWT fill+projection pair-evals/s; solves/s with p50/p99 latency"

# Algorithmic FP64 flops of one regular triangle pair in the fill kernel
# (FMA = 2 flops; square roots, reciprocals, sines/cosines not counted):
#   49 point pairs x 73 (distance 12, Green's functions of both media 24,
#   inner accumulations 40 -- less 3 for the folded weight products)
#   + 7 outer points x 190 (T moments 84, K moments 106)
#   + 9 local pairs x 110 (K 38, two media X_i 36, two output operators 36)
FLOP_PER_PAIR = 49 * 73 + 7 * 190 + 9 * 110
PEAK_FP64_VALU = 78.6e12
PEAK_FP64_MFMA = 78.6e12
PEAK_HBM = 8.0e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_cube1728.txt")

# timer family -> (kernel, bound, peak, unit, scale of the timer's work unit)
FAMILIES = {
    "fill_regular": ("fill_regular_kernel<double>", "alu", PEAK_FP64_VALU, "TFLOP/s", FLOP_PER_PAIR),
    "gemm": ("zgemm_batched_kernel", "mfma", PEAK_FP64_MFMA, "TFLOP/s", 1.0),
    "gmres_dots": ("dots2_kernel", "hbm", PEAK_HBM, "GB/s", 1.0),
    "gmres_update": ("dcgs_update_kernel", "hbm", PEAK_HBM, "GB/s", 1.0),
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


def measured_traffic():
    """Per-kernel HBM bytes per launch from the committed counter summary,
    kept only where the kernel's source file still has the hash recorded
    with the measurement."""
    out = {}
    if not os.path.exists(TRAFFIC_FILE):
        return out
    for line in open(TRAFFIC_FILE):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        src = os.path.join(ROOT, f["source"])
        if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == f["sha256"]:
            out[f["kernel"]] = float(f["bytes_per_dispatch"])
    return out


# timer family -> (substring of the kernel symbol, source file)
FAMILY_SOURCES = {
    "fill_regular": ("fill_regular_kernel<double", "paper_2111_11058_amd/csrc/fill.hip"),
    "gemm": ("zgemm_batched_kernel", "paper_2111_11058_amd/csrc/gemm.hip"),
    "gmres_dots": ("dots2_kernel", "paper_2111_11058_amd/csrc/solve.hip"),
    "gmres_update": ("dcgs_update_kernel", "paper_2111_11058_amd/csrc/solve.hip"),
}


def write_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, cmd):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of this
    benchmark, then of the 1 GiB copy) into the traffic summary: per kernel
    family the mean KiB per dispatch, scaled so that the copy reads and
    writes exactly 1 GiB, with the hash of the kernel's source."""
    import csv
    from collections import defaultdict

    def per_dispatch(d, sub):
        acc = defaultdict(float)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if sub in r["Kernel_Name"]:
                acc[r["Dispatch_Id"]] += float(r["Counter_Value"])
        return list(acc.values())

    gib_kib = float(1 << 20)
    fs = gib_kib / np.mean(per_dispatch(cfetch_dir, "__amd_rocclr_copyBuffer"))
    ws = gib_kib / np.mean(per_dispatch(cwrite_dir, "__amd_rocclr_copyBuffer"))
    lines = ["# HBM traffic per dispatch, cube1728 bench step (FP64), from rocprofv3 --pmc",
             f"# command: {cmd}",
             f"# calibration: a 1 GiB device copy reads {1 / fs:.4f} GiB by FETCH_SIZE and writes "
             f"{1 / ws:.4f} GiB by WRITE_SIZE; scales fetch x{fs:.4f}, write x{ws:.4f}"]
    for fam, (sub, src) in FAMILY_SOURCES.items():
        f, w = per_dispatch(fetch_dir, sub), per_dispatch(write_dir, sub)
        if not f or not w:
            continue
        sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        fk, wk = float(np.mean(f)), float(np.mean(w))
        b = (fk * fs + wk * ws) * 1024.0
        lines.append(f"kernel={fam} symbol={sub.split('<')[0]} source={src} sha256={sha} dispatches={len(f)} "
                     f"fetch_kib={fk:.1f} write_kib={wk:.1f} bytes_per_dispatch={b:.0f}")
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def rooflines(cbfm, step):
    """One step with every timer family on: achieved rate of each family
    against its peak; the dominant family is the one with the most time."""
    cbfm.timer_enable(list(FAMILIES))
    step()
    traffic = measured_traffic()
    rows = {}
    for fam, (kernel, bound, peak, unit, scale) in FAMILIES.items():
        n, ms, work = cbfm.timer_read(fam, with_work=True)
        if n == 0 or ms <= 0:
            continue
        per_launch = work * scale / n
        avg_s = ms * 1e-3 / n
        ach = per_launch / avg_s
        div = 1e12 if unit == "TFLOP/s" else 1e9
        rows[fam] = {"bound": bound, "achieved": ach / div, "peak": peak / div, "unit": unit, "frac": ach / peak,
                     "traffic": traffic.get(fam), "kernel": kernel, "launches": n, "avg_launch_ms": ms / n,
                     "total_ms": ms, "work_per_launch": per_launch}
    cbfm.timer_enable(None)
    dom = max(rows, key=lambda k: rows[k]["total_ms"])
    return rows[dom], rows


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
            "unknowns": {"min": int(min(r.unknowns for r in stream)), "max": int(max(r.unknowns for r in stream))}}


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


def cpu_baseline(w, sample, seed=5):
    """The oracle's fill timed on a bounded, seeded sample of the workload's
    triangle pairs (regular and near pairs in the workload's proportion)."""
    from oracle import fill, mesh as om
    m = om.build(w.V, w.T)
    k, _ = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    near = om.near_pairs(m)
    frac = len(near) / m.nt ** 2
    rng = np.random.default_rng(seed)
    n_near = max(1, int(round(sample * frac)))
    n_reg = sample - n_near
    isn = set(map(tuple, near.tolist()))
    P = rng.integers(0, m.nt, n_reg * 2)
    Q = rng.integers(0, m.nt, n_reg * 2)
    keep = np.array([(p, q) not in isn for p, q in zip(P.tolist(), Q.tolist())])
    P, Q = P[keep][:n_reg], Q[keep][:n_reg]
    pick = near[rng.choice(len(near), n_near, replace=False)]
    t0 = time.perf_counter()
    for s in range(0, len(P), 4096):
        fill.regular_local(m, k, P[s:s + 4096], Q[s:s + 4096])
    for p, q in pick:
        fill.near_local(m, k, int(p), int(q))
    dt = time.perf_counter() - t0
    return {"value": (n_reg + n_near) / dt, "unit": "pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FP64 fill of {n_reg} regular + {n_near} near triangle pairs "
                      f"(seeded, of {m.nt ** 2} in the workload), {dt:.1f} s on one core; "
                      f"projection, CBF build and solve not included"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube1728", choices=["cube1728", "sphere320", "sphere5120", "cylinder19968",
                                                                "sphere_array4x4x2", "sphere_array8x16x2",
                                                                "cube_array8x2x2"])
    ap.add_argument("--cpu-sample", type=int, default=250000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the precision-form legs (FP32 fill, mixed FP32 and split-BF16)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for the HBM byte counters)")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the traffic summary from four rocprofv3 --pmc output folders (no GPU use)")
    ap.add_argument("--traffic-command", default="", help="command line recorded in the traffic summary")
    ap.add_argument("--serve", type=int, default=32,
                    help="requests of the serving leg (mixed-size stream, Poisson arrivals); 0 skips it")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg (both budgets)")
    ap.add_argument("--serve-slots", type=int, default=4)
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, args.traffic_command)
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
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported",
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
    log(f"bench: {w.name} nt={w.nt} cells={w.nblocks} nrhs={len(w.inc)}")
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    solver = dict(tol=1e-6)
    state = {}

    def step(precision, inner_fp32=False):
        cb = cbfm.build_cbf(mesh, med, w.gen, w.delta_svd, max_L=w.extra.get("max_L", 0))
        n = cb.n_cbf
        Zr = state.get(n)
        if Zr is None:
            Zr = state[n] = torch.empty((n, n), dtype=torch.complex128, device="cuda")
        t0 = time.perf_counter()
        cbfm.project(mesh, med, cb, Zr, precision)
        # (the caller's stream only: the CMP inverse that the CBF build left
        # on the library's side stream may still run beside the projection)
        torch.cuda.current_stream().synchronize()
        t1 = time.perf_counter()
        # full (unrestarted) GMRES while the Krylov basis of all right-hand
        # sides stays small, else cycles of 1000
        m = n if n * n * len(w.inc) * 16 * 3 < 8 << 30 else 1000
        out = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=(3 if inner_fp32 else 1) * max(n, 3000),
                         restart=m, inner_fp32=inner_fp32, **solver)
        t2 = time.perf_counter()
        return cb, out, t1 - t0, t2 - t1

    for i in range(args.warmup):
        log(f"warmup {i}")
        step(cbfm.FP64)
    torch.cuda.synchronize()
    proj_t, solve_t, iters = [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        cb, out, tp, ts = step(cbfm.FP64)
        proj_t.append(tp)
        solve_t.append(ts)
        iters.append(out["iters"])
        log(f"step {i}: project {tp * 1e3:.1f} ms, solve {ts * 1e3:.1f} ms, N_CBF={cb.n_cbf}, "
            f"iters max {out['iters'].max()} status {out['status']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    nt = w.nt
    roof, roofs = rooflines(cbfm, lambda: step(cbfm.FP64))
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {nt} triangles, {3 * nt // 2} RWGs, {3 * nt} unknowns, "
                               f"{w.nblocks} cells, {nrhs} incidences, {len(w.gen)} generating waves",
                   "n_cbf": int(cb.n_cbf), "solver": solver},
        "fill_projection_pair_evals_per_s": nt * nt / float(np.median(proj_t)),
        "solves_per_s": nrhs * args.steps / float(lat.sum()),
        "solve_batch_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                   "p99": float(np.percentile(lat, 99) * 1e3)},
        "gmres_iterations": {"mean": float(np.mean(iters)), "max": int(np.max(iters))},
        "roofline": roof,
        "roofline_kernels": roofs,
        "flop_per_pair": FLOP_PER_PAIR,
    }
    if w.extra.get("max_L"):
        # the paper's comparison on its array: the same CBFs solved without
        # the CMP (the K-diagonal CBFM without G^CBF), full GMRES up to 1000
        # iterations
        nc = state[cb.n_cbf]
        o = cbfm.solve(mesh, med, cb, nc, w.inc, use_cmp=False, max_iter=1000, restart=1000, **solver)
        result["without_cmp"] = {"gmres_iterations_max": int(o["iters"].max()), "status": o["status"],
                                 "relres_max": float(o["relres"].max())}
        log(f"without CMP: {result['without_cmp']}")
        # iterations to 1e-4 against eps_r, with and without the CMP (the
        # paper's figure for the 4 x 4 x 2 array)
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
        # the precision forms on the same workload: FP32 regular fill with the
        # FP64 projection and solve; and the mixed forms (FP32 fill, FP32 or
        # split-BF16 matrix-core projection, float GMRES cycles refined
        # against the double residual).  CBF build, near pairs, the SVD and
        # the refinement residual stay FP64.  RCS error against this run's
        # FP64 step.
        rcs64 = out["rcs"]
        forms = {}
        for name, prec, inner in (("fp32_fill", cbfm.FP32, False), ("mixed_fp32", cbfm.MIXED_FP32, True),
                                  ("mixed_bf16x3", cbfm.MIXED_BF16X3, True)):
            step(prec, inner)
            tp_l, ts_l, tt = [], [], time.perf_counter()
            k = max(1, args.steps // 2)
            for _ in range(k):
                _, o, tp, ts = step(prec, inner)
                tp_l.append(tp)
                ts_l.append(ts)
            torch.cuda.synchronize()
            tt = time.perf_counter() - tt
            forms[name] = {"value": nt * nt * k / tt, "ms_per_step": tt / k * 1e3,
                           "fill_projection_pair_evals_per_s": nt * nt / float(np.median(tp_l)),
                           "solves_per_s": nrhs * k / float(np.sum(ts_l)),
                           "gmres_iterations_max": int(o["iters"].max()), "status": o["status"],
                           "rcs_max_rel_err_vs_fp64": float(np.max(np.abs(o["rcs"] - rcs64) / rcs64))}
            log(f"{name}: {forms[name]}")
        result["precision_forms"] = forms
    if args.serve > 0:
        log("serving")
        result["serving"] = serving_legs(cbfm, torch, args.serve, args.serve_slots)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
