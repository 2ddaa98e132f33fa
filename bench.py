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
the whole step.  The roofline entry is for the dominant kernel, the
regular-pair fill, from HIP events recorded around its launches.
"""
from __future__ import annotations

import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from synth import configs
    if name == "cube1728":
        return configs.cube_c2()
    if name == "sphere320":
        return configs.sphere_c1()
    raise SystemExit(f"unknown workload {name}")


def cell_supports(w):
    """Triangle count of each cell's RWG support (the CBF build fills each
    cell's support against itself)."""
    from synth.meshes import edges_canonical
    E = edges_canonical(w.T)
    key = {(int(a), int(b)): i for i, (a, b) in enumerate(E)}
    tri_of = [[] for _ in range(len(E))]
    for t, (a, b, c) in enumerate(w.T.tolist()):
        for u, v in ((a, b), (b, c), (c, a)):
            tri_of[key[(min(u, v), max(u, v))]].append(t)
    sizes = []
    for c in range(w.nblocks):
        ts = set()
        for e in np.nonzero(w.edge_block == c)[0]:
            ts.update(tri_of[e])
        sizes.append(len(ts))
    return np.array(sizes)


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
    ap.add_argument("--workload", default="cube1728", choices=["cube1728", "sphere320"])
    ap.add_argument("--cpu-sample", type=int, default=250000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-fill comparison leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
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
    w = workload(args.workload)
    log(f"bench: {w.name} nt={w.nt} cells={w.nblocks} nrhs={len(w.inc)}")
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    solver = dict(tol=1e-6)
    state = {}

    def step(precision):
        cb = cbfm.build_cbf(mesh, med, w.gen, w.delta_svd)
        n = cb.n_cbf
        Zr = state.get(n)
        if Zr is None:
            Zr = state[n] = torch.empty((n, n), dtype=torch.complex128, device="cuda")
        t0 = time.perf_counter()
        cbfm.project(mesh, med, cb, Zr, precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # full (unrestarted) GMRES: the Krylov dimension is bounded by N_CBF
        out = cbfm.solve(mesh, med, cb, Zr, w.inc, use_cmp=True, max_iter=n, restart=n, **solver)
        t2 = time.perf_counter()
        return cb, out, t1 - t0, t2 - t1

    for i in range(args.warmup):
        log(f"warmup {i}")
        step(cbfm.FP64)
    torch.cuda.synchronize()
    cbfm.timer_enable(["fill_regular"])
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
    nl, ms = cbfm.timer_read("fill_regular")
    cbfm.timer_enable(None)
    nt = w.nt
    pairs_per_step = nt * nt + int((cell_supports(w) ** 2).sum())
    flops = FLOP_PER_PAIR * pairs_per_step * args.steps
    achieved = flops / (ms * 1e-3) if ms > 0 else 0.0
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
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": None,
                     "kernel": "fill_regular_kernel<double>", "launches": nl,
                     "avg_launch_ms": ms / max(nl, 1), "flop_per_pair": FLOP_PER_PAIR,
                     "pairs_per_step": pairs_per_step},
    }
    if not args.no_fp32:
        # same step with the regular-pair fill in FP32 (near pairs, CBFs, solve in FP64)
        step(cbfm.FP32)
        t32 = []
        for _ in range(max(1, args.steps // 2)):
            _, out32, tp, ts = step(cbfm.FP32)
            t32.append(tp)
        result["fp32_fill"] = {"fill_projection_pair_evals_per_s": nt * nt / float(np.median(t32))}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
