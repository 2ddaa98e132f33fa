"""The serving form through the C ABI: continuous batching of mixed-size
scattering solves on one device, each result the same alone and in the mix,
admission within the memory budget, resident scatterers shared by key, and
a served result checked against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _req(cbfm, w, tol=1e-9, key=0, inc=None, inner_fp32=False):
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    return cbfm.make_request(w.V, w.T, w.edge_block, w.nblocks, med, w.gen, w.delta_svd,
                             w.inc if inc is None else inc, tol=tol, key=key, inner_fp32=inner_fp32)


def test_results_same_alone_and_in_the_mix(torch_cuda):
    from paper_2111_11058_amd import cbfm
    from synth import configs
    stream = configs.serving_stream(6, seed=7, max_unknowns=2200)
    srv = cbfm.Server(slots=3, budget_bytes=24 << 30)
    try:
        alone = []
        for r in stream:
            print(f"alone {r.work.name} {r.unknowns} unknowns nrhs={len(r.work.inc)}", flush=True)
            req, keep = _req(cbfm, r.work)
            alone.append(srv.wait(srv.submit(req)))
        print("mix", flush=True)
        built = [_req(cbfm, r.work) for r in stream]
        tickets = [srv.submit(req) for req, _ in built]
        mix = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    print(st)
    for r, a, b in zip(stream, alone, mix):
        assert a["status"] == "OK" and b["status"] == "OK", (r.work.name, a["status"], b["status"])
        assert np.array_equal(a["iters"], b["iters"])
        assert np.max(np.abs(a["rcs"] - b["rcs"]) / a["rcs"]) < 1e-12
    assert st["max_running"] >= 2 and st["peak_bytes"] <= 24 << 30
    # the mix overlapped on the device: some run intervals intersect
    iv = sorted((m["t_start"], m["t_end"]) for m in mix)
    assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))


def test_tight_budget_serialises_and_keys_share(torch_cuda):
    from paper_2111_11058_amd import cbfm
    from synth import configs
    w = configs.sphere_c1()
    req, keep = _req(cbfm, w)
    fp = cbfm.request_footprint(req)
    # a budget for one request at a time: never two running
    srv = cbfm.Server(slots=3, budget_bytes=int(fp * 1.5))
    try:
        ts = [srv.submit(_req(cbfm, w)[0]) for _ in range(3)]
        outs = [srv.wait(t) for t in ts]
        st = srv.stats()
    finally:
        srv.close()
    assert st["max_running"] == 1 and all(o["status"] == "OK" for o in outs)
    assert all(np.array_equal(o["rcs"], outs[0]["rcs"]) for o in outs)
    # equal keys: one resident scatterer, the later request only solves
    incs = configs.random_incidences(4, 99)
    srv = cbfm.Server(slots=2, budget_bytes=8 << 30)
    try:
        ref = srv.wait(srv.submit(_req(cbfm, w, inc=incs)[0]))
        k1 = srv.wait(srv.submit(_req(cbfm, w, inc=incs, key=42)[0]))
        k2 = srv.wait(srv.submit(_req(cbfm, w, inc=incs[::-1].copy(), key=42)[0]))
        st = srv.stats()
    finally:
        srv.close()
    assert st["resident"] == 1
    assert np.array_equal(k1["rcs"], ref["rcs"])
    assert np.max(np.abs(k2["rcs"][::-1] - ref["rcs"]) / ref["rcs"]) < 1e-12


def test_served_rcs_matches_oracle(torch_cuda):
    """The 320-triangle sphere served end to end (GPU-built CBFs) against the
    oracle's CBFM solution with its own CBFs: same spanned subspaces, so the
    RCS agrees to the solver tolerance."""
    from conftest import oracle_problem
    from oracle import cbf, excitation, reduced
    from paper_2111_11058_amd import cbfm
    P = oracle_problem("c1")
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, w.delta_svd)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    j = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ P["v"])
    ref = excitation.monostatic_rcs(m, j, w.inc, w.k0, w.eta0)
    srv = cbfm.Server(slots=1, budget_bytes=8 << 30)
    try:
        out = srv.wait(srv.submit(_req(cbfm, w, tol=1e-12)[0]))
    finally:
        srv.close()
    err = np.max(np.abs(out["rcs"] - ref) / ref)
    print("served vs oracle RCS", err)
    assert out["status"] == "OK" and err < 1e-8


def test_admission_keeps_within_budget(torch_cuda):
    """A budget for about two requests at a time: keyless requests hold their
    own mesh, CBFs and Z_r while they run, so admission counts them, and the
    admitted peak never exceeds the budget while several requests run."""
    from paper_2111_11058_amd import cbfm
    from synth import configs
    stream = configs.serving_stream(8, seed=9, max_unknowns=2200)
    built = [_req(cbfm, r.work) for r in stream]
    fps = [cbfm.request_footprint(req) for req, _ in built]
    budget = int(2.2 * max(fps))
    srv = cbfm.Server(slots=4, budget_bytes=budget)
    try:
        print(f"admission: 8 requests, budget {budget / 2**30:.2f} GiB", flush=True)
        tickets = [srv.submit(req) for req, _ in built]
        outs = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    print(st)
    assert all(o["status"] == "OK" for o in outs)
    assert st["peak_bytes"] <= budget


def test_served_mixed_solve_meets_the_rcs_bar(torch_cuda):
    """A request with inner_fp32 (float Krylov cycles refined against the
    double residual) against the oracle's FP64 CBFM RCS of the same sphere:
    within the mixed form's 1e-4, and the same result alone and beside FP64
    requests."""
    from conftest import oracle_problem
    from oracle import cbf, excitation, reduced
    from paper_2111_11058_amd import cbfm
    P = oracle_problem("c1")
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, w.delta_svd)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    j = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ P["v"])
    ref = excitation.monostatic_rcs(m, j, w.inc, w.k0, w.eta0)
    srv = cbfm.Server(slots=2, budget_bytes=8 << 30)
    try:
        alone = srv.wait(srv.submit(_req(cbfm, w, tol=1e-6, inner_fp32=True)[0]))
        built = [_req(cbfm, w, tol=1e-6, inner_fp32=f) for f in (True, False)]
        mix = [srv.wait(t) for t in [srv.submit(r) for r, _ in built]]
    finally:
        srv.close()
    err = np.max(np.abs(alone["rcs"] - ref) / ref)
    print("served mixed vs oracle RCS", err, "iterations", alone["iters"], mix[1]["iters"])
    assert alone["status"] == "OK" and err < 1e-4
    assert np.array_equal(alone["rcs"], mix[0]["rcs"]) and np.array_equal(alone["iters"], mix[0]["iters"])
