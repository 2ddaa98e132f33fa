"""GPU parity of the paths the full-size workloads take, against the FP64
oracle, through the C ABI: the projection split into several row panels,
the lossy FP32 fill and the mixed forms on a lossy body, the Gauss-Jordan
CMP inverse at orders that need three pivot rounds, the single-RHS GMRES
with long vectors, and sampled outputs of the 19,968-triangle cylinder
(fill rows and Z_r blocks in the launch configuration of the benchmark).

Every comparison reports the normwise error ||X - R|| / ||R|| and the
elementwise one max |X - R| / max |R|, and bounds both."""
import numpy as np
import pytest

from conftest import oracle_problem
from test_gpu_cbf_solve import _gpu_handles, _oracle_cbf

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _elem(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _both(a, b, what):
    r, e = _rel(a, b), _elem(a, b)
    print(f"{what}: normwise {r:.2e} elementwise {e:.2e}", flush=True)
    return r, e


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.mark.parametrize("name", ["c1", "cyl_small"])
def test_multipanel_projection_parity(torch_cuda, name):
    """Row panels of one cell each, and of a few cells each (a budget that
    splits the cells raggedly): the per-panel near lists, the row offsets of
    each panel into the W products and the per-panel Z_r rows, in FP64, with
    the FP32 fill and in the mixed FP32 form."""
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf(name)
    w = O["P"]["w"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    # one cell per panel (budget 1 byte), then a budget halved from the
    # whole-mesh scratch until three or more panels form (some holding
    # several cells) in the mixed form, whose panels need the least
    # scratch (so the other precisions split at least as finely)
    nb = mesh.nblocks
    budgets = [1]
    Z = torch_cuda.full((n, n), complex(np.nan, np.nan), dtype=torch_cuda.complex128, device="cuda")
    b = 64 << 20
    while b > 1 << 16:
        if cbfm.project(mesh, med, cbf, Z, cbfm.MIXED_FP32, panel_bytes=b) >= 3:
            budgets.append(b)
            break
        b //= 2
    assert len(budgets) == 2
    for budget in budgets:
        Z = torch_cuda.full((n, n), complex(np.nan, np.nan), dtype=torch_cuda.complex128, device="cuda")
        print(f"multi-panel projection {w.name} budget {budget}", flush=True)
        np_ = cbfm.project(mesh, med, cbf, Z, cbfm.FP64, panel_bytes=budget)
        print("panels", np_)
        assert np_ >= 3 and (budget > 1 or np_ == nb)
        r, e = _both(Z.cpu().numpy(), O["Zr"], f"Z_r fp64 {np_} panels")
        assert r < 1e-10 and e < 1e-10
        np32 = cbfm.project(mesh, med, cbf, Z, cbfm.FP32, panel_bytes=budget)
        r, e = _both(Z.cpu().numpy(), O["Zr"], f"Z_r fp32 fill {np32} panels")
        assert np32 >= 3 and r < 1e-4 and e < 1e-4
        npm = cbfm.project(mesh, med, cbf, Z, cbfm.MIXED_FP32, panel_bytes=budget)
        r, e = _both(Z.cpu().numpy(), O["Zr"], f"Z_r mixed fp32 {npm} panels")
        assert npm >= 3 and r < 1e-4 and e < 1e-4


def test_fp32_fill_lossy(torch_cuda):
    """The FP32 regular fill with the attenuation factor of a lossy interior
    (eps_r = 4 - 0.1j, the permittivity of the lossy sphere workload)."""
    from paper_2111_11058_amd import cbfm
    P = oracle_problem("cyl_lossy")
    w = P["w"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    ne = mesh.ne
    for layout, refs in ((cbfm.LAYOUT_MEDIA3, (P["Kop"], P["T1"], P["T2"])),
                         (cbfm.LAYOUT_OPS3, (P["Kc"], P["TE"], P["TH"]))):
        out = torch_cuda.full((3, ne, ne), complex(np.nan, np.nan), dtype=torch_cuda.complex64, device="cuda")
        print(f"fp32 lossy fill layout {layout}", flush=True)
        cbfm.fill_pmchwt(mesh, med, out, cbfm.FP32, layout)
        got = out.cpu().numpy().astype(np.complex128)
        for o, R_ in enumerate(refs):
            r, e = _both(got[o], R_, f"fp32 lossy op {o}")
            assert r < 2e-5 and e < 2e-5


def test_mixed_forms_on_a_lossy_body(torch_cuda):
    """FP32 fill with FP32 and split-BF16 matrix-core projection on the lossy
    cylinder, then the refined float GMRES: Z_r within 1e-4 of the oracle,
    the monostatic RCS within 1e-4, the current error stated."""
    from oracle import excitation
    O = _oracle_cbf("cyl_lossy")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    vr = O["CJM"].conj().T @ excitation.rhs(m, w.inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    rcs_ref = excitation.monostatic_rcs(m, jref, w.inc, w.k0, w.eta0)
    Z = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    jt = torch_cuda.zeros((len(w.inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    for prec, name in ((cbfm.FP32, "fp32 fill"), (cbfm.MIXED_FP32, "mixed fp32"), (cbfm.MIXED_BF16X3, "split bf16")):
        print(f"lossy {name}", flush=True)
        cbfm.project(mesh, med, cbf, Z, prec)
        r, e = _both(Z.cpu().numpy(), O["Zr"], f"lossy Z_r {name}")
        assert r < 1e-4 and e < 1e-4
        out = cbfm.solve(mesh, med, cbf, Z, w.inc, tol=1e-8, max_iter=4 * n, restart=n, inner_fp32=prec != cbfm.FP32,
                         j_out=jt)
        assert out["status"] == "OK"
        rcs_err = np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref)
        cur_err = _rel(jt.cpu().numpy().T, jref)
        print(f"lossy {name}: RCS max rel err {rcs_err:.2e}, current rel err {cur_err:.2e}")
        assert rcs_err < 1e-4


_C3 = {}


def _c3_random_dual_cbfs():
    """Dual CBFs of the 5,120-triangle lossy sphere (64 cells) built by the
    oracle's orthogonalisation from seeded random current sets of 40
    columns per cell: sum L > 2048, so the CMP's B needs three tournament
    rounds of pivot choice, and N_CBF > 2048 (long Krylov vectors)."""
    if _C3:
        return _C3
    from oracle import cbf, mesh as om, reduced
    from synth import configs
    w = configs.sphere_c3()
    m = om.build(w.V, w.T)
    sizes = np.bincount(w.edge_block, minlength=w.nblocks)
    cur = configs.random_cell_sets(sizes, 40, seed=21)
    Gs = cbf.rwg_gram_sparse(m)
    cb = cbf.dual_from_currents(m, w.edge_block, cur, 1e-3, G=Gs)
    _C3.update(w=w, m=m, cb=cb, B=reduced.gram_b(Gs, cb))
    return _C3


def test_cmp_apply_three_pivot_rounds(torch_cuda):
    from oracle import reduced
    from paper_2111_11058_amd import cbfm
    D = _c3_random_dual_cbfs()
    w, cb, B = D["w"], D["cb"], D["B"]
    NL = B.shape[0]
    print("sum L", NL, flush=True)
    assert NL > 2048
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    h = cbfm.cbf_import(mesh, cb.CM, cb.CJ, cb.sigma)
    n = h.n_cbf
    from synth import configs
    y = configs.random_complex((2, n), 22)
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(h, yt, xt)
    x = xt.cpu().numpy()
    ref = reduced.cmp_solve(B, y.T).T
    cond = np.linalg.cond(B)
    back = max(np.linalg.norm(-B.conj().T @ x[:, :NL].T - y[:, :NL].T), np.linalg.norm(B @ x[:, NL:].T - y[:, NL:].T)) \
        / (np.linalg.norm(B, 2) * np.linalg.norm(x))
    r, e = _both(x, ref, f"cmp apply order {NL} (cond {cond:.1e})")
    print("backward error", back)
    assert back < 1e-14 and r < max(1e-10, 1e-14 * cond) and e < max(1e-10, 1e-14 * cond)


def test_single_rhs_long_vector_solve(torch_cuda):
    """GMRES with N_CBF > 2048 and fewer than 16 right-hand sides (the
    unrolled dot pass of long vectors) on Z_r = I + E (E seeded, spectral
    norm about 0.4), without the CMP, against LU of the same Z_r: currents
    and monostatic RCS; one and three right-hand sides."""
    from oracle import excitation, reduced
    from paper_2111_11058_amd import cbfm
    from synth import configs
    D = _c3_random_dual_cbfs()
    w, m, cb = D["w"], D["m"], D["cb"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    h = cbfm.cbf_import(mesh, cb.CM, cb.CJ, cb.sigma)
    n = h.n_cbf
    assert n > 2048
    E = configs.random_complex((n, n), 23) * (0.4 / (2.0 * np.sqrt(n)))
    Zr = np.eye(n) + E
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zt = torch_cuda.tensor(Zr, dtype=torch_cuda.complex128, device="cuda")
    for inc in (w.inc, configs.random_incidences(3, 24)):
        nr = len(inc)
        v = excitation.rhs(m, inc, w.k0, w.eta0)
        jref = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ v)
        rcs_ref = excitation.monostatic_rcs(m, jref, inc, w.k0, w.eta0)
        jt = torch_cuda.zeros((nr, 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
        print(f"long-vector solve n={n} nrhs={nr}", flush=True)
        out = cbfm.solve(mesh, med, h, Zt, inc, tol=1e-12, max_iter=200, restart=200, use_cmp=False, j_out=jt)
        print(out["iters"], out["relres"])
        assert out["status"] == "OK"
        r, e = _both(jt.cpu().numpy().T, jref, f"currents nrhs={nr}")
        assert r < 1e-9 and e < 1e-9
        assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9


def test_block_solve_groups_of_32(torch_cuda):
    """Block GMRES in groups of 32 right-hand sides (the automatic size for
    N_CBF > 1,056) on Z_r = I + E (E seeded, spectral norm about 0.4; the
    5,120-triangle sphere's imported dual CBFs, N_CBF > 2048), without the
    CMP, against LU of the same Z_r: 34 incidences (groups of 32 and 2), two
    of them repeated so that the first group's block is rank deficient
    (random vectors take the dependent directions), and groups of 8 forced;
    currents and monostatic RCS at tol 1e-12."""
    from oracle import excitation, reduced
    from paper_2111_11058_amd import cbfm
    from synth import configs
    D = _c3_random_dual_cbfs()
    w, m, cb = D["w"], D["m"], D["cb"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    h = cbfm.cbf_import(mesh, cb.CM, cb.CJ, cb.sigma)
    n = h.n_cbf
    assert n > 33 * 32
    E = configs.random_complex((n, n), 27) * (0.4 / (2.0 * np.sqrt(n)))
    Zr = np.eye(n) + E
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zt = torch_cuda.tensor(Zr, dtype=torch_cuda.complex128, device="cuda")
    inc = configs.random_incidences(32, 28)
    inc = np.concatenate([inc[:30], inc[3:5], inc[30:]])
    v = excitation.rhs(m, inc, w.k0, w.eta0)
    jref = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ v)
    rcs_ref = excitation.monostatic_rcs(m, jref, inc, w.k0, w.eta0)
    for block in (1, 8):
        jt = torch_cuda.zeros((len(inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
        print(f"block solve n={n} nrhs={len(inc)} block={block}", flush=True)
        out = cbfm.solve(mesh, med, h, Zt, inc, tol=1e-12, max_iter=200, restart=n, use_cmp=False, j_out=jt,
                         block=block)
        print(out["iters"], out["relres"].max())
        assert out["status"] == "OK" and np.all(out["relres"] <= 1e-12)
        r, e = _both(jt.cpu().numpy().T, jref, f"block currents, block={block}")
        assert r < 1e-9 and e < 1e-9
        assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9


_C5 = {}


def _c5():
    if _C5:
        return _C5
    from oracle import fill, mesh as om
    from synth import configs
    w = configs.cylinder_c5()
    m = om.build(w.V, w.T)
    k, eta = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    print("c5 near pairs", flush=True)
    _C5.update(w=w, m=m, k=k, eta=eta, near=om.near_pairs(m))
    return _C5


def test_c5_sampled_fill_rows(torch_cuda):
    """Rows of K, T1, T2 of the 19,968-triangle cylinder (29,952 RWGs), FP64
    and FP32, against the oracle row by row."""
    from oracle import fill
    from paper_2111_11058_amd import cbfm
    C = _c5()
    w, m = C["w"], C["m"]
    rows = np.array([0, 7777, 15000, 29951])
    ref = fill.fill_block(m, C["k"], rows, np.arange(m.ne), near=C["near"])
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    for prec, tol in ((cbfm.FP64, 1e-10), (cbfm.FP32, 2e-5)):
        dt = torch_cuda.complex128 if prec == cbfm.FP64 else torch_cuda.complex64
        for i, r0 in enumerate(rows):
            out = torch_cuda.full((3, 1, m.ne), complex(np.nan, np.nan), dtype=dt, device="cuda")
            print(f"c5 fill row {r0} prec {prec}", flush=True)
            cbfm.fill_pmchwt(mesh, med, out, prec, cbfm.LAYOUT_MEDIA3, int(r0), 1)
            got = out.cpu().numpy().astype(np.complex128)
            for o in range(3):
                r, e = _both(got[o, 0], ref[o][i], f"c5 row {r0} op {o} prec {prec}")
                assert r < tol and e < tol


def test_c5_projection_sampled_blocks(torch_cuda):
    """Z_r of the 19,968-triangle cylinder with imported seeded CBFs (24 per
    current per cell, any matrices define a projection), projected as the
    benchmark does (default panel budget, FP64 and FP32 fill); blocks of
    cell pairs (self, neighbours, distant) against the oracle's fill of that
    cell pair projected with the same CBFs."""
    from oracle import fill, reduced
    from paper_2111_11058_amd import cbfm
    from synth import configs
    C = _c5()
    w, m = C["w"], C["m"]
    eb = w.edge_block
    sizes = np.bincount(eb, minlength=w.nblocks)
    L = 24
    sets = configs.random_cell_sets(sizes, L, seed=25)
    CM = [a for a, _ in sets]
    CJ = [b for _, b in sets]
    mesh = cbfm.Mesh(w.V, w.T, eb, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    h = cbfm.cbf_import(mesh, CM, CJ, [np.ones(L)] * w.nblocks)
    n = h.n_cbf
    NL = n // 2
    cells = [np.nonzero(eb == c)[0] for c in range(w.nblocks)]
    pairs = [(0, 0), (0, 1), (40, 95)]
    refs = []
    for a, b in pairs:
        print(f"c5 oracle block ({a},{b})", flush=True)
        Kab, T1, T2 = fill.fill_block(m, C["k"], cells[a], cells[b], near=C["near"])
        _, TE, TH = fill.combine(Kab, T1, T2, C["eta"])
        refs.append(reduced.project_block(Kab, TE, TH, CM[a], CJ[a], CM[b], CJ[b]))
    Z = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    for prec, tol in ((cbfm.FP64, 1e-10), (cbfm.FP32, 1e-4)):
        print(f"c5 projection prec {prec}", flush=True)
        cbfm.project(mesh, med, h, Z, prec)
        Zh = Z.cpu().numpy()
        for (a, b), ref in zip(pairs, refs):
            ra = np.r_[a * L:(a + 1) * L, NL + a * L:NL + (a + 1) * L]
            cb_ = np.r_[b * L:(b + 1) * L, NL + b * L:NL + (b + 1) * L]
            r, e = _both(Zh[np.ix_(ra, cb_)], ref, f"c5 Z_r block ({a},{b}) prec {prec}")
            assert r < tol and e < tol


def test_no_cmp_solve_parity(torch_cuda):
    """The K-diagonal CBFM without G^CBF (use_cmp = 0): GMRES on Z_r itself
    reaches the oracle's LU solution of the reduced system; currents and
    monostatic RCS."""
    from oracle import excitation
    O = _oracle_cbf("c1")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.tensor(O["Zr"], dtype=torch_cuda.complex128, device="cuda")
    jt = torch_cuda.zeros((1, 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    out = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, use_cmp=False, j_out=jt)
    print("no-CMP solve", out)
    assert out["status"] == "OK"
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], O["vr"])
    r, e = _both(jt.cpu().numpy().T, jref, "no-CMP currents")
    assert r < 1e-9 and e < 1e-9
    rcs_ref = excitation.monostatic_rcs(m, jref, w.inc, w.k0, w.eta0)
    assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9


def _golden_c3():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere5120_oracle_rcs.txt")
    mono, th, bi = None, [], []
    for line in open(path):
        if line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "monostatic":
            mono = float(f[1])
        else:
            th.append(float(f[1]))
            bi.append(float(f[2]))
    return mono, np.array(th), np.array(bi)


def test_precision_forms_on_the_lossy_sphere_against_the_oracle(torch_cuda):
    """The precision workload end to end (5,120 triangles, eps_r 4 - 0.1j,
    15,360 unknowns, 64 cells; GPU-built CBFs), each form against the
    oracle's CBFM RCS stored in tests/golden/sphere5120_oracle_rcs.txt
    (written by make_sphere5120_rcs.py from oracle/ alone; the oracle's
    CBFs span the same spaces, so the RCS agrees to the solver tolerance):
    the monostatic RCS and the bistatic pattern (theta = 0..180 deg, phi =
    0, error relative to the pattern's maximum).  FP64, and FP64 with the
    Krylov basis stored in float (compressed basis), within 1e-7; FP32 fill
    and mixed FP32 within 1e-4; split BF16 and BF16 reported, bounded by
    1e-3 and 0.1."""
    from paper_2111_11058_amd import cbfm
    from synth import configs
    mono_ref, th, bi_ref = _golden_c3()
    w = configs.sphere_c3()
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    cb = cbfm.build_cbf(mesh, med, w.gen, w.delta_svd)
    n = cb.n_cbf
    assert n == 3532  # the oracle's N_CBF (same singular-value counts)
    t = np.deg2rad(th)
    dirs = np.stack([np.sin(t), np.zeros_like(t), np.cos(t)], axis=1)
    Z = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    f32, b32 = dict(inner_fp32=True), dict(basis_fp32=True)
    forms = {"fp64": (cbfm.FP64, {}, 1e-7), "compressed_basis": (cbfm.FP64, b32, 1e-7),
             "fp32_fill": (cbfm.FP32, {}, 1e-4), "mixed_fp32": (cbfm.MIXED_FP32, f32, 1e-4),
             "split_bf16": (cbfm.MIXED_BF16X3, f32, 1e-3), "bf16": (cbfm.MIXED_BF16, f32, 0.1)}
    for name, (prec, kw, bar) in forms.items():
        print(f"sphere5120 {name}", flush=True)
        cbfm.project(mesh, med, cb, Z, prec)
        mo = cbfm.solve(mesh, med, cb, Z, w.inc, tol=1e-10, max_iter=4 * n, restart=n, **kw)
        bo = cbfm.solve(mesh, med, cb, Z, w.inc, tol=1e-10, max_iter=4 * n, restart=n, dirs=dirs, **kw)
        assert mo["status"] == "OK" and bo["status"] == "OK", (name, mo["status"], bo["status"])
        em = abs(mo["rcs"][0] - mono_ref) / mono_ref
        eb = np.abs(bo["rcs"][0] - bi_ref).max() / bi_ref.max()
        print(f"sphere5120 {name}: monostatic RCS rel err {em:.2e}, bistatic pattern err {eb:.2e}, "
              f"iterations {mo['iters'][0]}")
        assert em < bar and eb < bar, name
