"""GPU parity of the CBF build, the projection Z_r = (C^JM)^H Z C^MJ, the
Calderon preconditioner and the reduced GMRES solve against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

from conftest import oracle_problem

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


_ORA = {}


def _oracle_cbf(name, delta=1e-3, max_L=None):
    key = (name, delta, max_L)
    if key in _ORA:
        return _ORA[key]
    from oracle import cbf, reduced
    P = oracle_problem(name)
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, delta)
    if max_L:
        cb = cbf.CBFSet(cb.cells, [c[:, :max_L] for c in cb.CM], [c[:, :max_L] for c in cb.CJ],
                        [s[:max_L] for s in cb.sigma], cb.sigma_all)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    G = cbf.rwg_gram(m)
    out = dict(P=P, cb=cb, CJM=CJM, CMJ=CMJ, G=G, Zr=reduced.project(P["Z"], CJM, CMJ),
               Gc=reduced.gram_cbf(G, CJM, CMJ), vr=CJM.conj().T @ P["v"])
    _ORA[key] = out
    return out


def _gpu_handles(w, O):
    from paper_2111_11058_amd import cbfm
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    cbf = cbfm.cbf_import(mesh, O["cb"].CM, O["cb"].CJ, O["cb"].sigma)
    return cbfm, mesh, med, cbf


@pytest.mark.parametrize("name", ["c1", "cyl_small"])
def test_project_parity_with_imported_cbfs(torch_cuda, name):
    O = _oracle_cbf(name)
    w = O["P"]["w"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    assert n == O["Zr"].shape[0]
    print(f"project {w.name} N_CBF={n}", flush=True)
    Zr = torch_cuda.full((n, n + 3), complex(np.nan, np.nan), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64, ldz=n + 3)
    got = Zr.cpu().numpy()[:, :n]
    err = _rel(got, O["Zr"])
    print("Zr fp64 rel err", err)
    assert err < 1e-10
    Zr32 = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr32, cbfm.FP32)
    err32 = _rel(Zr32.cpu().numpy(), O["Zr"])
    print("Zr fp32-fill rel err", err32)
    assert err32 < 1e-4


def test_cmp_apply_parity(torch_cuda):
    O = _oracle_cbf("cyl_small")
    w = O["P"]["w"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    rng = np.random.default_rng(11)
    y = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(cbf, yt, xt)
    ref = np.linalg.solve(O["Gc"], y.T).T
    err = _rel(xt.cpu().numpy(), ref)
    print("cmp err", err)
    assert err < 1e-10
    cbfm.cmp_apply(cbf, yt, yt)  # in place
    assert _rel(yt.cpu().numpy(), ref) < 1e-10


def test_cmp_apply_parity_two_pivot_rounds(torch_cuda):
    """c1 with delta_SVD = 1e-5 keeps 290 CBFs per current, so B (order 290,
    cells coupled) is inverted over panels whose first pivot rows come from
    two groups of 256 rows and a second tournament round."""
    O = _oracle_cbf("c1", delta=1e-5)
    w = O["P"]["w"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    assert n // 2 == 290
    rng = np.random.default_rng(13)
    y = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(cbf, yt, xt)
    x = xt.cpu().numpy()
    Gc = O["Gc"]
    back = np.linalg.norm(x @ Gc.T - y) / (np.linalg.norm(Gc, 2) * np.linalg.norm(x))
    fwd = _rel(x, np.linalg.solve(Gc, y.T).T)
    cond = np.linalg.cond(Gc)
    print("cmp backward", back, "forward", fwd, "cond", cond)
    assert back < 1e-14 and fwd < 1e-14 * cond


@pytest.mark.parametrize("name", ["cyl_small", "array2"])
def test_cmp_singular_b_reports_rank(torch_cuda, name):
    """With the magnetic CBFs set to zero, B = (C^M)^H G C^J is zero: the
    Gauss-Jordan inverse (dense for the coupled cylinder cells, block by
    block for the two disjoint spheres) finds no nonzero pivot and
    cmp_apply returns E_RANK; every kernel still runs to its end."""
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf(name)
    w = O["P"]["w"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    cbf = cbfm.cbf_import(mesh, [np.zeros_like(c) for c in O["cb"].CM], O["cb"].CJ, O["cb"].sigma)
    n = cbf.n_cbf
    y = torch_cuda.ones((1, n), dtype=torch_cuda.complex128, device="cuda")
    x = torch_cuda.empty_like(y)
    with pytest.raises(cbfm.CBFMError) as e:
        cbfm.cmp_apply(cbf, y, x)
    print(e.value)
    assert e.value.code == -6 and "singular" in str(e.value)


def test_cmp_inverse_formed_beside_the_projection(torch_cuda):
    """cbfm_build_cbf leaves the CMP inverse on the library's side stream,
    where it runs beside what is queued next (here the projection);
    cmp_apply waits for it.  Its result equals that of the inverse formed
    on first use (the same CBFs exported and imported again), whose parity
    with the oracle test_cmp_apply_parity checks."""
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf("c1")
    P = O["P"]
    w = P["w"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    cb = cbfm.build_cbf(mesh, med, w.gen, 1e-3)
    n = cb.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cb, Zr, cbfm.FP64)
    from synth import configs
    y = configs.random_complex((2, n), 14)
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(cb, yt, xt)
    CM, CJ = cb.export()
    again = cbfm.cbf_import(mesh, CM, CJ, [cb.sigma[a:b] for a, b in
                                           zip(np.r_[0, np.cumsum(cb.L)[:-1]], np.cumsum(cb.L))])
    xs = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(again, yt, xs)
    d = _rel(xt.cpu().numpy(), xs.cpu().numpy())
    print("side-stream inverse vs first-use inverse", d)
    assert d < 1e-13


def test_build_cbf_one_cell_order_960(torch_cuda):
    """The whole c1 body as one cell: its isolated system has order 960 (the
    first panels' pivot rows come from four groups of 256 rows and a second
    round) with 144 right-hand sides; kept count, singular values and the
    duality relation as the oracle's."""
    from oracle import cbf
    from paper_2111_11058_amd import cbfm
    P = oracle_problem("c1")
    w, m = P["w"], P["m"]
    eb = np.zeros(m.ne, dtype=np.int32)
    ref = cbf.build(m, P["Kc"], P["TE"], P["TH"], eb, w.gen, w.k0, w.eta0, 1e-3)
    mesh = cbfm.Mesh(w.V, w.T, eb, 1)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    print("build_cbf c1 as one cell", flush=True)
    cb = cbfm.build_cbf(mesh, med, w.gen, 1e-3)
    assert np.array_equal(cb.L, ref.L)
    s = ref.sigma[0]
    assert np.max(np.abs(cb.sigma - s)) < 1e-10 * s[0]
    CM, CJ = cb.export()
    G = cbf.rwg_gram(m)[np.ix_(ref.cells[0], ref.cells[0])]
    assert np.abs(CM[0].conj().T @ G @ CJ[0] - np.diag(s)).max() < 1e-9 * s[0]


def test_disjoint_cells_block_cmp_parity(torch_cuda):
    """Two disjoint spheres, one per cell: no triangle carries RWGs of both
    cells, so G^CBF is block-diagonal and the library inverts it block by
    block and forms the preconditioned operator per cell.  The CMP apply and
    the CMP-preconditioned solve against the oracle's dense G^CBF and LU."""
    from oracle import excitation
    O = _oracle_cbf("array2")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    NL = n // 2
    assert np.allclose(O["Gc"][:NL, :NL][:cbf.L[0], cbf.L[0]:], 0.0)  # the oracle's B couples no cells
    rng = np.random.default_rng(12)
    y = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    cbfm.cmp_apply(cbf, yt, xt)
    assert _rel(xt.cpu().numpy(), np.linalg.solve(O["Gc"], y.T).T) < 1e-10
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    jt = torch_cuda.zeros((len(w.inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    out = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, use_cmp=True, j_out=jt)
    assert out["status"] == "OK"
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], O["vr"])
    assert _rel(jt.cpu().numpy().T, jref) < 1e-9
    rcs_ref = excitation.monostatic_rcs(m, jref, w.inc, w.k0, w.eta0)
    assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9


def test_translated_cells_share_cbfs_and_offset_blocks(torch_cuda):
    """Two translated copies of one sphere.  The GPU build gives both cells
    one CBF set (identical, still dual in each cell).  With the oracle's
    cell-0 CBFs imported into both cells, the projection fills one block per
    cell offset (three here) and copies it to the pairs sharing that offset;
    against the oracle's dense projection with the same CBFs."""
    from oracle import cbf as ocbf, reduced
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf("array2")
    P = O["P"]
    w, m = P["w"], P["m"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    cb = cbfm.build_cbf(mesh, med, w.gen, 1e-3)
    CM, CJ = cb.export()
    assert np.array_equal(cb.L, [cb.L[0]] * 2) and np.array_equal(CM[0], CM[1]) and np.array_equal(CJ[0], CJ[1])
    for c, ix in enumerate(O["cb"].cells):  # still dual CBFs of each cell: (C^M)^H G C^J = Sigma
        D = CM[c].conj().T @ O["G"][np.ix_(ix, ix)] @ CJ[c]
        assert np.abs(D - np.diag(np.diag(D))).max() < 1e-9 * np.abs(D).max()
    cm0, cj0, s0 = O["cb"].CM[0], O["cb"].CJ[0], O["cb"].sigma[0]
    shared = cbfm.cbf_import(mesh, [cm0, cm0], [cj0, cj0], [s0, s0])
    n = shared.n_cbf
    Zr = torch_cuda.zeros((n, n + 2), dtype=torch_cuda.complex128, device="cuda")
    groups = cbfm.project(mesh, med, shared, Zr, cbfm.FP64, ldz=n + 2, panel_bytes=0)
    sets = ocbf.CBFSet(O["cb"].cells, [cm0, cm0], [cj0, cj0], [s0, s0], O["cb"].sigma_all)
    CJM, CMJ = reduced.cbf_matrices(sets, m.ne)
    ref = reduced.project(P["Z"], CJM, CMJ)
    got = Zr.cpu().numpy()[:, :n]
    err, ee = _rel(got, ref), np.abs(got - ref).max() / np.abs(ref).max()
    print("translated projection rel err", err, "elementwise", ee, "offset groups", groups)
    assert err < 1e-10 and ee < 1e-10


@pytest.mark.parametrize("name", ["c1", "cyl_small"])
def test_build_cbf_invariants(torch_cuda, name):
    """CBFs are unique only up to unitary mixing inside degenerate singular
    multiplets; compare what is unique: kept counts, singular values, the
    spanned subspaces (when the cut falls in a gap) and the duality
    relation (C^M)^H G_m C^J = Sigma."""
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf(name)
    P = O["P"]
    w, m = P["w"], P["m"]
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    print(f"build_cbf {w.name}", flush=True)
    cb = cbfm.build_cbf(mesh, med, w.gen, 1e-3)
    assert np.array_equal(cb.L, O["cb"].L)
    sig_ref = np.concatenate(O["cb"].sigma)
    assert np.max(np.abs(cb.sigma - sig_ref) / sig_ref.max()) < 1e-10
    CM, CJ = cb.export()
    for c, ix in enumerate(O["cb"].cells):
        G = O["G"][np.ix_(ix, ix)]
        D = CM[c].conj().T @ G @ CJ[c]
        s = O["cb"].sigma[c]
        assert np.abs(D - np.diag(s)).max() < 1e-9 * s[0]
        S = O["cb"].sigma_all[c]
        L = len(s)
        if L < len(S) and S[L] < S[L - 1] * (1 - 1e-6):
            for Cg, Co in ((CM[c], O["cb"].CM[c]), (CJ[c], O["cb"].CJ[c])):
                Q, _ = np.linalg.qr(Co)
                assert np.linalg.norm(Cg - Q @ (Q.conj().T @ Cg)) < 1e-8 * np.linalg.norm(Cg)


def test_solve_parity_and_rcs(torch_cuda):
    """GMRES (tol 1e-12, full Krylov space) on the GPU vs LU of the oracle's
    reduced system with the same CBFs: currents and monostatic RCS."""
    from oracle import excitation, reduced
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    inc = w.inc
    jt = torch_cuda.zeros((len(inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    print("solve", flush=True)
    out = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-12, max_iter=n + 10, restart=n + 10, use_cmp=True, j_out=jt)
    print(out)
    assert out["status"] == "OK"
    vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    jg = jt.cpu().numpy().T
    assert _rel(jg, jref) < 1e-9
    rcs_ref = excitation.monostatic_rcs(m, jref, inc, w.k0, w.eta0)
    assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9
    # bistatic total RCS on a few directions
    dirs = np.array([[0, 0, 1.0], [1, 0, 0], [0, 0.6, 0.8]])
    out2 = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-12, max_iter=n + 10, restart=n + 10, dirs=dirs)
    ref2 = excitation.rcs(m, jref, dirs, w.k0, w.eta0)
    assert np.max(np.abs(out2["rcs"] - ref2) / ref2.max()) < 1e-9
    # an iteration cap below convergence is reported, with the residual reached
    out5 = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-12, max_iter=5, restart=5)
    assert out5["status"] == "E_NOCONV" and np.all(out5["relres"] > 1e-12) and np.all(out5["iters"] == 5)


def test_single_sphere_worked_example_end_to_end(torch_cuda):
    """The paper's single-cell sphere (diameter lambda/3, 960 unknowns, Table I
    waves): GPU CBF build keeps 70 per current (groups l = 1..5), the CMP solve
    converges in far fewer iterations than without it, and currents/RCS match
    the oracle's CBFM with the same 70 CBFs."""
    from oracle import excitation, reduced
    from paper_2111_11058_amd import cbfm
    O = _oracle_cbf("x1_er3", delta=0.0, max_L=70)
    P = O["P"]
    w, m = P["w"], P["m"]
    mesh = cbfm.Mesh(w.V, w.T, None)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    cb = cbfm.build_cbf(mesh, med, w.gen, 0.0, max_L=70)
    assert cb.n_cbf == 140
    n = cb.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cb, Zr, cbfm.FP64)
    a = cbfm.solve(mesh, med, cb, Zr, w.inc, tol=1e-6, max_iter=200, restart=200, use_cmp=True)
    b = cbfm.solve(mesh, med, cb, Zr, w.inc, tol=1e-6, max_iter=200, restart=200, use_cmp=False)
    print("iters CMP", a["iters"], "no CMP", b["iters"])
    assert a["iters"][0] * 2 < b["iters"][0]
    jt = torch_cuda.zeros((1, 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    c = cbfm.solve(mesh, med, cb, Zr, w.inc, tol=1e-12, max_iter=200, restart=200, j_out=jt)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], O["vr"])
    assert c["status"] == "OK"
    assert _rel(jt.cpu().numpy().T, jref) < 1e-8
    # restarted GMRES (restart 3: several cycles) reaches the same solution
    d = cbfm.solve(mesh, med, cb, Zr, w.inc, tol=1e-12, max_iter=2000, restart=3, j_out=jt)
    print("restarted", d)
    assert d["status"] == "OK"
    assert _rel(jt.cpu().numpy().T, jref) < 1e-8


def test_graph_replayed_solve_matches_eager(torch_cuda):
    """Arnoldi chunks captured in a HIP graph and replayed (many replays per
    solve, host reads of the convergence flags between them) give the same
    currents as plain launches; two graph solves in a row, and the mixed form."""
    from oracle import excitation
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    nr, ne2 = len(w.inc), 2 * m.ne
    j0 = torch_cuda.zeros((nr, ne2), dtype=torch_cuda.complex128, device="cuda")
    e = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=j0)
    ref = j0.cpu().numpy()
    for rep in range(2):
        jg = torch_cuda.zeros((nr, ne2), dtype=torch_cuda.complex128, device="cuda")
        g = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=jg, use_graph=True)
        print("graph solve", rep, g["iters"], e["iters"])
        assert g["status"] == "OK" and np.array_equal(g["iters"], e["iters"])
        assert _rel(jg.cpu().numpy(), ref) < 1e-13
        _ = Zr.sum().item()  # eager work between the graph solves
    # a single right-hand side (its own update-pass split and matrix-vector
    # kernel), eager and replayed, against the first column of the batch
    inc1 = np.ascontiguousarray(w.inc[:1])
    j1 = torch_cuda.zeros((1, ne2), dtype=torch_cuda.complex128, device="cuda")
    e1 = cbfm.solve(mesh, med, cbf, Zr, inc1, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=j1)
    assert e1["status"] == "OK" and _rel(j1.cpu().numpy(), ref[:1]) < 1e-9
    j1g = torch_cuda.zeros((1, ne2), dtype=torch_cuda.complex128, device="cuda")
    g1 = cbfm.solve(mesh, med, cbf, Zr, inc1, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=j1g, use_graph=True)
    print("single graph solve", g1["iters"], e1["iters"])
    assert g1["status"] == "OK" and np.array_equal(g1["iters"], e1["iters"])
    assert _rel(j1g.cpu().numpy(), j1.cpu().numpy()) < 1e-13
    # the mixed form: float cycles refined in double, one graph per cycle
    jg = torch_cuda.zeros((nr, ne2), dtype=torch_cuda.complex128, device="cuda")
    g = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-11, max_iter=4 * n, restart=n, j_out=jg, use_graph=True,
                   inner_fp32=True)
    print("mixed graph solve", g)
    assert g["status"] == "OK" and _rel(jg.cpu().numpy(), ref) < 1e-9


def test_compressed_basis_solve(torch_cuda):
    """The compressed-basis form (double arithmetic, Krylov basis stored in
    float, cycles restarted from the double residual): at tol 1e-12 it
    reaches LU of the oracle's reduced system like the plain form, for the
    batch, a single right-hand side (the split update pass) and graph
    replays; at tol 1e-6 its true residual meets the tolerance (a right-hand
    side still above it after the first cycle takes a short second one) in
    about the plain form's iteration count."""
    from oracle import excitation
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    inc = w.inc
    nr, ne2 = len(inc), 2 * m.ne
    vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    rcs_ref = excitation.monostatic_rcs(m, jref, inc, w.k0, w.eta0)
    for graph in (False, True):
        jt = torch_cuda.zeros((nr, ne2), dtype=torch_cuda.complex128, device="cuda")
        out = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-12, max_iter=6 * n, restart=n + 10, j_out=jt,
                         basis_fp32=True, use_graph=graph)
        e, r = _rel(jt.cpu().numpy().T, jref), np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref)
        print("compressed basis, graph", graph, out["iters"], out["relres"], "currents", e, "rcs", r)
        assert out["status"] == "OK" and np.all(out["relres"] <= 1e-12)
        assert e < 1e-9 and r < 1e-9
    j1 = torch_cuda.zeros((1, ne2), dtype=torch_cuda.complex128, device="cuda")
    o1 = cbfm.solve(mesh, med, cbf, Zr, np.ascontiguousarray(inc[:1]), tol=1e-12, max_iter=6 * n, restart=n + 10,
                    j_out=j1, basis_fp32=True)
    e1 = _rel(j1.cpu().numpy().T, jref[:, :1])
    print("compressed basis, one right-hand side", o1["iters"], e1)
    assert o1["status"] == "OK" and e1 < 1e-9
    # tol 1e-6: the true residual meets it, in about the plain form's count
    a = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-6, max_iter=6 * n, restart=n + 10)
    b = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-6, max_iter=6 * n, restart=n + 10, basis_fp32=True)
    print("tol 1e-6 iterations plain", a["iters"], "compressed", b["iters"], "relres", b["relres"])
    assert b["status"] == "OK" and np.all(b["relres"] <= 1e-6)
    assert np.all(b["iters"] <= 1.5 * a["iters"] + 10)
    # forms that do not combine with it
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, inc, basis_fp32=True, inner_fp32=True, raise_noconv=True)
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, inc, basis_fp32=True, cmp_mode=cbfm.CMP_INNER_GMRES, raise_noconv=True)


def test_sstep_solve(torch_cuda):
    """s-step cycles (blocks of 4 or 8 iterations: Newton basis, two block
    Gram-Schmidt and two Cholesky QR passes, Hessenberg columns rebuilt)
    solve the oracle's reduced system like plain cycles: at tol 1e-12 the
    currents match LU (batch and one right-hand side); at tol 1e-6 the true
    residual meets the tolerance, with blocks of 4 in about the plain
    iteration count (the first plain cycle of S + 1 iterations that gives
    the shifts included).  Blocks of 8 break down on this operator (a
    Cholesky pivot vanishes mid-solve; the solve then goes on in plain
    cycles), so only their result is checked."""
    from oracle import excitation
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    inc = w.inc
    vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    plain = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-6, max_iter=6 * n, restart=n + 10)
    for S in (4, 8):
        for sel in (slice(None), slice(0, 1)):
            ii = np.ascontiguousarray(inc[sel])
            jt = torch_cuda.zeros((len(ii), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
            out = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-12, max_iter=6 * n, restart=n + 10, j_out=jt, sstep=S)
            e = _rel(jt.cpu().numpy().T, jref[:, sel])
            print("s-step", S, "right-hand sides", len(ii), out["iters"], out["relres"], e)
            assert out["status"] == "OK" and np.all(out["relres"] <= 1e-12) and e < 1e-9, (S, len(ii))
        b = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-6, max_iter=6 * n, restart=n + 10, sstep=S)
        print("tol 1e-6 iterations plain", plain["iters"], "s-step", S, b["iters"], b["relres"])
        assert b["status"] == "OK" and np.all(b["relres"] <= 1e-6)
        if S == 4:
            assert np.all(b["iters"] <= plain["iters"] + 2 * S + 2)
    # an iteration limit that whole blocks cannot reach (the first cycle
    # of S + 1, two blocks, then 3 iterations in a plain cycle) and a
    # tolerance no solve meets: the solve stops at the limit, unconverged
    # (a right-hand side whose block broke down counts that block out)
    for S in (4, 8):
        lim = S + 1 + 2 * S + 3
        c = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-30, max_iter=lim, restart=n + 10, sstep=S)
        print("s-step", S, "iteration limit", lim, c["iters"], c["relres"], c["status"])
        assert c["status"] == "E_NOCONV" and c["iters"].max() == lim and np.all(c["iters"] <= lim), S
        assert np.all(c["relres"] < 1), S
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, inc, sstep=5, raise_noconv=True)
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, inc, sstep=8, inner_fp32=True, raise_noconv=True)


def test_block_solve(torch_cuda):
    """Block GMRES (the right-hand sides of a group share one Krylov space;
    two block Gram-Schmidt passes with Cholesky QR on a double-double Gram
    matrix, pivoted, dependent directions replaced by random vectors) solves
    the oracle's reduced system.  N_CBF is 200 here, so the automatic groups
    hold 6 right-hand sides (cycles of 32 block iterations).  At tol 1e-12
    the currents match LU for 40 incidences: 30 plane waves one degree apart
    (numerically dependent: their right-hand sides have rank about 12 at
    1e-13), one repeated exactly, 8 random; for 32 of them; for one; and
    for one group of 6 in cycles of 24 block iterations (restarted from the
    true residual;
    cycles of 8 stagnate on this operator).
    At tol 1e-6 the true residual meets the tolerance in fewer block
    iterations than plain GMRES needs iterations.  An iteration limit stops
    the solve there, unconverged."""
    from oracle import excitation
    from synth.configs import random_incidences, sph_dir
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    th = np.deg2rad(np.arange(30.0))
    r, t, _ = sph_dir(th, np.zeros_like(th))
    inc = np.concatenate([np.concatenate([-r, t], axis=1), w.inc[:1], w.inc[:1], random_incidences(8, 29)])
    assert len(inc) == 40
    vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
    sv = np.linalg.svd(vr[:, :30] / np.linalg.norm(vr[:, :30], axis=0), compute_uv=False)
    print("right-hand sides of the 30 plane waves: rank at 1e-13", int((sv > 1e-13 * sv[0]).sum()))
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    for sel, restart in ((slice(None), n), (slice(0, 32), n), (slice(0, 1), n), (slice(0, 6), 24)):
        ii = np.ascontiguousarray(inc[sel])
        jt = torch_cuda.zeros((len(ii), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
        out = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-12, max_iter=2000, restart=restart, j_out=jt, block=True)
        got = jt.cpu().numpy().T
        e = _rel(got, jref[:, sel])
        emax = np.max(np.abs(got - jref[:, sel])) / np.max(np.abs(jref[:, sel]))
        print("block", len(ii), "restart", restart, "iters", out["iters"].max(), "relres", out["relres"].max(),
              "current err", e, emax, flush=True)
        assert out["status"] == "OK" and np.all(out["relres"] <= 1e-12) and e < 1e-9 and emax < 1e-9, (len(ii), restart)
        if len(ii) >= 32:
            assert np.allclose(got[:, 30], got[:, 31], rtol=0, atol=1e-12 * np.abs(got[:, 30]).max())
    ii = np.ascontiguousarray(inc[:32])
    plain = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-6, max_iter=6 * n, restart=n + 10)
    b = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-6, max_iter=400, restart=n, block=True)
    print("tol 1e-6: plain iterations", plain["iters"].max(), "block iterations", b["iters"].max(), b["relres"].max())
    assert b["status"] == "OK" and np.all(b["relres"] <= 1e-6) and b["iters"].max() < plain["iters"].max()
    c = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-30, max_iter=3, restart=n, block=True)
    print("iteration limit 3:", c["iters"], c["status"], c["relres"].max())
    assert c["status"] == "E_NOCONV" and np.all(c["iters"] == 3) and np.all(c["relres"] < 1)
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, ii, block=True, sstep=4, raise_noconv=True)
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, ii, block=True, inner_fp32=True, raise_noconv=True)
    with pytest.raises(RuntimeError):
        cbfm.solve(mesh, med, cbf, Zr, ii, block=33, raise_noconv=True)


def test_block_cycle_matches_the_oracle_minimiser(torch_cuda):
    """One cycle of block GMRES stopped after J block iterations returns, for
    every right-hand side, the minimiser of its residual over the block
    Krylov space K_J(A, B), A = Z_r (G^CBF)^{-1}: against the oracle's
    block Arnoldi and least squares, for groups of 4 (4 and 8 random
    incidences, whose right-hand sides are independent) and J = 2, 6."""
    from oracle import excitation, reduced
    from synth.configs import random_incidences
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    Gi = np.linalg.inv(O["Gc"])
    A = O["Zr"] @ Gi
    for nr in (4, 8):
        inc = random_incidences(nr, 31 + nr)
        vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
        for g0 in range(0, nr, 4):
            sv = np.linalg.svd(vr[:, g0:g0 + 4], compute_uv=False)
            assert sv[-1] > 1e-6 * sv[0]
        for J in (2, 6):
            y = np.concatenate([reduced.block_krylov_minimiser(lambda X: A @ X, vr[:, g0:g0 + 4], J)
                                for g0 in range(0, nr, 4)], axis=1)
            jref = O["CMJ"] @ (Gi @ y)
            jt = torch_cuda.zeros((nr, 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
            out = cbfm.solve(mesh, med, cbf, Zr, inc, tol=1e-30, max_iter=J, restart=n, j_out=jt, block=4)
            got = jt.cpu().numpy().T
            e = _rel(got, jref)
            emax = np.max(np.abs(got - jref)) / np.max(np.abs(jref))
            print(f"block cycle nrhs={nr} J={J}: iters {out['iters']}, current err {e:.2e} {emax:.2e}", flush=True)
            assert out["status"] == "E_NOCONV" and np.all(out["iters"] == J) and e < 1e-9 and emax < 1e-9


def test_every_gemm_launch_shape_solves_alike(torch_cuda, monkeypatch):
    """Every launch shape of the complex GEMM (CBFM_GEMM_SHAPE forces it on
    each product it applies to; the tuner may pick any of them for the
    GMRES matrix-vector product): four tiles per block, K split over 4 or 8
    wavefronts, wide tiles of 2 or 4 column blocks, K split over 5
    wavefronts, over 3 wavefronts x 2 blocks and 2 wavefronts x 3 blocks
    (partial tiles added by a second kernel), the vector-unit
    matrix-vector kernel (a single right-hand side), and the row-block
    kernel (64 rows x 32 columns per block, K split so that 2 or 3 blocks
    per compute unit hold the launch; partial tiles added by the second
    kernel).  Each solve, at tol 1e-12 with the full Krylov space, matches
    LU of the oracle's reduced system."""
    from oracle import excitation
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    inc = w.inc
    vr = O["CJM"].conj().T @ excitation.rhs(m, inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    for shape in range(11):
        monkeypatch.setenv("CBFM_GEMM_SHAPE", str(shape))
        for sel in (slice(None), slice(0, 1)):
            ii = np.ascontiguousarray(inc[sel])
            jt = torch_cuda.zeros((len(ii), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
            out = cbfm.solve(mesh, med, cbf, Zr, ii, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=jt)
            e = _rel(jt.cpu().numpy().T, jref[:, sel])
            print("GEMM shape", shape, "right-hand sides", len(ii), out["iters"], e)
            assert out["status"] == "OK" and e < 1e-9, (shape, len(ii))
    monkeypatch.delenv("CBFM_GEMM_SHAPE")


def test_batched_projection_matches_single(torch_cuda):
    """Several scatterers (own sizes and media) through one persistent fill
    launch and batched GEMMs give each one's Z_r as cbfm_project does, and
    the FP64 oracle's."""
    from paper_2111_11058_amd import cbfm
    names = ["c1", "cyl_small"]
    Os = [_oracle_cbf(nm) for nm in names]
    hs = [_gpu_handles(O["P"]["w"], O) for O in Os]
    for prec, tol in ((cbfm.FP64, 1e-13), (cbfm.MIXED_FP32, 1e-5)):
        items, singles = [], []
        for (cb_, mesh, med, cbf), O in zip(hs, Os):
            n = cbf.n_cbf
            zb = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
            zs = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
            cbfm.project(mesh, med, cbf, zs, prec)
            items.append((mesh, med, cbf, zb))
            singles.append(zs)
        print("batched projection", prec, flush=True)
        cbfm.project_batch(items, prec)
        for (mesh, med, cbf, zb), zs, O in zip(items, singles, Os):
            e = _rel(zb.cpu().numpy(), zs.cpu().numpy())
            print("batch vs single", e)
            assert e < tol
            if prec == cbfm.FP64:
                assert _rel(zb.cpu().numpy(), O["Zr"]) < 1e-10


def test_inexact_cmp_and_flexible_gmres(torch_cuda):
    """The paper's inexact CMP through the C ABI: cmp_apply_ex with the inner
    GMRES (D^CBF preconditioner) meets its allowance against the oracle's
    G^CBF and reaches the exact inverse as the allowance goes to 0; the
    reduced solve with the inexact CMP inside flexible GMRES reaches the LU
    solution, and at the paper's 1e-5 inner allowance converges in about the
    iterations of the exact CMP and of the oracle's flexible GMRES."""
    from oracle import reduced
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    from synth import configs
    y = configs.random_complex((2, n), 32)
    yt = torch_cuda.tensor(y, dtype=torch_cuda.complex128, device="cuda")
    xt = torch_cuda.empty_like(yt)
    Gc = O["Gc"]
    xe = np.linalg.solve(Gc, y.T).T
    cbfm.cmp_apply(cbf, yt, xt, mode=cbfm.CMP_INNER_GMRES, inner_tol=1e-13)
    e0 = _rel(xt.cpu().numpy(), xe)
    cbfm.cmp_apply(cbf, yt, xt, mode=cbfm.CMP_INNER_GMRES, inner_tol=1e-5)
    x5 = xt.cpu().numpy()
    res5 = np.linalg.norm(x5 @ Gc.T - y, axis=1) / np.linalg.norm(y, axis=1)
    print("inner CMP: allowance 1e-13 error", e0, "allowance 1e-5 residuals", res5)
    assert e0 < 1e-9 and np.all(res5 <= 1e-5)
    Zr = torch_cuda.tensor(O["Zr"], dtype=torch_cuda.complex128, device="cuda")
    jt = torch_cuda.zeros((len(w.inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    out = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=jt,
                     cmp_mode=cbfm.CMP_INNER_GMRES, cmp_inner_tol=1e-10)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], O["vr"])
    print("flexible GMRES, inner 1e-10:", out["iters"], out["status"])
    assert out["status"] == "OK" and _rel(jt.cpu().numpy().T, jref) < 1e-9
    ex = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-6, max_iter=n + 10, restart=n + 10)
    inx = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-6, max_iter=n + 10, restart=n + 10, j_out=jt,
                     cmp_mode=cbfm.CMP_INNER_GMRES, cmp_inner_tol=1e-5)
    ora = [reduced.fgmres(lambda u: O["Zr"] @ u, lambda q: reduced.cmp_inner(Gc, q, 1e-5)[:, 0], O["vr"][:, c], 1e-6,
                          n + 10, n + 10)[1] for c in range(O["vr"].shape[1])]
    print("iterations to 1e-6: exact CMP", ex["iters"], "inexact (GPU)", inx["iters"], "inexact (oracle)", ora)
    assert inx["status"] == "OK" and np.all(inx["relres"] <= 1e-6)
    assert np.all(np.abs(inx["iters"] - np.array(ora)) <= 2) and np.all(inx["iters"] <= ex["iters"] + 5)
    assert _rel(jt.cpu().numpy().T, jref) < 1e-4
