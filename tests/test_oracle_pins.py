"""Pins of the CPU oracle against things the paper and the mathematics fix
(closed forms, brute force on tiny inputs, invariants, the Mie series, and
the paper's single-sphere worked example).  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from conftest import oracle_problem
from oracle import cbf, excitation, fill, mesh, mie, potentials, quadrature, reduced
from synth import configs
from synth.blocks import octant_blocks, rcb_blocks
from synth.meshes import cube, cylinder, edges_canonical, icosphere

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- quadrature
def test_quadrature_degree5_exact_degree6_not():
    """int over the unit right triangle of x^a y^b = a! b! / (a+b+2)!."""
    tri = np.array([[[0.0, 0, 0], [1, 0, 0], [0, 1, 0]]])
    p = quadrature.points(tri)[0]
    w = quadrature.WEIGHTS * 0.5
    worst5 = 0.0
    for a in range(7):
        for b in range(7 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = (w * p[:, 0] ** a * p[:, 1] ** b).sum()
            err = abs(got - exact) / exact
            if a + b <= 5:
                worst5 = max(worst5, err)
            elif a + b == 6 and a == 6:
                assert err > 1e-6
    assert worst5 < 1e-13
    assert abs(quadrature.WEIGHTS.sum() - 1) < 1e-15


# ---------------------------------------------------------------- potentials
TRI = np.array([[0.0, 0, 0], [1.0, 0.1, 0], [0.3, 0.8, 0.05]])


def _brute(r):
    v0, v1, v2 = TRI
    A2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0))

    def I(fun):
        return integrate.dblquad(lambda t, s: fun(v0 + s * (v1 - v0) + t * (v2 - v0)) * A2,
                                 0, 1, 0, lambda s: 1 - s, epsabs=1e-13, epsrel=1e-12)[0]

    R = lambda p: np.linalg.norm(r - p)
    return dict(
        Im1=I(lambda p: 1 / R(p)), I1=I(lambda p: R(p)),
        Vm1=np.array([I(lambda p, i=i: (p - r)[i] / R(p)) for i in range(3)]),
        V1=np.array([I(lambda p, i=i: (p - r)[i] * R(p)) for i in range(3)]),
        Gm3=np.array([I(lambda p, i=i: (r - p)[i] / R(p) ** 3) for i in range(3)]))


@pytest.mark.parametrize("r", [[0.4, 0.3, 0.5], [0.4, 0.3, -0.05], [2.0, -1.0, 0.3],
                               [1.5, 0.15, 0.0], [0.4, 0.3, 0.01]],
                         ids=["above", "below-near", "far", "in-plane-outside", "very-near"])
def test_potentials_vs_adaptive_quadrature(r):
    r = np.array(r)
    a = potentials.triangle_potentials(r, TRI)
    b = _brute(r)
    for key in b:
        err = np.max(np.abs(a[key] - b[key])) / np.max(np.abs(b[key]))
        assert err < 1e-9, (key, err)


# ---------------------------------------------------------------- meshes, RWG
@pytest.mark.parametrize("gen", [lambda: icosphere(2, 0.5), lambda: cube(4), lambda: cylinder(2, 4, 0.3, 0.8)])
def test_mesh_closed_oriented(gen):
    V, T = gen()
    m = mesh.build(V, T)
    assert len(V) - m.ne + m.nt == 2                    # Euler characteristic
    assert 3 * m.nt == 2 * m.ne                         # unknowns 2 ne = 3 nt
    assert np.array_equal(m.edges, edges_canonical(T))
    vol = np.einsum("ij,ij->i", m.xyz[:, 0], np.cross(m.xyz[:, 1], m.xyz[:, 2])).sum() / 6
    assert vol > 0                                      # outward orientation
    # RWG: total divergence over T+ and T- cancels (charge neutrality)
    for e in range(0, m.ne, 7):
        p, q = m.tplus[e], m.tminus[e]
        ap, aq = m.aplus[e], m.aminus[e]
        flux = (m.tri_sign[p, ap] * m.length[e] / m.area[p]) * m.area[p] + \
               (m.tri_sign[q, aq] * m.length[e] / m.area[q]) * m.area[q]
        assert abs(flux) < 1e-14
        # normal current continuity across the edge: f . n_edge equal on both sides
        a, b = m.V[m.edges[e, 0]], m.V[m.edges[e, 1]]
        mid = (a + b) / 2
        for t, loc in ((p, ap), (q, aq)):
            pass
        fp = m.tri_sign[p, ap] * m.length[e] / (2 * m.area[p]) * (mid - m.xyz[p, ap])
        fq = m.tri_sign[q, aq] * m.length[e] / (2 * m.area[q]) * (mid - m.xyz[q, aq])
        np_ = np.cross(b - a, m.normal[p])
        nq_ = np.cross(b - a, m.normal[q])
        assert abs(fp @ np_ / np.linalg.norm(np_) - fq @ nq_ / np.linalg.norm(nq_)) < 1e-12


def test_counts_match_paper():
    """320-triangle sphere -> 960 unknowns (Sec. IV-A); arrays 32 x 960 and
    256 x 960 unknowns (Sec. IV-A array examples)."""
    V, T = icosphere(2, 1 / 6)
    m = mesh.build(V, T)
    assert 2 * m.ne == 960
    assert 32 * 2 * m.ne == 30720 and 256 * 2 * m.ne == 245760


def test_cells_partition_edges():
    V, T = cube(12)
    b = rcb_blocks(V, T, 27)
    assert len(np.unique(b)) == 27 and np.bincount(b).min() > 0
    V, T = icosphere(2, 0.5)
    assert len(np.unique(octant_blocks(V, T))) == 8


# ---------------------------------------------------------------- Gram matrix
def test_rwg_gram_closed_form():
    """int_T (n x f_a) . f_b = eps_ab l_a l_b / 6 (eps = +1 for (a, b) cyclic,
    -1 anticyclic, 0 on the diagonal) times the RWG signs, summed over the
    two triangles; G is real and antisymmetric (the paper notes G_ffff is
    singular)."""
    V, T = icosphere(1, 0.4)
    m = mesh.build(V, T)
    G = cbf.rwg_gram(m)
    ref = np.zeros_like(G)
    eps = np.array([[0, 1, -1], [-1, 0, 1], [1, -1, 0]], dtype=float)
    for t in range(m.nt):
        L = m.length[m.tri_edge[t]]
        s = m.tri_sign[t]
        for a in range(3):
            for b in range(3):
                ref[m.tri_edge[t, a], m.tri_edge[t, b]] += eps[a, b] * L[a] * L[b] / 6 * s[a] * s[b]
    assert np.abs(G - ref).max() < 1e-15 * np.abs(ref).max() * 10
    assert np.abs(G + G.T).max() < 1e-16
    assert np.linalg.matrix_rank(G) < m.ne             # singular


# ---------------------------------------------------------------- fill
def test_extraction_matches_plain_rule_on_separated_pair():
    """On a well-separated pair the singularity-subtracted route and the plain
    7x7 rule evaluate the same integrals; they must agree to quadrature
    error.  A dropped or mis-signed term in the extraction breaks this."""
    V, T = icosphere(2, 0.5)
    m = mesh.build(V, T)
    k, _ = fill.media(2 * np.pi, configs.ETA0, 4.0 - 0.3j, 1.0)
    c = m.xyz.mean(axis=1)
    p = 0
    d = np.linalg.norm(c - c[p], axis=1)
    h = np.linalg.norm(m.xyz[p, 1] - m.xyz[p, 0])
    q = int(np.argmin(np.abs(d - 4 * h)))
    Kr, Tr = fill.regular_local(m, k, np.array([p]), np.array([q]))
    Kn, Tn = fill.near_local(m, k, p, q)
    assert np.abs(Kn - Kr[0]).max() < 1e-4 * np.abs(Kr[0]).max()
    assert np.abs(Tn - Tr[:, 0]).max() < 1e-5 * np.abs(Tr[:, 0]).max()


def test_inner_integral_extraction_vs_brute_force():
    """Inner integral int_Q G(r, r') (r' - q) dS' and int_Q grad'G x (r'-q)
    for an observation point close to Q: extraction + 7-point remainder vs
    adaptive quadrature of the full kernel."""
    Q = np.array([[0.0, 0, 0], [0.1, 0, 0], [0.02, 0.09, 0.0]])
    r = np.array([0.05, 0.03, 0.02])
    k = 2 * np.pi * 2.0
    A2 = np.linalg.norm(np.cross(Q[1] - Q[0], Q[2] - Q[0]))

    def I(fun):
        return integrate.dblquad(lambda t, s: fun(Q[0] + s * (Q[1] - Q[0]) + t * (Q[2] - Q[0])) * A2,
                                 0, 1, 0, lambda s: 1 - s, epsabs=1e-14, epsrel=1e-11)[0]

    def G(p):
        R = np.linalg.norm(r - p)
        return np.exp(-1j * k * R) / (4 * np.pi * R)

    def cI(fun):
        return I(lambda p: fun(p).real) + 1j * I(lambda p: fun(p).imag)

    ref0 = cI(G)
    ref1 = np.array([cI(lambda p, i=i: G(p) * p[i]) for i in range(3)])
    pot = potentials.triangle_potentials(r, Q)
    rq = quadrature.points(Q[None])[0]
    R = np.linalg.norm(r - rq, axis=1)
    A = A2 / 2
    Gr = fill._Gr(k, R)
    J0 = (pot["Im1"] - 0.5 * k * k * pot["I1"]) / (4 * np.pi) + A * (Gr * quadrature.WEIGHTS).sum()
    J1 = ((pot["Vm1"] + r * pot["Im1"]) - 0.5 * k * k * (pot["V1"] + r * pot["I1"])) / (4 * np.pi) \
        + A * (Gr * quadrature.WEIGHTS) @ rq
    assert abs(J0 - ref0) < 1e-4 * abs(ref0)
    assert np.abs(J1 - ref1).max() < 1e-4 * np.abs(ref1).max()

    def g(p):
        R = np.linalg.norm(r - p)
        return -(1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)

    refV = np.array([cI(lambda p, i=i: g(p) * (r - p)[i]) for i in range(3)])
    Vs = -(pot["Gm3"] - 0.5 * k * k * pot["Vm1"]) / (4 * np.pi)
    V = Vs + A * (fill._gr(k, R) * quadrature.WEIGHTS) @ (r - rq)
    assert np.abs(V - refV).max() < 1e-4 * np.abs(refV).max()


def test_symmetry_and_coplanar_zero():
    """Reciprocity: far-pair blocks of K and T are symmetric to rounding
    (same 7x7 rule both ways); K vanishes on coplanar near pairs."""
    w = configs.small_cylinder()
    m = mesh.build(w.V, w.T)
    k, _ = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    K, T = fill.local_blocks(m, k)
    near = mesh.near_pairs(m)
    isn = np.zeros((m.nt, m.nt), bool)
    isn[near[:, 0], near[:, 1]] = True
    for X in (K, T[0], T[1]):
        Xt = X.transpose(1, 0, 3, 2)
        d = np.abs(X - Xt)[~isn].max()
        assert d < 1e-13 * np.abs(X).max()
    ncop = 0
    for p, q in near:
        if mesh.coplanar(m, p, q):
            assert np.all(K[p, q] == 0)
            ncop += 1
    assert ncop > m.nt  # caps and side rows give many coplanar pairs


def test_mie_sphere_c1_and_refinement():
    """MoM with the paper's operators vs the Mie series: the 320-triangle
    eps_r = 4 sphere of radius 0.5 agrees at the discretisation level (a
    wrong operator sign gives O(1) errors), and the error shrinks when the
    mesh is refined (80 -> 320 triangles on a smaller sphere)."""
    P = oracle_problem("c1")
    m, w = P["m"], P["w"]
    j = np.linalg.solve(P["Z"], P["v"])
    th = np.deg2rad(np.arange(0, 181, 2.0))
    dE = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    dH = np.stack([0 * th, np.sin(th), np.cos(th)], 1)
    sE = excitation.rcs(m, j, dE, w.k0, w.eta0)[0]
    sH = excitation.rcs(m, j, dH, w.k0, w.eta0)[0]
    mE, mH = mie.bistatic_rcs(0.5, w.k0, w.eps_r, np.pi - th)
    eE = np.linalg.norm(sE - mE) / np.linalg.norm(mE)
    eH = np.linalg.norm(sH - mH) / np.linalg.norm(mH)
    assert eE < 0.15 and eH < 0.12, (eE, eH)
    errs = []
    for level in (1, 2):
        V, T = icosphere(level, 0.25)
        mm = mesh.build(V, T)
        k, eta = fill.media(2 * np.pi, configs.ETA0, 2.0, 1.0)
        Kc, TE, TH = fill.combine(*fill.fill_ops(mm, k), eta)
        v = excitation.rhs(mm, np.array([[0, 0, -1, 1, 0, 0.0]]), 2 * np.pi, configs.ETA0)
        jj = np.linalg.solve(fill.assemble_Z(Kc, TE, TH), v)
        s = excitation.rcs(mm, jj, dE, 2 * np.pi, configs.ETA0)[0]
        ref, _ = mie.bistatic_rcs(0.25, 2 * np.pi, 2.0, np.pi - th)
        errs.append(np.linalg.norm(s - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.6 * errs[0], errs


def test_mie_lossless_optical_theorem():
    """Independent check of the Mie code itself: for a lossless sphere the
    extinction from the forward amplitude equals the integrated scattering."""
    x, mrel = 2.0, np.sqrt(3.0)
    a, b = mie.coefficients(x, mrel)
    n = np.arange(1, len(a) + 1)
    qext = 2 / x ** 2 * ((2 * n + 1) * (a + b).real).sum()
    qsca = 2 / x ** 2 * ((2 * n + 1) * (abs(a) ** 2 + abs(b) ** 2)).sum()
    assert abs(qext - qsca) < 1e-12 * qsca
    S1, S2 = mie.amplitudes(x, mrel, np.array([0.0]))
    assert abs(S1[0] - S2[0]) < 1e-12 * abs(S1[0])
    assert abs(4 / x ** 2 * S1[0].real - qext) < 1e-10 * qext


def test_transparent_sphere_scatters_nothing():
    """eps_r = mu_r = 1: the scattered far field vanishes to discretisation
    level."""
    V, T = icosphere(2, 0.5)
    m = mesh.build(V, T)
    inc = np.array([[0, 0, -1, 1, 0, 0.0]])
    th = np.deg2rad(np.arange(0, 181, 10.0))
    d = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    out = {}
    for er in (1.0, 4.0):
        k, eta = fill.media(2 * np.pi, configs.ETA0, er, 1.0)
        Kc, TE, TH = fill.combine(*fill.fill_ops(m, k), eta)
        j = np.linalg.solve(fill.assemble_Z(Kc, TE, TH), excitation.rhs(m, inc, 2 * np.pi, configs.ETA0))
        out[er] = excitation.rcs(m, j, d, 2 * np.pi, configs.ETA0)[0]
    assert out[1.0].max() < 1e-3 * out[4.0].max()


# ---------------------------------------------------------------- CBFs, reduced system
def test_x1_singular_value_groups_and_cmp():
    """The paper's single-sphere worked example: the normalised singular
    values of G' fall in groups of 2(2l+1) (largest log-gaps after 6, 16, 30,
    48, 70); with the first 70 kept, G^CBF is diagonal, the duality relation
    holds, the CMP solve converges in far fewer iterations than the
    unpreconditioned one and reproduces the MoM currents."""
    rows = np.loadtxt(os.path.join(GOLDEN, "x1_singular_value_groups.txt"))
    cum = rows[:, 2].astype(int)
    P = oracle_problem("x1_er3")
    m = P["m"]
    JM, JJ = cbf.primary_currents(m, P["Kc"], P["TE"], P["TH"], np.arange(m.ne),
                                  P["w"].gen, P["w"].k0, P["w"].eta0)
    G = cbf.rwg_gram(m)
    CM, CJ, S, Sall = cbf.dual_cbfs(JM, JJ, G, 0.0)
    lr = np.log10(Sall[:80] / Sall[0])
    gaps = lr[:-1] - lr[1:]
    for c in cum:
        # the boundary after each cumulative count is a gap of > 1 decade
        assert gaps[c - 1] > 1.0, (c, gaps[c - 1])
    L = int(cum[-1])
    cb = cbf.CBFSet([np.arange(m.ne)], [CM[:, :L]], [CJ[:, :L]], [S[:L]], [Sall])
    D = CM[:, :L].conj().T @ G @ CJ[:, :L]
    assert np.abs(D - np.diag(S[:L])).max() < 1e-12 * S[0]
    assert np.all(S[:L] > 0)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    assert CJM.shape[1] == 140
    Zr = reduced.project(P["Z"], CJM, CMJ)
    Gc = reduced.gram_cbf(G, CJM, CMJ)
    # G^CBF = blkdiag(-S, +S) for one closed body per cell
    ref = np.diag(np.concatenate([-S[:L], S[:L]]))
    assert np.abs(Gc - ref).max() < 1e-12 * S[0]
    vr = CJM.conj().T @ P["v"]
    jc, its, _ = reduced.solve_reduced(Zr, Gc, vr, 1e-6)
    _, its0, _ = reduced.solve_reduced(Zr, np.eye(len(Zr)), vr, 1e-6)
    assert its[0] * 2 < its0[0], (its, its0)
    j = np.linalg.solve(P["Z"], P["v"])
    assert np.linalg.norm(CMJ @ jc - j) / np.linalg.norm(j) < 1e-3


def test_gmres_equals_lu_and_cbf_invariance():
    """GMRES to 1e-12 reproduces the LU solution of the reduced system; the
    reduced solution's currents do not depend on the column order or phase
    of the generating solutions (C = J U is invariant)."""
    P = oracle_problem("cyl_small")
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, 1e-3)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    Gc = reduced.gram_cbf(cbf.rwg_gram(m), CJM, CMJ)
    vr = CJM.conj().T @ P["v"]
    jc, its, _ = reduced.solve_reduced(Zr, Gc, vr, 1e-12, restart=400, max_iter=400)
    jlu = np.linalg.solve(Zr, vr)
    assert np.linalg.norm(jc - jlu) < 1e-9 * np.linalg.norm(jlu)
    # permute + rephase the generating waves
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(w.gen))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, len(w.gen)))
    cell = cb.cells[0]
    JM, JJ = cbf.primary_currents(m, P["Kc"], P["TE"], P["TH"], cell, w.gen, w.k0, w.eta0)
    G = cbf.rwg_gram(m)[np.ix_(cell, cell)]
    CM1, CJ1, S1, _ = cbf.dual_cbfs(JM, JJ, G, 1e-3)
    CM2, CJ2, S2, _ = cbf.dual_cbfs(JM[:, perm] * ph[perm], JJ[:, perm] * ph[perm], G, 1e-3)
    assert np.allclose(S1, S2, rtol=1e-10, atol=1e-12 * S1[0])
    # same span: projector onto span(CM1) reproduces CM2
    Qm, _ = np.linalg.qr(CM1)
    assert np.linalg.norm(CM2 - Qm @ (Qm.conj().T @ CM2)) < 1e-8 * np.linalg.norm(CM2)


# ------------------------------------------------------- block forms of the oracle
def test_block_forms_equal_the_dense_definitions():
    """The block routines that let large meshes be sampled cheaply agree with
    the dense definitions on the c1 sphere: fill_block with the sub-block of
    fill_ops (ragged row and column sets, near and far pairs), the sparse
    RWG Gram with the dense one, G^CBF = blkdiag(-B^H, B) from the cell-pair
    form of B (G real antisymmetric), cmp_solve with a dense solve of G^CBF,
    and project_block with the blocks of the dense projection."""
    P = oracle_problem("c1")
    m, w = P["m"], P["w"]
    rows = np.array([0, 5, 77, 200, 479])
    cols = np.array([3, 4, 150, 151, 300, 478])
    got = fill.fill_block(m, P["k"], rows, cols)
    for X, R_ in zip(got, (P["Kop"], P["T1"], P["T2"])):
        ref = R_[np.ix_(rows, cols)]
        assert np.abs(X - ref).max() <= 1e-13 * np.abs(ref).max()
    G = cbf.rwg_gram(m)
    Gs = cbf.rwg_gram_sparse(m)
    assert np.abs(Gs.toarray() - G).max() <= 1e-15 * np.abs(G).max()
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, 1e-3)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Gc = reduced.gram_cbf(G, CJM, CMJ)
    B = reduced.gram_b(Gs, cb)
    NL = B.shape[0]
    assert np.abs(Gc[NL:, NL:] - B).max() <= 1e-13 * np.abs(B).max()
    assert np.abs(Gc[:NL, :NL] + B.conj().T).max() <= 1e-13 * np.abs(B).max()
    assert np.abs(Gc[:NL, NL:]).max() == 0 and np.abs(Gc[NL:, :NL]).max() == 0
    y = configs.random_complex((2 * NL, 2), 3)
    assert np.linalg.norm(reduced.cmp_solve(B, y) - np.linalg.solve(Gc, y)) <= 1e-12 * np.linalg.norm(
        np.linalg.solve(Gc, y))
    Zr = reduced.project(P["Z"], CJM, CMJ)
    off = np.concatenate([[0], np.cumsum(cb.L)])
    for a, b in ((0, 0), (2, 5)):
        ia, ib = cb.cells[a], cb.cells[b]
        blk = reduced.project_block(P["Kc"][np.ix_(ia, ib)], P["TE"][np.ix_(ia, ib)], P["TH"][np.ix_(ia, ib)],
                                    cb.CM[a], cb.CJ[a], cb.CM[b], cb.CJ[b])
        ra = np.r_[off[a]:off[a + 1], NL + off[a]:NL + off[a + 1]]
        cbix = np.r_[off[b]:off[b + 1], NL + off[b]:NL + off[b + 1]]
        ref = Zr[np.ix_(ra, cbix)]
        assert np.abs(blk - ref).max() <= 1e-12 * np.abs(ref).max()
    # dual CBFs from given currents: the primary currents reproduce build()
    cur = [cbf.primary_currents(m, P["Kc"], P["TE"], P["TH"], ix, w.gen, w.k0, w.eta0) for ix in cb.cells]
    cb2 = cbf.dual_from_currents(m, w.edge_block, cur, 1e-3)
    for s1, s2 in zip(cb.sigma, cb2.sigma):
        assert len(s1) == len(s2) and np.abs(s1 - s2).max() <= 1e-12 * s1[0]


# ------------------------------------------------ MoM arrangement, IPCBF, T-diagonal
def test_mom_arrangement_gmres_equals_lu():
    """GMRES on Z_t D^{-1} (the MoM arrangement with the diagonal
    preconditioner) to 1e-12 reaches the LU solution of Z, reordered, and
    needs fewer iterations than GMRES on Z_t itself; the residual history
    falls below each looser allowance at the reported iteration."""
    from oracle import mom
    P = oracle_problem("c1")
    Zt = mom.mom_t_matrix(P["Kc"], P["TE"], P["TH"])
    ne = P["m"].ne
    # the arrangement is Z with its two column blocks swapped
    assert np.array_equal(Zt[:, :ne], P["Z"][:, ne:]) and np.array_equal(Zt[:, ne:], P["Z"][:, :ne])
    ref = np.linalg.solve(P["Z"], P["v"])
    j, its, hists = mom.mom_t_solve(Zt, P["v"], 1e-12, 2 * ne, 2 * ne)
    assert np.linalg.norm(j - ref) <= 1e-9 * np.linalg.norm(ref)
    _, its_plain, _ = reduced.gmres(lambda y: Zt @ y, P["v"][:, 0], 1e-6, 2 * ne, 2 * ne)
    _, its_diag, _ = mom.mom_t_solve(Zt, P["v"], 1e-6, 2 * ne, 2 * ne)
    assert its_diag[0] < its_plain
    j2, its2, _ = mom.mom_t_solve(Zt, P["v"], 1e-2, 2 * ne, 2 * ne)
    res = np.linalg.norm(P["v"] - P["Z"] @ j2) / np.linalg.norm(P["v"])
    assert res <= 1e-2 and abs(res - hists[0][its2[0]]) <= 1e-8


def test_ipcbf_limits_and_invariances():
    """IPCBF currents (Sec. III-A, GMRES version): (1) as delta_r -> 0 they
    are the MoM solutions of the generating waves restricted to each cell;
    (2) with delta_SVD = 0 the CBFM on those CBFs reproduces the MoM
    solution of a generating incidence (it lies in the CBF span); (3) the
    kept singular values do not depend on the order of the waves; (4) at a
    loose delta_r every wave's residual is within delta_r."""
    from oracle import mom
    P = oracle_problem("cyl_small")
    w, m = P["w"], P["m"]
    ne = m.ne
    Zt = mom.mom_t_matrix(P["Kc"], P["TE"], P["TH"])
    gen = w.gen[::12][:10]
    Vg = excitation.rhs(m, gen, w.k0, w.eta0)
    cur, its = mom.ipcbf_currents(Zt, Vg, w.edge_block, 1e-12, max_iter=2 * ne)
    exact = np.linalg.solve(P["Z"], Vg)
    for c in range(w.nblocks):
        ix = np.nonzero(w.edge_block == c)[0]
        JM, JJ = cur[c]
        assert np.linalg.norm(JM - exact[:ne][ix]) <= 1e-9 * np.linalg.norm(exact[:ne][ix])
        assert np.linalg.norm(JJ - exact[ne:][ix]) <= 1e-9 * np.linalg.norm(exact[ne:][ix])
    cb = cbf.dual_from_currents(m, w.edge_block, cur, 0.0, G=cbf.rwg_gram(m))
    CJM, CMJ = reduced.cbf_matrices(cb, ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    jc = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ Vg[:, [3]])
    assert np.linalg.norm(jc[:, 0] - exact[:, 3]) <= 1e-7 * np.linalg.norm(exact[:, 3])
    perm = np.random.default_rng(4).permutation(len(gen))
    cur2, _ = mom.ipcbf_currents(Zt, Vg[:, perm], w.edge_block, 1e-12, max_iter=2 * ne)
    cb2 = cbf.dual_from_currents(m, w.edge_block, cur2, 0.0, G=cbf.rwg_gram(m))
    for s1, s2 in zip(cb.sigma, cb2.sigma):
        assert np.abs(np.sort(s1) - np.sort(s2)).max() <= 1e-9 * s1.max()
    curl, itl = mom.ipcbf_currents(Zt, Vg, w.edge_block, 1e-2, max_iter=2 * ne)
    J = np.zeros((2 * ne, len(gen)), complex)
    for c in range(w.nblocks):
        ix = np.nonzero(w.edge_block == c)[0]
        J[ix], J[ne + ix] = curl[c]
    res = np.linalg.norm(Vg - P["Z"] @ J, axis=0) / np.linalg.norm(Vg, axis=0)
    assert np.all(res <= 1e-2) and max(itl) < min(its)


def test_t_diagonal_cbfm_is_the_column_swapped_reduced_matrix():
    """(C^JM)^H Z_t C^JM equals Z_r = (C^JM)^H Z C^MJ with its two column
    halves swapped, so the T-diagonal CBFM reaches the same currents as the
    K-diagonal one (GMRES 1e-12 against LU)."""
    from oracle import mom
    P = oracle_problem("c1")
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, 1e-3)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    Zt = mom.mom_t_matrix(P["Kc"], P["TE"], P["TH"])
    Ztr = mom.t_diagonal_operator(Zt, CJM)
    NL = Zr.shape[0] // 2
    sw = np.r_[NL:2 * NL, 0:NL]
    assert np.abs(Ztr - Zr[:, sw]).max() <= 1e-12 * np.abs(Zr).max()
    vr = CJM.conj().T @ P["v"][:, 0]
    y, it, _ = reduced.gmres(lambda u: Ztr @ u, vr, 1e-12, 2 * NL, 2 * NL)
    j_t = CJM @ y
    j = np.concatenate([j_t[m.ne:], j_t[:m.ne]])
    jref = CMJ @ np.linalg.solve(Zr, vr)
    assert np.linalg.norm(j - jref) <= 1e-9 * np.linalg.norm(jref)


def test_rmse_closed_forms():
    """RMSE (Sec. IV-A): a constant offset delta over a range R gives
    10 log10(delta / R); a scaled error scales inside the log."""
    from oracle import mom
    sm = np.linspace(1.0, 5.0, 31)
    assert abs(mom.rmse_db(sm + 0.04, sm) - 10 * np.log10(0.01)) < 1e-12
    e = np.sin(np.arange(31.0))
    assert abs(mom.rmse_db(sm + 2 * e, sm) - mom.rmse_db(sm + e, sm) - 10 * np.log10(2)) < 1e-12


def test_media_apart_sum_to_the_combined_fill():
    """K1 and K2 filled apart (one medium each) sum to the fill of both
    media, and T1, T2 are the combined fill's (the K operator is linear in
    the media's kernels g_i)."""
    P = oracle_problem("c1")
    K1, K2, T1, T2 = fill.fill_media(P["m"], P["k"])
    assert np.abs(K1 + K2 - P["Kop"]).max() <= 1e-13 * np.abs(P["Kop"]).max()
    assert np.array_equal(T1, P["T1"]) and np.array_equal(T2, P["T2"])
    assert np.abs(K1 - K2).max() > 1e-3 * np.abs(K1).max()  # the media differ


def test_inexact_cmp_and_flexible_gmres():
    """The inexact inner CMP (GMRES with D^CBF) reaches the exact inverse as
    its allowance goes to 0 and meets its allowance otherwise; flexible
    GMRES with the exact inverse takes the iterations of right-preconditioned
    GMRES and reaches LU; with the inexact inner solve at the paper's 1e-5
    it still reaches the LU solution of the reduced system."""
    P = oracle_problem("cyl_small")
    w, m = P["w"], P["m"]
    cb = cbf.build(m, P["Kc"], P["TE"], P["TH"], w.edge_block, w.gen, w.k0, w.eta0, 1e-3)
    CJM, CMJ = reduced.cbf_matrices(cb, m.ne)
    Zr = reduced.project(P["Z"], CJM, CMJ)
    Gc = reduced.gram_cbf(cbf.rwg_gram(m), CJM, CMJ)
    n = Gc.shape[0]
    y = configs.random_complex((n, 2), 31)
    xe = np.linalg.solve(Gc, y)
    x0 = reduced.cmp_inner(Gc, y, 1e-14)
    assert np.linalg.norm(x0 - xe) <= 1e-8 * np.linalg.norm(xe)
    x5 = reduced.cmp_inner(Gc, y, 1e-5)
    assert np.all(np.linalg.norm(Gc @ x5 - y, axis=0) <= 1e-5 * np.linalg.norm(y, axis=0))
    vr = CJM.conj().T @ P["v"][:, 0]
    Gi = np.linalg.inv(Gc)
    ref = np.linalg.solve(Zr, vr)
    yv, it_r, _ = reduced.gmres(lambda u: Zr @ (Gi @ u), vr, 1e-10, n, n)
    xf, it_f, _ = reduced.fgmres(lambda u: Zr @ u, lambda q: Gi @ q, vr, 1e-10, n, n)
    assert it_f == it_r and np.linalg.norm(xf - Gi @ yv) <= 1e-8 * np.linalg.norm(ref)
    assert np.linalg.norm(xf - ref) <= 1e-8 * np.linalg.norm(ref)
    xi, it_i, _ = reduced.fgmres(lambda u: Zr @ u, lambda q: reduced.cmp_inner(Gc, q, 1e-5)[:, 0], vr, 1e-12, n, n)
    assert np.linalg.norm(xi - ref) <= 1e-9 * np.linalg.norm(ref)


def test_block_krylov_minimiser():
    """The oracle's block GMRES iterate (the minimiser of each column's
    residual over K_J(A, B)), on a random well-conditioned complex system
    (n 60, p 4): with J p >= n the space is everything and the iterate is
    the exact solution; with one column it is plain GMRES after J
    iterations (the oracle's MGS GMRES, independent code); permuting the
    columns of B permutes the iterates; each residual is orthogonal to
    A K_J (the least-squares condition, checked on a Krylov basis built by
    plain powers of A); and the residuals do not grow with J."""
    rng = np.random.default_rng(5)
    n, p = 60, 4
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    B = rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))
    mv = lambda X: A @ X
    x = reduced.block_krylov_minimiser(mv, B, n // p)
    assert np.linalg.norm(x - np.linalg.solve(A, B)) / np.linalg.norm(np.linalg.solve(A, B)) < 1e-11
    for J in (3, 7):
        x1 = reduced.block_krylov_minimiser(mv, B[:, :1], J)[:, 0]
        g, its, _ = reduced.gmres(lambda v: A @ v, B[:, 0], tol=0.0, restart=J, max_iter=J)
        assert its == J and np.linalg.norm(x1 - g) / np.linalg.norm(g) < 1e-11
    perm = [2, 0, 3, 1]
    xp = reduced.block_krylov_minimiser(mv, B[:, perm], 5)
    x5 = reduced.block_krylov_minimiser(mv, B, 5)
    assert np.linalg.norm(xp - x5[:, perm]) / np.linalg.norm(x5) < 1e-11
    K = np.hstack([np.linalg.matrix_power(A, j) @ B for j in range(5)])
    r = B - A @ x5
    assert np.max(np.abs((A @ K).conj().T @ r)) < 1e-9 * np.linalg.norm(A @ K) * np.linalg.norm(B)
    res = [np.linalg.norm(B - A @ reduced.block_krylov_minimiser(mv, B, J), axis=0) for J in (1, 2, 4, 8)]
    assert all(np.all(res[i + 1] <= res[i] * (1 + 1e-12)) for i in range(3))
