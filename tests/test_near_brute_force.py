"""The near-pair rule on touching triangle pairs against a converged
brute-force reference (Sec. II-A: the operators' principal-value and
finite-part integrals; Sec. II-B entries).

The near rule (the oracle's, which the GPU kernels match to 1e-10) takes the
7-point rule on the test triangle and integrates the singular parts over the
source triangle in closed form.  The reference here shares nothing with it:
the test triangle is cut into 4^L congruent triangles, each with a collapsed
n x n Gauss-Legendre rule, and for every outer point the source integrals
are split at the point's projection into three signed triangles, each mapped
to the unit square (the polar Duffy map, radius graded as t^3) with a
Gauss-Legendre product rule, which takes the 1/R and 1/R^2 singularities
without subtraction.  Two levels of the reference bound its own error; the
near rule's error is then reported per pair class of the 1,728-triangle
cube (self, edge- and vertex-adjacent, in one plane or across a cube edge,
and the separated near pairs) and held below the bounds listed."""
import numpy as np
import pytest

FOUR_PI = 4.0 * np.pi


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _outer_rule(V, L, n):
    """Points and weights of a composite rule on triangle V (3 x 3)."""
    tris = [V]
    for _ in range(L):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nxt
    s, ws = _gl01(n)
    S, T = np.meshgrid(s, s, indexing="ij")
    pts, wts = [], []
    for v0, v1, v2 in tris:
        A2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
        pts.append((v0 + S[..., None] * (v1 - v0) + (S * T)[..., None] * (v2 - v1)).reshape(-1, 3))
        wts.append((np.outer(ws, ws) * S * A2).reshape(-1))
    return np.concatenate(pts), np.concatenate(wts)


def _source_integrals(r, V, k, nu, nv, grade=3):
    """int_Q G_i, int_Q G_i r' (per medium) and int_Q (g_1 + g_2)(r - r') for
    every outer point r, by the signed polar split of Q at r's projection."""
    nrm = np.cross(V[1] - V[0], V[2] - V[0])
    nrm /= np.linalg.norm(nrm)
    h = (r - V[0]) @ nrm
    r0 = r - h[:, None] * nrm
    t, wt = _gl01(nu)
    u, wu = t ** grade, wt * grade * t ** (grade - 1)
    s, ws = _gl01(nv)
    N = len(r)
    J0 = np.zeros((len(k), N), complex)
    J1 = np.zeros((len(k), N, 3), complex)
    Vg = np.zeros((N, 3), complex)
    for i in range(3):
        a, b = V[i], V[(i + 1) % 3]
        e = (a[None, None] - r0[:, None]) + s[None, :, None] * (b - a)[None, None]
        jac = np.cross(a[None] - r0, (b - a)[None]) @ nrm          # signed, twice the area
        rp = r0[:, None, None] + u[None, :, None, None] * e[:, None]
        W = (wu[:, None] * ws[None, :])[None] * u[None, :, None] * jac[:, None, None]
        d = r[:, None, None] - rp
        R = np.sqrt((d * d).sum(-1))
        gs = 0.0
        for m, ki in enumerate(k):
            E = np.exp(-1j * ki * R)
            G = E / (FOUR_PI * R)
            J0[m] += (W * G).sum((1, 2))
            J1[m] += np.einsum("nuv,nuvi->ni", W * G, rp)
            gs = gs - (1.0 + 1j * ki * R) * E / (FOUR_PI * R ** 3)
        Vg += np.einsum("nuv,nuvi->ni", W * gs, d)
    return J0, J1, Vg


def _reference_blocks(m, k, p, q, L, n, nsrc):
    """(K, [T_1, T_2]) local 3 x 3 blocks of the pair, as the fill defines
    them: T_i = j k_i int int G_i (f_a . f_b - div f_a div f_b / k_i^2),
    K = int int f_a . (grad' G x f_b) summed over the media."""
    Vp, Vq = m.xyz[p], m.xyz[q]
    r, w = _outer_rule(Vp, L, n)
    J0, J1, Vg = _source_integrals(r, Vq, k, nsrc, nsrc)
    ca = m.tri_sign[p] * m.length[m.tri_edge[p]]
    cb = m.tri_sign[q] * m.length[m.tri_edge[q]]
    Ap, Aq = m.area[p], m.area[q]
    fa = (ca / (2 * Ap))[None, :, None] * (r[:, None, :] - Vp[None])
    da = ca / Ap
    Ts = []
    for mi, ki in enumerate(k):
        f_in = (cb / (2 * Aq))[None, :, None] * (J1[mi][:, None, :] - Vq[None] * J0[mi][:, None, None])
        d_in = (cb / Aq)[None, :] * J0[mi][:, None]
        Ts.append(1j * ki * (np.einsum("n,nai,nbi->ab", w, fa, f_in) - np.einsum("n,a,nb->ab", w, da, d_in) / ki ** 2))
    # int_Q grad'G x f_b = -(c_b / 2A_Q) (int_Q g (r - r')) x (r - q_b)
    k_in = -(cb / (2 * Aq))[None, :, None] * np.cross(Vg[:, None, :], r[:, None, :] - Vq[None])
    K = np.einsum("n,nai,nbi->ab", w, fa, k_in)
    return K, np.stack(Ts)


# pair class -> bounds on the near rule's error relative to the largest entry
# of the reference block (T, K), as measured (with margin)
BOUNDS = {"self_coplanar": (1e-2, None), "edge_coplanar": (5e-3, None), "vertex_coplanar": (5e-4, None),
          "apart_coplanar": (1e-4, None), "edge_bent": (2e-3, 0.2), "vertex_bent": (1e-3, 3e-2),
          "apart_bent": (3e-4, 3e-3)}


def test_near_rule_against_brute_force():
    from oracle import fill, mesh as om
    from synth import configs
    w = configs.cube_c2()
    m = om.build(w.V, w.T)
    k, _ = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    cases = {}
    for p, q in om.near_pairs(m):
        shared = len(set(map(tuple, m.xyz[p].round(12))) & set(map(tuple, m.xyz[q].round(12))))
        cop = p == q or om.coplanar(m, p, q)
        key = ("self" if p == q else {2: "edge", 1: "vertex", 0: "apart"}[shared]) + ("_coplanar" if cop else "_bent")
        cases.setdefault(key, (int(p), int(q)))
    assert set(cases) == set(BOUNDS), sorted(cases)
    for key, (p, q) in sorted(cases.items()):
        Kn, Tn = fill.near_local(m, k, p, q)
        K2, T2 = _reference_blocks(m, k, p, q, 2, 6, 24)
        K3, T3 = _reference_blocks(m, k, p, q, 3, 6, 32)
        sT = np.abs(T3).max()
        ref_T, err_T = np.abs(T3 - T2).max() / sT, np.abs(Tn - T3).max() / sT
        msg = f"{key} ({p}, {q}): reference change T {ref_T:.1e}; near rule error T {err_T:.1e}"
        bT, bK = BOUNDS[key]
        assert ref_T < 0.2 * bT, msg
        assert err_T < bT, msg
        if bK is None:
            assert np.abs(Kn).max() == 0.0 and np.abs(K3).max() < 1e-12 * sT, msg  # coplanar: K vanishes
        else:
            sK = np.abs(K3).max()
            ref_K, err_K = np.abs(K3 - K2).max() / sK, np.abs(Kn - K3).max() / sK
            msg += f", reference change K {ref_K:.1e}; near rule error K {err_K:.1e}"
            assert ref_K < 0.2 * bK and err_K < bK, msg
        print(msg)
