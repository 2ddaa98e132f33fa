"""Galerkin fill of the PMCHWT operators (Sec. II-B, eqs. for [K_i]_mn and
[T_i]_mn and the block matrix Z of the discretised system).

Definitions used (Sec. II-A operators, e^{jwt}):
  G_i(R) = e^{-j k_i R} / (4 pi R)
  [T_i]_mn = j k_i int int G_i [ f_m(r) . f_n(r') - div f_m div' f_n / k_i^2 ]
             (the grad-grad term moved onto the divergences)
  [K_i]_mn = int int f_m(r) . ( grad' G_i(r, r') x f_n(r') )
             grad' G_i = -g_i(R) (r - r'),  g_i = -(1 + j k_i R) e^{-j k_i R} / (4 pi R^3)
  Z = [[K1 + K2, -(eta1 T1 + eta2 T2)], [T1/eta1 + T2/eta2, K1 + K2]]
  unknown order [alpha^M ; alpha^J], test order [t^J ; t^M].

Far triangle pairs: the 7 x 7 point product rule applied to the integrands
exactly as written above.  Near pairs (``oracle.mesh.near_pairs``): the
7-point rule on the test triangle; on the source triangle the terms
1/R - k^2 R / 2 of 4 pi G and 1/R^3 + k^2 / (2R) of -4 pi g are integrated in
closed form (``oracle.potentials``) and the bounded remainders with the
7-point rule.  K of a coplanar near pair (including P == Q) is 0: the
integrand is a triple product of three vectors in one plane.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as qd
from .mesh import RWGMesh, coplanar, near_pairs
from .potentials import triangle_potentials

FOUR_PI = 4.0 * np.pi


def media(k0, eta0, eps_r, mu_r):
    """Wavenumbers and impedances (k_i, eta_i) of exterior vacuum and the
    interior medium: k2 = k0 sqrt(eps_r mu_r), eta2 = eta0 sqrt(mu_r/eps_r),
    principal square roots (Im k2 <= 0 for a lossy eps_r = e' - j e'')."""
    eps_r, mu_r = complex(eps_r), complex(mu_r)
    k = np.array([k0, k0 * np.sqrt(eps_r * mu_r)], dtype=np.complex128)
    eta = np.array([eta0, eta0 * np.sqrt(mu_r / eps_r)], dtype=np.complex128)
    return k, eta


def _rwg_values(m: RWGMesh, tris, pts):
    """f_a at points ``pts`` (n, np, 3) of triangles ``tris`` -> (n, np, 3a, 3)
    and the divergences (n, 3a), signs and edge lengths included."""
    s = m.tri_sign[tris].astype(np.float64)            # (n,3)
    L = m.length[m.tri_edge[tris]]                     # (n,3)
    A = m.area[tris]
    coef = s * L / (2.0 * A[:, None])                  # (n,3)
    f = coef[:, None, :, None] * (pts[:, :, None, :] - m.xyz[tris][:, None, :, :])
    div = s * L / A[:, None]
    return f, div


def regular_local(m: RWGMesh, k, P, Q):
    """Local 3x3 blocks of K1+K2, T1, T2 for far pairs (P[i], Q[i]) by the
    7x7 product rule.  Returns (K, T) with shapes (n,3,3) and (2,n,3,3)."""
    w = qd.WEIGHTS
    rp = qd.points(m.xyz[P])
    rq = qd.points(m.xyz[Q])
    fa, da = _rwg_values(m, P, rp)
    fb, db = _rwg_values(m, Q, rq)
    diff = rp[:, :, None, :] - rq[:, None, :, :]        # r - r'   (n,7,7,3)
    R = np.sqrt((diff * diff).sum(axis=-1))
    wA = (w[:, None] * w[None, :])[None] * (m.area[P] * m.area[Q])[:, None, None]
    fafb = np.einsum("nkai,njbi->nkjab", fa, fb)
    dd = da[:, :, None] * db[:, None, :]
    Ts = []
    gsum = 0.0
    for ki in k:
        e = np.exp(-1j * ki * R)
        G = e / (FOUR_PI * R)
        g = -(1.0 + 1j * ki * R) * e / (FOUR_PI * R ** 3)
        gsum = gsum + g
        Ts.append(1j * ki * np.einsum("nkj,nkjab->nab", wA * G, fafb)
                  - (1j / ki) * (wA * G).sum(axis=(1, 2))[:, None, None] * dd)
    # grad' G x f_b = -g (r - r') x f_b(r')
    cr = np.cross(diff[:, :, :, None, :], fb[:, None, :, :, :])   # (n,7,7,3b,3)
    K = -np.einsum("nkj,nkai,nkjbi->nab", wA * gsum, fa, cr)
    return K, np.stack(Ts)


def _Gr(k, R):
    """4 pi G - (1/R - k^2 R/2), bounded; its limit -jk at R = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (np.exp(-1j * k * R) - 1.0) / R + 0.5 * k * k * R
    return np.where(R == 0.0, -1j * k, v) / FOUR_PI


def _gr(k, R):
    """g + (1/R^3 + k^2/(2R))/(4 pi), bounded; its limit j k^3/(12 pi) at 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (-(1.0 + 1j * k * R) * np.exp(-1j * k * R) + 1.0 + 0.5 * k * k * R * R) / R ** 3
    return np.where(R == 0.0, 1j * k ** 3 / 3.0, v) / FOUR_PI


def near_local(m: RWGMesh, k, p, q):
    """Local 3x3 blocks (K, T1, T2) of one near pair with singularity
    subtraction on the source triangle."""
    w = qd.WEIGHTS
    rp = qd.points(m.xyz[[p]])[0]                       # (7,3)
    rq = qd.points(m.xyz[[q]])[0]
    fa, da = _rwg_values(m, np.array([p]), rp[None])
    fa, da = fa[0], da[0]                               # (7,3a,3), (3,)
    sq = m.tri_sign[q].astype(np.float64)
    Lq = m.length[m.tri_edge[q]]
    Aq, Ap = m.area[q], m.area[p]
    vq = m.xyz[q]                                       # free vertices q_b
    pot = triangle_potentials(rp, np.broadcast_to(vq, (7, 3, 3)))
    diff = rp[:, None, :] - rq[None, :, :]              # (7,7,3)
    R = np.sqrt((diff * diff).sum(axis=-1))
    Ts = []
    for ki in k:
        Gr = _Gr(ki, R)                                 # (7,7)
        J0 = (pot["Im1"] - 0.5 * ki * ki * pot["I1"]) / FOUR_PI + Aq * (Gr * w[None]).sum(1)
        # int G r' = int G (r' - r) + r int G
        J1 = ((pot["Vm1"] + rp * pot["Im1"][:, None])
              - 0.5 * ki * ki * (pot["V1"] + rp * pot["I1"][:, None])) / FOUR_PI \
            + Aq * np.einsum("kj,j,ji->ki", Gr, w, rq)
        # int_Q G f_b = s_b l_b / (2 Aq) (J1 - q_b J0); int_Q G div f_b = s_b l_b / Aq J0
        cb = sq * Lq
        inner_f = (cb / (2 * Aq))[None, :, None] * (J1[:, None, :] - vq[None, :, :] * J0[:, None, None])
        inner_d = (cb / Aq)[None, :] * J0[:, None]      # (7,3b)
        T = 1j * ki * Ap * (np.einsum("k,kai,kbi->ab", w, fa, inner_f)
                            - np.einsum("k,a,kb->ab", w, da, inner_d) / (ki * ki))
        Ts.append(T)
    if p == q or coplanar(m, p, q):
        K = np.zeros((3, 3), dtype=np.complex128)
    else:
        # V(r) = int_Q g (r - r') summed over the media in k
        ksq = k[0] * k[0]
        grs = _gr(k[0], R)
        for ki in k[1:]:
            ksq = ksq + ki * ki
            grs = grs + _gr(ki, R)
        # int (r - r')/R = -Vm1
        Vs = -(float(len(k)) * pot["Gm3"] - 0.5 * ksq * pot["Vm1"]) / FOUR_PI
        Vk = Vs + Aq * np.einsum("kj,j,kji->ki", grs, w, diff)
        # int_Q grad'G x f_b = -(s_b l_b / 2Aq) V x (r - q_b)
        rmq = rp[:, None, :] - vq[None, :, :]           # (7,3b,3)
        inner = -(cb / (2 * Aq))[None, :, None] * np.cross(Vk[:, None, :], rmq)
        K = Ap * np.einsum("k,kai,kbi->ab", w, fa, inner)
    return K, np.stack(Ts)


def local_blocks(m: RWGMesh, k, chunk=4096):
    """All triangle-pair blocks: returns (K, T) of shapes (nt,nt,3,3) and
    (2,nt,nt,3,3).  Memory O(nt^2); meant for small meshes."""
    nt = m.nt
    K = np.zeros((nt, nt, 3, 3), dtype=np.complex128)
    T = np.zeros((2, nt, nt, 3, 3), dtype=np.complex128)
    near = near_pairs(m)
    is_near = np.zeros((nt, nt), dtype=bool)
    is_near[near[:, 0], near[:, 1]] = True
    PP, QQ = np.nonzero(~is_near)
    for s in range(0, len(PP), chunk):
        P, Q = PP[s:s + chunk], QQ[s:s + chunk]
        Kc, Tc = regular_local(m, k, P, Q)
        K[P, Q] = Kc
        T[:, P, Q] = Tc
    for p, q in near:
        Kc, Tc = near_local(m, k, p, q)
        K[p, q] = Kc
        T[:, p, q] = Tc
    return K, T


def assemble_ops(m: RWGMesh, K, T):
    """Scatter triangle-pair blocks into RWG matrices K (=K1+K2), T1, T2."""
    ne = m.ne
    out = [np.zeros((ne, ne), dtype=np.complex128) for _ in range(3)]
    rows = m.tri_edge                                   # (nt,3)
    for X, Y in zip(out, [K, T[0], T[1]]):
        # Y[p, q, a, b] -> X[tri_edge[p,a], tri_edge[q,b]]
        ii = np.broadcast_to(rows[:, None, :, None], Y.shape)
        jj = np.broadcast_to(rows[None, :, None, :], Y.shape)
        np.add.at(X, (ii.ravel(), jj.ravel()), Y.ravel())
    return out


def fill_ops(m: RWGMesh, k):
    """RWG matrices (K, T1, T2) with K = K1 + K2."""
    K, T = local_blocks(m, k)
    return assemble_ops(m, K, T)


def fill_media(m: RWGMesh, k):
    """The four operators of the two media apart, (K1, K2, T1, T2): K_i is the
    K operator of medium i alone (the fill with the single wavenumber k_i)."""
    K1, T1 = _one_medium(m, k[0])
    K2, T2 = _one_medium(m, k[1])
    return K1, K2, T1, T2


def _one_medium(m: RWGMesh, ki):
    K, T = local_blocks(m, np.array([ki]))
    ne = m.ne
    out = [np.zeros((ne, ne), dtype=np.complex128) for _ in range(2)]
    rows = m.tri_edge
    for X, Y in zip(out, [K, T[0]]):
        ii = np.broadcast_to(rows[:, None, :, None], Y.shape)
        jj = np.broadcast_to(rows[None, :, None, :], Y.shape)
        np.add.at(X, (ii.ravel(), jj.ravel()), Y.ravel())
    return out


def combine(Kop, T1, T2, eta):
    """The three operator combinations of the PMCHWT blocks: K = K1+K2,
    TE = eta1 T1 + eta2 T2, TH = T1/eta1 + T2/eta2."""
    return Kop, eta[0] * T1 + eta[1] * T2, T1 / eta[0] + T2 / eta[1]


def assemble_Z(Kop, TE, TH):
    """Z = [[K, -TE], [TH, K]] acting on [alpha^M; alpha^J]."""
    return np.block([[Kop, -TE], [TH, Kop]])


def fill_rows(m: RWGMesh, k, rows, chunk=4096):
    """Rows ``rows`` (RWG ids) of K (=K1+K2), T1, T2, each (len(rows), ne),
    computing only the triangle pairs those rows need."""
    rows = np.asarray(rows)
    tris = np.unique(np.concatenate([m.tplus[rows], m.tminus[rows]]))
    near = near_pairs(m)
    near_set = set(map(tuple, near.tolist()))
    nt = m.nt
    K = np.zeros((len(tris), nt, 3, 3), dtype=np.complex128)
    T = np.zeros((2, len(tris), nt, 3, 3), dtype=np.complex128)
    PP, QQ, II = [], [], []
    for i, p in enumerate(tris):
        for q in range(nt):
            if (p, q) in near_set:
                Kc, Tc = near_local(m, k, p, q)
                K[i, q] = Kc
                T[:, i, q] = Tc
            else:
                PP.append(p)
                QQ.append(q)
                II.append(i)
    PP, QQ, II = map(np.asarray, (PP, QQ, II))
    for s in range(0, len(PP), chunk):
        Kc, Tc = regular_local(m, k, PP[s:s + chunk], QQ[s:s + chunk])
        K[II[s:s + chunk], QQ[s:s + chunk]] = Kc
        T[:, II[s:s + chunk], QQ[s:s + chunk]] = Tc
    pos = {int(t): i for i, t in enumerate(tris)}
    out = [np.zeros((len(rows), m.ne), dtype=np.complex128) for _ in range(3)]
    for r, e in enumerate(rows):
        for tp, ap in ((m.tplus[e], m.aplus[e]), (m.tminus[e], m.aminus[e])):
            i = pos[int(tp)]
            for X, Y in zip(out, (K, T[0], T[1])):
                # Y[i, q, ap, b] -> column tri_edge[q, b]
                np.add.at(X[r], m.tri_edge.ravel(), Y[i, :, ap, :].ravel())
    return out


def fill_block(m: RWGMesh, k, rows, cols, chunk=4096, near=None):
    """Rows ``rows`` and columns ``cols`` (RWG ids) of K (=K1+K2), T1, T2,
    each (len(rows), len(cols)), from the triangle pairs that carry them
    only: every entry is the sum over the two triangles of the test RWG and
    the two of the trial RWG of the pair blocks defined above (same far and
    near rules), so a sub-block of a large mesh costs only its own pairs.
    ``near``: the mesh's near-pair array if already at hand."""
    rows, cols = np.asarray(rows), np.asarray(cols)
    rt = np.unique(np.concatenate([m.tplus[rows], m.tminus[rows]]))
    ct = np.unique(np.concatenate([m.tplus[cols], m.tminus[cols]]))
    near_set = set(map(tuple, (near_pairs(m) if near is None else near).tolist()))
    K = np.zeros((len(rt), len(ct), 3, 3), dtype=np.complex128)
    T = np.zeros((2, len(rt), len(ct), 3, 3), dtype=np.complex128)
    PP, QQ, II, JJ = [], [], [], []
    for i, p in enumerate(rt.tolist()):
        for j, q in enumerate(ct.tolist()):
            if (p, q) in near_set:
                Kc, Tc = near_local(m, k, p, q)
                K[i, j] = Kc
                T[:, i, j] = Tc
            else:
                PP.append(p)
                QQ.append(q)
                II.append(i)
                JJ.append(j)
    PP, QQ, II, JJ = map(np.asarray, (PP, QQ, II, JJ))
    for s in range(0, len(PP), chunk):
        Kc, Tc = regular_local(m, k, PP[s:s + chunk], QQ[s:s + chunk])
        K[II[s:s + chunk], JJ[s:s + chunk]] = Kc
        T[:, II[s:s + chunk], JJ[s:s + chunk]] = Tc
    rpos = {int(t): i for i, t in enumerate(rt)}
    cpos = {int(t): j for j, t in enumerate(ct)}
    out = [np.zeros((len(rows), len(cols)), dtype=np.complex128) for _ in range(3)]
    for r, e in enumerate(rows.tolist()):
        for tp, ap in ((m.tplus[e], m.aplus[e]), (m.tminus[e], m.aminus[e])):
            i = rpos[int(tp)]
            for c, f in enumerate(cols.tolist()):
                for tq, bq in ((m.tplus[f], m.aplus[f]), (m.tminus[f], m.aminus[f])):
                    j = cpos[int(tq)]
                    out[0][r, c] += K[i, j, ap, bq]
                    out[1][r, c] += T[0, i, j, ap, bq]
                    out[2][r, c] += T[1, i, j, ap, bq]
    return out
