"""Reduced CBFM system with the Calderon multiplicative preconditioner
(Sec. III-C).

  C^JM = blkdiag(C^J_1..C^J_M, C^M_1..C^M_M)       (N x N_CBF)
  C^MJ = blkdiag(C^M_1..C^M_M, C^J_1..C^J_M)
  G^CBF = (C^JM)^H G_ffff C^MJ,  G_ffff = blkdiag(G, G)
  outer:  [(C^JM)^H Z C^MJ] (G^CBF)^{-1} y = (C^JM)^H v
  inner:  G^CBF j_CBF = y
  j = C^MJ j_CBF

The outer system is solved by restarted GMRES with modified Gram-Schmidt
Arnoldi (Saad 2003), x0 = 0, stopping on the relative residual of the
preconditioned system; the inner system by a dense LU (an exact inverse).
"""
from __future__ import annotations

import numpy as np

from .cbf import CBFSet


def expand(cb: CBFSet, ne: int, which: str):
    """Dense ne x (sum L) block matrix of C^M or C^J (columns cell by cell)."""
    Ls = cb.L
    off = np.concatenate([[0], np.cumsum(Ls)])
    C = np.zeros((ne, off[-1]), dtype=np.complex128)
    mats = cb.CM if which == "M" else cb.CJ
    for c, ix in enumerate(cb.cells):
        C[np.ix_(ix, np.arange(off[c], off[c + 1]))] = mats[c]
    return C


def cbf_matrices(cb: CBFSet, ne: int):
    CM = expand(cb, ne, "M")
    CJ = expand(cb, ne, "J")
    Z0 = np.zeros_like(CM)
    CJM = np.block([[CJ, Z0], [Z0, CM]])
    CMJ = np.block([[CM, Z0], [Z0, CJ]])
    return CJM, CMJ


def project(Z, CJM, CMJ):
    """Z_r = (C^JM)^H Z C^MJ."""
    return CJM.conj().T @ Z @ CMJ


def gram_cbf(G, CJM, CMJ):
    ne = G.shape[0]
    Gff = np.zeros((2 * ne, 2 * ne))
    Gff[:ne, :ne] = G
    Gff[ne:, ne:] = G
    return CJM.conj().T @ Gff @ CMJ


def gram_b(G, cb: CBFSet):
    """B = (C^M)^H G C^J (sum L x sum L) built cell pair by cell pair from a
    dense or scipy-sparse RWG Gram G.  Since G is real antisymmetric,
    G^CBF = blkdiag((C^J)^H G C^M, (C^M)^H G C^J) = blkdiag(-B^H, B)."""
    Ls = cb.L
    off = np.concatenate([[0], np.cumsum(Ls)])
    B = np.zeros((off[-1], off[-1]), dtype=np.complex128)
    for a, ia in enumerate(cb.cells):
        Ga = G[ia] if isinstance(G, np.ndarray) else G[ia].toarray()
        for b, ib in enumerate(cb.cells):
            Gab = Ga[:, ib]
            if np.any(Gab):
                B[off[a]:off[a + 1], off[b]:off[b + 1]] = cb.CM[a].conj().T @ Gab @ cb.CJ[b]
    return B


def cmp_solve(B, y):
    """x = (G^CBF)^{-1} y for G^CBF = blkdiag(-B^H, B), columns of y of
    length 2 sum L (inner CBFM equation, solved exactly by LU)."""
    NL = B.shape[0]
    y = np.asarray(y)
    x = np.empty_like(y, dtype=np.complex128)
    x[:NL] = np.linalg.solve(-B.conj().T, y[:NL])
    x[NL:] = np.linalg.solve(B, y[NL:])
    return x


def project_block(Kab, TEab, THab, CMa, CJa, CMb, CJb):
    """Block (cell a rows, cell b columns) of Z_r = (C^JM)^H Z C^MJ from the
    cell-pair blocks of K, TE, TH: the four quadrants
    [[(C^J_a)^H K C^M_b, -(C^J_a)^H TE C^J_b], [(C^M_a)^H TH C^M_b, (C^M_a)^H K C^J_b]]."""
    return np.block([[CJa.conj().T @ Kab @ CMb, -(CJa.conj().T @ TEab @ CJb)],
                     [CMa.conj().T @ THab @ CMb, CMa.conj().T @ Kab @ CJb]])


def gmres(matvec, b, tol=1e-12, restart=100, max_iter=1000):
    """Restarted GMRES(restart) for one right-hand side.  Returns
    (x, iterations, relative residual history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0:
        return x, 0, hist
    it = 0
    r = b.copy()
    while it < max_iter:
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            break
        m = min(restart, max_iter - it)
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        Vb[0] = r / beta
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        kk = 0
        for kk in range(m):
            wv = matvec(Vb[kk])
            for i in range(kk + 1):
                H[i, kk] = np.vdot(Vb[i], wv)
                wv = wv - H[i, kk] * Vb[i]
            H[kk + 1, kk] = np.linalg.norm(wv)
            if H[kk + 1, kk] != 0:
                Vb[kk + 1] = wv / H[kk + 1, kk]
            for i in range(kk):                         # previous rotations
                t = cs[i] * H[i, kk] + sn[i] * H[i + 1, kk]
                H[i + 1, kk] = -np.conj(sn[i]) * H[i, kk] + np.conj(cs[i]) * H[i + 1, kk]
                H[i, kk] = t
            a, bb = H[kk, kk], H[kk + 1, kk]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[kk] = np.conj(a) / den if den else 1.0
            sn[kk] = np.conj(bb) / den if den else 0.0
            H[kk, kk] = den
            H[kk + 1, kk] = 0
            g[kk + 1] = -np.conj(sn[kk]) * g[kk]
            g[kk] = cs[kk] * g[kk]
            it += 1
            hist.append(abs(g[kk + 1]) / bn)
            if hist[-1] <= tol:
                kk += 1
                break
        else:
            kk = m
        y = np.linalg.solve(np.triu(H[:kk, :kk]), g[:kk]) if kk else np.zeros(0)
        x = x + Vb[:kk].T @ y
        r = b - matvec(x)
        if hist[-1] <= tol:
            break
    return x, it, hist


def block_krylov_minimiser(matvec, B, J):
    """Block GMRES after J block iterations from x0 = 0, for the columns of
    B (n x p, full column rank) at once: every column's iterate minimises
    its own residual ||b_c - A x|| over the block Krylov space
    K_J(A, B) = span{B, A B, ..., A^(J-1) B}, the outer equation of Sec.
    III-C solved for many incidences together.  The space is spanned by
    block Arnoldi (each new block A Q_j projected twice against the earlier
    blocks, then a Householder QR); the minimiser is the least-squares
    solution over that basis.  matvec maps an n x k block to A times it."""
    B = np.asarray(B, dtype=np.complex128)
    Q, _ = np.linalg.qr(B)
    blocks = [Q]
    for _ in range(1, J):
        Vm = np.hstack(blocks)
        W = matvec(blocks[-1])
        for _ in range(2):
            W = W - Vm @ (Vm.conj().T @ W)
        Q, _ = np.linalg.qr(W)
        blocks.append(Q)
    K = np.hstack(blocks)
    Y = np.linalg.lstsq(matvec(K), B, rcond=None)[0]
    return K @ Y


def cmp_inner(Gcbf, y, tol, restart=None, max_iter=None):
    """The paper's inexact (G^CBF)^{-1} (Sec. III-C, the paragraph on D^CBF):
    GMRES on G^CBF D z = y with the diagonal preconditioner
    D = diag(1 / [G^CBF]_ii) (1 where that diagonal is 0), x0 = 0, to the
    relative residual tol; x = D z, for every column of y."""
    n = Gcbf.shape[0]
    dg = np.diag(Gcbf)
    D = np.where(dg != 0, 1.0 / np.where(dg != 0, dg, 1.0), 1.0)
    A = Gcbf * D[None, :]
    y = np.asarray(y).reshape(n, -1)
    out = np.zeros_like(y, dtype=np.complex128)
    for c in range(y.shape[1]):
        z, _, _ = gmres(lambda u: A @ u, y[:, c], tol, restart or min(n, 500), max_iter or 4 * n)
        out[:, c] = D * z
    return out


def fgmres(matvec, precond, b, tol=1e-12, restart=100, max_iter=1000):
    """Flexible GMRES (Saad 2003): right preconditioning by an operator that
    may change from one iteration to the next.  The preconditioned vectors
    z_j = precond(q_j) are kept and the iterate is x = x0 + Z y, y from the
    same least-squares problem as GMRES (modified Gram-Schmidt Arnoldi on
    A z_j).  Returns (x, iterations, relative residual history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0:
        return x, 0, hist
    it = 0
    r = b.copy()
    while it < max_iter:
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            break
        m = min(restart, max_iter - it)
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        Zb = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        Vb[0] = r / beta
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        kk = 0
        for kk in range(m):
            Zb[kk] = precond(Vb[kk])
            wv = matvec(Zb[kk])
            for i in range(kk + 1):
                H[i, kk] = np.vdot(Vb[i], wv)
                wv = wv - H[i, kk] * Vb[i]
            H[kk + 1, kk] = np.linalg.norm(wv)
            if H[kk + 1, kk] != 0:
                Vb[kk + 1] = wv / H[kk + 1, kk]
            for i in range(kk):
                t = cs[i] * H[i, kk] + sn[i] * H[i + 1, kk]
                H[i + 1, kk] = -np.conj(sn[i]) * H[i, kk] + np.conj(cs[i]) * H[i + 1, kk]
                H[i, kk] = t
            a, bb = H[kk, kk], H[kk + 1, kk]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[kk] = np.conj(a) / den if den else 1.0
            sn[kk] = np.conj(bb) / den if den else 0.0
            H[kk, kk] = den
            H[kk + 1, kk] = 0
            g[kk + 1] = -np.conj(sn[kk]) * g[kk]
            g[kk] = cs[kk] * g[kk]
            it += 1
            hist.append(abs(g[kk + 1]) / bn)
            if hist[-1] <= tol:
                kk += 1
                break
        else:
            kk = m
        y = np.linalg.solve(np.triu(H[:kk, :kk]), g[:kk]) if kk else np.zeros(0)
        x = x + Zb[:kk].T @ y
        r = b - matvec(x)
        if hist[-1] <= tol:
            break
    return x, it, hist


def solve_reduced(Zr, Gcbf, vr, tol=1e-12, restart=100, max_iter=1000):
    """Right-preconditioned GMRES on Z_r G^-1 y = v_r, then j_CBF = G^-1 y,
    for every column of ``vr``.  Returns (j_CBF, iterations, histories)."""
    vr = np.asarray(vr).reshape(Zr.shape[0], -1)
    Ginv = np.linalg.inv(Gcbf)
    out = np.zeros_like(vr)
    its, hists = [], []
    for c in range(vr.shape[1]):
        y, it, h = gmres(lambda u: Zr @ (Ginv @ u), vr[:, c], tol, restart, max_iter)
        out[:, c] = Ginv @ y
        its.append(it)
        hists.append(h)
    return out, its, hists
