"""Full-system solves of the discretised PMCHWT system: the MoM baseline of
the numerical section (Sec. IV, the MoM arrangement with the diagonal
preconditioner), the IPCBF currents obtained from it by GMRES with a loose
residual allowance (Sec. III-A, the IPCBF equation and the GMRES version
proposed after it), the T-diagonal CBFM of the sphere-array comparison
(Sec. IV-A) and the RMSE of the CBFM RCS against the MoM RCS (Sec. IV-A).

Reading of the MoM arrangement.  The paper tests the T blocks of its MoM
matrix with the Buffa-Christiansen functions g (out of scope here); with
the RWG-tested blocks that this fill computes in their place,
  Z_t = [[-(eta1 T1 + eta2 T2), K1 + K2], [K1 + K2, T1/eta1 + T2/eta2]]
acting on j_t = [alpha^J; alpha^M]: the matrix Z of Sec. II-B with its two
column blocks swapped.  D = diag(Z_t) (the large T diagonals) is the
diagonal preconditioner: GMRES solves Z_t D^{-1} u = v from u = 0 and
j_t = D^{-1} u; right preconditioning leaves the residual v - Z_t j_t, so the
relative residual allowance delta_r bounds ||v - Z j|| / ||v||.

Test infrastructure only: never imported by the product.
"""
from __future__ import annotations

import numpy as np

from . import reduced


def mom_t_matrix(Kop, TE, TH):
    """Z_t = [[-TE, K], [K, TH]] on j_t = [alpha^J; alpha^M]."""
    return np.block([[-TE, Kop], [Kop, TH]])


def mom_t_solve(Zt, v, tol, restart, max_iter):
    """Right-preconditioned GMRES on Z_t D^{-1} u = v (D = diag Z_t, x0 = 0)
    for every column of v; j_t = D^{-1} u, returned in the order of Z,
    [alpha^M; alpha^J].  Returns (j, iterations, residual histories)."""
    v = np.asarray(v).reshape(Zt.shape[0], -1)
    d = np.diag(Zt).copy()
    A = Zt / d[None, :]
    ne = Zt.shape[0] // 2
    out = np.zeros_like(v, dtype=np.complex128)
    its, hists = [], []
    for c in range(v.shape[1]):
        u, it, h = reduced.gmres(lambda y: A @ y, v[:, c], tol, restart, max_iter)
        jt = u / d
        out[:ne, c] = jt[ne:]
        out[ne:, c] = jt[:ne]
        its.append(it)
        hists.append(h)
    return out, its, hists


def ipcbf_currents(Zt, Vgen, edge_block, delta_r, restart=None, max_iter=1000):
    """IPCBF coefficient sets: each of the s generating plane waves (columns
    of Vgen) solved on the whole scatterer by GMRES in the MoM arrangement to
    the relative residual delta_r; cell m keeps the rows of its RWGs,
    J^M_m = alpha^M[cell m] and J^J_m = alpha^J[cell m] (N_m x s).  Returns
    (per-cell [(J^M_m, J^J_m)], iterations per wave)."""
    edge_block = np.asarray(edge_block)
    J, its, _ = mom_t_solve(Zt, Vgen, delta_r, restart or max_iter, max_iter)
    ne = J.shape[0] // 2
    cur = []
    for c in range(int(edge_block.max()) + 1):
        ix = np.nonzero(edge_block == c)[0]
        cur.append((J[:ne][ix], J[ne:][ix]))
    return cur, its


def t_diagonal_operator(Zt, CJM):
    """The T-diagonal CBFM matrix (C^JM)^H Z_t C^JM of the sphere-array
    comparison (solved without the CMP): j_t^CBF in the order [J CBFs; M
    CBFs], j_t = C^JM j_t^CBF."""
    return CJM.conj().T @ Zt @ CJM


def rmse_db(sig_c, sig_m):
    """RMSE of the CBFM RCS sigma^c against the MoM RCS sigma^m over the
    observation angles (linear sigma): 10 log10 of the root mean square
    difference over the range max sigma^m - min sigma^m, in dB."""
    sig_c, sig_m = np.asarray(sig_c, float), np.asarray(sig_m, float)
    rms = np.sqrt(np.mean((sig_c - sig_m) ** 2))
    return 10.0 * np.log10(rms / (sig_m.max() - sig_m.min()))
