"""Characteristic basis functions with the dual (Calderon-compatible)
orthogonalisation (Sec. III-A and III-B).

* Primary CBF currents (eq. of the primary CBFs): for cell m,
  Z_mm J_m = V_m with Z_mm the cell's own 2N_m x 2N_m PMCHWT block and V_m
  the tested incident fields of the s generating plane waves; solved by LU.
* RWG Gram of the cell (eq. of G_m): [G_m]_ij = int (n x f_i) . f_j, the
  rotated pairing of two RWG functions of the cell, integrated here by the
  7-point rule, which is exact for this degree-2 integrand.
* CBF Gram G'_m = (J^M)^H G_m J^J (s x s), its SVD U S V^H truncated to the
  L_m singular values with sigma_i / sigma_1 >= delta_SVD, and
  C^M = J^M U_L, C^J = J^J V_L (eq. of the CBFs), so that
  (C^M)^H G_m C^J = S_L (the duality relation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import quadrature as qd
from .excitation import rhs
from .mesh import RWGMesh


def rwg_gram(m: RWGMesh):
    """Full RWG Gram G (ne x ne, real): G_ij = int (n x f_i) . f_j."""
    pts = qd.points(m.xyz)
    s = m.tri_sign.astype(np.float64)
    L = m.length[m.tri_edge]
    coef = s * L / (2.0 * m.area[:, None])
    f = coef[:, None, :, None] * (pts[:, :, None, :] - m.xyz[:, None, :, :])   # (nt,7,3,3)
    nf = np.cross(m.normal[:, None, None, :], f)
    loc = np.einsum("q,t,tqai,tqbi->tab", qd.WEIGHTS, m.area, nf, f)          # (nt,3,3)
    G = np.zeros((m.ne, m.ne))
    ii = np.broadcast_to(m.tri_edge[:, :, None], loc.shape)
    jj = np.broadcast_to(m.tri_edge[:, None, :], loc.shape)
    np.add.at(G, (ii.ravel(), jj.ravel()), loc.ravel())
    return G


def rwg_gram_sparse(m: RWGMesh):
    """The RWG Gram of ``rwg_gram`` as a scipy CSR matrix (the same local
    3 x 3 integrals summed over each triangle's RWGs; nonzero only between
    RWGs that share a triangle), for meshes whose dense Gram is too large."""
    import scipy.sparse
    pts = qd.points(m.xyz)
    s = m.tri_sign.astype(np.float64)
    L = m.length[m.tri_edge]
    coef = s * L / (2.0 * m.area[:, None])
    f = coef[:, None, :, None] * (pts[:, :, None, :] - m.xyz[:, None, :, :])   # (nt,7,3,3)
    nf = np.cross(m.normal[:, None, None, :], f)
    loc = np.einsum("q,t,tqai,tqbi->tab", qd.WEIGHTS, m.area, nf, f)          # (nt,3,3)
    ii = np.broadcast_to(m.tri_edge[:, :, None], loc.shape)
    jj = np.broadcast_to(m.tri_edge[:, None, :], loc.shape)
    return scipy.sparse.coo_matrix((loc.ravel(), (ii.ravel(), jj.ravel())), shape=(m.ne, m.ne)).tocsr()


@dataclass
class CBFSet:
    cells: list            # per cell: sorted edge ids
    CM: list               # per cell (N_m, L_m)
    CJ: list
    sigma: list            # per cell (L_m,)
    sigma_all: list        # per cell, every singular value of G'_m

    @property
    def L(self):
        return np.array([c.shape[1] for c in self.CM])

    @property
    def n_cbf(self):
        return 2 * int(self.L.sum())


def primary_currents(m: RWGMesh, Kop, TE, TH, edges, gen, k0, eta0, V=None):
    """J_m = Z_mm^{-1} V_m for the cell's edges and generating waves."""
    ix = np.asarray(edges)
    Zmm = np.block([[Kop[np.ix_(ix, ix)], -TE[np.ix_(ix, ix)]],
                    [TH[np.ix_(ix, ix)], Kop[np.ix_(ix, ix)]]])
    if V is None:
        V = rhs(m, gen, k0, eta0)
    Vm = np.concatenate([V[ix], V[m.ne + ix]], axis=0)
    Jm = np.linalg.solve(Zmm, Vm)
    n = len(ix)
    return Jm[:n], Jm[n:]


def dual_cbfs(JM, JJ, Gm, delta_svd):
    """SVD of G'_m = JM^H Gm JJ, truncation, C^M = JM U_L, C^J = JJ V_L."""
    Gp = JM.conj().T @ Gm @ JJ
    # LAPACK's QR-iteration SVD (gesvd): robust on the numerically
    # rank-deficient G'_m (rank <= N_m < s)
    U, S, Vh = scipy.linalg.svd(Gp, lapack_driver="gesvd")
    L = int(np.count_nonzero(S / S[0] >= delta_svd))
    return JM @ U[:, :L], JJ @ Vh.conj().T[:, :L], S[:L], S


def build(m: RWGMesh, Kop, TE, TH, edge_block, gen, k0, eta0, delta_svd=1e-3):
    edge_block = np.asarray(edge_block)
    G = rwg_gram(m)
    V = rhs(m, gen, k0, eta0)
    cells, CM, CJ, sig, sall = [], [], [], [], []
    for c in range(int(edge_block.max()) + 1):
        ix = np.nonzero(edge_block == c)[0]
        JM, JJ = primary_currents(m, Kop, TE, TH, ix, gen, k0, eta0, V)
        cm, cj, s, S = dual_cbfs(JM, JJ, G[np.ix_(ix, ix)], delta_svd)
        cells.append(ix)
        CM.append(cm)
        CJ.append(cj)
        sig.append(s)
        sall.append(S)
    return CBFSet(cells, CM, CJ, sig, sall)


def dual_from_currents(m: RWGMesh, edge_block, currents, delta_svd, G=None):
    """Dual CBFs of every cell from given current coefficient sets
    ``currents`` = [(J^M_m, J^J_m), ...] (N_m x s each, cell by cell): the
    same orthogonalisation as ``build`` (G'_m, SVD, truncation) applied to
    currents that come from elsewhere (IPCBF solutions, or seeded test
    inputs)."""
    edge_block = np.asarray(edge_block)
    if G is None:
        G = rwg_gram_sparse(m)
    cells, CM, CJ, sig, sall = [], [], [], [], []
    for c, (JM, JJ) in enumerate(currents):
        ix = np.nonzero(edge_block == c)[0]
        Gm = G[np.ix_(ix, ix)] if isinstance(G, np.ndarray) else G[ix][:, ix].toarray()
        cm, cj, s, S = dual_cbfs(JM, JJ, Gm, delta_svd)
        cells.append(ix)
        CM.append(cm)
        CJ.append(cj)
        sig.append(s)
        sall.append(S)
    return CBFSet(cells, CM, CJ, sig, sall)
