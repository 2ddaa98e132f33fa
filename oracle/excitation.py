"""Incident plane waves, tested right-hand sides and the far field.

RHS (Sec. II-B, the tested incident fields):
  v^E_m =  int f_m . E_inc,    v^H_m = -int f_m . H_inc,   v = [v^E ; v^H]
  E_inc = p e^{-j k0 k.r},  H_inc = (1/eta0) k x E_inc   (|E0| = 1).

Far field of the solved currents (monostatic RCS definition cited by the
paper, Knott 1993): with N = int J e^{j k0 rhat.r'} and
L = int M e^{j k0 rhat.r'},
  E_s ~ (-j k0 e^{-j k0 r} / 4 pi r) (eta0 N_perp - rhat x L),
  sigma = (k0^2 / 4 pi) |eta0 N_perp - rhat x L|^2      (wavelength^2 units).
The currents enter quadratically, so the global sign of the solution (the
operator-sign reading) does not change sigma.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as qd
from .mesh import RWGMesh


def _rwg_at_points(m: RWGMesh):
    """f_a at the 7 points of every triangle: (nt,7,3a,3) and the points."""
    pts = qd.points(m.xyz)
    s = m.tri_sign.astype(np.float64)
    L = m.length[m.tri_edge]
    coef = s * L / (2.0 * m.area[:, None])
    f = coef[:, None, :, None] * (pts[:, :, None, :] - m.xyz[:, None, :, :])
    return pts, f


def rhs(m: RWGMesh, inc, k0, eta0):
    """v = [v^E; v^H] for each incidence row (k, p): returns (2 ne, nrhs)."""
    inc = np.atleast_2d(inc)
    pts, f = _rwg_at_points(m)
    wA = qd.WEIGHTS[None, :] * m.area[:, None]              # (nt,7)
    out = np.zeros((2 * m.ne, len(inc)), dtype=np.complex128)
    for c, row in enumerate(inc):
        kh, ph = row[:3], row[3:]
        ph_ = np.exp(-1j * k0 * (pts @ kh))                  # (nt,7)
        E = ph_[..., None] * ph[None, None, :]
        H = np.cross(kh, E) / eta0
        vE = np.einsum("tq,tqai,tqi->ta", wA, f, E)
        vH = -np.einsum("tq,tqai,tqi->ta", wA, f, H)
        np.add.at(out[:m.ne, c], m.tri_edge.ravel(), vE.ravel())
        np.add.at(out[m.ne:, c], m.tri_edge.ravel(), vH.ravel())
    return out


def radiation_vectors(m: RWGMesh, j, dirs, k0):
    """N and L for coefficient vectors j = [alpha^M; alpha^J] (2ne, nrhs)
    in directions ``dirs`` (ndir, 3): returns (N, L) of shape (nrhs, ndir, 3)."""
    j = np.asarray(j).reshape(2 * m.ne, -1)
    pts, f = _rwg_at_points(m)
    wA = qd.WEIGHTS[None, :] * m.area[:, None]
    aM, aJ = j[:m.ne], j[m.ne:]
    # currents at the quadrature points: (nrhs, nt, 7, 3)
    Jp = np.einsum("tqai,tar->rtqi", f, aJ[m.tri_edge])
    Mp = np.einsum("tqai,tar->rtqi", f, aM[m.tri_edge])
    ph = np.exp(1j * k0 * np.einsum("tqi,di->dtq", pts, dirs)) * wA[None]
    N = np.einsum("dtq,rtqi->rdi", ph, Jp)
    L = np.einsum("dtq,rtqi->rdi", ph, Mp)
    return N, L


def far_field(m: RWGMesh, j, dirs, k0, eta0):
    """eta0 N_perp - rhat x L, proportional to the scattered far field."""
    dirs = np.atleast_2d(dirs)
    N, L = radiation_vectors(m, j, dirs, k0)
    rn = np.einsum("di,rdi->rd", dirs, N)
    Nperp = N - rn[..., None] * dirs[None]
    return eta0 * Nperp - np.cross(dirs[None], L)


def rcs(m: RWGMesh, j, dirs, k0, eta0, pol=None):
    """Bistatic RCS sigma (wavelength^2) per (rhs, dir); total |E_s|^2, or the
    component along unit vectors ``pol`` (ndir, 3) if given."""
    F = far_field(m, j, dirs, k0, eta0)
    if pol is not None:
        F = np.einsum("rdi,di->rd", F, np.atleast_2d(pol))[..., None]
    return k0 ** 2 / (4 * np.pi) * (np.abs(F) ** 2).sum(axis=-1)


def monostatic_rcs(m: RWGMesh, j, inc, k0, eta0):
    """Co-polarised monostatic RCS: direction -k, polarisation p, per RHS."""
    inc = np.atleast_2d(inc)
    out = np.zeros(len(inc))
    for c, row in enumerate(inc):
        d = -row[None, :3]
        F = far_field(m, j[:, c:c + 1], d, k0, eta0)[0, 0]
        out[c] = k0 ** 2 / (4 * np.pi) * abs(F @ row[3:]) ** 2
    return out
