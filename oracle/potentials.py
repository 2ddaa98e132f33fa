"""Closed-form surface integrals over a flat triangle Q for an observation
point r, used to extract the singular part of the Green's function on near
triangle pairs.  The paper says only that K is a principal-value and T a
finite-part integral (operator definitions, Sec. II-A); these are the
classical potential integrals (Wilton et al. 1984; Graglia 1993), derived
here from the divergence theorem in the plane of Q:

With n the unit normal of Q, d = n . (r - v0) the signed height, rho the
projection of r on the plane, and for each directed edge i (v_i -> v_{i+1},
counter-clockwise about n) the unit tangent t_i, outward in-plane normal
u_i = t_i x n, t0_i = (v_i - rho) . u_i, l+- = (end/start - rho) . t_i,
R+- = |r - end/start|, R0^2 = t0^2 + d^2, f_i = ln((R+ + l+)/(R- + l-)),
beta_i = atan2(t0 l+, R0^2 + |d| R+) - atan2(t0 l-, R0^2 + |d| R-):

  int 1/R           = sum t0 f - |d| sum beta
  int R             = (d^2 int 1/R + sum t0 F1) / 3,   F1 = int_edge R dl
  int (rho'-rho)/R  = sum u F1
  int (rho'-rho) R  = sum u F3 / 3,                    F3 = int_edge R^3 dl
  int (r - r')/R^3  = sum u f + sign(d) n sum beta
with F1 = (l+R+ - l-R-)/2 + R0^2 f / 2 and
     F3 = (l+R+^3 - l-R-^3)/4 + 3 R0^2 (l+R+ - l-R-)/8 + 3 R0^4 f / 8.

All functions are vectorised: ``r`` is (..., 3) and ``tri`` (..., 3, 3).
"""
from __future__ import annotations

import numpy as np


def _edge_terms(r, tri):
    v0 = tri[..., 0, :]
    e1 = tri[..., 1, :] - v0
    e2 = tri[..., 2, :] - v0
    n = np.cross(e1, e2)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    d = np.einsum("...i,...i->...", r - v0, n)
    rho = r - d[..., None] * n
    out = []
    for i in range(3):
        a = tri[..., i, :]
        b = tri[..., (i + 1) % 3, :]
        L = np.linalg.norm(b - a, axis=-1)
        t = (b - a) / L[..., None]
        u = np.cross(t, n)
        t0 = np.einsum("...i,...i->...", a - rho, u)
        lp = np.einsum("...i,...i->...", b - rho, t)
        lm = np.einsum("...i,...i->...", a - rho, t)
        Rp = np.linalg.norm(r - b, axis=-1)
        Rm = np.linalg.norm(r - a, axis=-1)
        R02 = t0 * t0 + d * d
        # f = ln((R+ + l+)/(R- + l-)) = ln((R- - l-)/(R+ - l+)), whichever
        # form avoids cancellation
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((Rp + lp) / (Rm + lm))
            f_neg = np.log((Rm - lm) / (Rp - lp))
            f_mid = np.log((Rp + lp) * (Rm - lm) / R02)
        f = np.where(lm >= 0, f_pos, np.where(lp <= 0, f_neg, f_mid))
        ad = np.abs(d)
        beta = (np.arctan2(t0 * lp, R02 + ad * Rp) - np.arctan2(t0 * lm, R02 + ad * Rm))
        F1 = 0.5 * (lp * Rp - lm * Rm) + 0.5 * R02 * f
        F3 = (0.25 * (lp * Rp ** 3 - lm * Rm ** 3) + 0.375 * R02 * (lp * Rp - lm * Rm)
              + 0.375 * R02 * R02 * f)
        out.append(dict(u=u, t0=t0, f=f, beta=beta, F1=F1, F3=F3))
    return n, d, out


def triangle_potentials(r, tri):
    """Return a dict of the integrals over triangle ``tri`` of
    1/R ('Im1'), R ('I1'), (r'-r)/R ('Vm1'), (r'-r) R ('V1') and
    (r-r')/R^3 ('Gm3'), with R = |r - r'|."""
    n, d, E = _edge_terms(r, tri)
    sbeta = sum(e["beta"] for e in E)
    Im1 = sum(e["t0"] * e["f"] for e in E) - np.abs(d) * sbeta
    I1 = (d * d * Im1 + sum(e["t0"] * e["F1"] for e in E)) / 3.0
    pm1 = sum(e["u"] * e["F1"][..., None] for e in E)          # int (rho'-rho)/R
    p1 = sum(e["u"] * e["F3"][..., None] for e in E) / 3.0     # int (rho'-rho) R
    # r' - r = (rho' - rho) - d n
    Vm1 = pm1 - (d * Im1)[..., None] * n
    V1 = p1 - (d * I1)[..., None] * n
    Gm3 = sum(e["u"] * e["f"][..., None] for e in E) + (np.sign(d) * sbeta)[..., None] * n
    return dict(Im1=Im1, I1=I1, Vm1=Vm1, V1=V1, Gm3=Gm3, n=n, d=d)
