"""RWG tables of a closed triangle mesh (the basis f of Sec. II-B, after
Rao, Wilton and Glisson).

Canonical conventions (shared with the GPU library by specification, not by
code):
* edges are the unique undirected vertex pairs (min v, max v), sorted
  lexicographically; edge e is RWG function e;
* T+ of an edge is the triangle whose counter-clockwise (outward) vertex
  cycle traverses the edge from its smaller to its larger vertex id; T- is
  the other one;
* on triangle P, local function a has free vertex p_a = vertex a of P and
  lives on the edge opposite that vertex; f = s (l / 2A) (r - p_a) with
  s = +1 on T+ and -1 on T-, so the current flows from T+ into T-.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class RWGMesh:
    V: np.ndarray          # (nv, 3)
    T: np.ndarray          # (nt, 3)
    edges: np.ndarray      # (ne, 2) canonical
    tplus: np.ndarray      # (ne,)
    tminus: np.ndarray     # (ne,)
    aplus: np.ndarray      # (ne,) local index of the free vertex in T+
    aminus: np.ndarray     # (ne,)
    length: np.ndarray     # (ne,)
    tri_edge: np.ndarray   # (nt, 3) edge of local function a
    tri_sign: np.ndarray   # (nt, 3) +1 / -1
    xyz: np.ndarray        # (nt, 3, 3) vertex coordinates per triangle
    area: np.ndarray       # (nt,)
    normal: np.ndarray     # (nt, 3) unit outward normal

    @property
    def nt(self):
        return len(self.T)

    @property
    def ne(self):
        return len(self.edges)


def build(V, T) -> RWGMesh:
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    nt = len(T)
    # local function a <-> edge opposite vertex a: (v_{a+1}, v_{a+2})
    directed = np.stack([np.stack([T[:, (a + 1) % 3], T[:, (a + 2) % 3]], axis=1)
                         for a in range(3)], axis=1)          # (nt, 3, 2)
    lo = directed.min(axis=2)
    hi = directed.max(axis=2)
    keys = np.stack([lo.ravel(), hi.ravel()], axis=1)
    edges, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    if np.any(counts != 2):
        raise ValueError("mesh is not a closed 2-manifold (edge used by != 2 triangles)")
    inv = inv.reshape(nt, 3)
    forward = (directed[:, :, 0] == lo)                       # traverses min -> max
    ne = len(edges)
    tplus = np.full(ne, -1)
    tminus = np.full(ne, -1)
    aplus = np.full(ne, -1)
    aminus = np.full(ne, -1)
    for t in range(nt):
        for a in range(3):
            e = inv[t, a]
            if forward[t, a]:
                if tplus[e] >= 0:
                    raise ValueError("inconsistent orientation")
                tplus[e], aplus[e] = t, a
            else:
                if tminus[e] >= 0:
                    raise ValueError("inconsistent orientation")
                tminus[e], aminus[e] = t, a
    if np.any(tplus < 0) or np.any(tminus < 0):
        raise ValueError("inconsistent orientation")
    sign = np.where(forward, 1, -1)
    xyz = V[T]
    cr = np.cross(xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0])
    dbl = np.linalg.norm(cr, axis=1)
    length = np.linalg.norm(V[edges[:, 0]] - V[edges[:, 1]], axis=1)
    return RWGMesh(V, T, edges, tplus, tminus, aplus, aminus, length, inv, sign,
                   xyz, dbl / 2.0, cr / dbl[:, None])


def near_pairs(m: RWGMesh, alpha: float = 1.5) -> np.ndarray:
    """Triangle pairs (P, Q) given the singular treatment: P == Q, or P and Q
    share a vertex, or |c_P - c_Q|^2 < alpha^2 max(h_P^2, h_Q^2) with c the
    centroid and h the longest edge.  The paper only says the operators are
    principal-value / finite-part integrals; this near set is the reading.
    Returns an (n, 2) int array sorted by (P, Q)."""
    c = m.xyz.mean(axis=1)
    e = m.xyz[:, [1, 2, 0]] - m.xyz
    h2 = (e * e).sum(axis=2).max(axis=1)
    out = set()
    for p in range(m.nt):
        d = c - c[p]
        d2 = (d * d).sum(axis=1)
        thr = alpha * alpha * np.maximum(h2, h2[p])
        out.update((p, int(q)) for q in np.nonzero(d2 < thr)[0])
    # vertex sharing (may reach beyond the distance test on skewed meshes)
    vt = {}
    for t, tri in enumerate(m.T.tolist()):
        for v in tri:
            vt.setdefault(v, []).append(t)
    for ts in vt.values():
        for p in ts:
            for q in ts:
                out.add((p, q))
    return np.array(sorted(out), dtype=np.int64)


def coplanar(m: RWGMesh, p: int, q: int) -> bool:
    """P and Q lie in one plane (normals parallel and Q's centroid in P's
    plane), decided with absolute tolerances far from any value the meshes
    of this project produce for non-coplanar pairs."""
    n1, n2 = m.normal[p], m.normal[q]
    cr = np.cross(n1, n2)
    if (cr * cr).sum() > 1e-20:
        return False
    h = np.sqrt(m.area[p])
    dc = m.xyz[q].mean(axis=0) - m.xyz[p].mean(axis=0)
    return abs((n1 * dc).sum()) <= 1e-10 * h
