"""Closed triangle meshes of the scatterer classes the paper studies.

The paper's numerical section uses spheres (icosahedral tessellation), cubes
(square faces split into two triangles) and a connected circular cylinder
(Sec. IV-A, IV-B, IV-C).  Its mesh files are not published, so these
generators build meshes of the same classes from closed-form vertex sets.

Every generator returns ``(V, T)``: ``V`` is an ``(nv, 3)`` float64 array of
vertex coordinates in units of the free-space wavelength, ``T`` an ``(nt, 3)``
int32 array of vertex indices, each triangle ordered counter-clockwise when
seen from outside (so ``(v1 - v0) x (v2 - v0)`` is the outward normal).

This module is input generation only: topology and coordinates.  It holds no
integral-equation arithmetic and is shared by the CPU oracle and the GPU path.
"""
from __future__ import annotations

import numpy as np


def _orient_outward(V: np.ndarray, T: np.ndarray, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Flip triangles whose normal points towards ``centre`` (star-shaped bodies)."""
    c = np.asarray(centre, dtype=np.float64)
    a, b, d = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, d - a)
    mid = (a + b + d) / 3.0 - c
    flip = np.einsum("ij,ij->i", n, mid) < 0
    T = T.copy()
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def icosphere(level: int, radius: float = 1.0):
    """Icosahedron refined ``level`` times by midpoint subdivision, re-projected
    onto the sphere after each level: 20*4**level triangles.

    level 2 gives the paper's 320-triangle / 960-unknown sphere (Sec. IV-A).
    """
    p = (1.0 + np.sqrt(5.0)) / 2.0
    V = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            V += [(0.0, s1, s2 * p), (s1, s2 * p, 0.0), (s2 * p, 0.0, s1)]
    V = np.array(V, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # faces: every triple of mutually adjacent vertices (edge length 2/|v|)
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    emin = d[d > 1e-9].min()
    adj = np.abs(d - emin) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    T = np.array(faces, dtype=np.int64)
    assert T.shape == (20, 3)
    verts = [tuple(v) for v in V]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = (np.asarray(verts[i]) + np.asarray(verts[j])) / 2.0
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        newT = []
        for (a, b, c) in T:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newT += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        T = np.array(newT, dtype=np.int64)
    V = np.array(verts, dtype=np.float64) * radius
    T = _orient_outward(V, T)
    return V, T.astype(np.int32)


def geodesic(n: int, radius: float = 1.0):
    """Icosahedron with every face split into an n x n triangular grid, the
    grid points projected onto the sphere: 20 n^2 triangles (frequency-n
    geodesic sphere).  Points shared by faces are merged exactly: each is
    keyed by its integer barycentric weights on the icosahedron vertices."""
    V0, T0 = icosphere(0, 1.0)
    index, verts, tris = {}, [], []

    def vid(a, b, c, i, j):
        w = {}
        for v, wt in ((a, n - i - j), (b, i), (c, j)):
            if wt:
                w[int(v)] = w.get(int(v), 0) + wt
        key = tuple(sorted(w.items()))
        if key not in index:
            p = (V0[a] * (n - i - j) + V0[b] * i + V0[c] * j) / n
            index[key] = len(verts)
            verts.append(p / np.linalg.norm(p))
        return index[key]

    for a, b, c in T0:
        for i in range(n):
            for j in range(n - i):
                tris.append((vid(a, b, c, i, j), vid(a, b, c, i + 1, j), vid(a, b, c, i, j + 1)))
                if i + j + 1 < n:
                    tris.append((vid(a, b, c, i + 1, j), vid(a, b, c, i + 1, j + 1), vid(a, b, c, i, j + 1)))
    V = np.array(verts, dtype=np.float64) * radius
    T = _orient_outward(V, np.array(tris, dtype=np.int64))
    return V, T.astype(np.int32)


def cube(n: int, edge: float = 1.0):
    """Cube [-edge/2, edge/2]^3; each face an n x n grid of squares, each square
    split along its face-local (i, j) -> (i+1, j+1) diagonal: 12 n^2 triangles.

    n = 12 gives 1,728 triangles / 2,592 edges / 5,184 unknowns.
    """
    index = {}
    verts = []

    def vid(ijk):
        if ijk not in index:
            index[ijk] = len(verts)
            verts.append(ijk)
        return index[ijk]

    tris = []
    for axis in range(3):
        for side in (0, n):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            for i in range(n):
                for j in range(n):
                    def lat(a, b):
                        p = [0, 0, 0]
                        p[axis] = side
                        p[u_ax] = a
                        p[v_ax] = b
                        return vid(tuple(p))
                    q00, q10 = lat(i, j), lat(i + 1, j)
                    q11, q01 = lat(i + 1, j + 1), lat(i, j + 1)
                    tris.append((q00, q10, q11))
                    tris.append((q00, q11, q01))
    V = (np.array(verts, dtype=np.float64) / n - 0.5) * edge
    T = _orient_outward(V, np.array(tris, dtype=np.int64))
    return V, T.astype(np.int32)


def _zip_rings(inner, outer, ang_in, ang_out):
    """Triangulate the annulus between two concentric closed rings of vertex
    ids sorted by angle, advancing along whichever ring's next vertex comes
    first in angle (inner ring first on ties)."""
    tris = []
    ni, no = len(inner), len(outer)
    i = o = 0
    while i < ni or o < no:
        a_i = ang_in[(i + 1) % ni] + (2 * np.pi if i + 1 >= ni else 0.0)
        a_o = ang_out[(o + 1) % no] + (2 * np.pi if o + 1 >= no else 0.0)
        if o >= no or (i < ni and a_i <= a_o):
            tris.append((inner[i % ni], outer[o % no], inner[(i + 1) % ni]))
            i += 1
        else:
            tris.append((inner[i % ni], outer[o % no], outer[(o + 1) % no]))
            o += 1
    return tris


def cylinder(K: int, n_h: int, radius: float = 1.0, height: float = 6.0):
    """Closed circular cylinder along z, centred at the origin.

    The side is a (6K) x n_h grid of quads (two triangles each); each cap is a
    disk of K concentric rings with 6k vertices on ring k (the rim, ring K, is
    shared with the side) plus the centre: 12 K^2 + 12 K n_h triangles.

    K = 16, n_h = 88, radius 1, height 6 gives 19,968 triangles.
    """
    nc = 6 * K
    verts = []
    tris = []
    ang_rim = 2 * np.pi * np.arange(nc) / nc
    rows = []
    for h in range(n_h + 1):
        z = -height / 2 + height * h / n_h
        ids = []
        for a in ang_rim:
            ids.append(len(verts))
            verts.append((radius * np.cos(a), radius * np.sin(a), z))
        rows.append(ids)
    for h in range(n_h):
        lo, hi = rows[h], rows[h + 1]
        for i in range(nc):
            j = (i + 1) % nc
            tris.append((lo[i], lo[j], hi[j]))
            tris.append((lo[i], hi[j], hi[i]))
    for z, rim in ((-height / 2, rows[0]), (height / 2, rows[-1])):
        centre = len(verts)
        verts.append((0.0, 0.0, z))
        prev_ids, prev_ang = [centre], np.array([0.0])
        for k in range(1, K + 1):
            if k == K:
                ids, ang = rim, ang_rim
            else:
                ang = 2 * np.pi * np.arange(6 * k) / (6 * k)
                r = radius * k / K
                ids = []
                for a in ang:
                    ids.append(len(verts))
                    verts.append((r * np.cos(a), r * np.sin(a), z))
            if k == 1:
                for i in range(6):
                    tris.append((centre, ids[i], ids[(i + 1) % 6]))
            else:
                tris += _zip_rings(prev_ids, ids, prev_ang, ang)
            prev_ids, prev_ang = ids, ang
    V = np.array(verts, dtype=np.float64)
    T = np.array(tris, dtype=np.int64)
    # orientation: side/caps are convex pieces of a convex body
    T = _orient_outward(V, T)
    return V, T.astype(np.int32)


def edges_canonical(T: np.ndarray) -> np.ndarray:
    """Unique undirected edges as (min v, max v), sorted lexicographically.

    This is the canonical RWG order used by every interface in this project:
    edge e of the mesh is row e of this array.
    """
    T = np.asarray(T, dtype=np.int64)
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    return np.unique(e, axis=0)
