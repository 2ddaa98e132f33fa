"""Cell division of a mesh's RWG edges (Sec. III-A: every edge lies in exactly
one cell).  The paper shows a division figure but states no rule, so two
deterministic rules are provided:

* ``octant_blocks``: cell = sign pattern of the edge midpoint (x, y, z); a
  coordinate with ``|c| < 1e-12 * scale`` counts as positive.  Eight cells.
* ``rcb_blocks``: recursive coordinate bisection of edge midpoints.  A set of
  edges destined for ``n`` cells is split along the longest axis of its
  midpoints' bounding box (ties x < y < z); edges are sorted by
  (coordinate, edge id) and the first ``round(|E| * (n // 2) / n)`` go left
  with ``n // 2`` cells, the rest right with ``n - n // 2`` cells.  Cells are
  numbered left-first.  Gives exactly ``n`` non-empty cells when |E| >= n.

Both return an int32 array, one cell id per edge in canonical edge order
(:func:`synth.meshes.edges_canonical`).  Input generation only.
"""
from __future__ import annotations

import numpy as np

from .meshes import edges_canonical


def edge_midpoints(V, T):
    E = edges_canonical(T)
    return (V[E[:, 0]] + V[E[:, 1]]) / 2.0


def octant_blocks(V, T) -> np.ndarray:
    M = edge_midpoints(V, T)
    scale = np.abs(V).max()
    pos = M >= -1e-12 * scale
    return (pos[:, 0] * 1 + pos[:, 1] * 2 + pos[:, 2] * 4).astype(np.int32)


def rcb_blocks(V, T, n: int) -> np.ndarray:
    M = edge_midpoints(V, T)
    out = np.empty(len(M), dtype=np.int32)

    def split(ids, ncell, first):
        if ncell == 1:
            out[ids] = first
            return
        P = M[ids]
        ext = P.max(axis=0) - P.min(axis=0)
        ax = int(np.argmax(ext))  # argmax returns the first maximum: x < y < z
        order = np.lexsort((ids, P[:, ax]))
        ids = ids[order]
        nl = ncell // 2
        cut = int(round(len(ids) * nl / ncell))
        split(ids[:cut], nl, first)
        split(ids[cut:], ncell - nl, first + nl)

    split(np.arange(len(M)), n, 0)
    return out
