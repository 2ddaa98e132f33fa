"""Seven-point degree-5 symmetric triangle rule (Radon's rule, as tabulated by
Strang & Fix and Dunavant).  The paper does not name its quadrature; this is
the reading used for the fill, the incident-field vectors and the far field.

Barycentric points and weights (weights sum to 1; multiply by the area):
  centroid (1/3, 1/3, 1/3)                            weight 9/40
  (1-2a, a, a) and rotations, a = (6 - sqrt 15)/21    weight (155 - sqrt 15)/1200
  (1-2b, b, b) and rotations, b = (6 + sqrt 15)/21    weight (155 + sqrt 15)/1200
"""
import numpy as np

_s15 = np.sqrt(15.0)
_a = (6.0 - _s15) / 21.0
_b = (6.0 + _s15) / 21.0
_wa = (155.0 - _s15) / 1200.0
_wb = (155.0 + _s15) / 1200.0

BARY = np.array([
    [1 / 3, 1 / 3, 1 / 3],
    [1 - 2 * _a, _a, _a], [_a, 1 - 2 * _a, _a], [_a, _a, 1 - 2 * _a],
    [1 - 2 * _b, _b, _b], [_b, 1 - 2 * _b, _b], [_b, _b, 1 - 2 * _b],
], dtype=np.float64)
WEIGHTS = np.array([9 / 40, _wa, _wa, _wa, _wb, _wb, _wb], dtype=np.float64)


def points(tri_xyz: np.ndarray) -> np.ndarray:
    """Quadrature points of triangles ``tri_xyz`` (n, 3 vertices, 3) -> (n, 7, 3)."""
    return np.einsum("qa,nai->nqi", BARY, tri_xyz)
