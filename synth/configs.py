"""Seeded synthetic workloads shaped like the paper's experiments.

Units: free-space wavelength lambda0 = 1, so k0 = 2 pi.  Exterior medium is
vacuum, interior (eps_r, mu_r = 1).  An incidence is a row
``(kx, ky, kz, px, py, pz)``: unit propagation direction k and unit
polarisation p (p . k = 0), amplitude 1, phase reference at the origin.

Only geometry, block ids and directions are produced here; every
integral-equation quantity is computed separately by the oracle and by the
GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .blocks import octant_blocks, rcb_blocks
from .meshes import cube, cylinder, edges_canonical, geodesic, icosphere

ETA0 = 376.730313668  # free-space wave impedance (ohm); passed to both sides


def sph_dir(theta, phi):
    """Unit vector r(theta, phi) and the spherical unit vectors theta, phi."""
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    r = np.stack([st * cp, st * sp, ct], axis=-1)
    th = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ph = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    return r, th, ph


def generating_set(theta_s=0.0, dtheta=30.0, n_theta=12, phi_s=0.0, dphi=30.0,
                   n_phi=6, pols=("theta", "phi")) -> np.ndarray:
    """Plane waves used to generate CBFs (eq. for the spherical sampling and
    Table I): propagation along r(theta, phi) for theta = theta_s + i dtheta,
    i < n_theta, phi = phi_s + j dphi, j < n_phi; polarisation theta-hat
    and/or phi-hat.  Table I defaults give s = 12 * 6 * 2 = 144 waves.
    Column order: theta index slowest, then phi, then polarisation.
    """
    rows = []
    for i in range(n_theta):
        for j in range(n_phi):
            th = np.deg2rad(theta_s + i * dtheta)
            ph = np.deg2rad(phi_s + j * dphi)
            r, t, p = sph_dir(np.array(th), np.array(ph))
            for pol in pols:
                rows.append(np.concatenate([r, t if pol == "theta" else p]))
    return np.array(rows, dtype=np.float64)


def random_incidences(n: int, seed: int) -> np.ndarray:
    """Arrival directions d = normalise(N(0, I3)); k = -d, p = theta-hat(d)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    _, th, _ = sph_dir(theta, phi)
    return np.concatenate([-d, th], axis=1)


def random_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex normal entries (real and imaginary parts N(0, 1/2)):
    stand-in coefficient sets for tests that need matrices of a given shape
    and no particular physics (imported CBFs, current sets, perturbations)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def random_cell_sets(sizes, cols: int, seed: int):
    """One (N_m x cols) pair of seeded complex normal matrices per cell size
    N_m in ``sizes`` (cell after cell, one seed for all)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        a = (rng.standard_normal((n, cols)) + 1j * rng.standard_normal((n, cols))) / np.sqrt(2.0)
        b = (rng.standard_normal((n, cols)) + 1j * rng.standard_normal((n, cols))) / np.sqrt(2.0)
        out.append((a, b))
    return out


@dataclass
class Workload:
    name: str
    V: np.ndarray
    T: np.ndarray
    edge_block: np.ndarray
    nblocks: int
    eps_r: complex
    mu_r: complex
    inc: np.ndarray            # (nrhs, 6)
    gen: np.ndarray            # (s, 6) CBF generating waves
    delta_svd: float = 1e-3
    k0: float = 2 * np.pi
    eta0: float = ETA0
    extra: dict = field(default_factory=dict)

    @property
    def nt(self):
        return len(self.T)


def sphere_c1() -> Workload:
    """Dielectric sphere radius 0.5, eps_r 4, 320 triangles, octant cells,
    one x-polarised plane wave travelling along -z."""
    V, T = icosphere(2, 0.5)
    return Workload("sphere320_er4", V, T, octant_blocks(V, T), 8, 4.0 + 0j, 1.0 + 0j,
                    np.array([[0, 0, -1, 1, 0, 0]], dtype=np.float64), generating_set())


def cube_c2(nrhs: int = 64) -> Workload:
    """Dielectric cube edge 1, eps_r 2.5, 12x12 squares per face (1728 tri),
    27 RCB cells, 64 seeded incidences."""
    V, T = cube(12, 1.0)
    return Workload("cube1728_er2.5", V, T, rcb_blocks(V, T, 27), 27, 2.5 + 0j, 1.0 + 0j,
                    random_incidences(nrhs, 2111), generating_set())


def sphere_c3() -> Workload:
    """Lossy sphere radius 2, eps_r 4 - 0.1j, 5120 tri, 64 RCB cells."""
    V, T = icosphere(4, 2.0)
    return Workload("sphere5120_er4-0.1j", V, T, rcb_blocks(V, T, 64), 64, 4.0 - 0.1j, 1.0 + 0j,
                    np.array([[0, 0, -1, 1, 0, 0]], dtype=np.float64), generating_set())


def cylinder_c5() -> Workload:
    """Cylinder r 1, h 6, eps_r 3, 19,968 tri, 96 RCB cells, 32 monostatic
    theta-polarised incidences over theta = 45 deg * k / 31, phi = 0."""
    V, T = cylinder(16, 88, 1.0, 6.0)
    th = np.deg2rad(45.0 * np.arange(32) / 31.0)
    r, t, _ = sph_dir(th, np.zeros_like(th))
    inc = np.concatenate([-r, t], axis=1)
    return Workload("cylinder19968_er3", V, T, rcb_blocks(V, T, 96), 96, 3.0 + 0j, 1.0 + 0j,
                    inc, generating_set())


def sphere_array(nx: int = 4, ny: int = 4, nz: int = 2, pitch: float = 0.5, eps_r: complex = 3.0 + 0j,
                 level: int = 2) -> Workload:
    """The paper's sphere array (Sec. IV-A, 4 x 4 x 2 spheres): copies of the
    single-cell sphere (radius lambda/6, 320 triangles, 960 unknowns) at a
    centre pitch of lambda/2 along x, y and z, centred on the origin; one
    cell per sphere; one theta-polarised wave travelling along -z (x
    polarisation); the Table I generating waves.  The paper keeps 70 CBFs per
    current per cell (the singular-value groups l = 1..5): ``extra["max_L"]``
    and ``delta_svd = 0``.  ``level`` < 2 gives coarser spheres (level 1: 80
    triangles) for tests small enough for the oracle."""
    V0, T0 = icosphere(level, 1.0 / 6.0)
    Vs, Ts = [], []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                off = pitch * np.array([ix - (nx - 1) / 2, iy - (ny - 1) / 2, iz - (nz - 1) / 2])
                Ts.append(T0 + len(V0) * len(Vs))
                Vs.append(V0 + off)
    V, T = np.concatenate(Vs), np.concatenate(Ts).astype(T0.dtype)
    # an edge's cell is the sphere of its vertices
    blocks = (edges_canonical(T)[:, 0] // len(V0)).astype(np.int32)
    return Workload(f"sphere_array{nx}x{ny}x{nz}_er{eps_r.real:g}", V, T, blocks, nx * ny * nz, eps_r, 1.0 + 0j,
                    np.array([[0, 0, -1, 1, 0, 0]], dtype=np.float64), generating_set(), delta_svd=0.0,
                    extra={"max_L": 70})


# Table II (cube array): (dtheta, N_theta, dphi, N_phi) of the generating
# waves and the singular-value group l kept, per condition 1..6
CUBE_ARRAY_CONDITIONS = {1: (30.0, 12, 30.0, 6, 4), 2: (30.0, 12, 30.0, 6, 5), 3: (30.0, 12, 30.0, 6, 6),
                         4: (10.0, 36, 10.0, 18, 4), 5: (10.0, 36, 10.0, 18, 5), 6: (10.0, 36, 10.0, 18, 6)}


def cube_array(condition: int = 6, nx: int = 8, ny: int = 2, nz: int = 2, pitch: float = 0.5,
               eps_r: complex = 3.0 + 0j) -> Workload:
    """The paper's cube array (Sec. IV-B): 8 x 2 x 2 cubes of edge 0.4
    lambda (12 mm at lambda = 30 mm) meshed with 6 x 6 squares per face (432
    triangles, 1296 unknowns each) at a centre pitch of lambda/2, one cell per
    cube, eps_r 3, one theta-polarised wave along -z.  The generating waves
    and the CBFs kept per current follow Table II: groups l = 1..L of sizes
    2 (2 l + 1), i.e. 48, 70 or 96 CBFs for L = 4, 5, 6."""
    dth, nth, dph, nph, lmax = CUBE_ARRAY_CONDITIONS[condition]
    V0, T0 = cube(6, 0.4)
    Vs, Ts = [], []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                off = pitch * np.array([ix - (nx - 1) / 2, iy - (ny - 1) / 2, iz - (nz - 1) / 2])
                Ts.append(T0 + len(V0) * len(Vs))
                Vs.append(V0 + off)
    V, T = np.concatenate(Vs), np.concatenate(Ts).astype(T0.dtype)
    blocks = (edges_canonical(T)[:, 0] // len(V0)).astype(np.int32)
    gen = generating_set(0.0, dth, nth, 0.0, dph, nph)
    max_L = sum(2 * (2 * l + 1) for l in range(1, lmax + 1))
    return Workload(f"cube_array{nx}x{ny}x{nz}_cond{condition}", V, T, blocks, nx * ny * nz, eps_r, 1.0 + 0j,
                    np.array([[0, 0, -1, 1, 0, 0]], dtype=np.float64), gen, delta_svd=0.0,
                    extra={"max_L": max_L})


def small_cylinder(K=2, n_h=4, nblocks=4, eps_r=3.0 + 0j) -> Workload:
    V, T = cylinder(K, n_h, 0.3, 0.8)
    return Workload(f"cyl{len(T)}", V, T, rcb_blocks(V, T, nblocks), nblocks, eps_r, 1.0 + 0j,
                    random_incidences(3, 7), generating_set())


# ---------------------------------------------------------------- serving
@dataclass
class ServeRequest:
    t_arrival: float     # seconds after the stream starts
    shape: str
    unknowns: int
    work: Workload


def _serve_ladder():
    """(shape, unknowns, mesh parameters) of the sizes a request may take:
    sphere r 0.5 (icosphere-2, geodesic n = 5..11), cube edge 1 (n = 6..14
    squares per face edge), cylinder r 0.5, h 2 (K = 3..6 rings, rows
    keeping the side squares near unit aspect)."""
    lad = {"sphere": [(960, ("ico", 2))] + [(60 * n * n, ("geo", n)) for n in range(5, 12)],
           "cube": [(36 * n * n, ("cube", n)) for n in range(6, 15)],
           "cylinder": []}
    for K in range(3, 7):
        nh = int(round(2.0 * 6 * K / np.pi))
        lad["cylinder"].append((3 * (12 * K * nh + 12 * K * K), ("cyl", K, nh)))
    return lad


_SERVE_MESHES = {}


def _serve_mesh(spec):
    if spec not in _SERVE_MESHES:
        if spec[0] == "ico":
            V, T = icosphere(spec[1], 0.5)
        elif spec[0] == "geo":
            V, T = geodesic(spec[1], 0.5)
        elif spec[0] == "cube":
            V, T = cube(spec[1], 1.0)
        else:
            V, T = cylinder(spec[1], spec[2], 0.5, 2.0)
        ne = 3 * len(T) // 2
        nb = max(1, int(round(ne / 100.0)))
        _SERVE_MESHES[spec] = (V, T, rcb_blocks(V, T, nb), nb)
    return _SERVE_MESHES[spec]


def serving_stream(n_requests: int = 512, seed: int = 2113, rate: float = 200.0, max_unknowns: float = 8000.0):
    """Seeded request stream: Poisson arrivals at `rate` per second, shape
    uniform over sphere / cube / cylinder, target unknowns uniform in
    [960, max_unknowns] snapped to the nearest size of the shape's ladder,
    eps_r uniform in [1.5, 6], 1-16 seeded incidences, RCB cells of about
    100 edges, the Table-I generating waves."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    lad = _serve_ladder()
    out = []
    for i in range(n_requests):
        shape = ("sphere", "cube", "cylinder")[int(rng.integers(3))]
        target = rng.uniform(960.0, max_unknowns)
        eps = float(rng.uniform(1.5, 6.0))
        nrhs = int(rng.integers(1, 17))
        iseed = int(rng.integers(1 << 31))
        opts = [(u, spec) for u, spec in lad[shape] if u <= max_unknowns] or lad[shape][:1]
        u, spec = min(opts, key=lambda o: abs(o[0] - target))
        V, T, eb, nb = _serve_mesh(spec)
        w = Workload(f"{shape}{len(T)}_er{eps:.2f}", V, T, eb, nb, eps + 0j, 1.0 + 0j,
                     random_incidences(nrhs, iseed), generating_set())
        out.append(ServeRequest(float(t[i]), shape, u, w))
    return out
