"""Writes sphere5120_oracle_rcs.txt: the oracle's CBFM RCS of the lossy
precision workload (radius 2 wavelengths, eps_r = 4 - 0.1j, 5,120
triangles, 15,360 unknowns, 64 cells, the Table-I generating waves,
delta_SVD 1e-3; one x-polarised wave along -z): the monostatic
co-polarised RCS and the bistatic RCS (total field) at theta = 0..180 deg
by 10 deg, phi = 0, in wavelength^2.  Calls only oracle/ and synth/ (the
dense FP64 fill in worker processes, then the CBF build, the projection and
an LU solve of the reduced system, Sec. III).  Takes several minutes.

    python tests/golden/make_sphere5120_rcs.py [workers]
"""
import os
import sys
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cbf, excitation, fill, mesh, reduced  # noqa: E402
from synth import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere5120_oracle_rcs.txt")


def _rows(args):
    rows = args
    w = configs.sphere_c3()
    m = mesh.build(w.V, w.T)
    k, _ = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    return rows, fill.fill_rows(m, k, rows)


def bistatic_dirs():
    th = np.deg2rad(np.arange(0.0, 181.0, 10.0))
    return np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else min(8, os.cpu_count() or 1)
    w = configs.sphere_c3()
    m = mesh.build(w.V, w.T)
    k, eta = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    ne = m.ne
    chunks = np.array_split(np.arange(ne), 4 * workers)
    Kop = np.zeros((ne, ne), np.complex128)
    T1 = np.zeros_like(Kop)
    T2 = np.zeros_like(Kop)
    with get_context("fork").Pool(workers) as pool:
        for rows, (a, b, c) in pool.imap_unordered(_rows, chunks):
            Kop[rows], T1[rows], T2[rows] = a, b, c
            print(f"rows {rows[0]}..{rows[-1]}", flush=True)
    Kc, TE, TH = fill.combine(Kop, T1, T2, eta)
    del Kop, T1, T2
    cb = cbf.build(m, Kc, TE, TH, w.edge_block, w.gen, w.k0, w.eta0, w.delta_svd)
    CJM, CMJ = reduced.cbf_matrices(cb, ne)
    Z = fill.assemble_Z(Kc, TE, TH)
    del Kc, TE, TH
    Zr = reduced.project(Z, CJM, CMJ)
    del Z
    v = excitation.rhs(m, w.inc, w.k0, w.eta0)
    j = CMJ @ np.linalg.solve(Zr, CJM.conj().T @ v)
    mono = excitation.monostatic_rcs(m, j, w.inc, w.k0, w.eta0)
    bi = excitation.rcs(m, j, bistatic_dirs(), w.k0, w.eta0)[0]
    with open(OUT, "w") as fh:
        fh.write("# oracle CBFM RCS (wavelength^2) of sphere5120_er4-0.1j: one x-polarised wave along -z;\n")
        fh.write(f"# N_CBF = {2 * sum(c.shape[1] for c in cb.CM)}; written by tests/golden/make_sphere5120_rcs.py\n")
        fh.write(f"monostatic {mono[0]:.17e}\n")
        for t, s in zip(np.arange(0, 181, 10), bi):
            fh.write(f"bistatic_theta_deg {t:d} {s:.17e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
