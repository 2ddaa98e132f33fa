import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs longer than a few seconds")


_cache = {}


def oracle_problem(name):
    """Oracle fill of a named small workload, cached per test session."""
    if name in _cache:
        return _cache[name]
    from oracle import excitation, fill, mesh
    from synth import configs
    from synth.meshes import icosphere
    if name == "x1_er3":
        V, T = icosphere(2, 1.0 / 6.0)
        w = configs.Workload("x1", V, T, np.zeros(480, np.int32), 1, 3.0 + 0j, 1.0 + 0j,
                             np.array([[0, 0, -1, 1, 0, 0.0]]), configs.generating_set())
    elif name == "c1":
        w = configs.sphere_c1()
    elif name == "cyl_small":
        w = configs.small_cylinder()
    elif name == "cyl_lossy":
        w = configs.small_cylinder(eps_r=4.0 - 0.1j)
    elif name == "array2":
        w = configs.sphere_array(2, 1, 1, level=1)
    else:
        raise KeyError(name)
    m = mesh.build(w.V, w.T)
    k, eta = fill.media(w.k0, w.eta0, w.eps_r, w.mu_r)
    Kop, T1, T2 = fill.fill_ops(m, k)
    Kc, TE, TH = fill.combine(Kop, T1, T2, eta)
    out = dict(w=w, m=m, k=k, eta=eta, Kop=Kop, T1=T1, T2=T2, Kc=Kc, TE=TE, TH=TH,
               Z=fill.assemble_Z(Kc, TE, TH), v=excitation.rhs(m, w.inc, w.k0, w.eta0))
    _cache[name] = out
    return out
