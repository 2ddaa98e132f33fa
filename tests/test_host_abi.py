"""Host-side tests of libcbfm that need no GPU: the C ABI loads and exports
every symbol include/cbfm.h declares; the host mesh tables (canonical
edges, RWG signs, near pairs, coplanar flags) equal the oracle's; invalid
meshes and arguments are rejected with the documented status codes."""
import os
import re

import numpy as np
import pytest

from oracle import mesh as om
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cb():
    from paper_2111_11058_amd import cbfm
    if not os.path.exists(cbfm.LIB_PATH):
        pytest.fail("libcbfm.so is not built (run __graft_entry__.build())")
    cbfm.lib()
    return cbfm


def test_exports_every_declared_symbol(cb):
    hdr = open(os.path.join(ROOT, "include", "cbfm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = sorted(set(re.findall(r"\b(cbfm_[a-z0-9_]+)\s*\(", hdr)))
    assert len(names) >= 17
    L = cb.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.cbfm_version() == 7


@pytest.mark.parametrize("make", [configs.sphere_c1, configs.cube_c2, configs.small_cylinder],
                         ids=["sphere320", "cube1728", "cylinder144"])
def test_host_tables_match_oracle(cb, make):
    w = make()
    E, TE, TS, N = cb.mesh_analyze(w.V, w.T, w.edge_block, w.nblocks)
    m = om.build(w.V, w.T)
    assert np.array_equal(E, m.edges)
    assert np.array_equal(TE, m.tri_edge)
    assert np.array_equal(TS, m.tri_sign)
    ref = om.near_pairs(m)
    assert np.array_equal(N[:, :2], ref)
    cop = np.array([p == q or om.coplanar(m, p, q) for p, q in ref])
    assert np.array_equal(N[:, 2].astype(bool), cop)


def _expect(cb, code, V, T, eb=None, nb=None):
    with pytest.raises(cb.CBFMError) as e:
        cb.mesh_analyze(V, T, eb, nb)
    assert e.value.code == code, str(e.value)


def test_invalid_meshes_rejected(cb):
    w = configs.sphere_c1()
    V, T = w.V, w.T
    flipped = T.copy()
    flipped[3] = flipped[3][::-1]
    _expect(cb, -2, V, flipped)                          # inconsistent orientation
    _expect(cb, -2, V, T[1:])                            # open surface
    inward = T[:, ::-1].copy()
    _expect(cb, -2, V, inward)                           # negative volume
    bad = T.copy()
    bad[0, 0] = len(V) + 5
    _expect(cb, -2, V, bad)                              # index out of range
    rep = T.copy()
    rep[0, 1] = rep[0, 0]
    _expect(cb, -2, V, rep)                              # repeated vertex
    nanV = V.copy()
    nanV[0, 0] = np.nan
    _expect(cb, -2, nanV, T)
    eb = w.edge_block.copy()
    eb[0] = 99
    _expect(cb, -1, V, T, eb, 8)                         # cell id out of range
    eb = w.edge_block.copy()
    eb[eb == 3] = 2
    _expect(cb, -2, V, T, eb, 8)                         # empty cell
    _expect(cb, -1, V[:3], T[:2])                        # too small


def test_error_message_is_thread_local_text(cb):
    with pytest.raises(cb.CBFMError) as e:
        cb.mesh_analyze(np.zeros((3, 3)), np.zeros((1, 3), np.int32))
    assert "nv" in str(e.value)
