"""Host-side pieces of the serving form: the request footprint estimate,
the seeded request stream and its meshes (no GPU)."""
import numpy as np

from synth import configs, meshes


def test_geodesic_sphere_is_closed_and_outward():
    for n in (1, 3, 5):
        V, T = meshes.geodesic(n, 0.5)
        assert len(T) == 20 * n * n
        E = meshes.edges_canonical(T)
        assert len(V) - len(E) + len(T) == 2  # sphere topology
        assert np.allclose(np.linalg.norm(V, axis=1), 0.5)
        a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        nrm = np.cross(b - a, c - a)
        assert np.all(np.einsum("ij,ij->i", nrm, a + b + c) > 0)
        # every edge shared by exactly two triangles with opposite directions
        directed = {(int(u), int(v)) for t in T for u, v in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert len(directed) == 3 * len(T) and all((v, u) in directed for u, v in directed)


def test_serving_stream_is_seeded_and_on_the_ladder():
    a = configs.serving_stream(40, seed=5)
    b = configs.serving_stream(40, seed=5)
    lad = {k: {u for u, _ in v} for k, v in configs._serve_ladder().items()}
    for x, y in zip(a, b):
        assert x.t_arrival == y.t_arrival and x.unknowns == y.unknowns and np.array_equal(x.work.inc, y.work.inc)
        assert x.unknowns in lad[x.shape] and 960 <= x.unknowns <= 8000
        assert 3 * len(x.work.T) == x.unknowns
        assert 1 <= len(x.work.inc) <= 16 and 1.5 <= x.work.eps_r.real <= 6.0
        ne = 3 * len(x.work.T) // 2
        assert abs(ne / x.work.nblocks - 100) < 60
    t = np.array([x.t_arrival for x in a])
    assert np.all(np.diff(t) > 0)


def test_request_footprint_grows_with_size_and_rhs():
    from paper_2111_11058_amd import cbfm
    w = configs.sphere_c1()
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    fp = []
    for inc in (w.inc, configs.random_incidences(16, 3)):
        req, keep = cbfm.make_request(w.V, w.T, w.edge_block, w.nblocks, med, w.gen, w.delta_svd, inc)
        fp.append(cbfm.request_footprint(req))
    assert 0 < fp[0] < fp[1]
    big = configs.cube_c2(1)
    req, keep = cbfm.make_request(big.V, big.T, big.edge_block, big.nblocks, med, big.gen, big.delta_svd, big.inc)
    assert cbfm.request_footprint(req) > fp[0]
