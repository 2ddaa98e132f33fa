"""The allocation-free fill (cbfm_fill_pmchwt_noalloc), through the C ABI,
against the allocating fill (cbfm_fill_pmchwt) on the same inputs: two calls
in a row on the library's fixed workspace, the second smaller, in FP64 and
FP32; a range beyond the workspace is rejected before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_fill_matches_allocating_fill():
    import torch
    from paper_2111_11058_amd import cbfm
    from synth import configs
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = configs.sphere_c1()
    mesh = cbfm.Mesh(w.V, w.T, w.edge_block, w.nblocks)
    med = cbfm.Medium.make(w.k0, w.eta0, w.eps_r, w.mu_r)
    ne = mesh.ne
    for prec, dt in ((cbfm.FP64, torch.complex128), (cbfm.FP32, torch.complex64)):
        # the whole 480 x 480 fill, then a ragged sub-range with a padded ld
        for row0, nrow, col0, ncol, ld in ((0, ne, 0, ne, ne), (17, 101, 250, 77, 80)):
            print(f"noalloc fill prec={prec} rows={row0}+{nrow} cols={col0}+{ncol}", flush=True)
            a = torch.full((3, nrow, ld), complex(np.nan, np.nan), dtype=dt, device="cuda")
            b = torch.full((3, nrow, ld), complex(np.nan, np.nan), dtype=dt, device="cuda")
            cbfm.fill_pmchwt(mesh, med, a, prec, cbfm.LAYOUT_OPS3, row0, nrow, col0, ncol, ld)
            cbfm.fill_pmchwt(mesh, med, b, prec, cbfm.LAYOUT_OPS3, row0, nrow, col0, ncol, ld, noalloc=True)
            ga, gb = a.cpu().numpy()[:, :, :ncol], b.cpu().numpy()[:, :, :ncol]
            assert np.all(np.isfinite(gb))
            d = np.abs(ga - gb).max() / np.abs(ga).max()
            print("max rel difference", d)
            assert d <= (1e-15 if prec == cbfm.FP64 else 1e-7)
    # a range whose workspace exceeds the fixed array: E_ARG, output untouched
    big = configs.cylinder_c5()
    mb = cbfm.Mesh(big.V, big.T, big.edge_block, big.nblocks)
    mdb = cbfm.Medium.make(big.k0, big.eta0, big.eps_r, big.mu_r)
    out = torch.zeros((3, 200, mb.ne), dtype=torch.complex128, device="cuda")
    with pytest.raises(cbfm.CBFMError) as e:
        cbfm.fill_pmchwt(mb, mdb, out, cbfm.FP64, cbfm.LAYOUT_OPS3, 0, 200, 0, mb.ne, noalloc=True)
    print(e.value)
    assert e.value.code == -1 and "workspace" in str(e.value)
    assert float(out.abs().max()) == 0.0
