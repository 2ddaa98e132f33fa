"""Device memory from the caller's allocator (cbfm_set_allocator) through
the C ABI: with PyTorch's caching allocator set, the projection, the CMP
and the solve keep their parity with the oracle, the library's handles and
scratch show up in PyTorch's allocated bytes, and the library makes no
hipMalloc allocation of its own; its own allocations return afterwards."""
import numpy as np
import pytest

from test_gpu_cbf_solve import _gpu_handles, _oracle_cbf

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_torch_allocator_carries_all_device_memory():
    import torch
    from oracle import excitation
    from paper_2111_11058_amd import cbfm
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    torch.cuda.synchronize()
    cbfm.use_torch_allocator(True)
    try:
        own0 = cbfm.memory_stats()["held"]
        t0 = torch.cuda.memory_allocated()
        print("allocator set: library-held bytes", own0, "torch allocated", t0, flush=True)
        cb_, mesh, med, cbf = _gpu_handles(w, O)
        n = cbf.n_cbf
        Zr = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
        assert _rel(Zr.cpu().numpy(), O["Zr"]) < 1e-10
        op = cbfm.MomOperator(mesh, med, cbfm.FP64)
        t1 = torch.cuda.memory_allocated()
        print("with handles: torch allocated", t1, "operator bytes", op.n * op.n * 16, flush=True)
        assert t1 - t0 >= op.n * op.n * 16  # the operator's matrix is torch memory
        jt = torch.zeros((len(w.inc), 2 * m.ne), dtype=torch.complex128, device="cuda")
        out = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-12, max_iter=n + 10, restart=n + 10, j_out=jt)
        jref = O["CMJ"] @ np.linalg.solve(O["Zr"], O["CJM"].conj().T @ P["v"])
        assert out["status"] == "OK" and _rel(jt.cpu().numpy().T, jref) < 1e-9
        rcs_ref = excitation.monostatic_rcs(m, jref, w.inc, w.k0, w.eta0)
        assert np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref) < 1e-9
        own1 = cbfm.memory_stats()["held"]
        print("library-held bytes after the work", own1, flush=True)
        assert own1 <= own0  # nothing came from the library's own hipMalloc
        op.close()
        cbf.close()
        mesh.close()
        torch.cuda.synchronize()
        t2 = torch.cuda.memory_allocated()
        print("handles freed: torch allocated", t2, flush=True)
        assert t2 < t1
    finally:
        cbfm.use_torch_allocator(False)
    # the library's own allocations again
    cb_, mesh, med, cbf = _gpu_handles(w, O)
    Zr = torch.zeros((cbf.n_cbf, cbf.n_cbf), dtype=torch.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    assert _rel(Zr.cpu().numpy(), O["Zr"]) < 1e-10
    assert cbfm.memory_stats()["held"] > 0
