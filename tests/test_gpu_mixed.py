"""The precision form through the C ABI: FP32 fill with FP32 or BF16
matrix-core projection (FP32 accumulation), and GMRES with float Krylov
cycles refined against the double residual, checked against the FP64
oracle (same imported CBFs)."""
import numpy as np
import pytest

from test_gpu_cbf_solve import _gpu_handles, _oracle_cbf, _rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.mark.parametrize("name", ["c1", "cyl_small"])
def test_mixed_projection_error(torch_cuda, name):
    """Z_r from the float fill and FP32 matrix cores stays within 1e-4 of the
    FP64 oracle, and so does split BF16; plain BF16 inputs (8-bit
    significands) within 2e-2."""
    O = _oracle_cbf(name)
    w = O["P"]["w"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    print(f"mixed project {w.name} N_CBF={n}", flush=True)
    Z = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Z, cbfm.MIXED_FP32)
    e32 = _rel(Z.cpu().numpy(), O["Zr"])
    cbfm.project(mesh, med, cbf, Z, cbfm.MIXED_BF16)
    e16 = _rel(Z.cpu().numpy(), O["Zr"])
    cbfm.project(mesh, med, cbf, Z, cbfm.MIXED_BF16X3)
    e3 = _rel(Z.cpu().numpy(), O["Zr"])
    print(f"Z_r rel err: fp32 {e32:.2e}  bf16 {e16:.2e}  split bf16 {e3:.2e}")
    assert e32 < 1e-4 and e3 < 1e-4
    assert e16 < 2e-2


def test_refined_solve_matches_fp64(torch_cuda):
    """Float Krylov cycles refined against the double residual reach the
    double solution of the same system (tol 1e-11)."""
    from oracle import excitation
    O = _oracle_cbf("cyl_small")
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    Zr = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    cbfm.project(mesh, med, cbf, Zr, cbfm.FP64)
    jt = torch_cuda.zeros((len(w.inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    print("refined solve", flush=True)
    out = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-11, max_iter=4 * n, restart=n, j_out=jt, inner_fp32=True)
    print(out)
    assert out["status"] == "OK" and np.all(out["relres"] < 1.1e-10)
    vr = O["CJM"].conj().T @ excitation.rhs(m, w.inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    err = _rel(jt.cpu().numpy().T, jref)
    print("currents rel err", err)
    assert err < 1e-8
    # a loose inner tolerance only adds cycles
    out2 = cbfm.solve(mesh, med, cbf, Zr, w.inc, tol=1e-11, max_iter=4 * n, restart=n, j_out=jt, inner_fp32=True,
                      inner_tol=1e-2)
    assert out2["status"] == "OK" and _rel(jt.cpu().numpy().T, jref) < 1e-8


@pytest.mark.parametrize("name", ["c1", "cyl_small", "cyl_lossy"])
def test_mixed_end_to_end_rcs(torch_cuda, name):
    """Each precision form against the FP64 oracle (same CBFs, LU of the
    oracle's Z_r): FP32 regular fill with FP64 projection and solve; float
    fill + FP32 matrix-core projection + refined float GMRES; the same with
    split-BF16 and with plain BF16 projection.  Monostatic RCS within 1e-4
    of the oracle (plain BF16: reported, bounded by 5e-2); the surface
    current error (relative Frobenius over all incidences) is reported and
    bounded by 1e-3 (0.2 for plain BF16).  cyl_lossy has the lossy
    permittivity of the precision workload (4 - 0.1j)."""
    from oracle import excitation
    O = _oracle_cbf(name)
    P = O["P"]
    w, m = P["w"], P["m"]
    cbfm, mesh, med, cbf = _gpu_handles(w, O)
    n = cbf.n_cbf
    vr = O["CJM"].conj().T @ excitation.rhs(m, w.inc, w.k0, w.eta0)
    jref = O["CMJ"] @ np.linalg.solve(O["Zr"], vr)
    rcs_ref = excitation.monostatic_rcs(m, jref, w.inc, w.k0, w.eta0)
    Z = torch_cuda.zeros((n, n), dtype=torch_cuda.complex128, device="cuda")
    J = torch_cuda.zeros((len(w.inc), 2 * m.ne), dtype=torch_cuda.complex128, device="cuda")
    errs, cerr = {}, {}
    forms = {"fp32_fill": (cbfm.FP32, False), "mixed_fp32": (cbfm.MIXED_FP32, True),
             "split_bf16": (cbfm.MIXED_BF16X3, True), "bf16": (cbfm.MIXED_BF16, True)}
    for name_f, (prec, f32) in forms.items():
        cbfm.project(mesh, med, cbf, Z, prec)
        out = cbfm.solve(mesh, med, cbf, Z, w.inc, tol=1e-8, max_iter=4 * n, restart=n, inner_fp32=f32, j_out=J)
        assert out["status"] == "OK"
        errs[name_f] = np.max(np.abs(out["rcs"] - rcs_ref) / rcs_ref)
        cerr[name_f] = _rel(J.cpu().numpy().T, jref)
    print(f"{w.name}: vs the FP64 oracle, monostatic RCS / current rel err: " +
          ", ".join(f"{k} {errs[k]:.2e} / {cerr[k]:.2e}" for k in forms))
    for k in ("fp32_fill", "mixed_fp32", "split_bf16"):
        assert errs[k] < 1e-4 and cerr[k] < 1e-3, k
    assert errs["bf16"] < 5e-2 and cerr["bf16"] < 0.2
