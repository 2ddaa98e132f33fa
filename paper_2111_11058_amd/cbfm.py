"""Thin ctypes binding of libcbfm (include/cbfm.h).

Argument marshalling only: every computation happens in the HIP library.
PyTorch supplies device memory (tensors passed by ``data_ptr``) and streams
(``torch.cuda.current_stream().cuda_stream``).  Importing this module does not
load the library; the first call does, and raises if it is not built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbfm.so")

FP64, FP32, MIXED_FP32, MIXED_BF16, MIXED_BF16X3 = 0, 1, 2, 3, 4
LAYOUT_MEDIA3, LAYOUT_OPS3, LAYOUT_MEDIA4 = 0, 1, 2

STATUS = {0: "OK", -1: "E_ARG", -2: "E_MESH", -3: "E_NOMEM", -4: "E_HIP", -5: "E_NOCONV",
          -6: "E_RANK", -7: "E_STATE"}


class CBFMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Medium(C.Structure):
    _fields_ = [("k0", C.c_double), ("eta0", C.c_double), ("eps_re", C.c_double),
                ("eps_im", C.c_double), ("mu_re", C.c_double), ("mu_im", C.c_double)]

    @classmethod
    def make(cls, k0, eta0, eps_r, mu_r=1.0):
        e, m = complex(eps_r), complex(mu_r)
        return cls(float(k0), float(eta0), e.real, e.imag, m.real, m.imag)


class CbfParams(C.Structure):
    _fields_ = [("gen_host", C.POINTER(C.c_double)), ("n_gen", C.c_int32),
                ("delta_svd", C.c_double), ("max_L", C.c_int32)]


CMP_EXACT, CMP_INNER_GMRES = 0, 1


class SolverParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("use_cmp", C.c_int32), ("inner_fp32", C.c_int32), ("inner_tol", C.c_double),
                ("use_graph", C.c_int32), ("cmp_mode", C.c_int32), ("cmp_inner_tol", C.c_double),
                ("basis_fp32", C.c_int32), ("sstep", C.c_int32), ("block", C.c_int32)]


class IpcbfParams(C.Structure):
    _fields_ = [("gen_host", C.POINTER(C.c_double)), ("n_gen", C.c_int32), ("delta_r", C.c_double),
                ("delta_svd", C.c_double), ("max_L", C.c_int32), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("block", C.c_int32)]


_lib = None
_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32


def lib():
    """Load libcbfm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2111_11058_amd.build`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "cbfm_last_error": (C.c_char_p, []),
        "cbfm_set_allocator": (_I32, [_P, _P]),
        "cbfm_memory_stats": (_I32, [C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
        "cbfm_timer_enable": (_I32, [_I32]),
        "cbfm_request_footprint": (_I32, [_P, C.POINTER(_I64)]),
        "cbfm_project_batch": (_I32, [_I32, _P, _P, _P, _I32, _P, _P, _P]),
        "cbfm_server_create": (_I32, [_I32, _I64, C.POINTER(_P)]),
        "cbfm_server_submit": (_I32, [_P, _P, C.POINTER(_I64)]),
        "cbfm_server_wait": (_I32, [_P, _I64, _P, _P, _P]),
        "cbfm_server_stats": (_I32, [_P, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I32)]),
        "cbfm_server_destroy": (None, [_P]),
        "cbfm_timer_read": (_I32, [C.c_char_p, C.POINTER(_I64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "cbfm_version": (_I32, []),
        "cbfm_mesh_load": (_I32, [_P, _I64, _P, _I64, _P, _I32, C.POINTER(_P)]),
        "cbfm_mesh_info": (_I32, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I64)]),
        "cbfm_mesh_edges": (_I32, [_P, _P, _P]),
        "cbfm_mesh_free": (None, [_P]),
        "cbfm_mesh_analyze": (_I32, [_P, _I64, _P, _I64, _P, _I32, C.POINTER(_I64), _P, _P, _P,
                                     C.POINTER(_I64), _P, _I64]),
        "cbfm_fill_pmchwt": (_I32, [_P, C.POINTER(Medium), _I32, _I64, _I64, _I64, _I64, _I32, _P, _I64, _P]),
        "cbfm_fill_pmchwt_noalloc": (_I32, [_P, C.POINTER(Medium), _I32, _I64, _I64, _I64, _I64, _I32, _P, _I64,
                                            _P]),
        "cbfm_rhs": (_I32, [_P, C.POINTER(Medium), _P, _I64, _P, _P]),
        "cbfm_build_cbf": (_I32, [_P, C.POINTER(Medium), C.POINTER(CbfParams), _P, C.POINTER(_P)]),
        "cbfm_cbf_import": (_I32, [_P, _P, _P, _P, _P, _P, C.POINTER(_P)]),
        "cbfm_cbf_info": (_I32, [_P, C.POINTER(_I64), _P, _P]),
        "cbfm_cbf_export": (_I32, [_P, _P, _P]),
        "cbfm_cbf_free": (None, [_P]),
        "cbfm_project": (_I32, [_P, C.POINTER(Medium), _P, _I32, _P, _I64, _P]),
        "cbfm_project_ex": (_I32, [_P, C.POINTER(Medium), _P, _I32, _P, _I64, _I64, C.POINTER(_I32), _P]),
        "cbfm_cmp_apply": (_I32, [_P, _I64, _P, _P, _P]),
        "cbfm_cmp_apply_ex": (_I32, [_P, _I64, _P, _P, _I32, C.c_double, _P]),
        "cbfm_mom_build": (_I32, [_P, C.POINTER(Medium), _I32, _I64, _P, C.POINTER(_P)]),
        "cbfm_mom_info": (_I32, [_P, C.POINTER(_I64), C.POINTER(_I32)]),
        "cbfm_mom_export": (_I32, [_P, _I64, _I64, _P, _I64, _P, _P]),
        "cbfm_mom_free": (None, [_P]),
        "cbfm_mom_solve": (_I32, [_P, _P, _I64, C.POINTER(SolverParams), _P, _P, _P, _P, _I64, _P, _P]),
        "cbfm_build_ipcbf": (_I32, [_P, C.POINTER(IpcbfParams), _P, C.POINTER(_P), _P, _P]),
        "cbfm_solve_matfree": (_I32, [_P, _P, _P, _I64, C.POINTER(SolverParams), _P, _P, _P, _P, _I64, _P, _P]),
        "cbfm_solve": (_I32, [_P, C.POINTER(Medium), _P, _P, _I64, _P, _I64, C.POINTER(SolverParams), _P,
                              _P, _P, _P, _I64, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise CBFMError(code, lib().cbfm_last_error().decode())
    return code


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, numel=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what} has {t.numel()} elements, need {numel}")
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator_hooks = []  # the ctypes callbacks live as long as the process


def use_torch_allocator(enable=True):
    """cbfm_set_allocator with PyTorch's caching allocator: every device
    buffer of the library (handles and scratch) then comes from
    torch.cuda.caching_allocator_alloc on the stream the library names, and
    goes back through caching_allocator_delete.  enable=False restores the
    library's own allocations."""
    import torch
    if not enable:
        _check(lib().cbfm_set_allocator(None, None))
        return

    def _alloc(nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _release(p, stream):
        torch.cuda.caching_allocator_delete(int(p))

    hooks = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _allocator_hooks.append(hooks)
    _check(lib().cbfm_set_allocator(C.cast(hooks[0], _P), C.cast(hooks[1], _P)))


def memory_stats():
    """cbfm_memory_stats: dict(held, peak, cached) bytes of the library's own
    device allocations."""
    h, p, c = _I64(), _I64(), _I64()
    _check(lib().cbfm_memory_stats(C.byref(h), C.byref(p), C.byref(c)))
    return dict(held=h.value, peak=p.value, cached=c.value)


TIMERS = ("fill_regular", "fill_near", "assemble", "gemm", "gmres_dots", "gmres_update", "fill_regular_f32", "xgemm",
          "gemm_panel")


def timer_enable(names=TIMERS):
    """Clear the library's per-kernel event timers and time the kernel
    families in ``names`` (an empty sequence or None disables timing)."""
    mask = 0
    for n in names or ():
        mask |= 1 << TIMERS.index(n)
    _check(lib().cbfm_timer_enable(mask))


def timer_read(name, with_work=False):
    """(launches, total milliseconds[, algorithmic work]) recorded for kernel
    family ``name`` (work units: see TIMERS in include/cbfm.h)."""
    n, ms, wk = _I64(), C.c_double(), C.c_double()
    _check(lib().cbfm_timer_read(name.encode(), C.byref(n), C.byref(ms), C.byref(wk)))
    return (n.value, ms.value, wk.value) if with_work else (n.value, ms.value)


def mesh_analyze(V, T, edge_block=None, nblocks=None):
    """Host-only mesh validation (cbfm_mesh_analyze): returns (edges,
    tri_edge, tri_sign, near) with near rows (P, Q, coplanar).  Needs no
    GPU."""
    L = lib()
    V, pV = _host(V, np.float64)
    T, pT = _host(T, np.int32)
    if edge_block is not None:
        eb, peb = _host(edge_block, np.int32)
        nb = int(nblocks if nblocks is not None else eb.max() + 1)
    else:
        peb, nb = None, 1
    ne, nn = _I64(), _I64()
    _check(L.cbfm_mesh_analyze(pV, len(V), pT, len(T), peb, nb, C.byref(ne), None, None, None, C.byref(nn),
                               None, 0))
    E = np.zeros((ne.value, 2), np.int32)
    TE = np.zeros((len(T), 3), np.int32)
    TS = np.zeros((len(T), 3), np.int32)
    N = np.zeros((nn.value, 3), np.int32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(L.cbfm_mesh_analyze(pV, len(V), pT, len(T), peb, nb, C.byref(ne), ptr(E), ptr(TE), ptr(TS), C.byref(nn),
                               ptr(N), nn.value))
    return E, TE, TS, N


class Mesh:
    """Handle of a loaded mesh (cbfm_mesh)."""

    def __init__(self, V, T, edge_block=None, nblocks=None):
        L = lib()
        V, pV = _host(V, np.float64)
        T, pT = _host(T, np.int32)
        if edge_block is not None:
            eb, peb = _host(edge_block, np.int32)
            nb = int(nblocks if nblocks is not None else eb.max() + 1)
        else:
            peb, nb = None, 1
        h = C.c_void_p()
        _check(L.cbfm_mesh_load(pV, len(V), pT, len(T), peb, nb, C.byref(h)))
        self._h = h
        ne, nt, nbk, nn = _I64(), _I64(), _I32(), _I64()
        _check(L.cbfm_mesh_info(h, C.byref(ne), C.byref(nt), C.byref(nbk), C.byref(nn)))
        self.ne, self.nt, self.nblocks, self.n_near = ne.value, nt.value, nbk.value, nn.value

    @property
    def handle(self):
        return self._h

    def edges(self):
        ev = np.zeros((self.ne, 2), np.int32)
        eb = np.zeros(self.ne, np.int32)
        _check(lib().cbfm_mesh_edges(self._h, ev.ctypes.data_as(C.c_void_p), eb.ctypes.data_as(C.c_void_p)))
        return ev, eb

    def close(self):
        if getattr(self, "_h", None):
            lib().cbfm_mesh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FILL_NOALLOC_MAX_BYTES = 64 << 20  # CBFM_FILL_NOALLOC_MAX_BYTES


def fill_pmchwt(mesh: Mesh, medium: Medium, out, precision=FP64, layout=LAYOUT_MEDIA3,
                row0=0, nrow=None, col0=0, ncol=None, ld=None, stream=None, noalloc=False):
    """cbfm_fill_pmchwt into ``out`` (3 x nrow x ld complex tensor, 4 x for
    LAYOUT_MEDIA4); with noalloc, cbfm_fill_pmchwt_noalloc (the library's
    fixed workspace)."""
    import torch
    nrow = mesh.ne - row0 if nrow is None else nrow
    ncol = mesh.ne - col0 if ncol is None else ncol
    ld = ncol if ld is None else ld
    dt = torch.complex128 if precision == FP64 else torch.complex64
    p = _dev(out, dt, (4 if layout == LAYOUT_MEDIA4 else 3) * nrow * ld, "out")
    f = lib().cbfm_fill_pmchwt_noalloc if noalloc else lib().cbfm_fill_pmchwt
    _check(f(mesh.handle, C.byref(medium), precision, row0, nrow, col0, ncol, layout, p, ld, _stream(stream)))
    return out


def rhs(mesh: Mesh, medium: Medium, inc, out, stream=None):
    """cbfm_rhs: ``out`` is (nrhs, 2 ne) complex128."""
    import torch
    inc, pi = _host(inc, np.float64)
    inc = inc.reshape(-1, 6)
    p = _dev(out, torch.complex128, len(inc) * 2 * mesh.ne, "out")
    _check(lib().cbfm_rhs(mesh.handle, C.byref(medium), pi, len(inc), p, _stream(stream)))
    return out


class CBF:
    """Handle of a CBF set (cbfm_cbf)."""

    def __init__(self, h, mesh):
        self._h = h
        self.mesh = mesh
        n = _I64()
        L = np.zeros(mesh.nblocks, np.int32)
        _check(lib().cbfm_cbf_info(h, C.byref(n), L.ctypes.data_as(C.c_void_p), None))
        self.n_cbf = n.value
        self.L = L
        sig = np.zeros(int(L.sum()))
        _check(lib().cbfm_cbf_info(h, None, None, sig.ctypes.data_as(C.c_void_p)))
        self.sigma = sig

    @property
    def handle(self):
        return self._h

    def export(self):
        """(CM, CJ) as lists of per-cell (N_m, L_m) complex arrays."""
        ev, eb = self.mesh.edges()
        N = np.bincount(eb, minlength=self.mesh.nblocks)
        tot = int((N * self.L).sum())
        CM = np.zeros(tot, np.complex128)
        CJ = np.zeros(tot, np.complex128)
        _check(lib().cbfm_cbf_export(self._h, CM.ctypes.data_as(C.c_void_p), CJ.ctypes.data_as(C.c_void_p)))
        outM, outJ, o = [], [], 0
        for n, l in zip(N, self.L):
            outM.append(CM[o:o + n * l].reshape(n, l))
            outJ.append(CJ[o:o + n * l].reshape(n, l))
            o += n * l
        return outM, outJ

    def close(self):
        if getattr(self, "_h", None):
            lib().cbfm_cbf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_cbf(mesh: Mesh, medium: Medium, gen, delta_svd=1e-3, max_L=0, stream=None) -> CBF:
    gen, _ = _host(gen, np.float64)
    gen = gen.reshape(-1, 6)
    prm = CbfParams(gen.ctypes.data_as(C.POINTER(C.c_double)), len(gen), float(delta_svd), int(max_L))
    h = C.c_void_p()
    _check(lib().cbfm_build_cbf(mesh.handle, C.byref(medium), C.byref(prm), _stream(stream), C.byref(h)))
    return CBF(h, mesh)


def cbf_import(mesh: Mesh, CM_cells, CJ_cells, sigma_cells, stream=None) -> CBF:
    L = np.array([c.shape[1] for c in CM_cells], np.int32)
    CM = np.ascontiguousarray(np.concatenate([np.asarray(c, np.complex128).ravel() for c in CM_cells]))
    CJ = np.ascontiguousarray(np.concatenate([np.asarray(c, np.complex128).ravel() for c in CJ_cells]))
    sg = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64) for s in sigma_cells]))
    h = C.c_void_p()
    _check(lib().cbfm_cbf_import(mesh.handle, L.ctypes.data_as(C.c_void_p), CM.ctypes.data_as(C.c_void_p),
                                 CJ.ctypes.data_as(C.c_void_p), sg.ctypes.data_as(C.c_void_p),
                                 _stream(stream), C.byref(h)))
    return CBF(h, mesh)


def project(mesh: Mesh, medium: Medium, cbf: CBF, out, precision=FP64, ldz=None, stream=None, panel_bytes=None):
    """cbfm_project into ``out`` (n x ldz complex128); with ``panel_bytes``
    cbfm_project_ex with that panel budget, returning the panel count."""
    import torch
    n = cbf.n_cbf
    ldz = n if ldz is None else ldz
    p = _dev(out, torch.complex128, n * ldz, "Zr")
    if panel_bytes is None:
        _check(lib().cbfm_project(mesh.handle, C.byref(medium), cbf.handle, precision, p, ldz, _stream(stream)))
        return out
    npan = _I32()
    _check(lib().cbfm_project_ex(mesh.handle, C.byref(medium), cbf.handle, precision, p, ldz, int(panel_bytes),
                                 C.byref(npan), _stream(stream)))
    return npan.value


def project_batch(items, precision=FP64, stream=None):
    """cbfm_project_batch over items = [(mesh, medium, cbf, Zr tensor), ...]
    (Zr row-major n x n complex128, ldz = n)."""
    import torch
    k = len(items)
    meshes = (_P * k)(*[it[0].handle for it in items])
    media = (Medium * k)(*[it[1] for it in items])
    cbfs = (_P * k)(*[it[2].handle for it in items])
    zr = (_P * k)(*[_dev(it[3], torch.complex128, it[2].n_cbf ** 2, "Zr") for it in items])
    ldz = (_I64 * k)(*[it[2].n_cbf for it in items])
    _check(lib().cbfm_project_batch(k, meshes, media, cbfs, int(precision), zr, ldz, _stream(stream)))


def cmp_apply(cbf: CBF, y, x, stream=None, mode=CMP_EXACT, inner_tol=0.0):
    """cbfm_cmp_apply_ex: x = (G^CBF)^{-1} y, exact or by the inner GMRES."""
    import torch
    nrhs = y.numel() // cbf.n_cbf
    py = _dev(y, torch.complex128, nrhs * cbf.n_cbf, "y")
    px = _dev(x, torch.complex128, nrhs * cbf.n_cbf, "x")
    _check(lib().cbfm_cmp_apply_ex(cbf.handle, nrhs, py, px, int(mode), float(inner_tol), _stream(stream)))
    return x


class MomOperator:
    """The whole system in the MoM arrangement with its diagonal
    preconditioner (cbfm_mom): A = Z_t D^{-1} stored on the device."""

    def __init__(self, mesh: Mesh, medium: Medium, precision=FP64, panel_bytes=0, stream=None):
        h = _P()
        _check(lib().cbfm_mom_build(mesh.handle, C.byref(medium), int(precision), int(panel_bytes), _stream(stream),
                                    C.byref(h)))
        self._h, self.mesh, self.medium = h, mesh, medium
        n, p = _I64(), _I32()
        _check(lib().cbfm_mom_info(h, C.byref(n), C.byref(p)))
        self.n, self.precision = n.value, p.value

    @property
    def handle(self):
        return self._h

    def export(self, row0=0, nrow=None, stream=None):
        """(rows row0.. of A, D) as torch tensors (cell order, see the header)."""
        import torch
        nrow = self.n - row0 if nrow is None else nrow
        dt = torch.complex128 if self.precision == FP64 else torch.complex64
        A = torch.empty((nrow, self.n), dtype=dt, device="cuda")
        d = torch.empty(self.n, dtype=torch.complex128, device="cuda")
        _check(lib().cbfm_mom_export(self._h, int(row0), int(nrow), _dev(A, dt, nrow * self.n, "A"), self.n,
                                     _dev(d, torch.complex128, self.n, "d"), _stream(stream)))
        torch.cuda.synchronize()
        return A, d

    def close(self):
        if getattr(self, "_h", None):
            lib().cbfm_mom_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solve_outputs(nrhs, dirs):
    iters = np.zeros(nrhs, np.int32)
    relres = np.zeros(nrhs)
    if dirs is not None:
        dirs, pd = _host(dirs, np.float64)
        dirs = dirs.reshape(-1, 3)
        rcs = np.zeros((nrhs, len(dirs)))
        return iters, relres, rcs, dirs, pd, len(dirs)
    return iters, relres, np.zeros(nrhs), None, None, 0


def mom_solve(mom: MomOperator, inc, tol=1e-6, max_iter=1000, restart=1000, j_out=None, dirs=None, stream=None,
              inner_fp32=False, inner_tol=0.0, use_graph=False, basis_fp32=False, block=False):
    """cbfm_mom_solve (the MoM baseline; block as in solve(), FP64 operator
    only).  Returns dict(iters, relres, rcs, status)."""
    import torch
    inc, pi = _host(inc, np.float64)
    inc = inc.reshape(-1, 6)
    nrhs = len(inc)
    pj = _dev(j_out, torch.complex128, nrhs * mom.n, "j") if j_out is not None else None
    iters, relres, rcs, dirs, pd, nd = _solve_outputs(nrhs, dirs)
    prm = SolverParams(float(tol), int(max_iter), int(restart), 0, int(bool(inner_fp32)), float(inner_tol),
                       int(bool(use_graph)), basis_fp32=int(bool(basis_fp32)), block=int(block))
    code = lib().cbfm_mom_solve(mom.handle, pi, nrhs, C.byref(prm), pj, iters.ctypes.data_as(C.c_void_p),
                                relres.ctypes.data_as(C.c_void_p), pd, nd, rcs.ctypes.data_as(C.c_void_p),
                                _stream(stream))
    if code not in (0, -5):
        _check(code)
    return dict(iters=iters, relres=relres, rcs=rcs, status=STATUS.get(code, code))


def build_ipcbf(mom: MomOperator, gen, delta_r=1e-3, delta_svd=1e-3, max_L=0, max_iter=1000, restart=0, block=False,
                stream=None):
    """cbfm_build_ipcbf: returns (CBF, iterations per wave, residual per wave)
    (block: True or a group size, block GMRES; the iterations are then block
    iterations of the wave's group)."""
    gen, _ = _host(gen, np.float64)
    gen = gen.reshape(-1, 6)
    prm = IpcbfParams(gen.ctypes.data_as(C.POINTER(C.c_double)), len(gen), float(delta_r), float(delta_svd),
                      int(max_L), int(max_iter), int(restart), int(block))
    h = _P()
    its = np.zeros(len(gen), np.int32)
    res = np.zeros(len(gen))
    _check(lib().cbfm_build_ipcbf(mom.handle, C.byref(prm), _stream(stream), C.byref(h),
                                  its.ctypes.data_as(C.c_void_p), res.ctypes.data_as(C.c_void_p)))
    return CBF(h, mom.mesh), its, res


def solve_matfree(mom: MomOperator, cbf: CBF, inc, tol=1e-6, max_iter=1000, restart=100, use_cmp=True, j_out=None,
                  dirs=None, stream=None):
    """cbfm_solve_matfree: the reduced CBFM solve with (C^JM)^H Z C^MJ applied
    from the stored operator, Z_r never formed."""
    import torch
    inc, pi = _host(inc, np.float64)
    inc = inc.reshape(-1, 6)
    nrhs = len(inc)
    pj = _dev(j_out, torch.complex128, nrhs * mom.n, "j") if j_out is not None else None
    iters, relres, rcs, dirs, pd, nd = _solve_outputs(nrhs, dirs)
    prm = SolverParams(float(tol), int(max_iter), int(restart), int(use_cmp), 0, 0.0, 0)
    code = lib().cbfm_solve_matfree(mom.handle, cbf.handle, pi, nrhs, C.byref(prm), pj,
                                    iters.ctypes.data_as(C.c_void_p), relres.ctypes.data_as(C.c_void_p), pd, nd,
                                    rcs.ctypes.data_as(C.c_void_p), _stream(stream))
    if code not in (0, -5):
        _check(code)
    return dict(iters=iters, relres=relres, rcs=rcs, status=STATUS.get(code, code))


def solve(mesh: Mesh, medium: Medium, cbf: CBF, Zr, inc, tol=1e-6, max_iter=1000, restart=100,
          use_cmp=True, j_out=None, dirs=None, ldz=None, stream=None, raise_noconv=False, inner_fp32=False,
          inner_tol=0.0, use_graph=False, cmp_mode=CMP_EXACT, cmp_inner_tol=0.0, basis_fp32=False, sstep=0,
          block=False):
    """cbfm_solve.  Returns dict(iters, relres, rcs, status).  inner_fp32
    selects the mixed form (float Krylov cycles refined against the double
    residual, each cycle reducing it by inner_tol); basis_fp32 the
    compressed-basis form (double cycles with the basis stored in float,
    restarted the same way); sstep (4 or 8) the s-step cycles of blocks of
    that many iterations; block the block GMRES (True or 1: one Krylov space
    per group of up to 32 right-hand sides, sized for cycles of at least 32
    block iterations; 2..32: groups of that many; max_iter, restart and the
    returned iters count block iterations); use_graph replays the Arnoldi iterations from a
    captured HIP graph."""
    import torch
    inc, pi = _host(inc, np.float64)
    inc = inc.reshape(-1, 6)
    nrhs = len(inc)
    n = cbf.n_cbf
    ldz = n if ldz is None else ldz
    pz = _dev(Zr, torch.complex128, n * ldz, "Zr")
    pj = _dev(j_out, torch.complex128, nrhs * 2 * mesh.ne, "j") if j_out is not None else None
    iters = np.zeros(nrhs, np.int32)
    relres = np.zeros(nrhs)
    if dirs is not None:
        dirs, pd = _host(dirs, np.float64)
        dirs = dirs.reshape(-1, 3)
        nd = len(dirs)
        rcs = np.zeros((nrhs, nd))
    else:
        pd, nd = None, 0
        rcs = np.zeros(nrhs)
    prm = SolverParams(float(tol), int(max_iter), int(restart), int(use_cmp), int(bool(inner_fp32)),
                       float(inner_tol), int(bool(use_graph)), int(cmp_mode), float(cmp_inner_tol),
                       int(bool(basis_fp32)), int(sstep), int(block))
    code = lib().cbfm_solve(mesh.handle, C.byref(medium), cbf.handle, pz, ldz, pi, nrhs, C.byref(prm), pj,
                            iters.ctypes.data_as(C.c_void_p), relres.ctypes.data_as(C.c_void_p), pd, nd,
                            rcs.ctypes.data_as(C.c_void_p), _stream(stream))
    if code != 0 and (code != -5 or raise_noconv):
        _check(code)
    return dict(iters=iters, relres=relres, rcs=rcs, status=STATUS.get(code, code))


class Request(C.Structure):
    """cbfm_request (see include/cbfm.h)."""
    _fields_ = [("xyz_host", _P), ("nv", _I64), ("tri_host", _P), ("nt", _I64), ("edge_block", _P),
                ("nblocks", _I32), ("medium", Medium), ("gen_host", _P), ("n_gen", _I32), ("delta_svd", C.c_double),
                ("precision", _I32), ("inc_host", _P), ("nrhs", _I64), ("tol", C.c_double), ("max_iter", _I32),
                ("restart", _I32), ("inner_fp32", _I32), ("scatterer_key", C.c_uint64)]


def make_request(V, T, edge_block, nblocks, medium, gen, delta_svd, inc, tol=1e-6, max_iter=0, restart=0,
                 precision=FP64, key=0, inner_fp32=False):
    """A Request and the host arrays it points to (keep both alive until
    the request is submitted; submission copies them)."""
    V, pv = _host(V, np.float64)
    T, pt = _host(T, np.int32)
    gen, pg = _host(gen, np.float64)
    inc, pi = _host(inc, np.float64)
    keep = [V, T, gen, inc]
    pe, nb = None, 1
    if edge_block is not None:
        eb, pe = _host(edge_block, np.int32)
        keep.append(eb)
        nb = int(nblocks)
    r = Request(pv, V.size // 3, pt, T.size // 3, pe, nb, medium, pg, gen.size // 6, float(delta_svd), int(precision),
                pi, inc.size // 6, float(tol), int(max_iter), int(restart), int(bool(inner_fp32)), int(key))
    return r, keep


def request_footprint(req):
    b = _I64()
    _check(lib().cbfm_request_footprint(C.byref(req), C.byref(b)))
    return b.value


class Server:
    """cbfm_server: continuous batching of scattering solves (slots worker
    streams, admission by estimated device footprint within budget_bytes)."""

    def __init__(self, slots=2, budget_bytes=None):
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = free // 2
        h = _P()
        _check(lib().cbfm_server_create(int(slots), int(budget_bytes), C.byref(h)))
        self._h = h
        self._nrhs = {}

    def submit(self, req):
        t = _I64()
        _check(lib().cbfm_server_submit(self._h, C.byref(req), C.byref(t)))
        self._nrhs[t.value] = req.nrhs
        return t.value

    def wait(self, ticket):
        n = self._nrhs.pop(ticket)
        rcs = np.zeros(n)
        iters = np.zeros(n, np.int32)
        times = np.zeros(3)
        code = lib().cbfm_server_wait(self._h, int(ticket), rcs.ctypes.data_as(_P), iters.ctypes.data_as(_P),
                                      times.ctypes.data_as(_P))
        if code not in (0, -5):
            _check(code)
        return dict(rcs=rcs, iters=iters, t_submit=times[0], t_start=times[1], t_end=times[2],
                    status=STATUS.get(code, code))

    def stats(self):
        pb, mr, res = _I64(), _I32(), _I32()
        _check(lib().cbfm_server_stats(self._h, C.byref(pb), C.byref(mr), C.byref(res)))
        return dict(peak_bytes=pb.value, max_running=mr.value, resident=res.value)

    def close(self):
        if self._h:
            lib().cbfm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
