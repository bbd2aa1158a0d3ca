"""ctypes binding of libmas (include/mas.h): argument marshalling only.

Every step of the preconditioner and of FGMRES runs in the HIP library; this
module converts host arrays and torch device tensors to the C-ABI's pointers.
Importing it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libmas.so")

MAS_OK, MAS_NOT_CONVERGED = 0, 1
MAS_EINVAL, MAS_ESINGULAR_PATCH, MAS_ENOMEM, MAS_EHIP, MAS_ENAN = -1, -2, -3, -4, -5
MAS_TH, MAS_SV = 0, 1
MAS_RELAX_VANKA, MAS_RELAX_DLSC, MAS_RELAX_VANKA_DLSC = 0, 1, 2
MAS_DC_ALL, MAS_DC_SKIP1, MAS_DC_SKIP0, MAS_HO_AMG = 0, 1, 2, 3
MAS_FP64, MAS_FP32 = 0, 1
MAS_SOC_EVOLUTION, MAS_SOC_SYMMETRIC = 0, 1
MAS_GS_CLASSICAL, MAS_GS_MODIFIED = 0, 1


class mas_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("indptr", C.c_void_p),
                ("indices", C.c_void_p), ("data", C.c_void_p)]


class mas_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("disc", C.c_int32), ("K0", mas_csr), ("K1", mas_csr), ("Ap", mas_csr),
                ("field0", C.c_void_p), ("field1", C.c_void_p), ("dir0", C.c_void_p), ("dir1", C.c_void_p),
                ("p_nullspace", C.c_int32), ("p_weight0", C.c_void_p), ("mu_diag0", C.c_void_p),
                ("n_elem", C.c_int64), ("elem_p0", C.c_void_p), ("Pp0", mas_csr), ("Mdg", mas_csr),
                ("Mcg", mas_csr), ("n_prebuilt", C.c_int32), ("prebuilt_P", C.c_void_p),
                ("prebuilt_null_p", C.c_void_p)]


class mas_params(C.Structure):
    _fields_ = [("relax", C.c_int32), ("schedule", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("omega0", C.c_double), ("omega", C.c_double), ("eta_u", C.c_double), ("eta_p", C.c_double),
                ("cheb_deg", C.c_int32 * 3), ("precision", C.c_int32), ("restart", C.c_int32),
                ("max_coarse", C.c_int32), ("max_levels", C.c_int32), ("theta", C.c_double),
                ("seed", C.c_uint64), ("mass_rtol", C.c_double), ("nrhs_max", C.c_int32),
                ("krylov_its", C.c_int32), ("nu_dlsc", C.c_int32), ("dlsc_amg", C.c_int32),
                ("soc", C.c_int32), ("soc_eps", C.c_double), ("gram_schmidt", C.c_int32), ("autotune", C.c_int32),
                ("graphs", C.c_int32), ("full_patch_min", C.c_int32), ("bucket_min", C.c_int32),
                ("factor_blocked", C.c_int32), ("device_galerkin", C.c_int32), ("share_blocks", C.c_int32),
                ("patch_kernel", C.c_int32), ("device_sa", C.c_int32), ("spgemm_cap", C.c_int32)]


class mas_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("conv_factor", C.c_double)]


class mas_hier_info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n", C.c_int64 * 16), ("nnz", C.c_int64 * 16),
                ("n_vel", C.c_int64 * 16), ("n_patches", C.c_int64 * 16), ("patch_dofs", C.c_int64 * 16),
                ("factor_entries", C.c_int64 * 16), ("p_nnz", C.c_int64 * 16), ("coarse_n", C.c_int64),
                ("device_bytes", C.c_int64), ("bucket_patches", C.c_int64 * 16), ("patch_kernel", C.c_int32 * 16),
                ("bucket_shapes", (C.c_int32 * 16) * 16), ("patch_layout", C.c_int32 * 16)]


def _load():
    # torch first: the process must hold ONE HIP runtime, and torch ships its
    # own libamdhip64.so.7.  Loaded after libmas, torch would start a second
    # runtime beside the one libmas pulled in, and the two cannot share the GPU.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmas is not built ({LIB_PATH}); run paper_2306_06795_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.mas_default_params.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(mas_params)]
    lib.mas_default_params.restype = None
    lib.mas_setup.argtypes = [P(mas_problem), P(mas_params), C.c_void_p, P(C.c_void_p)]
    lib.mas_analyze.argtypes = [P(mas_problem), P(mas_params), P(C.c_void_p)]
    lib.mas_upload.argtypes = [C.c_void_p, C.c_void_p]
    lib.mas_workspace_size.argtypes = [C.c_void_p, P(C.c_size_t)]
    lib.mas_upload_ws.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    lib.mas_release.argtypes = [C.c_void_p]
    lib.mas_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.mas_apply_static.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.mas_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                              P(mas_solve_info), C.c_void_p]
    lib.mas_solve_rtols.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, P(C.c_double), C.c_int32,
                                    P(mas_solve_info), C.c_void_p]
    lib.mas_solve_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, P(C.c_double), P(C.c_int32),
                                   C.c_int32, P(mas_solve_info), C.c_void_p]
    lib.mas_get_info.argtypes = [C.c_void_p, P(mas_hier_info)]
    lib.mas_export_level.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64), C.c_void_p,
                                     C.c_void_p, C.c_void_p]
    lib.mas_scale_rows.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double), C.c_int32,
                                   C.c_void_p]
    lib.mas_set_timing.argtypes = [C.c_void_p, C.c_int32]
    lib.mas_get_timing.argtypes = [C.c_void_p, P(C.c_double), C.c_int32]
    lib.mas_destroy.argtypes = [C.c_void_p]
    lib.mas_error_string.argtypes = [C.c_int]
    lib.mas_error_string.restype = C.c_char_p
    lib.mas_last_error.argtypes = []
    lib.mas_last_error.restype = C.c_char_p
    for name in ("mas_setup", "mas_analyze", "mas_upload", "mas_release", "mas_workspace_size", "mas_upload_ws",
                 "mas_solve_rtols", "mas_solve_step", "mas_apply_static", "mas_scale_rows", "mas_apply", "mas_solve", "mas_get_info", "mas_export_level", "mas_set_timing",
                 "mas_get_timing", "mas_destroy"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()

EXPORTED = ("mas_default_params", "mas_setup", "mas_analyze", "mas_upload", "mas_workspace_size", "mas_upload_ws",
            "mas_release", "mas_apply", "mas_apply_static", "mas_solve", "mas_solve_rtols", "mas_solve_step",
            "mas_get_info", "mas_scale_rows", "mas_export_level", "mas_set_timing", "mas_get_timing", "mas_destroy",
            "mas_error_string", "mas_last_error")


class MasError(RuntimeError):
    def __init__(self, code: int):
        self.code = code
        super().__init__(f"{lib.mas_error_string(code).decode()}: {lib.mas_last_error().decode()}")


def _check(rc: int) -> int:
    if rc < 0:
        raise MasError(rc)
    return rc


def default_params(dim: int, disc: int = MAS_TH, relax: int = MAS_RELAX_VANKA, **over) -> mas_params:
    p = mas_params()
    lib.mas_default_params(dim, disc, relax, C.byref(p))
    for k, v in over.items():
        if k == "cheb_deg":
            for i in range(3):
                p.cheb_deg[i] = int(v[i])
        else:
            setattr(p, k, v)
    return p


def _csr(A, keep: list) -> mas_csr:
    A = A.tocsr()
    if not A.has_sorted_indices:
        A = A.sorted_indices()
    ptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ind = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    keep += [ptr, ind, val]
    return mas_csr(A.shape[0], A.shape[1], ptr.ctypes.data, ind.ctypes.data, val.ctypes.data)


def _arr(a, dtype, keep: list):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    keep.append(a)
    return a.ctypes.data


def make_problem_struct(prob, keep: list, prebuilt=None) -> mas_problem:
    """mas_problem from an object with the fields of include/mas.h (a StokesProblem).
    prebuilt: None, or (Ps, null_p) with Ps[l][f] the interpolation of field f
    from hierarchy level l + 1 to level l (scipy sparse) and null_p the
    coarsest pressure near-null vector."""
    s = mas_problem()
    s.dim = prob.dim
    s.disc = MAS_SV if prob.disc == "SV" else MAS_TH
    s.K0 = _csr(prob.K0, keep)
    s.K1 = _csr(prob.K1, keep)
    s.Ap = _csr(prob.Ap, keep)
    s.field0 = _arr(prob.field0, np.int8, keep)
    s.field1 = _arr(prob.field1, np.int8, keep)
    s.dir0 = _arr(prob.dir0, np.uint8, keep)
    s.dir1 = _arr(prob.dir1, np.uint8, keep)
    s.p_nullspace = 1 if prob.p_nullspace else 0
    s.p_weight0 = _arr(prob.p_weight0, np.float64, keep)
    s.mu_diag0 = _arr(getattr(prob, "mu_diag0", None), np.float64, keep)
    if prob.disc == "SV":
        s.n_elem = prob.elem_p0.shape[0]
        s.elem_p0 = _arr(prob.elem_p0, np.int64, keep)
        s.Pp0 = _csr(prob.Pp0, keep)
        s.Mdg = _csr(prob.Mdg, keep)
        s.Mcg = _csr(prob.Mcg, keep)
    if prebuilt is not None:
        Ps, null_p = prebuilt
        flat = [_csr(P, keep) for level in Ps for P in level]
        arr = (mas_csr * len(flat))(*flat)
        keep.append(arr)
        s.n_prebuilt = len(Ps)
        s.prebuilt_P = C.cast(arr, C.c_void_p)
        s.prebuilt_null_p = _arr(null_p, np.float64, keep)
    return s


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


class Handle:
    """Owns one mas_handle.  Device arrays are torch tensors (float64, on the GPU)."""

    def __init__(self, prob, params: mas_params, stream=None, analyze_only: bool = False, prebuilt=None):
        keep: list = []
        s = make_problem_struct(prob, keep, prebuilt)
        h = C.c_void_p()
        if analyze_only:
            _check(lib.mas_analyze(C.byref(s), C.byref(params), C.byref(h)))
        else:
            _check(lib.mas_setup(C.byref(s), C.byref(params), _stream(stream), C.byref(h)))
        self.h = h
        self.params = params
        self.n0 = prob.K0.shape[0]

    def upload(self, stream=None):
        """Device half of the setup for an analysed or released handle."""
        _check(lib.mas_upload(self.h, _stream(stream)))

    def release(self):
        """Free the device memory, keep the host analysis."""
        _check(lib.mas_release(self.h))

    def workspace_size(self) -> int:
        """Device bytes upload_ws needs (analysed handle; no device is touched)."""
        n = C.c_size_t()
        _check(lib.mas_workspace_size(self.h, C.byref(n)))
        return n.value

    def upload_ws(self, ws, stream=None):
        """Device half of the setup inside a caller-owned device tensor ``ws``
        (kept alive by the caller until release/close)."""
        _check(lib.mas_upload_ws(self.h, C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                 _stream(stream)))

    def apply(self, r, z, nrhs: int = 1, stream=None):
        _check(lib.mas_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), nrhs, _stream(stream)))

    def apply_static(self, r, z, nrhs: int = 1, stream=None):
        """mas_apply with the cycle scratch in the library's static device array."""
        _check(lib.mas_apply_static(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), nrhs,
                                    _stream(stream)))

    def solve(self, b, x, rtol=1e-8, max_it: int = 1000, nrhs: int = 1, stream=None):
        """rtol: one tolerance, or a sequence of nrhs (mas_solve_rtols)."""
        info = (mas_solve_info * nrhs)()
        if np.ndim(rtol) == 0:
            rc = _check(lib.mas_solve(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, float(rtol),
                                      max_it, info, _stream(stream)))
        else:
            tols = (C.c_double * nrhs)(*[float(v) for v in rtol])
            rc = _check(lib.mas_solve_rtols(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, tols,
                                            max_it, info, _stream(stream)))
        out = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, conv_factor=i.conv_factor)
               for i in info]
        return rc, out

    def solve_step(self, b, x, rtol, fresh, cycles: int = 1, nrhs: int = 1, stream=None):
        """One continuous-batching step (mas_solve_step): rtol and fresh are
        sequences of nrhs; returns (status, per-column info of this step)."""
        info = (mas_solve_info * nrhs)()
        tols = (C.c_double * nrhs)(*[float(v) for v in rtol])
        fr = (C.c_int32 * nrhs)(*[1 if f else 0 for f in fresh])
        rc = _check(lib.mas_solve_step(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, tols, fr,
                                       cycles, info, _stream(stream)))
        return rc, [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres) for i in info]

    def info(self) -> dict:
        hi = mas_hier_info()
        _check(lib.mas_get_info(self.h, C.byref(hi)))
        L = hi.n_levels
        return dict(n_levels=L, n=list(hi.n[:L]), nnz=list(hi.nnz[:L]), n_vel=list(hi.n_vel[:L]),
                    n_patches=list(hi.n_patches[:L]), patch_dofs=list(hi.patch_dofs[:L]),
                    factor_entries=list(hi.factor_entries[:L]), p_nnz=list(hi.p_nnz[:L]), coarse_n=hi.coarse_n,
                    device_bytes=hi.device_bytes, bucket_patches=list(hi.bucket_patches[:L]),
                    patch_kernel=list(hi.patch_kernel[:L]), patch_layout=list(hi.patch_layout[:L]),
                    bucket_shapes=[[tuple(hi.bucket_shapes[l][4 * q:4 * q + 4]) for q in range(4)
                                    if hi.bucket_shapes[l][4 * q + 3] > 0] for l in range(L)])

    def scale_rows(self, x, s_u, s_p, nrhs: int = 1, dirichlet_inverse: bool = False, stream=None):
        su = (C.c_double * nrhs)(*[float(v) for v in s_u])
        sp = (C.c_double * nrhs)(*[float(v) for v in s_p])
        _check(lib.mas_scale_rows(self.h, C.c_void_p(x.data_ptr()), nrhs, su, sp, 1 if dirichlet_inverse else 0,
                                  _stream(stream)))

    def export_level(self, level: int):
        import scipy.sparse as sp
        nr, nnz = C.c_int64(), C.c_int64()
        _check(lib.mas_export_level(self.h, level, C.byref(nr), C.byref(nnz), None, None, None))
        ptr = np.empty(nr.value + 1, np.int64)
        ind = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value, np.float64)
        _check(lib.mas_export_level(self.h, level, C.byref(nr), C.byref(nnz), ptr.ctypes.data, ind.ctypes.data,
                                    val.ctypes.data))
        return sp.csr_matrix((val, ind, ptr), shape=(nr.value, nr.value))

    def set_timing(self, on: bool):
        _check(lib.mas_set_timing(self.h, 1 if on else 0))

    TIMED_KINDS = ("tpp", "generic", "batched", "sell", "csr", "spmm")

    def timing(self):
        """{kind: (ms, launches, bytes)} for the kernel kinds of mas_get_timing."""
        out = (C.c_double * 18)()
        _check(lib.mas_get_timing(self.h, out, 18))
        return {k: (out[3 * i], int(out[3 * i + 1]), out[3 * i + 2]) for i, k in enumerate(self.TIMED_KINDS)}

    def close(self):
        if getattr(self, "h", None):
            lib.mas_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
