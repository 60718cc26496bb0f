"""ctypes binding of libbras.so (argument marshalling only).

Every function keeps the C name.  Host helpers take and return NumPy arrays;
device entry points take torch tensors on the GPU (PyTorch is used only for
device memory and streams) and the current torch stream.  There is no
fallback: if the library is missing or fails to load, LibraryMissing is
raised.
"""
import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbras.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bras.h")

BRAS_OK, BRAS_EINVAL, BRAS_ENOTSPD, BRAS_EHIP, BRAS_ENOCONV, BRAS_EBREAKDOWN, BRAS_ENOMEM = 0, -1, -2, -3, -4, -5, -6
H1, HCURL, HDIV, H1_BERNSTEIN, HCURL2, HDIV2 = 0, 1, 2, 3, 4, 5
ELEM_EXPLICIT, ELEM_SCALED_REF, ELEM_METRIC_REF = 0, 1, 2
FP64, FP32, BF16 = 0, 1, 2
PC_NONE, PC_JACOBI, PC_BRAS = 0, 1, 2
PC = {"none": PC_NONE, "jacobi": PC_JACOBI, "bras": PC_BRAS}
INFO = {"n": 0, "E": 1, "nloc": 2, "nbr": 3, "prec": 4, "form": 5, "maxrhs": 6, "restarts": 7, "variant": 8,
        "solve_path": 9, "patches": 10, "patch_on": 11}
EXPORT_MULT, EXPORT_ROWPTR, EXPORT_SLOT, EXPORT_DIAG = 0, 1, 2, 3
OPT_GRAPH_ITERS, OPT_MAX_RESTART, OPT_VARIANT, OPT_SMALL_CG, OPT_PATCH, OPT_FLEXIBLE = 0, 1, 2, 3, 4, 5
NOALLOC_SCRATCH_BYTES = 32 << 20   # BRAS_NOALLOC_SCRATCH_BYTES
FAMILY = {"P": H1, "N1curl": HCURL, "RT": HDIV, "B": H1_BERNSTEIN, "N2curl": HCURL2, "BDM": HDIV2}


def is_h1(family):
    return family in (H1, H1_BERNSTEIN)
PREC = {"f64": FP64, "f32": FP32, "bf16": BF16}


class LibraryMissing(RuntimeError):
    pass


class BrasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%d: %s" % (code, msg))
        self.code = code


_lib = None

vp = C.c_void_p
i32, i64, dbl, u64 = C.c_int, C.c_int64, C.c_double, C.c_uint64
P_i64, P_i32, P_dbl = C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)

_SIGS = {
    "bras_mesh_size": [i32, i32, P_i64, P_i64],
    "bras_mesh_structured": [i32, i32, dbl, u64, P_dbl, P_i32],
    "bras_element_info": [i32, i32, i32, C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "bras_reference_mass": [i32, i32, i32, P_dbl],
    "bras_dofmap": [i32, i32, i32, i64, i64, P_i32, P_i64, P_i32],
    "bras_geometry": [i32, i32, i64, vp, i64, vp, vp, vp, vp],
    "bras_setup": [C.POINTER(vp), i64, i64, i32, vp, i32, vp, vp, i32, i32, i32, vp],
    "bras_update": [vp, vp, vp],
    "bras_destroy": [vp],
    "bras_apply": [vp, vp, vp, i32, vp],
    "bras_apply_noalloc": [vp, vp, vp, i32, vp],
    "mass_apply": [vp, vp, vp, i32, vp],
    "jacobi_apply": [vp, vp, vp, i32, vp],
    "pcg_solve": [vp, i32, vp, vp, i32, dbl, i32, C.POINTER(C.c_int), P_dbl, vp],
    "bras_lambda_max": [vp, i32, vp, i32, P_dbl, vp],
    "fixed_point_solve": [vp, i32, dbl, vp, vp, i32, dbl, i32, C.POINTER(C.c_int), P_dbl, vp],
    "chebyshev_solve": [vp, i32, dbl, dbl, vp, vp, i32, dbl, i32, C.POINTER(C.c_int), P_dbl, vp],
    "bras_rho_grad": [vp, vp, vp, vp, vp, i32, vp],
    "bras_info": [vp, i32, P_i64],
    "bras_export": [vp, i32, vp, vp],
    "bras_set_option": [vp, i32, dbl],
    "bras_autotune": [vp, i32, vp],
    "bras_bench_bf16_local_gemm": [i32, i32, i32, vp, C.POINTER(C.c_longlong), vp],
    "bras_csr_rowptr": [vp, vp, P_i64, vp],
    "bras_csr_assemble": [vp, i32, vp, vp, vp, vp],
    "bras_csr_apply": [i64, vp, vp, vp, vp, vp, vp],
    "bras_spgemm_rowptr": [i64, i64, vp, vp, vp, vp, vp, P_i64, vp],
    "bras_spgemm_fill": [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
    "bras_csr_transpose": [i64, i64, vp, vp, vp, vp, vp, vp, vp],
    "bras_csr_add_rowptr": [i64, vp, vp, vp, vp, vp, P_i64, vp],
    "bras_csr_jacobi": [vp, vp, vp, vp, vp],
    "bras_csr_add_fill": [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
}


def header_functions():
    """Names of the functions declared in include/bras.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", txt, flags=re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing("libbras.so is not built (run python -m paper_2607_12138_amd.build)")
        try:
            L = C.CDLL(LIB_PATH)
        except OSError as e:
            raise LibraryMissing("libbras.so failed to load: %s" % e)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.bras_last_error.argtypes = []
        L.bras_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(code):
    if code != BRAS_OK:
        raise BrasError(code, lib().bras_last_error().decode())
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------
def bras_mesh_size(dim, N):
    nv, nc = C.c_int64(), C.c_int64()
    check(lib().bras_mesh_size(dim, N, C.byref(nv), C.byref(nc)))
    return nv.value, nc.value


def bras_mesh_structured(dim, N, jitter=0.0, seed=0):
    nv, nc = bras_mesh_size(dim, N)
    coords = np.empty((nv, dim), dtype=np.float64)
    cells = np.empty((nc, dim + 1), dtype=np.int32)
    check(lib().bras_mesh_structured(dim, N, float(jitter), C.c_uint64(seed), _ptr(coords, C.c_double),
                                     _ptr(cells, C.c_int32)))
    return coords, cells


def bras_element_info(family, dim, degree):
    nl = C.c_int()
    cnt = (C.c_int * 4)()
    check(lib().bras_element_info(family, dim, degree, C.byref(nl), cnt))
    return nl.value, tuple(cnt[: dim + 1])


def nsym(dim):
    return dim * (dim + 1) // 2


def bras_reference_mass(family, dim, degree):
    nl, _ = bras_element_info(family, dim, degree)
    k = 1 if is_h1(family) else nsym(dim)
    out = np.empty((k, nl, nl), dtype=np.float64)
    check(lib().bras_reference_mass(family, dim, degree, _ptr(out, C.c_double)))
    return out[0] if is_h1(family) else out


def bras_dofmap(family, dim, degree, nvert, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    nl, _ = bras_element_info(family, dim, degree)
    l2g = np.empty((len(cells), nl), dtype=np.int32)
    n = C.c_int64()
    check(lib().bras_dofmap(family, dim, degree, nvert, len(cells), _ptr(cells, C.c_int32), C.byref(n),
                            _ptr(l2g, C.c_int32)))
    return n.value, l2g


# ---------------------------------------------------------------------------
# device entry points (torch tensors on the GPU)
# ---------------------------------------------------------------------------
def _dev(t):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def bras_geometry(family, dim, coords_d, cells_d, rho_d, elem_d, stream=None):
    check(lib().bras_geometry(family, dim, coords_d.shape[0], _dev(coords_d), cells_d.shape[0], _dev(cells_d),
                              _dev(rho_d), _dev(elem_d), _stream(stream)))


def bras_setup(n, E, n_loc, l2g_d, form, ref_d, elem_d, nsym_, prec, max_rhs, stream=None):
    h = C.c_void_p()
    check(lib().bras_setup(C.byref(h), n, E, n_loc, _dev(l2g_d), form, _dev(ref_d), _dev(elem_d), nsym_, prec,
                           max_rhs, _stream(stream)))
    return h


def bras_update(h, elem_d, stream=None):
    check(lib().bras_update(h, _dev(elem_d), _stream(stream)))


def bras_destroy(h):
    check(lib().bras_destroy(h))


def _nrhs(x):
    return 1 if x.dim() == 1 else x.shape[1]


def bras_apply(h, x_d, y_d, stream=None):
    check(lib().bras_apply(h, _dev(x_d), _dev(y_d), _nrhs(x_d), _stream(stream)))


def bras_apply_noalloc(h, x_d, y_d, stream=None):
    check(lib().bras_apply_noalloc(h, _dev(x_d), _dev(y_d), _nrhs(x_d), _stream(stream)))


def bras_bench_bf16_local_gemm(n_loc, iters, blocks, out_d=None, stream=None):
    """Microbenchmark launch (asynchronous); returns the issued matrix-core FLOPs."""
    fl = C.c_longlong(0)
    launch = int(blocks) > 0
    check(lib().bras_bench_bf16_local_gemm(int(n_loc), int(iters), int(blocks), _dev(out_d) if launch else None,
                                           C.byref(fl), _stream(stream) if launch else None))
    return int(fl.value)


def mass_apply(h, x_d, y_d, stream=None):
    check(lib().mass_apply(h, _dev(x_d), _dev(y_d), _nrhs(x_d), _stream(stream)))


def jacobi_apply(h, x_d, y_d, stream=None):
    check(lib().jacobi_apply(h, _dev(x_d), _dev(y_d), _nrhs(x_d), _stream(stream)))


def pcg_solve(h, pc, b_d, x_d, rtol, maxit, stream=None, raise_on=(BRAS_EINVAL, BRAS_EHIP, BRAS_ENOMEM)):
    """Returns (status, iterations [nrhs], true relative residuals [nrhs])."""
    R = _nrhs(b_d)
    its = (C.c_int * R)()
    rel = (C.c_double * R)()
    st = lib().pcg_solve(h, pc, _dev(b_d), _dev(x_d), R, float(rtol), int(maxit), its, rel, _stream(stream))
    if st in raise_on:
        check(st)
    return st, np.array(its[:]), np.array(rel[:])


def bras_lambda_max(h, pc, v0_d, iters=50, stream=None):
    lam = C.c_double()
    check(lib().bras_lambda_max(h, pc, _dev(v0_d), int(iters), C.byref(lam), _stream(stream)))
    return lam.value


def fixed_point_solve(h, pc, omega, b_d, x_d, rtol, maxit, stream=None,
                      raise_on=(BRAS_EINVAL, BRAS_EHIP, BRAS_ENOMEM)):
    """Returns (status, updates [nrhs], relative residuals [nrhs])."""
    R = _nrhs(b_d)
    its = (C.c_int * R)()
    rel = (C.c_double * R)()
    st = lib().fixed_point_solve(h, pc, float(omega), _dev(b_d), _dev(x_d), R, float(rtol), int(maxit), its, rel,
                                 _stream(stream))
    if st in raise_on:
        check(st)
    return st, np.array(its[:]), np.array(rel[:])


def chebyshev_solve(h, pc, lmin, lmax, b_d, x_d, rtol, maxit, stream=None,
                    raise_on=(BRAS_EINVAL, BRAS_EHIP, BRAS_ENOMEM)):
    """Returns (status, updates [nrhs], relative residuals [nrhs])."""
    R = _nrhs(b_d)
    its = (C.c_int * R)()
    rel = (C.c_double * R)()
    st = lib().chebyshev_solve(h, pc, float(lmin), float(lmax), _dev(b_d), _dev(x_d), R, float(rtol), int(maxit),
                               its, rel, _stream(stream))
    if st in raise_on:
        check(st)
    return st, np.array(its[:]), np.array(rel[:])


def bras_rho_grad(h, x_d, lam_d, dcoef_d, g_d, stream=None):
    check(lib().bras_rho_grad(h, _dev(x_d), _dev(lam_d), _dev(dcoef_d), _dev(g_d), _nrhs(x_d), _stream(stream)))


def bras_info(h, what):
    v = C.c_int64()
    check(lib().bras_info(h, INFO[what] if isinstance(what, str) else what, C.byref(v)))
    return v.value


def bras_export(h, what, dst_d, stream=None):
    check(lib().bras_export(h, what, _dev(dst_d), _stream(stream)))


OP_MASS, OP_BRAS, OP_JACOBI = 0, 1, 2


def bras_csr_rowptr(h, rowptr_d, stream=None):
    nnz = C.c_int64()
    check(lib().bras_csr_rowptr(h, _dev(rowptr_d), C.byref(nnz), _stream(stream)))
    return nnz.value


def bras_csr_assemble(h, op, rowptr_d, col_d, val_d, stream=None):
    check(lib().bras_csr_assemble(h, op, _dev(rowptr_d), _dev(col_d), _dev(val_d), _stream(stream)))


def bras_csr_apply(n, rowptr_d, col_d, val_d, x_d, y_d, stream=None):
    check(lib().bras_csr_apply(n, _dev(rowptr_d), _dev(col_d), _dev(val_d), _dev(x_d), _dev(y_d), _stream(stream)))


def bras_spgemm_rowptr(m, k, a, b, c_rowptr_d, stream=None):
    """Row pointers of C = A B (a, b: (rowptr, col, val) device tensors); returns nnz(C)."""
    nnz = C.c_int64()
    check(lib().bras_spgemm_rowptr(m, k, _dev(a[0]), _dev(a[1]), _dev(b[0]), _dev(b[1]), _dev(c_rowptr_d),
                                   C.byref(nnz), _stream(stream)))
    return nnz.value


def bras_spgemm_fill(m, k, a, b, c, stream=None):
    check(lib().bras_spgemm_fill(m, k, _dev(a[0]), _dev(a[1]), _dev(a[2]), _dev(b[0]), _dev(b[1]), _dev(b[2]),
                                 _dev(c[0]), _dev(c[1]), _dev(c[2]), _stream(stream)))


def bras_csr_transpose(m, n, a, t, stream=None):
    check(lib().bras_csr_transpose(m, n, _dev(a[0]), _dev(a[1]), _dev(a[2]), _dev(t[0]), _dev(t[1]), _dev(t[2]),
                                   _stream(stream)))


def bras_csr_jacobi(h, rowptr_d, col_d, val_d, stream=None):
    check(lib().bras_csr_jacobi(h, _dev(rowptr_d), _dev(col_d), _dev(val_d), _stream(stream)))


def bras_csr_add_rowptr(m, a, b, c_rowptr_d, stream=None):
    """Row pointers of C = A + B; returns nnz(C)."""
    nnz = C.c_int64()
    check(lib().bras_csr_add_rowptr(m, _dev(a[0]), _dev(a[1]), _dev(b[0]), _dev(b[1]), _dev(c_rowptr_d),
                                    C.byref(nnz), _stream(stream)))
    return nnz.value


def bras_csr_add_fill(m, a, b, c, stream=None):
    check(lib().bras_csr_add_fill(m, _dev(a[0]), _dev(a[1]), _dev(a[2]), _dev(b[0]), _dev(b[1]), _dev(b[2]),
                                  _dev(c[0]), _dev(c[1]), _dev(c[2]), _stream(stream)))


def bras_set_option(h, opt, value):
    check(lib().bras_set_option(h, opt, float(value)))


def bras_autotune(h, nrhs, stream=None):
    check(lib().bras_autotune(h, nrhs, _stream(stream)))


def bras_last_error():
    return lib().bras_last_error().decode()
