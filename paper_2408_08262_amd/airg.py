"""Python binding of the AIRG HIP library (libairg.so), argument marshalling only.

Every function here forwards to the C entry point of the same name declared in
include/airg.h and include/airg_steps.h; all arithmetic runs in the library's
HIP kernels.  Device memory and streams come from PyTorch: matrices and
vectors are passed as contiguous CUDA (ROCm) tensors, and each call runs on
``torch.cuda.current_stream()`` unless a stream is given.  A missing library
raises immediately -- there is no fallback path.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libairg.so")

OK, NOT_CONVERGED = 0, 1
F_POINT, C_POINT = 1, 2
OUTER_RICHARDSON, OUTER_FGMRES = 0, 1
PHASES = ("cf", "extract", "poly", "restrictor", "prolongator", "coarse", "finalize")


class AirgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("airg status %d: %s" % (status, msg))
        self.status = status


class Opts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("pmisr_max_rounds", C.c_int32),
                ("strong_threshold", C.c_double), ("ddc_threshold", C.c_double), ("ddc_fraction", C.c_double),
                ("drop_R", C.c_double), ("drop_A", C.c_double), ("poly_order", C.c_int32),
                ("poly_sparsity_order", C.c_int32), ("coarse_poly_order", C.c_int32),
                ("coarse_iters", C.c_int32), ("truncate_n", C.c_int64), ("max_levels", C.c_int32),
                ("up_smooths", C.c_int32), ("down_smooths", C.c_int32), ("precond_precision", C.c_int32),
                ("outer", C.c_int32), ("fgmres_restart", C.c_int32), ("seed", C.c_uint64),
                ("build_adjoint", C.c_int32), ("onepoint_weight", C.c_int32), ("use_graph", C.c_int32),
                ("autotune", C.c_int32), ("device_bytes_cap", C.c_int64),
                ("coarse_matrix_free", C.c_int32), ("time_phases", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("seconds", C.c_double)]


class LevelInfo(C.Structure):
    _fields_ = [("level", C.c_int32), ("coarsest", C.c_int32), ("n", C.c_int64), ("n_f", C.c_int64),
                ("n_c", C.c_int64), ("nnz_a", C.c_int64), ("nnz_aff", C.c_int64), ("nnz_afc", C.c_int64),
                ("nnz_ainv", C.c_int64), ("nnz_z", C.c_int64), ("nnz_w", C.c_int64),
                ("poly_terms", C.c_int32), ("poly_requested", C.c_int32), ("alpha", C.c_double * 16),
                ("setup_seconds", C.c_double * 7), ("setup_bytes", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("reserved", C.c_int32), ("grid_complexity", C.c_double),
                ("operator_complexity", C.c_double), ("storage_complexity", C.c_double),
                ("setup_seconds", C.c_double), ("phase_seconds", C.c_double * 7),
                ("vcycle_bytes_fp64", C.c_int64), ("vcycle_bytes_fp32", C.c_int64),
                ("top_spmv_bytes_fp64", C.c_int64), ("device_bytes", C.c_int64),
                ("resetup_seconds", C.c_double), ("vcycle_nnz", C.c_int64), ("top_nnz", C.c_int64),
                ("cycles_eager", C.c_int64), ("cycles_graph", C.c_int64), ("setup_bytes", C.c_int64),
                ("vcycle_index_bytes", C.c_int64), ("vcycle_vec_entries", C.c_int64)]


_VP, _I32, _I64, _U64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
_SIGS = {
    "airg_default_opts": [C.POINTER(Opts)],
    "airg_setup": [C.POINTER(Opts), _I64, _I64, _VP, _VP, _VP, _I32, _VP, _VP, _VP, C.POINTER(_VP)],
    "airg_solve": [_VP, _I32, _VP, _VP, _D, _I32, _VP, C.POINTER(SolveInfo)],
    "airg_adjoint_solve": [_VP, _I32, _VP, _VP, _D, _I32, _VP, C.POINTER(SolveInfo)],
    "airg_get_stats": [_VP, C.POINTER(Stats)],
    "airg_resetup": [_VP, _VP, _VP],
    "airg_vcycle": [_VP, _I32, _VP, _VP, _I32, _VP],
    "airg_batch_vcycle": [_VP, _I32, _VP, _VP, _VP],
    "airg_vcycle_profile": [_VP, _I32, _I32, _I32, _VP, _I32, _VP],
    "airg_batch_vcycle_profile": [_VP, _I32, _I32, _VP, _I32, _VP],
    "airg_get_level": [_VP, _I32, _I32, C.POINTER(LevelInfo), _VP],
    "airg_get_level_matrix": [_VP, _I32, _I32, _I32, _VP, _VP, _VP],
    "airg_csr_info": [_VP, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)],
    "airg_csr_to_host": [_VP, _VP, _VP, _VP],
    "airg_strength": [_I64, _I64, _VP, _VP, _VP, _D, _VP, _VP, _VP],
    "airg_pmisr": [_I64, _I64, _VP, _VP, _VP, _D, _VP, _U64, _I32, _I32, _VP, C.POINTER(_I32), _VP],
    "airg_ddc": [_I64, _I64, _VP, _VP, _VP, _D, _VP, _VP, _VP, _VP],
    "airg_ddc_fraction_threshold": [_I64, _I64, _VP, _VP, _VP, _VP, _D, C.POINTER(_D), _VP],
    "airg_ddc_fraction_threshold_noalloc": [_I64, _I64, _VP, _VP, _VP, _VP, _D, C.POINTER(_D), _VP],
    "airg_cf_split": [_I64, _I64, _VP, _VP, _VP, C.POINTER(Opts), _I32, _VP, C.POINTER(_I64), C.POINTER(_I64),
                      _VP],
    "airg_extract": [_I64, _I64, _VP, _VP, _VP, _VP, C.c_int8, C.c_int8, C.POINTER(_VP), _VP],
    "airg_spmv": [_I64, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _VP],
    "airg_gauss_rhs": [_I64, _U64, _I32, _VP, _VP],
    "airg_tsqr_r": [_I64, _I32, _VP, _VP, _VP, _VP],
    "airg_gmres_poly": [_I64, _I64, _VP, _VP, _VP, _U64, _I32, _I32, _VP, _VP, _VP, C.POINTER(_I32), _VP],
    "airg_poly_fixed_sparsity": [_I64, _I64, _VP, _VP, _VP, _I32, _VP, _VP, _VP],
    "airg_spgemm": [_I64, _I64, _I64, _VP, _VP, _VP, _I64, _I64, _VP, _VP, _VP, C.POINTER(_VP), _VP],
    "airg_drop": [_I64, _I64, _I64, _VP, _VP, _VP, _D, _I32, _I32, C.POINTER(_VP), _VP],
    "airg_onepoint_w": [_I64, _I64, _VP, _VP, _VP, _VP, _I32, C.POINTER(_VP), _VP],
    "airg_transpose": [_I64, _I64, _I64, _VP, _VP, _VP, C.POINTER(_VP), _VP],
    "airg_level_build": [_I64, _I64, _VP, _VP, _VP, C.POINTER(Opts), _I32, _VP, _VP, _VP, C.POINTER(_VP),
                         C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP), _VP],
}
_SIGS["airg_kernel_timing"] = [_I32]
_SIGS["airg_blockdiag_axpy"] = [_I64, _I32, _VP, _VP, _VP, _VP, _VP, _VP]
_SIGS["airg_blockdiag_apply"] = [_I64, _I32, _VP, _VP, _VP, _VP]
_SIGS["airg_blockdiag_bilinear"] = [_I64, _I32, _VP, _VP, _VP, _D, _VP, _VP]
_SIGS["airg_kernel_timing_read"] = [C.POINTER(_I64), C.POINTER(_D), C.POINTER(_D)]
EXPORTS = tuple(_SIGS) + ("airg_destroy", "airg_status_string", "airg_last_error", "airg_csr_free",
                         "airg_ddc_fraction_threshold_noalloc_max_rows")

_lib = None


def lib():
    """Loads libairg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libairg.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.airg_destroy.argtypes = [_VP]
        L.airg_destroy.restype = None
        L.airg_csr_free.argtypes = [_VP]
        L.airg_csr_free.restype = None
        L.airg_status_string.argtypes = [C.c_int]
        L.airg_status_string.restype = C.c_char_p
        L.airg_last_error.argtypes = []
        L.airg_last_error.restype = C.c_char_p
        L.airg_ddc_fraction_threshold_noalloc_max_rows.argtypes = []
        L.airg_ddc_fraction_threshold_noalloc_max_rows.restype = _I64
        _lib = L
    return _lib


def _check(st, allow=(OK,)):
    if st in allow:
        return st
    msg = lib().airg_last_error().decode() or lib().airg_status_string(st).decode()
    raise AirgError(st, msg)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _ptr(t, dtype):
    return C.c_void_p(0) if t is None else _dev(t, dtype)


def to_device(rowptr, col, val=None, device="cuda"):
    """numpy CSR -> (int32 rowptr, int32 col, float64 val) device tensors."""
    out = [torch.as_tensor(np.ascontiguousarray(rowptr, dtype=np.int32), device=device),
           torch.as_tensor(np.ascontiguousarray(col, dtype=np.int32), device=device)]
    if val is not None:
        out.append(torch.as_tensor(np.ascontiguousarray(val, dtype=np.float64), device=device))
    return tuple(out)


def default_opts(**kw):
    o = Opts()
    _check(lib().airg_default_opts(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------- library matrices --
class DevCsr:
    """Matrix returned by the library (airg_csr); freed with the object."""

    def __init__(self, ptr):
        self.ptr = C.c_void_p(ptr)

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value and _lib is not None:
            _lib.airg_csr_free(self.ptr)
            self.ptr = None

    def info(self):
        nr, nc, nz = _I64(), _I64(), _I64()
        _check(lib().airg_csr_info(self.ptr, C.byref(nr), C.byref(nc), C.byref(nz)))
        return nr.value, nc.value, nz.value

    def to_host(self):
        nr, nc, nz = self.info()
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(nz, np.int32)
        v = np.zeros(nz, np.float64)
        _check(lib().airg_csr_to_host(self.ptr, rp.ctypes.data_as(_VP), ci.ctypes.data_as(_VP),
                                      v.ctypes.data_as(_VP)))
        return rp, ci, v, nc


def _out_csr(call):
    p = _VP()
    call(C.byref(p))
    return DevCsr(p.value)


# ------------------------------------------------------------- hierarchy --
class Handle:
    def __init__(self, ptr, n):
        self.ptr = C.c_void_p(ptr)
        self.n = n

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value and _lib is not None:
            _lib.airg_destroy(self.ptr)
            self.ptr = None


def airg_setup(rowptr, col, val, opts=None, seg_offsets=None, seg_seeds=None, stream=None):
    """Builds the hierarchy of the CSR matrix given as device tensors."""
    opts = opts if opts is not None else default_opts()
    n = rowptr.numel() - 1
    nnz = col.numel()
    nseg = 1
    offs = seeds = None
    if seg_offsets is not None:
        offs = np.ascontiguousarray(seg_offsets, dtype=np.int64)
        nseg = len(offs) - 1
        if seg_seeds is not None:
            seeds = np.ascontiguousarray(seg_seeds, dtype=np.uint64)
    out = _VP()
    _check(lib().airg_setup(C.byref(opts), n, nnz, _dev(rowptr, torch.int32), _dev(col, torch.int32),
                            _dev(val, torch.float64), nseg,
                            None if offs is None else offs.ctypes.data_as(_VP),
                            None if seeds is None else seeds.ctypes.data_as(_VP), _stream(stream), C.byref(out)))
    return Handle(out.value, n)


def _solve(fn, h, b, rtol, max_it, stream, allow_not_converged):
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    x = torch.empty_like(b)
    info = SolveInfo()
    st = fn(h.ptr, nrhs, _dev(b, torch.float64), _dev(x, torch.float64), rtol, max_it, _stream(stream),
            C.byref(info))
    _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
    return x, {"iterations": info.iterations, "converged": bool(info.converged),
               "rel_residual": info.rel_residual, "seconds": info.seconds}


def airg_solve(h, b, rtol=1e-10, max_it=200, stream=None, allow_not_converged=False):
    """x with A x = b (b: (n,) or (n, nrhs) float64 device tensor)."""
    return _solve(lib().airg_solve, h, b, rtol, max_it, stream, allow_not_converged)


def airg_adjoint_solve(h, g, rtol=1e-10, max_it=200, stream=None, allow_not_converged=False):
    """lambda with A^T lambda = g, by an AIRG hierarchy built on A^T."""
    return _solve(lib().airg_adjoint_solve, h, g, rtol, max_it, stream, allow_not_converged)


def airg_resetup(h, val, stream=None):
    """Numeric re-setup with new values (device float64 tensor, nnz entries in
    the order of the matrix given to airg_setup)."""
    _check(lib().airg_resetup(h.ptr, _dev(val, torch.float64), _stream(stream)))


def airg_vcycle(h, g, precision=64, segment=0, stream=None):
    """e = V(g): one V-cycle of the hierarchy, natural order."""
    e = torch.empty_like(g)
    _check(lib().airg_vcycle(h.ptr, segment, _dev(g, torch.float64), _dev(e, torch.float64), precision,
                             _stream(stream)))
    return e


def airg_vcycle_profile(h, precision=32, reps=10, segment=0, stream=None):
    """Mean device seconds per V-cycle of each level's own work (eager cycles
    with events around every level), as a list indexed by level."""
    nl = airg_get_stats(h)["levels"]
    out = (C.c_double * max(nl, 1))()
    _check(lib().airg_vcycle_profile(h.ptr, segment, precision, reps, out, nl, _stream(stream)))
    return list(out)[:nl]


def airg_batch_vcycle_profile(h, nrhs=4, reps=10, stream=None):
    """Mean device seconds per batched FP32 cycle of each level's own stages."""
    nl = airg_get_stats(h)["levels"]
    out = (C.c_double * max(nl, 1))()
    _check(lib().airg_batch_vcycle_profile(h.ptr, nrhs, reps, out, nl, _stream(stream)))
    return list(out)[:nl]


def airg_batch_vcycle(h, g, stream=None):
    """E = V(G): one batched FP32 V-cycle over every segment and right-hand
    side (G: (n, nrhs) float64 device tensor, natural order)."""
    nrhs = 1 if g.dim() == 1 else g.shape[1]
    e = torch.empty_like(g)
    _check(lib().airg_batch_vcycle(h.ptr, nrhs, _dev(g, torch.float64), _dev(e, torch.float64), _stream(stream)))
    return e


def airg_get_stats(h):
    s = Stats()
    _check(lib().airg_get_stats(h.ptr, C.byref(s)))
    d = {k: getattr(s, k) for k, _ in Stats._fields_ if k not in ("phase_seconds", "reserved")}
    d["phase_seconds"] = dict(zip(PHASES, list(s.phase_seconds)))
    return d


def airg_get_level(h, level, segment=0, with_cf=True):
    info = LevelInfo()
    _check(lib().airg_get_level(h.ptr, segment, level, C.byref(info), None))
    d = {k: getattr(info, k) for k, _ in LevelInfo._fields_ if k not in ("alpha", "setup_seconds")}
    d["alpha"] = np.array(list(info.alpha)[:info.poly_requested])
    d["setup_seconds"] = dict(zip(PHASES, list(info.setup_seconds)))
    if with_cf:
        cf = np.zeros(info.n, np.int8)
        _check(lib().airg_get_level(h.ptr, segment, level, C.byref(info), cf.ctypes.data_as(_VP)))
        d["cf"] = cf
    return d


_WHICH = {"A": (0, "nnz_a", "n", "n"), "Ainv": (1, "nnz_ainv", "n_f", "n_f"), "Z": (2, "nnz_z", "n_c", "n_f"),
          "W": (3, "nnz_w", "n_f", "n_c"), "Aff": (4, "nnz_aff", "n_f", "n_f"), "Afc": (5, "nnz_afc", "n_f", "n_c")}


def airg_get_level_matrix(h, level, which, segment=0):
    """(rowptr, col, val, ncols) numpy arrays of one level matrix."""
    info = airg_get_level(h, level, segment, with_cf=False)
    code, nzk, rk, ck = _WHICH[which]
    nr, nc = info[rk], info[ck]
    if info["coarsest"] and which in ("A", "Ainv"):
        nr = nc = info["n"]
    nz = info[nzk]
    rp = np.zeros(nr + 1, np.int32)
    ci = np.zeros(nz, np.int32)
    v = np.zeros(nz, np.float64)
    _check(lib().airg_get_level_matrix(h.ptr, segment, level, code, rp.ctypes.data_as(_VP),
                                       ci.ctypes.data_as(_VP), v.ctypes.data_as(_VP)))
    return rp, ci, v, nc


def airg_kernel_timing(enable):
    """Turns event timing of the finest-operator SpMV kernel on (clearing) or off."""
    _check(lib().airg_kernel_timing(1 if enable else 0))


def airg_kernel_timing_read():
    """(launches, algorithmic bytes, event seconds) recorded since enabling."""
    n, b, t = _I64(), _D(), _D()
    _check(lib().airg_kernel_timing_read(C.byref(n), C.byref(b), C.byref(t)))
    return n.value, b.value, t.value


def airg_blockdiag_axpy(mass, sigma, pos, base, val, stream=None):
    """val[pos] = base[pos] + sigma_K M_K (mass: (ncell, bs, bs))."""
    ncell, bs = mass.shape[0], mass.shape[1]
    _check(lib().airg_blockdiag_axpy(ncell, bs, _dev(mass, torch.float64), _dev(sigma, torch.float64),
                                     _dev(pos, torch.int32), _dev(base, torch.float64), _dev(val, torch.float64),
                                     _stream(stream)))


def airg_blockdiag_apply(mass, x, stream=None):
    ncell, bs = mass.shape[0], mass.shape[1]
    y = torch.empty_like(x)
    _check(lib().airg_blockdiag_apply(ncell, bs, _dev(mass, torch.float64), _dev(x, torch.float64),
                                      _dev(y, torch.float64), _stream(stream)))
    return y


def airg_blockdiag_bilinear(mass, u, lam, scale=1.0, stream=None):
    ncell, bs = mass.shape[0], mass.shape[1]
    out = torch.empty(ncell, dtype=torch.float64, device=u.device)
    _check(lib().airg_blockdiag_bilinear(ncell, bs, _dev(mass, torch.float64), _dev(u, torch.float64),
                                         _dev(lam, torch.float64), scale, _dev(out, torch.float64),
                                         _stream(stream)))
    return out


# ----------------------------------------------------------------- steps --
def _csr_args(A):
    rp, ci, v = A[0], A[1], A[2]
    return rp.numel() - 1, ci.numel(), _dev(rp, torch.int32), _dev(ci, torch.int32), _dev(v, torch.float64)


def airg_strength(A, alpha, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    strong = torch.empty(nnz, dtype=torch.uint8, device=A[0].device)
    deg = torch.empty(n, dtype=torch.int32, device=A[0].device)
    _check(lib().airg_strength(n, nnz, rp, ci, v, alpha, _dev(strong, torch.uint8), _dev(deg, torch.int32),
                               _stream(stream)))
    return strong, deg


def airg_pmisr(A, alpha, max_rounds, h=None, seed=0, level=0, stream=None):
    """h: optional int32 device tensor holding the 32-bit random parts."""
    n, nnz, rp, ci, v = _csr_args(A)
    cf = torch.empty(n, dtype=torch.int8, device=A[0].device)
    rounds = _I32()
    _check(lib().airg_pmisr(n, nnz, rp, ci, v, alpha, _ptr(h, torch.int32), seed, level, max_rounds,
                            _dev(cf, torch.int8), C.byref(rounds), _stream(stream)))
    return cf, rounds.value


def airg_ddc(A, alpha_diag, cf_in, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    cf = torch.empty_like(cf_in)
    theta = torch.empty(n, dtype=torch.float64, device=A[0].device)
    _check(lib().airg_ddc(n, nnz, rp, ci, v, alpha_diag, _dev(cf_in, torch.int8), _dev(cf, torch.int8),
                          _dev(theta, torch.float64), _stream(stream)))
    return cf, theta


def airg_ddc_fraction_threshold(A, cf, fraction, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    out = _D()
    _check(lib().airg_ddc_fraction_threshold(n, nnz, rp, ci, v, _dev(cf, torch.int8), fraction, C.byref(out),
                                             _stream(stream)))
    return out.value


def airg_ddc_fraction_threshold_noalloc(A, cf, fraction, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    out = _D()
    _check(lib().airg_ddc_fraction_threshold_noalloc(n, nnz, rp, ci, v, _dev(cf, torch.int8), fraction,
                                                     C.byref(out), _stream(stream)))
    return out.value


def ddc_fraction_noalloc_max_rows():
    return int(lib().airg_ddc_fraction_threshold_noalloc_max_rows())


def airg_cf_split(A, opts, level=0, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    cf = torch.empty(n, dtype=torch.int8, device=A[0].device)
    nf, nc = _I64(), _I64()
    _check(lib().airg_cf_split(n, nnz, rp, ci, v, C.byref(opts), level, _dev(cf, torch.int8), C.byref(nf),
                               C.byref(nc), _stream(stream)))
    return cf, nf.value, nc.value


def airg_extract(A, cf, rowsel, colsel, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    return _out_csr(lambda o: _check(lib().airg_extract(n, nnz, rp, ci, v, _dev(cf, torch.int8), rowsel, colsel, o,
                                                        _stream(stream))))


def airg_spmv(A, x, ncols=None, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    y = torch.empty(n, dtype=torch.float64, device=x.device)
    _check(lib().airg_spmv(n, ncols if ncols is not None else x.numel(), nnz, rp, ci, v, _dev(x, torch.float64),
                           _dev(y, torch.float64), _stream(stream)))
    return y


def airg_gauss_rhs(n, seed, level, device="cuda", stream=None):
    b = torch.empty(n, dtype=torch.float64, device=device)
    _check(lib().airg_gauss_rhs(n, seed, level, _dev(b, torch.float64), _stream(stream)))
    return b


def airg_tsqr_r(K, stream=None):
    """K: (cols, rows) device tensor holding the columns of the tall matrix."""
    cols, rows = K.shape
    R = np.zeros((cols, cols))
    nrm = np.zeros(cols)
    _check(lib().airg_tsqr_r(rows, cols, _dev(K, torch.float64), R.ctypes.data_as(_VP), nrm.ctypes.data_as(_VP),
                             _stream(stream)))
    return R, nrm


def airg_gmres_poly(A, seed, level, m, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    alpha = np.zeros(m)
    R = np.zeros((m + 1, m + 1))
    nrm = np.zeros(m + 1)
    used = _I32()
    _check(lib().airg_gmres_poly(n, nnz, rp, ci, v, seed, level, m, alpha.ctypes.data_as(_VP),
                                 R.ctypes.data_as(_VP), nrm.ctypes.data_as(_VP), C.byref(used), _stream(stream)))
    return alpha, used.value, R, nrm


def airg_poly_fixed_sparsity(A, alpha, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    out = torch.empty(nnz, dtype=torch.float64, device=A[0].device)
    _check(lib().airg_poly_fixed_sparsity(n, nnz, rp, ci, v, len(alpha), alpha.ctypes.data_as(_VP),
                                          _dev(out, torch.float64), _stream(stream)))
    return out


def airg_spgemm(A, B, a_cols, b_cols, stream=None):
    m, nza, arp, aci, av = _csr_args(A)
    k, nzb, brp, bci, bv = _csr_args(B)
    return _out_csr(lambda o: _check(lib().airg_spgemm(m, a_cols, nza, arp, aci, av, b_cols, nzb, brp, bci, bv, o,
                                                       _stream(stream))))


def airg_drop(A, ncols, tau, keep_diag, negate=False, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    return _out_csr(lambda o: _check(lib().airg_drop(n, ncols, nnz, rp, ci, v, tau, int(keep_diag), int(negate), o,
                                                     _stream(stream))))


def airg_onepoint_w(A, cf, weight_mode=0, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    return _out_csr(lambda o: _check(lib().airg_onepoint_w(n, nnz, rp, ci, v, _dev(cf, torch.int8), weight_mode, o,
                                                           _stream(stream))))


def airg_transpose(A, ncols, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    return _out_csr(lambda o: _check(lib().airg_transpose(n, ncols, nnz, rp, ci, v, o, _stream(stream))))


def airg_level_build(A, opts, level, alpha_in=None, stream=None):
    n, nnz, rp, ci, v = _csr_args(A)
    m = opts.poly_order + 1
    cf = torch.empty(n, dtype=torch.int8, device=A[0].device)
    aout = np.zeros(m)
    ain = None if alpha_in is None else np.ascontiguousarray(alpha_in, dtype=np.float64)
    ptrs = [_VP() for _ in range(4)]
    _check(lib().airg_level_build(n, nnz, rp, ci, v, C.byref(opts), level,
                                  None if ain is None else ain.ctypes.data_as(_VP), _dev(cf, torch.int8),
                                  aout.ctypes.data_as(_VP), *[C.byref(p) for p in ptrs], _stream(stream)))
    Ainv, Z, W, Ac = [DevCsr(p.value) for p in ptrs]
    return {"cf": cf, "alpha": aout, "Ainv": Ainv, "Z": Z, "W": W, "Ac": Ac}
