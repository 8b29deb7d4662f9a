"""CPU oracle of AIRG setup and solve -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C reference in
``airg_oracle.c`` (built with gcc, -O2 -ffp-contract=off) with numpy
marshalling, and shares no code with the HIP library.

CSR matrices cross this boundary as (rowptr, col, val) numpy triples.
CF markers: 1 = F point, 2 = C point.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "airg_oracle.c")

F_POINT, C_POINT = 1, 2


def build():
    """Compile the oracle shared library (always recompiles)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)


class _Csr(C.Structure):
    _fields_ = [("nr", C.c_int64), ("nc", C.c_int64), ("rp", C.POINTER(C.c_int64)),
                ("ci", C.POINTER(C.c_int32)), ("v", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("strong_threshold", C.c_double), ("ddc_threshold", C.c_double),
                ("ddc_fraction", C.c_double), ("pmisr_max_rounds", C.c_int32),
                ("poly_order", C.c_int32), ("drop_R", C.c_double), ("drop_A", C.c_double),
                ("coarse_poly_order", C.c_int32), ("coarse_iters", C.c_int32),
                ("truncate_n", C.c_int64), ("max_levels", C.c_int32), ("up_smooths", C.c_int32),
                ("onepoint_weight", C.c_int32), ("seed", C.c_uint64),
                ("poly_sparsity_order", C.c_int32), ("coarse_matrix_free", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        cs = P(_Csr)
        sig = {
            "orc_default_params": (None, [P(Params)]),
            "orc_set_threads": (None, [C.c_int32]),
            "orc_get_threads": (C.c_int32, []),
            "orc_csr_free": (None, [cs]),
            "orc_splitmix64": (C.c_uint64, [C.c_uint64]),
            "orc_counter": (C.c_uint64, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64]),
            "orc_strength": (None, [cs, C.c_double, C.c_void_p]),
            "orc_sym_graph": (C.c_int, [cs, C.c_void_p, cs]),
            "orc_pmisr_keys": (None, [cs, C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p]),
            "orc_pmisr": (C.c_int32, [cs, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
            "orc_ddc_fraction_threshold": (C.c_double, [cs, C.c_void_p, C.c_double]),
            "orc_ddc": (C.c_int64, [cs, C.c_double, C.c_void_p, C.c_void_p]),
            "orc_cf_split": (C.c_int, [cs, P(Params), C.c_int32, C.c_void_p]),
            "orc_submatrix": (C.c_int, [cs, C.c_void_p, C.c_int8, C.c_int8, cs]),
            "orc_spmv": (None, [cs, C.c_void_p, C.c_void_p]),
            "orc_spgemm": (C.c_int, [cs, cs, cs]),
            "orc_drop": (C.c_int, [cs, C.c_double, C.c_int, cs]),
            "orc_transpose": (C.c_int, [cs, cs]),
            "orc_gauss_rhs": (None, [C.c_int64, C.c_uint64, C.c_int32, C.c_void_p]),
            "orc_power_basis": (None, [cs, C.c_void_p, C.c_int32, C.c_void_p]),
            "orc_householder_r": (None, [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
            "orc_poly_coeffs_from_r": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
            "orc_gmres_poly": (C.c_int, [cs, C.c_uint64, C.c_int32, C.c_int32, C.c_void_p]),
            "orc_poly_fixed_sparsity": (C.c_int, [cs, C.c_void_p, C.c_int32, cs]),
            "orc_poly_fixed_sparsity_pattern": (C.c_int, [cs, cs, C.c_void_p, C.c_int32, cs]),
            "orc_power_pattern": (C.c_int, [cs, C.c_int32, cs]),
            "orc_onepoint_w": (C.c_int, [cs, C.c_void_p, C.c_int32, cs]),
            "orc_restrictor": (C.c_int, [cs, cs, C.c_double, cs]),
            "orc_coarse_operator": (C.c_int, [cs, C.c_void_p, cs, cs, C.c_double, cs]),
            "orc_level_build": (C.c_int, [cs, P(Params), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          cs, cs, cs, cs]),
            "orc_setup": (C.c_void_p, [cs, P(Params)]),
            "orc_setup_replay": (C.c_void_p, [cs, P(Params), C.c_int32, C.c_void_p]),
            "orc_level_renumeric": (C.c_int, [cs, C.c_void_p, P(Params), C.c_int32, C.c_void_p, cs, cs, cs,
                                              C.c_void_p, cs, cs, cs, cs]),
            "orc_resetup": (C.c_void_p, [C.c_void_p, C.c_void_p]),
            "orc_hier_free": (None, [C.c_void_p]),
            "orc_hier_levels": (C.c_int32, [C.c_void_p]),
            "orc_hier_matrix": (cs, [C.c_void_p, C.c_int32, C.c_int32]),
            "orc_hier_cf": (C.c_void_p, [C.c_void_p, C.c_int32]),
            "orc_hier_alpha": (C.c_void_p, [C.c_void_p, C.c_int32, P(C.c_int32)]),
            "orc_vcycle": (None, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
            "orc_richardson": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                         P(C.c_double)]),
            "orc_fgmres": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                                     P(C.c_double)]),
            "orc_hier_complexity": (None, [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's row-parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def default_params(**kw):
    p = Params()
    lib().orc_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# -------------------------------------------------------------- marshalling --
class _In:
    """Keeps numpy buffers alive while a _Csr view of them is in use."""

    def __init__(self, rowptr, col, val=None, ncols=None):
        self.rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.ci = np.ascontiguousarray(col, dtype=np.int32)
        self.v = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
        n = len(self.rp) - 1
        self.s = _Csr(n, n if ncols is None else ncols,
                      self.rp.ctypes.data_as(C.POINTER(C.c_int64)),
                      self.ci.ctypes.data_as(C.POINTER(C.c_int32)),
                      None if self.v is None else self.v.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def ref(self):
        return C.byref(self.s)


def _csr_in(A, ncols=None):
    if isinstance(A, _In):
        return A
    if len(A) == 4:
        return _In(A[0], A[1], A[2], A[3])
    return _In(A[0], A[1], A[2] if len(A) > 2 else None, ncols)


def _csr_out(s, free=True):
    nnz = s.rp[s.nr]
    rp = np.ctypeslib.as_array(s.rp, shape=(s.nr + 1,)).copy()
    ci = np.ctypeslib.as_array(s.ci, shape=(nnz,)).copy() if nnz else np.zeros(0, np.int32)
    v = None
    if s.v:
        v = np.ctypeslib.as_array(s.v, shape=(nnz,)).copy() if nnz else np.zeros(0)
    nc = s.nc
    if free:
        lib().orc_csr_free(C.byref(s))
    return (rp, ci, v, nc)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------- step API --
def splitmix64(x):
    return int(lib().orc_splitmix64(C.c_uint64(x)))


def counter(seed, stream, level, i):
    return int(lib().orc_counter(seed, stream, level, i))


def strength(A, alpha):
    a = _csr_in(A)
    out = np.zeros(len(a.ci), np.uint8)
    lib().orc_strength(a.ref, alpha, _ptr(out))
    return out


def sym_graph(A, strong):
    a = _csr_in(A)
    strong = np.ascontiguousarray(strong, np.uint8)
    g = _Csr()
    lib().orc_sym_graph(a.ref, _ptr(strong), C.byref(g))
    return _csr_out(g)


def pmisr_keys(G, seed, level):
    g = _csr_in(G)
    n = len(g.rp) - 1
    deg = np.zeros(n, np.int32)
    h = np.zeros(n, np.uint32)
    lib().orc_pmisr_keys(g.ref, seed, level, _ptr(deg), _ptr(h))
    return deg, h


def pmisr(G, deg, h, max_rounds):
    g = _csr_in(G)
    n = len(g.rp) - 1
    cf = np.zeros(n, np.int8)
    deg = np.ascontiguousarray(deg, np.int32)
    h = np.ascontiguousarray(h, np.uint32)
    rounds = lib().orc_pmisr(g.ref, _ptr(deg), _ptr(h), max_rounds, _ptr(cf))
    return cf, int(rounds)


def ddc(A, cf, alpha_diag):
    a = _csr_in(A)
    cf = np.array(cf, dtype=np.int8, copy=True)
    theta = np.zeros(len(cf))
    cnt = lib().orc_ddc(a.ref, alpha_diag, _ptr(cf), _ptr(theta))
    return cf, theta, int(cnt)


def ddc_fraction_threshold(A, cf, fraction):
    a = _csr_in(A)
    cf = np.ascontiguousarray(cf, np.int8)
    return float(lib().orc_ddc_fraction_threshold(a.ref, _ptr(cf), fraction))


def cf_split(A, params, level):
    a = _csr_in(A)
    cf = np.zeros(len(a.rp) - 1, np.int8)
    lib().orc_cf_split(a.ref, C.byref(params), level, _ptr(cf))
    return cf


def submatrix(A, cf, rowsel, colsel):
    a = _csr_in(A)
    cf = np.ascontiguousarray(cf, np.int8)
    o = _Csr()
    lib().orc_submatrix(a.ref, _ptr(cf), rowsel, colsel, C.byref(o))
    return _csr_out(o)


def spmv(A, x):
    a = _csr_in(A)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(len(a.rp) - 1)
    lib().orc_spmv(a.ref, _ptr(x), _ptr(y))
    return y


def spgemm(A, B):
    a, b = _csr_in(A), _csr_in(B)
    o = _Csr()
    lib().orc_spgemm(a.ref, b.ref, C.byref(o))
    return _csr_out(o)


def drop(A, tau, keep_diag):
    a = _csr_in(A)
    o = _Csr()
    lib().orc_drop(a.ref, tau, int(keep_diag), C.byref(o))
    return _csr_out(o)


def transpose(A):
    a = _csr_in(A)
    o = _Csr()
    lib().orc_transpose(a.ref, C.byref(o))
    return _csr_out(o)


def gauss_rhs(n, seed, level):
    b = np.zeros(n)
    lib().orc_gauss_rhs(n, seed, level, _ptr(b))
    return b


def power_basis(A, b, m):
    a = _csr_in(A)
    n = len(a.rp) - 1
    K = np.zeros((m + 1, n))          # row c = column c of K (column-major storage)
    b = np.ascontiguousarray(b, np.float64)
    lib().orc_power_basis(a.ref, _ptr(b), m, _ptr(K))
    return K.T


def householder_r(K):
    """R factor (cols x cols) and column norms of the column-scaled K."""
    rows, cols = K.shape
    Kc = np.ascontiguousarray(K.T)
    R = np.zeros((cols, cols))
    nrm = np.zeros(cols)
    lib().orc_householder_r(rows, cols, _ptr(Kc), _ptr(R), _ptr(nrm))
    return R, nrm


def poly_coeffs_from_r(R, colnorm):
    m = R.shape[0] - 1
    R = np.ascontiguousarray(R, np.float64)
    colnorm = np.ascontiguousarray(colnorm, np.float64)
    alpha = np.zeros(m)
    used = lib().orc_poly_coeffs_from_r(_ptr(R), _ptr(colnorm), m, _ptr(alpha))
    return alpha, int(used)


def gmres_poly(A, seed, level, m):
    a = _csr_in(A)
    alpha = np.zeros(m)
    used = lib().orc_gmres_poly(a.ref, seed, level, m, _ptr(alpha))
    return alpha, int(used)


def poly_fixed_sparsity(A, alpha):
    a = _csr_in(A)
    alpha = np.ascontiguousarray(alpha, np.float64)
    o = _Csr()
    lib().orc_poly_fixed_sparsity(a.ref, _ptr(alpha), len(alpha), C.byref(o))
    return _csr_out(o)


def poly_fixed_sparsity_pattern(A, S, alpha):
    """Fixed-sparsity polynomial with row patterns from S (plus diagonals)."""
    a, sp_ = _csr_in(A), _csr_in(S)
    alpha = np.ascontiguousarray(alpha, np.float64)
    o = _Csr()
    lib().orc_poly_fixed_sparsity_pattern(a.ref, sp_.ref, _ptr(alpha), len(alpha), C.byref(o))
    return _csr_out(o)


def power_pattern(A, order):
    a = _csr_in(A)
    o = _Csr()
    lib().orc_power_pattern(a.ref, order, C.byref(o))
    return _csr_out(o)


def onepoint_w(A, cf, weight_mode=0):
    a = _csr_in(A)
    cf = np.ascontiguousarray(cf, np.int8)
    o = _Csr()
    lib().orc_onepoint_w(a.ref, _ptr(cf), weight_mode, C.byref(o))
    return _csr_out(o)


def restrictor(Acf, Ainv, drop_R):
    a, b = _csr_in(Acf), _csr_in(Ainv)
    o = _Csr()
    lib().orc_restrictor(a.ref, b.ref, drop_R, C.byref(o))
    return _csr_out(o)


def coarse_operator(A, cf, Z, W, drop_A):
    a, z, w = _csr_in(A), _csr_in(Z), _csr_in(W)
    cf = np.ascontiguousarray(cf, np.int8)
    o = _Csr()
    lib().orc_coarse_operator(a.ref, _ptr(cf), z.ref, w.ref, drop_A, C.byref(o))
    return _csr_out(o)


def level_build(A, params, level, alpha_in=None):
    """One setup level for replay; returns dict(cf, alpha, Ainv, Z, W, Ac)."""
    a = _csr_in(A)
    n = len(a.rp) - 1
    m = params.poly_order + 1
    cf = np.zeros(n, np.int8)
    alpha = np.zeros(m)
    ain = None if alpha_in is None else np.ascontiguousarray(alpha_in, np.float64)
    outs = [_Csr() for _ in range(4)]
    lib().orc_level_build(a.ref, C.byref(params), level, None if ain is None else _ptr(ain), _ptr(cf),
                          _ptr(alpha), *[C.byref(o) for o in outs])
    Ainv, Z, W, Ac = [_csr_out(o) for o in outs]
    return {"cf": cf, "alpha": alpha, "Ainv": Ainv, "Z": Z, "W": W, "Ac": Ac}


def level_renumeric(A, cf, params, level, W, Z, Ac, alpha_in=None):
    """Numeric re-setup of one level on given patterns (W, Z, Ac: CSR tuples
    whose values are ignored); returns dict(alpha, Ainv, Z, W, Ac)."""
    a = _csr_in(A)
    cf = np.ascontiguousarray(cf, np.int8)
    w = _csr_in(W, W[3] if len(W) > 3 else None)
    z = _csr_in(Z, Z[3] if len(Z) > 3 else None)
    ac = _csr_in(Ac, Ac[3] if len(Ac) > 3 else None)
    m = params.poly_order + 1
    alpha = np.zeros(m)
    ain = None if alpha_in is None else np.ascontiguousarray(alpha_in, np.float64)
    outs = [_Csr() for _ in range(4)]
    lib().orc_level_renumeric(a.ref, _ptr(cf), C.byref(params), level, None if ain is None else _ptr(ain),
                              w.ref, z.ref, ac.ref, _ptr(alpha), *[C.byref(o) for o in outs])
    Ainv, Zo, Wo, Aco = [_csr_out(o) for o in outs]
    return {"alpha": alpha, "Ainv": Ainv, "Z": Zo, "W": Wo, "Ac": Aco}


class Hierarchy:
    """Oracle AIRG hierarchy (setup) with V-cycle, Richardson and FGMRES."""

    MATS = {"A": 0, "Ainv": 1, "Z": 2, "W": 3, "Aff": 4, "Afc": 5}

    ALPHA_STRIDE = 16

    def __init__(self, A, params, alphas=None):
        """alphas (optional): one coefficient vector per level, used instead of
        the coefficients computed from the random rhs (hierarchy replay)."""
        self._a = _csr_in(A)
        self.params = params
        self.n = len(self._a.rp) - 1
        if alphas is None:
            self.h = lib().orc_setup(self._a.ref, C.byref(params))
        else:
            tab = np.zeros((max(len(alphas), 1), self.ALPHA_STRIDE))
            for l, a in enumerate(alphas):
                a = np.asarray(a, np.float64)
                tab[l, :len(a)] = a
            self.h = lib().orc_setup_replay(self._a.ref, C.byref(params), len(alphas), _ptr(tab))
        if not self.h:
            raise ValueError("oracle setup rejected the matrix")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_hier_free(self.h)
            self.h = None

    def resetup(self, vals):
        """Numeric re-setup with new values on the canonical level-0 pattern:
        same CF splittings and patterns, recomputed values (a new Hierarchy)."""
        vals = np.ascontiguousarray(vals, np.float64)
        nnz = self.matrix(0, "A")[0][-1]
        if vals.shape != (nnz,):
            raise ValueError("values must match the canonical level-0 pattern")
        out = Hierarchy.__new__(Hierarchy)
        out._a = self._a
        out.params = self.params
        out.n = self.n
        out.h = lib().orc_resetup(self.h, _ptr(vals))
        return out

    @property
    def nlevels(self):
        return int(lib().orc_hier_levels(self.h))

    def matrix(self, level, which):
        p = lib().orc_hier_matrix(self.h, level, self.MATS[which])
        if not p:
            return None
        return _csr_out(p.contents, free=False)

    def cf(self, level):
        p = lib().orc_hier_cf(self.h, level)
        if not p:
            return None
        n = self.matrix(level, "A")[0].shape[0] - 1
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_int8)), shape=(n,)).copy()

    def alpha(self, level):
        na = C.c_int32(0)
        p = lib().orc_hier_alpha(self.h, level, C.byref(na))
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_double)), shape=(na.value,)).copy()

    def vcycle(self, g, level=0):
        g = np.ascontiguousarray(g, np.float64)
        e = np.zeros_like(g)
        lib().orc_vcycle(self.h, level, _ptr(g), _ptr(e))
        return e

    def richardson(self, b, rtol=1e-10, maxit=200):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros_like(b)
        rr = C.c_double(0)
        its = lib().orc_richardson(self.h, _ptr(b), _ptr(x), rtol, maxit, C.byref(rr))
        return x, int(its), rr.value

    def fgmres(self, b, rtol=1e-10, maxit=200, restart=30):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros_like(b)
        rr = C.c_double(0)
        its = lib().orc_fgmres(self.h, _ptr(b), _ptr(x), rtol, maxit, restart, C.byref(rr))
        return x, int(its), rr.value

    def complexity(self):
        g, o, s = C.c_double(), C.c_double(), C.c_double()
        lib().orc_hier_complexity(self.h, C.byref(g), C.byref(o), C.byref(s))
        return g.value, o.value, s.value
