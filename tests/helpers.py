"""Small shared helpers for the tests (dense conversion, tiny random matrices)."""
import numpy as np
import scipy.sparse as sp


def dense(A):
    rp, ci, v = A[0], A[1], A[2]
    nc = A[3] if len(A) > 3 else len(rp) - 1
    n = len(rp) - 1
    D = np.zeros((n, nc))
    rows = np.repeat(np.arange(n), np.diff(rp))
    D[rows, np.asarray(ci, dtype=np.int64)] = v
    return D


def pattern(A):
    rp, ci = A[0], A[1]
    nc = A[3] if len(A) > 3 else len(rp) - 1
    n = len(rp) - 1
    P = np.zeros((n, nc), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(rp))
    P[rows, np.asarray(ci, dtype=np.int64)] = True
    return P


def from_dense(D):
    S = sp.csr_matrix(D)
    S.sort_indices()
    return (S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64), D.shape[1])


def with_diag(D):
    """CSR of D keeping the diagonal even where it is zero."""
    n = D.shape[0]
    S = sp.csr_matrix(D + 0.0)
    S = S + sp.csr_matrix((np.full(n, 1e-300), (np.arange(n), np.arange(n))), shape=D.shape)
    S.sort_indices()
    S.data[S.indices == np.repeat(np.arange(n), np.diff(S.indptr))] -= 1e-300
    return (S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64), D.shape[1])


def random_nonsym(n, density, seed, dominance=2.0):
    """Random nonsymmetric sparse matrix with a dominant positive diagonal."""
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < density, -rng.random((n, n)), 0.0)
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, dominance * np.abs(D).sum(1) + 0.5 + rng.random(n))
    return D


def csr_of(P):
    return (P.rowptr, P.col, P.val)


_PROBLEMS = {}


def full_problem(name):
    """The full-size workloads, generated once per test session (the 3D mesh
    takes tens of seconds to build).  Callers must not modify the arrays."""
    if name not in _PROBLEMS:
        from workloads import dg_square, p0_cube, batch
        make = {"dg_square_512": lambda: dg_square(512), "p0_cube_128": lambda: p0_cube(128),
                "batch48": lambda: batch()}[name]
        _PROBLEMS[name] = make()
    return _PROBLEMS[name]
