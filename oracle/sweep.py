"""Exact solve of an upwind streaming operator by a topological-order sweep.

Test infrastructure, not part of the product: only the tests, the smoke
check and the benchmark's CPU-baseline leg use anything under ``oracle/``.

The streaming operator couples a cell only to its upwind neighbours, so in a
flow-consistent (topological) order of the cells the matrix is block lower
triangular and one block forward substitution inverts it exactly -- the
classical sweep that source iteration relies on (Introduction).  Upwinded
straight-edged triangulations with a constant direction, and the Kuhn
(regular) tetrahedral split, have acyclic cell dependency graphs; the sweep
checks acyclicity with Kahn's algorithm and otherwise falls back to a sparse
direct solve.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _cell_graph(rowptr, col, bs, ncell):
    n = ncell * bs
    rows = np.repeat(np.arange(n), np.diff(rowptr)) // bs
    cols = np.asarray(col) // bs
    keep = rows != cols
    G = sp.csr_matrix((np.ones(int(keep.sum()), dtype=np.int8), (rows[keep], cols[keep])), shape=(ncell, ncell))
    G.sum_duplicates()
    return G          # row K lists the upwind cells K depends on


def sweep_levels(rowptr, col, bs=1):
    """Kahn level sets of the cell dependency graph, or None if it has a cycle."""
    n = len(rowptr) - 1
    ncell = n // bs
    G = _cell_graph(rowptr, col, bs, ncell)
    indeg = np.diff(G.indptr).astype(np.int64)
    down = G.T.tocsr()           # row J lists the downwind cells of J
    levels = []
    frontier = np.nonzero(indeg == 0)[0]
    done = 0
    while frontier.size:
        levels.append(frontier)
        done += frontier.size
        starts = down.indptr[frontier]
        ends = down.indptr[frontier + 1]
        cnt = ends - starts
        if cnt.sum() == 0:
            break
        idx = np.repeat(starts - np.cumsum(np.concatenate([[0], cnt[:-1]])), cnt) + np.arange(cnt.sum())
        nb = down.indices[idx]
        np.subtract.at(indeg, nb, 1)
        cand = np.unique(nb)
        frontier = cand[indeg[cand] == 0]
    if done != ncell:
        return None
    return levels


def sweep_solve(rowptr, col, val, b, bs=1, transpose=False):
    """x = A^{-1} b (or A^{-T} b) by block forward substitution in sweep order.

    ``bs`` is the number of dofs per cell (1 for P0, 3 for DG-P1).  b may be
    (n,) or (n, k).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    A = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col, dtype=np.int64), rowptr), shape=(n, n))
    if transpose:
        A = A.T.tocsr()
        A.sort_indices()
    levels = sweep_levels(A.indptr, A.indices, bs)
    b = np.asarray(b, dtype=np.float64)
    if levels is None:
        return spla.splu(A.tocsc()).solve(b)
    vec = b.ndim == 1
    B = b.reshape(n, -1)
    X = np.zeros_like(B)
    ncell = n // bs
    # diagonal blocks
    D = np.zeros((ncell, bs, bs))
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    same = (rows // bs) == (A.indices // bs)
    D[rows[same] // bs, rows[same] % bs, A.indices[same] % bs] = A.data[same]
    Aoff = sp.csr_matrix((np.where(same, 0.0, A.data), A.indices, A.indptr), shape=(n, n))
    Aoff.eliminate_zeros()
    for lev in levels:
        dofs = (lev[:, None] * bs + np.arange(bs)[None]).ravel()
        rhs = B[dofs] - Aoff[dofs] @ X
        rhs = rhs.reshape(lev.size, bs, -1)
        X[dofs] = np.linalg.solve(D[lev], rhs).reshape(-1, B.shape[1])
    return X[:, 0] if vec else X
