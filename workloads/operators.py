"""Upwinded streaming-limit operators (advection plus a removal term).

Both discretisations solve  Omega . grad(u) + sigma u = s  with vacuum
(zero) inflow.  The paper's own operator is a stabilised CG Schur
complement (Discretisation section); the build substitutes these upwind
operators, which have the same hyperbolic, non-normal character and are
block lower triangular in a flow-ordered (sweep) numbering.

* P0 finite volume (any simplex mesh):
    a_KK = sum_{outflow faces f} (Omega.n_f)|f| + sigma_K |K|
    a_KJ = (Omega.n_f)|f| < 0  for the interior inflow face f shared with J
    b_K  = s_K |K|
* DG-P1 on triangles (nodal basis, 3 dofs per cell, cell-major numbering)
  from  sum_K [ -int_K u Omega.grad v + int_K sigma u v
               + int_{dK} (Omega.n) u_upwind v ]
  with exact P1 integrals: a 3x3 block per cell and a 2x2 block per interior
  inflow edge.  b = M s for nodal s.

CSR output: int32 row pointers and columns (sorted, unique), float64 values.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import triangle_edges, tet_faces

__all__ = ["p0_upwind", "dgp1_upwind", "to_csr", "dgp1_mass_blocks"]


def to_csr(rows, cols, vals, n):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def p0_upwind(faces, omega, sigma, src=None):
    """P0 upwind operator on a simplex mesh given its face connectivity.

    ``faces`` comes from ``triangle_edges`` (2D, key 'length'/'area') or
    ``tet_faces`` (3D, key 'area'/'vol').
    """
    if "length" in faces:
        meas = faces["length"]
        vol = faces["area"]
    else:
        meas = faces["area"]
        vol = faces["vol"]
    nbr = faces["nbr"]
    nt, nf = nbr.shape
    flux = np.einsum("tfd,d->tf", faces["nrm"], np.asarray(omega, dtype=np.float64)) * meas
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (nt,))
    diag = np.where(flux > 0, flux, 0.0).sum(axis=1) + sigma * vol
    t = np.repeat(np.arange(nt), nf).reshape(nt, nf)
    inflow = (flux < 0) & (nbr >= 0)
    rows = np.concatenate([np.arange(nt), t[inflow]])
    cols = np.concatenate([np.arange(nt), nbr[inflow]])
    vals = np.concatenate([diag, flux[inflow]])
    A = to_csr(rows, cols, vals, nt)
    b = None if src is None else np.asarray(src, dtype=np.float64) * vol
    return A, b, vol


def dgp1_mass_blocks(area):
    """Per-cell P1 mass blocks |K|/12 [[2,1,1],[1,2,1],[1,1,2]]  (nt,3,3)."""
    base = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    return area[:, None, None] * base[None]


def dgp1_upwind(xy, tri, omega, sigma, src=None, edges=None):
    """DG-P1 upwind operator on a counter-clockwise triangle mesh.

    dof of node a in triangle t is 3 t + a.  ``sigma`` is per cell, ``src``
    is nodal (nt,3) or flat (3 nt).  Returns ((rowptr, col, val), b, edges).
    """
    if edges is None:
        edges = triangle_edges(xy, tri)
    nt = tri.shape[0]
    omega = np.asarray(omega, dtype=np.float64)
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (nt,))
    area = edges["area"]
    p = xy[tri]                                            # nt,3,2
    # grad phi_a = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / (2|K|)
    p1 = p[:, [1, 2, 0], :]
    p2 = p[:, [2, 0, 1], :]
    grad = np.stack([p1[..., 1] - p2[..., 1], p2[..., 0] - p1[..., 0]], axis=-1) / (2.0 * area[:, None, None])
    og = grad @ omega                                      # nt,3  Omega . grad phi_a
    M = dgp1_mass_blocks(area)
    # cell block: test a (row), trial b (col)
    blk = -og[:, :, None] * (area[:, None, None] / 3.0) + sigma[:, None, None] * M
    flux = np.einsum("tkd,d->tk", edges["nrm"], omega) * edges["length"]   # (Omega.n)|f|
    fm = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    loc = np.array([[0, 1], [1, 2], [2, 0]])               # local nodes of edge k
    # cell blocks: entry (a, b) of cell t sits at row 3t+a, column 3t+b
    cell_r = np.repeat(3 * np.arange(nt)[:, None] + np.arange(3)[None], 3, axis=1)
    cell_c = np.tile(3 * np.arange(nt)[:, None] + np.arange(3)[None], (1, 3))
    rows = [cell_r.ravel()]
    cols = [cell_c.ravel()]
    vals_cell = blk.copy()
    nbr = edges["nbr"]
    for k in range(3):
        la, lb = loc[k]
        out = flux[:, k] > 0
        # outflow edge: own trace, (Omega.n)|f| times the edge mass on its two nodes
        for ia, a in enumerate((la, lb)):
            for ib, b_ in enumerate((la, lb)):
                vals_cell[out, a, b_] += flux[out, k] * fm[ia, ib]
    vals = [vals_cell.ravel()]
    # inflow edges: couple to the neighbour's trace at the same vertices
    for k in range(3):
        la, lb = loc[k]
        inn = (flux[:, k] < 0) & (nbr[:, k] >= 0)
        t = np.nonzero(inn)[0]
        if t.size == 0:
            continue
        J = nbr[t, k]
        va = tri[t, la]
        vb = tri[t, lb]
        tj = tri[J]                                        # neighbour vertices
        ja = np.argmax(tj == va[:, None], axis=1)
        jb = np.argmax(tj == vb[:, None], axis=1)
        assert np.all(tj[np.arange(t.size), ja] == va) and np.all(tj[np.arange(t.size), jb] == vb)
        f = flux[t, k]
        for ia, a in enumerate((la, lb)):
            for ib, jloc in enumerate((ja, jb)):
                rows.append(3 * t + a)
                cols.append(3 * J + jloc)
                vals.append(f * fm[ia, ib])
    A = to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), 3 * nt)
    b = None
    if src is not None:
        s = np.asarray(src, dtype=np.float64).reshape(nt, 3)
        b = np.einsum("tab,tb->ta", M, s).ravel()
    return A, b, edges
