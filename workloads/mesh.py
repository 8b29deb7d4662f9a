"""Seeded synthetic meshes for the streaming-limit test operators.

Three families are generated:

* ``square_triangles``: the unit square cut into N x N squares, each split
  into two counter-clockwise triangles along a diagonal picked per square by
  a seeded Bernoulli(1/2) draw; optionally every interior node is jittered by
  U(-j h, j h) in x and y (boundary nodes stay fixed).
* ``kuhn_tets``: the unit cube cut into N^3 cubes, each split into the six
  Kuhn (Freudenthal) tetrahedra x_{p1} >= x_{p2} >= x_{p3} over the
  permutations p; the split is conforming across cubes.
* ``faces``: interior/boundary face connectivity with outward unit normals
  and measures, shared by both operators in ``operators.py``.

The paper's own meshes (unstructured triangles of a 3x3 box, Results section)
are not available; these seeded meshes stand in for them.
Nothing here performs any of the multigrid method's arithmetic.
"""
import numpy as np

__all__ = ["square_triangles", "kuhn_tets", "triangle_edges", "tet_faces"]


def square_triangles(N, rng=None, jitter=0.0):
    """Triangulated unit square.

    Returns (xy[nv,2] float64, tri[nt,3] int64) with counter-clockwise
    triangles, nt = 2 N^2.  ``rng`` draws the per-square diagonal (and the
    jitter when ``jitter`` > 0, as a fraction of h = 1/N).
    """
    h = 1.0 / N
    nv1 = N + 1
    ix, iy = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="xy")
    xy = np.stack([ix.ravel() * h, iy.ravel() * h], axis=1).astype(np.float64)
    if rng is None:
        diag = np.zeros(N * N, dtype=np.int8)
    else:
        diag = rng.integers(0, 2, size=N * N).astype(np.int8)
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs an rng")
        interior = (ix.ravel() > 0) & (ix.ravel() < N) & (iy.ravel() > 0) & (iy.ravel() < N)
        d = rng.uniform(-jitter * h, jitter * h, size=(xy.shape[0], 2))
        xy = xy + d * interior[:, None]
    si, sj = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    si = si.ravel()
    sj = sj.ravel()
    a = sj * nv1 + si          # (i, j)
    b = a + 1                  # (i+1, j)
    c = a + nv1 + 1            # (i+1, j+1)
    d = a + nv1                # (i, j+1)
    t0 = np.where(diag[:, None] == 0, np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t1 = np.where(diag[:, None] == 0, np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tri = np.empty((2 * N * N, 3), dtype=np.int64)
    tri[0::2] = t0
    tri[1::2] = t1
    p = xy[tri]
    area2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
            (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    if not np.all(area2 > 0):
        raise RuntimeError("triangulation lost positive orientation (jitter too large)")
    return xy, tri


def triangle_edges(xy, tri):
    """Edge connectivity of a triangle mesh.

    Local edge k of triangle t joins tri[t,k] -> tri[t,(k+1)%3].  Returns a
    dict with
      nbr[nt,3]   neighbour triangle across edge k (-1 on the boundary),
      nrm[nt,3,2] outward unit normal of edge k,
      length[nt,3],
      area[nt].
    """
    nt = tri.shape[0]
    nv = xy.shape[0]
    p = xy[tri]                                   # nt,3,2
    q = p[:, [1, 2, 0], :]                        # edge end points
    e = q - p
    length = np.sqrt(e[..., 0] ** 2 + e[..., 1] ** 2)
    # counter-clockwise triangle: outward normal of edge p->q is (dy, -dx)
    nrm = np.stack([e[..., 1], -e[..., 0]], axis=-1) / length[..., None]
    area = 0.5 * (e[:, 0, 0] * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * e[:, 0, 1])
    va = tri
    vb = tri[:, [1, 2, 0]]
    key = np.minimum(va, vb) * nv + np.maximum(va, vb)
    key = key.ravel()
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    nbr = -np.ones(nt * 3, dtype=np.int64)
    i0 = order[:-1][same]
    i1 = order[1:][same]
    nbr[i0] = i1 // 3
    nbr[i1] = i0 // 3
    return {"nbr": nbr.reshape(nt, 3), "nrm": nrm, "length": length, "area": area}


_PERMS = np.array([[0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]])


def kuhn_tets(N):
    """Kuhn split of the unit cube into 6 N^3 tetrahedra.

    Returns (xyz[nv,3], tet[nt,4]); tet ordering is cube-major (cube index
    i + N j + N^2 k, then the six permutations in lexicographic order).
    """
    h = 1.0 / N
    nv1 = N + 1
    g = np.arange(nv1)
    vk, vj, vi = np.meshgrid(g, g, g, indexing="ij")       # raveled order = vertex id
    xyz = np.stack([vi.ravel(), vj.ravel(), vk.ravel()], axis=1) * h
    vid = lambda i, j, k: i + nv1 * j + nv1 * nv1 * k
    c = np.arange(N)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")       # raveled order = cube index
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    tet = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(_PERMS):
        cur = base.copy()
        tet[:, t, 0] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
        for s in range(3):
            cur[:, perm[s]] += 1
            tet[:, t, s + 1] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
    return xyz, tet.reshape(-1, 4)


def tet_faces(xyz, tet):
    """Face connectivity of a tetrahedral mesh.

    Face k of tetrahedron t is the one opposite vertex k.  Returns a dict with
      nbr[nt,4]   neighbour across face k (-1 on the boundary),
      nrm[nt,4,3] outward unit normal, area[nt,4], vol[nt].

    The normals are formed one face slot and one component at a time (the
    same products and differences as a vector cross product, in the same
    order), which keeps the temporaries at a few nt-long columns.
    """
    nt = tet.shape[0]
    nv = xyz.shape[0]
    X = [np.ascontiguousarray(xyz[:, d]) for d in range(3)]
    FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
    nrm = np.empty((nt, 4, 3))
    area = np.empty((nt, 4))
    for k, (a, b, c) in enumerate(FACES):
        ia, ib, ic, io = tet[:, a], tet[:, b], tet[:, c], tet[:, k]
        pa = [X[d][ia] for d in range(3)]
        u = [X[d][ib] - pa[d] for d in range(3)]
        v = [X[d][ic] - pa[d] for d in range(3)]
        n = [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]
        del u, v
        nlen = np.sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2])
        area[:, k] = 0.5 * nlen
        n = [n[d] / nlen for d in range(3)]
        s = n[0] * (pa[0] - X[0][io]) + n[1] * (pa[1] - X[1][io]) + n[2] * (pa[2] - X[2][io])
        sg = np.sign(s)
        for d in range(3):
            nrm[:, k, d] = n[d] * sg
        del n, pa, s, sg
    p0 = [X[d][tet[:, 0]] for d in range(3)]
    u = [X[d][tet[:, 1]] - p0[d] for d in range(3)]
    v = [X[d][tet[:, 2]] - p0[d] for d in range(3)]
    w = [X[d][tet[:, 3]] - p0[d] for d in range(3)]
    c = [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]
    vol = np.abs(c[0] * w[0] + c[1] * w[1] + c[2] * w[2]) / 6.0
    del p0, u, v, w, c
    # face key: sorted vertex ids, encoded relative to the smallest id
    fv = np.stack([tet[:, list(f)] for f in FACES], axis=1)
    fs = np.sort(fv.reshape(-1, 3), axis=1)
    del fv
    d1 = fs[:, 1] - fs[:, 0]
    d2 = fs[:, 2] - fs[:, 0]
    S = int(max(d1.max(), d2.max())) + 1
    if nv * S * S >= 2 ** 62:
        raise RuntimeError("face key overflow")
    key = fs[:, 0] * (S * S) + d1 * S + d2
    del fs, d1, d2
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    nbr = -np.ones(nt * 4, dtype=np.int64)
    i0 = order[:-1][same]
    i1 = order[1:][same]
    nbr[i0] = i1 // 4
    nbr[i1] = i0 // 4
    return {"nbr": nbr.reshape(nt, 4), "nrm": nrm, "area": area, "vol": vol}
