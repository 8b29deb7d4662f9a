"""The five seeded synthetic workloads, plus reduced-size variants for tests.

Every workload is a square CSR matrix (int32 row pointers and columns,
float64 values) with one or more right-hand sides.  All seeds are fixed
integers below; sizes follow from closed forms:

  p0_square   P0 upwind, unit square N x N squares -> 2 N^2 cells, seeded
              diagonal per square, theta = 0.3 rad, sigma = 1e-3, s ~ U(0,1).
              N = 64: n = 8,192, nnz = 20,352.
  dg_square   DG-P1 upwind, jittered (U(-0.2h, 0.2h)) N x N triangulation,
              3 dofs per cell, theta = 1.1 rad, sigma in {1e-4, 1} on a
              seeded 16 x 16 block checkerboard, nodal s ~ U(0,1).
              N = 512: n = 1,572,864, nnz = 7,860,224.
  p0_cube     P0 upwind, N^3 cubes x 6 Kuhn tetrahedra, Omega =
              (0.5, 0.3, 0.81)/|.|, sigma = 1e-4, s ~ U(0,1).
              N = 128: n = 12,582,912, nnz = 37,650,432.
  batch       48 DG-P1 problems, side N_p ~ U{64..384}, theta_p ~ U(0, 2 pi),
              sigma = 1e-3, 4 right-hand sides of nodal s ~ U(0,1) each.
  adjoint     DG-P1 on 256 x 256 squares, sigma_K = exp(N(log 1e-2, 1)),
              theta = 1.1, nodal s ~ U(0,1), a seeded 32 x 32-square
              detector patch; loss = sum of u^2 over the patch dofs.

The paper measures on the authors' unstructured SGS problem (a 3x3 box with
a central source, Results section), which is not available; these seeded
inputs stand in for it.
"""
from dataclasses import dataclass, field
import numpy as np

from .mesh import square_triangles, triangle_edges, kuhn_tets, tet_faces
from .operators import p0_upwind, dgp1_upwind, dgp1_mass_blocks

SEEDS = {
    "p0_square": {"mesh": 11, "src": 12, "airg": 13},
    "dg_square": {"mesh": 21, "sigma": 22, "src": 23, "airg": 24},
    "p0_cube": {"src": 32, "airg": 33},
    "batch": {"sizes": 41, "mesh": 42, "theta": 43, "src": 44, "airg": 45},
    "adjoint": {"mesh": 51, "sigma": 52, "src": 53, "patch": 54, "airg": 55},
}


@dataclass
class Problem:
    name: str
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray                      # (n,) or (n, nrhs)
    seed: int                          # AIRG seed (PMISR keys, random rhs)
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self):
        return int(self.rowptr[-1])


def p0_square(N=64, theta=0.3, sigma=1e-3):
    s = SEEDS["p0_square"]
    xy, tri = square_triangles(N, np.random.default_rng(s["mesh"]))
    faces = triangle_edges(xy, tri)
    src = np.random.default_rng(s["src"]).uniform(0.0, 1.0, tri.shape[0])
    (rp, ci, v), b, vol = p0_upwind(faces, (np.cos(theta), np.sin(theta)), sigma, src)
    return Problem("p0_square_%d" % N, tri.shape[0], rp, ci, v, b, s["airg"],
                   {"dofs_per_cell": 1, "cells": tri.shape[0]})


def _checker_sigma(xy, tri, rng, blocks=16, lo=1e-4, hi=1.0):
    pick = rng.integers(0, 2, size=(blocks, blocks))
    cen = xy[tri].mean(axis=1)
    bi = np.minimum((cen[:, 0] * blocks).astype(np.int64), blocks - 1)
    bj = np.minimum((cen[:, 1] * blocks).astype(np.int64), blocks - 1)
    return np.where(pick[bj, bi] == 1, hi, lo)


def dg_square(N=512, theta=1.1):
    s = SEEDS["dg_square"]
    rng = np.random.default_rng(s["mesh"])
    xy, tri = square_triangles(N, rng, jitter=0.2)
    sigma = _checker_sigma(xy, tri, np.random.default_rng(s["sigma"]))
    src = np.random.default_rng(s["src"]).uniform(0.0, 1.0, 3 * tri.shape[0])
    (rp, ci, v), b, edges = dgp1_upwind(xy, tri, (np.cos(theta), np.sin(theta)), sigma, src)
    return Problem("dg_square_%d" % N, 3 * tri.shape[0], rp, ci, v, b, s["airg"],
                   {"dofs_per_cell": 3, "cells": tri.shape[0]})


def p0_cube(N=128, sigma=1e-4):
    s = SEEDS["p0_cube"]
    xyz, tet = kuhn_tets(N)
    faces = tet_faces(xyz, tet)
    om = np.array([0.5, 0.3, 0.81])
    om = om / np.linalg.norm(om)
    src = np.random.default_rng(s["src"]).uniform(0.0, 1.0, tet.shape[0])
    (rp, ci, v), b, vol = p0_upwind(faces, om, sigma, src)
    return Problem("p0_cube_%d" % N, tet.shape[0], rp, ci, v, b, s["airg"],
                   {"dofs_per_cell": 1, "cells": tet.shape[0]})


def batch(count=48, lo=64, hi=384, nrhs=4, sigma=1e-3):
    """Independent DG-P1 problems with uneven sizes and directions."""
    s = SEEDS["batch"]
    sizes = np.random.default_rng(s["sizes"]).integers(lo, hi + 1, size=count)
    thetas = np.random.default_rng(s["theta"]).uniform(0.0, 2.0 * np.pi, size=count)
    out = []
    for p in range(count):
        N = int(sizes[p])
        xy, tri = square_triangles(N, np.random.default_rng([s["mesh"], p]), jitter=0.2)
        th = float(thetas[p])
        src = np.random.default_rng([s["src"], p]).uniform(0.0, 1.0, (nrhs, 3 * tri.shape[0]))
        (rp, ci, v), _, edges = dgp1_upwind(xy, tri, (np.cos(th), np.sin(th)), sigma)
        M = dgp1_mass_blocks(edges["area"])
        b = np.stack([np.einsum("tab,tb->ta", M, src[r].reshape(-1, 3)).ravel() for r in range(nrhs)], axis=1)
        out.append(Problem("batch_%d_N%d" % (p, N), 3 * tri.shape[0], rp, ci, v, b, s["airg"] + 1000 * p,
                           {"dofs_per_cell": 3, "cells": tri.shape[0], "theta": th}))
    return out


def adjoint(N=256, theta=1.1, patch=32):
    """DG-P1 problem with per-cell removal coefficients and a detector patch.

    meta holds what the gradient needs: the advection part A_adv (sigma=0),
    per-cell mass blocks, the nodal source and the patch dof mask.
    """
    s = SEEDS["adjoint"]
    xy, tri = square_triangles(N, np.random.default_rng(s["mesh"]), jitter=0.2)
    nt = tri.shape[0]
    sigma = np.exp(np.random.default_rng(s["sigma"]).normal(np.log(1e-2), 1.0, nt))
    src = np.random.default_rng(s["src"]).uniform(0.0, 1.0, 3 * nt)
    om = (np.cos(theta), np.sin(theta))
    (rp, ci, v), b, edges = dgp1_upwind(xy, tri, om, sigma, src)
    (rpa, cia, va), _, _ = dgp1_upwind(xy, tri, om, 0.0, None, edges=edges)
    assert np.array_equal(rp, rpa) and np.array_equal(ci, cia)
    # patch: squares [i0, i0+patch) x [j0, j0+patch); square of a cell from its centroid
    patch = min(patch, max(1, N // 2))          # reduced-size variants keep a proportionate patch
    p0 = np.random.default_rng(s["patch"]).integers(0, N - patch + 1, size=2)
    cen = xy[tri].mean(axis=1)
    sq = np.floor(cen * N).astype(np.int64)
    inpatch = (sq[:, 0] >= p0[0]) & (sq[:, 0] < p0[0] + patch) & (sq[:, 1] >= p0[1]) & (sq[:, 1] < p0[1] + patch)
    mask = np.repeat(inpatch, 3)
    M = dgp1_mass_blocks(edges["area"])
    return Problem("adjoint_%d" % N, 3 * nt, rp, ci, v, b, s["airg"],
                   {"dofs_per_cell": 3, "cells": nt, "sigma": sigma, "src": src, "val_adv": va,
                    "mass": M, "patch_mask": mask, "patch_origin": p0, "theta": theta})


def concat(problems):
    """Block-diagonal concatenation of independent problems.

    Returns (rowptr, col, val, b, offsets, seeds): one CSR with the problems'
    rows stacked in order, b stacked the same way ((n,) or (n, k)), segment row
    offsets (len(problems) + 1) and the per-problem AIRG seeds.
    """
    offs = np.zeros(len(problems) + 1, dtype=np.int64)
    for i, P in enumerate(problems):
        offs[i + 1] = offs[i] + P.n
    nz = np.zeros(len(problems) + 1, dtype=np.int64)
    for i, P in enumerate(problems):
        nz[i + 1] = nz[i] + P.nnz
    rp = np.concatenate([[0]] + [P.rowptr[1:].astype(np.int64) + nz[i] for i, P in enumerate(problems)])
    ci = np.concatenate([P.col.astype(np.int64) + offs[i] for i, P in enumerate(problems)])
    val = np.concatenate([P.val for P in problems])
    b = np.concatenate([P.b for P in problems], axis=0)
    if rp[-1] >= 2 ** 31 or offs[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 indices")
    return (rp.astype(np.int32), ci.astype(np.int32), val, b, offs,
            np.array([P.seed for P in problems], dtype=np.uint64))


def by_name(name, **kw):
    return {"p0_square": p0_square, "dg_square": dg_square, "p0_cube": p0_cube,
            "batch": batch, "adjoint": adjoint}[name](**kw)
