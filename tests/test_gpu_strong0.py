"""Strong tolerance 0.0 (the strong-tolerances subsection): the symmetrised
strong graph is the matrix's adjacency graph, PMISR gives an independent set
in it, A_ff is diagonal on every level and DDC has nothing to convert; on the
top grid the splitting does not depend on the direction.  Device against the
oracle: the splitting and the hierarchy replay bit for bit, and the solves
reach 1e-10 with one up F-point smooth (the paper's setting for this
tolerance)."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import dg_square, p0_square

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")

TOL0 = dict(strong_threshold=0.0, up_smooths=1, max_levels=128)


def setup(P, **kw):
    A = airg.to_device(P.rowptr, P.col, P.val)
    opts = airg.default_opts(seed=P.seed, **{**TOL0, **kw})
    return airg.airg_setup(*A, opts), opts


@pytest.mark.parametrize("make", [lambda: dg_square(48), lambda: p0_square(48)], ids=["dg48", "p0_48"])
def test_tol0_diagonal_ff_blocks_and_replay(make):
    P = make()
    h, opts = setup(P)
    prm = O.default_params(seed=P.seed, strong_threshold=0.0, up_smooths=1, max_levels=128)
    st = airg.airg_get_stats(h)
    assert st["levels"] > 10
    for l in range(st["levels"]):
        info = airg.airg_get_level(h, l)
        if info["coarsest"]:
            break
        assert info["nnz_aff"] == info["n_f"], l                       # A_ff diagonal
        A_l = airg.airg_get_level_matrix(h, l, "A")
        want = O.level_build(A_l, prm, l, alpha_in=info["alpha"])
        assert np.array_equal(info["cf"], want["cf"]), l
        for key in ("Ainv", "Z", "W"):
            got = airg.airg_get_level_matrix(h, l, key)
            assert all(np.array_equal(x, y) for x, y in zip(got[:3], want[key][:3])), (l, key)
        nxt = airg.airg_get_level_matrix(h, l + 1, "A")
        assert all(np.array_equal(x, y) for x, y in zip(nxt[:3], want["Ac"][:3])), l


def test_tol0_top_split_is_independent_of_direction():
    splits = []
    for theta in (0.3, 1.1, 2.0, 4.0):
        P = dg_square(40, theta=theta)
        h, _ = setup(P)
        cf = airg.airg_get_level(h, 0)["cf"]
        prm = O.default_params(seed=P.seed, strong_threshold=0.0)
        assert np.array_equal(cf, O.cf_split((P.rowptr, P.col, P.val), prm, 0))
        splits.append(cf)
    assert all(np.array_equal(splits[0], c) for c in splits[1:])


@pytest.mark.parametrize("outer,prec", [(0, 64), (1, 32)], ids=["richardson64", "fgmres32"])
def test_tol0_solves(outer, prec):
    P = dg_square(96)
    h, _ = setup(P, outer=outer, precond_precision=prec)
    x, info = airg.airg_solve(h, torch.as_tensor(P.b, device="cuda"), rtol=1e-10, max_it=300)
    assert info["converged"]
    r = P.b - O.spmv((P.rowptr, P.col, P.val), x.cpu().numpy())
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(P.b)
