"""Parity at the full workload sizes, in the configuration the benchmark
times, on what the oracle can check at that size:

* the level-0 CF splitting (bit-exact against the oracle's splitting of the
  whole operator),
* one replayed setup level (the oracle rebuilds level 1 from the device's
  level-0 operator and coefficients; bit-exact),
* the FP64 relative residual of the returned solution, recomputed by the
  oracle's SpMV, <= 1e-10 for every right-hand side.
"""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import concat
from tests.helpers import full_problem

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")


def check_split_and_first_level(h, P, opts_kw):
    prm = O.default_params(seed=P.seed, **opts_kw)
    A = (P.rowptr, P.col, P.val)
    lv = airg.airg_get_level(h, 0)
    assert np.array_equal(lv["cf"], O.cf_split(A, prm, 0))
    if lv["coarsest"]:
        return
    want = O.level_build(A, prm, 0, alpha_in=lv["alpha"])
    for key in ("Ainv", "Z", "W"):
        got = airg.airg_get_level_matrix(h, 0, key)
        assert all(np.array_equal(got[i], want[key][i]) for i in range(3)), key
    nxt = airg.airg_get_level_matrix(h, 1, "A")
    assert np.array_equal(nxt[0], want["Ac"][0]) and np.array_equal(nxt[1], want["Ac"][1])
    assert np.array_equal(nxt[2], want["Ac"][2])


def residual_ok(P, x, b):
    r = b - O.spmv((P.rowptr, P.col, P.val), x)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.timeout(300)
def test_dg_square_512_fp32_fgmres():
    P = full_problem("dg_square_512")
    A = airg.to_device(P.rowptr, P.col, P.val)
    kw = {"truncate_n": 98304, "coarse_iters": 6}      # as the benchmark times it
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed, outer=airg.OUTER_FGMRES, precond_precision=32, **kw))
    x, info = airg.airg_solve(h, torch.as_tensor(P.b, device="cuda"), rtol=1e-10, max_it=100)
    assert info["converged"]
    assert residual_ok(P, x.cpu().numpy(), P.b) <= 1.0001e-10
    check_split_and_first_level(h, P, kw)
    # and untruncated
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed, outer=airg.OUTER_FGMRES, precond_precision=32))
    x, info = airg.airg_solve(h, torch.as_tensor(P.b, device="cuda"), rtol=1e-10, max_it=100)
    assert info["converged"]
    assert residual_ok(P, x.cpu().numpy(), P.b) <= 1.0001e-10


@pytest.mark.timeout(400)
def test_p0_cube_128_truncated_fp32_fgmres():
    P = full_problem("p0_cube_128")
    A = airg.to_device(P.rowptr, P.col, P.val)
    kw = {"truncate_n": 65536}
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed, outer=airg.OUTER_FGMRES, precond_precision=32, **kw))
    st = airg.airg_get_stats(h)
    last = airg.airg_get_level(h, st["levels"] - 1, with_cf=False)
    assert last["coarsest"] and last["n"] <= 65536
    x, info = airg.airg_solve(h, torch.as_tensor(P.b, device="cuda"), rtol=1e-10, max_it=100)
    assert info["converged"]
    assert residual_ok(P, x.cpu().numpy(), P.b) <= 1.0001e-10
    check_split_and_first_level(h, P, kw)


@pytest.mark.timeout(300)
def test_batch_48_problems_4_rhs():
    probs = full_problem("batch48")
    rp, ci, val, b, offs, seeds = concat(probs)
    A = airg.to_device(rp, ci, val)
    opts = airg.default_opts(outer=airg.OUTER_FGMRES, precond_precision=32, use_graph=1, autotune=1)
    h = airg.airg_setup(*A, opts, seg_offsets=offs, seg_seeds=seeds)
    X, info = airg.airg_solve(h, torch.as_tensor(b, device="cuda"), rtol=1e-10, max_it=100)
    assert info["converged"]
    X = X.cpu().numpy()
    rng = np.random.default_rng(0)
    for p in rng.choice(len(probs), 6, replace=False):      # sampled segments, every rhs
        P = probs[p]
        for c in range(b.shape[1]):
            assert residual_ok(P, X[offs[p]:offs[p + 1], c], P.b[:, c]) <= 1.0001e-10
        lv = airg.airg_get_level(h, 0, segment=int(p))
        assert np.array_equal(lv["cf"], O.cf_split((P.rowptr, P.col, P.val), O.default_params(seed=P.seed), 0))
