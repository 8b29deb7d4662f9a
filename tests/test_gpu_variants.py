"""Polynomial variants and the V-cycle against the oracle, through the C ABI:

* sparsity orders 2 and 3 (the powers keep the pattern of A_ff^s): every
  device level replays bit for bit (Ainv on the power pattern, Z, W, A_c);
* the matrix-free coarse polynomial: one truncated level gives
  e = q(A) g + two corrections exactly (dense check with the device's
  coefficients); deeper hierarchies match the oracle's V-cycle and solves;
* the V-cycle entry point (FP64 and FP32) against the oracle's V-cycle on
  hierarchies whose structure coincides level by level;
* numeric re-setup keeps the power patterns.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests.helpers import dense
from workloads import p0_square, dg_square, p0_cube

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")


def setup(P, **kw):
    A = airg.to_device(P.rowptr, P.col, P.val)
    opts = airg.default_opts(seed=P.seed, **kw)
    return airg.airg_setup(*A, opts), opts


def replay(h, P, prm):
    st = airg.airg_get_stats(h)
    for l in range(st["levels"]):
        info = airg.airg_get_level(h, l)
        if info["coarsest"]:
            break
        A_l = airg.airg_get_level_matrix(h, l, "A")
        want = O.level_build(A_l, prm, l, alpha_in=info["alpha"])
        assert np.array_equal(info["cf"], want["cf"]), l
        for key in ("Ainv", "Z", "W"):
            got = airg.airg_get_level_matrix(h, l, key)
            assert all(np.array_equal(x, y) for x, y in zip(got[:3], want[key][:3])), (l, key)
        nxt = airg.airg_get_level_matrix(h, l + 1, "A")
        assert all(np.array_equal(x, y) for x, y in zip(nxt[:3], want["Ac"][:3])), l
    return st


@pytest.mark.parametrize("make,order", [(lambda: dg_square(40), 2), (lambda: p0_square(48), 3),
                                        (lambda: p0_cube(8), 2)], ids=["dg40_s2", "p0_48_s3", "cube8_s2"])
def test_sparsity_order_replay_and_power_patterns(make, order):
    P = make()
    h, _ = setup(P, poly_sparsity_order=order)
    prm = O.default_params(seed=P.seed, poly_sparsity_order=order)
    st = replay(h, P, prm)
    assert st["levels"] > 2
    Aff = airg.airg_get_level_matrix(h, 0, "Aff")
    S = O.power_pattern(Aff, order)
    Ainv = airg.airg_get_level_matrix(h, 0, "Ainv")
    assert np.array_equal(Ainv[0], S[0]) and np.array_equal(Ainv[1], S[1])


def test_matrix_free_coarse_on_one_level():
    P = p0_square(10)
    h, opts = setup(P, truncate_n=10 ** 6, coarse_matrix_free=1)
    info = airg.airg_get_level(h, 0)
    assert info["coarsest"] and info["nnz_ainv"] == 0
    D = dense((P.rowptr, P.col, P.val))
    Q = sum(a * np.linalg.matrix_power(D, k) for k, a in enumerate(info["alpha"]))
    g = np.random.default_rng(1).standard_normal(P.n)
    e = Q @ g
    for _ in range(opts.coarse_iters - 1):
        e = e + Q @ (g - D @ e)
    got = airg.airg_vcycle(h, torch.as_tensor(g, device="cuda")).cpu().numpy()
    assert np.allclose(got, e, rtol=1e-11, atol=1e-13 * np.abs(e).max())
    got32 = airg.airg_vcycle(h, torch.as_tensor(g, device="cuda"), precision=32).cpu().numpy()
    assert np.linalg.norm(got32 - e) <= 1e-4 * np.linalg.norm(e)


def same_structure(h, H):
    st = airg.airg_get_stats(h)
    if st["levels"] != H.nlevels:
        return False
    for l in range(H.nlevels):
        if not np.array_equal(airg.airg_get_level_matrix(h, l, "A")[1], H.matrix(l, "A")[1]):
            return False
    return True


@pytest.mark.parametrize("kw", [{}, {"poly_sparsity_order": 2}, {"coarse_matrix_free": 1, "truncate_n": 2000},
                                {"strong_threshold": 0.0, "up_smooths": 1, "max_levels": 128}],
                         ids=["default", "s2", "matrix_free", "tol0"])
def test_vcycle_matches_oracle(kw):
    P = dg_square(32)
    h, _ = setup(P, **kw)
    H = O.Hierarchy((P.rowptr, P.col, P.val), O.default_params(seed=P.seed, **kw))
    assert same_structure(h, H)
    g = np.random.default_rng(3).standard_normal(P.n)
    want = H.vcycle(g)
    got = airg.airg_vcycle(h, torch.as_tensor(g, device="cuda")).cpu().numpy()
    got32 = airg.airg_vcycle(h, torch.as_tensor(g, device="cuda"), precision=32).cpu().numpy()
    r64 = np.linalg.norm(got - want) / np.linalg.norm(want)
    r32 = np.linalg.norm(got32 - want) / np.linalg.norm(want)
    print("V-cycle against the oracle's: fp64 %.3e fp32 %.3e" % (r64, r32))
    # the hierarchies' coefficients differ at the TSQR's rounding (about 1e-9 here); the FP32 cycle adds
    # single-precision rounding, a few units of 6e-8 per level (measured 1.6e-7).  The matrix-free
    # coarse polynomial sums alpha_k A^k x over thirteen powers whose coefficients are large and of
    # alternating sign, which magnifies FP32 rounding (measured 6.0e-5)
    assert r64 <= 1e-9
    assert r32 <= (1e-4 if kw.get("coarse_matrix_free") else 1e-5)


@pytest.mark.parametrize("kw", [{"poly_sparsity_order": 2}, {"poly_sparsity_order": 3},
                                {"coarse_matrix_free": 1, "truncate_n": 4000}], ids=["s2", "s3", "matrix_free"])
def test_variant_solves_match_oracle_iterations(kw):
    P = dg_square(48)
    h, _ = setup(P, **kw)
    x, info = airg.airg_solve(h, torch.as_tensor(P.b, device="cuda"), rtol=1e-10, max_it=200)
    assert info["converged"]
    r = P.b - O.spmv((P.rowptr, P.col, P.val), x.cpu().numpy())
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(P.b)
    H = O.Hierarchy((P.rowptr, P.col, P.val), O.default_params(seed=P.seed, **kw))
    _, its, _ = H.richardson(P.b, 1e-10, 200)
    assert abs(its - info["iterations"]) <= 1


def test_resetup_keeps_power_patterns():
    P = dg_square(40)
    h, _ = setup(P, poly_sparsity_order=2)
    before = airg.airg_get_level_matrix(h, 0, "Ainv")
    vals = P.val * np.random.default_rng(4).uniform(0.8, 1.2, P.val.shape)
    airg.airg_resetup(h, torch.as_tensor(vals, device="cuda"))
    prm = O.default_params(seed=P.seed, poly_sparsity_order=2)
    info = airg.airg_get_level(h, 0)
    mats = {k: airg.airg_get_level_matrix(h, 0, k) for k in ("A", "Ainv", "Z", "W")}
    assert np.array_equal(mats["Ainv"][1], before[1])
    want = O.level_renumeric(mats["A"], info["cf"], prm, 0, mats["W"], mats["Z"],
                             airg.airg_get_level_matrix(h, 1, "A"), alpha_in=info["alpha"])
    for key in ("Ainv", "Z"):
        assert np.array_equal(mats[key][2], want[key][2]), key


def test_batched_form_rejects_matrix_free_coarse():
    from workloads import batch as batch_problems, concat
    rp, ci, val, b, offs, seeds = concat(batch_problems(count=2, lo=12, hi=16, nrhs=1))
    with pytest.raises(airg.AirgError) as e:
        airg.airg_setup(*airg.to_device(rp, ci, val),
                        airg.default_opts(outer=1, precond_precision=32, coarse_matrix_free=1),
                        seg_offsets=offs, seg_seeds=seeds)
    assert e.value.status == -1
