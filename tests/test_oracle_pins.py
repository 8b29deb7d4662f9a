"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-derive the oracle's own formulas: they use a hand-worked
example, published generator outputs, brute force on tiny inputs, textbook
special cases (sequential greedy MIS, dense inverse, dense products, numpy
least squares, dense Arnoldi GMRES), invariants stated in the CF splitting
section (H1R, H2R), and the exact sweep solution.
"""
import json
import os

import numpy as np
import pytest
import scipy.stats

import oracle as O
from oracle.sweep import sweep_solve
from tests.helpers import dense, pattern, from_dense, random_nonsym, csr_of
from workloads import p0_square, dg_square, p0_cube

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def hand_matrix():
    g = load("cf_hand.json")
    rp, ci, v = [0], [], []
    for row in g["rows"]:
        for c, x in row:
            ci.append(c)
            v.append(x)
        rp.append(len(ci))
    return g, (np.array(rp), np.array(ci), np.array(v))


# ------------------------------------------------------------ generator --
def test_splitmix64_published_outputs():
    g = load("splitmix64.json")
    gamma = int(g["gamma"], 16)
    for k, want in enumerate(g["outputs"]):
        state = (g["seed"] + k * gamma) % 2 ** 64
        assert O.splitmix64(state) == int(want)


def test_gauss_rhs_is_standard_normal():
    b = O.gauss_rhs(200000, seed=7, level=3)
    ks = scipy.stats.kstest(b, "norm")
    assert ks.pvalue > 1e-3
    assert abs(b.mean()) < 0.01 and abs(b.std() - 1.0) < 0.01
    b2 = O.gauss_rhs(1000, seed=7, level=4)
    assert not np.allclose(b[:1000], b2)                 # levels draw different streams


# ------------------------------------------------------- hand example ----
def test_hand_example_strength_graph_pmisr_ddc():
    g, A = hand_matrix()
    strong = O.strength(A, g["alpha"])
    rp, ci = A[0], A[1]
    for i in range(g["n"]):
        got = sorted(ci[rp[i]:rp[i + 1]][strong[rp[i]:rp[i + 1]] == 1].tolist())
        assert got == g["strong_sets"][i]
    G = O.sym_graph(A, strong)
    for i in range(g["n"]):
        assert G[1][G[0][i]:G[0][i + 1]].tolist() == g["graph"][i]
    deg, _ = O.pmisr_keys(G, 0, 0)
    assert deg.tolist() == g["deg"]
    h = np.array(g["h"], dtype=np.uint32)
    cf, rounds = O.pmisr(G, deg, h, 3)
    assert cf.tolist() == g["pmisr_rounds_3"]["cf"] and rounds == g["pmisr_rounds_3"]["rounds"]
    cf1, _ = O.pmisr(G, deg, h, 1)
    assert cf1.tolist() == g["pmisr_rounds_1"]["cf"]
    for case in g["ddc"]:
        out, theta, _ = O.ddc(A, cf, case["alpha_diag"])
        assert out.tolist() == case["cf"]
        if "theta" in case:
            assert np.array_equal(theta, np.array(case["theta"]))


# ------------------------------------------------------------ strength ---
@pytest.mark.parametrize("seed", range(4))
def test_strength_brute_force(seed):
    D = random_nonsym(30, 0.15, seed)
    A = from_dense(D)
    for alpha in (0.0, 0.25, 0.5, 0.99, 1.0):
        s = O.strength(A, alpha)
        S = np.zeros_like(D, dtype=bool)
        S[np.repeat(np.arange(30), np.diff(A[0])), A[1]] = s.astype(bool)
        off = np.abs(D) * (1 - np.eye(30))
        mx = off.max(axis=1, keepdims=True)
        want = (off > 0) & (off >= alpha * mx)
        assert np.array_equal(S, want)
        # the strongest off-diagonal entry of every row is strong for alpha <= 1
        for i in range(30):
            if mx[i, 0] > 0:
                assert S[i, np.argmax(off[i])]
    assert O.strength(A, 1.5).sum() == 0


def test_symmetrised_graph_brute_force():
    D = random_nonsym(40, 0.1, 9)
    A = from_dense(D)
    s = O.strength(A, 0.5)
    S = np.zeros((40, 40), dtype=bool)
    S[np.repeat(np.arange(40), np.diff(A[0])), A[1]] = s.astype(bool)
    G = O.sym_graph(A, s)
    Gd = pattern(G)
    assert np.array_equal(Gd, S | S.T)
    assert not Gd.diagonal().any()
    for i in range(40):
        row = G[1][G[0][i]:G[0][i + 1]]
        assert np.all(np.diff(row) > 0)


# -------------------------------------------------------------- PMISR ----
def greedy_mis(G, deg, h):
    """Sequential greedy MIS visiting nodes by ascending (deg, h, index)."""
    n = len(deg)
    order = sorted(range(n), key=lambda i: (int(deg[i]), int(h[i]), i))
    inF = np.zeros(n, dtype=bool)
    for i in order:
        nb = G[1][G[0][i]:G[0][i + 1]]
        if not inF[nb].any():
            inF[i] = True
    return inF


@pytest.mark.parametrize("seed", range(6))
def test_pmisr_matches_greedy_mis_and_is_maximal(seed):
    D = random_nonsym(120, 0.04, seed)
    A = from_dense(D)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, h = O.pmisr_keys(G, seed + 100, 2)
    cf, rounds = O.pmisr(G, deg, h, 0)
    F = cf == O.F_POINT
    Gd = pattern(G)
    assert not (Gd & np.outer(F, F)).any()                    # independence (H1R)
    C = cf == O.C_POINT
    assert np.all(Gd[C][:, F].any(axis=1))                    # maximality
    assert np.array_equal(F, greedy_mis(G, deg, h))           # lexicographically-first MIS
    cf3, r3 = O.pmisr(G, deg, h, 3)
    F3 = cf3 == O.F_POINT
    assert not (Gd & np.outer(F3, F3)).any()
    assert np.all(~F3 | F)                                    # capped rounds give a subset of it
    assert np.all(F[deg == 0]) and np.all(F3[deg == 0])


def test_strength_zero_gives_independent_set_in_adjacency():
    P = p0_square(16)
    A = csr_of(P)
    prm = O.default_params(strong_threshold=0.0, seed=3)
    cf = O.cf_split(A, prm, 0)
    Aff = dense(O.submatrix(A, cf, O.F_POINT, O.F_POINT))
    assert np.count_nonzero(Aff - np.diag(np.diag(Aff))) == 0   # A_ff diagonal
    # and DDC leaves diagonal rows alone
    G = O.sym_graph(A, O.strength(A, 0.0))
    deg, h = O.pmisr_keys(G, 3, 0)
    cf0, _ = O.pmisr(G, deg, h, 3)
    assert np.array_equal(cf0, cf)


# ---------------------------------------------------------------- DDC ----
@pytest.mark.parametrize("seed", range(3))
def test_ddc_invariants(seed):
    P = dg_square(12)
    A = csr_of(P)
    D = dense(A)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, h = O.pmisr_keys(G, seed, 0)
    cf, _ = O.pmisr(G, deg, h, 3)
    for ad in (0.1, 0.5, 0.9):
        out, theta, cnt = O.ddc(A, cf, ad)
        F0 = cf == O.F_POINT
        F1 = out == O.F_POINT
        off = np.abs(D) * (1 - np.eye(D.shape[0]))
        th0 = (off[:, F0].sum(1)) / np.abs(np.diag(D))
        conv = F0 & ~F1
        assert cnt == conv.sum()
        assert np.all(th0[conv] > ad)                      # converted rows broke the threshold
        assert np.all(th0[F1] <= ad + 1e-15)               # kept rows meet it
        # H2R on the final A_ff: removing F columns only lowers the sums
        thf = off[:, F1].sum(1) / np.abs(np.diag(D))
        assert np.all(thf[F1] <= ad + 1e-15)
        assert np.all(out[~F0] == cf[~F0])


def test_ddc_fraction_threshold_converts_about_the_fraction():
    P = dg_square(24)
    A = csr_of(P)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, h = O.pmisr_keys(G, 1, 0)
    cf, _ = O.pmisr(G, deg, h, 3)
    nF = int((cf == O.F_POINT).sum())
    ad = O.ddc_fraction_threshold(A, cf, 0.1)
    _, theta, cnt = O.ddc(A, cf, ad)
    assert abs(cnt - np.ceil(0.1 * nF)) <= max(3, 0.02 * nF)


# --------------------------------------------------------- extraction ----
def test_submatrix_is_dense_slicing():
    D = random_nonsym(50, 0.1, 4)
    A = from_dense(D)
    cf = O.cf_split(A, O.default_params(seed=1), 0)
    F = np.nonzero(cf == O.F_POINT)[0]
    C = np.nonzero(cf == O.C_POINT)[0]
    for rs, cs, R, Cc in [(1, 1, F, F), (1, 2, F, C), (2, 1, C, F), (2, 2, C, C)]:
        S = O.submatrix(A, cf, rs, cs)
        assert np.array_equal(dense(S), D[np.ix_(R, Cc)])


# ---------------------------------------------------------- products -----
def test_spmv_spgemm_transpose_drop_brute_force():
    rng = np.random.default_rng(5)
    Da = np.where(rng.random((40, 30)) < 0.1, rng.standard_normal((40, 30)), 0.0)
    Db = np.where(rng.random((30, 25)) < 0.15, rng.standard_normal((30, 25)), 0.0)
    A, B = from_dense(Da), from_dense(Db)
    x = rng.standard_normal(30)
    assert np.allclose(O.spmv(A, x), Da @ x, rtol=1e-14, atol=1e-14)
    Cm = O.spgemm(A, B)
    assert np.allclose(dense(Cm), Da @ Db, rtol=1e-14, atol=1e-14)
    assert np.array_equal(pattern(Cm), (pattern(A).astype(int) @ pattern(B).astype(int)) > 0)
    assert np.array_equal(dense(O.transpose(A)), Da.T)
    Dsq = random_nonsym(30, 0.3, 6)
    for tau, kd in [(0.01, 1), (0.3, 1), (0.3, 0)]:
        Dr = dense(O.drop(from_dense(Dsq), tau, kd))
        mx = np.abs(Dsq).max(axis=1, keepdims=True)
        keep = (np.abs(Dsq) >= tau * mx) & (Dsq != 0)
        if kd:
            keep |= np.eye(30, dtype=bool)
        assert np.array_equal(Dr, np.where(keep, Dsq, 0.0))


# --------------------------------------------------- GMRES polynomial ----
def small_operator(seed=0, n=60):
    D = random_nonsym(n, 0.08, seed, dominance=1.2)
    return D, from_dense(D)


def test_power_basis_and_householder_r():
    D, A = small_operator(1)
    b = O.gauss_rhs(60, 5, 0)
    K = O.power_basis(A, b, 7)
    for k in range(8):
        assert np.allclose(K[:, k], np.linalg.matrix_power(D, k) @ b, rtol=1e-12, atol=0)
    R, nrm = O.householder_r(K)
    Ks = K / np.linalg.norm(K, axis=0)
    assert np.allclose(nrm, np.linalg.norm(K, axis=0), rtol=1e-14)
    assert np.allclose(np.triu(R), R)
    assert np.allclose(R.T @ R, Ks.T @ Ks, rtol=1e-12, atol=1e-13)   # Gram identity
    Rn = np.linalg.qr(Ks, mode="r")
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rn)), rtol=1e-10)


@pytest.mark.parametrize("m", [2, 4, 7])
def test_poly_coeffs_equal_lstsq_and_gmres_residual(m):
    D, A = small_operator(2)
    b = O.gauss_rhs(60, 11, 1)
    alpha, used = O.gmres_poly(A, 11, 1, m)
    assert used == m
    K = O.power_basis(A, b, m)
    ref = np.linalg.lstsq(K[:, 1:], K[:, 0], rcond=None)[0]
    assert np.allclose(alpha, ref, rtol=1e-8)
    # residual of the polynomial equals the m-step GMRES residual (dense Arnoldi)
    q = sum(a * np.linalg.matrix_power(D, k) for k, a in enumerate(alpha))
    res_poly = np.linalg.norm(b - D @ (q @ b))
    V = np.zeros((60, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        w = D @ V[:, j]
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    e1 = np.zeros(m + 1)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(H, e1, rcond=None)[0]
    res_gmres = np.linalg.norm(e1 - H @ y)
    assert abs(res_poly - res_gmres) <= 1e-8 * np.linalg.norm(b)


def test_poly_special_cases():
    # A = c I: q == 1/c, found through the Krylov breakdown
    n = 20
    for c in (0.25, 3.0, -2.0):
        A = from_dense(c * np.eye(n))
        alpha, used = O.gmres_poly(A, 1, 0, 7)
        assert used == 1 and np.isclose(alpha[0], 1.0 / c, rtol=1e-13) and np.all(alpha[1:] == 0)
    # two distinct eigenvalues: q(l) = (l1 + l2 - l) / (l1 l2) exactly
    A = from_dense(np.diag(np.where(np.arange(n) % 2 == 0, 1.0, 2.0)))
    alpha, used = O.gmres_poly(A, 1, 0, 7)
    assert used == 2 and np.allclose(alpha[:2], [1.5, -0.5], rtol=1e-12)
    # m >= n with a full pattern: q(A) = A^{-1} (Cayley-Hamilton)
    rng = np.random.default_rng(3)
    Dn = rng.random((5, 5)) + 5 * np.eye(5)
    A = from_dense(Dn)
    alpha, used = O.gmres_poly(A, 2, 0, 8)
    Q = sum(a * np.linalg.matrix_power(Dn, k) for k, a in enumerate(alpha))
    assert np.allclose(Q, np.linalg.inv(Dn), rtol=1e-7, atol=1e-9)
    # scaling A by s scales alpha_k by s^-(k+1)
    D, A = small_operator(4)
    a1, _ = O.gmres_poly(A, 9, 0, 5)
    a2, _ = O.gmres_poly(from_dense(4.0 * D), 9, 0, 5)
    assert np.allclose(a2, a1 / 4.0 ** (np.arange(5) + 1), rtol=1e-9)


def test_fixed_sparsity_polynomial():
    D, A = small_operator(6, 40)
    mask = (D != 0) | np.eye(40, dtype=bool)
    rng = np.random.default_rng(1)
    # order <= 2: every reading equals mask(q(A))
    for d in (1, 2, 3):
        al = rng.standard_normal(d)
        Q = sum(a * np.linalg.matrix_power(D, k) for k, a in enumerate(al))
        assert np.allclose(dense(O.poly_fixed_sparsity(A, al)), np.where(mask, Q, 0.0), rtol=1e-12, atol=1e-14)
    # diagonal A: diag(q(a_ii)) exactly
    dg = rng.random(40) + 1
    al = rng.standard_normal(6)
    got = dense(O.poly_fixed_sparsity(from_dense(np.diag(dg)), al))
    assert np.allclose(np.diag(got), sum(a * dg ** k for k, a in enumerate(al)), rtol=1e-13)
    # full pattern: the dense polynomial
    Dn = rng.random((6, 6)) + np.eye(6)
    Q = sum(a * np.linalg.matrix_power(Dn, k) for k, a in enumerate(al))
    assert np.allclose(dense(O.poly_fixed_sparsity(from_dense(Dn), al)), Q, rtol=1e-12)
    # order 3 on a path: the row-local reading (e_i^T M_i^k on J_i) differs from
    # masking the exact power; brute force of the row-local definition
    Dp = np.diag(np.full(6, 2.0)) + np.diag(np.full(5, -1.0), -1) + np.diag(np.full(5, -0.5), 1)
    al = np.array([0.0, 0.0, 0.0, 1.0])
    got = dense(O.poly_fixed_sparsity(from_dense(Dp), al))
    want = np.zeros((6, 6))
    for i in range(6):
        J = np.nonzero(Dp[i])[0]
        e = (J == i).astype(float)
        v = e @ np.linalg.matrix_power(Dp[np.ix_(J, J)], 3)
        want[i, J] = v
    assert np.allclose(got, want, rtol=1e-14)
    masked_exact = np.where(Dp != 0, np.linalg.matrix_power(Dp, 3), 0.0)
    assert not np.allclose(got, masked_exact)



def golden_rows(rows):
    rp, ci, v = [0], [], []
    for row in rows:
        for c, x in row:
            ci.append(c)
            v.append(x)
        rp.append(len(ci))
    return (np.array(rp), np.array(ci), np.array(v))


@pytest.mark.parametrize("case", load("ddc_fraction_hand.json")["cases"], ids=lambda c: c["name"])
def test_ddc_fraction_threshold_hand_cases(case):
    """Hand-worked thresholds: the closest count, ties to the larger k, strict
    comparison with the boundary, the ceiling target over all F rows, and an
    infinite theta counted but not part of theta_max."""
    A = golden_rows(case["rows"])
    cf = np.array(case["cf"], np.int8)
    assert O.ddc_fraction_threshold(A, cf, case["fraction"]) == case["alpha_diag"]


@pytest.mark.parametrize("seed", range(4))
def test_ddc_fraction_threshold_brute_force(seed):
    """Brute force over all 1001 boundaries from theta computed densely."""
    P = dg_square(16)
    A = csr_of(P)
    D = dense(A)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, h = O.pmisr_keys(G, seed, 0)
    cf, _ = O.pmisr(G, deg, h, 3)
    F = cf == O.F_POINT
    off = np.abs(D) * (1 - np.eye(D.shape[0]))
    theta = off[:, F].sum(1)[F] / np.abs(np.diag(D))[F]
    for frac in (0.05, 0.1, 0.3):
        target = int(np.ceil(frac * F.sum()))
        tmax = theta[np.isfinite(theta)].max()
        best, bestd = None, None
        for k in range(1001):
            bk = tmax * k / 1000.0
            d = abs(int((theta > bk).sum()) - target)
            if bestd is None or d <= bestd:
                best, bestd = bk, d
        assert O.ddc_fraction_threshold(A, cf, frac) == pytest.approx(best, rel=1e-12)

# -------------------------------------------- grid transfer, RAP, cycle ---
@pytest.mark.parametrize("mode", [0, 1])
def test_onepoint_w_brute_force(mode):
    """Weight 1 (mode 0) or -a_ij*/a_ii (mode 1) at the strongest neighbour."""
    P = dg_square(10)
    A = csr_of(P)
    D = dense(A)
    cf = O.cf_split(A, O.default_params(seed=4), 0)
    W = dense(O.onepoint_w(A, cf, mode))
    F = np.nonzero(cf == O.F_POINT)[0]
    C = np.nonzero(cf == O.C_POINT)[0]
    crank = {c: k for k, c in enumerate(C)}
    for r, i in enumerate(F):
        off = np.abs(D[i]).copy()
        off[i] = 0
        if off.max() == 0:
            assert not W[r].any()
            continue
        j = int(np.argmax(off))                       # first maximum = smallest index
        assert cf[j] == O.C_POINT                     # strongest neighbour of an F point is C
        want = np.zeros(len(C))
        want[crank[j]] = 1.0 if mode == 0 else -D[i, j] / D[i, i]
        assert np.array_equal(W[r], want)


def test_coarse_operator_dense_and_ideal_identity():
    P = dg_square(8)
    A = csr_of(P)
    D = dense(A)
    prm = O.default_params(seed=2)
    cf = O.cf_split(A, prm, 0)
    F = np.nonzero(cf == O.F_POINT)[0]
    C = np.nonzero(cf == O.C_POINT)[0]
    Aff, Afc, Acf, Acc = D[np.ix_(F, F)], D[np.ix_(F, C)], D[np.ix_(C, F)], D[np.ix_(C, C)]
    W = O.onepoint_w(A, cf, 0)
    Wd = dense(W)
    # ideal restrictor, no drop: R A P = Schur complement whatever W is
    Zi = -Acf @ np.linalg.inv(Aff)
    Ac = dense(O.coarse_operator(A, cf, from_dense(Zi), W, 0.0))
    S = Acc - Acf @ np.linalg.solve(Aff, Afc)
    assert np.allclose(Ac, S, rtol=1e-10, atol=1e-12 * np.abs(S).max())
    # approximate restrictor with drops: dense R A P then the row drop
    Ainv = O.poly_fixed_sparsity(O.submatrix(A, cf, 1, 1), O.gmres_poly(O.submatrix(A, cf, 1, 1), 2, 0, 7)[0])
    Z = O.restrictor(O.submatrix(A, cf, 2, 1), Ainv, 0.01)
    Zraw = -Acf @ dense(Ainv)
    mx = np.abs(Zraw).max(axis=1, keepdims=True)
    assert np.allclose(dense(Z), np.where(np.abs(Zraw) >= 0.01 * mx, Zraw, 0.0), rtol=1e-12, atol=1e-18)
    n = D.shape[0]
    Pm = np.zeros((n, len(C)))
    Pm[F] = Wd
    Pm[C, np.arange(len(C))] = 1.0
    Rm = np.zeros((len(C), n))
    Rm[:, F] = dense(Z)
    Rm[np.arange(len(C)), C] = 1.0
    RAP = Rm @ D @ Pm
    Acd = dense(O.coarse_operator(A, cf, Z, W, 0.001))
    mx = np.abs(RAP).max(axis=1, keepdims=True)
    keep = (np.abs(RAP) >= 0.001 * mx) | np.eye(len(C), dtype=bool)
    assert np.allclose(Acd, np.where(keep, RAP, 0.0), rtol=1e-11, atol=1e-14 * np.abs(RAP).max())


def test_two_level_cycle_is_exact_with_ideal_operators():
    """Strength 0 makes A_ff diagonal; two diagonal values make the GMRES
    polynomial exact; no drops give the ideal restrictor and the Schur
    complement; a long coarse solve is exact -> one cycle solves A x = b."""
    rng = np.random.default_rng(8)
    n = 40
    D = np.where(rng.random((n, n)) < 0.06, -0.2 * rng.random((n, n)), 0.0)
    np.fill_diagonal(D, np.where(rng.random(n) < 0.5, 1.0, 2.0))
    A = from_dense(D)
    prm = O.default_params(strong_threshold=0.0, drop_R=0.0, drop_A=0.0, max_levels=2,
                           coarse_iters=200, seed=5, poly_order=6)
    H = O.Hierarchy(A, prm)
    assert H.nlevels == 2
    b = rng.standard_normal(n)
    e = H.vcycle(b)
    assert np.linalg.norm(D @ e - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("make,bs", [(lambda: p0_square(48), 1), (lambda: dg_square(24), 3),
                                     (lambda: p0_cube(8), 1)])
def test_richardson_and_fgmres_reach_sweep_solution(make, bs):
    P = make()
    A = csr_of(P)
    H = O.Hierarchy(A, O.default_params(seed=P.seed))
    xs = sweep_solve(P.rowptr, P.col, P.val, P.b, bs)
    x, its, rr = H.richardson(P.b, 1e-10, 100)
    Dm = dense(A)
    assert rr <= 1e-10 and np.linalg.norm(Dm @ x - P.b) <= 1e-10 * np.linalg.norm(P.b) * 1.0001
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert its <= 30
    x2, its2, rr2 = H.fgmres(P.b, 1e-10, 100, 30)
    assert rr2 <= 1e-10 and np.linalg.norm(x2 - xs) <= 1e-8 * np.linalg.norm(xs)


def test_hierarchy_structure_and_storage():
    P = dg_square(32)
    H = O.Hierarchy(csr_of(P), O.default_params(seed=P.seed))
    ns = [H.matrix(l, "A")[0].shape[0] - 1 for l in range(H.nlevels)]
    assert all(a > b for a, b in zip(ns, ns[1:]))                 # strictly coarser
    assert ns[-1] < 100
    g, o, s = H.complexity()
    assert 1.0 < g < 4.0 and 1.0 < o < 10.0 and 1.0 < s < 10.0
    for l in range(H.nlevels - 1):
        cf = H.cf(l)
        Aff = dense(H.matrix(l, "Aff"))
        # every F row of A_ff meets the dominance threshold (H2R after DDC)
        off = np.abs(Aff).sum(1) - np.abs(np.diag(Aff))
        assert np.all(off <= 0.9 * np.abs(np.diag(Aff)) * (1 + 1e-14))
        assert (cf == O.F_POINT).sum() == Aff.shape[0]


def test_pmisr_index_breaks_exact_ties():
    """With every random part equal, the index decides (greedy by index)."""
    D = random_nonsym(80, 0.05, 21)
    A = from_dense(D)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, _ = O.pmisr_keys(G, 0, 0)
    h = np.zeros(80, dtype=np.uint32)
    cf, _ = O.pmisr(G, deg, h, 0)
    assert np.array_equal(cf == O.F_POINT, greedy_mis(G, deg, h))


def test_drop_keeps_small_diagonal():
    D = np.array([[1e-6, 2.0, -3.0], [1.0, 1e-9, 0.5], [0.25, -4.0, 1.0]])
    got = dense(O.drop(from_dense(D), 0.1, 1))
    want = np.array([[1e-6, 2.0, -3.0], [1.0, 1e-9, 0.5], [0.0, -4.0, 1.0]])
    assert np.array_equal(got, want)
    got0 = dense(O.drop(from_dense(D), 0.1, 0))
    assert got0[0, 0] == 0.0 and got0[1, 1] == 0.0


def test_householder_is_stable_for_nearly_aligned_columns():
    """Columns close to e_1 are where the reflector sign matters."""
    rng = np.random.default_rng(2)
    K = np.zeros((500, 4))
    K[0] = 1.0
    K[1:] = 1e-9 * rng.standard_normal((499, 4))
    R, nrm = O.householder_r(K)
    Ks = K / np.linalg.norm(K, axis=0)
    Rn = np.linalg.qr(Ks, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rn), rtol=1e-6, atol=1e-15)


# ------------------------------------------------------ numeric re-setup ---
# Reuse of the CF splitting and the symbolic products (Results section,
# padded-sparsity reading): the re-setup keeps every level's splitting and the
# patterns of W, Z and the coarse operators, and recomputes the values.

def _levels_equal(H, G):
    assert H.nlevels == G.nlevels
    for l in range(H.nlevels):
        if l < H.nlevels - 1:
            assert np.array_equal(H.cf(l), G.cf(l)), l
        assert np.array_equal(H.alpha(l), G.alpha(l)), l
        for key in ("A", "Ainv", "Z", "W", "Aff", "Afc"):
            a, b = H.matrix(l, key), G.matrix(l, key)
            assert (a is None) == (b is None), (l, key)
            if a is not None:
                assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])), (l, key)


def test_resetup_with_the_same_values_reproduces_the_hierarchy():
    P = dg_square(24)
    H = O.Hierarchy(csr_of(P), O.default_params(seed=P.seed))
    _levels_equal(H, H.resetup(H.matrix(0, "A")[2]))


def test_resetup_of_a_doubled_operator_equals_its_setup():
    """Scaling by 2 is exact in binary floating point: the splitting, every
    pattern after the drops, Z and the coarse patterns of setup(2A) equal
    those of setup(A); the coefficients halve per power.  So re-setup with
    2A must reproduce setup(2A) bit for bit."""
    P = p0_square(24)
    prm = O.default_params(seed=P.seed)
    H = O.Hierarchy(csr_of(P), prm)
    A2 = (P.rowptr, P.col, 2.0 * P.val)
    _levels_equal(O.Hierarchy(A2, prm), H.resetup(2.0 * H.matrix(0, "A")[2]))
    assert H.nlevels > 3


def test_resetup_values_are_the_products_on_the_old_patterns():
    """Level 0 against dense products: Z' = -A'_cf Ainv' on Z's pattern,
    W' = W (weight 1), A'_1 = R' A' P' on the old coarse pattern; and the
    re-set-up hierarchy solves the new system."""
    P = p0_square(12)
    prm = O.default_params(seed=P.seed)
    H = O.Hierarchy(csr_of(P), prm)
    vals = H.matrix(0, "A")[2] * np.random.default_rng(3).uniform(0.5, 1.5, H.matrix(0, "A")[2].shape)
    G = H.resetup(vals)
    Ad = dense((P.rowptr, P.col, vals))
    cf = G.cf(0)
    F, Cc = np.nonzero(cf == 1)[0], np.nonzero(cf == 2)[0]
    Ainv = dense(G.matrix(0, "Ainv"))
    Zd = -Ad[np.ix_(Cc, F)] @ Ainv
    Z = G.matrix(0, "Z")
    Zpat = H.matrix(0, "Z")
    assert np.array_equal(Z[0], Zpat[0]) and np.array_equal(Z[1], Zpat[1])
    rows = np.repeat(np.arange(len(Z[0]) - 1), np.diff(Z[0]))
    assert np.allclose(Z[2], Zd[rows, Z[1]], rtol=1e-13, atol=1e-16)
    W = G.matrix(0, "W")
    assert np.array_equal(W[2], np.ones_like(W[2]))
    n, nC = Ad.shape[0], len(Cc)
    R = np.zeros((nC, n))
    R[np.ix_(np.arange(nC), F)] = dense(Z)
    R[np.arange(nC), Cc] = 1.0
    Pm = np.zeros((n, nC))
    Pm[np.ix_(F, np.arange(nC))] = dense(W)
    Pm[Cc, np.arange(nC)] = 1.0
    Acd = R @ Ad @ Pm
    A1 = G.matrix(1, "A")
    assert np.array_equal(A1[1], H.matrix(1, "A")[1])
    r1 = np.repeat(np.arange(len(A1[0]) - 1), np.diff(A1[0]))
    scale = np.abs(Acd).max()
    assert np.allclose(A1[2], Acd[r1, A1[1]], rtol=1e-12, atol=1e-14 * scale)
    b = P.b
    x, its, rr = G.richardson(b, 1e-10, 200)
    xs = sweep_solve(P.rowptr, P.col, vals, b, 1)
    assert rr <= 1e-10 and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_tolerance_zero_hierarchy_has_diagonal_ff_and_direction_free_top_split():
    """Strong tolerance 0.0: A_ff diagonal on every level (an independent set
    in the adjacency graph), and the top splitting the same for every
    direction on one mesh (its symmetrised adjacency does not depend on it)."""
    prm = O.default_params(strong_threshold=0.0, up_smooths=1, max_levels=128)
    tops = []
    for theta in (0.3, 1.1, 2.5):
        P = dg_square(16, theta=theta)
        prm.seed = P.seed
        H = O.Hierarchy(csr_of(P), prm)
        for l in range(H.nlevels - 1):
            Aff = H.matrix(l, "Aff")
            assert np.array_equal(np.diff(Aff[0]), np.ones(len(Aff[0]) - 1, int)), l
            assert np.array_equal(Aff[1], np.arange(len(Aff[0]) - 1)), l
        tops.append(H.cf(0))
        x, its, rr = H.fgmres(P.b, 1e-10, 200)
        assert rr <= 1e-10
    assert all(np.array_equal(tops[0], t) for t in tops[1:])


# ------------------------------------------------ polynomial variants ---
# Sparsity order s (GMRES polynomial order subsection): the powers keep the
# pattern of A^s; the coarse polynomial may be applied matrix-free.

def test_power_pattern_brute_force():
    D, A = small_operator(6, 40)
    for order in (1, 2, 3):
        S = O.power_pattern(A, order)
        want = np.linalg.matrix_power((D != 0).astype(float), order) != 0
        assert np.array_equal(dense((S[0], S[1], np.ones(len(S[1])))) != 0, want), order


def test_sparsity_order_polynomial():
    D, A = small_operator(6, 40)
    rng = np.random.default_rng(4)
    n = D.shape[0]
    for s in (2, 3):
        S = O.power_pattern(A, s)
        # degree <= s: the row-local reading is the exact polynomial
        for d in range(1, s + 2):
            al = rng.standard_normal(d)
            Q = sum(a * np.linalg.matrix_power(D, k) for k, a in enumerate(al))
            got = dense(O.poly_fixed_sparsity_pattern(A, S, al))
            assert np.allclose(got, Q, rtol=1e-12, atol=1e-13), (s, d)
        # degree > s: e_i^T M_i^k on J_i = pattern(A^s)_i, brute force
        al = rng.standard_normal(s + 3)
        got = dense(O.poly_fixed_sparsity_pattern(A, S, al))
        Sd = dense((S[0], S[1], np.ones(len(S[1])))) != 0
        want = np.zeros((n, n))
        for i in range(n):
            J = np.nonzero(Sd[i] | (np.arange(n) == i))[0]
            M = D[np.ix_(J, J)]
            e = (J == i).astype(float)
            want[i, J] = sum(a * (e @ np.linalg.matrix_power(M, k)) for k, a in enumerate(al))
        assert np.allclose(got, want, rtol=1e-11, atol=1e-12), s


def test_matrix_free_coarse_polynomial_cycle():
    """One-level hierarchy (truncated at the top): the cycle is
    e = q(A) g, then e += q(A)(g - A e) twice, with q applied exactly."""
    P = p0_square(8)
    prm = O.default_params(seed=P.seed, truncate_n=10 ** 6, coarse_matrix_free=1)
    H = O.Hierarchy(csr_of(P), prm)
    assert H.nlevels == 1 and H.matrix(0, "Ainv") is None
    D = dense(csr_of(P))
    al = H.alpha(0)
    Q = sum(a * np.linalg.matrix_power(D, k) for k, a in enumerate(al))
    g = np.random.default_rng(6).standard_normal(D.shape[0])
    e = Q @ g
    for _ in range(prm.coarse_iters - 1):
        e = e + Q @ (g - D @ e)
    assert np.allclose(H.vcycle(g), e, rtol=1e-11, atol=1e-13 * np.abs(e).max())
    # and the assembled form differs from it (first-order fixed sparsity)
    prm.coarse_matrix_free = 0
    H1 = O.Hierarchy(csr_of(P), prm)
    assert not np.allclose(H1.vcycle(g), e, rtol=1e-6)


def test_sparsity_order_two_hierarchy_solves():
    P = dg_square(24)
    its = {}
    for s in (1, 2):
        H = O.Hierarchy(csr_of(P), O.default_params(seed=P.seed, poly_sparsity_order=s))
        x, its[s], rr = H.richardson(P.b, 1e-10, 200)
        assert rr <= 1e-10
        xs = sweep_solve(P.rowptr, P.col, P.val, P.b, 3)
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
        Ainv, Aff = H.matrix(0, "Ainv"), H.matrix(0, "Aff")
        S = O.power_pattern(Aff, s)
        assert np.array_equal(Ainv[0], S[0]) and np.array_equal(Ainv[1], S[1])
    assert its[2] <= its[1]


# ------------------------------------------------------------ complexities --
def test_complexity_hand_worked_two_level_hierarchy():
    g = load("complexity_hand.json")
    A = golden_rows(g["rows"])
    for vc, key in ((3, "storage_vc3"), (1, "storage_vc1")):
        H = O.Hierarchy(A, O.default_params(coarse_iters=vc, **g["params"]))
        assert H.nlevels == g["levels"]
        gr, op, st = H.complexity()
        assert gr == pytest.approx(g["grid"], rel=1e-15)
        assert op == pytest.approx(g["operator"], rel=1e-15)
        assert st == pytest.approx(g[key], rel=1e-15)


def test_complexity_single_level_diagonal():
    """A diagonal matrix is its own coarsest level: grid = operator = 1 and the
    storage is Ainv (n entries) plus A when more than one coarse iteration runs."""
    n = 10
    A = (np.arange(n + 1), np.arange(n), np.linspace(1.0, 2.0, n))
    for vc, want in ((1, 1.0), (3, 2.0)):
        H = O.Hierarchy(A, O.default_params(coarse_iters=vc))
        assert H.nlevels == 1
        assert H.complexity() == (1.0, 1.0, want)


@pytest.mark.parametrize("make,kw", [(lambda: dg_square(24), {}), (lambda: p0_square(32), {"coarse_iters": 1}),
                                     (lambda: dg_square(16), {"strong_threshold": 0.0, "max_levels": 40})])
def test_complexity_counted_from_the_assembled_matrices(make, kw):
    """The storage equation counted from the hierarchy's matrices, with R and P
    assembled densely as [Z I] and [W; I] in the level's full index space."""
    P = make()
    prm = O.default_params(seed=P.seed, **kw)
    H = O.Hierarchy(csr_of(P), prm)
    L = H.nlevels
    assert L >= 3
    nnz = lambda M: int(np.count_nonzero(pattern(M)))
    A = [H.matrix(l, "A") for l in range(L)]
    n = [len(a[0]) - 1 for a in A]
    store = 0
    for l in range(L - 1):
        cf = H.cf(l)
        F, C = np.nonzero(cf == O.F_POINT)[0], np.nonzero(cf == O.C_POINT)[0]
        R = np.zeros((len(C), n[l]), bool)
        R[:, F] = pattern(H.matrix(l, "Z"))
        R[np.arange(len(C)), C] = True
        Pm = np.zeros((n[l], len(C)), bool)
        Pm[F] = pattern(H.matrix(l, "W"))
        Pm[C, np.arange(len(C))] = True
        Dl = pattern(A[l])
        assert np.array_equal(pattern(H.matrix(l, "Aff")), Dl[np.ix_(F, F)])
        assert np.array_equal(pattern(H.matrix(l, "Afc")), Dl[np.ix_(F, C)])
        store += nnz(H.matrix(l, "Ainv")) + Dl[np.ix_(F, F)].sum() + Dl[np.ix_(F, C)].sum() + R.sum() + Pm.sum()
    store += nnz(H.matrix(L - 1, "Ainv")) + min(prm.coarse_iters - 1, 1) * nnz(A[L - 1])
    gr, op, st = H.complexity()
    assert gr == pytest.approx(sum(n) / n[0], rel=1e-14)
    assert op == pytest.approx(sum(nnz(a) for a in A) / nnz(A[0]), rel=1e-14)
    assert st == pytest.approx(store / nnz(A[0]), rel=1e-14)


# ------------------------------------------------------------------ replay --
def test_setup_replay_with_own_coefficients_is_identical():
    """Fed its own coefficients, the replay setup rebuilds the same hierarchy
    bit for bit; fed other coefficients, only the values change."""
    P = dg_square(24)
    A = csr_of(P)
    prm = O.default_params(seed=P.seed)
    H = O.Hierarchy(A, prm)
    al = [H.alpha(l) for l in range(H.nlevels)]
    R = O.Hierarchy(A, prm, alphas=al)
    assert R.nlevels == H.nlevels
    for l in range(H.nlevels):
        assert np.array_equal(R.alpha(l), H.alpha(l))
        for key in ("A", "Ainv", "Z", "W"):
            a, b = H.matrix(l, key), R.matrix(l, key)
            assert (a is None) == (b is None)
            if a is not None:
                assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])), (l, key)
    # level-0 coefficients scaled by 1 + 2^-20: level 0's Ainv changes, its splitting does not
    al2 = [a.copy() for a in al]
    al2[0] = al2[0] * (1 + 2.0 ** -20)
    R2 = O.Hierarchy(A, prm, alphas=al2[:1])
    assert np.array_equal(R2.cf(0), H.cf(0))
    assert np.array_equal(R2.alpha(0), al2[0])
    assert not np.array_equal(R2.matrix(0, "Ainv")[2], H.matrix(0, "Ainv")[2])
    assert np.array_equal(R2.alpha(1), O.Hierarchy(A, prm, alphas=al2[:1]).alpha(1))


# ----------------------------------------------------------------- threads --
@pytest.mark.parametrize("make", [lambda: dg_square(40), lambda: p0_cube(10)], ids=["dg40", "cube10"])
def test_thread_count_does_not_change_results(make):
    """The oracle's row-parallel loops leave every result bit for bit equal
    to the single-threaded run: hierarchy, cycle, Richardson and FGMRES."""
    P = make()
    A = csr_of(P)
    prm = O.default_params(seed=P.seed)
    nthreads = max(4, O.get_threads())
    runs = []
    try:
        for t in (1, nthreads):
            O.set_threads(t)
            H = O.Hierarchy(A, prm)
            mats = [[H.matrix(l, k) for k in ("A", "Ainv", "Z", "W")] for l in range(H.nlevels)]
            g = np.random.default_rng(3).standard_normal(P.n)
            runs.append((H.nlevels, mats, H.vcycle(g), H.richardson(P.b, 1e-10, 50), H.fgmres(P.b, 1e-10, 50, 30),
                         H.complexity()))
    finally:
        O.set_threads(nthreads)
    a, b = runs
    assert a[0] == b[0]
    for la, lb in zip(a[1], b[1]):
        for x, y in zip(la, lb):
            assert (x is None) == (y is None)
            if x is not None:
                assert all(np.array_equal(p, q) for p, q in zip(x[:3], y[:3]))
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3][0], b[3][0]) and a[3][1:] == b[3][1:]
    assert np.array_equal(a[4][0], b[4][0]) and a[4][1:] == b[4][1:]
    assert a[5] == b[5]
