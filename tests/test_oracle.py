"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses an
independent route (exact rational arithmetic, LAPACK through numpy/scipy,
closed forms, the textbook error bound of Gaussian elimination, the
iteration-count law the paper states for Algorithm 1).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import exact
from oracle import oracle as O
from synth import gen

U_D = 2.0 ** -53
U_S = 2.0 ** -24


def _perm_matrix(ipiv, n):
    """P with P A = rows of A after applying the swap sequence ipiv."""
    order = np.arange(n)
    for k, p in enumerate(ipiv):
        order[[k, p]] = order[[p, k]]
    P = np.zeros((n, n))
    P[np.arange(n), order] = 1.0
    return P


def _split_lu(LU):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U


# ------------------------------------------------------------ factorization

@pytest.mark.parametrize("n", [1, 2, 7, 64, 150])
def test_getrf_backward_error_bound(n):
    """|PA - LU| <= gamma_n |L||U| elementwise (Higham, Thm 9.3): the textbook
    bound for Gaussian elimination; the product is formed in long double so
    its own rounding is far below the bound."""
    A = gen.uniform_system(n, 10 + n)[0]
    LU, ipiv, info = O.getrf(A)
    assert info == 0
    L, U = _split_lu(LU)
    P = _perm_matrix(ipiv, n)
    ld = np.longdouble
    PA = (P.astype(ld) @ A.astype(ld))
    prod = L.astype(ld) @ U.astype(ld)
    absprod = np.abs(L).astype(ld) @ np.abs(U).astype(ld)
    gamma = n * U_D / (1 - n * U_D)
    assert np.all(np.abs(PA - prod) <= gamma * absprod + 1e-300)
    # partial pivoting: every multiplier has magnitude at most one
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)


def test_getrf_pivots_match_lapack():
    """Same pivot sequence as LAPACK dgetrf (scipy) on a random matrix."""
    A = gen.uniform_system(120, 3)[0]
    LU, ipiv, info = O.getrf(A)
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert info == 0
    np.testing.assert_array_equal(ipiv, piv_ref)
    np.testing.assert_allclose(LU, lu_ref, rtol=0, atol=1e-12 * np.abs(lu_ref).max())


def _gamma(n, u):
    return n * u / (1 - n * u)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (17, 2), (64, 3), (150, 4), (150, 5)])
def test_sgetrf_backward_error_and_lapack_pivots(n, seed):
    """The FP32 elimination of Algorithm 1 step 1: |PA - LU| <= gamma_n u_s
    |L||U| elementwise for the FP32 input (Higham, Thm 9.3 with the single
    precision unit roundoff), |l_ij| <= 1, and the same pivot sequence as
    LAPACK's sgetrf (scipy on the FP32 matrix) on random inputs."""
    A = gen.uniform_system(n, 900 + seed)[0].astype(np.float32)
    LU, ipiv, info = O.sgetrf(A)
    assert info == 0 and LU.dtype == np.float32
    L, U = _split_lu(LU.astype(np.float64))
    P = _perm_matrix(ipiv, n)
    ld = np.longdouble
    PA = P.astype(ld) @ A.astype(ld)
    prod = L.astype(ld) @ U.astype(ld)
    absprod = np.abs(L).astype(ld) @ np.abs(U).astype(ld)
    assert np.all(np.abs(PA - prod) <= _gamma(n, U_S) * absprod + 1e-300)
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert lu_ref.dtype == np.float32
    np.testing.assert_array_equal(ipiv, piv_ref)
    # the factors agree with LAPACK's to a few FP32 units of |L||U|
    assert np.all(np.abs(LU.astype(np.float64) - lu_ref) <=
                  8 * _gamma(n, U_S) * (np.abs(L) @ np.abs(U)) + 1e-30)


@pytest.mark.parametrize("n", [1, 9, 80, 150])
def test_sgetrs_triangular_solve_backward_error(n):
    """The FP32 solves with the FP32 factors (Algorithm 1 steps 2-3): the
    computed x satisfies |P b - L U x| <= (2 gamma_n + gamma_n^2) |L||U||x|
    elementwise (Higham, the proof of Thm 9.4, in single precision), with
    L, U, x exact FP32 numbers and the check evaluated in long double."""
    A, b, _ = gen.prescribed_cond_system(n, 1e3, 950 + n, nrhs=2)
    LU, ipiv, info = O.sgetrf(A.astype(np.float32))
    assert info == 0
    b32 = b.astype(np.float32)
    x = O.sgetrs(LU, ipiv, b32)
    assert x.dtype == np.float32
    L, U = _split_lu(LU.astype(np.float64))
    P = _perm_matrix(ipiv, n)
    ld = np.longdouble
    lhs = P.astype(ld) @ b32.astype(ld) - L.astype(ld) @ (U.astype(ld) @ x.astype(ld))
    g = _gamma(n, U_S)
    bound = (2 * g + g * g) * (np.abs(L).astype(ld) @ (np.abs(U).astype(ld) @ np.abs(x).astype(ld)))
    assert np.all(np.abs(lhs) <= bound + 1e-300)


@pytest.mark.parametrize("n", [1, 5, 64, 130])
def test_spotrf_spotrs_backward_error(n):
    """FP32 Cholesky (the SPOTRF of Section 3.1.1): |A - L L^T| <= gamma_{n+1}
    u_s |L||L^T| (Higham, Thm 10.3), agreement with LAPACK's spotrf through
    numpy on the FP32 matrix, and the FP32 solves satisfy |b - L L^T x| <=
    (2 gamma_n + gamma_n^2) |L||L^T||x|."""
    A, B, _ = gen.spd_system(n, 1e2, 960 + n, nrhs=2)
    A32 = A.astype(np.float32)
    L, info = O.spotrf(A32)
    assert info == 0 and L.dtype == np.float32
    Ld = L.astype(np.float64)
    ld = np.longdouble
    err = np.abs(A32.astype(ld) - Ld.astype(ld) @ Ld.T.astype(ld))
    absprod = np.abs(Ld).astype(ld) @ np.abs(Ld.T).astype(ld)
    assert np.all(err <= _gamma(n + 1, U_S) * absprod + 1e-300)
    L_ref = np.linalg.cholesky(A32)
    assert L_ref.dtype == np.float32
    assert np.all(np.abs(Ld - L_ref) <= 8 * _gamma(n + 1, U_S) * np.sqrt(np.abs(np.diag(A32)))[None, :]
                  * np.ones((n, 1)) + 1e-30)
    b32 = B.astype(np.float32)
    x = O.spotrs(L, b32)
    g = _gamma(n, U_S)
    lhs = b32.astype(ld) - Ld.astype(ld) @ (Ld.T.astype(ld) @ x.astype(ld))
    bound = (2 * g + g * g) * (np.abs(Ld).astype(ld) @ (np.abs(Ld.T).astype(ld) @ np.abs(x).astype(ld)))
    assert np.all(np.abs(lhs) <= bound + 1e-300)


def test_getrf_tiny_pivot_swaps():
    """2x2 with a tiny leading entry must exchange the rows."""
    A = np.array([[1e-20, 1.0], [1.0, 1.0]])
    LU, ipiv, info = O.getrf(A)
    assert info == 0 and list(ipiv) == [1, 1]
    x = O.gesv_ir(A, np.array([1.0, 2.0])).x
    # exact solution: x1 = 1/(1-1e-20) ~ 1, x0 = 1 - x1*... both within u of 1
    exact_x = exact.solve([[Fraction(1e-20), 1], [1, 1]], [1, 2])
    np.testing.assert_allclose(x, [float(v) for v in exact_x], rtol=4 * U_D)


def test_getrf_ties_take_first_index():
    A = np.array([[1.0, 2.0, 0.0], [-1.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    _, ipiv, info = O.getrf(A)
    assert info == 0 and ipiv[0] == 0


def test_getrf_singular_reports_column():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    _, _, info = O.getrf(A)
    assert info == 3  # column 2 (1-based 3) has no nonzero pivot left
    assert O.getrf(np.zeros((2, 2)))[2] == 1


# ------------------------------------------------------------------- solves

def test_exact_solver_is_exact():
    """The rational solver's x satisfies A x = b exactly, and matches Cramer's
    rule on a 3x3 (brute force via determinants)."""
    A, b, _ = gen.integer_system(6, 5)
    x = exact.solve(A.tolist(), b[:, 0].tolist())
    assert all(r == 0 for r in exact.residual(A.tolist(), x, b[:, 0].tolist()))
    M = [[2, -1, 3], [4, 0, -2], [1, 5, 1]]
    rhs = [3, -7, 2]

    def det3(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))

    d = det3(M)
    cramer = []
    for c in range(3):
        Mc = [row[:] for row in M]
        for i in range(3):
            Mc[i][c] = rhs[i]
        cramer.append(Fraction(det3(Mc), d))
    assert exact.solve(M, rhs) == cramer


@pytest.mark.parametrize("seed", range(6))
def test_refined_solution_vs_exact_rational(seed):
    """Integer systems n <= 12: the refined FP64 oracle x agrees with the exact
    rational solution to within a few units of the condition-weighted
    roundoff (in practice to the last bits)."""
    n = 4 + 2 * seed
    g = np.random.default_rng(100 + seed)
    A = g.integers(-9, 10, (n, n)).astype(float)
    b = g.integers(-9, 10, (n, 1)).astype(float)
    try:
        xe = exact.solve(A.tolist(), b[:, 0].tolist())
    except ZeroDivisionError:
        pytest.skip("singular draw")
    xe = np.array([float(v) for v in xe])
    res = O.gesv_ir(A, b)
    assert res.info == 0 and res.iters >= 0
    kappa = np.linalg.cond(A, np.inf)
    err = np.abs(res.x[:, 0] - xe).max() / np.abs(xe).max()
    assert err <= 4 * kappa * U_D


@pytest.mark.parametrize("n", [3, 8, 12])
def test_planted_integer_solution_recovered(n):
    A, b, x_true = gen.integer_system(n, 40 + n)
    res = O.gesv_ir(A, b)
    kappa = np.linalg.cond(A, np.inf)
    err = np.abs(res.x - x_true).max() / np.abs(x_true).max()
    assert res.iters >= 0 and err <= 4 * kappa * U_D
    # the mixed-precision Algorithm 1 recovers it too
    res32 = O.gesv_ir(A, b, lowp=True)
    assert res32.iters >= 0
    assert np.abs(res32.x - x_true).max() / np.abs(x_true).max() <= 4 * kappa * U_D


def test_special_cases():
    # n = 1: x = fl(b / a), no correction needed
    r = O.gesv_ir(np.array([[3.0]]), np.array([1.0]))
    assert r.x[0] == 1.0 / 3.0 and r.iters == 0
    # identity: x = b bitwise, zero corrections
    b = np.random.default_rng(1).uniform(-1, 1, 17)
    r = O.gesv_ir(np.eye(17), b)
    assert np.array_equal(r.x, b) and r.iters == 0
    # diagonal: correctly rounded quotients
    d = np.random.default_rng(2).uniform(1, 2, 9)
    r = O.gesv_ir(np.diag(d), b[:9])
    assert np.array_equal(r.x, b[:9] / d)
    # permutation matrix: exact
    p = np.random.default_rng(3).permutation(11)
    Pm = np.eye(11)[p]
    r = O.gesv_ir(Pm, b[:11])
    assert np.array_equal(Pm @ r.x, b[:11])
    # n = 0 is a no-op
    r = O.gesv_ir(np.zeros((0, 0)), np.zeros(0))
    assert r.iters == 0 and r.x.shape == (0,)


@pytest.mark.parametrize("n,kappa", [(50, 1e2), (200, 1e6)])
def test_against_lapack_solve(n, kappa):
    A, b, x_true = gen.prescribed_cond_system(n, kappa, 7)
    r = O.gesv_ir(A, b)
    ref = np.linalg.solve(A, b)
    assert np.abs(r.x - ref).max() / np.abs(ref).max() <= 8 * kappa * U_D
    assert np.abs(r.x - x_true).max() / np.abs(x_true).max() <= 8 * kappa * U_D * np.sqrt(n)
    assert O.metrics(A, r.x, b)["passes"]


def test_multiple_rhs_all_columns_certified():
    A, b, x_true = gen.prescribed_cond_system(80, 1e3, 9, nrhs=5)
    for lowp in (False, True):
        r = O.gesv_ir(A, b, lowp=lowp)
        assert r.iters >= 0
        m = O.metrics(A, r.x, b)
        assert m["passes"]
        ref = np.linalg.solve(A, b)
        assert (np.abs(r.x - ref).max(axis=0) / np.abs(ref).max(axis=0)).max() <= 1e-12 * 1e3


def test_transposed_solve_and_adjoint_identity():
    """A^T solve vs LAPACK, and <A^{-1} b, w> = <b, A^{-T} w>."""
    n = 60
    A, b, _ = gen.prescribed_cond_system(n, 1e2, 11)
    w = np.random.default_rng(12).standard_normal((n, 1))
    rt = O.gesv_ir(A, w, trans=True)
    ref = np.linalg.solve(A.T, w)
    assert np.abs(rt.x - ref).max() / np.abs(ref).max() <= 1e-13
    x = O.gesv_ir(A, b).x
    lhs = float((x * w).sum())
    rhs = float((b * rt.x).sum())
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(x).sum() * np.abs(w).max())


def test_getrs_trans_matches_direct_definition():
    n = 30
    A = gen.uniform_system(n, 13)[0]
    LU, ipiv, _ = O.getrf(A)
    B = np.random.default_rng(14).standard_normal((n, 3))
    X = O.getrs(LU, ipiv, B, trans=True)
    np.testing.assert_allclose(A.T @ X, B, atol=1e-12)
    X = O.getrs(LU, ipiv, B, trans=False)
    np.testing.assert_allclose(A @ X, B, atol=1e-12)


# ---------------------------------------------------------------- Cholesky

@pytest.mark.parametrize("n", [1, 5, 64, 130])
def test_cholesky_matches_lapack(n):
    A, B, X = gen.spd_system(n, 1e3, 20 + n, nrhs=3)
    L, info = O.potrf(A)
    assert info == 0
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=0, atol=1e-12)
    ld = np.longdouble
    rec = L.astype(ld) @ L.T.astype(ld)
    gamma = (n + 1) * U_D / (1 - (n + 1) * U_D)
    assert np.all(np.abs(rec - A.astype(ld)) <= gamma * (np.abs(L) @ np.abs(L).T) + 1e-300)
    for lowp in (False, True):
        r = O.posv_ir(A, B, lowp=lowp)
        assert r.info == 0 and r.iters >= 0
        assert O.metrics(A, r.x, B)["passes"]
        assert np.abs(r.x - X).max() <= 1e-12 * 1e3 * np.sqrt(n)


def test_cholesky_indefinite_breaks_down():
    A = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 3.0], [0.0, 3.0, 5.0]])
    _, info = O.potrf(A)
    assert info == 2
    assert O.posv_ir(A, np.ones(3)).iters == -1


# -------------------------------------------------------------- residuals

def test_extended_residual_matches_exact():
    A, b, _ = gen.integer_system(5, 31)
    x = np.array([0.1, -0.3, 1.0 / 3.0, 2.5, -7.25])
    rn, cb = O.residual_ld(A, x, b)
    r = exact.residual(A.tolist(), [Fraction(v) for v in x], b[:, 0].tolist())
    assert abs(rn[0] - float(max(abs(v) for v in r))) <= 1e-18 * max(1.0, rn[0])
    # exact solution -> zero residual, zero backward errors
    xe = exact.solve(A.tolist(), b[:, 0].tolist())
    assert all(v.denominator == 1 for v in xe)
    m = O.metrics(A, np.array([float(v) for v in xe]), b)
    assert m["rnorm"][0] == 0.0 and m["nbe"][0] == 0.0 and m["cbe"][0] == 0.0


def test_fp64_residual_sign_and_transpose():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    x = np.array([1.0, 1.0])
    b = np.array([10.0, 20.0])
    np.testing.assert_array_equal(O.residual(A, x, b), [7.0, 13.0])
    np.testing.assert_array_equal(O.residual(A, x, b, trans=True), [6.0, 14.0])


def test_norm_inf():
    A = np.array([[1.0, -2.0], [-3.0, 0.5]])
    assert O.norm_inf(A) == 3.5


# ---------------------------------------------- iteration-count law (Sec. 4)

def _datta(kappa, eps_s=U_S, eps_d=U_D):
    return math.ceil(math.log(eps_d) / (math.log(eps_s) + math.log(kappa)))


def test_mixed_iteration_count_follows_law():
    """Algorithm 1 with an FP32 factor on random 200x200 matrices of
    prescribed condition number (the protocol of Section 4, fewer matrices).
    The generalized Datta formula ceil(ln eps_d / (ln eps_s + ln kappa)) takes
    the worst-case contraction kappa*eps_s per step, so the observed number of
    solves (x_0 plus corrections) lies between its kappa -> 1 limit
    ceil(ln eps_d / ln eps_s) = 3 and the formula, and grows with kappa."""
    means = []
    for kappa in (1e1, 1e3, 1e5, 1e6):
        g = np.random.default_rng(int(kappa))
        counts = []
        for _ in range(10):
            A, b, _ = gen.prescribed_cond_system(200, kappa, g)
            r = O.gesv_ir(A, b, lowp=True)
            assert r.iters >= 0
            counts.append(r.iters + 1)
        mean = float(np.mean(counts))
        assert _datta(1.0) <= mean <= _datta(kappa), (kappa, mean, _datta(kappa))
        means.append(mean)
    assert means == sorted(means) and means[-1] > means[0]


def test_mixed_fails_when_kappa_eps_s_above_one():
    """kappa * eps_s > 1: no convergence within 30 iterations (Section 4)."""
    g = np.random.default_rng(77)
    fails = 0
    for _ in range(4):
        A, b, _ = gen.prescribed_cond_system(200, 1e9, g)
        r = O.gesv_ir(A, b, lowp=True)
        fails += r.iters == -31
    assert fails >= 3


# ---------------------------------------------------------------- inputs

def test_generators_are_seeded_and_well_formed():
    A1, b1, x1 = gen.prescribed_cond_system(64, 1e4, 5)
    A2, b2, x2 = gen.prescribed_cond_system(64, 1e4, 5)
    assert np.array_equal(A1, A2) and np.array_equal(b1, b2)
    s = np.linalg.svd(A1, compute_uv=False)
    assert abs(s[0] / s[-1] / 1e4 - 1) < 1e-8
    Q = gen.haar_orthogonal(40, np.random.default_rng(0))
    np.testing.assert_allclose(Q.T @ Q, np.eye(40), atol=1e-13)
    A, B, X = gen.spd_system(50, 1e3, 6, nrhs=4)
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[-1] - 1) < 1e-12 and abs(ev[0] * 1e3 - 1) < 1e-9
    As, bs, xs, ks = gen.batched_systems(count=5, seed=401, nmin=16, nmax=40)
    assert all(16 <= a.shape[0] <= 40 for a in As) and all(1e1 <= k <= 1e5 for k in ks)


def _golden_exact_systems():
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "exact_systems.json")
    with open(path) as f:
        return json.load(f)["systems"]


@pytest.mark.parametrize("case", _golden_exact_systems(), ids=lambda c: f"n{c['n']}")
def test_golden_exact_systems(case):
    """Stored exact solutions satisfy A x = b exactly, and the refined FP64
    oracle reproduces them to the condition-weighted roundoff."""
    A, b = case["A"], case["b"]
    x = [Fraction(s) for s in case["x"]]
    assert all(r == 0 for r in exact.residual(A, x, b))
    xf = np.array([float(v) for v in x])
    r = O.gesv_ir(np.array(A, float), np.array(b, float))
    kappa = np.linalg.cond(np.array(A, float), np.inf)
    assert np.abs(r.x - xf).max() <= 4 * kappa * U_D * np.abs(xf).max()


# ---------------------------------------------------------------- kappa_1
def test_condest_diagonal_is_exact():
    """For diagonal A the first sweep moves to the smallest |d_j| and the
    estimate is kappa_1 = max|d| / min|d| exactly."""
    g = np.random.default_rng(21)
    d = g.uniform(0.5, 2.0, 30) * np.where(g.random(30) < 0.5, -1.0, 1.0)
    d[11] = 3e-5
    A = np.diag(d)
    assert O.condest1(A) == pytest.approx(np.abs(d).max() / np.abs(d).min(), rel=1e-14)


def test_condest_bidiagonal_closed_form():
    """A = I - 2 N (N the shift above the diagonal): (A^{-1})_ij = 2^(j-i)
    for j >= i, so ||A^{-1}||_1 = 2^n - 1 (last column) and ||A||_1 = 3;
    the method reaches that column in one sweep."""
    for n in (2, 5, 20, 40):
        A = np.eye(n) - 2.0 * np.eye(n, k=1)
        assert O.condest1(A) == pytest.approx(3.0 * (2.0 ** n - 1.0), rel=1e-13)


def test_condest_special_cases():
    assert O.condest1(np.array([[-4.0]])) == 1.0
    assert O.condest1(np.eye(7)) == 1.0
    P = np.eye(9)[[3, 0, 8, 1, 2, 7, 6, 5, 4]]
    assert O.condest1(P) == pytest.approx(1.0, rel=1e-15)
    assert O.condest1(np.zeros((0, 0))) == 0.0


def test_condest_bounds_on_random_matrices():
    """A lower bound of the true kappa_1 (||A^{-1}||_1 computed column by
    column from the inverse), and never below a third of it on these seeded
    matrices: iid uniform, a badly scaled column, prescribed singular values."""
    for seed in range(45):
        g = np.random.default_rng(300 + seed)
        n = int(g.choice([3, 8, 20, 60]))
        if seed % 3 == 0:
            A = g.uniform(-1, 1, (n, n))
        elif seed % 3 == 1:
            A = g.standard_normal((n, n))
            A[:, 0] *= 1e-4
        else:
            A, _, _ = gen.prescribed_cond_system(n, 1e6, g)
        true = np.abs(A).sum(axis=0).max() * np.abs(np.linalg.inv(A)).sum(axis=0).max()
        est = O.condest1(A)
        assert est <= true * (1 + 1e-9), (seed, est, true)
        assert est >= true / 3.0, (seed, est, true)


# --------------------------------------------- sparse inner-outer FGMRES
def _dense_from_csr(rp, ci, v):
    n = len(rp) - 1
    A = np.zeros((n, n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            A[i, ci[p]] += v[p]
    return A


def test_sparse_generator_and_matvec():
    """The 3-D Poisson matrix (Peclet 0) has the closed-form eigenvalues
    6 - 2 (cos(a pi/(k+1)) + cos(b pi/(k+1)) + cos(c pi/(k+1))); its
    upwind convection-diffusion variant has zero interior row sums; the CRS
    product equals the dense product built entry by entry."""
    from oracle import sparse_ir as S

    k = 5
    rp, ci, v, b, x = gen.sparse_convdiff3d(k, 0.0, 1)
    A = _dense_from_csr(rp, ci, v)
    t = np.cos(np.arange(1, k + 1) * np.pi / (k + 1))
    lam = np.sort((6 - 2 * (t[:, None, None] + t[None, :, None] + t[None, None, :])).ravel())
    assert np.allclose(np.linalg.eigvalsh(A), lam, atol=1e-12)
    assert np.allclose(A @ x, b, atol=1e-14)
    rp2, ci2, v2, b2, x2 = gen.sparse_convdiff3d(k, 0.7, 2)
    A2 = _dense_from_csr(rp2, ci2, v2)
    interior = [i + k * j + k * k * l for l in range(1, k - 1) for j in range(1, k - 1)
                for i in range(1, k - 1)]
    assert np.allclose(A2[interior].sum(axis=1), 0.0, atol=1e-13)
    g = np.random.default_rng(4)
    u = g.standard_normal(k ** 3)
    assert np.allclose(S.csr_matvec(rp2, ci2, v2, u), A2 @ u, atol=1e-13)
    assert S.norm_inf_csr(rp2, v2) == pytest.approx(np.abs(A2).sum(axis=1).max())


def test_gmres_cycle_closed_forms():
    """GMRES(1) from zero is the minimal-residual step z = (v.Av / Av.Av) v;
    GMRES(n) in FP64 exhausts the Krylov space and solves the system."""
    from oracle import sparse_ir as S

    rp, ci, v, _, _ = gen.sparse_convdiff3d(3, 0.4, 5)
    A = _dense_from_csr(rp, ci, v)
    g = np.random.default_rng(6)
    w = g.standard_normal(27)
    mv = lambda u: A @ u
    z, k = S.gmres_cycle(mv, w, 1, np.float64)
    Aw = A @ w
    assert k == 1 and np.allclose(z, (w @ Aw) / (Aw @ Aw) * w, rtol=1e-13)
    z, k = S.gmres_cycle(mv, w, 27, np.float64)
    assert np.linalg.norm(A @ z - w) <= 1e-12 * np.linalg.norm(w)
    # single precision: the residual stalls near the FP32 unit roundoff, not below
    z32, _ = S.gmres_cycle(lambda u: (A.astype(np.float32) @ u), w.astype(np.float32), 27,
                           np.float32)
    rel = np.linalg.norm(A @ z32.astype(np.float64) - w) / np.linalg.norm(w)
    assert 1e-9 < rel < 1e-5


def test_fgmres_gmres_sp_solves():
    """Algorithm 2 on Poisson and convection-diffusion: the stopping rule
    holds for the returned x, which matches the dense direct solution; FP64
    inner solves (the GMRES_DP variant) also converge; on the identity FP64
    inner cycles finish in at most two applications, while FP32 inner cycles
    need a few outer steps to remove their rounding."""
    from oracle import sparse_ir as S

    for k, p in ((6, 0.0), (7, 1.5)):
        rp, ci, v, b, x_true = gen.sparse_convdiff3d(k, p, 10 + k)
        A = _dense_from_csr(rp, ci, v)
        for dt in (np.float32, np.float64):
            r = S.fgmres_gmres(rp, ci, v, b, m_out=8, m_in=10, inner_dtype=dt)
            assert r.converged, (k, p, dt)
            res = b - A @ r.x
            assert np.abs(res).max() <= np.sqrt(len(b)) * 2.0 ** -53 * np.abs(A).sum(1).max() * \
                np.abs(r.x).max()
            xs = np.linalg.solve(A, b)
            assert np.abs(r.x - xs).max() <= 1e-12 * np.linalg.cond(A) * np.abs(xs).max()
    n = 10
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(1).uniform(-1, 1, n)
    # FP64 inner solves invert the identity up to FP64 rounding: at most a
    # second application removes it
    r = S.fgmres_gmres(rp, ci, np.ones(n), b, m_out=5, m_in=5, inner_dtype=np.float64)
    assert r.converged and r.inner_calls <= 2 and np.abs(r.x - b).max() <= 4e-16
    # FP32 inner solves leave a rounding-size residual for the outer steps to remove
    r = S.fgmres_gmres(rp, ci, np.ones(n), b, m_out=5, m_in=5)
    assert r.converged and 1 < r.inner_calls <= 5 and np.abs(r.x - b).max() <= 4e-16
