"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests uses the GPU. Each pin is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign, an off-by-one index, a
transposed operand, a missing diagonal division) fails at least one of them.
"""

from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth


def exact_int_inverse_check(L_int, X):
    """L X == I in exact Python integer arithmetic (X must be integral)."""
    n = L_int.shape[0]
    Xi = [[int(v) for v in row] for row in X]
    Li = [[int(v) for v in row] for row in L_int]
    for i in range(n):
        for j in range(n):
            s = sum(Li[i][k] * Xi[k][j] for k in range(n))
            assert s == (1 if i == j else 0), (i, j, s)


# ---------------------------------------------------------------- worked example
def test_paper_4x4_example_exact(golden):
    """Section 3 worked example: T^{-1} printed as exact integers."""
    g = golden("combinatorix_4x4.txt")
    T, S = g["T"], g["S"]
    L = T.T.copy()  # lower by transposition (eq. defT remark)
    X = oracle.tril_inverse(L, unit=True)
    np.testing.assert_array_equal(X, S.T)
    Xn = oracle.tril_inverse(L, unit=False)  # diagonal is 1 anyway
    np.testing.assert_array_equal(Xn, S.T)
    Xc = oracle.chain_sum_inverse(L, unit=True)
    np.testing.assert_array_equal(Xc, S.T)


def test_hopscotch_listing_h15(golden):
    """Example examplek15: H(1,5) has the 8 listed chains; the count is 2^(5-1-1)."""
    seqs = golden("hopscotch_h15.txt")
    assert len(seqs) == 8 == oracle.chain_count(1, 5)
    assert len({tuple(s) for s in seqs}) == 8
    for s in seqs:
        assert s[0] == 1 and s[-1] == 5 and all(a < b for a, b in zip(s, s[1:]))


@pytest.mark.parametrize("a,b", [(1, 2), (1, 3), (2, 7), (5, 8), (3, 15)])
def test_chain_count_closed_form(a, b):
    """Proposition corrTranlation: |H(a,b)| = 2^(b-a-1); Corollary Translation:
    the count depends on b - a only."""
    assert oracle.chain_count(a, b) == 2 ** (b - a - 1)
    assert oracle.chain_count(a + 4, b + 4) == oracle.chain_count(a, b)


def test_chain_sum_matches_listed_sequences(golden):
    """S_15 of a 5x5 unit upper T from the eight listed chains of H(1,5), with
    sign (-1)^(len-1) and the product over consecutive chain pairs
    (Theorem Combinatorix), against the oracle's enumeration."""
    seqs = golden("hopscotch_h15.txt")
    rng = np.random.default_rng(11)
    T = np.triu(rng.integers(-4, 5, size=(5, 5)).astype(np.float64), 1) + np.eye(5)
    s15 = 0.0
    for s in seqs:
        p = 1.0
        for a, b in zip(s, s[1:]):
            p *= T[a - 1, b - 1]
        s15 += (-1.0) ** (len(s) - 1) * p
    X = oracle.chain_sum_inverse(T.T.copy(), unit=True)
    assert X[4, 0] == s15
    assert s15 == np.linalg.inv(T)[0, 4].round()


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("unit", [False, True])
def test_chain_sum_vs_recurrence(n, unit):
    """Theorem Combinatorix by enumeration (n <= 8) against the recurrence."""
    L = synth.lower_triangular(n, seed=100 + n)
    L[np.tril_indices(n, -1)] *= n  # O(1) off-diagonals so every chain matters
    Xr = oracle.tril_inverse(L, unit=unit)
    Xc = oracle.chain_sum_inverse(L, unit=unit)
    np.testing.assert_allclose(Xc, Xr, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [4, 7])
def test_chain_sum_exact_rational(n):
    """Integer non-unit input: chain sum equals the exact rational inverse."""
    rng = np.random.default_rng(n)
    L = np.tril(rng.integers(-3, 4, size=(n, n)), -1).astype(np.float64)
    d = rng.choice([-2, -1, 1, 2, 4], size=n).astype(np.float64)
    L[np.arange(n), np.arange(n)] = d
    # exact inverse by Fraction forward substitution of L x = e_j
    exact = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):
        x = [Fraction(0)] * n
        for i in range(n):
            rhs = Fraction(1 if i == j else 0) - sum(Fraction(int(L[i, k])) * x[k] for k in range(i))
            x[i] = rhs / Fraction(int(L[i, i]))
        for i in range(n):
            exact[i][j] = x[i]
    Xc = oracle.chain_sum_inverse(L)
    Xr = oracle.tril_inverse(L)
    ex = np.array([[float(v) for v in row] for row in exact])
    np.testing.assert_allclose(Xc, ex, rtol=1e-15, atol=0)
    np.testing.assert_allclose(Xr, ex, rtol=1e-15, atol=0)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 9, 64, 300])
def test_minus_one_bidiagonal_gives_all_ones(n):
    """Unit bidiagonal with -1 sub-diagonal: inverse is the all-ones lower triangle."""
    L = np.eye(n)
    L[np.arange(1, n), np.arange(n - 1)] = -1.0
    X = oracle.tril_inverse(L)
    np.testing.assert_array_equal(X, np.tril(np.ones((n, n))))
    if n <= 9:
        np.testing.assert_array_equal(oracle.chain_sum_inverse(L), np.tril(np.ones((n, n))))


@pytest.mark.parametrize("n", [3, 10, 40])
def test_all_minus_one_gives_powers_of_two(n):
    """Strict lower all -1: X_ij = 2^(i-j-1) for i > j (one per chain, all signs +)."""
    L = np.eye(n) - np.tril(np.ones((n, n)), -1)
    X = oracle.tril_inverse(L, unit=True)
    i, j = np.indices((n, n))
    expect = np.where(i > j, 2.0 ** (i - j - 1), np.where(i == j, 1.0, 0.0))
    np.testing.assert_array_equal(X, expect)
    if n <= 10:
        np.testing.assert_array_equal(oracle.chain_sum_inverse(L, unit=True), expect)


@pytest.mark.parametrize("a,n", [(0.5, 60), (3.0, 20), (-2.0, 30)])
def test_geometric_bidiagonal(a, n):
    """L = I - a * subdiag: X_ij = a^(i-j)."""
    L = np.eye(n)
    L[np.arange(1, n), np.arange(n - 1)] = -a
    X = oracle.tril_inverse(L)
    i, j = np.indices((n, n))
    expect = np.where(i >= j, a ** np.maximum(i - j, 0), 0.0)
    np.testing.assert_array_equal(X, expect)


def test_toeplitz_preserved():
    """Corollary Translation: chain sets of each diagonal band are shifts of
    each other, so a Toeplitz lower matrix has a Toeplitz inverse."""
    n = 48
    c = synth.uniform01(5, np.arange(n)) - 0.5
    c[0] = 1.5
    i, j = np.indices((n, n))
    L = np.where(i >= j, c[np.clip(i - j, 0, n - 1)], 0.0)
    X = oracle.tril_inverse(L)
    for k in range(n):
        band = np.diagonal(X, offset=-k)
        np.testing.assert_allclose(band, band[0], rtol=1e-12, atol=1e-15)


def test_integer_closure_exact():
    """Corollary after the worked example: integer unit lower -> integer inverse."""
    n = 14
    L = synth.integer_unit_lower(n, seed=9)
    X = oracle.tril_inverse(L, unit=True)
    assert np.all(X == np.round(X))
    assert np.max(np.abs(X)) < 2.0 ** 50
    exact_int_inverse_check(L, X)


# ---------------------------------------------------------------- library special case
@pytest.mark.parametrize("n,seed", [(64, 1), (200, 2), (257, 3)])
def test_matches_scipy_triangular_solve(n, seed):
    L = synth.lower_triangular(n, seed)
    X = oracle.tril_inverse(L)
    ref = scipy.linalg.solve_triangular(L, np.eye(n), lower=True)
    np.testing.assert_allclose(X, ref, rtol=1e-12, atol=1e-15)


def test_unit_flag_ignores_stored_diagonal():
    n = 50
    L = synth.lower_triangular(n, 4)
    Lu = L.copy()
    Lu[np.arange(n), np.arange(n)] = 1.0
    ref = scipy.linalg.solve_triangular(Lu, np.eye(n), lower=True, unit_diagonal=True)
    np.testing.assert_allclose(oracle.tril_inverse(L, unit=True), ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- invariants
def test_invariants():
    n = 300
    L = synth.lower_triangular(n, 1)
    X = oracle.tril_inverse(L)
    assert np.all(np.triu(X, 1) == 0.0)
    np.testing.assert_array_equal(np.diag(X), 1.0 / np.diag(L))
    r = oracle.residuals(L, X)
    assert r["rel_lx"] < 1e-16 * 10 and r["rel_xl"] < 1e-16 * 10
    # numpy's own product as an outside check of both residual directions
    I = np.eye(n)
    assert np.linalg.norm(L @ X - I) / (np.linalg.norm(L) * np.linalg.norm(X)) < 1e-15
    assert np.linalg.norm(X @ L - I) / (np.linalg.norm(L) * np.linalg.norm(X)) < 1e-15


def test_principal_blocks_bitwise():
    """X[:k,:k] = inv(L[:k,:k]) and X[k:,k:] = inv(L[k:,k:]) exactly: each entry
    only uses entries of L inside the block."""
    n = 70
    L = synth.lower_triangular(n, 6)
    X = oracle.tril_inverse(L)
    for k in (1, 17, 35, 69):
        np.testing.assert_array_equal(X[:k, :k], oracle.tril_inverse(L[:k, :k]))
        np.testing.assert_array_equal(X[k:, k:], oracle.tril_inverse(L[k:, k:]))


def test_power_of_two_scaling_bitwise():
    n = 64
    L = synth.lower_triangular(n, 7)
    X = oracle.tril_inverse(L)
    np.testing.assert_array_equal(oracle.tril_inverse(L * 8.0), X / 8.0)


def test_upper_garbage_ignored():
    n = 90
    L = synth.lower_triangular(n, 8)
    Lg = synth.lower_triangular(n, 8, upper_garbage=True)
    assert np.any(np.triu(Lg, 1) != 0)
    np.testing.assert_array_equal(oracle.tril_inverse(Lg), oracle.tril_inverse(L))


def test_columns_match_full():
    n = 120
    L = synth.lower_triangular(n, 9)
    X = oracle.tril_inverse(L)
    cols = [0, 1, 59, 119]
    np.testing.assert_array_equal(oracle.tril_inverse_columns(L, cols), X[:, cols])


def test_singular_reports_first_zero_diagonal():
    n = 20
    L = synth.lower_triangular(n, 10)
    L[5, 5] = 0.0
    L[12, 12] = 0.0
    with pytest.raises(oracle.SingularMatrix) as e:
        oracle.tril_inverse(L)
    assert e.value.index == 6
    # unit flag: the stored diagonal is not read, so no error
    oracle.tril_inverse(L, unit=True)


# ---------------------------------------------------------------- residual metric
def test_residual_planted_perturbation():
    """X = exact inverse + delta e_p e_q^T: ||LX - I||_F = |delta| ||L(:,p)||_2 and
    ||XL - I||_F = |delta| ||L(q,:)||_2."""
    n = 12
    L = synth.integer_unit_lower(n, seed=3)
    X = oracle.tril_inverse(L, unit=True)
    r0 = oracle.residuals(L, X)
    assert r0["lx"] == 0.0 and r0["xl"] == 0.0
    p, q, delta = 7, 2, 2.0 ** -10
    Xp = X.copy()
    Xp[p, q] += delta
    r = oracle.residuals(L, Xp)
    assert r["lx"] == pytest.approx(delta * np.linalg.norm(L[:, p]), rel=1e-12)
    assert r["xl"] == pytest.approx(delta * np.linalg.norm(L[q, :]), rel=1e-12)
    # a non-zero in the strict upper part of X is seen as well
    Xu = X.copy()
    Xu[1, 5] = delta
    assert oracle.residuals(L, Xu)["lx"] == pytest.approx(delta * np.linalg.norm(L[:, 1]), rel=1e-12)
    cols = oracle.residual_columns(L, Xp, np.arange(n))
    assert np.sqrt(cols.sum()) == pytest.approx(r["lx"], rel=1e-12)
    assert cols[q] == pytest.approx(r["lx"] ** 2, rel=1e-12)


def test_residual_matrix_planted_integer_perturbation():
    """R = I - L X entry by entry: exactly zero for an integer unit lower L
    and its exact integer inverse; for X + E with E an integer matrix (lower
    and upper entries), exactly -L E, which a pure-Python triple loop over
    tril(L) gives in integers. A transposed operand, a dropped diagonal term,
    a sign error or reading triu(L) fails it."""
    n = 11
    L = synth.integer_unit_lower(n, seed=5)
    L_full = L.copy()
    L_full[np.triu_indices(n, 1)] = 7.0  # garbage above the diagonal: must be ignored
    X = oracle.tril_inverse(L, unit=True)
    np.testing.assert_array_equal(oracle.residual_matrix(L_full, X), np.zeros((n, n)))
    rng = np.random.default_rng(4)
    E = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
    R = oracle.residual_matrix(L_full, X + E)
    Li = [[int(L[i, k]) if k <= i else 0 for k in range(n)] for i in range(n)]
    Ei = [[int(v) for v in row] for row in E]
    want = [[-sum(Li[i][k] * Ei[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    np.testing.assert_array_equal(R, np.array(want, dtype=np.float64))
    # its Frobenius norm is the residual metric's
    assert np.linalg.norm(R) == pytest.approx(oracle.residuals(L_full, X + E)["lx"], rel=1e-14)


# ---------------------------------------------------------------- factored inverse
def test_skul_printed_example(golden):
    """Section 6: from the printed L and U, K = L^{-1} and S = U^{-1} match the
    printed values to the four printed decimals; A * (S K) = I to the precision
    of the printed A."""
    g = golden("skul_5x5.txt")
    A, U, L, S, K = g["A"], g["U"], g["L"], g["S"], g["K"]
    np.testing.assert_allclose(L @ U, A, atol=2e-4)  # fixture sanity: L U = A
    Linv, Uinv, Ainv = oracle.factored_inverse(L, U, l_unit=False, u_unit=True)
    np.testing.assert_allclose(Linv, K, atol=1e-4)
    np.testing.assert_allclose(Uinv, S, atol=1e-4)
    np.testing.assert_allclose(A @ Ainv, np.eye(5), atol=1e-3)
    np.testing.assert_allclose(Ainv, S @ K, atol=2e-4)


def test_factored_inverse_identities():
    n = 80
    L = synth.lower_triangular(n, 3, unit=True)
    U = synth.upper_triangular(n, 4)
    Linv, Uinv, Ainv = oracle.factored_inverse(L, U, l_unit=True, u_unit=False)
    I = np.eye(n)
    assert np.max(np.abs(L @ Linv - I)) < 1e-14
    assert np.max(np.abs(U @ Uinv - I)) < 1e-14
    assert np.all(np.tril(Uinv, -1) == 0) and np.all(np.triu(Linv, 1) == 0)
    assert np.max(np.abs((L @ U) @ Ainv - I)) < 1e-13
    np.testing.assert_allclose(Uinv, scipy.linalg.solve_triangular(U, I, lower=False), rtol=1e-12,
                               atol=1e-15)


# ---------------------------------------------------------------- gradient
def _loss(L, W):
    return float(np.sum(W * oracle.tril_inverse(L)))


def test_backward_finite_differences():
    """grad of f(L) = sum(W .* L^{-1}) against FP64 central differences, h = 1e-6."""
    n = 16
    L = synth.lower_triangular(n, 7)
    W = synth.normal(n, n, seed=7)
    g = oracle.tril_inverse_backward(L, W)
    h = 1e-6
    fd = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            Lp = L.copy()
            Lm = L.copy()
            Lp[i, j] += h
            Lm[i, j] -= h
            fd[i, j] = (_loss(Lp, W) - _loss(Lm, W)) / (2 * h)
    assert np.all(np.triu(g, 1) == 0)
    assert np.linalg.norm(fd - g) / np.linalg.norm(g) < 1e-7


def test_backward_closed_forms():
    # 1x1: d(w / l)/dl = -w / l^2
    g = oracle.tril_inverse_backward(np.array([[2.0]]), np.array([[3.0]]))
    assert g[0, 0] == -3.0 / 4.0
    # 2x2: X = [[1/a, 0], [-c/(ab), 1/b]]
    a, c, b = 1.5, 0.25, -2.0
    w11, w12, w21, w22 = 0.5, 9.0, -1.25, 2.0
    L = np.array([[a, 0.0], [c, b]])
    W = np.array([[w11, w12], [w21, w22]])
    g = oracle.tril_inverse_backward(L, W)
    np.testing.assert_allclose(g[0, 0], -w11 / a**2 + w21 * c / (a**2 * b), rtol=1e-15)
    np.testing.assert_allclose(g[1, 0], -w21 / (a * b), rtol=1e-15)
    np.testing.assert_allclose(g[1, 1], -w22 / b**2 + w21 * c / (a * b**2), rtol=1e-15)
    assert g[0, 1] == 0.0


def test_backward_linear_in_g_and_rows():
    n = 24
    L = synth.lower_triangular(n, 12)
    G1 = synth.normal(n, n, 1)
    G2 = synth.normal(n, n, 2)
    g = oracle.tril_inverse_backward(L, G1 + 2.0 * G2)
    np.testing.assert_allclose(g, oracle.tril_inverse_backward(L, G1) + 2.0 * oracle.tril_inverse_backward(L, G2),
                               rtol=1e-12, atol=1e-13)
    # only tril(G) matters (X lower => the strict upper of G drops out)
    np.testing.assert_allclose(oracle.tril_inverse_backward(L, np.tril(G1)), oracle.tril_inverse_backward(L, G1),
                               rtol=1e-12, atol=1e-14)
    rows = [0, 5, 23]
    np.testing.assert_array_equal(oracle.tril_inverse_backward_rows(L, G1, rows),
                                  oracle.tril_inverse_backward(L, G1)[rows])


# ---------------------------------------------------------------- SKUL factorization


def test_crout_printed_example(golden):
    """Section 6: the Crout factors of the printed A are the printed L and U
    (four decimals), and the whole SKUL output reproduces the printed S, K."""
    g = golden("skul_5x5.txt")
    L, U, S, K, Ainv = oracle.skul(g["A"])
    np.testing.assert_allclose(L, g["L"], atol=1.5e-4)
    np.testing.assert_allclose(U, g["U"], atol=1.5e-4)
    np.testing.assert_allclose(S, g["S"], atol=1.5e-4)
    np.testing.assert_allclose(K, g["K"], atol=1.5e-4)
    np.testing.assert_allclose(g["A"] @ Ainv, np.eye(5), atol=1e-12)


def test_crout_integer_factors_exact():
    """A = L0 U0 with integer L0 (diagonal +-1) and integer unit-upper U0:
    every step of the recurrence is exact, so the factors come back bitwise."""
    rng = np.random.default_rng(11)
    n = 12
    L0 = np.tril(rng.integers(-3, 4, (n, n)), -1).astype(float) + np.diag(rng.choice([-1.0, 1.0], n))
    U0 = np.triu(rng.integers(-3, 4, (n, n)), 1).astype(float) + np.eye(n)
    L, U = oracle.crout_lu(L0 @ U0)
    np.testing.assert_array_equal(L, L0)
    np.testing.assert_array_equal(U, U0)


def test_crout_matches_scipy_lu():
    """For a column diagonally dominant matrix partial pivoting never swaps, so
    scipy's A = P L1 U1 (unit lower L1) has P = I, and the Crout factors are
    L = L1 diag(U1), U = diag(U1)^{-1} U1."""
    import scipy.linalg as sl

    rng = np.random.default_rng(3)
    n = 40
    A = rng.uniform(-1, 1, (n, n))
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=0) + 1.0
    P, L1, U1 = sl.lu(A)
    np.testing.assert_array_equal(P, np.eye(n))
    d = np.diag(U1)
    L, U = oracle.crout_lu(A)
    np.testing.assert_allclose(L, L1 * d[None, :], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(U, U1 / d[:, None], rtol=1e-12, atol=1e-13)


def test_crout_invariants_and_zero_pivot():
    rng = np.random.default_rng(4)
    n = 60
    A = rng.uniform(-1, 1, (n, n)) + n * np.eye(n)
    L, U = oracle.crout_lu(A)
    assert np.all(np.triu(L, 1) == 0) and np.all(np.tril(U, -1) == 0) and np.all(np.diag(U) == 1.0)
    np.testing.assert_allclose(L @ U, A, rtol=0, atol=1e-12 * np.abs(A).max())
    with pytest.raises(oracle.SingularMatrix) as e:
        oracle.crout_lu(np.array([[0.0, 1.0], [1.0, 1.0]]))
    assert e.value.index == 1
    with pytest.raises(oracle.SingularMatrix) as e:  # second pivot 1 - 1 * 1 = 0
        oracle.crout_lu(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 2.0], [0.0, 3.0, 1.0]]))
    assert e.value.index == 2


# ---------------------------------------------------------------- SQR
def test_sqr_printed_example(golden):
    """Section 6: the SQR factors Q, R, S and Q^T of the printed 5x5 matrix,
    to the four printed decimals (the printed A is itself rounded, so the
    last printed digit may differ by one)."""
    g = golden("sqr_5x5.txt")
    np.testing.assert_allclose(g["QT"], g["Q"].T, atol=0)  # fixture sanity
    Q, R, S, Ainv = oracle.sqr(g["A"])
    np.testing.assert_allclose(Q, g["Q"], atol=2e-4)
    np.testing.assert_allclose(R, g["R"], atol=2e-4)
    np.testing.assert_allclose(S, g["S"], atol=2e-4)
    np.testing.assert_allclose(Ainv, g["S"] @ g["QT"], atol=5e-4)
    np.testing.assert_allclose(g["A"] @ Ainv, np.eye(5), atol=1e-12)


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (7, 3), (60, 4), (200, 5)])
def test_sqr_matches_householder_qr(n, seed):
    """Against numpy's Householder QR (an independent algorithm) after the
    sign normalisation R(j, j) > 0 that makes the QR factors unique."""
    A = synth.normal(n, n, seed) / np.sqrt(n) + 2.0 * np.eye(n)
    Q, R, S, Ainv = oracle.sqr(A)
    Qh, Rh = np.linalg.qr(A)
    sg = np.sign(np.diag(Rh))
    Qh, Rh = Qh * sg, (Rh.T * sg).T
    cond = np.linalg.cond(A)
    tol = 1e-13 * cond * max(n, 1)
    np.testing.assert_allclose(Q, Qh, atol=tol)
    np.testing.assert_allclose(R, Rh, atol=tol * np.abs(Rh).max())
    assert np.all(np.tril(R, -1) == 0) and np.all(np.tril(S, -1) == 0)
    assert np.all(np.diag(R) > 0)
    I = np.eye(n)
    assert np.abs(Q.T @ Q - I).max() < tol
    assert np.abs(S @ R - I).max() < 1e-13 * cond
    # S Q^T A - I = S (Q^T Q - I) R: the loss of orthogonality times cond(R)
    assert np.abs(Ainv @ A - I).max() < 1e-13 * cond * cond
    np.testing.assert_allclose(S, np.linalg.inv(Rh), atol=tol * np.abs(S).max())


def test_sqr_upper_input_is_exact():
    """For upper triangular A with a positive power-of-two diagonal,
    Gram-Schmidt meets orthogonal columns e_1, e_2, ... and every norm and
    reciprocal is exact: Q = I and R = A exactly, and S is the triangular
    inverse of A (checked against the column recurrence applied to A^T)."""
    n = 40
    A = synth.upper_triangular(n, 9)
    A[np.arange(n), np.arange(n)] = 2.0 ** (np.arange(n) % 5 - 2)
    Q, R, S, _ = oracle.sqr(A)
    assert np.array_equal(Q, np.eye(n))
    assert np.array_equal(R, A)
    np.testing.assert_allclose(S, oracle.tril_inverse(A.T).T, rtol=1e-13, atol=1e-15)


def test_sqr_zero_column_reports_index():
    A = synth.normal(6, 6, 7)
    A[:, 3] = 0.0
    with pytest.raises(oracle.SingularMatrix) as e:
        oracle.sqr(A)
    assert e.value.index == 4
    B = synth.normal(6, 6, 8)
    B[:, 4] = B[:, 1] * 2.0  # dependent column: its residual is (numerically) zero only by luck
    Q, R, S, _ = oracle.sqr(B)
    assert abs(R[4, 4]) < 1e-12 * np.abs(R).max()


# ---------------------------------------------------------------- general inverse
def test_inverse_closed_forms():
    a, b, c, d = 3.0, -2.0, 5.0, 7.0
    X = oracle.inverse(np.array([[a, b], [c, d]]))
    det = a * d - b * c
    np.testing.assert_allclose(X, np.array([[d, -b], [-c, a]]) / det, rtol=1e-15)
    P = np.eye(9)[[3, 0, 8, 1, 7, 2, 6, 4, 5]]
    assert np.array_equal(oracle.inverse(P), P.T)
    D = np.diag(2.0 ** np.arange(-4, 5))
    assert np.array_equal(oracle.inverse(D), np.diag(2.0 ** -np.arange(-4, 5)))


@pytest.mark.parametrize("n,seed", [(1, 1), (5, 2), (64, 3), (257, 4)])
def test_inverse_matches_lapack(n, seed):
    A = synth.normal(n, n, seed)
    X = oracle.inverse(A)
    cond = np.linalg.cond(A)
    np.testing.assert_allclose(X, np.linalg.inv(A), atol=1e-14 * cond * np.abs(X).max())
    assert np.abs(A @ X - np.eye(n)).max() < 1e-14 * cond * n


def test_inverse_singular_reports_column():
    A = synth.normal(5, 5, 3)
    A[2] = A[0] + A[1]
    A[:, 4] = 0.0
    with pytest.raises(oracle.SingularMatrix) as e:
        oracle.inverse(A)
    assert e.value.index == 5


# ---------------------------------------------------------------- BRSI (gamma = 2)
@pytest.mark.parametrize("n,base", [(2, 1), (3, 1), (17, 4), (64, 8), (130, 16), (300, 64)])
def test_brsi_matches_inverse(n, base):
    A = synth.diag_dominant(n, 30 + n)
    X = oracle.brsi(A, base)
    np.testing.assert_allclose(X, oracle.inverse(A), atol=1e-13)
    assert np.abs(A @ X - np.eye(n)).max() < 1e-13


def test_brsi_2x2_closed_form():
    a, b, c, d = 4.0, 1.0, -2.0, 3.0
    X = oracle.brsi(np.array([[a, b], [c, d]]), base=1)
    np.testing.assert_allclose(X, np.array([[d, -b], [-c, a]]) / (a * d - b * c), rtol=1e-15)


def test_brsi_block_upper_input():
    """A21 = 0: W = I and the inverse is the block triangular inverse
    [[S11, -S11 A12 S22], [0, S22]] with an exactly zero lower block."""
    n, h = 96, 48
    A = synth.diag_dominant(n, 41)
    A[h:, :h] = 0.0
    X = oracle.brsi(A, base=16)
    assert np.all(X[h:, :h] == 0.0)
    S11 = oracle.inverse(A[:h, :h])
    S22 = oracle.inverse(A[h:, h:])
    np.testing.assert_allclose(X[:h, :h], S11, atol=1e-14)
    np.testing.assert_allclose(X[h:, h:], S22, atol=1e-14)
    np.testing.assert_allclose(X[:h, h:], -S11 @ A[:h, h:] @ S22, atol=1e-14)


def test_brsi_split_factorization():
    """Steps of BRSI with gamma = 2: A = U0 U1 L with U0 block upper, U1 block
    diagonal, L unit block lower, and S = U0^{-1}."""
    n, h = 80, 40
    A = synth.diag_dominant(n, 43)
    U0, U1, Lb, S = oracle.brsi_split(A)
    assert np.all(U0[h:, :h] == 0) and np.all(U1[h:, :h] == 0) and np.all(U1[:h, h:] == 0)
    assert np.all(Lb[:h, h:] == 0)
    np.testing.assert_allclose(np.diag(Lb), 1.0, atol=1e-15)
    np.testing.assert_allclose(U0 @ S, np.eye(n), atol=1e-14)
    np.testing.assert_allclose(U0 @ U1 @ Lb, A, atol=1e-14)
    np.testing.assert_allclose(oracle.inverse(Lb) @ oracle.inverse(U1) @ S, oracle.brsi(A, 8), atol=1e-13)
