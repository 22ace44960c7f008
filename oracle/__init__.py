"""CPU FP64 oracle for the triangular-inverse engine (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never imports, links or calls it, and
this package imports nothing from the GPU library: the two share only the
seeded input generators of the ``synth`` package.

The arithmetic lives in ``oracle.c`` (plain FP64 C, built by ``build.py`` in
this directory); this module marshals numpy arrays to it.

What each function follows, and what pins it (tests/test_oracle_pins.py):

* ``tril_inverse`` -- column recurrence CRIT (Section 4.2), transposed to the
  lower case. Pinned by: the worked 4x4 example of Section 3 (exact integers);
  the chain-sum theorem by brute force (n <= 8); the closed forms
  (-1 sub-diagonal -> all-ones lower; all -1 strict lower -> 2^(i-j-1);
  a-bidiagonal -> a^(i-j)); Toeplitz preservation (Corollary Translation);
  integer closure (Corollary after the worked example) checked in exact
  integer arithmetic; scipy's triangular solve on random inputs;
  L X = X L = I, tril(X) = X, X_ii = 1/L_ii bitwise, the principal-block
  property and power-of-two scaling equivariance.
* ``chain_sum_inverse`` -- Theorem Combinatorix (Section 3) by enumeration of
  the Hopscotch series. Pinned by the worked 4x4 example, by the chain count
  2^(b-a-1) (Proposition corrTranlation) and the H(1,5) listing, by exact
  rational arithmetic on integer inputs, and by agreement with the
  recurrence (an independent derivation).
* ``crout_lu`` / ``skul`` -- the Crout factorization steps of SKUL (Section 5;
  L lower, U unit upper, no pivoting), then ``factored_inverse``. Pinned by
  the printed 5x5 example of Section 6 (L, U, S, K), exact recovery of integer
  factors with unit-modulus pivots, agreement with scipy's LU (partial
  pivoting is the identity for column diagonally dominant matrices) after the
  Crout rescaling, L U = A, and zero pivots reported by index.
* ``factored_inverse`` -- the output statement of SKUL (Section 5): S K =
  A^{-1} with S = U^{-1}, K = L^{-1}. Pinned by the printed 5x5 example of
  Section 6 (L, U, S, K to four decimals) and by A * Ainv = I.
* ``sqr`` -- algorithm SQR (Section 5): modified Gram-Schmidt with S = R^{-1}
  grown column by column (the column of S uses R(j, j) of the same column),
  S = D S' at the end. Pinned by the printed 5x5 example of Section 6 (Q, R,
  S, Q^T to four decimals), agreement with numpy's Householder QR after the
  sign normalisation R(j, j) > 0, exact Q = I, R = A for an upper triangular
  input with positive diagonal, Q^T Q = I, S R = I, S Q^T A = I, and a zero
  column reported by index.
* ``inverse`` -- the textbook definition of A^{-1} (Gauss-Jordan with partial
  pivoting). Pinned by numpy's LAPACK inverse, the 2x2 closed form, exact
  inverses of permutation and diagonal power-of-two matrices, A X = I and a
  singular input reported by column.
* ``brsi`` / ``brsi_split`` -- BRSI with gamma = 2 (Section 5, Steps of BRSI
  and the gamma = 2 derivation). Pinned by agreement with ``inverse`` (odd
  and even orders, several recursion depths), the block upper triangular case
  (A21 = 0 gives X21 = 0 exactly and the triangular blocks), the 2x2 closed
  form, and the factorization A = U0 U1 L of the Steps.
* ``tril_inverse_backward`` -- grad = -tril(X^T G X^T), derived from
  dX = -X dL X (not in the paper). Pinned by FP64 central finite differences
  at n = 16, the 1x1 and 2x2 closed forms, and linearity in G.
* ``residuals`` -- ||LX - I||_F, ||XL - I||_F, ||L||_F, ||X||_F. Pinned by a
  planted perturbation whose residual has a closed form.
* ``residual_matrix`` -- R = I - L X entry by entry. Pinned by exact zeros
  for an integer matrix and its exact integer inverse, and by a planted
  integer perturbation E of that inverse, whose residual is exactly -L E
  (checked against a pure-Python triple loop in integers).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # compile on first use (plain gcc, seconds)
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_tril_inverse.argtypes = [_i64, _dp, _i64, _i32, _dp, _i64]
    lib.oracle_tril_inverse.restype = _i64
    lib.oracle_tril_inverse_columns.argtypes = [_i64, _dp, _i64, _i32, _lp, _i64, _dp]
    lib.oracle_tril_inverse_columns.restype = _i64
    lib.oracle_chain_sum_inverse.argtypes = [_i64, _dp, _i64, _i32, _dp, _i64]
    lib.oracle_chain_sum_inverse.restype = _i64
    lib.oracle_chain_count.argtypes = [_i64, _i64]
    lib.oracle_chain_count.restype = _i64
    lib.oracle_crout_lu.argtypes = [_i64, _dp, _i64, _dp, _dp]
    lib.oracle_crout_lu.restype = _i64
    lib.oracle_factored_inverse.argtypes = [_i64, _dp, _i64, _i32, _dp, _i64, _i32, _dp, _dp, _dp]
    lib.oracle_factored_inverse.restype = _i64
    lib.oracle_tril_inverse_backward.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp]
    lib.oracle_tril_inverse_backward.restype = _i64
    lib.oracle_tril_inverse_backward_rows.argtypes = [_i64, _dp, _i64, _dp, _i64, _lp, _i64, _dp]
    lib.oracle_tril_inverse_backward_rows.restype = _i64
    lib.oracle_residuals.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp]
    lib.oracle_residuals.restype = None
    lib.oracle_residual_matrix.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp]
    lib.oracle_residual_matrix.restype = None
    lib.oracle_residual_columns.argtypes = [_i64, _dp, _i64, _dp, _i64, _lp, _i64, _dp]
    lib.oracle_residual_columns.restype = None
    lib.oracle_sqr.argtypes = [_i64, _dp, _i64, _dp, _dp, _dp]
    lib.oracle_sqr.restype = _i64
    lib.oracle_inverse.argtypes = [_i64, _dp, _i64, _dp]
    lib.oracle_inverse.restype = _i64
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = _i32
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp)


class SingularMatrix(ValueError):
    """Raised with the 1-based index of the first zero diagonal entry."""

    def __init__(self, index: int):
        super().__init__(f"zero diagonal entry at (1-based) index {index}")
        self.index = index


def tril_inverse(L, unit: bool = False) -> np.ndarray:
    """X = L^{-1} in FP64 by the column recurrence; only tril(L) is read."""
    L = _f64(L)
    n = L.shape[0]
    X = np.empty((n, n), dtype=np.float64)
    bad = _load().oracle_tril_inverse(n, _p(L), n, int(unit), _p(X), n)
    if bad:
        raise SingularMatrix(int(bad))
    return X


def tril_inverse_columns(L, cols, unit: bool = False) -> np.ndarray:
    """Columns ``cols`` of L^{-1}, returned as an n x len(cols) array."""
    L = _f64(L)
    n = L.shape[0]
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty((len(cols), n), dtype=np.float64)
    bad = _load().oracle_tril_inverse_columns(n, _p(L), n, int(unit), cols.ctypes.data_as(_lp),
                                              len(cols), _p(out))
    if bad:
        raise SingularMatrix(int(bad))
    return out.T.copy()


def chain_sum_inverse(L, unit: bool = False) -> np.ndarray:
    """L^{-1} by brute-force enumeration of Theorem Combinatorix (n <= 20)."""
    L = _f64(L)
    n = L.shape[0]
    if n > 20:
        raise ValueError("chain-sum enumeration is exponential; n <= 20 only")
    X = np.empty((n, n), dtype=np.float64)
    bad = _load().oracle_chain_sum_inverse(n, _p(L), n, int(unit), _p(X), n)
    if bad:
        raise SingularMatrix(int(bad))
    return X


def chain_count(a: int, b: int) -> int:
    """|H(a, b)| counted by enumerating the chains."""
    return int(_load().oracle_chain_count(a, b))


def factored_inverse(L, U, l_unit: bool = False, u_unit: bool = False, want_ainv: bool = True):
    """(Linv, Uinv, Ainv) from lower L and upper U with A = L U."""
    L = _f64(L)
    U = _f64(U)
    n = L.shape[0]
    Linv = np.empty((n, n))
    Uinv = np.empty((n, n))
    Ainv = np.empty((n, n)) if want_ainv else None
    bad = _load().oracle_factored_inverse(n, _p(L), n, int(l_unit), _p(U), n, int(u_unit), _p(Linv),
                                          _p(Uinv), _p(Ainv) if want_ainv else None)
    if bad:
        raise SingularMatrix(int(abs(bad)))
    return Linv, Uinv, Ainv


def crout_lu(A):
    """(L, U) with A = L U, L lower, U unit upper, no pivoting (the
    factorization steps of algorithm SKUL)."""
    A = _f64(A)
    n = A.shape[0]
    L = np.empty((n, n))
    U = np.empty((n, n))
    bad = _load().oracle_crout_lu(n, _p(A), n, _p(L), _p(U))
    if bad:
        raise SingularMatrix(int(bad))
    return L, U


def skul(A, want_ainv: bool = True):
    """Algorithm SKUL's outputs (L, U, S, K, Ainv): L U = A, S = U^{-1},
    K = L^{-1}, Ainv = S K (None if not wanted)."""
    L, U = crout_lu(A)
    K, S, Ainv = factored_inverse(L, U, l_unit=False, u_unit=True, want_ainv=want_ainv)
    return L, U, S, K, Ainv


def sqr(A, want_ainv: bool = True):
    """Algorithm SQR's outputs (Q, R, S, Ainv): modified Gram-Schmidt
    A = Q R with S = R^{-1} grown column by column, Ainv = S Q^T (a plain
    matrix product; None if not wanted)."""
    A = _f64(A)
    n = A.shape[0]
    Q = np.empty((n, n))
    R = np.empty((n, n))
    S = np.empty((n, n))
    bad = _load().oracle_sqr(n, _p(A), n, _p(Q), _p(R), _p(S))
    if bad:
        raise SingularMatrix(int(bad))
    return Q, R, S, (S @ Q.T if want_ainv else None)


def inverse(A) -> np.ndarray:
    """A^{-1} by Gauss-Jordan elimination with partial pivoting."""
    A = _f64(A)
    n = A.shape[0]
    X = np.empty((n, n))
    bad = _load().oracle_inverse(n, _p(A), n, _p(X))
    if bad:
        raise SingularMatrix(int(bad))
    return X


def brsi_split(A):
    """One pass of the gamma = 2 split of BRSI (Section 5, Steps of BRSI and
    the gamma = 2 derivation), for A with invertible diagonal blocks
    (h = n // 2): U0 is the block upper part of A, S = U0^{-1} with blocks
    S11 = A11^{-1}, S22 = A22^{-1}, S12 = -S11 A12 S22; A1 = I + S (A - U0)
    = [[I + S12 A21, 0], [S22 A21, I]]; U1 = diag(I + S12 A21, I) is the
    block upper part of A1 and L = I + U1^{-1} (A1 - U1) = [[I, 0],
    [S22 A21, I]]. Then A = U0 U1 L. Returns (U0, U1, L, S)."""
    A = _f64(A)
    n = A.shape[0]
    h = n // 2
    A11, A12, A21, A22 = A[:h, :h], A[:h, h:], A[h:, :h], A[h:, h:]
    S11 = inverse(A11)
    S22 = inverse(A22)
    S12 = -(S11 @ A12) @ S22
    U0 = A.copy()
    U0[h:, :h] = 0.0
    S = np.zeros((n, n))
    S[:h, :h], S[:h, h:], S[h:, h:] = S11, S12, S22
    A1 = np.eye(n) + S @ (A - U0)
    U1 = A1.copy()
    U1[h:, :h] = 0.0
    U1inv = np.eye(n)
    U1inv[:h, :h] = inverse(A1[:h, :h])
    Lb = np.eye(n) + U1inv @ (A1 - U1)
    return U0, U1, Lb, S


def brsi(A, base: int = 64) -> np.ndarray:
    """A^{-1} by BRSI with gamma = 2 (Section 5, the gamma = 2 derivation):
    with h = n // 2, S11 = A11^{-1}, S22 = A22^{-1} (both by this recursion),
    S12 = -S11 A12 S22, W = (I + S12 A21)^{-1} (by this recursion),
        A^{-1} = [[W S11, W S12], [-S22 A21 W S11, S22 - S22 A21 W S12]].
    Orders <= base are inverted by ``inverse``. No pivoting: the diagonal
    blocks met on the way must be invertible."""
    A = _f64(A)
    n = A.shape[0]
    if n <= base:
        return inverse(A)
    h = n // 2
    A11, A12, A21, A22 = A[:h, :h], A[:h, h:], A[h:, :h], A[h:, h:]
    S11 = brsi(A11, base)
    S22 = brsi(A22, base)
    S12 = -(S11 @ A12) @ S22
    W = brsi(np.eye(h) + S12 @ A21, base)
    T = S22 @ A21
    X = np.empty((n, n))
    X[:h, :h] = W @ S11
    X[:h, h:] = W @ S12
    X[h:, :h] = -T @ X[:h, :h]
    X[h:, h:] = S22 - T @ X[:h, h:]
    return X


def tril_inverse_backward(L, G) -> np.ndarray:
    """-tril(X^T G X^T) with X = L^{-1} computed here from L."""
    L = _f64(L)
    G = _f64(G)
    n = L.shape[0]
    grad = np.empty((n, n))
    bad = _load().oracle_tril_inverse_backward(n, _p(L), n, _p(G), n, _p(grad))
    if bad:
        raise SingularMatrix(int(bad))
    return grad


def tril_inverse_backward_rows(L, G, rows) -> np.ndarray:
    """Rows ``rows`` of -tril(X^T G X^T), as a len(rows) x n array."""
    L = _f64(L)
    G = _f64(G)
    n = L.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), n))
    bad = _load().oracle_tril_inverse_backward_rows(n, _p(L), n, _p(G), n, rows.ctypes.data_as(_lp),
                                                    len(rows), _p(out))
    if bad:
        raise SingularMatrix(int(bad))
    return out


def residuals(L, X) -> dict:
    """Residual norms of candidate X for lower L (tril(L) read, X in full)."""
    L = _f64(L)
    X = _f64(X)
    n = L.shape[0]
    out = np.empty(4)
    _load().oracle_residuals(n, _p(L), n, _p(X), n, _p(out))
    denom = out[2] * out[3]
    return {
        "lx": out[0], "xl": out[1], "norm_l": out[2], "norm_x": out[3],
        "rel_lx": out[0] / denom if denom else 0.0,
        "rel_xl": out[1] / denom if denom else 0.0,
    }


def residual_matrix(L, X) -> np.ndarray:
    """R = I - tril(L) X in FP64 (X read in full)."""
    L = _f64(L)
    X = _f64(X)
    n = L.shape[0]
    out = np.empty((n, n))
    _load().oracle_residual_matrix(n, _p(L), n, _p(X), n, _p(out))
    return out


def residual_columns(L, X, cols) -> np.ndarray:
    """||(L X - I)(:, j)||_2^2 for each j in ``cols``."""
    L = _f64(L)
    X = _f64(X)
    n = L.shape[0]
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(len(cols))
    _load().oracle_residual_columns(n, _p(L), n, _p(X), n, cols.ctypes.data_as(_lp), len(cols), _p(out))
    return out


def num_threads() -> int:
    return int(_load().oracle_num_threads())
