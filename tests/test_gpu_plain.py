"""GPU parity of the plain recursion (FP64 and FP32) against the CPU oracle.

Every case calls the HIP library through its C ABI (via the thin Python
binding) and compares element by element with the oracle on the same seeded
inputs. Tolerances: FP64 results differ from the oracle only in summation
order, so the relative forward error is bounded by a small multiple of
kappa * n * eps (kappa ~ 2 for this generator): 1e-12 is used, and the
relative residual ||LX - I||_F / (||L||_F ||X||_F) must be <= 1e-13. FP32:
forward error <= 1e-5 and residual <= 1e-5. Exact-arithmetic cases (integer
and power-of-two inputs) must match bitwise.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, dev, host, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trinv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07611_amd as P

    P.load()
    return P


def inv(trinv, L, **kw):
    import torch

    X, info = trinv.tril_inverse(L, return_info=True, **kw)
    torch.cuda.synchronize()
    return X, info


# ---------------------------------------------------------------- configuration 1
def test_n256_fp64_leaf32_vs_oracle(trinv):
    banner("plain f64 n=256 leaf=32 seed=1")
    L = synth.lower_triangular(256, 1)
    X, info = inv(trinv, dev(L), leaf=32, check=True)
    Xo = oracle.tril_inverse(L)
    Xg = host(X)
    assert rel_fro(Xg, Xo) < 1e-12
    assert np.max(np.abs(Xg - Xo)) < 1e-12
    assert np.all(np.triu(Xg, 1) == 0.0)
    np.testing.assert_array_equal(np.diag(Xg), 1.0 / np.diag(L))
    r = oracle.residuals(L, Xg)
    assert r["rel_lx"] <= 1e-13 and r["rel_xl"] <= 1e-13
    assert info["rel_residual"] <= 1e-13
    assert abs(info["rel_residual"] - r["rel_lx"]) <= 1e-15


def test_gpu_residual_helper_matches_oracle(trinv):
    banner("residual helper n=300 planted perturbation")
    n = 300
    L = synth.lower_triangular(n, 2)
    Xo = oracle.tril_inverse(L)
    Xo[200, 17] += 1e-6
    r = trinv.residual(dev(L), dev(Xo))
    ro = oracle.residuals(L, Xo)
    assert r["lx"] == pytest.approx(ro["lx"], rel=1e-9)
    assert r["norm_l"] == pytest.approx(ro["norm_l"], rel=1e-13)
    assert r["norm_x"] == pytest.approx(ro["norm_x"], rel=1e-13)


# ---------------------------------------------------------------- exact pins
def test_minus_one_bidiagonal_all_ones_bitwise(trinv):
    for n in (1, 2, 33, 256, 1000):
        banner(f"bidiagonal -1 n={n}")
        L = np.eye(n)
        L[np.arange(1, n), np.arange(n - 1)] = -1.0
        X, _ = inv(trinv, dev(L), leaf=32)
        np.testing.assert_array_equal(host(X), np.tril(np.ones((n, n))))
        X32, _ = inv(trinv, dev(L, __import__("torch").float32))
        np.testing.assert_array_equal(host(X32), np.tril(np.ones((n, n), dtype=np.float32)))


def test_paper_example_and_powers_of_two_bitwise(trinv, golden):
    banner("paper 4x4 example, all -1 n=40")
    g = golden("combinatorix_4x4.txt")
    X, _ = inv(trinv, dev(g["T"].T.copy()), leaf=16)
    np.testing.assert_array_equal(host(X), g["S"].T)
    n = 40
    L = np.eye(n) - np.tril(np.ones((n, n)), -1)
    X, _ = inv(trinv, dev(L), leaf=16)
    i, j = np.indices((n, n))
    np.testing.assert_array_equal(host(X), np.where(i > j, 2.0 ** (i - j - 1), np.where(i == j, 1.0, 0.0)))


def test_integer_closure_bitwise(trinv):
    banner("integer unit lower n=14")
    L = synth.integer_unit_lower(14, seed=9)
    X, _ = inv(trinv, dev(L), leaf=16, unit_diag=True)
    np.testing.assert_array_equal(host(X), oracle.tril_inverse(L, unit=True))


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("n,leaf", [(1, 32), (2, 32), (31, 32), (32, 32), (33, 32), (100, 16), (257, 32),
                                    (300, 64), (513, 128), (640, 32)])
def test_ragged_sizes_fp64(trinv, n, leaf):
    banner(f"ragged f64 n={n} leaf={leaf}")
    L = synth.lower_triangular(n, 10 + n)
    X, _ = inv(trinv, dev(L), leaf=leaf)
    Xg = host(X)
    assert rel_fro(Xg, oracle.tril_inverse(L)) < 1e-12
    assert np.all(np.triu(Xg, 1) == 0.0)


def test_leading_dimension_and_garbage(trinv):
    import torch

    banner("ld > n, garbage in the strict upper part, n=300")
    n, ld = 300, 333
    L = synth.lower_triangular(n, 5, upper_garbage=True)
    big = np.full((n, ld), 7.0)
    big[:, :n] = L
    Lt = dev(big)[:, :n]
    Xbig = torch.full((n, ld), -3.0, dtype=torch.float64, device="cuda")
    X = Xbig[:, :n]
    trinv.tril_inverse(Lt, leaf=32, out=X)
    torch.cuda.synchronize()
    Xh = host(Xbig)
    assert rel_fro(Xh[:, :n], oracle.tril_inverse(L)) < 1e-12
    assert np.all(Xh[:, n:] == -3.0)  # padding untouched
    assert np.all(np.triu(Xh[:, :n], 1) == 0.0)


def test_unit_and_upper_flags(trinv):
    banner("unit_diag and upper flags n=200")
    n = 200
    L = synth.lower_triangular(n, 6)
    X, _ = inv(trinv, dev(L), leaf=32, unit_diag=True)
    assert rel_fro(host(X), oracle.tril_inverse(L, unit=True)) < 1e-12
    U = np.ascontiguousarray(L.T)
    Xu, _ = inv(trinv, dev(U), leaf=32, upper=True)
    assert rel_fro(host(Xu), oracle.tril_inverse(L).T) < 1e-12
    assert np.all(np.tril(host(Xu), -1) == 0.0)


def test_singular_reports_index(trinv):
    from paper_2307_07611_amd import _lib

    banner("singular n=100 zero at 37 and 80")
    L = synth.lower_triangular(100, 7)
    L[37, 37] = 0.0
    L[80, 80] = 0.0
    with pytest.raises(_lib.TrinvError) as e:
        trinv.tril_inverse(dev(L), leaf=32)
    assert e.value.code == _lib.ERR_SINGULAR and e.value.info["first_bad_index"] == 38


# ---------------------------------------------------------------- FP32
@pytest.mark.parametrize("n", [64, 256, 1000])
def test_fp32(trinv, n):
    import torch

    banner(f"plain f32 n={n}")
    L32 = synth.lower_triangular(n, 20 + n, dtype=np.float32)
    X, _ = inv(trinv, dev(L32))
    Xo = oracle.tril_inverse(L32.astype(np.float64))
    Xg = host(X).astype(np.float64)
    assert rel_fro(Xg, Xo) < 1e-5
    assert oracle.residuals(L32, Xg)["rel_lx"] < 1e-5
    assert np.all(np.triu(Xg, 1) == 0.0)
    del torch


# ---------------------------------------------------------------- configuration 2 (scale)
def test_n8192_fp64_leaf64_sampled(trinv):
    import torch

    banner("plain f64 n=8192 leaf=64 seed=2")
    n = 8192
    L = synth.lower_triangular(n, 2)
    Ld = dev(L)
    X, info = inv(trinv, Ld, leaf=64, check=True)
    assert info["rel_residual"] <= 1e-13
    cols = np.array([0, 1, 63, 64, 1000, 4095, 4096, 6000, 8190, 8191])
    Xo = oracle.tril_inverse_columns(L, cols)
    Xg = host(X[:, torch.from_numpy(cols).cuda()])
    assert rel_fro(Xg, Xo) < 1e-12
    assert np.max(np.abs(Xg - Xo)) < 1e-12
    rows = np.array([0, 5000, 8191])
    Xr = host(X[torch.from_numpy(rows).cuda()])
    assert np.all(Xr[0, 1:] == 0) and np.all(Xr[1, 5001:] == 0)
    Xh = host(X)
    sq = oracle.residual_columns(L, Xh, cols)
    assert np.sqrt(sq.sum()) / (np.linalg.norm(np.tril(L)) * np.linalg.norm(Xh)) < 1e-13


# ---------------------------------------------------------------- factored inverse
def test_factored_printed_example(trinv, golden):
    banner("factored inverse, printed 5x5 example")
    g = golden("skul_5x5.txt")
    Linv, Uinv, Ainv = trinv.factored_inverse(dev(g["L"]), dev(g["U"]), u_unit=True, leaf=16)
    np.testing.assert_allclose(host(Linv), g["K"], atol=1e-4)
    np.testing.assert_allclose(host(Uinv), g["S"], atol=1e-4)
    np.testing.assert_allclose(g["A"] @ host(Ainv), np.eye(5), atol=1e-3)


def test_factored_n512_full(trinv):
    banner("factored inverse n=512 full oracle")
    n = 512
    L = synth.lower_triangular(n, 3, unit=True)
    U = synth.upper_triangular(n, 4)
    Linv, Uinv, Ainv = trinv.factored_inverse(dev(L), dev(U), l_unit=True, leaf=64)
    Lo, Uo, Ao = oracle.factored_inverse(L, U, l_unit=True)
    assert rel_fro(host(Linv), Lo) < 1e-12
    assert rel_fro(host(Uinv), Uo) < 1e-12
    assert rel_fro(host(Ainv), Ao) < 1e-12
    assert np.all(np.triu(host(Linv), 1) == 0) and np.all(np.tril(host(Uinv), -1) == 0)


def test_factored_n4096_sampled(trinv):
    banner("factored inverse n=4096 (configuration size) sampled")
    n = 4096
    L = synth.lower_triangular(n, 3, unit=True)
    U = synth.upper_triangular(n, 4)
    Linv, Uinv, Ainv = trinv.factored_inverse(dev(L), dev(U), l_unit=True, leaf=64)
    Lh, Uh, Ah = host(Linv), host(Uinv), host(Ainv)
    cols = np.array([0, 777, 2048, 4095])
    Lc = oracle.tril_inverse_columns(L, cols, unit=True)  # columns of L^-1
    assert rel_fro(Lh[:, cols], Lc) < 1e-12
    rows = np.array([0, 100, 2047, 4095])
    Ur = oracle.tril_inverse_columns(np.ascontiguousarray(U.T), rows).T  # rows of U^-1
    assert rel_fro(Uh[rows], Ur) < 1e-12
    Aref = Ur @ Lc  # Ainv(rows, cols) = U^-1(rows, :) L^-1(:, cols)
    assert rel_fro(Ah[np.ix_(rows, cols)], Aref) < 1e-12


# ---------------------------------------------------------------- adjoint
@pytest.mark.parametrize("n,dtype", [(16, "f64"), (100, "f64"), (256, "f64"), (300, "f32")])
def test_backward_vs_oracle(trinv, n, dtype):
    import torch

    banner(f"backward n={n} {dtype}")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    L = synth.lower_triangular(n, 40 + n)
    W = synth.normal(n, n, 50 + n)
    if dtype == "f32":
        L = L.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    Xg = oracle.tril_inverse(L)  # the backward consumes the forward's X
    g = trinv.tril_inverse_backward(dev(Xg, tdt), dev(W, tdt))
    torch.cuda.synchronize()
    go = oracle.tril_inverse_backward(L, W)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_fro(host(g), go) < tol
    assert np.all(np.triu(host(g), 1) == 0)


def test_autograd_function(trinv):
    import torch

    banner("autograd TrilInverse n=128 f64")
    n = 128
    L = synth.lower_triangular(n, 77)
    W = synth.normal(n, n, 78)
    Lt = dev(L).requires_grad_(True)
    X = trinv.TrilInverse.apply(Lt)
    loss = (dev(W) * X).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert rel_fro(host(Lt.grad), oracle.tril_inverse_backward(L, W)) < 1e-12
