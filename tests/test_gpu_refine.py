"""GPU parity of the mixed-precision path (BF16 MFMA products + FP64 leaves and
residual + Newton-Schulz refinement) against the CPU oracle.

Tolerance: the relative residual ||LX - I||_F / (||L||_F ||X||_F) after
refinement must be <= 1e-12 (the stopping rule stops at rho + its estimated
error <= 1e-12), checked independently with
the oracle's FP64 residual (CPU) or the FP64-MFMA residual helper (n = 16384,
itself checked against the oracle in the plain-path tests). The forward error
against the oracle is bounded by kappa times that residual times the norm
ratio; for this generator kappa ~ 2, and 1e-10 is used (relative Frobenius).
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


def run(trinv, L, mode="bf16_refine", **kw):
    import torch

    X, info = trinv.tril_inverse(L, mode, return_info=True, **kw)
    torch.cuda.synchronize()
    return X, info


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
@pytest.mark.parametrize("n,leaf", [(256, 64), (300, 64), (1024, 64), (1500, 128), (2048, 128)])
def test_refine_vs_oracle(trinv, mode, n, leaf):
    banner(f"{mode} n={n} leaf={leaf}")
    L = synth.lower_triangular(n, 60 + n)
    X, info = run(trinv, dev(L), mode, leaf=leaf)
    Xg = host(X)
    r = oracle.residuals(L, Xg)
    print(f"n={n}: iterations={info['iterations']} rho_gpu={info['rel_residual']:.3e} "
          f"rho_oracle={r['rel_lx']:.3e} fwd={rel_fro(Xg, oracle.tril_inverse(L)):.3e}", flush=True)
    assert r["rel_lx"] <= 1e-12
    assert info["rel_residual"] + info["resid_error_est"] <= 1e-12
    Xo = oracle.tril_inverse(L)
    assert rel_fro(Xg, Xo) < 1e-10
    # the strictly lower part (what the products compute; the diagonal is 1 / L_ii)
    se = rel_fro(np.tril(Xg, -1), np.tril(Xo, -1))
    print(f"n={n}: strict fwd {se:.3e}", flush=True)
    assert se < 1e-6
    assert np.all(np.triu(Xg, 1) == 0.0)
    # the in-loop residual agrees with the FP64 one within its estimated error
    assert abs(info["rel_residual"] - r["rel_lx"]) <= max(info["resid_error_est"], 1e-15)


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
def test_exact_bidiagonal(trinv, mode):
    """All values +-1: every product and every partial sum is exact in BF16 /
    FP16 (with power-of-two scales) and FP32, so X is the exact all-ones lower
    triangle and no correction runs."""
    n = 1000
    banner(f"{mode} bidiagonal -1 n={n}")
    L = np.eye(n)
    L[np.arange(1, n), np.arange(n - 1)] = -1.0
    X, info = run(trinv, dev(L), mode, leaf=64)
    np.testing.assert_array_equal(host(X), np.tril(np.ones((n, n))))
    assert info["iterations"] == 0 and info["rel_residual"] == 0.0


def test_bf16_not_converged_reports_forward_residual(trinv):
    from paper_2307_07611_amd import _lib

    n = 1024
    banner(f"bf16_refine max_iter=0 n={n}")
    L = synth.lower_triangular(n, 9)
    with pytest.raises(_lib.TrinvError) as e:
        trinv.tril_inverse(dev(L), "bf16_refine", leaf=64, max_iter=0)
    assert e.value.code == _lib.ERR_NOT_CONVERGED
    assert 1e-12 < e.value.info["rel_residual"] < 1e-3
    assert e.value.info["iterations"] == 0


def _bf16_exact(v):
    f = v.astype(np.float32)
    return (f.astype(np.float64) == v) & ((f.view(np.uint32) & 0xFFFF) == 0)


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
@pytest.mark.parametrize("n,leaf", [(640, 64), (1000, 128)])
def test_first_iterate_exact_in_low_precision(trinv, mode, n, leaf):
    """The first iterate keeps the FP64 diagonal 1 / L_ii (bitwise) and holds,
    below it, values of the low-precision type times one power-of-two scale
    (1 for BF16; for FP16 2^(11 - e) with 1 / min |L_ii| < 2^e), so the first
    residual's two-product form is exact in X. max_iter = 0 returns it."""
    import torch
    from paper_2307_07611_amd import _lib

    banner(f"{mode} first iterate n={n} leaf={leaf}")
    L = synth.lower_triangular(n, 12)
    X = torch.empty((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.TrinvError) as e:
        trinv.tril_inverse(dev(L), mode, leaf=leaf, max_iter=0, out=X)
    assert e.value.code == _lib.ERR_NOT_CONVERGED
    Xh = host(X)
    d = np.diag(L)
    np.testing.assert_array_equal(np.diag(Xh), 1.0 / d)
    off = Xh[np.tril_indices(n, -1)]
    if mode == "bf16_refine":
        assert np.all(_bf16_exact(off))
    else:
        ex = np.frexp(np.max(1.0 / np.abs(d)))[1]  # 1 / min |L_ii| < 2^ex
        scaled = off * 2.0 ** (11 - ex)
        assert np.all(scaled.astype(np.float16).astype(np.float64) == scaled)
    np.testing.assert_array_equal(np.triu(Xh, 1), 0.0)
    # it is the low-precision forward: close to the oracle, not equal
    Xo = oracle.tril_inverse(L)
    assert 0.0 < rel_fro(Xh, Xo) < 1e-2


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
def test_singular(trinv, mode):
    from paper_2307_07611_amd import _lib

    banner(f"{mode} singular n=512")
    L = synth.lower_triangular(512, 3)
    L[300, 300] = 0.0
    with pytest.raises(_lib.TrinvError) as e:
        trinv.tril_inverse(dev(L), mode, leaf=64)
    assert e.value.code == _lib.ERR_SINGULAR and e.value.info["first_bad_index"] == 301


def test_bf16_ill_conditioned_is_honest(trinv):
    """Unit lower with U[-1,1] off-diagonals (no 1/n scale): the condition
    number grows exponentially with n. The path must either certify a
    residual that the FP64 check confirms, or report NOT_CONVERGED."""
    from paper_2307_07611_amd import _lib

    n = 512
    banner(f"bf16_refine ill-conditioned n={n}")
    L = synth.lower_triangular(n, 4, unit=True)
    L[np.tril_indices(n, -1)] *= n
    try:
        X, info = run(trinv, dev(L), leaf=64, max_iter=6)
        assert oracle.residuals(L, host(X))["rel_lx"] <= 1e-12
    except _lib.TrinvError as e:
        assert e.code in (_lib.ERR_NOT_CONVERGED, _lib.ERR_NONFINITE)


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
def test_refine_n16384_configuration(trinv, mode):
    """Configuration size: residual by the FP64-MFMA helper, sampled columns
    against the oracle."""
    import torch

    n = 16384
    banner(f"{mode} n={n} leaf=128 seed=5")
    L = synth.lower_triangular(n, 5)
    Ld = dev(L)
    X, info = run(trinv, Ld, mode, leaf=128)
    r = trinv.residual(Ld, X)
    print(f"n={n}: iterations={info['iterations']} rho_gpu={info['rel_residual']:.3e} rho_fp64={r['rel']:.3e}",
          flush=True)
    assert r["rel"] <= 1e-12 and info["rel_residual"] + info["resid_error_est"] <= 1e-12
    assert abs(info["rel_residual"] - r["rel"]) <= info["resid_error_est"]
    cols = np.array([0, 4095, 8192, 16000, 16382])
    Xo = oracle.tril_inverse_columns(L, cols)
    Xg = host(X[:, torch.from_numpy(cols).cuda()])
    assert rel_fro(Xg, Xo) < 1e-10
    strict = np.arange(n)[:, None] > cols[None, :]
    se = np.linalg.norm((Xg - Xo)[strict]) / np.linalg.norm(Xo[strict])
    print(f"n={n}: sampled strict fwd {se:.3e}", flush=True)
    assert se < 1e-6


def test_bf16_n16384_leaf32_more_corrections(trinv):
    """Configuration size with 32-wide FP64 leaves: more BF16 levels leave a
    larger first residual, so the path may need a second correction after one
    whose epilogue wrote the next residual's slices of X itself (the A-role
    slice is then re-split from X). Whatever the count, the certified residual
    must hold under the FP64 check and sampled columns must match the oracle."""
    import torch

    n = 16384
    banner(f"bf16_refine n={n} leaf=32 seed=5")
    L = synth.lower_triangular(n, 5)
    Ld = dev(L)
    X, info = run(trinv, Ld, "bf16_refine", leaf=32)
    r = trinv.residual(Ld, X)
    print(f"n={n} leaf=32: iterations={info['iterations']} rho_gpu={info['rel_residual']:.3e} "
          f"rho_fp64={r['rel']:.3e}", flush=True)
    assert r["rel"] <= 1e-12 and info["rel_residual"] + info["resid_error_est"] <= 1e-12
    assert abs(r["rel"] - info["rel_residual"]) <= max(info["resid_error_est"], 1e-15)
    cols = np.array([1, 5000, 12345])
    Xo = oracle.tril_inverse_columns(L, cols)
    Xg = host(X[:, torch.from_numpy(cols).cuda()])
    assert rel_fro(Xg, Xo) < 1e-10
    # a tolerance just under what one correction reached: a further correction
    # runs (with the BF16 residual while its floor allows it)
    tol = 0.9 * info["rel_residual"]
    X2, info2 = run(trinv, Ld, "bf16_refine", leaf=32, tol=tol, max_iter=4)
    r2 = trinv.residual(Ld, X2)
    print(f"n={n} leaf=32 tol={tol:.3e}: iterations={info2['iterations']} rho_gpu={info2['rel_residual']:.3e} "
          f"rho_fp64={r2['rel']:.3e} est={info2['resid_error_est']:.3e}", flush=True)
    assert info2["iterations"] >= 2
    assert r2["rel"] <= tol and info2["rel_residual"] + info2["resid_error_est"] <= tol
    Xg2 = host(X2[:, torch.from_numpy(cols).cuda()])
    assert rel_fro(Xg2, Xo) < 1e-10


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
def test_residual_precision_choice(trinv, mode):
    """AUTO chooses the residual product's precision from the first iterate's
    norms: with a tolerance below the split product's estimated error it runs
    exactly as resid="fp64" (bitwise), with a loose one exactly as
    resid="split" (whose norms are read with the residual's sums)."""
    import torch

    n = 2048
    banner(f"residual precision choice {mode} n={n}")
    Ld = dev(synth.lower_triangular(n, 12))

    def go(resid, tol):
        X = torch.empty_like(Ld)
        try:
            _, info = trinv.tril_inverse(Ld, mode, leaf=128, tol=tol, max_iter=3, resid=resid, out=X,
                                         return_info=True)
            st = 0
        except trinv.TrinvError as e:
            info, st = e.info or {}, e.code
        torch.cuda.synchronize()
        return X, info, st

    tight = 1e-16  # below the split product's estimated error at this order
    Xa, ia, sa = go("auto", tight)
    Xf, i_f, sf = go("fp64", tight)
    print(f"tight: auto status {sa} est {ia.get('resid_error_est')}, fp64 status {sf} est {i_f.get('resid_error_est')}",
          flush=True)
    assert sa == sf and torch.equal(Xa, Xf)
    assert ia.get("resid_error_est") == i_f.get("resid_error_est")
    Xa, ia, sa = go("auto", 1e-9)
    Xs, i_s, ss = go("split", 1e-9)
    assert sa == ss == 0 and torch.equal(Xa, Xs)
    assert ia["resid_error_est"] == i_s["resid_error_est"]
