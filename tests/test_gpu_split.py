"""GPU parity of the refinement's split residual product (the dominant kernel
of the mixed-precision path) and of the refinement loop when it runs on that
product, against the CPU oracle.

The split product forms N_L N_X from low-precision slices (hi + lo) of both
factors with FP32 accumulation: its error per entry is at most 3 u^2
(|N_L||N_X|)_ij from the slices (u = 2^-8 BF16, 2^-11 FP16) plus the FP32
rounding of the sums (about sqrt(m) 2^-24 (|N_L||N_X|)_ij for m products per
entry). The tests allow 16 u^2 + 8 sqrt(m) 2^-24 times |N_L||N_X| per entry
(plus the FP32 storage of R), and, over the whole matrix, twice the library's
own estimate of the relative error (resid_error_est, whose constant is twice
the one measured). Forward errors are checked through the exact identity
X - X_o = -X_o (L X - I): entrywise |X - X_o| <= |X_o| |R| and
||X - X_o||_F <= ||X_o||_2 ||R||_F, with R the oracle's FP64 residual of the
GPU result; the strictly lower part is reported as
||N_X - N_Xo||_F / ||N_Xo||_F.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, dev, host, rel_fro

pytestmark = pytest.mark.gpu

U_LP = {"bf16_refine": 2.0 ** -8, "f16_refine": 2.0 ** -11}


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07611_amd as P

    P.load()
    return P


def iterate(P, Ld, mode, leaf, corrections):
    """The refinement's iterate after `corrections` corrections (split residual)."""
    import torch
    from paper_2307_07611_amd import _lib

    X = torch.empty_like(Ld)
    with pytest.raises(_lib.TrinvError) as e:
        P.tril_inverse(Ld, mode, leaf=leaf, max_iter=corrections, tol=1e-300, resid="split", out=X)
    assert e.value.code == _lib.ERR_NOT_CONVERGED
    torch.cuda.synchronize()
    return X, e.value.info


def strict_err(X, Xo):
    return rel_fro(np.tril(X, -1), np.tril(Xo, -1))


def norm2_bound(A):
    """||A||_2 <= sqrt(||A||_1 ||A||_inf)."""
    return float(np.sqrt(np.abs(A).sum(axis=0).max() * np.abs(A).sum(axis=1).max()))


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
@pytest.mark.parametrize("n,leaf", [(1000, 64), (1536, 128), (2048, 128), (4096, 128)])
def test_split_residual_elementwise(P, mode, n, leaf):
    """Two-product form on the first iterate (exact in one slice) and
    three-product form on the iterate after one correction, element by
    element against the oracle's FP64 R = I - L X of the same X."""
    banner(f"split residual {mode} n={n} leaf={leaf}")
    L = synth.lower_triangular(n, 70 + n)
    Ld = dev(L)
    u = U_LP[mode]
    NLa = np.abs(np.tril(L, -1))
    nl = np.linalg.norm(np.tril(L))
    for corrections, nsplit in ((0, 2), (1, 3)):
        X, _ = iterate(P, Ld, mode, leaf, corrections)
        Xh = host(X)
        banner(f"split residual {mode} n={n} nsplit={nsplit}")
        r = P.refine_residual(Ld, X, mode, nsplit=nsplit)
        Rg = host(r["R"]).astype(np.float64)
        Ro = oracle.residual_matrix(L, Xh)
        A = NLa @ np.abs(np.tril(Xh, -1))
        # FP64 rounding of both sides: the oracle's sums (gamma_n) and the
        # GPU's FP64 assembly of the diagonal terms, over |L||X|
        F = np.abs(np.tril(L)) @ np.abs(Xh)
        tol = ((16 * u * u + 8 * np.sqrt(nsplit * n) * 2.0 ** -24) * A + 2.0 ** -23 * np.abs(Ro)
               + (n + 8) * 2.0 ** -53 * F + 1e-300)
        low = np.tril_indices(n)
        d = np.abs(Rg - Ro)
        worst = float(np.max(d[low] / tol[low]))
        nx = np.linalg.norm(Xh)
        fro = np.linalg.norm(np.tril(Rg - Ro)) / (nl * nx)
        rho_o = np.linalg.norm(Ro) / (nl * nx)
        print(f"n={n} nsplit={nsplit}: worst entry / tol {worst:.3f}, ||dR||/(||L|| ||X||) {fro:.3e}, "
              f"est {r['est']:.3e}, bound {r['bound']:.3e}, rho {r['rel']:.3e} (oracle {rho_o:.3e})", flush=True)
        assert worst <= 1.0
        assert np.all(np.triu(Rg, 1) == 0.0)
        assert fro <= 2.0 * r["est"] <= r["bound"]
        assert abs(r["rel"] - rho_o) <= r["est"]
        assert r["norm_l"] == pytest.approx(nl, rel=1e-12)
        assert r["norm_x"] == pytest.approx(nx, rel=1e-12)


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
@pytest.mark.parametrize("n,leaf", [(1000, 64), (1536, 128), (2048, 128), (4096, 128)])
def test_refine_on_split_residual(P, mode, n, leaf):
    """The whole refinement with the split residual (fused correction
    epilogue for BF16 at orders divisible by 256), to a tolerance above the
    split product's estimated floor at this order."""
    banner(f"refine on split residual {mode} n={n} leaf={leaf}")
    L = synth.lower_triangular(n, 80 + n)
    Ld = dev(L)
    _, info0 = iterate(P, Ld, mode, leaf, 0)
    tol = max(1e-12, 4.0 * info0["resid_error_est"])
    X, info = P.tril_inverse(Ld, mode, leaf=leaf, tol=tol, max_iter=6, resid="split", return_info=True)
    Xh = host(X)
    Xo = oracle.tril_inverse(L)
    Ro = oracle.residual_matrix(L, Xh)
    nl, nx = np.linalg.norm(np.tril(L)), np.linalg.norm(Xh)
    rho_o = np.linalg.norm(Ro) / (nl * nx)
    se = strict_err(Xh, Xo)
    print(f"n={n}: tol {tol:.2e} iterations {info['iterations']} rho {info['rel_residual']:.3e} "
          f"(oracle {rho_o:.3e}) est {info['resid_error_est']:.3e} strict fwd {se:.3e} "
          f"full fwd {rel_fro(Xh, Xo):.3e}", flush=True)
    assert info["rel_residual"] + info["resid_error_est"] <= tol
    assert abs(info["rel_residual"] - rho_o) <= info["resid_error_est"]
    assert rho_o <= tol
    assert np.all(np.triu(Xh, 1) == 0.0)
    # forward error through X - X* = -X* R, with the oracle's Xo for X* and
    # its own error |Xo - X*| <= n 2^-53 |Xo||L||Xo| (column recurrence)
    d = np.abs(Xh - Xo)
    Ea = n * 2.0 ** -53 * (np.abs(Xo) @ (np.abs(np.tril(L)) @ np.abs(Xo)))
    assert np.all(d <= 1.01 * (np.abs(Xo) @ np.abs(Ro)) + Ea + 1e-300)
    assert np.linalg.norm(Xh - Xo) <= 1.01 * norm2_bound(Xo) * np.linalg.norm(Ro) + np.linalg.norm(Ea)
    assert se < 1e-6


def test_bf16_split_ragged_large(P):
    """A ragged large order (edge tiles in every product, no fused correction)
    on the split residual to 1e-12: FP64-MFMA residual check, the in-loop
    residual within its estimate, sampled columns against the oracle."""
    import torch

    n = 12345
    banner(f"bf16_refine split residual n={n} leaf=128")
    L = synth.lower_triangular(n, 11)
    Ld = dev(L)
    X, info = P.tril_inverse(Ld, "bf16_refine", leaf=128, resid="split", return_info=True)
    torch.cuda.synchronize()
    r = P.residual(Ld, X)
    print(f"n={n}: iterations {info['iterations']} rho {info['rel_residual']:.3e} (fp64 {r['rel']:.3e}) "
          f"est {info['resid_error_est']:.3e}", flush=True)
    assert r["rel"] <= 1e-12
    assert info["rel_residual"] + info["resid_error_est"] <= 1e-12
    assert abs(info["rel_residual"] - r["rel"]) <= info["resid_error_est"]
    cols = np.array([0, 1, 255, 256, 4096, 6172, 12000, 12288, 12343, 12344])
    Xo = oracle.tril_inverse_columns(L, cols)
    Xg = host(X[:, torch.from_numpy(cols).cuda()])
    rows = np.arange(n)[:, None]
    strict = rows > cols[None, :]
    se = np.linalg.norm((Xg - Xo)[strict]) / np.linalg.norm(Xo[strict])
    print(f"n={n}: sampled strict fwd {se:.3e}", flush=True)
    assert se < 1e-6
    np.testing.assert_array_equal(Xg[~(rows >= cols[None, :])], 0.0)
