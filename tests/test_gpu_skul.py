"""GPU parity of algorithm SKUL (Section 5: Crout A = L U with S = U^-1,
K = L^-1, S K = A^-1) through the C ABI, against the oracle (Crout
factorization + factored inverse). Tolerances: FP64 relative Frobenius error
<= 1e-11 per output (kappa ~ 2 for the diagonally dominant generator), FP32
<= 1e-4; at n = 4096, ||L U - A|| / ||A|| <= 1e-13 and ||A Ainv - I||_F <=
1e-11 sqrt(n) (the oracle's O(n^3) single-thread loops are too slow there)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, dev, host, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07611_amd as P

    P.load()
    return P


def test_skul_printed_example(P, golden):
    banner("skul printed 5x5")
    g = golden("skul_5x5.txt")
    L, U, S, K, Ainv = (host(t) for t in P.skul(dev(g["A"])))
    for got, name in ((L, "L"), (U, "U"), (S, "S"), (K, "K")):
        np.testing.assert_allclose(got, g[name], atol=1.5e-4)
    ref = oracle.skul(g["A"])
    for got, want in zip((L, U, S, K, Ainv), ref):
        assert rel_fro(got, want) <= 1e-13


@pytest.mark.parametrize("n,dt", [(128, "f64"), (300, "f64"), (1000, "f64"), (500, "f32")])
def test_skul_vs_oracle(P, n, dt):
    import torch

    banner(f"skul n={n} {dt}")
    A = synth.diag_dominant(n, 40 + n)
    tdt = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    outs = [host(t).astype(np.float64) for t in P.skul(dev(A, tdt))]
    ref = oracle.skul(A)
    tol = 1e-11 if dt == "f64" else 1e-4
    for got, want, name in zip(outs, ref, "LUSKA"):
        e = rel_fro(got, want)
        print(f"n={n} {dt} {name}: {e:.3e}", flush=True)
        assert e <= tol, name
    L, U = outs[0], outs[1]
    assert np.all(np.triu(L, 1) == 0) and np.all(np.tril(U, -1) == 0) and np.all(np.diag(U) == 1.0)


def test_skul_n4096_properties(P):
    import torch

    n = 4096
    banner(f"skul n={n} f64 properties")
    A = dev(synth.diag_dominant(n, 77))
    L, U, S, K, Ainv = P.skul(A)
    lu = torch.linalg.norm(L @ U - A) / torch.linalg.norm(A)
    inv = torch.linalg.norm(A @ Ainv - torch.eye(n, dtype=A.dtype, device=A.device))
    sk = torch.linalg.norm(S @ K - Ainv) / torch.linalg.norm(Ainv)
    print(f"n={n}: |LU-A|/|A| {lu.item():.3e}, |A Ainv - I| {inv.item():.3e}, |SK - Ainv| {sk.item():.3e}",
          flush=True)
    assert lu.item() <= 1e-13 and inv.item() <= 1e-11 * np.sqrt(n) and sk.item() <= 1e-13


def test_skul_zero_pivot_reports_index(P):
    from paper_2307_07611_amd import _lib

    banner("skul zero pivots")
    n = 400
    A = synth.diag_dominant(n, 9)
    A[0, 0] = 0.0
    with pytest.raises(_lib.TrinvError) as e:
        P.skul(dev(A))
    assert e.value.code == _lib.ERR_SINGULAR and e.value.info["first_bad_index"] == 1
    # A = L0 U0 with L0[199, 199] = 0: the Crout pivot 200 (1-based) vanishes exactly
    L0 = np.tril(synth.diag_dominant(n, 10))
    U0 = np.triu(synth.diag_dominant(n, 11), 1) + np.eye(n)
    L0[199, 199] = 0.0
    L0 = np.round(L0 * 64) / 64  # dyadic entries: every product and sum is exact
    U0 = np.round(U0 * 64) / 64
    np.fill_diagonal(U0, 1.0)
    with pytest.raises(_lib.TrinvError) as e:
        P.skul(dev(L0 @ U0))
    assert e.value.code == _lib.ERR_SINGULAR and e.value.info["first_bad_index"] == 200
