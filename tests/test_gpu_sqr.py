"""GPU parity of algorithm SQR (Section 5: modified Gram-Schmidt A = Q R with
S = R^-1 and S Q^T = A^-1) through the C ABI, against the oracle (the
algorithm's column-by-column steps).

Tolerances: for the diagonally dominant inputs (kappa below 10) FP64
relative Frobenius error <= 1e-11 per output, FP32 <= 1e-4; for a Gaussian
input the Gram-Schmidt variants differ by O(eps kappa^2), so the bound there
is 1e-14 kappa^2. At n = 4096 (beyond the oracle's seconds): Q^T Q = I,
Q R = A, S R = I and A Ainv = I to stated bounds."""

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


def test_sqr_printed_example(P, golden):
    banner("sqr printed 5x5")
    g = golden("sqr_5x5.txt")
    Q, R, S, Ainv = (host(t) for t in P.sqr(dev(g["A"])))
    for got, name in ((Q, "Q"), (R, "R"), (S, "S")):
        np.testing.assert_allclose(got, g[name], atol=2e-4)
    ref = oracle.sqr(g["A"])
    for got, want in zip((Q, R, S, Ainv), ref):
        assert rel_fro(got, want) <= 1e-13


@pytest.mark.parametrize("n,dt", [(16, "f64"), (100, "f64"), (300, "f64"), (1000, "f64"), (1100, "f64"),
                                  (500, "f32"), (1300, "f32")])
def test_sqr_vs_oracle(P, n, dt):
    import torch

    banner(f"sqr n={n} {dt}")
    A = synth.diag_dominant(n, 50 + n)
    tdt = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    outs = [host(t).astype(np.float64) for t in P.sqr(dev(A, tdt))]
    ref = oracle.sqr(A)
    tol = 1e-11 if dt == "f64" else 1e-4
    for got, want, name in zip(outs, ref, ("Q", "R", "S", "Ainv")):
        e = rel_fro(got, want)
        print(f"n={n} {dt} {name}: {e:.3e}", flush=True)
        assert e <= tol, name
    R, S = outs[1], outs[2]
    assert np.all(np.tril(R, -1) == 0) and np.all(np.tril(S, -1) == 0) and np.all(np.diag(R) > 0)


def test_sqr_gaussian(P):
    n = 512
    banner(f"sqr n={n} gaussian")
    A = synth.normal(n, n, 21)
    kappa = np.linalg.cond(A)
    Q, R, S, Ainv = (host(t) for t in P.sqr(dev(A)))
    Qo, Ro, So, Ao = oracle.sqr(A)
    tol = 1e-14 * kappa * kappa
    e = [rel_fro(Q, Qo), rel_fro(R, Ro), rel_fro(Ainv, Ao)]
    print(f"gaussian kappa {kappa:.3e}: Q {e[0]:.3e} R {e[1]:.3e} Ainv {e[2]:.3e} (tol {tol:.1e})", flush=True)
    assert max(e) <= tol
    assert np.abs(Q @ R - A).max() <= 1e-13 * np.abs(A).max() * np.sqrt(n)


def test_sqr_n4096_properties(P):
    import torch

    n = 4096
    banner(f"sqr n={n} f64 properties")
    A = dev(synth.diag_dominant(n, 22))
    Q, R, S, Ainv = P.sqr(A)
    I = torch.eye(n, dtype=A.dtype, device=A.device)
    orth = (torch.linalg.norm(Q.T @ Q - I) / np.sqrt(n)).item()
    qr = (torch.linalg.norm(Q @ R - A) / torch.linalg.norm(A)).item()
    sr = (torch.linalg.norm(S @ R - I) / np.sqrt(n)).item()
    inv = (torch.linalg.norm(A @ Ainv - I) / np.sqrt(n)).item()
    print(f"n={n}: |QtQ-I| {orth:.3e} |QR-A|/|A| {qr:.3e} |SR-I| {sr:.3e} |A Ainv-I| {inv:.3e}", flush=True)
    assert orth <= 1e-13 and qr <= 1e-14 and sr <= 1e-13 and inv <= 1e-12
    assert bool(torch.all(torch.tril(R, -1) == 0)) and bool(torch.all(torch.diagonal(R) > 0))


def test_sqr_zero_column_reports_index(P):
    from paper_2307_07611_amd import _lib

    banner("sqr zero column")
    n = 200
    A = synth.diag_dominant(n, 23)
    A[:, 37] = 0.0
    with pytest.raises(_lib.TrinvError) as e:
        P.sqr(dev(A))
    assert e.value.code == _lib.ERR_SINGULAR and e.value.info["first_bad_index"] == 38
