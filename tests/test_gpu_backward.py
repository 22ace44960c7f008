"""GPU parity of the hand-written adjoint gradL = -tril(X^T G X^T) through
autograd (TrilInverse) and the C ABI: the 64 x 1024 FP32 configuration on
sampled rows against the oracle, central finite differences at n = 16 (FP64),
and a batched FP32 case in full.

Tolerance: gradient relative error <= 1e-4 (Frobenius, over the rows
compared); finite differences with h = 1e-6 in FP64 carry an error of order
h^2 plus 1e-16 / h, far below that.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07611_amd as P

    P.load()
    return P


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_backward_64x1024_configuration(P):
    """64 FP32 matrices of order 1024 (L seeds 2000 + b, upstream gradients
    N(0, 1) with seeds 3000 + b): forward through the batched path, backward
    through autograd; rows of three matrices against the oracle, the forward
    on sampled columns, and exact zeros above the diagonal everywhere."""
    import torch

    batch, n = 64, 1024
    banner(f"backward configuration {batch} x {n} f32")
    L = np.stack([synth.lower_triangular(n, 2000 + b, dtype=np.float32) for b in range(batch)])
    W = np.stack([synth.normal(n, n, 3000 + b, dtype=np.float32) for b in range(batch)])
    Lt = torch.from_numpy(L).cuda().requires_grad_(True)
    Wt = torch.from_numpy(W).cuda()
    X = P.TrilInverse.apply(Lt)
    (Wt * X).sum().backward()
    torch.cuda.synchronize()
    g = Lt.grad
    assert bool(torch.all(torch.triu(g, 1) == 0))
    assert bool(torch.all(torch.triu(X.detach(), 1) == 0))
    rows = np.array([1, 257, 640, 1023])
    cols = np.array([0, 300, 1000])
    for b in (0, 37, 63):
        Lb = L[b].astype(np.float64)
        go = oracle.tril_inverse_backward_rows(Lb, W[b].astype(np.float64), rows)
        gg = g[b][torch.from_numpy(rows).cuda()].double().cpu().numpy()
        e = rel(gg, go)
        xo = oracle.tril_inverse_columns(Lb, cols)
        xg = X.detach()[b][:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
        ex = rel(xg, xo)
        print(f"matrix {b}: gradient rows rel err {e:.3e}, forward columns rel err {ex:.3e}", flush=True)
        assert e <= 1e-4
        assert ex <= 1e-4


def test_gradient_finite_differences_n16(P):
    """Autograd gradient of f(L) = sum(W * L^-1) against FP64 central
    differences of the GPU forward, over the 136 lower entries."""
    import torch

    n, h = 16, 1e-6
    banner("backward finite differences n=16 f64")
    L = synth.lower_triangular(n, 7)
    W = synth.normal(n, n, 8)
    Lt = torch.from_numpy(L).cuda().requires_grad_(True)
    Wt = torch.from_numpy(W).cuda()
    X = P.TrilInverse.apply(Lt)
    (Wt * X).sum().backward()
    g = Lt.grad.cpu().numpy()

    def f(M):
        Xm = P.tril_inverse(torch.from_numpy(M).cuda(), "f64")
        return float((Wt * Xm).sum().item())

    gfd = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            Lp = L.copy()
            Lp[i, j] += h
            Lm = L.copy()
            Lm[i, j] -= h
            gfd[i, j] = (f(Lp) - f(Lm)) / (2 * h)
    e = rel(g, gfd)
    print(f"finite differences: rel err {e:.3e}", flush=True)
    assert e <= 1e-4
    assert rel(g, oracle.tril_inverse_backward(L, W)) <= 1e-12


def test_batched_autograd_f32(P):
    import torch

    batch, n = 8, 200
    banner(f"backward batched autograd {batch} x {n} f32")
    L = np.stack([synth.lower_triangular(n, 400 + b, dtype=np.float32) for b in range(batch)])
    W = np.stack([synth.normal(n, n, 500 + b, dtype=np.float32) for b in range(batch)])
    Lt = torch.from_numpy(L).cuda().requires_grad_(True)
    X = P.TrilInverse.apply(Lt)
    (torch.from_numpy(W).cuda() * X).sum().backward()
    torch.cuda.synchronize()
    g = Lt.grad.double().cpu().numpy()
    for b in range(batch):
        go = oracle.tril_inverse_backward(L[b].astype(np.float64), W[b].astype(np.float64))
        assert rel(g[b], go) <= 1e-4, b
