"""Failure reporting, determinism, strided views and the residual helper at
configuration size, through the C ABI.

- A NaN in the input shows as TRINV_ERR_NONFINITE (plain blocking calls,
  refine modes, factored inverse) or as status -2 for that matrix (batched);
  TrilInverse raises on a batch with a singular matrix.
- The FP64 and refine paths are bitwise deterministic run to run (fixed
  reduction orders, no atomics in the arithmetic).
- The upper case of the refine path goes through the transposed view.
- The FP64-MFMA residual helper at n = 4096 against a planted perturbation
  with a closed-form residual.
"""

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


@pytest.mark.parametrize("mode,dtype", [("f64", np.float64), ("f32", np.float32), ("bf16_refine", np.float64),
                                        ("f16_refine", np.float64)])
def test_nan_input_reports_nonfinite(P, mode, dtype):
    from paper_2307_07611_amd import _lib

    n = 300
    banner(f"NaN input {mode} n={n}")
    L = synth.lower_triangular(n, 21).astype(dtype)
    L[200, 50] = np.nan
    with pytest.raises(_lib.TrinvError) as e:
        P.tril_inverse(dev(L), mode, leaf=64)
    assert e.value.code == _lib.ERR_NONFINITE
    # a NaN above the diagonal is never read
    L2 = synth.lower_triangular(n, 21).astype(dtype)
    L2[50, 200] = np.nan
    X = P.tril_inverse(dev(L2), mode, leaf=64)
    assert np.all(np.isfinite(host(X)))


def test_nan_factored(P):
    from paper_2307_07611_amd import _lib

    n = 256
    banner(f"NaN factored n={n}")
    L = synth.lower_triangular(n, 3, unit=True)
    U = synth.upper_triangular(n, 4)
    U[10, 100] = np.inf
    with pytest.raises(_lib.TrinvError) as e:
        P.factored_inverse(dev(L), dev(U), l_unit=True, leaf=32)
    assert e.value.code == _lib.ERR_NONFINITE


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batched_nonfinite_status(P, dt):
    """Uneven batch (persistent launch) and a uniform one (level path): the
    matrix with a NaN gets status -2, the singular one its pivot index, the
    others 0."""
    import torch

    dtype = np.float32 if dt == "f32" else np.float64
    for sizes in ([40, 300, 17, 128, 513], [160] * 5):
        banner(f"batched nonfinite {dt} sizes={sizes}")
        offs = np.zeros(len(sizes), dtype=np.int64)
        offs[1:] = np.cumsum(np.asarray(sizes[:-1], dtype=np.int64) ** 2)
        packed = np.zeros(int(offs[-1]) + sizes[-1] ** 2, dtype=dtype)
        for i, n in enumerate(sizes):
            Li = synth.lower_triangular(n, 500 + i, dtype=dtype)
            if i == 1:
                Li[n - 1, 3] = np.nan
            if i == 3:
                Li[9, 9] = 0.0
            packed[offs[i]:offs[i] + n * n] = Li.ravel()
        X, status = P.tril_inverse_batched(torch.from_numpy(packed).cuda(), sizes, offs, dt)
        st = status.cpu().numpy()
        assert list(st) == [0, -2, 0, 10, 0], st


def test_trilinverse_raises_on_singular_batch(P):
    import torch
    from paper_2307_07611_amd import _lib

    banner("TrilInverse batch with a singular matrix")
    batch, n = 4, 64
    L = np.stack([synth.lower_triangular(n, 600 + b, dtype=np.float32) for b in range(batch)])
    L[2, 30, 30] = 0.0
    Lt = torch.from_numpy(L).cuda().requires_grad_(True)
    with pytest.raises(_lib.TrinvError) as e:
        P.TrilInverse.apply(Lt)
    assert e.value.code == _lib.ERR_SINGULAR
    assert e.value.info["matrices"] == [2] and e.value.info["status"] == [31]


@pytest.mark.parametrize("mode,n", [("f64", 4096), ("f32", 2048), ("bf16_refine", 2048), ("f16_refine", 1536)])
def test_bitwise_run_to_run(P, mode, n):
    import torch

    banner(f"run-to-run determinism {mode} n={n}")
    dtype = np.float32 if mode == "f32" else np.float64
    Ld = dev(synth.lower_triangular(n, 31, dtype=dtype))
    X1 = P.tril_inverse(Ld, mode)
    X2 = P.tril_inverse(Ld, mode)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)


@pytest.mark.parametrize("mode", ["bf16_refine", "f16_refine"])
def test_refine_upper(P, mode):
    banner(f"{mode} upper n=1000")
    n = 1000
    L = synth.lower_triangular(n, 41)
    U = np.ascontiguousarray(L.T)
    X, info = P.tril_inverse(dev(U), mode, leaf=64, upper=True, return_info=True)
    Xh = host(X)
    Xo = oracle.tril_inverse(L).T
    assert np.all(np.tril(Xh, -1) == 0.0)
    assert rel_fro(Xh, Xo) < 1e-10
    # the residual of the upper problem: U X = I, i.e. X^T L^T... = (L X^T)^T
    assert oracle.residuals(L, np.ascontiguousarray(Xh.T))["rel_lx"] <= 1e-12


def test_factored_strided_views(P):
    """L and U as row-strided views of larger buffers (leading dimensions
    n + 24 and n + 40), garbage outside the triangles."""
    import torch

    n = 700
    banner(f"factored inverse strided views n={n}")
    L = synth.lower_triangular(n, 3, unit=True)
    U = synth.upper_triangular(n, 4)
    Lb = np.full((n, n + 24), 5.0)
    Lb[:, :n] = L + np.triu(np.full((n, n), 9.0), 1)
    Ub = np.full((n, n + 40), -7.0)
    Ub[:, :n] = U + np.tril(np.full((n, n), 3.0), -1)
    Lt = torch.from_numpy(Lb).cuda()[:, :n]
    Ut = torch.from_numpy(Ub).cuda()[:, :n]
    assert Lt.stride(0) == n + 24 and Ut.stride(0) == n + 40
    Linv, Uinv, Ainv = P.factored_inverse(Lt, Ut, l_unit=True, leaf=64)
    Lo, Uo, Ao = oracle.factored_inverse(L, U, l_unit=True)
    assert rel_fro(host(Linv), Lo) < 1e-12
    assert rel_fro(host(Uinv), Uo) < 1e-12
    assert rel_fro(host(Ainv), Ao) < 1e-12


def test_residual_helper_n4096_planted(P):
    """trinv_residual (FP64 MFMA) at n = 4096: X = X_o + delta e_p e_q^T has
    ||L X - I||_F = |delta| ||L(:, p)||_2 up to the tiny residual of X_o."""
    n = 4096
    banner(f"residual helper n={n} planted perturbation")
    L = synth.lower_triangular(n, 2)
    Xo = oracle.tril_inverse(L)
    p, q, delta = 3000, 1234, 1e-6
    Xp = Xo.copy()
    Xp[p, q] += delta
    r = P.residual(dev(L), dev(Xp))
    want = delta * np.linalg.norm(L[p:, p])
    assert r["lx"] == pytest.approx(want, rel=1e-6)
    assert r["norm_l"] == pytest.approx(np.linalg.norm(np.tril(L)), rel=1e-12)
    assert r["norm_x"] == pytest.approx(np.linalg.norm(Xp), rel=1e-12)
    cols = np.array([0, q, 4095])
    c = oracle.residual_columns(L, Xp, cols)
    assert np.sqrt(c[1]) == pytest.approx(want, rel=1e-6)


def test_profile_select_and_dispatch_events(P):
    """The launch profiler: every class by default, only the selected ones
    after profile_select; the timed intervals lie inside the step's own time
    and the results are those of an unprofiled run (bitwise)."""
    import torch

    banner("launch profiler classes bf16_refine n=2048")
    n = 2048
    Ld = dev(synth.lower_triangular(n, 41))
    kw = dict(resid="split", tol=1e-9)  # every product on BF16 MFMA at this order
    X0 = P.tril_inverse(Ld, "bf16_refine", **kw)
    torch.cuda.synchronize()
    P.profile_select(None)
    P.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    X1 = P.tril_inverse(Ld, "bf16_refine", **kw)
    e1.record()
    torch.cuda.synchronize()
    every = P.profile_read()
    P.profile_enable(False)
    step_ms = e0.elapsed_time(e1)
    for cls in ("split", "leaf_f64", "bf16_level_T", "bf16_level_X21", "bf16_residual2", "bf16_correction",
                "bf16_residual"):
        assert every[cls]["launches"] >= 1, cls
    assert all(v["total_ms"] > 0.0 for v in every.values())
    assert sum(v["total_ms"] for v in every.values()) <= step_ms * 1.05
    P.profile_select(["bf16_residual2", "bf16_level_T"])
    P.profile_enable(True)
    X2 = P.tril_inverse(Ld, "bf16_refine", **kw)
    torch.cuda.synchronize()
    some = P.profile_read()
    P.profile_enable(False)
    P.profile_select(None)
    assert sorted(some) == ["bf16_level_T", "bf16_residual2"]
    assert some["bf16_level_T"]["launches"] == every["bf16_level_T"]["launches"]
    assert torch.equal(X0, X1) and torch.equal(X0, X2)
