"""The allocation-free batched entry point (trinv_tril_inverse_batched_noalloc)
against the workspace one (trinv_tril_inverse_batched), through the C ABI:
both run the same persistent kernels, so on uneven batches the results must
be bitwise equal, with equal statuses. Two calls in a row on the library's
per-device scratch, the second with a smaller batch; then the oracle on a
sample. Batch limit and argument errors are checked on the host."""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_07611_amd import _lib

    return _lib.load()


def make(sizes, dtype, seed0):
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(np.asarray(sizes[:-1], dtype=np.int64) ** 2)
    packed = np.zeros(int(offs[-1]) + int(sizes[-1]) ** 2, dtype=dtype)
    mats = []
    for i, n in enumerate(sizes):
        L = synth.lower_triangular(int(n), seed0 + i, dtype=dtype)
        packed[offs[i]:offs[i] + n * n] = L.ravel()
        mats.append(L)
    return packed, offs, mats


def run_both(lib, mode, sizes, packed, offs):
    import torch
    from paper_2307_07611_amd import _lib

    n_np = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    off_np = np.ascontiguousarray(offs)
    Ld = torch.from_numpy(packed).cuda()
    n_dev = torch.from_numpy(n_np).cuda()
    off_dev = torch.from_numpy(off_np).cuda()
    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    o.blocking = 1
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    batch = len(sizes)
    # the workspace entry point
    Xw = torch.full_like(Ld, float("nan"))
    sw = torch.full((batch,), 7, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(int(lib.trinv_batched_workspace_bytes(mode, batch, n_np.ctypes.data, ctypes.byref(o))), 1),
                     dtype=torch.uint8, device="cuda")
    st = lib.trinv_tril_inverse_batched(mode, batch, n_np.ctypes.data, n_dev.data_ptr(), off_np.ctypes.data,
                                        off_dev.data_ptr(), Ld.data_ptr(), Xw.data_ptr(), sw.data_ptr(),
                                        ctypes.byref(o), ws.data_ptr(), ws.numel(), stream)
    assert st == _lib.OK
    # the allocation-free one
    Xn = torch.full_like(Ld, float("nan"))
    sn = torch.full((batch,), 7, dtype=torch.int32, device="cuda")
    st = lib.trinv_tril_inverse_batched_noalloc(mode, batch, n_np.ctypes.data, n_dev.data_ptr(), off_np.ctypes.data,
                                                off_dev.data_ptr(), Ld.data_ptr(), Xn.data_ptr(), sn.data_ptr(),
                                                ctypes.byref(o), stream)
    assert st == _lib.OK
    torch.cuda.synchronize()
    return Xw.cpu().numpy(), sw.cpu().numpy(), Xn.cpu().numpy(), sn.cpu().numpy()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_workspace_entry_point(lib, dt):
    from paper_2307_07611_amd import _lib

    mode = _lib.F32 if dt == "f32" else _lib.F64
    dtype = np.float32 if dt == "f32" else np.float64
    first = list(synth.batch_sizes(600))  # uneven orders 16..512
    second = [1, 2, 17, 64, 129, 300, 5, 33]  # a smaller batch on the same scratch
    for k, sizes in enumerate((first, second)):
        banner(f"noalloc vs workspace {dt} call {k + 1}: {len(sizes)} matrices")
        packed, offs, mats = make(sizes, dtype, 4000 + 100 * k)
        Xw, sw, Xn, sn = run_both(lib, mode, sizes, packed, offs)
        np.testing.assert_array_equal(sn, sw)
        assert np.all(sn == 0)
        assert np.array_equal(Xn, Xw, equal_nan=False)
        for i in range(0, len(sizes), max(1, len(sizes) // 8)):
            n, o = int(sizes[i]), int(offs[i])
            Xo = oracle.tril_inverse(mats[i].astype(np.float64))
            err = np.linalg.norm(Xn[o:o + n * n].reshape(n, n) - Xo) / np.linalg.norm(Xo)
            assert err <= (1e-4 if dt == "f32" else 1e-11), (i, n, err)


def test_noalloc_limits(lib):
    from paper_2307_07611_amd import _lib

    n = np.array([16, 40], dtype=np.int32)
    off = np.array([0, 256], dtype=np.int64)
    call = lambda batch, L, X, nn=n: lib.trinv_tril_inverse_batched_noalloc(  # noqa: E731
        _lib.F32, batch, nn.ctypes.data, 4096, off.ctypes.data, 8192, L, X, 1 << 32, None, None)
    assert call(0, None, None) == _lib.OK
    assert call(-1, 1 << 30, 1 << 31) == _lib.ERR_ARG
    assert call(65537, 1 << 30, 1 << 31) == _lib.ERR_ARG  # above the scratch's plan capacity
    assert call(2, 1 << 30, (1 << 30) + 100) == _lib.ERR_ARG  # overlapping input and output
    bad = np.array([16, 2000], dtype=np.int32)
    assert call(2, 1 << 30, 1 << 31, bad) == _lib.ERR_ARG
