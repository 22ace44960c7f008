"""C-ABI checks that need no GPU: the library loads, exports every function
that include/trinv.h declares, and its host-only calls (workspace queries,
argument validation, status strings) behave as documented."""

import ctypes

import numpy as np
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "trinv.h")
LIB = os.path.join(ROOT, "paper_2307_07611_amd", "libtrinv.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trinv_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2307_07611_amd.build as b

        b.build()
    from paper_2307_07611_amd import _lib

    return _lib.load()


def test_header_declares_the_four_calls():
    fns = declared_functions()
    for name in ("trinv_tril_inverse", "trinv_tril_inverse_batched", "trinv_tril_inverse_backward",
                 "trinv_factored_inverse"):
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    from paper_2307_07611_amd import _lib

    fns = declared_functions()
    assert sorted(_lib.EXPORTS) == fns
    for name in fns:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    from paper_2307_07611_amd import _lib

    assert _lib.status_string(0) == "ok"
    assert "singular" in _lib.status_string(_lib.ERR_SINGULAR)
    assert _lib.status_string(99) == "unknown status"


def test_default_opts(lib):
    from paper_2307_07611_amd import _lib

    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    assert (o.leaf, o.unit_diag, o.upper, o.max_iter, o.tol, o.blocking, o.check, o.beta, o.resid) == \
        (0, 0, 0, 4, 1e-12, 0, 0, 0, _lib.RESID_AUTO)


def test_workspace_queries(lib):
    from paper_2307_07611_amd import _lib

    assert lib.trinv_workspace_bytes(_lib.F64, 0, None) == 0
    # T workspace of the top level: (n/2)^2 elements
    w = lib.trinv_workspace_bytes(_lib.F64, 1024, None)
    assert 512 * 512 * 8 <= w < 512 * 512 * 8 + 64 * 1024
    w32 = lib.trinv_workspace_bytes(_lib.F32, 1024, None)
    assert 512 * 512 * 4 <= w32 < 512 * 512 * 4 + 64 * 1024
    assert lib.trinv_backward_workspace_bytes(_lib.F32, 4, 100) >= 4 * 100 * 100 * 4
    assert lib.trinv_residual_workspace_bytes(_lib.F64, 300) > 0


def test_argument_errors_before_any_launch(lib):
    from paper_2307_07611_amd import _lib

    info = _lib.Info()
    # n < 0, ld < n, NULL pointers and unknown modes are rejected on the host
    assert lib.trinv_tril_inverse(_lib.F64, -1, None, 0, None, 0, None, None, 0, None, ctypes.byref(info)) == \
        _lib.ERR_ARG
    assert lib.trinv_tril_inverse(_lib.F64, 10, 8, 5, 16, 10, None, None, 0, None, None) == _lib.ERR_ARG
    assert lib.trinv_tril_inverse(_lib.F64, 10, None, 10, None, 10, None, None, 0, None, None) == _lib.ERR_ARG
    assert lib.trinv_tril_inverse(9, 10, 8, 10, 4096, 10, None, None, 0, None, None) == _lib.ERR_UNSUPPORTED
    # overlapping input and output
    assert lib.trinv_tril_inverse(_lib.F64, 10, 4096, 10, 4096 + 8, 10, None, None, 0, None, None) == _lib.ERR_ARG
    # n == 0 is a no-op
    assert lib.trinv_tril_inverse(_lib.F64, 0, None, 0, None, 0, None, None, 0, None, ctypes.byref(info)) == _lib.OK
    assert info.rel_residual == -1.0 and info.first_bad_index == 0
    assert lib.trinv_tril_inverse_backward(_lib.F64, 1, 4, None, None, None, 16, None, 0, None) == _lib.ERR_ARG
    assert lib.trinv_tril_inverse_backward(_lib.F64, 1, 4, 4096, 8192, 16384, 8, None, 0, None) == _lib.ERR_ARG
    fac = lambda n, L, ldl, U, ldu, Li, ldli, Ui, ldui, Ai, ldai: lib.trinv_factored_inverse(  # noqa: E731
        _lib.F64, n, L, ldl, 0, U, ldu, 0, Li, ldli, Ui, ldui, Ai, ldai, None, None, 0, None, None)
    assert fac(4, None, 4, None, 4, None, 4, None, 4, None, 4) == _lib.ERR_ARG
    A, B, C, D, E = 1 << 30, 1 << 31, 1 << 32, 1 << 33, 1 << 34
    assert fac(4, A, 3, B, 4, C, 4, D, 4, None, 0) == _lib.ERR_ARG   # ldl < n
    assert fac(4, A, 4, B, 4, C, 4, D, 3, None, 0) == _lib.ERR_ARG   # ldui < n
    assert fac(4, A, 4, B, 4, C, 4, D, 4, E, 2) == _lib.ERR_ARG      # ldai < n with Ainv
    assert fac(4, A, 4, B, 4, C, 4, D, 4, None, 0) == _lib.ERR_WORKSPACE  # ldai ignored without Ainv
    # an output overlapping an input through a leading dimension larger than n
    assert fac(4, A, 64, B, 4, A + 8 * 5, 4, D, 4, None, 0) == _lib.ERR_ARG
    assert fac(4, A, 4, B, 4, C, 4, C + 8, 4, None, 0) == _lib.ERR_ARG  # outputs overlap
    assert lib.trinv_residual(_lib.F64, -2, None, 0, None, 0, None, 0, None, None) == _lib.ERR_ARG


def test_refine_options_before_any_launch(lib):
    """The residual-precision option is validated, and refine orders whose
    low-precision planes would need more than 32-bit per-lane offsets within a
    256-row panel are rejected (workspace query 0, call UNSUPPORTED) before
    anything is launched."""
    from paper_2307_07611_amd import _lib

    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    o.resid = 3
    assert lib.trinv_tril_inverse(_lib.BF16_REFINE, 64, 1 << 30, 64, 1 << 34, 64, ctypes.byref(o), None, 0, None,
                                  None) == _lib.ERR_ARG
    o.resid = -1
    assert lib.trinv_tril_inverse(_lib.F64, 64, 1 << 30, 64, 1 << 34, 64, ctypes.byref(o), None, 0, None,
                                  None) == _lib.ERR_ARG
    for r in (_lib.RESID_AUTO, _lib.RESID_SPLIT, _lib.RESID_FP64):  # valid, but no workspace
        o.resid = r
        assert lib.trinv_tril_inverse(_lib.BF16_REFINE, 64, 1 << 30, 64, 1 << 34, 64, ctypes.byref(o), None, 0,
                                      None, None) == _lib.ERR_WORKSPACE
    big = (1 << 23) - 127  # first unsupported order
    assert lib.trinv_workspace_bytes(_lib.BF16_REFINE, big, None) == 0
    assert lib.trinv_workspace_bytes(_lib.F16_REFINE, big + 1000, None) == 0
    assert lib.trinv_refine_residual_workspace_bytes(_lib.BF16_REFINE, big) == 0
    L, X = 1 << 40, (1 << 40) + 8 * big * big + 4096
    assert lib.trinv_tril_inverse(_lib.BF16_REFINE, big, L, big, X, big, None, 1 << 20, 1 << 20, None, None) == \
        _lib.ERR_UNSUPPORTED
    # orders past the old 32-bit wrap of whole-plane offsets (2 n^2 >= 2^32) are supported
    assert lib.trinv_workspace_bytes(_lib.BF16_REFINE, 46341, None) > 6 * 2 * 46341 * 46341
    assert lib.trinv_workspace_bytes(_lib.BF16_REFINE, big - 1, None) > 0
    out = (ctypes.c_double * 5)()
    rr = lambda mode, n, L, X, nsplit, R, ldr: lib.trinv_refine_residual(  # noqa: E731
        mode, n, L, n, X, n, nsplit, R, ldr, None, 0, None, out)
    assert rr(_lib.BF16_REFINE, -1, 1 << 30, 1 << 34, 3, 1 << 36, 1) == _lib.ERR_ARG
    assert rr(_lib.BF16_REFINE, 0, None, None, 3, None, 0) == _lib.OK
    assert rr(_lib.F64, 64, 1 << 30, 1 << 34, 3, 1 << 36, 64) == _lib.ERR_UNSUPPORTED
    assert rr(_lib.BF16_REFINE, 64, 1 << 30, 1 << 34, 4, 1 << 36, 64) == _lib.ERR_ARG
    assert rr(_lib.BF16_REFINE, 64, 1 << 30, 1 << 34, 3, 1 << 36, 63) == _lib.ERR_ARG
    assert rr(_lib.BF16_REFINE, 64, 1 << 30, 1 << 34, 3, (1 << 30) + 8, 64) == _lib.ERR_ARG  # R overlaps L
    assert rr(_lib.F16_REFINE, 64, 1 << 30, 1 << 34, 2, 1 << 36, 64) == _lib.ERR_WORKSPACE
    assert lib.trinv_refine_residual(_lib.BF16_REFINE, 64, 1 << 30, 64, 1 << 34, 64, 3, 1 << 36, 64, None, 0, None,
                                     None) == _lib.ERR_ARG


def test_batched_argument_errors_before_any_launch(lib):
    from paper_2307_07611_amd import _lib

    n = np.array([16, 40, 7], dtype=np.int32)
    off = np.array([0, 256, 256 + 1600], dtype=np.int64)
    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    call = lambda mode, batch, n_arr, off_arr, L, X, st, opts: lib.trinv_tril_inverse_batched(  # noqa: E731
        mode, batch, n_arr.ctypes.data, 4096, off_arr.ctypes.data, 8192, L, X, st, ctypes.byref(opts), 1 << 20,
        1 << 20, None)
    assert lib.trinv_tril_inverse_batched(_lib.F32, 0, None, None, None, None, None, None, None, None, None, 0,
                                          None) == _lib.OK
    assert call(_lib.F32, -1, n, off, 1 << 30, 1 << 31, 1 << 32, o) == _lib.ERR_ARG
    assert call(_lib.BF16_REFINE, 3, n, off, 1 << 30, 1 << 31, 1 << 32, o) == _lib.ERR_UNSUPPORTED
    bad = n.copy()
    bad[1] = 0
    assert call(_lib.F32, 3, bad, off, 1 << 30, 1 << 31, 1 << 32, o) == _lib.ERR_ARG
    bad[1] = 1025
    assert call(_lib.F32, 3, bad, off, 1 << 30, 1 << 31, 1 << 32, o) == _lib.ERR_ARG
    neg = off.copy()
    neg[2] = -5
    assert call(_lib.F32, 3, n, neg, 1 << 30, 1 << 31, 1 << 32, o) == _lib.ERR_ARG
    # input and output ranges overlap (extent 1649 elements of 4 bytes)
    assert call(_lib.F32, 3, n, off, 1 << 30, (1 << 30) + 4000, 1 << 32, o) == _lib.ERR_ARG
    up = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(up))
    up.upper = 1
    # upper input: staged through transposes in the workspace, which grows by
    # two densely packed copies of the batch and the dense offsets
    w_lo = lib.trinv_batched_workspace_bytes(_lib.F32, 3, n.ctypes.data, ctypes.byref(o))
    w_up = lib.trinv_batched_workspace_bytes(_lib.F32, 3, n.ctypes.data, ctypes.byref(up))
    assert w_up >= w_lo + 2 * 4 * int((n.astype(np.int64) ** 2).sum()) + 8 * 3
    assert lib.trinv_tril_inverse_batched(_lib.F32, 3, n.ctypes.data, 4096, off.ctypes.data, 8192, 1 << 30,
                                          1 << 31, 1 << 32, ctypes.byref(up), 1 << 20, w_lo, None) == \
        _lib.ERR_WORKSPACE
    assert lib.trinv_tril_inverse_batched_noalloc(_lib.F32, 3, n.ctypes.data, 4096, off.ctypes.data, 8192, 1 << 30,
                                                  1 << 31, 1 << 32, ctypes.byref(up), None) == _lib.ERR_UNSUPPORTED
    lf = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(lf))
    for leaf in (16, 128):  # the persistent launch takes leaf 0, 32 or 64
        lf.leaf = leaf
        assert call(_lib.F32, 3, n, off, 1 << 30, 1 << 31, 1 << 32, lf) == _lib.ERR_ARG
    # too small a workspace
    assert lib.trinv_tril_inverse_batched(_lib.F32, 3, n.ctypes.data, 4096, off.ctypes.data, 8192, 1 << 30,
                                          1 << 31, 1 << 32, ctypes.byref(o), 1 << 20, 8, None) == \
        _lib.ERR_WORKSPACE
    assert lib.trinv_batched_workspace_bytes(_lib.F32, 3, n.ctypes.data, ctypes.byref(o)) >= 3 * 4 + 4


def test_combrit_argument_errors_before_any_launch(lib):
    from paper_2307_07611_amd import _lib

    def call(mode, n, ldl, ldx, **kw):
        o = _lib.Opts()
        lib.trinv_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return lib.trinv_tril_inverse(mode, n, 1 << 30, ldl, 1 << 34, ldx, ctypes.byref(o), None, 0, None, None)

    assert call(_lib.F64, 1000, 1000, 1000, beta=1) == _lib.ERR_ARG
    assert call(_lib.F64, 1000, 1000, 1000, beta=-2) == _lib.ERR_ARG
    assert call(_lib.F64, 1088, 1088, 1088, beta=17) == _lib.ERR_ARG
    assert call(_lib.F64, 1000, 1000, 1000, beta=3) == _lib.ERR_ARG        # 1000 % 3 != 0
    assert call(_lib.F64, 1024, 1024, 1030, beta=4) == _lib.ERR_ARG        # ldl != ldx
    assert call(_lib.F64, 1024, 1024, 1024, beta=4, upper=1) == _lib.ERR_UNSUPPORTED
    assert call(_lib.BF16_REFINE, 1024, 1024, 1024, beta=4) == _lib.ERR_UNSUPPORTED
    assert call(_lib.F64, 1024, 1024, 1024, beta=4) == _lib.ERR_WORKSPACE  # valid, but no workspace
    w2 = lib.trinv_workspace_bytes(_lib.F64, 1024, None)
    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    o.beta = 4
    w4 = lib.trinv_workspace_bytes(_lib.F64, 1024, ctypes.byref(o))
    assert w4 >= 2 * 1024 * 1024 * 8 > w2  # B and its inverse, n x n each


def test_sqr_brsi_argument_errors_before_any_launch(lib):
    from paper_2307_07611_amd import _lib

    o = _lib.Opts()
    lib.trinv_default_opts(ctypes.byref(o))
    A, Q, R, S, X = 1 << 30, 1 << 34, 1 << 35, 1 << 36, 1 << 37

    def sqr(mode, n, **kw):
        oo = _lib.Opts()
        lib.trinv_default_opts(ctypes.byref(oo))
        for k, v in kw.items():
            setattr(oo, k, v)
        return lib.trinv_sqr(mode, n, A, Q, R, S, X, ctypes.byref(oo), None, 0, None, None)

    assert sqr(_lib.F64, -1) == _lib.ERR_ARG
    assert sqr(_lib.F64, 0) == _lib.OK
    assert lib.trinv_sqr(_lib.F64, 10, A, None, R, S, X, ctypes.byref(o), None, 0, None, None) == _lib.ERR_ARG
    assert lib.trinv_sqr(_lib.F64, 10, A, A + 8, R, S, X, ctypes.byref(o), None, 0, None, None) == _lib.ERR_ARG
    assert sqr(_lib.BF16_REFINE, 10) == _lib.ERR_UNSUPPORTED
    assert sqr(_lib.F64, 4097) == _lib.ERR_UNSUPPORTED
    assert sqr(_lib.F64, 100, upper=1) == _lib.ERR_UNSUPPORTED
    assert sqr(_lib.F64, 100) == _lib.ERR_WORKSPACE
    assert lib.trinv_sqr_workspace_bytes(_lib.F64, 1000, None) >= 1000 * 1000 * 8

    def brsi(mode, n, lda, ldx, **kw):
        oo = _lib.Opts()
        lib.trinv_default_opts(ctypes.byref(oo))
        for k, v in kw.items():
            setattr(oo, k, v)
        return lib.trinv_brsi(mode, n, A, lda, X, ldx, ctypes.byref(oo), None, 0, None, None)

    assert brsi(_lib.F64, -1, 1, 1) == _lib.ERR_ARG
    assert brsi(_lib.F64, 0, 0, 0) == _lib.OK
    assert brsi(_lib.F64, 100, 99, 100) == _lib.ERR_ARG
    assert brsi(_lib.F64, 100, 100, 99) == _lib.ERR_ARG
    assert lib.trinv_brsi(_lib.F64, 100, A, 100, A + 800, 100, ctypes.byref(o), None, 0, None, None) == _lib.ERR_ARG
    assert brsi(_lib.F16_REFINE, 100, 100, 100) == _lib.ERR_UNSUPPORTED
    assert brsi(_lib.F64, 100, 100, 100, unit_diag=1) == _lib.ERR_UNSUPPORTED
    assert brsi(_lib.F64, 100, 100, 100) == _lib.ERR_WORKSPACE
    # about 4 n^2 elements for n = b 2^k; padded orders round up
    w = lib.trinv_brsi_workspace_bytes(_lib.F64, 1024, None)
    assert 3 * 1024 * 1024 * 8 <= w <= 5 * 1024 * 1024 * 8
    assert lib.trinv_brsi_workspace_bytes(_lib.F64, 129, None) >= 2 * 130 * 130 * 8


def test_batched_tuner_argument_errors(lib):
    """The autotuner validates like the batched call; pinning a configuration
    checks its fields (no launch in either)."""
    from paper_2307_07611_amd import _lib

    cfg = _lib.BatchedConfig(64, 0, -1.0)
    sizes = np.array([16, 300, 1024], dtype=np.int32)
    assert lib.trinv_batched_set_config(_lib.F32, 3, sizes.ctypes.data, ctypes.byref(cfg)) == _lib.OK
    bad = _lib.BatchedConfig(16, 0, -1.0)
    assert lib.trinv_batched_set_config(_lib.F32, 3, sizes.ctypes.data, ctypes.byref(bad)) == _lib.ERR_ARG
    assert lib.trinv_batched_set_config(_lib.F32, 3, None, ctypes.byref(cfg)) == _lib.ERR_ARG
    assert lib.trinv_batched_set_config(_lib.BF16_REFINE, 3, sizes.ctypes.data, ctypes.byref(cfg)) == \
        _lib.ERR_UNSUPPORTED
    big = np.array([16, 2000], dtype=np.int32)
    assert lib.trinv_batched_set_config(_lib.F32, 2, big.ctypes.data, ctypes.byref(cfg)) == _lib.ERR_ARG
    out = _lib.BatchedConfig()
    assert lib.trinv_batched_autotune(_lib.F32, 0, None, None, None, None, None, None, None, None, None, 0, None,
                                      ctypes.byref(out)) == _lib.OK
    assert out.ms == -1.0
    assert lib.trinv_batched_autotune(_lib.F32, 3, None, None, None, None, None, None, None, None, None, 0, None,
                                      ctypes.byref(out)) == _lib.ERR_ARG


def test_batched_get_config_host_side(lib):
    """trinv_batched_get_config: argument errors, and the defaults for a
    signature nothing has set (no device needed)."""
    import numpy as np

    from paper_2307_07611_amd import _lib

    n = np.array([5, 64, 100], dtype=np.int32)
    cfg = _lib.BatchedConfig()
    assert lib.trinv_batched_get_config(_lib.F32, 0, n.ctypes.data, ctypes.byref(cfg)) == _lib.ERR_ARG
    assert lib.trinv_batched_get_config(_lib.F32, 3, None, ctypes.byref(cfg)) == _lib.ERR_ARG
    assert lib.trinv_batched_get_config(_lib.F32, 3, n.ctypes.data, None) == _lib.ERR_ARG
    assert lib.trinv_batched_get_config(_lib.BF16_REFINE, 3, n.ctypes.data, ctypes.byref(cfg)) == \
        _lib.ERR_UNSUPPORTED
    bad = np.array([5, 2000, 100], dtype=np.int32)
    assert lib.trinv_batched_get_config(_lib.F32, 3, bad.ctypes.data, ctypes.byref(cfg)) == _lib.ERR_ARG
    assert lib.trinv_batched_get_config(_lib.F32, 3, n.ctypes.data, ctypes.byref(cfg)) == _lib.OK
    assert (cfg.leaf, cfg.wgs_per_cu, cfg.ms, cfg.tile) == (64, 0, -1.0, 128)
    assert lib.trinv_batched_get_config(_lib.F64, 3, n.ctypes.data, ctypes.byref(cfg)) == _lib.OK
    assert (cfg.leaf, cfg.wgs_per_cu) == (32, 0)
    # set_config pins a signature for the rest of the process
    pin = _lib.BatchedConfig(32, 2, -1.0, 64)
    assert lib.trinv_batched_set_config(_lib.F32, 3, n.ctypes.data, ctypes.byref(pin)) == _lib.OK
    assert lib.trinv_batched_get_config(_lib.F32, 3, n.ctypes.data, ctypes.byref(cfg)) == _lib.OK
    assert (cfg.leaf, cfg.wgs_per_cu, cfg.tile) == (32, 2, 64)
    bad_tile = _lib.BatchedConfig(32, 2, -1.0, 96)
    assert lib.trinv_batched_set_config(_lib.F32, 3, n.ctypes.data, ctypes.byref(bad_tile)) == _lib.ERR_ARG


def test_profile_select_host_side(lib):
    """Class selection parses a comma-separated list (empty names ignored);
    NULL restores every class. No launch happens, so the profile stays empty."""
    assert lib.trinv_profile_select(b"bf16_residual,,f64_level_T,") == 0
    assert lib.trinv_profile_enable(1) == 0
    assert lib.trinv_profile_read(None, 0) == 0
    assert lib.trinv_profile_enable(0) == 0
    assert lib.trinv_profile_select(None) == 0
    assert lib.trinv_profile_select(b"") == 0
