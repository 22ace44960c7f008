"""C-ABI checks that need no GPU: the library loads, exports every function
that include/trinv.h declares, and its host-only calls (workspace queries,
argument validation, status strings) behave as documented."""

import ctypes
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
    assert (o.leaf, o.unit_diag, o.upper, o.max_iter, o.tol, o.blocking, o.check) == (0, 0, 0, 4, 1e-12, 0, 0)


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
    assert lib.trinv_factored_inverse(_lib.F64, 4, None, 0, None, 0, None, None, None, None, None, 0, None,
                                      None) == _lib.ERR_ARG
    assert lib.trinv_residual(_lib.F64, -2, None, 0, None, 0, None, 0, None, None) == _lib.ERR_ARG
