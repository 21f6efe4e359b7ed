"""The C-ABI library loads and exports every symbol include/isvd.h declares
(CPU only: no call here reaches the GPU)."""

import ctypes as ct
import os

import pytest

from paper_2111_06312_amd import isvd

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2111_06312_amd",
                   "libisvd.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libisvd.so not built (run __graft_entry__.build())")
    return isvd.load()


def test_every_header_symbol_is_exported(lib):
    names = isvd.exported_symbols_from_header()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.isvd_version()
    for code in range(7):
        assert len(lib.isvd_status_string(code)) > 0
    assert lib.isvd_status_string(99) == b"unknown status"


def test_argument_errors_are_reported_without_a_gpu(lib):
    h = ct.c_void_p()
    assert lib.isvd_create_operator(None, None, 1, None, ct.byref(h)) == isvd.ISVD_E_INVALID
    assert b"null" in lib.isvd_last_error()
    r, c = ct.c_int64(), ct.c_int64()
    assert lib.isvd_operator_shape(None, ct.byref(r), ct.byref(c)) == isvd.ISVD_E_INVALID
    assert lib.isvd_truncated_svd(None, None, None, 0, None, None, 0, None, None) == isvd.ISVD_E_INVALID
    assert lib.isvd_matmul_block(None, 0, None, 1, 1, None, 1, None) == isvd.ISVD_E_INVALID
    assert lib.isvd_small_svd(0, None, None, None, None, None) == isvd.ISVD_E_INVALID
    lib.isvd_destroy_operator(None)


def test_graph_validation_before_any_device_work(lib):
    g = isvd._Graph(n=0, nnz=0)
    d = isvd._Design(form=0, K=1)
    h = ct.c_void_p()
    assert lib.isvd_create_operator(ct.byref(g), ct.byref(d), 1, None, ct.byref(h)) == isvd.ISVD_E_INVALID
    assert b"n > 0" in lib.isvd_last_error()
