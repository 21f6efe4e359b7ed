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
    assert lib.isvd_profile_phases_read(None, None) == isvd.ISVD_E_INVALID
    lib.isvd_destroy_operator(None)


def test_graph_validation_before_any_device_work(lib):
    g = isvd._Graph(n=0, nnz=0)
    d = isvd._Design(form=0, K=1)
    h = ct.c_void_p()
    assert lib.isvd_create_operator(ct.byref(g), ct.byref(d), 1, None, ct.byref(h)) == isvd.ISVD_E_INVALID
    assert b"n > 0" in lib.isvd_last_error()


def test_symbolic_dag_shapes_and_validation_without_a_gpu(lib):
    # building dense leaves, sums, products, transposes and concatenations is
    # host bookkeeping (a dense leaf's pointer is only kept, never read here)
    i64 = ct.c_int64
    dag = ct.c_void_p()
    assert lib.isvd_dag_create(isvd.BF16, ct.byref(dag)) == isvd.ISVD_E_INVALID   # FP32 / FP64 only
    assert lib.isvd_dag_create(isvd.FP32, ct.byref(dag)) == isvd.ISVD_OK
    buf = (ct.c_float * 64)()
    ptr = ct.cast(buf, ct.c_void_p)

    def dense(r, c):
        out = i64()
        assert lib.isvd_dag_dense(dag, r, c, ptr, c, ct.byref(out)) == isvd.ISVD_OK
        return out.value

    def shape(node):
        r, c = i64(), i64()
        assert lib.isvd_dag_shape(dag, node, ct.byref(r), ct.byref(c)) == isvd.ISVD_OK
        return r.value, c.value

    def ids(*xs):
        return (i64 * len(xs))(*xs)

    a, b = dense(100, 7), dense(7, 5)          # shapes only: the leaf rows are never multiplied here
    out = i64()
    assert lib.isvd_dag_product(dag, 2, ids(a, b), ct.byref(out)) == isvd.ISVD_OK
    ab = out.value
    assert shape(ab) == (100, 5)
    assert lib.isvd_dag_transpose(dag, ab, ct.byref(out)) == isvd.ISVD_OK
    assert shape(out.value) == (5, 100)
    assert lib.isvd_dag_concat_cols(dag, 2, ids(a, ab), ct.byref(out)) == isvd.ISVD_OK
    assert shape(out.value) == (100, 12)
    w = (ct.c_double * 2)(1.0, -2.0)
    assert lib.isvd_dag_sum(dag, 2, ids(ab, ab), w, ct.byref(out)) == isvd.ISVD_OK
    assert shape(out.value) == (100, 5)
    # errors: inner dimensions, term shapes, concatenation rows, node ids, leaf widths
    assert lib.isvd_dag_product(dag, 2, ids(a, a), ct.byref(out)) == isvd.ISVD_E_INVALID
    assert lib.isvd_dag_sum(dag, 2, ids(a, ab), None, ct.byref(out)) == isvd.ISVD_E_INVALID
    assert lib.isvd_dag_concat_cols(dag, 2, ids(a, b), ct.byref(out)) == isvd.ISVD_E_INVALID
    assert lib.isvd_dag_transpose(dag, 999, ct.byref(out)) == isvd.ISVD_E_INVALID
    assert lib.isvd_dag_dense(dag, 10, 4096, ptr, 4096, ct.byref(out)) == isvd.ISVD_E_INVALID
    assert lib.isvd_dag_dense(dag, 10, 4, ptr, 3, ct.byref(out)) == isvd.ISVD_E_INVALID
    lib.isvd_dag_destroy(dag)


def test_learner_argument_errors_without_a_gpu(lib):
    # checks that fail before any device work
    p = ct.c_void_p(16)
    assert lib.isvd_ne_embeddings(10, 10, 4, isvd.BF16, p, 4, p, p, 4, p, 4, p, 4, None) == isvd.ISVD_E_INVALID
    assert lib.isvd_ne_scores(0, isvd.FP32, p, 4, 10, p, p, 4, 10, 1, p, p, p, None) == isvd.ISVD_E_INVALID
    assert lib.isvd_nc_fit(10, 10, 4, 2045, isvd.FP32, p, 4, p, p, 4, p, 2045, None, -1, 0.0, p, 2045,
                           None) == isvd.ISVD_E_INVALID                       # k + ny > 2048
    assert lib.isvd_nc_fit(10, 10, 4, 2, isvd.FP32, p, 4, p, p, 4, p, 2, None, 5, 0.0, p, 2,
                           None) == isvd.ISVD_E_INVALID                       # nsub > 0 without rows
    assert lib.isvd_orthonormalize_householder(3, 5, isvd.FP32, p, 5, None, None) == isvd.ISVD_E_INVALID


def test_binding_rejects_nodes_of_another_dag(lib):
    # a node id indexes one DAG's node store; handing it to another DAG must
    # fail in the binding instead of silently naming a different node
    buf = (ct.c_float * 64)()
    ptr = ct.cast(buf, ct.c_void_p)
    d1, d2 = isvd.Dag(isvd.FP32), isvd.Dag(isvd.FP32)
    a = d1._node(lib.isvd_dag_dense, 8, 8, ptr, 8)       # host pointer: shape bookkeeping only
    b = d2._node(lib.isvd_dag_dense, 8, 8, ptr, 8)
    assert d1.sum([a, a]).shape == (8, 8)
    for bad in (lambda: d1.sum([a, b]), lambda: d1.product([a, b]), lambda: d1.concat_cols([b]),
                lambda: a + b, lambda: a @ b, lambda: d1.operator(b)):
        with pytest.raises(ValueError):
            bad()
    d1.close()
    d2.close()
