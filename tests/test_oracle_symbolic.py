"""Pins for the oracle's symbolic DAG (CPU only): every node type against
the explicit matrix it stands for, built by dense NumPy algebra; the Fig. 1
construction against the NE design matrix; the feature form as a
concatenation against the feature-propagation matrix."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.graph import adjacency, degrees, sym_normalized, transition
from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix
from oracle import symbolic as sym
from synth import sbm_graph


def _check(pf, explicit, rng):
    explicit = np.asarray(explicit, dtype=np.float64)
    assert pf.shape == explicit.shape and pf.T.shape == explicit.T.shape
    g = rng.standard_normal((explicit.shape[1], 3))
    q = rng.standard_normal((explicit.shape[0], 3))
    assert np.allclose(pf.dot(g), explicit @ g, atol=1e-12)
    assert np.allclose(pf.T.dot(q), explicit.T @ q, atol=1e-12)
    assert np.allclose(pf.dense(), explicit, atol=1e-12)


def test_every_node_against_dense_algebra():
    rng = np.random.default_rng(0)
    a = sp.random(12, 9, density=0.3, random_state=1, format="csr")
    b = rng.standard_normal((9, 12))
    c = sp.random(12, 12, density=0.25, random_state=2, format="csr")
    d = rng.uniform(0.5, 2.0, 12)
    A, B, C, D = sym.sparse(a), sym.dense(b), sym.sparse(c), sym.diag(d)
    ad, cd = a.toarray(), c.toarray()
    _check(A, ad, rng)
    _check(B, b, rng)
    _check(D, np.diag(d), rng)
    _check(A @ B, ad @ b, rng)
    _check(A @ B + 2.5 * C, ad @ b + 2.5 * cd, rng)
    _check(C - D, cd - np.diag(d), rng)
    _check(C ** 3, cd @ cd @ cd, rng)
    _check((A @ B).T, (ad @ b).T, rng)
    _check(D @ C @ D, np.diag(d) @ cd @ np.diag(d), rng)
    rows = rng.choice(12, 5, replace=False)
    _check(sym.take_rows(C @ A, rows), (cd @ ad)[rows], rng)
    _check(sym.take_rows(C @ A, rows).T, (cd @ ad)[rows].T, rng)
    _check(sym.hstack([A, C, D]), np.hstack([ad, cd, np.diag(d)]), rng)
    _check(sym.vstack([B, A.T]), np.vstack([b, ad.T]), rng)
    _check(sym.chain([sym.hstack([A, C]), sym.vstack([B, C])]), np.hstack([ad, cd]) @ np.vstack([b, cd]), rng)
    _check(sym.lincomb([A @ B, C @ C], [0.3, -0.7]).T, (0.3 * ad @ b - 0.7 * cd @ cd).T, rng)


def test_fig1_construction_is_the_ne_design_matrix():
    # Fig. 1: t = D^-1 A, row1 = a ones row, M = q1 t + q2 t@t + q3 t@t@t - lambda (row1^T row1 - A)
    g = sbm_graph(60, 3, 0.15, 0.02, seed=3)
    a = adjacency(g.n, g.indptr, g.indices)
    t = sym.sparse(transition(a))
    A = sym.sparse(a)
    row1 = sym.dense(np.ones((1, g.n)))
    q1, q2, q3 = np.array([3, 2, 1]) / 6.0
    lam = 0.07
    m = q1 * t + q2 * (t @ t) + q3 * (t @ t @ t)
    m = m - lam * (row1.T @ row1 - A)
    ref = NEDesignMatrix(a, [q1, q2, q3], lam)
    rng = np.random.default_rng(4)
    for pf, op in ((m, ref), (m.T, ref.T)):
        y = rng.standard_normal((g.n, 4))
        assert np.allclose(pf.dot(y), op.dot(y), atol=1e-12)


def test_feature_form_as_a_concatenation():
    g = sbm_graph(50, 2, 0.2, 0.03, seed=5)
    x = np.random.default_rng(6).standard_normal((50, 3))
    a = adjacency(g.n, g.indptr, g.indices)
    ah = sym.sparse(sym_normalized(a))
    X = sym.dense(x)
    m = sym.hstack([X] + [(ah ** j) @ X for j in range(1, 4)])
    ref = FeatPropDesignMatrix(a, x, 3)
    assert np.allclose(m.dense(), ref.dense(), atol=1e-12)


def test_degree_diagonal_matches_transition():
    g = sbm_graph(40, 2, 0.2, 0.05, seed=7)
    a = adjacency(g.n, g.indptr, g.indices)
    dg = degrees(a)
    dinv = np.where(dg > 0, 1.0 / np.where(dg > 0, dg, 1.0), 0.0)
    m = sym.diag(dinv) @ sym.sparse(a)
    assert np.allclose(m.dense(), transition(a).toarray(), atol=1e-14)


def test_shape_mismatch_is_refused():
    with pytest.raises(ValueError):
        sym.chain([sym.dense(np.ones((3, 4))), sym.dense(np.ones((3, 4)))])
    with pytest.raises(ValueError):
        sym.lincomb([sym.dense(np.ones((3, 4))), sym.dense(np.ones((4, 3)))])
    with pytest.raises(ValueError):
        sym.power(sym.dense(np.ones((3, 3))), 0)
    with pytest.raises(ValueError):
        sym.power(sym.dense(np.ones((3, 4))), 2)
    with pytest.raises(ValueError):
        sym.take_rows(sym.dense(np.ones((3, 3))), [0, 0])


def test_label_reuse_operator_has_a_zero_diagonal():
    # Section 5.3 (label re-use): A_hat - (D + I)^-1 zeroes the diagonal of A_hat,
    # so row i of (A_hat - (D+I)^-1) Y_train never sees label i
    g = sbm_graph(80, 3, 0.1, 0.02, seed=9)
    a = adjacency(g.n, g.indptr, g.indices)
    dg = degrees(a)
    b = sym.sparse(sym_normalized(a)) - sym.diag(1.0 / (dg + 1.0))
    dense = b.dense()
    assert np.abs(np.diag(dense)).max() < 1e-15
    y = np.eye(g.n)[:, :5]
    assert np.allclose(b.dot(y)[np.arange(5), np.arange(5)], 0.0, atol=1e-15)
    # off the diagonal it is A_hat itself
    off = ~np.eye(g.n, dtype=bool)
    assert np.allclose(dense[off], sym_normalized(a).toarray()[off], atol=1e-15)


def test_symmetric_ne_variant_is_symmetric():
    # replacing T by A_hat (Section 3.1) gives a symmetric M on an undirected graph
    g = sbm_graph(60, 3, 0.15, 0.02, seed=10)
    a = adjacency(g.n, g.indptr, g.indices)
    ah = sym.sparse(sym_normalized(a))
    one = sym.dense(np.ones((g.n, 1)))
    m = sym.lincomb([ah ** j for j in (1, 2, 3)], [0.5, 0.3, 0.2]) - 0.05 * (one @ one.T - sym.sparse(a))
    dense = m.dense()
    assert np.allclose(dense, dense.T, atol=1e-14)
