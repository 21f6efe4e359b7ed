"""Pins for the oracle's design-matrix products (CPU only).

The oracle is checked against things other than itself: closed-form
spectra of circulant graphs, brute-force enumeration of random walks on
tiny graphs, the adjoint identity and the weights printed in Fig. 1.
"""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.graph import adjacency, degrees, sym_normalized, transition
from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix, RowGather, context_weights
from synth import complete_graph, cycle_graph

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _explicit(op):
    """Columns of M obtained by products with the unit vectors."""
    return op.dot(np.eye(op.shape[1]))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("loops", [False, True])
def test_cycle_spectrum_closed_form(loops):
    # C_n is circulant: A has eigenvalues 2 cos(theta_j), theta_j = 2 pi j / n,
    # with the Fourier vectors as eigenvectors; so do T, 11^T and M.
    n, coeffs, lam = 24, np.array([0.5, 0.3, 0.2]), 0.07
    g = cycle_graph(n)
    m = NEDesignMatrix.from_graph(g, coeffs, lam, add_self_loops=loops)
    dense = _explicit(m)
    assert np.allclose(dense, dense.T, atol=1e-14)
    theta = 2 * np.pi * np.arange(n) / n
    a_eig = 2 * np.cos(theta) + (1.0 if loops else 0.0)
    t_eig = a_eig / (3.0 if loops else 2.0)
    ones_eig = np.where(np.arange(n) == 0, n, 0.0)
    mu = sum(c * t_eig ** (j + 1) for j, c in enumerate(coeffs)) - lam * (ones_eig - a_eig)
    got = np.sort(np.linalg.eigvalsh(dense))
    assert np.allclose(got, np.sort(mu), atol=1e-13)


def test_complete_graph_closed_form():
    # K_n: 11^T - A = I and T = (11^T - I)/(n-1), eigenvalues 1 and -1/(n-1).
    n, coeffs, lam = 9, np.array([0.2, 0.2, 0.2, 0.2, 0.2]), 0.3
    m = NEDesignMatrix.from_graph(complete_graph(n), coeffs, lam)
    got = np.sort(np.linalg.eigvalsh(_explicit(m)))
    top = coeffs.sum() - lam
    rest = sum(c * (-1.0 / (n - 1)) ** (j + 1) for j, c in enumerate(coeffs)) - lam
    want = np.sort(np.r_[top, np.full(n - 1, rest)])
    assert np.allclose(got, want, atol=1e-14)


def test_fig1_weights_are_printed_values():
    # Fig. 1 sets q1, q2, q3 = [3, 2, 1] / 6 for a window of 3.
    assert np.allclose(context_weights(3), np.array([3.0, 2.0, 1.0]) / 6.0, atol=0, rtol=0)
    for C in (3, 5, 10):
        assert abs(context_weights(C).sum() - 1.0) < 1e-15


def test_eq3_printed_weights_sum_to_one_over_C():
    # The weights as printed in Eq. 3, (2/((C+1)C)) (C-q+1)/C, sum to 1/C, not 1:
    # the reason the coefficients are taken as explicit inputs.
    for C in (3, 5, 10):
        w = [(2.0 / ((C + 1) * C)) * (C - q + 1) / C for q in range(1, C + 1)]
        assert abs(sum(w) - 1.0 / C) < 1e-15


# ---------------------------------------------------------------- brute force

def _tiny_directed_graph():
    # 6 nodes, weighted, directed; node 5 has no out-edges (zero degree).
    rows = [0, 0, 1, 1, 2, 2, 2, 3, 4, 4, 0]
    cols = [1, 3, 2, 4, 0, 3, 5, 4, 0, 5, 0]
    vals = [1.0, 2.0, 0.5, 1.5, 1.0, 3.0, 1.0, 2.0, 1.0, 0.25, 0.5]
    a = sp.csr_matrix((vals, (rows, cols)), shape=(6, 6))
    a.sum_duplicates()
    a.sort_indices()
    return a


def _walk_weight(a_dense, i, j, steps):
    """Sum over all walks i -> ... -> j of length `steps` of the product of
    transition probabilities A_uv / sum_w A_uw (zero from a node with no
    out-weight), by explicit enumeration."""
    n = a_dense.shape[0]
    out_w = [sum(a_dense[u, w] for w in range(n)) for u in range(n)]
    total = 0.0
    for mid in itertools.product(range(n), repeat=steps - 1):
        path = (i,) + mid + (j,)
        p = 1.0
        for u, v in zip(path[:-1], path[1:]):
            if out_w[u] == 0 or a_dense[u, v] == 0:
                p = 0.0
                break
            p *= a_dense[u, v] / out_w[u]
        total += p
    return total


def _brute_ne(a_dense, coeffs, lam):
    n = a_dense.shape[0]
    m = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for s, c in enumerate(coeffs, start=1):
                acc += c * _walk_weight(a_dense, i, j, s)
            acc -= lam * (1.0 - a_dense[i, j])
            m[i, j] = acc
    return m


def test_ne_product_matches_walk_enumeration():
    a = _tiny_directed_graph()
    coeffs, lam = np.array([0.5, -0.25, 0.125]), 0.3
    m = NEDesignMatrix(a, coeffs, lam)
    brute = _brute_ne(a.toarray(), coeffs, lam)
    assert np.allclose(_explicit(m), brute, atol=1e-14)
    assert np.allclose(_explicit(m.T), brute.T, atol=1e-14)
    assert m.T.T.transposed is False


def test_transition_rows_and_zero_degree():
    a = _tiny_directed_graph()
    t = transition(a).toarray()
    d = degrees(a)
    assert d[5] == 0
    assert np.all(t[5] == 0)
    assert np.allclose(t[:5].sum(axis=1), 1.0, atol=1e-15)


def test_adjoint_identity_random_weighted():
    rng = np.random.default_rng(3)
    n = 40
    a = sp.random(n, n, density=0.1, random_state=4, format="csr")
    m = NEDesignMatrix(a, rng.standard_normal(4), 0.2)
    y = rng.standard_normal((n, 3))
    z = rng.standard_normal((n, 3))
    lhs = np.sum(m.T.dot(y) * z)
    rhs = np.sum(y * m.dot(z))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_vector_and_block_products_agree():
    a = _tiny_directed_graph()
    m = NEDesignMatrix(a, [0.4, 0.6], 0.1)
    g = np.random.default_rng(0).standard_normal((6, 4))
    block = m.dot(g)
    for c in range(4):
        assert np.allclose(m.dot(g[:, c]), block[:, c], atol=1e-15)


# ---------------------------------------------------------------- featprop

def test_sym_normalized_entries_by_hand():
    a = _tiny_directed_graph()
    ad = a.toarray()
    n = ad.shape[0]
    d = ad.sum(axis=1)
    want = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            want[i, j] = (ad[i, j] + (1.0 if i == j else 0.0)) / np.sqrt((d[i] + 1) * (d[j] + 1))
    assert np.allclose(sym_normalized(a).toarray(), want, atol=1e-15)


def test_featprop_cycle_closed_form():
    # On C_n, A_hat = (A + I)/3 has eigenvector f_j = cos(theta_j i) with
    # eigenvalue (1 + 2 cos theta_j)/3, so [f, A_hat f, ..] = f (1, e, e^2, ..):
    # rank one with singular value |f| sqrt(sum_m e^(2m)).
    n, L, j = 30, 3, 4
    g = cycle_graph(n)
    theta = 2 * np.pi * j / n
    f = np.cos(theta * np.arange(n))[:, None]
    e = (1 + 2 * np.cos(theta)) / 3
    m = FeatPropDesignMatrix.from_graph(g, f, L)
    dense = _explicit(m)
    assert np.allclose(dense, f * (e ** np.arange(L + 1))[None, :], atol=1e-14)
    s = np.linalg.svd(dense, compute_uv=False)
    assert abs(s[0] - np.linalg.norm(f) * np.sqrt(np.sum(e ** (2 * np.arange(L + 1))))) < 1e-12
    assert s[1] < 1e-12


def test_featprop_adjoint_and_shape():
    rng = np.random.default_rng(5)
    n, d, L = 50, 3, 2
    a = sp.random(n, n, density=0.08, random_state=6, format="csr")
    a = ((a + a.T) > 0).astype(np.float64).tocsr()
    x = rng.standard_normal((n, d))
    m = FeatPropDesignMatrix(a, x, L)
    assert m.shape == (n, d * (L + 1)) and m.T.shape == (d * (L + 1), n)
    g = rng.standard_normal((d * (L + 1), 2))
    q = rng.standard_normal((n, 2))
    assert abs(np.sum(m.dot(g) * q) - np.sum(g * m.T.dot(q))) < 1e-10
    # block j of M is A_hat^j X, built here by repeated dense products
    ah = sym_normalized(a).toarray()
    dense = _explicit(m)
    p = x.copy()
    for j in range(L + 1):
        assert np.allclose(dense[:, j * d:(j + 1) * d], p, atol=1e-13)
        p = ah @ p


def test_adjacency_self_loops_enter_degree_and_lambda_term():
    g = cycle_graph(5)
    a = adjacency(g.n, g.indptr, g.indices, add_self_loops=True)
    assert np.allclose(degrees(a), 3.0)
    m = NEDesignMatrix(a, [1.0], 0.5)
    dense = _explicit(m)
    # diagonal: T_ii = 1/3, and the lambda term is 0 on looped nodes
    assert np.allclose(np.diag(dense), 1.0 / 3.0)
    # non-neighbours: -lambda
    assert abs(dense[0, 2] + 0.5) < 1e-15


@pytest.mark.parametrize("form", ["ne", "featprop"])
def test_row_gather_is_the_row_submatrix(form):
    # Section 3.2 option (ii): M[rows, :] without forming M; checked against
    # the explicit matrix built column by column from unit vectors
    rng = np.random.default_rng(11)
    n = 40
    a = sp.random(n, n, density=0.1, random_state=12, format="csr")
    a = ((a + a.T) > 0).astype(np.float64).tocsr()
    if form == "ne":
        m = NEDesignMatrix(a, [0.5, 0.3, 0.2], 0.07)
    else:
        m = FeatPropDesignMatrix(a, rng.standard_normal((n, 3)), 2)
    rows = rng.choice(n, 13, replace=False)
    sub = RowGather(m, rows)
    assert sub.shape == (13, m.shape[1]) and sub.T.shape == (m.shape[1], 13)
    full = _explicit(m)
    assert np.allclose(_explicit(sub), full[rows], atol=1e-13)
    assert np.allclose(_explicit(sub.T), full[rows].T, atol=1e-13)
    # repeated rows are refused (the transpose scatters without adding)
    with pytest.raises(AssertionError):
        RowGather(m, [1, 2, 1])
