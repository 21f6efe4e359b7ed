"""Pins for the oracle's Algorithm 1 / Algorithm 2 and residual (CPU only).

Pins: exact recovery when k >= rank (Section 2.3, Eckart-Young with zero
error), closed-form spectra of circulant graphs, Eckart-Young's lower
bound and singular-value interlacing against LAPACK's SVD of the
explicit matrix, orthonormality, span equality of the two Algorithm 2
routines (its footnote), and a zero residual at an exact SVD.
"""

import numpy as np
import pytest

from oracle.isvd import (canonical_signs, isvd, orthonorm_cholesky, orthonorm_qr,
                         principal_angles, triplet_residuals)
from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix
from synth import cycle_graph, gaussian_block, sbm_graph


class _Dense:
    """A plain explicit matrix with the symbolic interface (test helper)."""

    def __init__(self, m):
        self.m = m
        self.shape = m.shape

    def dot(self, g):
        return self.m @ g

    @property
    def T(self):
        return _Dense(self.m.T)


def _known_matrix(r, c, sig, seed):
    rng = np.random.default_rng(seed)
    u0, _ = np.linalg.qr(rng.standard_normal((r, len(sig))))
    v0, _ = np.linalg.qr(rng.standard_normal((c, len(sig))))
    return u0 @ np.diag(sig) @ v0.T, u0, v0


def test_exact_when_k_reaches_rank_featprop_L0():
    # M^(NC) with L = 0 is X itself; with k = rank(X) = d the range finder
    # captures range(X) exactly and the SVD is exact (zero Frobenius error).
    sig = np.array([9.0, 5.0, 4.0, 2.5, 1.0, 0.5])
    x, u0, v0 = _known_matrix(80, 6, sig, seed=1)
    g = cycle_graph(80)
    m = FeatPropDesignMatrix.from_graph(g, x, L=0)
    u, s, v = isvd(m, 6, gaussian_block(6, 6, seed=2), iterations=0)
    assert np.allclose(s, sig, rtol=1e-13)
    assert np.allclose(u @ np.diag(s) @ v.T, x, atol=1e-12)
    assert principal_angles(u, u0).max() < 1e-12
    assert principal_angles(v, v0).max() < 1e-12


def test_exact_low_rank_with_oversampling():
    sig = np.array([10.0, 3.0, 1.0])
    x, _, _ = _known_matrix(50, 40, sig, seed=7)
    u, s, v = isvd(_Dense(x), 3, gaussian_block(40, 8, seed=8), iterations=1)
    assert np.allclose(s, sig, rtol=1e-12)
    assert np.linalg.norm(x - u @ np.diag(s) @ v.T) < 1e-12


def test_cycle_top_singular_values_closed_form():
    n, coeffs, lam = 64, np.full(4, 0.25), 0.05
    m = NEDesignMatrix.from_graph(cycle_graph(n), coeffs, lam)
    theta = 2 * np.pi * np.arange(n) / n
    t_eig = np.cos(theta)
    mu = sum(c * t_eig ** (j + 1) for j, c in enumerate(coeffs)) \
        - lam * (np.where(np.arange(n) == 0, n, 0.0) - 2 * np.cos(theta))
    want = np.sort(np.abs(mu))[::-1]
    k = 5   # sigma_1 plus two complete pairs (Fourier modes j and n-j are degenerate)
    u, s, v = isvd(m, k, gaussian_block(n, 12, seed=3), iterations=40)
    assert np.allclose(s, want[:k], rtol=1e-10)
    rho, _ = triplet_residuals(m, u, s, v)
    assert rho.max() < 1e-8


def test_eckart_young_and_interlacing_on_sbm():
    g = sbm_graph(300, 3, 0.05, 0.005, seed=11)
    m = NEDesignMatrix.from_graph(g, np.full(3, 1 / 3), 0.05, add_self_loops=True)
    dense = m.dot(np.eye(300))
    exact = np.linalg.svd(dense, compute_uv=False)
    k = 10
    prev_err = np.inf
    for q in (0, 1, 3, 8, 150):
        u, s, v = isvd(m, k, gaussian_block(300, 16, seed=4), iterations=q)
        # interlacing: Ritz values never exceed the true singular values
        assert np.all(s <= exact[:k] * (1 + 1e-12))
        # Eckart-Young: no rank-k matrix beats the truncated SVD
        err = np.linalg.norm(dense - u @ np.diag(s) @ v.T) ** 2
        assert err >= np.sum(exact[k:] ** 2) * (1 - 1e-12)
        assert err <= prev_err * (1 + 1e-9)
        prev_err = err
        assert np.allclose(u.T @ u, np.eye(k), atol=1e-13)
        assert np.allclose(v.T @ v, np.eye(k), atol=1e-13)
    # with enough iterations the error reaches the optimum
    assert prev_err <= np.sum(exact[k:] ** 2) * (1 + 1e-5)


def test_qr_and_cholesky_orthonormalisation_span_the_same_space():
    y = np.random.default_rng(9).standard_normal((200, 12)) @ np.diag(np.logspace(0, 3, 12))
    a = orthonorm_qr(y)
    b = orthonorm_cholesky(y)
    assert np.allclose(b.T @ b, np.eye(12), atol=1e-12)
    assert principal_angles(a, b).max() < 1e-12
    assert principal_angles(a, y).max() < 1e-12
    # Q (L^-1)^T: the factor relating b and y is upper triangular
    r = np.linalg.lstsq(b, y, rcond=None)[0]
    assert np.allclose(np.tril(r, -1), 0, atol=1e-10)


def test_isvd_with_cholesky_matches_qr_variant():
    g = sbm_graph(400, 4, 0.04, 0.004, seed=12)
    m = NEDesignMatrix.from_graph(g, np.full(2, 0.5), 0.02)
    om = gaussian_block(400, 14, seed=5)
    u1, s1, v1 = isvd(m, 8, om, 2, orthonorm_qr)
    u2, s2, v2 = isvd(m, 8, om, 2, orthonorm_cholesky)
    assert np.allclose(s1, s2, rtol=1e-10)
    assert principal_angles(u1, u2).max() < 1e-8


def test_residual_zero_at_exact_svd_and_positive_otherwise():
    sig = np.array([4.0, 2.0, 1.0])
    x, u0, v0 = _known_matrix(30, 20, sig, seed=13)
    rho, rho1 = triplet_residuals(_Dense(x), u0, sig, v0)
    assert rho.max() < 1e-14 and rho1.max() < 1e-14
    v_bad = v0.copy()
    v_bad[:, 2] = np.roll(v_bad[:, 2], 1)
    rho, rho1 = triplet_residuals(_Dense(x), u0, sig, v_bad)
    assert rho[2] > 0.1 and rho[0] < 1e-14
    assert np.isclose(rho1[2] * sig[0], rho[2] * sig[2])


def test_principal_angles_known_value():
    a = np.array([[1.0], [0.0], [0.0]])
    b = np.array([[np.cos(0.3)], [np.sin(0.3)], [0.0]])
    assert abs(principal_angles(a, b)[0] - 0.3) < 1e-14


def test_canonical_signs():
    u = np.array([[0.1, -0.9], [-0.8, 0.2]])
    v = np.array([[1.0, 2.0], [3.0, 4.0]])
    cu, cv = canonical_signs(u, v)
    assert np.all(cu[np.argmax(np.abs(cu), axis=0), [0, 1]] > 0)
    assert np.allclose(cu @ cv.T, u @ v.T)


def test_isvd_rejects_bad_sizes():
    x = np.ones((5, 4))
    with pytest.raises(ValueError):
        isvd(_Dense(x), 3, np.ones((4, 5)), 0)   # l > min(r, c)
    with pytest.raises(ValueError):
        isvd(_Dense(x), 3, np.ones((5, 3)), 0)   # wrong number of rows
