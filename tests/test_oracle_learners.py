"""Pins for the closed-form learners of the oracle (CPU only).

Pins: Theorem 1 (W* = V S^+ U^T Y equals LAPACK's least-norm least-squares
solution when k >= rank M, also for a rank-deficient M), the row-subset
option equals the fit on the explicitly gathered rows, Eq. 5 scores
reconstruct M's entries at full rank and reduce to U_i^T S V_j, and S^+
reciprocates exactly the entries above the threshold.
"""

import numpy as np
import pytest

from oracle import learners


def _rank_r(n, f, r, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, r)) @ rng.standard_normal((r, f))


def _svd_k(m, k):
    u, s, vt = np.linalg.svd(m, full_matrices=False)
    return u[:, :k], s[:k], vt[:k].T


@pytest.mark.parametrize("n,f,r,k", [(60, 25, 25, 25), (80, 30, 12, 12), (80, 30, 12, 20)])
def test_theorem1_least_norm(n, f, r, k):
    m = _rank_r(n, f, r, seed=n + r)
    y = np.random.default_rng(1).standard_normal((n, 3))
    u, s, v = _svd_k(m, k)
    w = learners.nc_fit(u, s, v, y, rcond=1e-10)
    want = np.linalg.lstsq(m, y, rcond=None)[0]   # least-norm minimiser
    assert np.abs(w - want).max() <= 1e-10 * max(1.0, np.abs(want).max())
    # the residual is orthogonal to the range of M (normal equations)
    assert np.abs(m.T @ (m @ w - y)).max() <= 1e-9 * np.abs(m).max() ** 2


def test_rank_deficient_literal_rule_blows_up():
    # rcond = 0 reciprocates round-off singular values (why a threshold is needed)
    m = _rank_r(50, 20, 5, seed=3)
    y = np.random.default_rng(2).standard_normal((50, 2))
    u, s, v = _svd_k(m, 20)
    assert s[5:].max() < 1e-12 * s[0]
    w0 = learners.nc_fit(u, s, v, y, rcond=0.0)
    w1 = learners.nc_fit(u, s, v, y, rcond=1e-10)
    assert np.abs(w0).max() > 1e6 * np.abs(w1).max()


def test_row_subset_equals_gathered_rows():
    rng = np.random.default_rng(4)
    u = rng.standard_normal((40, 6))
    v = rng.standard_normal((15, 6))
    s = np.sort(rng.uniform(0.5, 3.0, 6))[::-1]
    y = rng.standard_normal((40, 4))
    rows = rng.choice(40, size=17, replace=False)
    w = learners.nc_fit(u, s, v, y, rows=rows)
    assert np.allclose(w, v @ np.diag(1.0 / s) @ u[rows].T @ y[rows], atol=1e-13)


def test_s_pinv_threshold():
    s = np.array([4.0, 2.0, 1e-3, 0.0])
    assert np.array_equal(learners.s_pinv(s), [0.25, 0.5, 1e3, 0.0])
    assert np.array_equal(learners.s_pinv(s, rcond=1e-3), [0.25, 0.5, 0.0, 0.0])


def test_ne_scores_reconstruct_full_rank():
    rng = np.random.default_rng(5)
    m = rng.standard_normal((12, 9))
    u, s, v = _svd_k(m, 9)
    lft, rgt = learners.ne_embeddings(u, s, v)
    assert np.abs(lft @ rgt.T - m).max() < 1e-12
    rows = rng.integers(0, 12, size=30)
    cols = rng.integers(0, 9, size=30)
    sc = learners.ne_scores(u, s, v, rows, cols)
    assert np.abs(sc - m[rows, cols]).max() < 1e-12
    # the same as U_i^T S V_j, term by term
    brute = [sum(u[i, t] * s[t] * v[j, t] for t in range(9)) for i, j in zip(rows, cols)]
    assert np.abs(sc - np.array(brute)).max() < 1e-12


def test_ne_symmetric_psd_gives_equal_embeddings():
    # Section 3.1: a symmetric (PSD) M gives L = R
    rng = np.random.default_rng(6)
    b = rng.standard_normal((10, 10))
    m = b @ b.T
    u, s, v = _svd_k(m, 10)
    lft, rgt = learners.ne_embeddings(u, s, v)
    assert np.abs(lft - rgt).max() < 1e-10
