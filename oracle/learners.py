"""Closed-form learners on a rank-k SVD (Section 3), FP64.

Test infrastructure only (see the package docstring).

- Node embeddings (Eq. 5): L = U S^(1/2), R = V S^(1/2); the score of the
  node pair (i, j) is <L_i, R_j> = U_i^T S V_j.
- Least-norm linear model (Eq. 8): W* = V S^+ U^T Y, multiplied right to
  left; S^+ reciprocates the non-zero singular values.  With labels on a
  subset of rows only, option (i) of Section 3.2 takes that subset of the
  rows of both U and Y.  Theorem 1: when k >= rank(M), W* is the
  least-norm minimiser of ||M W - Y||_F.

Reading: "non-zero" is s_t > rcond * s_1 (rcond = 0 is the literal rule;
a rank-deficient M computed in floating point needs rcond > 0, as LAPACK's
least-squares solvers use).
"""

from __future__ import annotations

import numpy as np


def ne_embeddings(u: np.ndarray, s: np.ndarray, v: np.ndarray):
    """(L, R) = (U S^(1/2), V S^(1/2)) (Eq. 5)."""
    r = np.sqrt(np.asarray(s, dtype=np.float64))
    return u * r[None, :], v * r[None, :]


def ne_scores(u: np.ndarray, s: np.ndarray, v: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """score_p = <L_{rows_p}, R_{cols_p}> = sum_t U[rows_p, t] s_t V[cols_p, t]."""
    lft, rgt = ne_embeddings(u, s, v)
    return np.einsum("pt,pt->p", lft[rows], rgt[cols])


def s_pinv(s: np.ndarray, rcond: float = 0.0) -> np.ndarray:
    """Diagonal of S^+: 1/s_t where s_t > rcond * s_1, else 0."""
    s = np.asarray(s, dtype=np.float64)
    cut = rcond * (s.max() if s.size else 0.0)
    out = np.zeros_like(s)
    keep = s > cut
    out[keep] = 1.0 / s[keep]
    return out


def nc_fit(u: np.ndarray, s: np.ndarray, v: np.ndarray, y: np.ndarray, rows=None, rcond: float = 0.0) -> np.ndarray:
    """W* = V S^+ U^T Y (Eq. 8), right to left; `rows` keeps the labelled rows
    of U and Y (option (i))."""
    if rows is not None:
        u = u[rows]
        y = y[rows]
    t = u.T @ y                            # k x ny
    t = s_pinv(s, rcond)[:, None] * t      # S^+ (U^T Y)
    return v @ t                           # V (S^+ U^T Y)
