"""Algorithm 1 (iSVD) and Algorithm 2 (orthonormalisation), FP64.

Test infrastructure only (see the package docstring).

`isvd` follows Algorithm 1 step by step: start from the c x l block
Omega, alternate orthonormalised products with M and M^T `iterations`
times, take one more orthonormalised product with M, project
B = (M^T Q)^T, take the SVD of the small B and lift its left vectors with
Q.  The width l = k + p replaces Algorithm 1's 2k (the start block is
passed in, so its width is the caller's choice).  The output is truncated
to k triplets.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def orthonorm_qr(q: np.ndarray) -> np.ndarray:
    """Algorithm 2, left: Householder QR (LAPACK), keep the reduced Q."""
    qhat, _ = np.linalg.qr(q, mode="reduced")
    return qhat


def orthonorm_cholesky(q: np.ndarray) -> np.ndarray:
    """Algorithm 2, right: L = chol(Q^T Q) (lower), return Q (L^-1)^T.

    Q (L^-1)^T is formed by a triangular solve with L rather than an
    explicit inverse: X = Q L^-T solves X L^T = Q.  Raises
    numpy.linalg.LinAlgError when Q^T Q is not numerically positive
    definite."""
    gram = q.T @ q
    low = np.linalg.cholesky(gram)
    return sla.solve_triangular(low, q.T, lower=True).T


def isvd(m, k: int, omega: np.ndarray, iterations: int, orthonorm=orthonorm_qr):
    """Rank-k SVD of the implicit matrix m from start block omega (c x l).

    m must offer `shape`, `dot` and `T` (the symbolic-matrix interface of
    the appendix).  Returns (U r x k, s k, V c x k), s descending."""
    r, c = m.shape
    omega = np.asarray(omega, dtype=np.float64)
    if omega.shape[0] != c:
        raise ValueError("omega must have c rows")
    l = omega.shape[1]
    if not (0 < k <= l <= min(r, c)):
        raise ValueError("need 0 < k <= l <= min(r, c)")
    mt = m.T
    q = omega
    for _ in range(iterations):
        q = orthonorm(m.dot(q))      # r x l
        q = orthonorm(mt.dot(q))     # c x l
    q = orthonorm(m.dot(q))          # r x l
    b = mt.dot(q).T                  # l x c
    ub, s, vt = np.linalg.svd(b, full_matrices=False)
    u = q @ ub
    return u[:, :k], s[:k], vt[:k].T


def canonical_signs(u: np.ndarray, v: np.ndarray):
    """Flip each pair (u_i, v_i) so that the entry of u_i largest in
    magnitude is positive (singular vectors are defined up to sign)."""
    idx = np.argmax(np.abs(u), axis=0)
    sgn = np.sign(u[idx, np.arange(u.shape[1])])
    sgn[sgn == 0] = 1.0
    return u * sgn, v * sgn


def triplet_residuals(m, u, s, v):
    """Per-triplet residuals of (u_i, s_i, v_i) against M, FP64.

    Returns (rho, rho_1) arrays of length k with
      rho_i   = sqrt(|M v_i - s_i u_i|^2 + |M^T u_i - s_i v_i|^2) / s_i
      rho_1,i = the same numerator / s_1.
    The definition is a reading (parity unpinned): the paper states no
    residual; M^T U - V S alone vanishes for Algorithm 1's output by
    construction, so the M V - U S side is included."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    left = m.dot(v) - u * s
    right = m.T.dot(u) - v * s
    num = np.sqrt(np.sum(left * left, axis=0) + np.sum(right * right, axis=0))
    return num / s, num / s[0]


def principal_angles(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Principal angles (radians, ascending) between span(a) and span(b)."""
    qa = orthonorm_qr(np.asarray(a, dtype=np.float64))
    qb = orthonorm_qr(np.asarray(b, dtype=np.float64))
    return sla.subspace_angles(qa, qb)[::-1]
