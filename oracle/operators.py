"""Products with the implicit design matrices, FP64.

Test infrastructure only (see the package docstring).

The interface is the one of the paper's symbolic matrices (Section 4 and
the appendix on symbolic representation): `shape`, `dot(G)` = M G for an
explicit G, and `T` = the implicit transpose.  Products are evaluated by
the naive power sum, in the order the definitions are written, without
Horner rearrangement or caching, so that they are independent of the GPU
path's evaluation order.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .graph import adjacency, sym_normalized, transition


class NEDesignMatrix:
    """M = sum_{j=1..K} c_j T^j - lambda (1 1^T - A), n x n (Eq. 3, Fig. 1).

    Eq. 3 takes the expectation of T^q under the context distribution; its
    weights are passed explicitly as `coeffs` = (c_1, ..., c_K) (the
    workloads use c_j = 1/K; Fig. 1 uses (3, 2, 1)/6).  "1" in the
    lambda term is the all-ones n x n matrix (Fig. 1 builds it as the
    outer product of a ones row with itself) and A is the same adjacency
    that defines T.
    """

    def __init__(self, a: sp.csr_matrix, coeffs, lam: float, transposed: bool = False):
        self.a = a.tocsr()
        self.t = transition(self.a)
        self.coeffs = np.asarray(coeffs, dtype=np.float64)
        self.lam = float(lam)
        self.transposed = transposed
        n = a.shape[0]
        self.shape = (n, n)
        if transposed:
            self._a_op = self.a.T.tocsr()
            self._t_op = self.t.T.tocsr()
        else:
            self._a_op = self.a
            self._t_op = self.t

    @classmethod
    def from_graph(cls, g, coeffs, lam, add_self_loops=False, values=None):
        return cls(adjacency(g.n, g.indptr, g.indices, values, add_self_loops), coeffs, lam)

    @property
    def T(self) -> "NEDesignMatrix":
        return NEDesignMatrix(self.a, self.coeffs, self.lam, transposed=not self.transposed)

    def dot(self, g: np.ndarray) -> np.ndarray:
        g = np.asarray(g, dtype=np.float64)
        vec = g.ndim == 1
        if vec:
            g = g[:, None]
        n = self.shape[0]
        out = np.zeros((n, g.shape[1]))
        p = g
        for cj in self.coeffs:          # P_j = T P_{j-1}; sum_j c_j P_j
            p = self._t_op @ p
            out += cj * p
        ones = np.ones((n, 1))
        ones_term = ones @ (ones.T @ g)  # (1 1^T) G kept in O(n) space
        out -= self.lam * (ones_term - self._a_op @ g)
        return out[:, 0] if vec else out


class FeatPropDesignMatrix:
    """M = [X, A_hat X, A_hat^2 X, ..., A_hat^L X], n x d(L+1) (Eq. 7).

    The blocks B_j = A_hat^j X are materialised here (the oracle may hold
    M explicitly); M G = sum_j B_j G_j over the row blocks G_j of G, and
    M^T Q stacks B_j^T Q.
    """

    def __init__(self, a: sp.csr_matrix, x: np.ndarray, L: int, transposed: bool = False,
                 blocks=None):
        self.a = a.tocsr()
        self.x = np.asarray(x, dtype=np.float64)
        self.L = int(L)
        self.transposed = transposed
        n, d = self.x.shape
        self.d = d
        if blocks is None:
            ahat = sym_normalized(self.a)
            blocks = [self.x]
            for _ in range(self.L):
                blocks.append(ahat @ blocks[-1])
        self.blocks = blocks
        full = (n, d * (self.L + 1))
        self.shape = full[::-1] if transposed else full

    @classmethod
    def from_graph(cls, g, x, L):
        return cls(adjacency(g.n, g.indptr, g.indices), x, L)

    @property
    def T(self) -> "FeatPropDesignMatrix":
        return FeatPropDesignMatrix(self.a, self.x, self.L, not self.transposed, self.blocks)

    def _mul(self, g):
        d = self.d
        out = np.zeros((self.x.shape[0], g.shape[1]))
        for j, b in enumerate(self.blocks):
            out += b @ g[j * d:(j + 1) * d]
        return out

    def _rmul(self, q):
        return np.vstack([b.T @ q for b in self.blocks])

    def dot(self, g):
        g = np.asarray(g, dtype=np.float64)
        vec = g.ndim == 1
        if vec:
            g = g[:, None]
        out = self._rmul(g) if self.transposed else self._mul(g)
        return out[:, 0] if vec else out

    def dense(self) -> np.ndarray:
        m = np.hstack(self.blocks)
        return m.T if self.transposed else m


class RowGather:
    """M_sub = M[rows, :] of an implicit M, without forming either (the
    implicit row gather of Section 3.2, option (ii), and Section 4).

    M_sub G takes the listed rows of M G; M_sub^T Q = M^T Q' where Q' has
    the rows of Q at the listed positions and zeros elsewhere (rows are
    distinct).
    """

    def __init__(self, m, rows, transposed: bool = False):
        self.m = m
        self.rows = np.asarray(rows, dtype=np.int64)
        assert self.rows.ndim == 1 and len(np.unique(self.rows)) == len(self.rows)
        self.transposed = transposed
        full = (len(self.rows), m.shape[1])
        self.shape = full[::-1] if transposed else full

    @property
    def T(self) -> "RowGather":
        return RowGather(self.m, self.rows, not self.transposed)

    def dot(self, g):
        g = np.asarray(g, dtype=np.float64)
        if not self.transposed:
            return self.m.dot(g)[self.rows]
        q = np.zeros((self.m.shape[0],) + g.shape[1:])
        q[self.rows] = g
        return self.m.T.dot(q)


def context_weights(C: int) -> np.ndarray:
    """Normalised context-window weights of Fig. 1: proportional to C - q + 1,
    q = 1..C, summing to one (Fig. 1 writes (3, 2, 1)/6 for C = 3)."""
    w = np.arange(C, 0, -1, dtype=np.float64)
    return w / w.sum()
