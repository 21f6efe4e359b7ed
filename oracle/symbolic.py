"""Symbolic (implicit) matrices as a DAG of product functions, FP64.

Test infrastructure only (see the package docstring).

Section 4 and the appendix on symbolic representation: a matrix is usable
once it offers `shape`, `dot(G)` = M G for an explicit G, and `T` = its
implicit transpose.  Leaf nodes hold a matrix explicitly; symbolic nodes
represent one as a function of other nodes, and a product walks the DAG
downwards to the leaves.  The node set here: dense, sparse and diagonal
leaves; sum (with weights), product, scalar multiple and power (sugar for a
product of copies), transpose, row gather, and column / row concatenation.
Products are evaluated exactly as the definitions read, without the lazy
cache of sub-products (the cache changes the cost, not the result).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class PF:
    """Base class: operator sugar building symbolic nodes."""

    shape: tuple

    def __add__(self, other):
        return SumPF([self, other])

    def __sub__(self, other):
        return SumPF([self, other], [1.0, -1.0])

    def __mul__(self, alpha):
        return SumPF([self], [float(alpha)])

    __rmul__ = __mul__

    def __matmul__(self, other):
        return ProductPF([self, other])

    def __pow__(self, p):
        assert int(p) >= 1
        return ProductPF([self] * int(p))

    def dense(self) -> np.ndarray:
        """The matrix, from products with the unit vectors (small cases)."""
        return self.dot(np.eye(self.shape[1]))


def _mat(g):
    g = np.asarray(g, dtype=np.float64)
    return g[:, None] if g.ndim == 1 else g


class DensePF(PF):
    def __init__(self, m):
        self.m = np.asarray(m, dtype=np.float64)
        self.shape = self.m.shape

    def dot(self, g):
        return self.m @ _mat(g)

    @property
    def T(self):
        return DensePF(self.m.T)


class SparsePF(PF):
    def __init__(self, m):
        self.m = sp.csr_matrix(m, dtype=np.float64)
        self.shape = self.m.shape

    def dot(self, g):
        return self.m @ _mat(g)

    @property
    def T(self):
        return SparsePF(self.m.T.tocsr())


class DiagPF(PF):
    def __init__(self, d):
        self.d = np.asarray(d, dtype=np.float64)
        self.shape = (len(self.d), len(self.d))

    def dot(self, g):
        return self.d[:, None] * _mat(g)

    @property
    def T(self):
        return self


class SumPF(PF):
    """sum_i w_i M_i (w_i = 1 when not given)."""

    def __init__(self, terms, weights=None):
        self.terms = list(terms)
        self.weights = [1.0] * len(self.terms) if weights is None else [float(w) for w in weights]
        assert len(self.weights) == len(self.terms) >= 1
        assert all(t.shape == self.terms[0].shape for t in self.terms)
        self.shape = self.terms[0].shape

    def dot(self, g):
        out = np.zeros((self.shape[0], _mat(g).shape[1]))
        for w, t in zip(self.weights, self.terms):
            out += w * t.dot(g)
        return out

    @property
    def T(self):
        return SumPF([t.T for t in self.terms], self.weights)


class ProductPF(PF):
    """M_1 M_2 ... M_m, multiplied onto G from the right."""

    def __init__(self, factors):
        self.factors = list(factors)
        for a, b in zip(self.factors, self.factors[1:]):
            assert a.shape[1] == b.shape[0]
        self.shape = (self.factors[0].shape[0], self.factors[-1].shape[1])

    def dot(self, g):
        out = _mat(g)
        for f in reversed(self.factors):
            out = f.dot(out)
        return out

    @property
    def T(self):
        return ProductPF([f.T for f in reversed(self.factors)])


class GatherRowsPF(PF):
    """M[rows, :]; the transpose places each row back (rows distinct)."""

    def __init__(self, m, rows, transposed=False):
        self.m = m
        self.rows = np.asarray(rows, dtype=np.int64)
        assert len(np.unique(self.rows)) == len(self.rows)
        self.transposed = transposed
        full = (len(self.rows), m.shape[1])
        self.shape = full[::-1] if transposed else full

    def dot(self, g):
        g = _mat(g)
        if not self.transposed:
            return self.m.dot(g)[self.rows]
        q = np.zeros((self.m.shape[0], g.shape[1]))
        q[self.rows] = g
        return self.m.T.dot(q)

    @property
    def T(self):
        return GatherRowsPF(self.m, self.rows, not self.transposed)


class ConcatColsPF(PF):
    """[M_1, M_2, ..., M_m] side by side (equal row counts)."""

    def __init__(self, parts):
        self.parts = list(parts)
        assert all(p.shape[0] == self.parts[0].shape[0] for p in self.parts)
        self.shape = (self.parts[0].shape[0], sum(p.shape[1] for p in self.parts))

    def dot(self, g):
        g = _mat(g)
        out = np.zeros((self.shape[0], g.shape[1]))
        off = 0
        for p in self.parts:
            out += p.dot(g[off:off + p.shape[1]])
            off += p.shape[1]
        return out

    @property
    def T(self):
        return ConcatRowsPF([p.T for p in self.parts])


class ConcatRowsPF(PF):
    """[M_1; M_2; ...; M_m] stacked (equal column counts)."""

    def __init__(self, parts):
        self.parts = list(parts)
        assert all(p.shape[1] == self.parts[0].shape[1] for p in self.parts)
        self.shape = (sum(p.shape[0] for p in self.parts), self.parts[0].shape[1])

    def dot(self, g):
        return np.vstack([p.dot(g) for p in self.parts])

    @property
    def T(self):
        return ConcatColsPF([p.T for p in self.parts])
