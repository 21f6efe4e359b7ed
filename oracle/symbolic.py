"""Implicit matrices as expression trees, evaluated in FP64 by their definitions.

Test infrastructure only (see the package docstring).

Section 4 of the paper treats a design matrix as usable once three things
are known about it: its shape, its product with an explicit block G, and the
product of its transpose with an explicit block.  Here an implicit matrix is
an immutable expression `Expr` -- a kind, a shape, child expressions and a
payload -- built by the constructor functions below, and one evaluator,
`matmul(e, G, adjoint)`, returns e G (or e^T G) by looking up the rule of
e's kind in a table.  Each rule is the defining identity of its kind:

  dense X, sparse X    X G                       X^T G
  diag(d)              rows of G scaled by d     (the same: D^T = D)
  lincomb(w, M_i)      sum_i w_i M_i G           sum_i w_i M_i^T G
  chain(M_1..M_m)      M_1 (M_2 (... (M_m G)))   M_m^T (... (M_1^T G))
  transpose(M)         M^T G                     M G
  take_rows(M, r)      (M G)[r]                  M^T S, S = G placed at rows r, zeros elsewhere
  hstack(M_1..M_m)     sum_i M_i G_i             [M_1^T G; ...; M_m^T G]
  vstack(M_1..M_m)     [M_1 G; ...; M_m G]       sum_i M_i^T G_i

(G_i: the row block of G that meets the columns of M_i.)  power(M, p) is a
chain of p copies of M.  Products are taken exactly as the identities read,
with no cache of shared sub-products: a cache changes the cost of a
product, never its value.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from numbers import Integral, Real

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True, eq=False)
class Expr:
    kind: str
    shape: tuple
    args: tuple = ()
    data: object = None
    weights: tuple = field(default=())

    # explicit products and the transpose, through the evaluator
    def dot(self, g):
        return matmul(self, g)

    @property
    def T(self):
        return transpose(self)

    def dense(self):
        return to_dense(self)


def _block(g) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)
    return g.reshape(-1, 1) if g.ndim == 1 else g


# ---------------------------------------------------------------- constructors

def dense(x) -> Expr:
    x = np.array(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("a dense leaf is a matrix")
    return Expr("dense", x.shape, data=x)


def sparse(x) -> Expr:
    x = sp.csr_matrix(x, dtype=np.float64)
    return Expr("sparse", x.shape, data=x)


def diag(d) -> Expr:
    d = np.array(d, dtype=np.float64).ravel()
    return Expr("diag", (d.shape[0], d.shape[0]), data=d)


def lincomb(terms, weights=None) -> Expr:
    terms = tuple(terms)
    if not terms:
        raise ValueError("a sum needs at least one term")
    w = tuple(1.0 for _ in terms) if weights is None else tuple(float(x) for x in weights)
    if len(w) != len(terms):
        raise ValueError("one weight per term")
    if any(t.shape != terms[0].shape for t in terms):
        raise ValueError(f"terms of a sum differ in shape: {[t.shape for t in terms]}")
    return Expr("lincomb", terms[0].shape, args=terms, weights=w)


def chain(factors) -> Expr:
    factors = tuple(factors)
    if not factors:
        raise ValueError("a product needs at least one factor")
    for left, right in zip(factors[:-1], factors[1:]):
        if left.shape[1] != right.shape[0]:
            raise ValueError(f"inner dimensions differ: {left.shape} times {right.shape}")
    return Expr("chain", (factors[0].shape[0], factors[-1].shape[1]), args=factors)


def power(m: Expr, p) -> Expr:
    if isinstance(p, bool) or not isinstance(p, Integral) or p < 1:
        raise ValueError(f"matrix powers are positive integers, got {p!r}")
    if m.shape[0] != m.shape[1]:
        raise ValueError(f"a power needs a square matrix, got {m.shape}")
    copies = []
    for _ in range(int(p)):
        copies.append(m)
    return chain(copies)


def transpose(m: Expr) -> Expr:
    return Expr("transpose", (m.shape[1], m.shape[0]), args=(m,))


def take_rows(m: Expr, rows) -> Expr:
    rows = np.array(rows, dtype=np.int64).ravel()
    if np.unique(rows).shape[0] != rows.shape[0]:
        raise ValueError("gathered rows must be distinct (the transpose places each row once)")
    if rows.size and (rows.min() < 0 or rows.max() >= m.shape[0]):
        raise ValueError("row index out of range")
    return Expr("take_rows", (rows.shape[0], m.shape[1]), args=(m,), data=rows)


def hstack(parts) -> Expr:
    parts = tuple(parts)
    if not parts or any(q.shape[0] != parts[0].shape[0] for q in parts):
        raise ValueError("side-by-side parts need equal row counts")
    return Expr("hstack", (parts[0].shape[0], sum(q.shape[1] for q in parts)), args=parts)


def vstack(parts) -> Expr:
    parts = tuple(parts)
    if not parts or any(q.shape[1] != parts[0].shape[1] for q in parts):
        raise ValueError("stacked parts need equal column counts")
    return Expr("vstack", (sum(q.shape[0] for q in parts), parts[0].shape[1]), args=parts)


# ---------------------------------------------------------------- evaluation

def _leaf(e, g, adjoint):
    x = e.data
    return (x.T @ g) if adjoint else (x @ g)


def _diag(e, g, adjoint):
    return e.data[:, None] * g


def _lincomb(e, g, adjoint):
    total = np.zeros((e.shape[1] if adjoint else e.shape[0], g.shape[1]))
    for w, t in zip(e.weights, e.args):
        total += w * matmul(t, g, adjoint)
    return total


def _chain(e, g, adjoint):
    # M_1 ... M_m G: the rightmost factor meets G first; for the transpose the
    # factors' transposes meet G in the opposite order
    order = e.args if adjoint else e.args[::-1]
    out = g
    for f in order:
        out = matmul(f, out, adjoint)
    return out


def _transpose(e, g, adjoint):
    return matmul(e.args[0], g, not adjoint)


def _take_rows(e, g, adjoint):
    m, rows = e.args[0], e.data
    if not adjoint:
        return matmul(m, g, False)[rows]
    placed = np.zeros((m.shape[0], g.shape[1]))
    placed[rows] = g
    return matmul(m, placed, True)


def _split(parts, g, along):
    """Row blocks of g that meet each part's columns (along=1) or rows (along=0)."""
    bounds = np.cumsum([0] + [q.shape[along] for q in parts])
    return [g[bounds[i]:bounds[i + 1]] for i in range(len(parts))]


def _hstack(e, g, adjoint):
    if adjoint:
        return np.vstack([matmul(q, g, True) for q in e.args])
    return sum(matmul(q, gi, False) for q, gi in zip(e.args, _split(e.args, g, 1)))


def _vstack(e, g, adjoint):
    if not adjoint:
        return np.vstack([matmul(q, g, False) for q in e.args])
    return sum(matmul(q, gi, True) for q, gi in zip(e.args, _split(e.args, g, 0)))


_RULES = {"dense": _leaf, "sparse": _leaf, "diag": _diag, "lincomb": _lincomb, "chain": _chain,
          "transpose": _transpose, "take_rows": _take_rows, "hstack": _hstack, "vstack": _vstack}


def matmul(e: Expr, g, adjoint: bool = False) -> np.ndarray:
    """e G (adjoint=False) or e^T G (adjoint=True), FP64, G explicit."""
    g = _block(g)
    inner = e.shape[0] if adjoint else e.shape[1]
    if g.shape[0] != inner:
        raise ValueError(f"block has {g.shape[0]} rows, the product needs {inner}")
    return np.asarray(_RULES[e.kind](e, g, adjoint))


def to_dense(e: Expr) -> np.ndarray:
    """The matrix itself, as the product with the identity (small cases)."""
    return matmul(e, np.eye(e.shape[1]))


# ---------------------------------------------------------------- Python operators

def _scaled(e, s):
    if not isinstance(s, Real):
        return NotImplemented
    return lincomb([e], [float(s)])


def _other_expr(fn):
    def op(a, b):
        return fn(a, b) if isinstance(b, Expr) else NotImplemented
    return op


# a + b, a - b, s * a, a @ b and a ** p build the nodes above
for _name, _fn in {
    "__add__": _other_expr(lambda a, b: lincomb([a, b])),
    "__sub__": _other_expr(lambda a, b: lincomb([a, b], [1.0, -1.0])),
    "__matmul__": _other_expr(lambda a, b: chain([a, b])),
    "__mul__": _scaled,
    "__rmul__": _scaled,
    "__pow__": power,
}.items():
    setattr(Expr, _name, _fn)
