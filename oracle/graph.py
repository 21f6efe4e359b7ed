"""Graph matrices of Section 2 (preliminaries and notation), in FP64 SciPy CSR.

Test infrastructure only (see the package docstring).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def adjacency(n, indptr, indices, values=None, add_self_loops=False) -> sp.csr_matrix:
    """A as an n x n FP64 CSR matrix: A_ij is the edge weight, 0 elsewhere.

    With add_self_loops, A + I is returned (the workload's "self-loops
    added"); every later quantity (D, T and the -lambda(11^T - A) term)
    then uses this A.
    """
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    nnz = int(indptr[-1])
    data = np.ones(nnz) if values is None else np.asarray(values, dtype=np.float64)
    a = sp.csr_matrix((data, indices, indptr), shape=(n, n))
    if add_self_loops:
        a = (a + sp.identity(n, format="csr")).tocsr()
    a.sort_indices()
    return a


def degrees(a: sp.csr_matrix) -> np.ndarray:
    """Diagonal of D: row sums of A."""
    return np.asarray(a.sum(axis=1)).ravel()


def transition(a: sp.csr_matrix) -> sp.csr_matrix:
    """Row-normalised transition matrix T = D^-1 A (Section 2).

    A node with zero degree has an all-zero row of A; its row of T is left
    zero (D^-1 read as the pseudo-inverse of D, the same convention as the
    S^+ of Eq. 8)."""
    d = degrees(a)
    dinv = np.zeros_like(d)
    nz = d != 0
    dinv[nz] = 1.0 / d[nz]
    return (sp.diags(dinv) @ a).tocsr()


def sym_normalized(a: sp.csr_matrix) -> sp.csr_matrix:
    """A_hat = (D + I)^-1/2 (A + I) (D + I)^-1/2 (Section 2), D = diag(A 1)."""
    n = a.shape[0]
    d = degrees(a)
    s = 1.0 / np.sqrt(d + 1.0)
    eye = sp.identity(n, format="csr")
    return (sp.diags(s) @ (a + eye) @ sp.diags(s)).tocsr()
