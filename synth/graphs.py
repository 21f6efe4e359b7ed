"""Random graph generators (stochastic block model, Chung-Lu) and CSR assembly.

Every generator is seeded and vectorised with NumPy so that graphs with
tens of millions of edges build in seconds.  Graphs are undirected and
simple: the CSR holds both (i, j) and (j, i), no duplicates and no
self-loops (self-loops, when a workload wants them, are added by the
design-matrix operator, not here).  Column indices are sorted inside each
row.  Edge weights are not drawn: every stored entry of A is 1.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Pattern of an undirected graph in CSR form.

    indptr  : int64 array of n+1 row offsets
    indices : int32 array of nnz column indices, sorted inside each row
    blocks  : optional int32 array of n block labels (SBM graphs)
    """

    n: int
    indptr: np.ndarray
    indices: np.ndarray
    blocks: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.indptr)


def edges_to_csr(n: int, src: np.ndarray, dst: np.ndarray, blocks=None) -> Graph:
    """Symmetric CSR from an undirected edge list (i != j).

    Duplicate pairs (in either orientation) are merged; self-pairs are
    dropped.  Row r holds its neighbours below r (pairs (lo, hi) with
    hi = r) followed by those above r (lo = r), each run sorted, so the
    CSR is assembled by placement after two sorts of the pair codes.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    code = np.minimum(src, dst) * n + np.maximum(src, dst)
    code.sort()
    if code.shape[0]:
        first = np.empty(code.shape[0], dtype=bool)
        first[0] = True
        np.not_equal(code[1:], code[:-1], out=first[1:])
        code = code[first]
    lo, hi = np.divmod(code, n)                 # sorted by (lo, hi)
    below = hi * n + lo
    below.sort()
    b_row, b_col = np.divmod(below, n)          # sorted by (hi, lo)
    cnt_b = np.bincount(b_row, minlength=n)
    cnt_a = np.bincount(lo, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_b + cnt_a, out=indptr[1:])
    start_b = np.cumsum(cnt_b) - cnt_b
    start_a = np.cumsum(cnt_a) - cnt_a
    rank = np.arange(code.shape[0], dtype=np.int64)
    indices = np.empty(2 * code.shape[0], dtype=np.int32)
    indices[indptr[b_row] + (rank - start_b[b_row])] = b_col
    indices[indptr[lo] + cnt_b[lo] + (rank - start_a[lo])] = hi
    return Graph(n=n, indptr=indptr, indices=indices, blocks=blocks)


def _block_sizes(n: int, num_blocks: int) -> np.ndarray:
    # When num_blocks does not divide n the first n mod B blocks get one extra node.
    base = n // num_blocks
    sizes = np.full(num_blocks, base, dtype=np.int64)
    sizes[: n - base * num_blocks] += 1
    return sizes


def sbm_graph(n: int, num_blocks: int, p_in: float, p_out: float, seed: int) -> Graph:
    """Stochastic block model with Bernoulli(p_in / p_out) edges over pairs i < j.

    Blocks are contiguous node ranges.  For n <= 6000 every pair is drawn
    explicitly.  For larger n each block pair draws its edge count from
    the binomial law and then that many distinct uniform pairs, which is
    the same distribution.
    """
    rng = np.random.default_rng(seed)
    sizes = _block_sizes(n, num_blocks)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    labels = np.repeat(np.arange(num_blocks, dtype=np.int32), sizes)
    if n <= 6000:
        iu, ju = np.triu_indices(n, k=1)
        same = labels[iu] == labels[ju]
        prob = np.where(same, p_in, p_out)
        hit = rng.random(iu.shape[0]) < prob
        return edges_to_csr(n, iu[hit], ju[hit], blocks=labels)
    srcs, dsts = [], []
    for a in range(num_blocks):
        for b in range(a, num_blocks):
            na, nb = int(sizes[a]), int(sizes[b])
            pairs = na * (na - 1) // 2 if a == b else na * nb
            p = p_in if a == b else p_out
            m = int(rng.binomial(pairs, p)) if pairs > 0 else 0
            if m == 0:
                continue
            got_s = np.empty(0, np.int64)
            got_d = np.empty(0, np.int64)
            need = m
            while need > 0:
                draw = int(need * 1.05) + 16
                if a == b:
                    s = rng.integers(0, na, draw)
                    d = rng.integers(0, na, draw)
                    ok = s != d
                    s, d = np.minimum(s[ok], d[ok]), np.maximum(s[ok], d[ok])
                else:
                    s = rng.integers(0, na, draw)
                    d = rng.integers(0, nb, draw)
                s = np.concatenate([got_s, s + starts[a]])
                d = np.concatenate([got_d, d + starts[b]])
                code, first = np.unique(s * n + d, return_index=True)
                first = np.sort(first)[:m]
                got_s, got_d = s[first], d[first]
                need = m - got_s.shape[0]
            srcs.append(got_s)
            dsts.append(got_d)
    src = np.concatenate(srcs) if srcs else np.empty(0, np.int64)
    dst = np.concatenate(dsts) if dsts else np.empty(0, np.int64)
    return edges_to_csr(n, src, dst, blocks=labels)


def sbm_graph_by_degree(n: int, num_blocks: int, mean_degree: float, frac_in: float, seed: int) -> Graph:
    """SBM whose p_in / p_out give an expected degree `mean_degree` with a
    fraction `frac_in` of each node's edges inside its block."""
    size = n / num_blocks
    p_in = mean_degree * frac_in / max(size - 1.0, 1.0)
    p_out = mean_degree * (1.0 - frac_in) / max(n - size, 1.0)
    return sbm_graph(n, num_blocks, p_in, p_out, seed)


def chung_lu_weights(n: int, beta: float, mean_degree: float) -> np.ndarray:
    """Expected degrees w_i proportional to (i+1)^(-1/(beta-1)), capped at
    sqrt(n * mean_degree) and rescaled so that their mean is mean_degree."""
    gamma = 1.0 / (beta - 1.0)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -gamma)
    cap = np.sqrt(n * mean_degree)
    w *= mean_degree / w.mean()
    for _ in range(50):
        w = np.minimum(w, cap)
        w *= mean_degree / w.mean()
        if w.max() <= cap * (1 + 1e-12):
            break
    return np.minimum(w, cap)


def chung_lu_graph(n: int, beta: float, mean_degree: float, seed: int) -> Graph:
    """Approximate Chung-Lu power-law graph by endpoint sampling.

    n*mean_degree/2 edges are drawn with both endpoints chosen
    independently with probability proportional to w; self-pairs and
    repeated pairs are then removed, so that node i ends with expected
    degree close to (slightly below, for the largest hubs) w_i.  Nodes
    are numbered by decreasing weight, so hubs sit at low indices.
    Isolated nodes are kept.
    """
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, beta, mean_degree)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2.0))
    chunk = 1 << 22
    srcs, dsts = [], []
    for start in range(0, m, chunk):
        cnt = min(chunk, m - start)
        s = np.searchsorted(cdf, rng.random(cnt), side="right")
        d = np.searchsorted(cdf, rng.random(cnt), side="right")
        srcs.append(np.minimum(s, n - 1))
        dsts.append(np.minimum(d, n - 1))
    return edges_to_csr(n, np.concatenate(srcs), np.concatenate(dsts))


def cycle_graph(n: int) -> Graph:
    """Cycle C_n (every node joined to its two ring neighbours), n >= 3."""
    i = np.arange(n, dtype=np.int64)
    return edges_to_csr(n, i, (i + 1) % n)


def complete_graph(n: int) -> Graph:
    """Complete graph K_n without self-loops."""
    iu, ju = np.triu_indices(n, k=1)
    return edges_to_csr(n, iu, ju)


def random_pattern(n_rows: int, n_cols: int, density: float, seed: int, hub_rows: int = 0,
                   hub_len: int = 0, empty_rows: int = 0):
    """Random (possibly rectangular, non-symmetric) CSR pattern for kernel tests.

    A few rows can be made dense "hubs" and a few left empty to exercise the
    long-row and empty-row cases.  Returns (indptr int64, indices int32).
    """
    rng = np.random.default_rng(seed)
    lens = rng.binomial(n_cols, density, size=n_rows).astype(np.int64)
    if hub_rows:
        hubs = rng.choice(n_rows, size=min(hub_rows, n_rows), replace=False)
        lens[hubs] = min(hub_len, n_cols)
    if empty_rows:
        empt = rng.choice(n_rows, size=min(empty_rows, n_rows), replace=False)
        lens[empt] = 0
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    indices = np.empty(int(indptr[-1]), dtype=np.int32)
    for r in range(n_rows):
        ln = int(lens[r])
        if ln:
            indices[indptr[r]:indptr[r + 1]] = np.sort(rng.choice(n_cols, size=ln, replace=False))
    return indptr, indices


@dataclass
class DirectedGraph:
    """Directed, optionally weighted graph: the CSR of A and the CSR of A^T.

    indptr / t_indptr : int64 arrays of n+1 row offsets of A / of A^T
    indices / t_indices : int32 column indices, sorted inside each row
    values / t_values : float32 edge weights in the same order, or None
                        (every stored entry is 1)
    """

    n: int
    indptr: np.ndarray
    indices: np.ndarray
    values: np.ndarray | None
    t_indptr: np.ndarray
    t_indices: np.ndarray
    t_values: np.ndarray | None
    blocks: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.indptr)


def csr_transpose(n_rows: int, n_cols: int, indptr, indices, values=None):
    """CSR arrays of the transpose (a format conversion: entries are only
    moved, never combined).  Returns (indptr int64, indices int32, values
    or None), column indices sorted inside each row."""
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(indptr))
    order = np.lexsort((rows, indices))          # by column, then by row
    t_indptr = np.zeros(n_cols + 1, dtype=np.int64)
    np.cumsum(np.bincount(indices, minlength=n_cols), out=t_indptr[1:])
    t_values = None if values is None else np.asarray(values)[order]
    return t_indptr, rows[order].astype(np.int32), t_values


def directed_graph(n: int, mean_degree: float, seed: int, weighted: bool = True, hub_rows: int = 0,
                   hub_len: int = 0, hub_cols: int = 0, hub_col_len: int = 0, empty_rows: int = 0,
                   w_range=(0.25, 2.0)) -> DirectedGraph:
    """Random directed graph for tests of a general (non-symmetric) A.

    Each node draws Binomial out-edges to uniform targets (mean
    `mean_degree`); `hub_rows` nodes get `hub_len` out-edges and
    `hub_cols` nodes receive `hub_col_len` extra in-edges (long rows of A
    and of A^T); `empty_rows` nodes have no out-edges at all (zero
    out-degree).  Self-pairs and repeated pairs are dropped.  With
    `weighted`, each edge carries a weight ~ U[w_range], rounded to
    float32."""
    rng = np.random.default_rng(seed)
    lens = rng.binomial(n - 1, min(mean_degree / max(n - 1, 1), 1.0), size=n).astype(np.int64)
    hubs = rng.choice(n, size=min(hub_rows, n), replace=False) if hub_rows else np.empty(0, np.int64)
    lens[hubs] = min(hub_len, n - 1)
    src = np.repeat(np.arange(n, dtype=np.int64), lens)
    dst = rng.integers(0, n, src.shape[0])
    if hub_cols:
        targets = rng.choice(n, size=min(hub_cols, n), replace=False)
        src = np.concatenate([src, rng.integers(0, n, targets.shape[0] * hub_col_len)])
        dst = np.concatenate([dst, np.repeat(targets, hub_col_len)])
    empty = rng.choice(np.setdiff1d(np.arange(n), hubs), size=min(empty_rows, n - hubs.shape[0]),
                       replace=False) if empty_rows else np.empty(0, np.int64)
    keep = (src != dst) & ~np.isin(src, empty)
    code = np.unique(src[keep] * n + dst[keep])
    rows, cols = code // n, code % n
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    values = None
    if weighted:
        values = rng.uniform(w_range[0], w_range[1], rows.shape[0]).astype(np.float32)
    t_indptr, t_indices, t_values = csr_transpose(n, n, indptr, cols, values)
    return DirectedGraph(n=n, indptr=indptr, indices=cols.astype(np.int32), values=values,
                         t_indptr=t_indptr, t_indices=t_indices, t_values=t_values)
