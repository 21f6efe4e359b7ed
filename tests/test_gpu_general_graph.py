"""The NE design matrix of a general A on the GPU: directed graphs (the CSR
of A^T passed beside A's) and weighted graphs, against the oracle's naive
power sum on the same A.

Section 2 defines T = D^-1 A for any adjacency A (D = row sums, so out-
degrees for a directed graph, weighted degrees for a weighted one), and
Eq. 3's M^T runs through T^T and A^T.  The graphs here have rows longer
than the 256-entry hub threshold in both A and A^T and rows with no
out-edges (zero out-degree: a zero row of T)."""

import numpy as np
import pytest
import torch

from gpu_helpers import col_rel_err, gapped_k, ne_pair_general, rounded, to_dev, to_np
from oracle.isvd import isvd as oracle_isvd, principal_angles
from synth import chung_lu_graph, directed_graph, gaussian_block

pytestmark = pytest.mark.gpu

DT = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}
TOL = {0: 1e-13, 1: 5e-6}


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def dgraph():
    g = directed_graph(5000, 6.0, seed=31, hub_rows=3, hub_len=600, hub_cols=3, hub_col_len=700,
                       empty_rows=50)
    lens, tlens = np.diff(g.indptr), np.diff(g.t_indptr)
    assert lens.max() > 256 and tlens.max() > 256          # hub rows in A and in A^T
    assert (lens == 0).sum() >= 50 and (tlens == 0).any()   # zero out-degree and zero in-degree
    return g


def _products(lib, g, coeffs, lam, loops, precision, ncols, weighted, seed=5):
    dt = DT[precision]
    gop, oop = ne_pair_general(lib, g, coeffs, lam, loops, precision, weighted=weighted)
    y = rounded(gaussian_block(g.n, ncols, seed=seed), dt)
    yd = to_dev(y, dt)
    for tr in (False, True):
        out = to_np(gop.matmul(yd, transpose=tr))
        want = (oop.T if tr else oop).dot(y)
        err = col_rel_err(out, want)
        assert err <= TOL[precision], (tr, err)
    gop.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("weighted", [True, False])
@pytest.mark.parametrize("loops", [False, True])
@pytest.mark.parametrize("K", [1, 3])
def test_directed_products(gpu_lib, dgraph, precision, weighted, loops, K):
    _case("directed", precision, weighted, loops, K)
    coeffs = np.array([0.6, -0.3, 0.2])[:K]
    _products(gpu_lib, dgraph, coeffs, 0.2, loops, precision, 42, weighted)


@pytest.mark.parametrize("ncols", [1, 80, 144, 288])
def test_directed_weighted_widths_fp32(gpu_lib, dgraph, ncols):
    _case("directed widths", ncols)
    _products(gpu_lib, dgraph, np.full(4, 0.25), 0.1, False, 1, ncols, True)


def test_symmetric_weighted_products(gpu_lib):
    # a weighted undirected graph: A symmetric, weights given once, no A^T arrays
    _case("symmetric weighted")
    g = chung_lu_graph(6000, 2.2, 12.0, seed=33)
    rng = np.random.default_rng(34)
    rows = np.repeat(np.arange(g.n), np.diff(g.indptr))
    cols = g.indices.astype(np.int64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    uniq, inv = np.unique(lo * g.n + hi, return_inverse=True)
    w = rng.uniform(0.5, 3.0, uniq.shape[0]).astype(np.float32)[inv]   # w_ij = w_ji
    from oracle.operators import NEDesignMatrix
    assert np.diff(g.indptr).max() > 256
    for precision in (0, 1):
        dt = DT[precision]
        gop = gpu_lib.Operator(g, form="ne", coeffs=np.full(3, 1 / 3), lam=0.05, precision=precision, values=w)
        oop = NEDesignMatrix.from_graph(g, np.full(3, 1 / 3), 0.05, values=w.astype(np.float64))
        y = rounded(gaussian_block(g.n, 37, seed=35), dt)
        for tr in (False, True):
            out = to_np(gop.matmul(to_dev(y, dt), transpose=tr))
            assert col_rel_err(out, (oop.T if tr else oop).dot(y)) <= TOL[precision], tr
        gop.close()


def test_directed_empty_graph(gpu_lib):
    _case("directed empty")
    from synth import DirectedGraph
    n = 12
    z = np.zeros(n + 1, dtype=np.int64)
    g = DirectedGraph(n=n, indptr=z, indices=np.empty(0, np.int32), values=np.empty(0, np.float32),
                      t_indptr=z, t_indices=np.empty(0, np.int32), t_values=np.empty(0, np.float32))
    _products(gpu_lib, g, np.array([0.5, 0.5]), 0.2, False, 0, 3, True)


@pytest.mark.parametrize("precision,s_tol", [(0, 1e-10), (1, 1e-4)])
def test_directed_weighted_svd_matches_oracle(gpu_lib, dgraph, precision, s_tol):
    # Algorithm 1 on a general A: every product runs both directions
    _case("directed svd", precision)
    k, p, q = 24, 8, 2
    dt = DT[precision]
    coeffs, lam = np.full(3, 1 / 3), 0.1
    gop, oop = ne_pair_general(gpu_lib, dgraph, coeffs, lam, False, precision)
    om = rounded(gaussian_block(dgraph.n, k + p, seed=36), dt)
    U, S, V, info = gop.truncated_svd(k, p, q=q, omega=to_dev(om, dt))
    uo, so, vo = oracle_isvd(oop, k + p, om, q)
    s = to_np(S)
    assert np.max(np.abs(s - so[:k]) / so[:k]) <= s_tol
    # top subspaces up to the last index whose Ritz gap separates them
    kk = gapped_k(so, k)
    assert kk >= k // 2, kk
    ang_u = principal_angles(to_np(U)[:, :kk].astype(np.float64), uo[:, :kk]).max()
    ang_v = principal_angles(to_np(V)[:, :kk].astype(np.float64), vo[:, :kk]).max()
    assert ang_u <= 1e-3 and ang_v <= 1e-3, (ang_u, ang_v)
    gop.close()


def test_directed_rejects_missing_transpose(gpu_lib, dgraph):
    _case("directed invalid")
    with pytest.raises(gpu_lib.IsvdError) as e:
        gpu_lib.Operator(dgraph, form="ne", coeffs=[1.0], symmetric=False)
    assert e.value.status == gpu_lib.ISVD_E_INVALID
    with pytest.raises(gpu_lib.IsvdError):
        gpu_lib.Operator(dgraph, form="ne", coeffs=[1.0], symmetric=False, values=dgraph.values,
                         t_indptr=dgraph.t_indptr, t_indices=dgraph.t_indices)
