"""Symbolic design matrices (Section 4 and the appendix) on the device, through
the C-ABI: every node type against the oracle's DAG, the Fig. 1 construction
against the NE design matrix (and the fused NE operator), the feature form as
a concatenation, the lazy cache (same products, fewer passes), and
Algorithm 1 on a DAG operator against the oracle."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_helpers import col_rel_err, gapped_k, rounded, to_dev, to_np
from oracle.isvd import isvd as oracle_isvd, principal_angles
from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix
from oracle import symbolic as sym
from synth import CONFIGS, block_features, chung_lu_graph, gaussian_block, sbm_graph
from synth.configs import make_graph

pytestmark = pytest.mark.gpu

DT = {0: torch.float64, 1: torch.float32}
TOL = {0: 1e-12, 1: 2e-5}


def _case(*a):
    print("CASE", *a, flush=True)


def _csr_of(g, loops=False):
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(g.n, g.n))
    if loops:
        a = (a + sp.identity(g.n, format="csr")).tocsr()
    a.sort_indices()
    return a


def _fig1(lib, g, coeffs, lam, precision, cache=True):
    """Fig. 1: t = (1/d) a, M = sum_j c_j t^j - lam (1 1^T - a), built from leaves."""
    dag = lib.Dag(precision)
    a = _csr_of(g)
    deg = np.diff(a.indptr).astype(np.float64)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    t = dag.diag(np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)) @ A
    one = dag.dense(torch.ones((g.n, 1), dtype=DT[precision], device="cuda"))
    m = coeffs[0] * t
    for j in range(2, len(coeffs) + 1):
        m = m + coeffs[j - 1] * (t ** j)
    m = m - lam * (one @ one.T - A)
    return dag, dag.operator(m, lazy_cache=cache)


def _check_products(op, ref, precision, l=13, seed=3):
    dt = DT[precision]
    y = rounded(gaussian_block(ref.shape[1], l, seed=seed), dt)
    assert col_rel_err(to_np(op.matmul(to_dev(y, dt))), ref.dot(y)) <= TOL[precision]
    z = rounded(gaussian_block(ref.shape[0], l, seed=seed + 1), dt)
    assert col_rel_err(to_np(op.matmul(to_dev(z, dt), transpose=True)), ref.T.dot(z)) <= TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("cache", [True, False])
def test_fig1_construction(gpu_lib, precision, cache):
    _case("fig1", precision, cache)
    g = chung_lu_graph(3000, 2.5, 8.0, seed=41)
    coeffs = np.array([3.0, 2.0, 1.0]) / 6.0
    dag, op = _fig1(gpu_lib, g, coeffs, 0.07, precision, cache)
    assert op.shape == (g.n, g.n)
    _check_products(op, NEDesignMatrix.from_graph(g, coeffs, 0.07), precision)
    op.close()
    dag.close()


def test_fig1_matches_the_fused_operator(gpu_lib):
    _case("fig1 vs fused")
    g = chung_lu_graph(5000, 2.3, 12.0, seed=42)
    coeffs = np.full(5, 0.2)
    dag, op = _fig1(gpu_lib, g, coeffs, 0.05, 0)
    fused = gpu_lib.Operator(g, form="ne", coeffs=coeffs, lam=0.05, precision=0)
    y = to_dev(gaussian_block(g.n, 24, seed=5), torch.float64)
    for tr in (False, True):
        a, b = to_np(op.matmul(y, transpose=tr)), to_np(fused.matmul(y, transpose=tr))
        assert col_rel_err(a, b) <= 1e-12
    op.close()
    fused.close()
    dag.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_feature_form_as_concatenation(gpu_lib, precision):
    _case("featprop concat", precision)
    g = sbm_graph(4000, 6, 0.005, 0.0004, seed=43)
    x = block_features(g.blocks, 16, seed=44)
    dt = DT[precision]
    xd = to_dev(x, dt)
    dag = gpu_lib.Dag(precision)
    a = _csr_of(g, loops=True)
    r = 1.0 / np.sqrt(np.diff(a.indptr).astype(np.float64))
    R = dag.diag(r)
    ah = R @ dag.sparse(a.indptr, a.indices, a.shape) @ R
    X = dag.dense(xd)
    m = dag.concat_cols([X] + [(ah ** j) @ X for j in range(1, 4)])
    op = dag.operator(m)
    _check_products(op, FeatPropDesignMatrix.from_graph(g, rounded(x, dt), 3), precision, l=11)
    op.close()
    dag.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_every_node_type_against_the_oracle(gpu_lib, precision):
    _case("dag nodes", precision)
    rng = np.random.default_rng(7)
    dt = DT[precision]
    a = sp.random(700, 500, density=0.02, random_state=8, format="csr", dtype=np.float64)
    a.data = rounded(a.data, torch.float32)
    c = sp.random(700, 700, density=0.01, random_state=9, format="csr", dtype=np.float64)
    c.data = rounded(c.data, torch.float32)
    at, ct_ = a.T.tocsr(), c.T.tocsr()
    b = rounded(rng.standard_normal((500, 33)), dt)
    d = rng.uniform(0.5, 2.0, 700)
    dag = gpu_lib.Dag(precision)
    A = dag.sparse(a.indptr, a.indices, a.shape, values=a.data, symmetric=False, t_indptr=at.indptr,
                   t_indices=at.indices, t_values=at.data)
    C = dag.sparse(c.indptr, c.indices, c.shape, values=c.data, symmetric=False, t_indptr=ct_.indptr,
                   t_indices=ct_.indices, t_values=ct_.data)
    B = dag.dense(to_dev(b, dt))
    D = dag.diag(d)
    oA, oC, oB, oD = sym.sparse(a), sym.sparse(c), sym.dense(b), sym.diag(d)
    rows = rng.choice(700, 250, replace=False)
    cols = np.random.default_rng(70).choice(500, 120, replace=False)
    cases = [
        (A, oA),
        (B, oB),
        (D @ C @ D, oD @ oC @ oD),
        (C ** 3 - 0.5 * D, oC ** 3 - 0.5 * oD),
        ((A @ B).T @ (C @ A @ B), (oA @ oB).T @ (oC @ oA @ oB)),
        ((C @ A).gather_rows(rows), sym.take_rows(oC @ oA, rows)),
        ((C @ A).gather_rows(rows).T, sym.take_rows(oC @ oA, rows).T),
        (dag.concat_cols([A, C, D @ A]), sym.hstack([oA, oC, oD @ oA])),
        (dag.concat_cols([A, C]).T, sym.hstack([oA, oC]).T),
        # a column gather M[:, cols] is the transpose of a row gather of M^T
        ((C @ A).T.gather_rows(cols).T, sym.take_rows((oC @ oA).T, cols).T),
        (2.0 * (C @ C + D) @ C - C, 2.0 * (oC @ oC + oD) @ oC - oC),
    ]
    for i, (node, ref) in enumerate(cases):
        print("node case", i, node.shape, flush=True)
        assert node.shape == ref.shape
        for cache in (True, False):
            op = dag.operator(node, lazy_cache=cache)
            _check_products(op, ref, precision, l=9, seed=10 + i)
            op.close()
    dag.close()


def test_dag_errors(gpu_lib):
    _case("dag errors")
    dag = gpu_lib.Dag(0)
    A = dag.sparse(np.array([0, 1, 2]), np.array([1, 0]), (2, 2))
    B = dag.dense(torch.ones((3, 2), dtype=torch.float64, device="cuda"))
    with pytest.raises(gpu_lib.IsvdError):
        A @ B                                   # inner dimensions differ
    with pytest.raises(gpu_lib.IsvdError):
        A + B                                   # shapes differ
    with pytest.raises(gpu_lib.IsvdError):
        A.gather_rows([0, 0])                   # repeated row
    with pytest.raises(gpu_lib.IsvdError):
        A.gather_rows([2])                      # out of range
    with pytest.raises(gpu_lib.IsvdError):
        dag.sparse(np.array([0, 1, 1]), np.array([1]), (2, 2), symmetric=False)   # no transpose CSR
    dag.close()


def test_svd_of_a_dag_operator_matches_the_oracle(gpu_lib):
    # Algorithm 1 on the Fig. 1 DAG of the C1 workload, same start block as the oracle
    cfg = CONFIGS["c1"]
    _case(cfg.name, "dag svd")
    g = make_graph(cfg)
    coeffs = cfg.coeffs
    dag = gpu_lib.Dag(0)
    a = _csr_of(g, loops=cfg.self_loops)
    deg = np.diff(a.indptr).astype(np.float64)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    t = dag.diag(np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)) @ A
    one = dag.dense(torch.ones((g.n, 1), dtype=torch.float64, device="cuda"))
    m = dag.sum([t ** j for j in range(1, len(coeffs) + 1)], coeffs) - cfg.lam * (one @ one.T - A)
    op = dag.operator(m)
    oop = NEDesignMatrix.from_graph(g, coeffs, cfg.lam, add_self_loops=cfg.self_loops)
    om = gaussian_block(g.n, cfg.k + cfg.p, seed=cfg.omega_seed)
    U, S, V, info = op.truncated_svd(cfg.k, cfg.p, q=cfg.q, omega=to_dev(om, torch.float64))
    uo, so_all, vo = oracle_isvd(oop, cfg.k + cfg.p, om, cfg.q)
    s = to_np(S)
    assert (np.abs(s - so_all[:cfg.k]) / so_all[:cfg.k]).max() <= 1e-10
    kk = gapped_k(so_all, cfg.k)
    assert principal_angles(to_np(U)[:, :kk], uo[:, :kk]).max() <= 1e-8
    op.close()
    dag.close()


def test_operator_outlives_its_dag_handle(gpu_lib):
    _case("dag lifetime")
    g = chung_lu_graph(2000, 2.5, 8.0, seed=44)
    coeffs = np.array([0.5, 0.5])
    dag, op = _fig1(gpu_lib, g, coeffs, 0.1, 0)
    y = to_dev(gaussian_block(g.n, 5, seed=6), torch.float64)
    before = to_np(op.matmul(y))
    keep = dag._keep                   # the leaves' device arrays stay alive (caller's side)
    dag.close()                        # the operator keeps the nodes
    after = to_np(op.matmul(y))
    assert np.array_equal(before, after)
    op.close()
    del keep
