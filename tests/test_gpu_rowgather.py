"""Implicit row gather (Section 3.2, option (ii)) through the C-ABI:
products with M[rows, :] and the SVD of the submatrix against the oracle's
RowGather, and the node-classification pipeline of Section 3.2 (SVD of the
labelled rows, then the least-norm model of Eq. 8, Theorem 1)."""

import numpy as np
import pytest
import torch

from gpu_helpers import RHO_SLACK, col_rel_err, featprop_pair, ne_pair, rounded, sampled_triplets, to_dev, to_np
from oracle import learners as ol
from oracle.isvd import triplet_residuals
from oracle.operators import RowGather
from synth import CONFIGS, block_features, chung_lu_graph, gaussian_block, sbm_graph
from synth.configs import make_graph

pytestmark = pytest.mark.gpu

DT = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}


def _case(*a):
    print("CASE", *a, flush=True)


def _products(gop, oop, rows, precision, l, tol, seed):
    dt = DT[precision]
    sub = RowGather(oop, rows)
    gop.gather_rows(torch.as_tensor(rows).cuda())
    assert gop.shape == sub.shape
    y = rounded(gaussian_block(sub.shape[1], l, seed=seed), dt)
    assert col_rel_err(to_np(gop.matmul(to_dev(y, dt))), sub.dot(y)) <= tol
    z = rounded(gaussian_block(sub.shape[0], l, seed=seed + 1), dt)
    assert col_rel_err(to_np(gop.matmul(to_dev(z, dt), transpose=True)), sub.T.dot(z)) <= tol


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-5)])
@pytest.mark.parametrize("L", [0, 2])
def test_featprop_row_gather_products(gpu_lib, precision, tol, L):
    _case("featprop gather", precision, L)
    g = sbm_graph(6000, 8, 0.004, 0.0003, seed=26)
    x = block_features(g.blocks, 24, seed=27)
    gop, oop = featprop_pair(gpu_lib, g, x, L, precision)
    rng = np.random.default_rng(L)
    for nsel in (1, 777, 6000):           # one row, a ragged subset, a permutation of all rows
        _products(gop, oop, rng.permutation(g.n)[:nsel], precision, 19, tol, seed=30 + nsel)
    gop.gather_rows(None)
    assert gop.shape == oop.shape
    gop.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 5e-6), (2, 3e-2)])
def test_ne_row_gather_products(gpu_lib, precision, tol):
    _case("ne gather", precision)
    g = chung_lu_graph(5000, 2.5, 10.0, seed=24)
    gop, oop = ne_pair(gpu_lib, g, np.full(3, 1 / 3), 0.1, False, precision)
    rows = np.sort(np.random.default_rng(3).choice(g.n, 1234, replace=False))
    _products(gop, oop, rows, precision, 40, tol, seed=41)
    gop.close()


def test_row_gather_errors_leave_the_operator_whole(gpu_lib):
    _case("gather errors")
    g = sbm_graph(500, 4, 0.02, 0.002, seed=3)
    gop, oop = ne_pair(gpu_lib, g, np.full(2, 0.5), 0.1, False, 0)
    for bad in ([0, 500], [-1], [3, 7, 3]):
        with pytest.raises(gpu_lib.IsvdError) as ei:
            gop.gather_rows(torch.tensor(bad))
        assert ei.value.status == gpu_lib.ISVD_E_INVALID
        gop.gather_rows(None)
        assert gop.shape == (500, 500)
    y = rounded(gaussian_block(500, 3, seed=4), torch.float64)
    assert col_rel_err(to_np(gop.matmul(to_dev(y, torch.float64))), oop.dot(y)) <= 1e-13
    gop.close()


def test_nc_pipeline_labelled_rows_least_norm(gpu_lib):
    # Section 3.2 option (ii): SVD of M[labelled, :] at full rank (k = F), then
    # W = V S^+ U^T Y_labelled is the least-norm least-squares fit (Theorem 1)
    _case("nc pipeline")
    g = sbm_graph(4000, 6, 0.005, 0.0004, seed=31)
    d, L = 12, 2
    x = block_features(g.blocks, d, seed=32)
    gop, oop = featprop_pair(gpu_lib, g, x, L, 0)
    F = d * (L + 1)
    labelled = np.sort(np.random.default_rng(33).choice(g.n, 900, replace=False))
    gop.gather_rows(torch.as_tensor(labelled).cuda())
    om = gaussian_block(F, F, seed=34)
    U, S, V, info = gop.truncated_svd(F, 0, q=0, omega=to_dev(om, torch.float64))
    m_sub = RowGather(oop, labelled).dot(np.eye(F))
    assert np.allclose(to_np(S), np.linalg.svd(m_sub, compute_uv=False), rtol=1e-10)
    y = np.zeros((g.n, int(g.blocks.max()) + 1))
    y[np.arange(g.n), g.blocks] = 1.0
    ysub = y[labelled]
    W = gpu_lib.nc_fit(U, S, V, to_dev(ysub, torch.float64))
    assert np.allclose(to_np(W), ol.nc_fit(to_np(U), to_np(S), to_np(V), ysub), rtol=1e-10, atol=1e-12)
    ls = np.linalg.lstsq(m_sub, ysub, rcond=None)[0]
    assert np.allclose(to_np(W), ls, rtol=1e-7, atol=1e-9 * np.abs(ls).max())
    gop.close()


def test_c3_full_size_labelled_rows_svd(gpu_lib):
    # the feature-propagation workload at full size (n = 170,000), half of the
    # rows labelled: sampled triplets of the device SVD of M[labelled, :]
    # against the oracle's residual
    cfg = CONFIGS["c3"]
    _case(cfg.name, "gathered rows")
    g = make_graph(cfg)
    x = block_features(g.blocks, cfg.d, seed=1000 + cfg.index)
    gop, oop = featprop_pair(gpu_lib, g, x, cfg.L, 1)
    labelled = np.sort(np.random.default_rng(35).choice(g.n, g.n // 2, replace=False))
    gop.gather_rows(torch.as_tensor(labelled).cuda())
    U, S, V, info = gop.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=0)
    print(info, flush=True)
    assert info.status == 0 and info.residual <= 1e-4
    u, s, v = to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64)
    idx = sampled_triplets(cfg.k)
    rho, _ = triplet_residuals(RowGather(oop, labelled), u[:, idx], s[idx], v[:, idx])
    print("sampled oracle residuals", rho, flush=True)
    assert rho.max() <= RHO_SLACK * 1e-4, rho
    assert np.abs(u.T @ u - np.eye(cfg.k)).max() < 1e-4
    gop.close()
