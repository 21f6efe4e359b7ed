"""Full-size parity of the paths beyond the hot path, in the configurations
bench.py times (--dag, --learners, --ablation): the Fig. 1 DAG of the
n = 200,000 NE workload against the fused operator and the oracle on sampled
columns; the learners on the device SVD outputs against the oracle; the
Householder QR of a 200,000 x 144 block (orthogonality and Q R = Y)."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_helpers import col_rel_err, ne_pair, rounded, to_dev, to_np
from oracle import learners as ol
from synth import CONFIGS, block_features, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def c2():
    cfg = CONFIGS["c2"]
    return cfg, make_graph(cfg)


def test_c2_fig1_dag_products_sampled_columns(gpu_lib, c2):
    cfg, g = c2
    _case(cfg.name, "fig1 dag")
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(g.n, g.n))
    deg = np.diff(a.indptr).astype(np.float64)
    dag = gpu_lib.Dag(gpu_lib.FP32)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    t = dag.diag(np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)) @ A
    one = dag.dense(torch.ones((g.n, 1), dtype=torch.float32, device="cuda"))
    m = dag.sum([t ** j for j in range(1, cfg.K + 1)], cfg.coeffs) - cfg.lam * (one @ one.T - A)
    op = dag.operator(m)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    y = rounded(gaussian_block(g.n, cfg.l, seed=21), torch.float32)
    yd = to_dev(y, torch.float32)
    cols = np.random.default_rng(21).choice(cfg.l, size=3, replace=False)
    for tr in (False, True):
        out = to_np(op.matmul(yd, transpose=tr))
        fused = to_np(gop.matmul(yd, transpose=tr))
        want = (oop.T if tr else oop).dot(y[:, cols])
        assert col_rel_err(out[:, cols], want) <= 5e-6
        assert col_rel_err(out, fused) <= 5e-6
    op.close()
    gop.close()
    dag.close()


def test_c2_learners_on_the_device_svd(gpu_lib, c2):
    cfg, g = c2
    _case(cfg.name, "learners")
    gop, _ = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    U, S, V, info = gop.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=0)
    gop.close()
    u, s, v = to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64)
    L, R = gpu_lib.ne_embeddings(U, S, V)
    lw, rw = ol.ne_embeddings(u, s, v)
    assert np.abs(to_np(L) - lw).max() <= 2.0 ** -23 * np.abs(lw).max()
    assert np.abs(to_np(R) - rw).max() <= 2.0 ** -23 * np.abs(rw).max()
    rng = np.random.default_rng(5)
    pi, pj = rng.integers(0, g.n, 2_000_000), rng.integers(0, g.n, 2_000_000)
    got = to_np(gpu_lib.ne_scores(U, S, V, torch.as_tensor(pi).cuda(), torch.as_tensor(pj).cuda()))
    want = ol.ne_scores(u, s, v, pi, pj)
    mag = np.einsum("pt,pt->p", np.abs(u[pi]) * s, np.abs(v[pj]))
    assert (np.abs(got - want) <= 4 * cfg.k * np.finfo(np.float64).eps * mag).all()


def test_c3_nc_fit_on_the_device_svd(gpu_lib):
    cfg = CONFIGS["c3"]
    _case(cfg.name, "nc fit")
    g = make_graph(cfg)
    x = torch.as_tensor(block_features(g.blocks, cfg.d, seed=1000 + cfg.index)).cuda()
    op = gpu_lib.Operator(g, form="featprop", X=x, L=cfg.L, precision=gpu_lib.FP32)
    U, S, V, info = op.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=0)
    op.close()
    ny = int(g.blocks.max()) + 1
    y = np.zeros((g.n, ny), dtype=np.float32)
    y[np.arange(g.n), g.blocks] = 1.0
    rows = np.sort(np.random.default_rng(6).choice(g.n, g.n // 2, replace=False))
    W = gpu_lib.nc_fit(U, S, V, torch.as_tensor(y).cuda(), rows=torch.as_tensor(rows).cuda())
    u, s, v = to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64)
    want = ol.nc_fit(u, s, v, y.astype(np.float64), rows=rows)
    bound = np.abs(v) @ (ol.s_pinv(s)[:, None] * (np.abs(u[rows]).T @ np.abs(y[rows].astype(np.float64))))
    assert (np.abs(to_np(W) - want) <= 4 * (len(rows) + cfg.k) * np.finfo(np.float64).eps * bound).all()


def test_householder_qr_full_block(gpu_lib):
    _case("householder 200000 x 144")
    Y = gpu_lib.gaussian_block(200000, 144, seed=9, dtype=torch.float32)
    y = to_np(Y).astype(np.float64)
    Q, R = gpu_lib.orthonormalize_householder(Y)
    q, r = to_np(Q).astype(np.float64), to_np(R)
    assert np.abs(q.T @ q - np.eye(144)).max() < 1e-5
    assert np.abs(q @ r - y).max() < 1e-4 * np.abs(y).max()
