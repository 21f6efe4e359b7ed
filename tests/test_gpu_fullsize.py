"""Parity at the benchmark sizes, in the configuration bench.py times.

The oracle cannot run a whole iSVD at these sizes, so it checks what it can
compute one by one or what holds at any size:
- sampled columns of M Y and M^T Y (the oracle's power sum on those columns);
- the returned triplets: the oracle's FP64 residual of ten sampled triplets,
  the last one included, against the tolerance the device stopped at
  (reading: rho as defined in the oracle), and orthonormality of U and V.
"""

import numpy as np
import pytest
import torch

from gpu_helpers import RHO_SLACK, col_rel_err, featprop_pair, ne_pair, rounded, sampled_triplets, to_dev, to_np
from oracle.isvd import triplet_residuals
from synth import CONFIGS, block_features, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu

SAMPLED = 3


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def c2_graph():
    return make_graph(CONFIGS["c2"])


def _sampled_products(gop, oop, n, l, dt, seed, tol):
    y = rounded(gaussian_block(n, l, seed=seed), dt)
    yd = to_dev(y, dt)
    cols = np.random.default_rng(seed).choice(l, size=SAMPLED, replace=False)
    for tr in (False, True):
        out = to_np(gop.matmul(yd, transpose=tr))
        want = (oop.T if tr else oop).dot(y[:, cols])
        err = col_rel_err(out[:, cols], want)
        assert err <= tol, (tr, err)
    return cols


def _sampled_triplets(gop, oop, k, p, tol, seed, **kw):
    U, S, V, info = gop.truncated_svd(k, p, tol=tol, max_iter=2000, seed=seed, **kw)
    print(info, flush=True)
    assert info.status == 0 and info.residual <= tol
    u = to_np(U).astype(np.float64)
    v = to_np(V).astype(np.float64)
    s = to_np(S)
    assert np.all(np.diff(s) <= 0)
    idx = sampled_triplets(k)
    rho, _ = triplet_residuals(oop, u[:, idx], s[idx], v[:, idx])
    print("sampled oracle residuals", rho, flush=True)
    assert rho.max() <= RHO_SLACK * tol, rho
    assert np.abs(u.T @ u - np.eye(k)).max() < 1e-4
    assert np.abs(v.T @ v - np.eye(k)).max() < 1e-4
    return info


def test_c2_full_products_sampled_columns(gpu_lib, c2_graph):
    cfg = CONFIGS["c2"]
    _case(cfg.name, "products")
    gop, oop = ne_pair(gpu_lib, c2_graph, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    _sampled_products(gop, oop, c2_graph.n, cfg.l, torch.float32, 11, 5e-6)
    gop.close()


def test_c2_full_svd_sampled_triplets(gpu_lib, c2_graph):
    cfg = CONFIGS["c2"]
    _case(cfg.name, "svd")
    gop, oop = ne_pair(gpu_lib, c2_graph, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    _sampled_triplets(gop, oop, cfg.k, cfg.p, 1e-4, 0)
    gop.close()


def test_c4_full_bf16_products_and_svd(gpu_lib):
    cfg = CONFIGS["c4"]
    _case(cfg.name)
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 2)
    # BF16 blocks with FP32 accumulation: each pass rounds its output to 2^-9
    _sampled_products(gop, oop, g.n, cfg.l, torch.bfloat16, 13, 3e-2)
    info = _sampled_triplets(gop, oop, cfg.k, cfg.p, 1e-4, 0, fp32_switch_tol=1e-2)
    assert info.bf16_iterations > 0
    gop.close()


def test_c3_full_featprop_products(gpu_lib):
    cfg = CONFIGS["c3"]
    _case(cfg.name)
    g = make_graph(cfg)
    x = block_features(g.blocks, cfg.d, seed=1000 + cfg.index)
    gop, oop = featprop_pair(gpu_lib, g, x, cfg.L, 1)
    r, c = oop.shape
    y = rounded(gaussian_block(c, cfg.l, seed=17), torch.float32)
    out = to_np(gop.matmul(to_dev(y, torch.float32)))
    cols = np.random.default_rng(17).choice(cfg.l, size=SAMPLED, replace=False)
    assert col_rel_err(out[:, cols], oop.dot(y[:, cols])) <= 5e-6
    z = rounded(gaussian_block(r, cfg.l, seed=18), torch.float32)
    outt = to_np(gop.matmul(to_dev(z, torch.float32), transpose=True))
    assert col_rel_err(outt[:, cols], oop.T.dot(z[:, cols])) <= 5e-6
    gop.close()
