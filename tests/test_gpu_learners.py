"""Parity of the closed-form learners (Section 3: Eq. 5 embeddings and pair
scores, Eq. 8 least-norm model) with the FP64 oracle, through the C-ABI.

Bounds: the device sums exact FP64 products in another order than numpy, so
each output is checked against c * eps64 * (the same sum over |terms|).
"""

import numpy as np
import pytest
import torch

from gpu_helpers import featprop_pair, rounded, to_dev, to_np
from oracle import learners as ol
from synth import CONFIGS, block_features, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _case(*a):
    print("CASE", *a, flush=True)


def _factors(rows_u, rows_v, k, seed):
    """Orthonormal U, V and descending S spanning several decades."""
    rng = np.random.default_rng(seed)
    u = np.linalg.qr(rng.standard_normal((rows_u, k)))[0]
    v = np.linalg.qr(rng.standard_normal((rows_v, k)))[0]
    s = np.sort(10.0 ** rng.uniform(-3, 3, k))[::-1].copy()
    return u, s, v


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("rows_u,rows_v,k", [(1000, 777, 37), (3001, 2500, 64), (257, 300, 128)])
def test_embeddings(gpu_lib, dt, rows_u, rows_v, k):
    _case("embeddings", dt, rows_u, rows_v, k)
    u, s, v = _factors(rows_u, rows_v, k, seed=rows_u + k)
    u, v = rounded(u, dt), rounded(v, dt)
    L, R = gpu_lib.ne_embeddings(to_dev(u, dt), to_dev(s, torch.float64), to_dev(v, dt))
    lw, rw = ol.ne_embeddings(u, s, v)
    # one rounding of an FP64 product (and of the square root), then to dt
    rel = 4 * EPS if dt == torch.float64 else 2.0 ** -24
    for got, want in ((L, lw), (R, rw)):
        assert got.dtype == dt
        err = np.abs(to_np(got) - rounded(want, dt))
        assert (err <= rel * np.abs(want)).all(), err.max()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("k,npairs", [(37, 5000), (64, 20001), (256, 1), (132, 4099)])
def test_pair_scores(gpu_lib, dt, k, npairs):
    _case("scores", dt, k, npairs)
    u, s, v = _factors(2000, 1500, k, seed=k)
    u, v = rounded(u, dt), rounded(v, dt)
    rng = np.random.default_rng(npairs)
    pi = rng.integers(0, 2000, npairs)
    pj = rng.integers(0, 1500, npairs)
    got = to_np(gpu_lib.ne_scores(to_dev(u, dt), to_dev(s, torch.float64), to_dev(v, dt),
                                  torch.as_tensor(pi).cuda(), torch.as_tensor(pj).cuda()))
    want = ol.ne_scores(u, s, v, pi, pj)
    mag = np.einsum("pt,pt->p", np.abs(u[pi]) * s, np.abs(v[pj]))
    assert (np.abs(got - want) <= 4 * k * EPS * mag).all()


def test_pair_scores_empty_and_bad_index(gpu_lib):
    _case("scores edge")
    u, s, v = _factors(100, 80, 16, seed=3)
    U, S, V = to_dev(u, torch.float64), to_dev(s, torch.float64), to_dev(v, torch.float64)
    e = torch.zeros(0, dtype=torch.int64, device="cuda")
    assert gpu_lib.ne_scores(U, S, V, e, e).shape == (0,)
    for pi, pj in (([0, 100], [0, 1]), ([0, 1], [-1, 2]), ([5], [80])):
        with pytest.raises(gpu_lib.IsvdError) as ei:
            gpu_lib.ne_scores(U, S, V, torch.tensor(pi, device="cuda"), torch.tensor(pj, device="cuda"))
        assert ei.value.status == gpu_lib.ISVD_E_INVALID


def _nc_bound(u, s, v, y, rows, rcond):
    """Sum of |terms| of each element of V S^+ (U^T Y)."""
    if rows is not None:
        u, y = u[rows], y[rows]
    return np.abs(v) @ (ol.s_pinv(s, rcond)[:, None] * (np.abs(u).T @ np.abs(y)))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("rows_u,rows_v,k,ny,subset,rcond", [
    (3001, 1999, 37, 7, None, 0.0),
    (20000, 5000, 128, 40, 2500, 0.0),
    (5000, 5000, 64, 1, 777, 1e-4),
    (1000, 300, 250, 130, None, 1e-5),
])
def test_nc_fit(gpu_lib, dt, rows_u, rows_v, k, ny, subset, rcond):
    _case("nc_fit", dt, rows_u, rows_v, k, ny, subset, rcond)
    u, s, v = _factors(rows_u, rows_v, k, seed=rows_u + ny)
    u, v = rounded(u, dt), rounded(v, dt)
    rng = np.random.default_rng(ny)
    y = np.zeros((rows_u, ny))
    y[np.arange(rows_u), rng.integers(0, ny, rows_u)] = 1.0       # one-hot labels
    rows = None if subset is None else np.sort(rng.choice(rows_u, subset, replace=False))
    W = gpu_lib.nc_fit(to_dev(u, dt), to_dev(s, torch.float64), to_dev(v, dt), to_dev(y, dt),
                       rows=None if rows is None else torch.as_tensor(rows).cuda(), rcond=rcond)
    want = ol.nc_fit(u, s, v, y, rows=rows, rcond=rcond)
    bound = _nc_bound(u, s, v, y, rows, rcond)
    n = rows_u if rows is None else subset
    assert W.shape == (rows_v, ny) and W.dtype == torch.float64
    assert (np.abs(to_np(W) - want) <= 4 * (n + k) * EPS * bound).all()


def test_nc_fit_edges(gpu_lib):
    _case("nc_fit edges")
    u, s, v = _factors(500, 400, 20, seed=9)
    U, S, V = to_dev(u, torch.float64), to_dev(s, torch.float64), to_dev(v, torch.float64)
    y = np.random.default_rng(1).standard_normal((500, 3))
    Y = to_dev(y, torch.float64)
    # empty subset: no labels, W = 0
    W = gpu_lib.nc_fit(U, S, V, Y, rows=torch.zeros(0, dtype=torch.int64, device="cuda"))
    assert torch.count_nonzero(W).item() == 0
    # repeated rows count twice (the subset is taken as given)
    rows = np.array([3, 3, 10, 499])
    W = gpu_lib.nc_fit(U, S, V, Y, rows=torch.as_tensor(rows).cuda())
    assert np.allclose(to_np(W), ol.nc_fit(u, s, v, y, rows=rows), rtol=1e-12, atol=1e-14)
    # an rcond above every ratio keeps s_1 only
    W = gpu_lib.nc_fit(U, S, V, Y, rcond=0.999999)
    assert np.allclose(to_np(W), np.outer(v[:, 0], u[:, 0] @ y) / s[0], rtol=1e-12, atol=1e-14)
    for bad in ([0, 500], [-1]):
        with pytest.raises(gpu_lib.IsvdError) as ei:
            gpu_lib.nc_fit(U, S, V, Y, rows=torch.tensor(bad, device="cuda"))
        assert ei.value.status == gpu_lib.ISVD_E_INVALID
    with pytest.raises(gpu_lib.IsvdError):
        gpu_lib.nc_fit(U, S, V, to_dev(np.zeros((500, 2040)), torch.float64))   # k + ny > 2048


def test_featprop_svd_then_least_norm_model(gpu_lib):
    # L = 0 and k = d: M = X exactly, so Eq. 8 on the device SVD gives the
    # least-norm least-squares solution of X W = Y (Theorem 1).
    _case("featprop + nc_fit")
    cfg = CONFIGS["c3"].scaled(4000)
    g = make_graph(cfg)
    d = 24
    x = block_features(g.blocks, d, seed=21)
    gop, oop = featprop_pair(gpu_lib, g, x, 0, 0)
    om = gaussian_block(d, d, seed=22)
    U, S, V, info = gop.truncated_svd(d, 0, q=0, omega=to_dev(om, torch.float64))
    xr = rounded(x, torch.float64)
    y = np.zeros((g.n, int(g.blocks.max()) + 1))
    y[np.arange(g.n), g.blocks] = 1.0
    labelled = np.sort(np.random.default_rng(23).choice(g.n, g.n // 10, replace=False))
    W = gpu_lib.nc_fit(U, S, V, to_dev(y, torch.float64), rows=torch.as_tensor(labelled).cuda())
    want = ol.nc_fit(to_np(U), to_np(S), to_np(V), y, rows=labelled)
    assert np.allclose(to_np(W), want, rtol=1e-10, atol=1e-12)
    # Theorem 1, all rows labelled: W is the least-norm least-squares solution of X W = Y
    Wf = gpu_lib.nc_fit(U, S, V, to_dev(y, torch.float64))
    lsf = np.linalg.lstsq(xr, y, rcond=None)[0]
    assert np.allclose(to_np(Wf), lsf, rtol=1e-8, atol=1e-10 * np.abs(lsf).max())
    gop.close()
