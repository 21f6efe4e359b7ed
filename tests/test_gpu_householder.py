"""Householder QR on the device (Algorithm 2's QR orthonormaliser) against
LAPACK's, and Algorithm 1 with it against the oracle (which orthonormalises
with Householder QR too)."""

import numpy as np
import pytest
import torch

from gpu_helpers import gapped_k, ne_pair, rounded, to_dev, to_np
from oracle.isvd import isvd as oracle_isvd, principal_angles
from synth import CONFIGS, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("rows,l", [(3001, 37), (20000, 144), (129, 128), (5000, 1)])
def test_householder_qr_matches_lapack(gpu_lib, dt, tol, rows, l):
    _case("householder", dt, rows, l)
    rng = np.random.default_rng(rows + l)
    # well conditioned: the factors agree with LAPACK's up to the signs of R's rows
    y = rounded(rng.standard_normal((rows, l)), dt)
    Q, R = gpu_lib.orthonormalize_householder(to_dev(y, dt))
    q, r = to_np(Q).astype(np.float64), to_np(R)
    ql, rl = np.linalg.qr(y)
    assert np.abs(np.tril(r, -1)).max() == 0.0
    sg = np.sign(np.diag(r)) * np.sign(np.diag(rl))
    assert np.abs(sg[:, None] * r - rl).max() <= 10 * tol * np.abs(rl).max()
    assert np.abs(q * sg[None, :] - ql).max() <= 100 * tol
    # ill conditioned (scales over three decades, a near-dependent pair): the
    # backward quantities only, orthogonality and Q R = Y
    y = rng.standard_normal((rows, l)) * np.logspace(0, -3, l)[None, :]
    if l > 2:
        y[:, 2] = y[:, 1] + 1e-6 * y[:, 2]
    y = rounded(y, dt)
    Q, R = gpu_lib.orthonormalize_householder(to_dev(y, dt))
    q, r = to_np(Q).astype(np.float64), to_np(R)
    assert np.abs(q.T @ q - np.eye(l)).max() <= tol * max(l, 16)
    assert np.abs(q @ r - y).max() <= tol * 10 * np.abs(y).max()


def test_svd_with_householder_matches_the_oracle(gpu_lib):
    cfg = CONFIGS["c1"]
    _case(cfg.name, "householder svd")
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 0)
    om = gaussian_block(g.n, cfg.k + cfg.p, seed=cfg.omega_seed)
    U, S, V, info = gop.truncated_svd(cfg.k, cfg.p, q=cfg.q, omega=to_dev(om, torch.float64), orth_method=1)
    uo, so_all, vo = oracle_isvd(oop, cfg.k + cfg.p, om, cfg.q)
    s = to_np(S)
    assert (np.abs(s - so_all[:cfg.k]) / so_all[:cfg.k]).max() <= 1e-10
    kk = gapped_k(so_all, cfg.k)
    assert principal_angles(to_np(U)[:, :kk], uo[:, :kk]).max() <= 1e-8
    assert principal_angles(to_np(V)[:, :kk], vo[:, :kk]).max() <= 1e-8
    with pytest.raises(gpu_lib.IsvdError):
        gop.truncated_svd(cfg.k, cfg.p, q=1, orth_method=2)
    gop.close()
