"""End-to-end parity of isvd_truncated_svd with the FP64 oracle on the same
start block: singular values to 1e-10 (FP64 path) / 1e-4 (FP32 path)
relative, top-k' subspaces (k' = largest index with a Ritz gap >= 1e-3)
within 1e-3 rad; tolerance mode checked against the oracle's residual."""

import numpy as np
import pytest
import torch

from gpu_helpers import featprop_pair, gapped_k, ne_pair, rounded, to_dev, to_np
from oracle.isvd import isvd as oracle_isvd, principal_angles, triplet_residuals
from synth import CONFIGS, block_features, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu

DT = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}


def _case(*a):
    print("CASE", *a, flush=True)


def _compare(gop, oop, k, p, q, precision, s_tol, ang_tol, omega_seed):
    dt = DT[precision]
    c = oop.shape[1]
    om = rounded(gaussian_block(c, k + p, seed=omega_seed), dt)
    U, S, V, info = gop.truncated_svd(k, p, q=q, omega=to_dev(om, dt))
    u, s, v = to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64)
    uo, so_all, vo = oracle_isvd(oop, k + p, om, q)
    so = so_all[:k]
    assert info.iterations == q
    rel = np.abs(s - so) / so
    assert rel.max() <= s_tol, rel.max()
    kk = gapped_k(so_all, k)
    if kk > 0:
        assert principal_angles(u[:, :kk], uo[:, :kk]).max() <= ang_tol
        assert principal_angles(v[:, :kk], vo[:, :kk]).max() <= ang_tol
    assert np.abs(u.T @ u - np.eye(k)).max() < (1e-12 if precision == 0 else 1e-4)
    assert np.abs(v.T @ v - np.eye(k)).max() < (1e-12 if precision == 0 else 1e-4)
    return rel.max(), kk


def test_config1_fp64(gpu_lib):
    cfg = CONFIGS["c1"]
    _case(cfg.name)
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 0)
    _compare(gop, oop, cfg.k, cfg.p, cfg.q, 0, 1e-10, 1e-8, cfg.omega_seed)
    gop.close()


def test_config2_shape_fp32_scaled(gpu_lib):
    cfg = CONFIGS["c2"].scaled(20000)
    _case(cfg.name, cfg.n)
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    _compare(gop, oop, cfg.k, cfg.p, cfg.q, 1, 1e-4, 1e-3, cfg.omega_seed)
    gop.close()


def test_config3_featprop_fp32_scaled(gpu_lib):
    cfg = CONFIGS["c3"].scaled(17000)
    _case(cfg.name, cfg.n)
    g = make_graph(cfg)
    x = block_features(g.blocks, cfg.d, seed=1000 + cfg.index)
    gop, oop = featprop_pair(gpu_lib, g, x, cfg.L, 1)
    _compare(gop, oop, cfg.k, cfg.p, cfg.q, 1, 1e-4, 1e-3, cfg.omega_seed)
    gop.close()


def test_featprop_exact_at_full_rank(gpu_lib):
    # L = 0, k = d: M = X and the SVD is exact (Section 2.3).
    _case("featprop exact")
    cfg = CONFIGS["c3"].scaled(3000)
    g = make_graph(cfg)
    d = 12
    x = block_features(g.blocks, d, seed=5)
    gop, oop = featprop_pair(gpu_lib, g, x, 0, 0)
    om = gaussian_block(d, d, seed=6)
    U, S, V, info = gop.truncated_svd(d, 0, q=0, omega=to_dev(om, torch.float64))
    s_exact = np.linalg.svd(rounded(x, torch.float64), compute_uv=False)
    assert np.allclose(to_np(S), s_exact, rtol=1e-12)
    recon = to_np(U) @ np.diag(to_np(S)) @ to_np(V).T
    assert np.abs(recon - x).max() < 1e-10 * np.abs(x).max()
    gop.close()


def test_device_start_block_is_used_when_omega_absent(gpu_lib):
    _case("device omega")
    cfg = CONFIGS["c1"]
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 0)
    from oracle import philox
    om = philox.gaussian_block(g.n, cfg.l, 77)
    _, S, _, _ = gop.truncated_svd(cfg.k, cfg.p, q=1, seed=77)
    _, so, _ = oracle_isvd(oop, cfg.k, om, 1)
    assert np.allclose(to_np(S), so, rtol=1e-10)
    gop.close()


def test_tolerance_mode_matches_fixed_mode_and_oracle_residual(gpu_lib):
    cfg = CONFIGS["c2"].scaled(5000)
    _case("tolerance", cfg.n)
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    k, p = 16, 16
    om = rounded(gaussian_block(g.n, k + p, seed=cfg.omega_seed), torch.float32)
    U, S, V, info = gop.truncated_svd(k, p, tol=1e-3, max_iter=300, omega=to_dev(om, torch.float32))
    assert info.status == 0 and info.residual <= 1e-3
    rho, _ = triplet_residuals(oop, to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64))
    assert rho.max() <= 1.5e-3, rho.max()
    assert abs(rho.max() - info.residual) <= 0.2 * info.residual + 1e-5
    _, so, _ = oracle_isvd(oop, k, om, info.iterations)
    assert np.abs(to_np(S) - so).max() / so.min() <= 1e-4
    gop.close()


def test_invalid_requests(gpu_lib):
    _case("invalid")
    cfg = CONFIGS["c1"]
    g = make_graph(cfg)
    gop, _ = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 0)
    with pytest.raises(gpu_lib.IsvdError) as e:
        gop.truncated_svd(1990, 20, q=1)
    assert e.value.status == gpu_lib.ISVD_E_INVALID
    with pytest.raises(gpu_lib.IsvdError):
        gop.truncated_svd(0, 4, q=1)
    gop.close()


@pytest.mark.parametrize("k,p,n", [(256, 32, 5003), (224, 32, 4000), (240, 32, 3001)])
def test_wide_blocks_fp32_against_oracle(gpu_lib, k, p, n):
    """Blocks of 288 and 256 columns take the LDS-resident wide triangular
    solve (with the FP64 column sums 1^T Q of the NE products); 272 columns
    take the general one.  Row counts leave a ragged last tile."""
    cfg = CONFIGS["c4"].scaled(n)
    _case("wide", cfg.name, n, k + p)
    g = make_graph(cfg)
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 1)
    _compare(gop, oop, k, p, 2, 1, 1e-4, 1e-3, cfg.omega_seed)
    gop.close()


@pytest.mark.parametrize("l", [288, 256])
def test_wide_orthonormalize_fp32_bf16(gpu_lib, l):
    """CholeskyQR2 through the wide solve against LAPACK's R (|diag|) and
    orthonormality, FP32 and BF16 storage, 20,007 rows (ragged)."""
    _case("wide orth", l)
    rows = 20007
    y = gaussian_block(rows, l, seed=9) @ np.diag(np.logspace(0, 3, l))
    _, rl = np.linalg.qr(y)
    for dt, tol in ((torch.float32, 1e-6), (torch.bfloat16, 2e-3)):
        yr = rounded(y, dt)
        q, r = gpu_lib.orthonormalize(to_dev(yr, dt))
        qn = to_np(q).astype(np.float64)
        assert np.abs(qn.T @ qn - np.eye(l)).max() < 10 * tol
        assert np.abs(qn @ to_np(r) - yr).max() <= 10 * tol * np.abs(yr).max()
        assert np.allclose(np.abs(np.diag(to_np(r))), np.abs(np.diag(rl)), rtol=1e3 * tol)
