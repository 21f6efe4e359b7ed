"""BF16-storage path: blocks stored as bfloat16 with FP32 accumulation.

- fixed q: singular values against the FP64 GPU run on the same start block,
  next to the FP32 run's errors (BF16 rounds every stored block to 2^-9);
- tolerance mode: BF16 while rho > 1e-2, then FP32 to rho <= tol; the returned
  triplets must meet tol by the oracle's own residual.
"""

import numpy as np
import pytest
import torch

from gpu_helpers import ne_pair, rounded, to_dev, to_np
from oracle.isvd import triplet_residuals
from synth import CONFIGS, gaussian_block
from synth.configs import make_graph

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def c4_small():
    cfg = CONFIGS["c4"].scaled(30000)
    return cfg, make_graph(cfg)


def test_bf16_fixed_q_tracks_fp64(gpu_lib, c4_small):
    cfg, g = c4_small
    _case("bf16 fixed", g.n)
    k, p, q = 64, 16, 2
    om = gaussian_block(g.n, k + p, seed=cfg.omega_seed)
    res = {}
    for prec in (0, 1, 2):
        dt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}[prec]
        gop, _ = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, prec)
        _, S, _, info = gop.truncated_svd(k, p, q=q, omega=to_dev(rounded(om, dt), dt))
        res[prec] = to_np(S)
        gop.close()
    e32 = np.max(np.abs(res[1] - res[0]) / res[0])
    e16 = np.max(np.abs(res[2] - res[0]) / res[0])
    print(f"relative sigma error vs FP64: fp32 {e32:.2e}, bf16 {e16:.2e}", flush=True)
    assert e32 <= 1e-4
    assert e16 <= 5e-2


def test_bf16_then_fp32_reaches_tolerance(gpu_lib, c4_small):
    cfg, g = c4_small
    _case("bf16 tolerance", g.n)
    k, p = 32, 16
    gop, oop = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 2)
    U, S, V, info = gop.truncated_svd(k, p, tol=1e-3, max_iter=400, seed=5, fp32_switch_tol=1e-2)
    print(info, flush=True)
    assert info.status == 0 and info.residual <= 1e-3
    assert 0 < info.bf16_iterations <= info.iterations + 1
    assert U.dtype == torch.float32 and V.dtype == torch.float32
    rho, _ = triplet_residuals(oop, to_np(U).astype(np.float64), to_np(S), to_np(V).astype(np.float64))
    assert rho.max() <= 1.5e-3, rho.max()
    gop.close()
