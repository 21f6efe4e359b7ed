"""Run-to-run determinism of a whole SVD: the same operator, seed and
parameters give bitwise-identical U, S, V and the same iteration count.

Every reduction on the device path has a fixed order (row-slice partial
sums of the Grams and column sums combined in index order, one workgroup
per hub row, no floating-point atomics), so nothing depends on the
scheduling of the waves."""

import numpy as np
import pytest
import torch

from gpu_helpers import ne_pair
from synth import CONFIGS
from synth.configs import make_graph

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


def _twice(op, **kw):
    outs = []
    for _ in range(2):
        U, S, V, info = op.truncated_svd(**kw)
        torch.cuda.synchronize()
        outs.append((U.clone(), S.clone(), V.clone(), info))
    return outs


@pytest.mark.parametrize("precision,name", [(1, "fp32"), (2, "bf16")])
def test_whole_svd_bitwise_repeatable_c2_scaled(gpu_lib, precision, name):
    cfg = CONFIGS["c2"].scaled(20000)
    _case("determinism", name, cfg.n)
    g = make_graph(cfg)
    gop, _ = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, precision)
    kw = dict(k=cfg.k, p=cfg.p, tol=1e-4, max_iter=2000, seed=3)
    if precision == 2:
        kw["fp32_switch_tol"] = 1e-2
    (u1, s1, v1, i1), (u2, s2, v2, i2) = _twice(gop, **kw)
    assert i1.status == 0 and i2.status == 0
    assert i1.iterations == i2.iterations and i1.applies == i2.applies
    assert i1.residual == i2.residual
    assert torch.equal(s1, s2)
    assert torch.equal(u1, u2)
    assert torch.equal(v1, v2)
    gop.close()


def test_fixed_q_fp64_bitwise_repeatable_c1(gpu_lib):
    cfg = CONFIGS["c1"]
    _case("determinism fp64", cfg.name)
    g = make_graph(cfg)
    gop, _ = ne_pair(gpu_lib, g, cfg.coeffs, cfg.lam, cfg.self_loops, 0)
    (u1, s1, v1, _), (u2, s2, v2, _) = _twice(gop, k=cfg.k, p=cfg.p, q=cfg.q, seed=cfg.omega_seed)
    assert torch.equal(s1, s2) and torch.equal(u1, u2) and torch.equal(v1, v2)
    gop.close()
