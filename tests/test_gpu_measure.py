"""Measurement entry points on the GPU: the peak-rate probes (a copy that
really copies, positive times, the MFMA flop count) and the per-storage
record of sparse passes (a BF16 operator's passes recorded as BF16), and
the phase record of a truncated SVD."""

import time

import numpy as np
import pytest
import torch

from gpu_helpers import print_case
from synth import chung_lu_graph

pytestmark = pytest.mark.gpu


def test_peak_copy_copies_and_times(gpu_lib):
    print_case("peak copy")
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    ms = gpu_lib.peak_copy(src, dst, 2)
    assert ms > 0.0
    assert torch.equal(src, dst)


def test_peak_read_and_mfma_report_positive_rates(gpu_lib):
    print_case("peak read / mfma")
    buf = torch.ones(1 << 22, dtype=torch.float32, device="cuda")
    assert gpu_lib.peak_read(buf, 3) > 0.0
    for prec in (gpu_lib.FP64, gpu_lib.FP32):
        fl, ms = gpu_lib.peak_mfma(prec, 10)
        assert ms > 0.0
        # 16 blocks of 4 waves per CU; per wave and trip 32 rounds of 8 MFMAs of 2048 flops
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert fl == cus * 16 * 4 * 10 * 32 * 8 * 2048


def test_profile_records_passes_by_storage(gpu_lib):
    print_case("profile by storage")
    g = chung_lu_graph(3000, 2.5, 8.0, seed=3)
    K = 3
    op = gpu_lib.Operator(g, form="ne", coeffs=np.full(K, 1.0 / K), lam=0.1, precision=gpu_lib.BF16)
    y = gpu_lib.gaussian_block(g.n, 24, seed=1, dtype=torch.bfloat16)
    torch.cuda.synchronize()
    gpu_lib.profile_spmm(True)
    op.matmul(op.matmul(y), transpose=True)
    ms16, gb16, cb16, n16 = gpu_lib.profile_spmm_read_storage(gpu_lib.BF16)
    ms32, _, _, n32 = gpu_lib.profile_spmm_read_storage(gpu_lib.FP32)
    ms, gb, cb, n = gpu_lib.profile_spmm_read()
    gpu_lib.profile_spmm(False)
    op.close()
    assert n16 == 2 * K and n32 == 0 and ms32 == 0.0
    assert n == n16 and gb == gb16 and cb == cb16 and ms == ms16
    assert gb16 > cb16 > 0.0


def test_phase_profile_covers_the_steps_of_a_truncated_svd(gpu_lib):
    print_case("phase profile")
    g = chung_lu_graph(4000, 2.5, 8.0, seed=5)
    op = gpu_lib.Operator(g, form="ne", coeffs=np.full(3, 1.0 / 3), lam=0.05, precision=gpu_lib.FP32)
    gpu_lib.profile_spmm(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, info = op.truncated_svd(8, 8, tol=1e-4, max_iter=300, seed=2)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0)
    ph = gpu_lib.profile_phases_read()
    gpu_lib.profile_spmm(False)
    assert set(ph) == set(gpu_lib.PHASES)
    # one product with M and one with M^T per iteration, plus the product that
    # feeds the last residual check
    assert ph["products"][1] == info.applies
    assert ph["orthonormalisation"][1] >= 2 * info.iterations
    assert ph["rayleigh_ritz"][1] == info.ritz_steps
    assert ph["residual_checks"][1] >= 1
    assert ph["output_products"][1] == 1
    total = sum(ms for ms, _ in ph.values())
    assert 0.0 < total <= wall_ms
    # read clears the record
    assert all(n == 0 for _, n in gpu_lib.profile_phases_read().values())
    op.close()
