"""isvd_gram_noalloc (the Gram product for callers that cannot allocate):
through the C ABI, against isvd_gram on the same inputs, two calls in a row,
the second with a smaller input, so the shared scratch array is reused."""

import numpy as np
import pytest
import torch

from gpu_helpers import print_case, to_dev

pytestmark = pytest.mark.gpu


def _rel(c, ref):
    return float((c - ref).abs().max() / ref.abs().max())


def test_gram_noalloc_matches_gram_on_two_calls(gpu_lib):
    rng = np.random.default_rng(21)
    # call 1: A^T A, 400,000 x 288 FP32 (the scratch holds fewer row slices
    # than isvd_gram's workspace, so the sums group differently)
    print_case("gram noalloc", "400000x288 fp32 A^T A")
    a = to_dev(rng.standard_normal((400_000, 288)), torch.float32)
    c1 = torch.full((288, 288), np.nan, dtype=torch.float64, device="cuda")
    gpu_lib.gram_noalloc(a, a, c1)
    ref1 = gpu_lib.gram(a)
    torch.cuda.synchronize()
    assert torch.isfinite(c1).all()
    assert _rel(c1, ref1) < 1e-12
    assert torch.equal(c1, c1.T)
    exact = a.double().T @ a.double()
    assert _rel(c1, exact) < 1e-12
    del a, exact
    # call 2: smaller, A^T B in FP64 (scratch keeps call 1's contents)
    print_case("gram noalloc", "5000x40 by 5000x24 fp64 A^T B")
    x = to_dev(rng.standard_normal((5000, 40)), torch.float64)
    y = to_dev(rng.standard_normal((5000, 24)), torch.float64)
    c2 = torch.full((40, 24), np.nan, dtype=torch.float64, device="cuda")
    gpu_lib.gram_noalloc(x, y, c2)
    ref2 = gpu_lib.gram(x, y)
    torch.cuda.synchronize()
    assert torch.isfinite(c2).all()
    assert _rel(c2, ref2) < 1e-12
    assert _rel(c2, x.T @ y) < 1e-12


def test_gram_noalloc_rejects_bad_sizes(gpu_lib):
    print_case("gram noalloc", "argument checks")
    a = torch.zeros((64, 1100), dtype=torch.float32, device="cuda")
    c = torch.zeros((1100, 1100), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.IsvdError) as e:
        gpu_lib.gram_noalloc(a, a, c)      # m + p above 2048
    assert e.value.status == gpu_lib.ISVD_E_INVALID
