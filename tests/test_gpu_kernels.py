"""GPU parity of the building blocks against the FP64 oracle / LAPACK:
device Philox, the FP64 Gram, CholeskyQR2, the Jacobi SVD, and one
product with each design matrix (NE and feature form, both directions)
through isvd_matmul_block, over widths, ragged tails, hubs, empty rows."""

import numpy as np
import pytest
import torch

from gpu_helpers import col_rel_err, featprop_pair, ne_pair, rounded, to_dev, to_np
from oracle import philox
from synth import chung_lu_graph, edges_to_csr, gaussian_block, sbm_graph, block_features

pytestmark = pytest.mark.gpu

DT = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}


def _print_case(*a):
    print("CASE", *a, flush=True)


# ---------------------------------------------------------------- Philox

def test_device_gaussian_matches_oracle_philox(gpu_lib):
    _print_case("gaussian")
    for rows, cols, seed in [(37, 11, 5), (1000, 144, 2 ** 40 + 7)]:
        z = to_np(gpu_lib.gaussian_block(rows, cols, seed, torch.float64))
        want = philox.gaussian_block(rows, cols, seed)
        assert np.abs(z - want).max() < 1e-12
        z32 = to_np(gpu_lib.gaussian_block(rows, cols, seed, torch.float32))
        assert np.abs(z32 - want).max() <= 1e-6 * max(1.0, np.abs(want).max())
    a = to_np(gpu_lib.gaussian_block(500, 33, 9, torch.float32))
    b = to_np(gpu_lib.gaussian_block(500, 33, 9, torch.float32))
    assert np.array_equal(a, b)


def test_device_bf16_rounding_is_round_to_nearest_even(gpu_lib):
    # BF16 blocks round on the device with the conversion instruction: the
    # device's own FP64 draws, rounded to FP32 and then to BF16 by torch on the
    # CPU (round to nearest, ties to even), must give the same bits.  (The
    # oracle's draws agree with the device's to 1e-12 only, which can move a
    # value across an FP32 rounding boundary.)
    _print_case("bf16 rounding")
    rows, cols, seed = 4099, 37, 11
    z = gpu_lib.gaussian_block(rows, cols, seed, torch.bfloat16).cpu()
    f32 = gpu_lib.gaussian_block(rows, cols, seed, torch.float64).cpu().float()
    # the block holds exact ties (low 16 bits 0x8000), which must go to the even neighbour
    assert int(((f32.view(torch.int32) & 0xffff) == 0x8000).sum()) >= 3
    want = f32.to(torch.bfloat16)
    assert torch.equal(z.view(torch.int16), want.view(torch.int16))
    # the reference's own tie rule
    x = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)], dtype=torch.float32)
    assert torch.equal(x.to(torch.bfloat16).float(), torch.tensor([1.0, 1.0 + 4 * 2.0 ** -8, -1.0]))


# ---------------------------------------------------------------- Gram

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("rows,m", [(1, 3), (1000, 42), (64, 80), (777, 17), (70001, 144), (5000, 288),
                                    (3001, 600),
                                    # job placements of A^T A: one group of 10 and 15 jobs, two of 21,
                                    # three of 36 and 45, four of 55 (a whole number of waves per SIMD)
                                    (20000, 192), (9000, 240), (20000, 256), (5000, 384), (3000, 432),
                                    (3000, 480)])
def test_gram_exact_products_fp64_sums(gpu_lib, dtype, rows, m):
    _print_case("gram", dtype, rows, m)
    y = gaussian_block(rows, m, seed=rows + m)
    y[:, 0] *= 1e3
    y = rounded(y, dtype)
    yd = to_dev(y, dtype)
    g = to_np(gpu_lib.gram(yd))
    want = y.T @ y
    assert np.abs(g - want).max() <= 1e-13 * np.abs(want).max()
    assert np.array_equal(g, g.T)


@pytest.mark.parametrize("rows,ma,pb", [(3001, 20, 70), (50000, 16, 128), (2000, 130, 5), (4099, 300, 300)])
def test_gram_rectangular(gpu_lib, rows, ma, pb):
    _print_case("gram rect", rows, ma, pb)
    a = rounded(gaussian_block(rows, ma, seed=1), torch.float32)
    b = rounded(gaussian_block(rows, pb, seed=2), torch.float32)
    c = to_np(gpu_lib.gram(to_dev(a, torch.float32), to_dev(b, torch.float32)))
    assert np.abs(c - a.T @ b).max() <= 1e-13 * np.abs(a.T @ b).max()


def test_gram_strided_columns(gpu_lib):
    # a column window of a wider block: leading dimension larger than the width
    _print_case("gram strided")
    wide = rounded(gaussian_block(5003, 160, seed=4), torch.float32)
    wd = to_dev(wide, torch.float32)
    g = to_np(gpu_lib.gram(wd[:, 7:151]))
    want = wide[:, 7:151].T @ wide[:, 7:151]
    assert np.abs(g - want).max() <= 1e-13 * np.abs(want).max()


# ---------------------------------------------------------------- CholeskyQR2

@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
@pytest.mark.parametrize("rows,l", [(2000, 42), (50000, 144), (20000, 288), (100, 17)])
def test_cholesky_qr2(gpu_lib, dtype, tol, rows, l):
    _print_case("cholqr2", dtype, rows, l)
    y = gaussian_block(rows, l, seed=3) @ np.diag(np.logspace(0, 4, l))
    y = rounded(y, dtype)
    yd = to_dev(y, dtype)
    q, r = gpu_lib.orthonormalize(yd)
    q = to_np(q).astype(np.float64)
    r = to_np(r)
    assert np.abs(q.T @ q - np.eye(l)).max() < tol * 10
    assert np.allclose(np.tril(r, -1), 0)
    assert np.abs(q @ r - y).max() <= tol * 10 * np.abs(y).max()
    _, rl = np.linalg.qr(y)
    assert np.allclose(np.abs(np.diag(r)), np.abs(np.diag(rl)), rtol=tol * 1e3)


def test_cholesky_qr_rank_deficient_reports_or_repairs(gpu_lib):
    _print_case("cholqr rank deficient")
    y = gaussian_block(3000, 16, seed=4)
    y[:, 5] = y[:, 3]
    yd = to_dev(y, torch.float64)
    try:
        q, _ = gpu_lib.orthonormalize(yd)
    except gpu_lib.IsvdError as e:
        assert e.status == gpu_lib.ISVD_E_NOT_SPD
        return
    q = to_np(q)
    assert np.all(np.isfinite(q))


# ---------------------------------------------------------------- Jacobi SVD

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("n", [1, 2, 7, 42, 64, 65, 144, 288, 300, 400, 512])
def test_small_svd_matches_lapack(gpu_lib, n):
    _print_case("jacobi", n)
    rng = np.random.default_rng(n)
    a = np.triu(rng.standard_normal((n, n))) @ np.diag(np.logspace(0, -6, n))
    u, s, v = (to_np(t) for t in gpu_lib.small_svd(to_dev(a, torch.float64)))
    sw = np.linalg.svd(a, compute_uv=False)
    assert np.allclose(s, sw, rtol=1e-11, atol=1e-14 * sw[0])
    assert np.all(np.diff(s) <= 0)
    # one-sided Jacobi: every rotation adds O(eps) relative error to the two
    # columns it touches; a column takes O(n) rotations per sweep, and the
    # block schedule converges within about ten sweeps
    assert np.abs(u @ np.diag(s) @ v.T - a).max() <= 20 * n * EPS * sw[0]
    assert np.abs(v.T @ v - np.eye(n)).max() < 1e-15 * 8 * max(n, 16)


@pytest.mark.parametrize("n", [40, 200])
def test_small_svd_repeated_values(gpu_lib, n):
    # clusters of equal singular values: any orthonormal basis of each
    # cluster's space is correct, so compare values and the reconstruction
    _print_case("jacobi repeated", n)
    rng = np.random.default_rng(100 + n)
    qa, _ = np.linalg.qr(rng.standard_normal((n, n)))
    qb, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sv = np.repeat([3.0, 1.0, 1e-3, 0.0], n // 4)
    a = (qa * sv) @ qb.T
    u, s, v = (to_np(t) for t in gpu_lib.small_svd(to_dev(a, torch.float64)))
    assert np.allclose(s, sv, atol=1e-12 * 3.0)
    assert np.abs(u @ np.diag(s) @ v.T - a).max() <= 20 * n * EPS * 3.0
    assert np.abs(v.T @ v - np.eye(n)).max() < 1e-15 * 8 * max(n, 16)


# ---------------------------------------------------------------- design-matrix products

def _apply_case(gpu_lib, g, coeffs, lam, loops, precision, ncols, tol, seed=7, ld_pad=0):
    dt = DT[precision]
    gop, oop = ne_pair(gpu_lib, g, coeffs, lam, loops, precision)
    y = rounded(gaussian_block(g.n, ncols, seed=seed), dt)
    if ld_pad:
        wide = torch.zeros((g.n, ncols + ld_pad), dtype=dt, device="cuda")
        wide[:, 1:ncols + 1] = to_dev(y, dt)
        yd = wide[:, 1:ncols + 1]         # unaligned start: the element-wise path
    else:
        yd = to_dev(y, dt)
    for tr in (False, True):
        out = to_np(gop.matmul(yd, transpose=tr))
        want = (oop.T if tr else oop).dot(y)
        err = col_rel_err(out, want)
        assert err <= tol, (tr, err)
    gop.close()


@pytest.mark.parametrize("ncols", [1, 2, 42, 80, 144, 288])
def test_ne_product_fp32_widths(gpu_lib, ncols):
    _print_case("ne fp32 width", ncols)
    g = chung_lu_graph(6000, 2.5, 12.0, seed=21)
    _apply_case(gpu_lib, g, np.full(4, 0.25), 0.1, False, 1, ncols, 5e-6)


def test_ne_product_fp64_c1_shape(gpu_lib):
    _print_case("ne fp64 c1")
    g = sbm_graph(2000, 7, 0.01, 0.0005, seed=1)
    _apply_case(gpu_lib, g, np.full(5, 0.2), 0.05, True, 0, 42, 1e-13)


def test_ne_product_hubs_and_isolated(gpu_lib):
    _print_case("ne hubs")
    g = chung_lu_graph(40000, 2.1, 20.0, seed=22)
    lens = g.row_lengths()
    assert lens.max() > 512 and (lens == 0).any()   # rows above the 256 hub threshold
    _apply_case(gpu_lib, g, np.full(3, 1 / 3), 0.05, False, 1, 144, 5e-6)
    _apply_case(gpu_lib, g, np.full(3, 1 / 3), 0.05, True, 0, 20, 1e-13)


@pytest.mark.parametrize("K", [1, 2, 10])
def test_ne_product_number_of_powers(gpu_lib, K):
    _print_case("ne K", K)
    g = sbm_graph(3000, 5, 0.01, 0.001, seed=23)
    rng = np.random.default_rng(K)
    _apply_case(gpu_lib, g, rng.uniform(-1, 1, K), 0.3, K == 2, 0, 24, 1e-13)


def test_ne_product_unaligned_blocks(gpu_lib):
    _print_case("ne unaligned")
    g = chung_lu_graph(5000, 2.5, 10.0, seed=24)
    _apply_case(gpu_lib, g, np.full(2, 0.5), 0.1, False, 1, 37, 5e-6, ld_pad=5)


def test_ne_product_bf16(gpu_lib):
    _print_case("ne bf16")
    g = chung_lu_graph(8000, 2.3, 15.0, seed=25)
    _apply_case(gpu_lib, g, np.full(5, 0.2), 0.05, False, 2, 288, 3e-2)


def test_ne_product_empty_graph(gpu_lib):
    _print_case("ne empty")
    g = edges_to_csr(10, np.empty(0, np.int64), np.empty(0, np.int64))
    _apply_case(gpu_lib, g, np.array([0.5, 0.5]), 0.2, False, 0, 3, 1e-14)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-5)])
@pytest.mark.parametrize("L", [0, 1, 3])
def test_featprop_product(gpu_lib, precision, tol, L):
    _print_case("featprop", precision, L)
    g = sbm_graph(6000, 8, 0.004, 0.0003, seed=26)
    x = block_features(g.blocks, 24, seed=27)
    dt = DT[precision]
    gop, oop = featprop_pair(gpu_lib, g, x, L, precision)
    l = 19
    gmat = rounded(gaussian_block(24 * (L + 1), l, seed=28), dt)
    out = to_np(gop.matmul(to_dev(gmat, dt)))
    assert col_rel_err(out, oop.dot(gmat)) <= tol
    q = rounded(gaussian_block(6000, l, seed=29), dt)
    out = to_np(gop.matmul(to_dev(q, dt), transpose=True))
    assert col_rel_err(out, oop.T.dot(q)) <= tol
    gop.close()


@pytest.mark.parametrize("d,l,L", [(16, 7, 0), (48, 19, 1), (128, 80, 3), (256, 37, 0), (128, 176, 1)])
def test_featprop_forward_gemm_shapes(gpu_lib, d, l, L):
    # X [G_0 .. G_L] by the tall GEMM: K = d multiples of 16 (register-A path),
    # ragged row count, column counts off the 16-column tiles
    _print_case("featprop gemm", d, l, L)
    g = sbm_graph(3001, 5, 0.004, 0.0004, seed=61)
    x = block_features(g.blocks, d, seed=62)
    gop, oop = featprop_pair(gpu_lib, g, x, L, 1)
    gmat = rounded(gaussian_block(d * (L + 1), l, seed=63), torch.float32)
    out = to_np(gop.matmul(to_dev(gmat, torch.float32)))
    assert col_rel_err(out, oop.dot(gmat)) <= 2e-5
    gop.close()
