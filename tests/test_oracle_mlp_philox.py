"""Pins for the warm-start oracle (features, MLP, loss, backward, Adam) and
for the Philox generator (CPU only)."""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import mlp, philox
from oracle.graph import adjacency
from synth import cycle_graph, edges_to_csr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        assert philox.philox4x32_10(r[0:4], r[4:6]) == tuple(r[6:10])


def test_philox_gaussian_block_layout_and_moments():
    z = philox.gaussian_block(300, 7, seed=123)
    assert z.shape == (300, 7)
    # pair g = 0 gives entries 0 and 1 (row-major) by Box-Muller
    x = philox.philox4x32_10((0, 0, 0, 0), (123, 0))
    u1 = ((x[0] >> 5) * 2.0 ** 26 + (x[1] >> 6) + 0.5) * 2.0 ** -53
    u2 = ((x[2] >> 5) * 2.0 ** 26 + (x[3] >> 6) + 0.5) * 2.0 ** -53
    r = math.sqrt(-2 * math.log(u1))
    assert abs(z[0, 0] - r * math.cos(2 * math.pi * u2)) < 1e-15
    assert abs(z[0, 1] - r * math.sin(2 * math.pi * u2)) < 1e-15
    assert abs(z.mean()) < 0.1 and abs(z.std() - 1) < 0.05
    assert not np.array_equal(z, philox.gaussian_block(300, 7, seed=124))


# ---------------------------------------------------------------- GELU

def test_gelu_textbook_values():
    xs = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    cdf = np.array([0.5 * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.allclose(mlp.gelu(xs), xs * cdf, atol=1e-16)
    assert np.allclose(mlp.gelu(xs) - mlp.gelu(-xs), xs, atol=1e-15)
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-16
    h = 1e-6
    fd = (mlp.gelu(xs + h) - mlp.gelu(xs - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(xs), fd, atol=1e-9)


# ---------------------------------------------------------------- loss

def _orth(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return q


def test_loss_is_mean_squared_sine_of_principal_angles():
    v = _orth(40, 4, 1)
    z = np.random.default_rng(2).standard_normal((40, 4))
    loss, _ = mlp.subspace_loss(z, v)
    ang = sla.subspace_angles(z, v)
    assert abs(loss - np.mean(np.sin(ang) ** 2)) < 1e-13
    assert 0.0 <= loss <= 1.0


def test_loss_zero_on_span_one_on_complement_and_invariant():
    v = _orth(30, 3, 3)
    r = np.random.default_rng(4).standard_normal((3, 3)) + 3 * np.eye(3)
    loss, grad = mlp.subspace_loss(v @ r, v)
    assert abs(loss) < 1e-14 and np.abs(grad).max() < 1e-13
    w = np.random.default_rng(5).standard_normal((30, 3))
    w -= v @ (v.T @ w)
    loss, _ = mlp.subspace_loss(w, v)
    assert abs(loss - 1.0) < 1e-13
    z = np.random.default_rng(6).standard_normal((30, 3))
    assert abs(mlp.subspace_loss(z, v)[0] - mlp.subspace_loss(z @ r, v)[0]) < 1e-13


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    v = _orth(25, 3, 8)
    z = rng.standard_normal((25, 3))
    _, grad = mlp.subspace_loss(z, v)
    h = 1e-6
    fd = np.zeros_like(z)
    for i in range(z.shape[0]):
        for j in range(z.shape[1]):
            zp, zm = z.copy(), z.copy()
            zp[i, j] += h
            zm[i, j] -= h
            fd[i, j] = (mlp.subspace_loss(zp, v)[0] - mlp.subspace_loss(zm, v)[0]) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-6 * np.abs(fd).max()


# ---------------------------------------------------------------- network

def test_backward_matches_central_differences():
    rng = np.random.default_rng(9)
    k, n = 3, 20
    params = mlp.init_params(k, seed=10)
    for p in params[1::2]:
        p += 0.1 * rng.standard_normal(p.shape)
    f = rng.standard_normal((n, 16))
    v = _orth(n, k, 11)

    def total(ps):
        z, _ = mlp.forward(ps, f)
        return mlp.subspace_loss(z, v)[0]

    z, cache = mlp.forward(params, f)
    _, dz = mlp.subspace_loss(z, v)
    grads = mlp.backward(params, cache, dz)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            fp = total(params)
            flat[i] = old - h
            fm = total(params)
            flat[i] = old
            fd = (fp - fm) / (2 * h)
            assert abs(g.reshape(-1)[i] - fd) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (pi, i)


def test_adam_first_step_is_signed_learning_rate():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    mlp.adam_step(p, g, m, v, t=1, lr=0.01, eps=1e-12)
    assert np.allclose(p[0], [0.99, -1.99, 2.99], atol=1e-9)


# ---------------------------------------------------------------- features

def test_features_on_star_graph_by_hand():
    # star K_{1,m}: centre 0 with degree m, leaves with degree 1.
    m = 5
    g = edges_to_csr(m + 1, np.zeros(m, np.int64), np.arange(1, m + 1))
    a = adjacency(g.n, g.indptr, g.indices)
    f = mlp.structural_features(a, raw=True)
    # T d: centre -> mean leaf degree 1, leaf -> centre degree m; alternates.
    assert np.allclose(f[0, 0], math.log1p(m)) and np.allclose(f[1:, 0], math.log(2))
    assert np.allclose(f[0, 1], math.log1p(1)) and np.allclose(f[1:, 1], math.log1p(m))
    assert np.allclose(f[0, 2], math.log1p(m)) and np.allclose(f[1:, 2], math.log1p(1))
    # (T^T) 1: centre -> sum over leaves of 1/1 = m; leaf -> 1/m.  Then m -> ...
    assert np.allclose(f[0, 9], math.log1p(m)) and np.allclose(f[1:, 9], math.log1p(1.0 / m))
    # (T^T)^2 1: centre -> sum of leaves' (1/m)/1 = 1; leaf -> m/m = 1.
    assert np.allclose(f[:, 10], math.log(2))


def test_features_constant_on_regular_graph():
    g = cycle_graph(12)
    f = mlp.structural_features(adjacency(g.n, g.indptr, g.indices))
    assert f.shape == (12, 16)
    assert np.all(f == 0.0)
    raw = mlp.structural_features(adjacency(g.n, g.indptr, g.indices), raw=True)
    assert np.allclose(raw[:, :9], math.log(3)) and np.allclose(raw[:, 9:], math.log(2))


def test_features_isolated_node_is_finite():
    g = edges_to_csr(4, np.array([0, 1]), np.array([1, 2]))   # node 3 isolated
    f = mlp.structural_features(adjacency(g.n, g.indptr, g.indices))
    assert np.all(np.isfinite(f))
