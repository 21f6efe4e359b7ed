"""Warm-start network: structural features, MLP, subspace loss, backward, Adam.

Test infrastructure only (see the package docstring).

The paper draws the start block of Algorithm 1 from N(0, 1).  The
learned warm start replaces its first k columns by the output of a small
MLP evaluated per node.  None of this is in the paper; the definitions
here are the readings the GPU path implements:

features (16 per node, for M's column side):
    log1p(d), log1p(T^j d) for j = 1..8, log1p((T^T)^j 1) for j = 1..7,
    each column z-scored over the nodes with its mean and (population)
    standard deviation; a column whose deviation is at most
    1e-9 (1 + |mean|) has no spread and is set to 0.  T^j 1 is not
    used: T is row-stochastic, so it is all ones.
network:  Z = GELU(GELU(F W1 + b1) W2 + b2) W3 + b3,  16 -> 128 -> 128 -> k,
          GELU(x) = x Phi(x) with the exact normal CDF.
loss:     L(Z) = tr((Z^T Z)^-1 Z^T (I - V V^T) Z) / k for orthonormal V
          (n x k): the mean squared sine of the principal angles between
          span(Z) and span(V); invariant to Z -> Z R for invertible R.
gradient: dL/dZ = (2/k) (I - Z G^-1 Z^T)(I - V V^T) Z G^-1, G = Z^T Z.
"""

from __future__ import annotations

import math

import numpy as np

from .graph import degrees, transition

LAYER_SIZES = (16, 128, 128)


def structural_features(a, raw: bool = False) -> np.ndarray:
    """n x 16 feature matrix of the nodes of A (see module docstring)."""
    t = transition(a)
    tt = t.T.tocsr()
    d = degrees(a)
    cols = [d]
    p = d.copy()
    for _ in range(8):
        p = t @ p
        cols.append(p)
    p = np.ones_like(d)
    for _ in range(7):
        p = tt @ p
        cols.append(p)
    f = np.log1p(np.stack(cols, axis=1))
    if raw:
        return f
    mu = f.mean(axis=0)
    sd = f.std(axis=0)
    out = np.zeros_like(f)
    ok = sd > 1e-9 * (1.0 + np.abs(mu))
    out[:, ok] = (f[:, ok] - mu[ok]) / sd[ok]
    return out


def _phi(x):
    return np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _cdf(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0)))


def gelu(x):
    return x * _cdf(x)


def gelu_grad(x):
    return _cdf(x) + x * _phi(x)


def init_params(k: int, seed: int):
    """Weights ~ N(0, 1/fan_in) (float64), biases 0."""
    rng = np.random.default_rng(seed)
    sizes = LAYER_SIZES + (k,)
    params = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        params.append(rng.standard_normal((fan_in, fan_out)) / math.sqrt(fan_in))
        params.append(np.zeros(fan_out))
    return params


def forward(params, f):
    """Returns (Z, cache) with cache holding the pre-activations."""
    w1, b1, w2, b2, w3, b3 = params
    h1p = f @ w1 + b1
    h1 = gelu(h1p)
    h2p = h1 @ w2 + b2
    h2 = gelu(h2p)
    z = h2 @ w3 + b3
    return z, (f, h1p, h1, h2p, h2)


def subspace_loss(z, v):
    """(loss, dL/dZ) for the subspace loss against orthonormal v."""
    k = z.shape[1]
    g = z.T @ z
    ginv = np.linalg.inv(g)
    pz = z - v @ (v.T @ z)                        # (I - V V^T) Z
    loss = np.trace(ginv @ (z.T @ pz)) / k
    x = pz @ ginv                                 # (I - V V^T) Z G^-1
    grad = (2.0 / k) * (x - z @ (ginv @ (z.T @ x)))
    return loss, grad


def backward(params, cache, dz):
    """Gradients of the parameters given dL/dZ, in the order of params."""
    w1, b1, w2, b2, w3, b3 = params
    f, h1p, h1, h2p, h2 = cache
    dw3 = h2.T @ dz
    db3 = dz.sum(axis=0)
    dh2 = (dz @ w3.T) * gelu_grad(h2p)
    dw2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ w2.T) * gelu_grad(h1p)
    dw1 = f.T @ dh1
    db1 = dh1.sum(axis=0)
    return [dw1, db1, dw2, db2, dw3, db3]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) in place; t counts from 1."""
    for p, g, mi, vi in zip(params, grads, m, v):
        mi *= beta1
        mi += (1 - beta1) * g
        vi *= beta2
        vi += (1 - beta2) * g * g
        mhat = mi / (1 - beta1 ** t)
        vhat = vi / (1 - beta2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
