"""Dense seeded inputs: node features and Gaussian start blocks."""

from __future__ import annotations

import numpy as np


def gaussian_block(rows: int, cols: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Row-major rows x cols block of i.i.d. N(0, 1) draws (NumPy PCG64).

    Drawn in FP64 and then rounded to `dtype` (round to nearest even)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols)).astype(dtype)


def block_features(labels: np.ndarray, d: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Node features X = N(0, 1)^(n x d) + mu_{b(i)}, with one mean vector
    mu_b ~ N(0, I_d) per block b."""
    rng = np.random.default_rng(seed)
    nb = int(labels.max()) + 1 if labels.size else 0
    mu = rng.standard_normal((nb, d))
    x = rng.standard_normal((labels.shape[0], d)) + mu[labels]
    return x.astype(dtype)
