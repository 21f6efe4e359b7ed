"""Philox4x32-10 and the Box-Muller Gaussian start block, in plain Python/NumPy.

Test infrastructure only (see the package docstring).

Philox4x32 is the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC 2011): ten
rounds of two 32x32 -> 64-bit multiplies, with the key bumped by the
Weyl constants between rounds.

The Gaussian block fixes how counters map to entries (a reading, since
the paper only says "sampled from standard normal"): entries are taken
in row-major order in pairs e = 2g, 2g+1; pair g uses counter
(g mod 2^32, g div 2^32, 0, 0) and key (seed mod 2^32, seed div 2^32);
its outputs x0..x3 give two 53-bit uniforms
u1 = ((x0 >> 5) 2^26 + (x1 >> 6) + 1/2) 2^-53 and u2 likewise from x2, x3;
then entry 2g = sqrt(-2 ln u1) cos(2 pi u2), entry 2g+1 = ... sin(2 pi u2).
"""

from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr = 4 uint32, key = 2 uint32 -> 4 uint32 (Python ints)."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox_stream(num_blocks: int, seed: int) -> np.ndarray:
    """num_blocks x 4 uint32 outputs for counters g = 0..num_blocks-1."""
    key = (seed & MASK, (seed >> 32) & MASK)
    out = np.empty((num_blocks, 4), dtype=np.uint32)
    for g in range(num_blocks):
        out[g] = philox4x32_10((g & MASK, (g >> 32) & MASK, 0, 0), key)
    return out


def gaussian_block(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols FP64 Gaussian block (see module docstring)."""
    total = rows * cols
    x = philox_stream((total + 1) // 2, seed).astype(np.uint64)
    u1 = ((x[:, 0] >> np.uint64(5)) * np.float64(2.0 ** 26) + (x[:, 1] >> np.uint64(6)) + 0.5) * 2.0 ** -53
    u2 = ((x[:, 2] >> np.uint64(5)) * np.float64(2.0 ** 26) + (x[:, 3] >> np.uint64(6)) + 0.5) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * x.shape[0])
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:total].reshape(rows, cols)
