"""Shared helpers of the GPU parity tests: build matching GPU / oracle operators
from one seeded graph, and compare blocks."""

from __future__ import annotations

import numpy as np
import torch

from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def to_np(t):
    return t.detach().float().cpu().numpy() if t.dtype == torch.bfloat16 else t.detach().cpu().numpy()


def rounded(a, dtype):
    """Host copy of `a` rounded to the device dtype, returned as float64."""
    return torch.as_tensor(a).to(dtype).to(torch.float64).numpy()


def ne_pair(lib, g, coeffs, lam, loops, precision):
    gop = lib.Operator(g, form="ne", coeffs=coeffs, lam=lam, self_loops=loops, precision=precision)
    oop = NEDesignMatrix.from_graph(g, coeffs, lam, add_self_loops=loops)
    return gop, oop


def featprop_pair(lib, g, x, L, precision):
    dt = lib._DTYPE[precision]
    xd = to_dev(x, dt)
    gop = lib.Operator(g, form="featprop", X=xd, L=L, precision=precision)
    oop = FeatPropDesignMatrix.from_graph(g, rounded(x, dt), L)
    return gop, oop


def col_rel_err(got, want):
    """Max over columns of max|got - want| / max|want| (per column)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.maximum(np.abs(want).max(axis=0), 1e-300)
    return float((np.abs(got - want).max(axis=0) / scale).max())


def gapped_k(s_all, k, rel_gap=1e-3):
    """Largest k' <= k whose Ritz gap (s_k' - s_k'+1)/s_k' is at least rel_gap."""
    for kk in range(k, 0, -1):
        if (s_all[kk - 1] - s_all[kk]) / s_all[kk - 1] >= rel_gap:
            return kk
    return 0


def ne_pair_general(lib, dg, coeffs, lam, loops, precision, weighted=True):
    """GPU and oracle NE operators of a directed (optionally weighted)
    synth.DirectedGraph: the GPU side gets the CSR of A and of A^T, the
    oracle builds its own transpose from A."""
    vals = dg.values if weighted else None
    tvals = dg.t_values if weighted else None
    gop = lib.Operator(dg, form="ne", coeffs=coeffs, lam=lam, self_loops=loops, precision=precision,
                       values=vals, symmetric=False, t_indptr=dg.t_indptr, t_indices=dg.t_indices,
                       t_values=tvals)
    oop = NEDesignMatrix.from_graph(dg, coeffs, lam, add_self_loops=loops,
                                    values=None if vals is None else vals.astype(np.float64))
    return gop, oop


def sampled_triplets(k):
    """Ten triplet indices spread over 0..k-1, the first two and the last
    two included."""
    return np.unique(np.concatenate([[0, 1], np.linspace(2, k - 3, 6).round().astype(int), [k - 2, k - 1]]))


# The device evaluates rho from the blocks it stores (FP32 products of the
# FP32 triplets; the FP64 oracle evaluates the same triplets exactly).  The
# two differ by the FP32 rounding of those products, about 1e-6 relative
# here, so a returned rho at the tolerance can read up to 1% above it.
RHO_SLACK = 1.01


def print_case(*a):
    """Name the case on stdout before its GPU work (flushed)."""
    print("CASE", *a, flush=True)
