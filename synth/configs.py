"""The five benchmark workloads, described by their sizes and seeds.

A workload names a graph recipe, the design matrix's form and its
constants, the rank k, the oversampling p and the number of power
iterations q.  Graph seed = workload index; start-block seed = 100 +
workload index.  `scale` shrinks a graph for quick tests while keeping
its shape (same degree law, same number of blocks).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .graphs import Graph, chung_lu_graph, sbm_graph, sbm_graph_by_degree
from .inputs import block_features, gaussian_block


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    index: int
    graph: str                 # "sbm" | "sbm_deg" | "chung_lu"
    n: int
    graph_args: dict = field(default_factory=dict)
    form: str = "ne"           # "ne": sum_k c_k T^k - lam (11^T - A);  "featprop": [X, AX, .., A^L X]
    K: int = 5                 # number of powers (ne)
    lam: float = 0.05          # lambda (ne)
    self_loops: bool = False   # add I to A before forming T (ne)
    d: int = 0                 # feature width (featprop)
    L: int = 0                 # propagation depth (featprop)
    k: int = 32
    p: int = 10
    q: int = 2
    precision: str = "fp32"    # "fp64" | "fp32" | "bf16"

    @property
    def l(self) -> int:
        return self.k + self.p

    @property
    def coeffs(self) -> np.ndarray:
        # uniform weights c_k = 1/K, k = 1..K
        return np.full(self.K, 1.0 / self.K)

    @property
    def omega_seed(self) -> int:
        return 100 + self.index

    def scaled(self, n: int) -> "WorkloadConfig":
        return replace(self, n=n)


CONFIGS = {
    "c1": WorkloadConfig("c1_sbm2k_fp64", 1, "sbm", 2000,
                         dict(num_blocks=7, p_in=0.01, p_out=0.0005),
                         form="ne", K=5, lam=0.05, self_loops=True, k=32, p=10, q=2,
                         precision="fp64"),
    "c2": WorkloadConfig("c2_chunglu200k_fp32", 2, "chung_lu", 200_000,
                         dict(beta=2.5, mean_degree=20.0),
                         form="ne", K=10, lam=0.1, k=128, p=16, q=3, precision="fp32"),
    "c3": WorkloadConfig("c3_featprop_sbm170k_fp32", 3, "sbm_deg", 170_000,
                         dict(num_blocks=40, mean_degree=14.0, frac_in=0.77),
                         form="featprop", d=128, L=3, k=64, p=16, q=2, precision="fp32"),
    "c4": WorkloadConfig("c4_chunglu2m_bf16", 4, "chung_lu", 2_000_000,
                         dict(beta=2.3, mean_degree=25.0),
                         form="ne", K=5, lam=0.05, k=256, p=32, q=2, precision="bf16"),
    "c5": WorkloadConfig("c5_chunglu1m_warmstart", 5, "chung_lu", 1_000_000,
                         dict(beta=2.5, mean_degree=20.0),
                         form="ne", K=10, lam=0.1, k=128, p=16, q=3, precision="fp32"),
}


def make_graph(cfg: WorkloadConfig, seed: int | None = None) -> Graph:
    s = cfg.index if seed is None else seed
    if cfg.graph == "sbm":
        return sbm_graph(cfg.n, seed=s, **cfg.graph_args)
    if cfg.graph == "sbm_deg":
        return sbm_graph_by_degree(cfg.n, seed=s, **cfg.graph_args)
    if cfg.graph == "chung_lu":
        return chung_lu_graph(cfg.n, seed=s, **cfg.graph_args)
    raise ValueError(cfg.graph)


def make_workload(cfg: WorkloadConfig, dtype=np.float64):
    """(graph, X or None, Omega) for a workload; Omega is c x l, FP64 draws
    rounded to `dtype`."""
    g = make_graph(cfg)
    x = None
    cols = g.n
    if cfg.form == "featprop":
        x = block_features(g.blocks, cfg.d, seed=1000 + cfg.index)
        cols = cfg.d * (cfg.L + 1)
    omega = gaussian_block(cols, cfg.l, cfg.omega_seed, dtype=dtype)
    return g, x, omega
