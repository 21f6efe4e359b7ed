"""The paper's NE/NC variants as symbolic DAGs on the device, against the
oracle's DAG: the symmetric NE form with A_hat in place of T (Section 3.1,
L = R), label re-use and pseudo-dropout (Section 5.3)."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_helpers import col_rel_err, gapped_k, rounded, to_dev, to_np
from oracle import symbolic as sym
from synth import block_features, gaussian_block, sbm_graph

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


def _leaves(lib, g, precision):
    """Device DAG and oracle leaves: A, A + I, (D+I)^-1/2 and (D+I)^-1."""
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(g.n, g.n))
    ai = (a + sp.identity(g.n, format="csr")).tocsr()
    ai.sort_indices()
    d1 = np.diff(ai.indptr).astype(np.float64)          # degree + 1
    dag = lib.Dag(precision)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    AI = dag.sparse(ai.indptr, ai.indices, ai.shape)
    R = dag.diag(1.0 / np.sqrt(d1))
    Dinv1 = dag.diag(1.0 / d1)
    ah = R @ AI @ R
    oah = sym.diag(1.0 / np.sqrt(d1)) @ sym.sparse(ai) @ sym.diag(1.0 / np.sqrt(d1))
    return dag, dict(A=A, ah=ah, Dinv1=Dinv1), dict(A=sym.sparse(a), ah=oah, Dinv1=sym.diag(1.0 / d1))


def _products(op, ref, dt, tol, l=10, seed=5):
    y = rounded(gaussian_block(ref.shape[1], l, seed=seed), dt)
    assert col_rel_err(to_np(op.matmul(to_dev(y, dt))), ref.dot(y)) <= tol
    z = rounded(gaussian_block(ref.shape[0], l, seed=seed + 1), dt)
    assert col_rel_err(to_np(op.matmul(to_dev(z, dt), transpose=True)), ref.T.dot(z)) <= tol


def test_symmetric_ne_form_gives_equal_left_and_right_embeddings(gpu_lib):
    _case("symmetric NE")
    g = sbm_graph(2000, 5, 0.01, 0.001, seed=51)
    dag, d, o = _leaves(gpu_lib, g, 0)
    one = dag.dense(torch.ones((g.n, 1), dtype=torch.float64, device="cuda"))
    c = [0.5, 0.3, 0.2]
    m = dag.sum([d["ah"] ** j for j in (1, 2, 3)], c) - 0.05 * (one @ one.T - d["A"])
    om = sym.dense(np.ones((g.n, 1)))
    ref = sym.lincomb([o["ah"] ** j for j in (1, 2, 3)], c) - 0.05 * (om @ om.T - o["A"])
    op = dag.operator(m)
    _products(op, ref, torch.float64, 1e-12)
    U, S, V, info = op.truncated_svd(24, 16, tol=1e-8, max_iter=2000, seed=3)
    u, s, v = to_np(U), to_np(S), to_np(V)
    kk = gapped_k(np.append(s, 0.0), 24, rel_gap=1e-2)
    # M = M^T: u_i = +-v_i for separated singular values, so L = U S^1/2 and R = V S^1/2 agree up to sign
    assert kk > 0
    assert np.abs(np.abs(np.sum(u[:, :kk] * v[:, :kk], axis=0)) - 1.0).max() < 1e-5
    op.close()
    dag.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-5)])
def test_label_reuse_design_matrix(gpu_lib, precision, tol):
    _case("label re-use", precision)
    g = sbm_graph(3000, 6, 0.006, 0.0005, seed=52)
    dt = {0: torch.float64, 1: torch.float32}[precision]
    x = rounded(block_features(g.blocks, 8, seed=53), dt)
    ytr = np.zeros((g.n, 6))
    train = np.random.default_rng(54).choice(g.n, g.n // 2, replace=False)
    ytr[train, g.blocks[train]] = 1.0
    dag, d, o = _leaves(gpu_lib, g, precision)
    X, Y = dag.dense(to_dev(x, dt)), dag.dense(to_dev(ytr, dt))
    b = d["ah"] - d["Dinv1"]
    m = dag.concat_cols([X, d["ah"] @ X, d["ah"] @ d["ah"] @ X, b @ Y, b @ b @ Y])
    ob = o["ah"] - o["Dinv1"]
    oX, oY = sym.dense(x), sym.dense(ytr)
    ref = sym.hstack([oX, o["ah"] @ oX, o["ah"] @ o["ah"] @ oX, ob @ oY, ob @ ob @ oY])
    op = dag.operator(m)
    assert op.shape == ref.shape == (g.n, 8 * 3 + 12)
    _products(op, ref, dt, tol)
    op.close()
    dag.close()


def test_pseudo_dropout_row_stacking(gpu_lib):
    # [M; PD(M)]: the feature design matrix stacked on the one built from a
    # dropped-out copy of X (each feature value zeroed with probability 0.2)
    _case("pseudo-dropout")
    g = sbm_graph(2500, 5, 0.006, 0.0006, seed=55)
    x = block_features(g.blocks, 10, seed=56).astype(np.float64)
    xpd = x * (np.random.default_rng(57).random(x.shape) >= 0.2)
    dag, d, o = _leaves(gpu_lib, g, 0)
    X, XPD = dag.dense(to_dev(x, torch.float64)), dag.dense(to_dev(xpd, torch.float64))
    m = dag.concat_cols([X, d["ah"] @ X, d["ah"] ** 2 @ X])
    mpd = dag.concat_cols([XPD, d["ah"] @ XPD, d["ah"] ** 2 @ XPD])
    stacked = dag.concat_cols([m.T, mpd.T]).T
    oX, oXPD = sym.dense(x), sym.dense(xpd)
    ref = sym.vstack([sym.hstack([oX, o["ah"] @ oX, o["ah"] ** 2 @ oX]),
                        sym.hstack([oXPD, o["ah"] @ oXPD, o["ah"] ** 2 @ oXPD])])
    op = dag.operator(stacked)
    assert op.shape == ref.shape == (2 * g.n, 30)
    _products(op, ref, torch.float64, 1e-12)
    # the stacked matrix keeps the width of M: its SVD is exact at full rank
    om = gaussian_block(30, 30, seed=58)
    U, S, V, info = op.truncated_svd(30, 0, q=0, omega=to_dev(om, torch.float64))
    dense = ref.dot(np.eye(30))
    assert np.allclose(to_np(S), np.linalg.svd(dense, compute_uv=False), rtol=1e-10)
    op.close()
    dag.close()
