"""GPU parity of the differentiable path: stress forward and the hand-written
backward with respect to coordinates and edge weights (adjoint PPR), against
the FP64 oracle gradient and central finite differences of the FP64 oracle
loss, plus invariants at the full n = 8192 size."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import ALPHA, get_ops

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    ops = get_ops()
    from paper_2112_14944_amd import autograd as AG
    return ops, AG


def _gpu_grads(ops, AG, g, X, T, budget=8 << 30):
    csr = ops.Csr.from_graph(g, "cuda", weighted=False)
    arc_edge, edge_arc = AG.edge_maps(g, "cuda")
    w = torch.as_tensor(g.weight, device="cuda").clone().requires_grad_(True)
    x = torch.as_tensor(X, device="cuda").clone().requires_grad_(True)
    loss = AG.pprviz_loss(w, x, csr, arc_edge, edge_arc, alpha=ALPHA, T=T, save_budget_bytes=budget)
    loss.backward()
    return loss.item(), w.grad.double().cpu().numpy(), x.grad.double().cpu().numpy()


@pytest.mark.parametrize("n,blocks", [(48, 3), (512, 8)])
def test_gradients_match_fp64_oracle(mods, n, blocks):
    ops, AG = mods
    g = synth.sbm(synth.equal_blocks(n, blocks), min(1.0, 24.0 * 0.8 / (n / blocks)), 24.0 * 0.2 / n, 900 + n,
                  weighted=(0.5, 2.0, 901 + n))
    X = synth.uniform_layout(n, 902 + n) * 4
    T = 100
    loss, gw, gx = _gpu_grads(ops, AG, g, X, T)
    ref = O.grad_weights(n, g.eu, g.ev, g.weight.astype(np.float64), X.astype(np.float64), ALPHA, T)
    assert abs(loss - ref["loss"]) <= 1e-5 * ref["loss"]
    assert np.abs(gx - ref["grad_x"]).max() <= 1e-4 * np.abs(ref["grad_x"]).max()
    assert np.abs(gw - ref["grad_w"]).max() <= 1e-3 * np.abs(ref["grad_w"]).max()
    rel = np.linalg.norm(gw - ref["grad_w"]) / np.linalg.norm(ref["grad_w"])
    assert rel <= 1e-4, rel


def test_gradients_against_central_differences(mods):
    # FD of the FP64 oracle loss, h = 1e-3, on sampled edges and coordinates
    ops, AG = mods
    n = 40
    g = synth.sbm(synth.equal_blocks(n, 2), 0.35, 0.05, 77, weighted=(0.5, 2.0, 78))
    X = synth.uniform_layout(n, 79) * 4
    T = 100
    _, gw, gx = _gpu_grads(ops, AG, g, X, T)
    w0 = g.weight.astype(np.float64)
    rng = np.random.default_rng(3)
    e_idx = rng.choice(len(w0), 16, replace=False)
    fd_w = O.central_difference(lambda wv: O.pipeline_forward(n, g.eu, g.ev, wv, X.astype(np.float64), ALPHA,
                                                              T)["loss"], w0, e_idx, 1e-3)
    scale = np.abs(gw).max()
    assert np.abs(gw[e_idx] - fd_w).max() <= 1e-3 * scale
    x_idx = rng.choice(2 * n, 16, replace=False)
    fd_x = O.central_difference(lambda xv: O.pipeline_forward(n, g.eu, g.ev, w0, xv.reshape(-1, 2), ALPHA,
                                                              T)["loss"], X.astype(np.float64).ravel(), x_idx, 1e-3)
    assert np.abs(gx.ravel()[x_idx] - fd_x).max() <= 1e-3 * np.abs(gx).max()


def test_sbm_8192_weighted_invariants_and_recompute(mods):
    # n = 8192 SBM (32 blocks of 256, mean degree 24, 80% of edges inside
    # blocks), weights U[0.5, 2], T = 100.  Checks that hold at any size:
    # translation / rotation invariance of dL/dX, the weight-scaling Euler
    # identity, and that recomputing PPR in backward gives the same bits.
    ops, AG = mods
    n = 8192
    g = synth.sbm(synth.equal_blocks(n, 32), 0.0753, 6.05e-4, synth.BASE_SEED + 3,
                  weighted=(0.5, 2.0, synth.BASE_SEED + 4))
    print(f"[sbm n=8192] n={n} nnz={g.nnz}", flush=True)
    X = synth.uniform_layout(n, synth.BASE_SEED + 5) * 20
    T = 100
    loss, gw, gx = _gpu_grads(ops, AG, g, X, T)
    assert np.isfinite(loss) and np.all(np.isfinite(gw)) and np.all(np.isfinite(gx))
    s = np.abs(gx).sum()
    assert np.abs(gx.sum(0)).max() <= 1e-4 * s
    assert abs((X[:, 0] * gx[:, 1] - X[:, 1] * gx[:, 0]).sum()) <= 1e-3 * (np.abs(X).max() * s)
    # Euler identity from the GPU's own intermediates
    csr = ops.Csr.from_graph(g, "cuda", weighted=True)
    _, dppr, _, _ = ops.ppr_matrix(csr, np.arange(n), tol=0.0, max_iter=T, want_ppr=False)
    delta = ops.pdist(dppr, n)
    _, gd = ops.stress_backward(delta, torch.as_tensor(X, device="cuda"), want_grad_x=False)
    dz = ops.pdist_backward(dppr, torch.ones_like(gd), n)  # -1/z inside the clamps, else 0
    inside = (dz != 0).double()
    rhs = -(gd.double() * inside).sum().item() / 2.0  # each unordered pair appears twice
    lhs = float((g.weight.astype(np.float64) * gw).sum())
    assert abs(lhs - rhs) <= 1e-3 * max(abs(rhs), np.abs(g.weight * gw).sum() * 1e-3), (lhs, rhs)
    _, gw2, gx2 = _gpu_grads(ops, AG, g, X, T, budget=0)
    np.testing.assert_array_equal(gw2, gw)
    np.testing.assert_array_equal(gx2, gx)
