"""GPU parity: PDist, stress, Jacobi layout step and their backward kernels on
seeded synthetic inputs, through the C ABI, against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import PDIST_REL, STEP_REL, STRESS_REL, get_ops, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    return get_ops()


def _dppr_like(k, seed, kinks=True):
    """Positive DPPR-like matrix with unreachable (0) pairs and (optionally)
    an entry exactly on the lower clamp kink."""
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(-12, 0.5, size=(k, k)))
    a[rng.random((k, k)) < 0.05] = 0.0
    if k >= 4 and kinks:
        a[0, 1], a[1, 0] = math.exp(-1) / 2, math.exp(-1) / 2     # z = 1/e: Delta = 2 exactly
        a[2, 3], a[3, 2] = 0.0, 0.0                                # unreachable pair
    return a.astype(np.float32)


@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 1000])
def test_pdist_matches_oracle(ops, k):
    a = _dppr_like(k, 100 + k)
    n_clamp = 3 * k + 7
    got = ops.pdist(torch.as_tensor(a, device="cuda"), n_clamp).double().cpu().numpy()
    want = O.pdist(a.astype(np.float64), n_clamp)
    assert np.all(np.diag(got) == 0)
    assert rel_err(got, want) <= PDIST_REL
    np.testing.assert_array_equal(got, got.T)  # exactly symmetric


# below 1025 nodes the row sweep, from 1025 on the pair-tile sweep (ragged
# last tile at 1100 and 2000)
@pytest.mark.parametrize("k", [1, 2, 17, 300, 1000, 1024, 1025, 1100, 2000])
def test_layout_step_and_stress(ops, k):
    D = synth.random_distance_matrix(k, 200 + k)
    X = synth.uniform_layout(k, 300 + k)
    d_t = torch.as_tensor(D, device="cuda")
    x_t = torch.as_tensor(X, device="cuda")
    x1, st = ops.layout_step(d_t, x_t, with_stress=True)
    s2 = ops.stress_eval(d_t, x_t)
    Dd, Xd = D.astype(np.float64), X.astype(np.float64)
    want_s = O.stress(Xd, Dd)
    if k == 1:
        assert st.item() == 0.0 and s2.item() == 0.0
        np.testing.assert_array_equal(x1.cpu().numpy(), X)
        return
    assert abs(st.item() - want_s) <= STRESS_REL * want_s
    assert st.item() == s2.item()
    want_x = O.jacobi_step(Xd, Dd)
    assert np.abs(x1.double().cpu().numpy() - want_x).max() <= STEP_REL * np.abs(want_x).max()


@pytest.mark.parametrize("k", [40, 1100])
def test_layout_coincident_points(ops, k):
    D = synth.random_distance_matrix(k, 5)
    X = synth.uniform_layout(k, 6)
    X[3] = X[7]
    X[10] = X[7]
    X[k - 1] = X[7]  # a coincident pair across 64-node tiles
    d_t = torch.as_tensor(D, device="cuda")
    x_t = torch.as_tensor(X, device="cuda")
    x1, st = ops.layout_step(d_t, x_t, with_stress=True)
    want_x = O.jacobi_step(X.astype(np.float64), D.astype(np.float64))
    assert np.all(np.isfinite(x1.cpu().numpy()))
    assert np.abs(x1.double().cpu().numpy() - want_x).max() <= STEP_REL * np.abs(want_x).max()
    assert abs(st.item() - O.stress(X.astype(np.float64), D.astype(np.float64))) <= STRESS_REL * st.item()
    gx, gd = ops.stress_backward(d_t, x_t)
    assert np.all(np.isfinite(gx.cpu().numpy())) and np.all(np.isfinite(gd.cpu().numpy()))


@pytest.mark.parametrize("k", [2, 33, 300])
def test_stress_backward(ops, k):
    D = synth.random_distance_matrix(k, 400 + k)
    X = synth.uniform_layout(k, 500 + k) * 3
    d_t = torch.as_tensor(D, device="cuda")
    x_t = torch.as_tensor(X, device="cuda")
    gx, gd = ops.stress_backward(d_t, x_t, grad_scale=0.5)
    Xd, Dd = X.astype(np.float64), D.astype(np.float64)
    want_gx = 0.5 * O.grad_x(Xd, Dd)
    want_gd = 0.5 * O.grad_delta_pair(Xd, Dd)
    assert np.abs(gx.double().cpu().numpy() - want_gx).max() <= 1e-5 * np.abs(want_gx).max()
    gdn = gd.double().cpu().numpy()
    assert np.abs(gdn - want_gd).max() <= 1e-5 * np.abs(want_gd).max()
    np.testing.assert_array_equal(gdn, gdn.T)
    gx_only, none = ops.stress_backward(d_t, x_t, grad_scale=0.5, want_grad_delta=False)
    assert none is None
    np.testing.assert_array_equal(gx_only.cpu().numpy(), gx.cpu().numpy())


@pytest.mark.parametrize("k", [3, 64, 257])
def test_pdist_backward(ops, k):
    # no pair on a kink: there the clamp decision depends on the precision
    a = _dppr_like(k, 600 + k, kinks=False)
    n_clamp = 2 * k + 3
    G = synth.random_distance_matrix(k, 700 + k) - 3.0  # any symmetric upstream gradient
    got = ops.pdist_backward(torch.as_tensor(a, device="cuda"), torch.as_tensor(G, device="cuda"),
                             n_clamp).double().cpu().numpy()
    want = G.astype(np.float64) * O.pdist_dz(a.astype(np.float64), n_clamp)
    np.fill_diagonal(want, 0.0)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-5 * scale
