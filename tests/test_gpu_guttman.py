"""GPU parity: the exact stress-majorization step (layout_step_exact, the
appendix's Guttman transform by conjugate gradients) through the C ABI,
against the FP64 oracle's pseudo-inverse step."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import get_ops

pytestmark = pytest.mark.gpu

CG_TOL = 1e-7


@pytest.fixture(scope="module")
def ops():
    return get_ops()


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _scale(a):
    return np.abs(a).max()


@pytest.mark.parametrize("k", [5, 97, 300, 1000])
def test_exact_step_matches_pseudo_inverse(ops, k):
    D = synth.random_distance_matrix(k, synth.BASE_SEED + k)
    Y = synth.uniform_layout(k, synth.BASE_SEED + k + 1)
    print(f"[guttman] k={k}", flush=True)
    x, iters = ops.layout_step_exact(_t(D), _t(Y), cg_tol=CG_TOL)
    want = O.majorization_step(Y.astype(np.float64), D.astype(np.float64))
    got = x.double().cpu().numpy()
    assert np.abs(got - want).max() <= 1e-4 * _scale(want), (np.abs(got - want).max(), _scale(want), iters)
    assert 0 < iters < 1000
    np.testing.assert_allclose(got.mean(axis=0), 0.0, atol=1e-5 * _scale(want))


def test_exact_steps_from_a_real_pdist_never_increase_stress(ops):
    # PDist of an ER graph (n = 500, mean degree 8) computed on the GPU, then
    # ten exact steps from a uniform start: the stress falls at every step.
    g = synth.erdos_renyi(500, 8, synth.BASE_SEED)
    csr = ops.Csr.from_graph(g, "cuda")
    _, dppr, _, _ = ops.ppr_matrix(csr, np.arange(g.n), tol=1e-6, want_ppr=False)
    delta = ops.pdist(dppr, g.n)
    D = delta.double().cpu().numpy()
    x = _t(synth.uniform_layout(g.n, synth.BASE_SEED + 1))
    s_prev = O.stress(x.double().cpu().numpy(), D)
    for step in range(10):
        X = x.double().cpu().numpy()
        x, iters = ops.layout_step_exact(delta, x, cg_tol=CG_TOL)
        got = x.double().cpu().numpy()
        want = O.majorization_step(X, D)
        assert np.abs(got - want).max() <= 1e-4 * _scale(want), step
        s = O.stress(got, D)
        assert s <= s_prev * (1 + 1e-6), (step, s, s_prev)
        s_prev = s


def test_planted_layout_is_a_fixed_point(ops):
    P, Dp = synth.planted_layout_distances(40, synth.BASE_SEED + 7)
    Pc = (P - P.mean(axis=0)).astype(np.float32)
    x, _ = ops.layout_step_exact(_t(Dp), _t(Pc), cg_tol=CG_TOL)
    assert np.abs(x.double().cpu().numpy() - Pc).max() <= 1e-4 * _scale(Pc)


def test_coincident_points_and_converged_start(ops):
    # two coincident points: L^Y has no term for them, nothing is NaN
    k = 64
    D = synth.random_distance_matrix(k, synth.BASE_SEED + 50)
    Y = synth.uniform_layout(k, synth.BASE_SEED + 51)
    Y[7] = Y[3]
    x, _ = ops.layout_step_exact(_t(D), _t(Y), cg_tol=CG_TOL)
    got = x.double().cpu().numpy()
    assert np.all(np.isfinite(got))
    want = O.majorization_step(Y.astype(np.float64), D.astype(np.float64))
    assert np.abs(got - want).max() <= 1e-4 * _scale(want)
    # a start that already solves its system stops before the first iteration
    x2, iters = ops.layout_step_exact(_t(D), x, cg_tol=1.0)
    assert iters == 0
    np.testing.assert_allclose(x2.double().cpu().numpy(), got - got.mean(axis=0), atol=1e-6 * _scale(got))


def test_iteration_cap_and_invalid_arguments(ops):
    from paper_2112_14944_amd import _lib
    k = 200
    D = _t(synth.random_distance_matrix(k, synth.BASE_SEED + 60))
    Y = _t(synth.uniform_layout(k, synth.BASE_SEED + 61))
    x, iters = ops.layout_step_exact(D, Y, cg_tol=0.0, cg_max_iter=3, allow_noconv=True)
    assert iters == 3 and torch.isfinite(x).all()
    for kwargs in (dict(cg_tol=-1.0), dict(cg_tol=float("nan")), dict(cg_max_iter=-1)):
        with pytest.raises(_lib.PprvizError) as ei:
            ops.layout_step_exact(D, Y, **kwargs)
        assert ei.value.status == _lib.PPR_EINVAL
    with pytest.raises(_lib.PprvizError) as ei:
        ops.layout_step_exact(D, Y, out=Y)
    assert ei.value.status == _lib.PPR_EINVAL


def test_4096_node_layout_solves_its_system(ops):
    # The size of the 4096-source layout of the 10^6-node graph: the defining
    # equation L^w X+ = L^Y(Y) Y checked in FP64 with the oracle's Laplacians.
    k = 4096
    D = synth.random_distance_matrix(k, synth.BASE_SEED + 70, hi=2.0 * np.log(1e6))
    Y = synth.uniform_layout(k, synth.BASE_SEED + 71)
    print("[guttman] k=4096", flush=True)
    x, iters = ops.layout_step_exact(_t(D), _t(Y), cg_tol=1e-6)
    X = x.double().cpu().numpy()
    D64 = D.astype(np.float64)
    rhs = O.laplacian_y(D64, Y.astype(np.float64)) @ Y.astype(np.float64)
    res = O.laplacian_w(D64) @ X - rhs
    assert np.linalg.norm(res[:, 0]) <= 2e-5 * np.linalg.norm(rhs[:, 0])
    assert np.linalg.norm(res[:, 1]) <= 2e-5 * np.linalg.norm(rhs[:, 1])
    np.testing.assert_allclose(X.mean(axis=0), 0.0, atol=1e-5 * _scale(X))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_exact_step_tiny_layouts(ops, k):
    # k = 1: L^w = 0 and the centred solution is the origin; k = 2, 3: the
    # pseudo-inverse solution of a tiny system
    D = synth.random_distance_matrix(max(k, 2), synth.BASE_SEED + 80 + k)[:k, :k].copy()
    Y = synth.uniform_layout(k, synth.BASE_SEED + 90 + k)
    x, _ = ops.layout_step_exact(_t(D), _t(Y), cg_tol=CG_TOL)
    want = O.majorization_step(Y.astype(np.float64), D.astype(np.float64))
    got = x.double().cpu().numpy()
    assert np.abs(got - want).max() <= 1e-4 * max(_scale(want), 1e-30) + 1e-7
