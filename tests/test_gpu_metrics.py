"""GPU parity: layout metrics (layout_metrics: ND and ULCV) through the C ABI
against the FP64 oracle's double loops."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import get_ops

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    return get_ops()


@pytest.mark.parametrize("n,seed", [(2, 1), (97, 2), (500, 3), (1000, 4)])
def test_metrics_match_oracle(ops, n, seed):
    g = synth.erdos_renyi(n, min(8, n - 1), synth.BASE_SEED + seed)
    X = synth.uniform_layout(n, synth.BASE_SEED + seed + 1)
    x = torch.as_tensor(X, device="cuda")
    nd, ul = ops.layout_metrics(x, ops.Csr.from_graph(g, "cuda"))
    X64 = X.astype(np.float64)
    nd_o = O.node_distribution(X64)
    assert abs(nd - nd_o) <= 1e-9 * nd_o
    ul_o = O.ulcv(X64, g.eu, g.ev)
    if math.isnan(ul_o):
        assert math.isnan(ul)
    else:
        assert abs(ul - ul_o) <= 1e-9 * ul_o


def test_metrics_special_cases(ops):
    # unit square with its 4 sides as edges: ND = 5, every edge length 1
    X = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float32)
    g = synth.build_graph(4, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 3]))
    nd, ul = ops.layout_metrics(torch.as_tensor(X, device="cuda"), ops.Csr.from_graph(g, "cuda"))
    assert abs(nd - 5.0) < 1e-12 and abs(ul) < 1e-12
    # a coincident pair: ND infinite; a graph without edges: ULCV undefined
    X[3] = X[0]
    g0 = synth.build_graph(4, np.zeros(0, np.int64), np.zeros(0, np.int64))
    nd, ul = ops.layout_metrics(torch.as_tensor(X, device="cuda"), ops.Csr.from_graph(g0, "cuda"))
    assert nd == math.inf and math.isnan(ul)
    nd_only, none = ops.layout_metrics(torch.as_tensor(X, device="cuda"))
    assert nd_only == math.inf and none is None


def test_metrics_of_a_computed_layout(ops):
    # the full path on the 500-node ER graph: PPR -> PDist -> 300 Jacobi
    # sweeps; ND and ULCV of the result against the oracle on the same layout
    g = synth.erdos_renyi(500, 8, synth.BASE_SEED)
    csr = ops.Csr.from_graph(g, "cuda")
    _, dppr, _, _ = ops.ppr_matrix(csr, np.arange(g.n), tol=1e-6, want_ppr=False)
    delta = ops.pdist(dppr, g.n)
    x = ops.layout(delta, torch.as_tensor(synth.uniform_layout(g.n, synth.BASE_SEED + 1), device="cuda"), 300)
    nd, ul = ops.layout_metrics(x, csr)
    X = x.double().cpu().numpy()
    assert abs(nd - O.node_distribution(X)) <= 1e-9 * nd
    assert abs(ul - O.ulcv(X, g.eu, g.ev)) <= 1e-9 * ul


def test_metrics_single_point(ops):
    x = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    g = synth.build_graph(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    nd, ul = ops.layout_metrics(x, ops.Csr.from_graph(g, "cuda"))
    assert nd == 0.0 and math.isnan(ul)
