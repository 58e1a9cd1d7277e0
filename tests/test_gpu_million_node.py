"""Large multi-source case at full size: Chung-Lu n = 10^6, exponent 2.2, mean
degree 30 (int32 CSR, ~3e7 arcs), PPR from 4096 seeded sources with at least
one arc, accumulated only at the 4096 source nodes as targets (the
4096 x 4096 DPPR block among the sources), to L1 residual 1e-6 (T = 86);
PDist among the sources with n_clamp = 10^6; a 4096-node stress layout with
Jacobi sweeps and gradient refinement.

The FP64 oracle rows come from tests/golden/chung_lu_1e6_rows.npz (written by
make_chung_lu_1e6_rows.py, which calls only the oracle): 16 of the 4096
sources (the four of highest degree and twelve seeded others) over all their
targets, and the four highest-degree nodes of the whole graph (hubs, where
pi_d(s, s) >= alpha d(s) is largest) as sources of a second call.  The oracle
also checks the PDist rows of the 16 sources, one Jacobi step and the stress
gradient of the 4096-node layout."""
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import (ALPHA, PDIST_REL, STEP_REL, STRESS_REL, assert_ppr_close, get_ops, oracle_ppr,
                      rel_err)

pytestmark = pytest.mark.gpu

N = 1_000_000
S = 4096


@pytest.fixture(scope="module")
def ops():
    return get_ops()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chung_lu_1e6_rows.npz")


def _golden(g, src):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_rows", os.path.join(os.path.dirname(GOLDEN), "make_chung_lu_1e6_rows.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    z = np.load(GOLDEN)
    assert str(z["digest"]) == mk.digest(g, src), "the seeded generators no longer give the stored graph"
    rows, hubs, tgt = mk.picks(g, src)
    np.testing.assert_array_equal(rows, z["rows"])
    np.testing.assert_array_equal(hubs, z["hubs"])
    np.testing.assert_array_equal(tgt, z["tgt"])
    assert int(z["T"]) == 86
    return z


def test_million_node_graph_4096_sources(ops):
    g = synth.chung_lu(N, 2.2, 30, synth.BASE_SEED + 4)
    src = synth.random_sources(g, S, synth.BASE_SEED + 5)
    print(f"[n=1e6] n={g.n} nnz={g.nnz} sources={S}", flush=True)
    z = _golden(g, src)
    deg = np.diff(g.row_ptr).astype(np.float64)
    csr = ops.Csr.from_graph(g, "cuda")
    ppr, dppr, T, resid = ops.ppr_matrix(csr, src, tgt=src, tol=1e-6, check_residual=True)
    torch.cuda.synchronize()
    print("[n=1e6] ppr done", flush=True)
    assert T == 86 and ppr.shape == (S, S)
    # residual over all 10^6 targets (FP64 sum of the FP32 iterate)
    assert np.abs(resid - (1 - ALPHA) ** 86).max() <= 2e-6

    # 16 sources over all 4096 targets: the four of highest degree among the
    # sources and twelve others
    pick = z["rows"]
    tpos = np.searchsorted(z["tgt"], src.astype(np.int64))
    est = z["ppr_tgt"][:16][:, tpos]
    d_src = deg[src[pick]]
    dppr_o = est * d_src[:, None]
    np.testing.assert_allclose(resid[pick], z["resid"][:16], rtol=0, atol=2e-6)
    pidx = torch.as_tensor(pick, device="cuda").long()
    err, errd = assert_ppr_close(ppr[pidx], dppr[pidx], est, dppr_o, d_src)
    print(f"[n=1e6] 16 sources (degrees {d_src[:4].astype(int).tolist()} + 12): PPR max-abs {err:.2e}, "
          f"DPPR per unit degree {errd:.2e}", flush=True)

    # the four hubs of the whole graph as sources, at the same targets plus
    # themselves (pi_d(s, s) of a hub is the largest DPPR value of the graph)
    hubs = z["hubs"]
    tgt_h = z["tgt"]
    ppr_h, dppr_h, T_h, resid_h = ops.ppr_matrix(csr, hubs.astype(np.int32), tgt=tgt_h.astype(np.int32), tol=1e-6,
                                                 check_residual=True)
    assert T_h == 86
    np.testing.assert_allclose(resid_h, z["resid"][16:], rtol=0, atol=2e-6)
    est_h = z["ppr_tgt"][16:]
    err_h, errd_h = assert_ppr_close(ppr_h, dppr_h, est_h, est_h * deg[hubs][:, None], deg[hubs])
    print(f"[n=1e6] 4 hubs (degrees {deg[hubs].astype(int).tolist()}): PPR max-abs {err_h:.2e}, "
          f"DPPR per unit degree {errd_h:.2e}", flush=True)
    del ppr_h, dppr_h
    del ppr

    # PDist among the sources, n_clamp = |V| of the whole graph.  The oracle's
    # row i needs pi_d(j, i) for every source j; on an undirected graph it
    # equals pi_d(i, j) (reversibility, pinned in the oracle tests).
    delta = ops.pdist(dppr, N)
    dl = delta.double().cpu().numpy()
    np.testing.assert_array_equal(dl, dl.T)
    off = ~np.eye(S, dtype=bool)
    assert dl[off].min() >= 2.0 and dl[off].max() <= 2.0 * np.log(N) * (1 + 1e-6)
    Drows = O.pdist_of_z(2.0 * dppr_o, N)
    Drows[np.arange(len(pick)), pick] = 0.0
    assert rel_err(dl[pick], Drows) <= PDIST_REL

    # 4096-node layout: one Jacobi step against the oracle, then 200 sweeps
    x0 = torch.as_tensor(synth.uniform_layout(S, synth.BASE_SEED + 6), device="cuda")
    x1, st0 = ops.layout_step(delta, x0, with_stress=True)
    X0 = x0.double().cpu().numpy()
    want = O.jacobi_step(X0, dl)
    assert np.abs(x1.double().cpu().numpy() - want).max() <= STEP_REL * np.abs(want).max()
    assert abs(st0.item() - O.stress(X0, dl)) <= STRESS_REL * st0.item()
    xl = ops.layout(delta, x0, 200)
    st_l = ops.stress_eval(delta, xl).item()
    assert np.isfinite(st_l) and st_l < st0.item()

    # gradient refinement: the stress gradient against the oracle, then a few
    # descent steps with a backtracking step size lower the stress further
    gx, _ = ops.stress_backward(delta, xl, want_grad_delta=False)
    XL = xl.double().cpu().numpy()
    g_o = O.grad_x(XL, dl)
    assert np.abs(gx.double().cpu().numpy() - g_o).max() <= 1e-4 * np.abs(g_o).max()
    x = xl.clone()
    st = st_l
    lr = 1e-3
    for _ in range(10):
        gx, _ = ops.stress_backward(delta, x, want_grad_delta=False)
        while True:
            xn = x - lr * gx
            sn = ops.stress_eval(delta, xn).item()
            if sn < st or lr < 1e-12:
                break
            lr *= 0.5
        x, st = xn, min(st, sn)
    assert st <= st_l
    print(f"[n=1e6] stress {st0.item():.4e} -> {st_l:.4e} (200 sweeps) -> {st:.4e} (gradient)", flush=True)
