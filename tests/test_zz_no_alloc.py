"""ppr_matrix_noalloc, the entry point that allocates nothing, against
ppr_matrix on the same inputs: two calls in a row on one GPU (the second on
a smaller graph, so that it runs over the first call's leftovers in the
shared scratch array), each compared bit for bit, since both entry points
run the same kernels in the same order; plus the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_util import ALPHA, get_ops

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    return get_ops()


def _both(ops, g, src, tgt, weighted):
    csr = ops.Csr.from_graph(g, "cuda", weighted=weighted)
    ppr, dppr, T, resid = ops.ppr_matrix(csr, src, tgt=tgt, alpha=ALPHA, tol=1e-6, check_residual=True)
    n_tgt = g.n if tgt is None else len(tgt)
    ppr2 = torch.full((len(src), n_tgt), float("nan"), device="cuda")
    dppr2 = torch.full_like(ppr2, float("nan"))
    T2, resid2 = ops.ppr_matrix_noalloc(csr, src, tgt=tgt, alpha=ALPHA, tol=1e-6, ppr=ppr2, dppr=dppr2,
                                        check_residual=True)
    torch.cuda.synchronize()
    assert T2 == T == 86
    assert torch.equal(ppr2, ppr) and torch.equal(dppr2, dppr)
    np.testing.assert_array_equal(resid2, resid)
    return ppr2


def test_noalloc_matches_ppr_matrix_two_calls(ops):
    # first call: weighted SBM, 1500 nodes (16-column tiles), all sources
    g1 = synth.sbm(synth.equal_blocks(1500, 6), 0.08, 0.004, 41, weighted=(0.5, 2.0, 42))
    print(f"[noalloc] call 1: n={g1.n} nnz={g1.nnz} weighted, all sources", flush=True)
    _both(ops, g1, np.arange(g1.n), None, True)
    # second call, smaller: unweighted ER, 300 nodes (64-column tiles), 70
    # sources and 90 targets
    g2 = synth.erdos_renyi(300, 8, 43)
    src = synth.random_sources(g2, 70, 44)
    tgt = np.sort(np.random.default_rng(45).choice(g2.n, 90, replace=False)).astype(np.int32)
    print(f"[noalloc] call 2: n={g2.n} nnz={g2.nnz}, {len(src)} sources x {len(tgt)} targets", flush=True)
    _both(ops, g2, src, tgt, False)


def test_noalloc_rejects_oversized_workspace(ops):
    from paper_2112_14944_amd import _lib as L
    g = synth.erdos_renyi(6000, 20, 46)  # mid-size path: its workspace exceeds the scratch array
    csr = ops.Csr.from_graph(g, "cuda")
    cg = csr.c()
    assert L.lib().ppr_matrix_workspace(C.byref(cg), g.n, g.n) > L.lib().ppr_matrix_noalloc_max_scratch()
    with pytest.raises(L.PprvizError) as ei:
        ops.ppr_matrix_noalloc(csr, np.arange(g.n), ppr=torch.empty((g.n, g.n), device="cuda"))
    assert ei.value.status == L.PPR_EUNSUPPORTED
