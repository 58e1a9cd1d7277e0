"""GPU parity: multi-source PPR / DPPR / PDist / layout on single graphs,
through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import (ALPHA, PDIST_REL, STEP_REL, assert_ppr_close, get_ops, oracle_ppr, rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    return get_ops()


def _csr(ops, g):
    return ops.Csr.from_graph(g, "cuda")


def test_erdos_renyi_500_all_pairs(ops):
    # ER n=500, mean degree 8, all 500 sources, L1 residual 1e-10 (T = 142),
    # then PDist and 300 Jacobi layout steps from U[-1,1]^2.
    g = synth.erdos_renyi(500, 8, synth.BASE_SEED)
    src = np.arange(g.n)
    print(f"[er n=500] n={g.n} nnz={g.nnz}", flush=True)
    ppr, dppr, T, resid = ops.ppr_matrix(_csr(ops, g), src, tol=1e-10, check_residual=True)
    est, dppr_o, T_o, res_o, d = oracle_ppr(g, src, tol=1e-10)
    assert T == T_o == 142
    assert_ppr_close(ppr, dppr, est, dppr_o, d[src])
    assert np.abs(resid - res_o).max() <= 2e-6
    delta = ops.pdist(dppr, g.n)
    D_o = O.pdist(dppr_o, g.n)
    assert rel_err(delta.double().cpu().numpy(), D_o) <= PDIST_REL
    x0 = torch.as_tensor(synth.uniform_layout(g.n, synth.BASE_SEED + 1), device="cuda")
    # one step from the same start, then the 300-step trajectory's final stress
    x1, s0 = ops.layout_step(delta, x0, with_stress=True)
    X0 = x0.double().cpu().numpy()
    assert abs(s0.item() - O.stress(X0, D_o)) <= 1e-5 * O.stress(X0, D_o)
    assert rel_err(x1.double().cpu().numpy(), O.jacobi_step(X0, D_o)) <= STEP_REL
    xf = ops.layout(delta, x0, 300)
    s_gpu = ops.stress_eval(delta, xf).item()
    Xo = X0
    for _ in range(300):
        Xo = O.jacobi_step(Xo, D_o)
    s_o = O.stress(Xo, D_o)
    assert abs(s_gpu - s_o) <= 1e-3 * s_o, (s_gpu, s_o)
    assert s_gpu < O.stress(X0, D_o)


@pytest.mark.parametrize("n", [300, 5000, 12000, 25000])
def test_weighted_isolated_subsets(ops, n):
    # weighted SBM with an isolated node, a ragged source subset, a shuffled
    # target subset, fixed T (tol <= 0); n = 300 runs the resident tile, the
    # others the mid-size kernel at 4, 2 and 1 columns per block
    blocks = 5 if n == 300 else 16
    p_in = 0.12 if n == 300 else 12.0 / (n / blocks)
    p_out = 0.01 if n == 300 else 2.0 / n
    g0 = synth.sbm(synth.equal_blocks(n, blocks), p_in, p_out, 77 + n, weighted=(0.5, 2.0, 78))
    keep = (g0.eu != 7) & (g0.ev != 7)
    g = synth.build_graph(n, g0.eu[keep], g0.ev[keep], g0.weight[keep])
    rng = np.random.default_rng(5)
    src = np.sort(rng.choice(n, 77, replace=False))
    src[3] = 7  # the isolated node is a source too
    src = np.unique(src)
    tgt = rng.permutation(n)
    tgt = np.concatenate([[7], tgt[tgt != 7]])[:123]  # shuffled, holds the isolated node
    tgt = np.roll(tgt, 40)
    print(f"[weighted] n={n} nnz={g.nnz} sources={len(src)}", flush=True)
    ppr, dppr, T, resid = ops.ppr_matrix(_csr(ops, g), src, tgt=tgt, tol=0.0, max_iter=60, check_residual=True)
    est, dppr_o, T_o, res_o, d = oracle_ppr(g, src, T=60)
    assert T == 60
    assert_ppr_close(ppr, dppr, est[:, tgt], dppr_o[:, tgt], d[src])
    assert np.abs(resid - res_o).max() <= 2e-6
    i7 = int(np.nonzero(src == 7)[0][0])
    # isolated source keeps its mass: pi(7,7) = 1 - (1-alpha)^T
    assert abs(ppr[i7].cpu().numpy()[tgt == 7].item() - (1 - (1 - ALPHA) ** 60)) <= 1e-6


@pytest.mark.parametrize("n", [576, 577, 1152, 1153, 2304, 2305, 3001, 10207, 10208, 20415, 20416, 40831, 40832])
def test_kernel_size_boundaries(ops, n):
    # 64/32/16-column resident tiles switch at 576/1152/2304; the mid-size
    # kernel keeps 4/2/1 columns of every node in LDS up to 10207/20415/40831;
    # above that the iterate streams through HBM.
    g = synth.erdos_renyi(n, 10, 1000 + n)
    src = synth.random_sources(g, 70, 2000 + n)
    print(f"[sizes] n={n} nnz={g.nnz}", flush=True)
    ppr, dppr, T, resid = ops.ppr_matrix(_csr(ops, g), src, tol=1e-6, check_residual=True)
    est, dppr_o, T_o, res_o, d = oracle_ppr(g, src, tol=1e-6)
    assert T == T_o == 86
    assert_ppr_close(ppr, dppr, est, dppr_o, d[src])
    assert np.abs(resid - res_o).max() <= 2e-6


@pytest.mark.parametrize("case", ["cl3000w", "cl12000", "cl25000", "star5000"])
def test_mid_split_long_rows(ops, case):
    # power-law graphs whose longest rows exceed a wave's share of a push: the
    # mid-size kernel cuts them into parts whose partial sums it adds back in
    # part order (4, 2 and 1 columns per block; a weighted case with a
    # shuffled target subset; a star whose hub becomes hundreds of parts)
    rng = np.random.default_rng(11)
    tgt = None
    if case == "cl3000w":
        g0 = synth.chung_lu(3000, 2.1, 40, 9)
        w = (0.5 + 1.5 * rng.random(g0.m_und)).astype(np.float32)
        g = synth.build_graph(g0.n, g0.eu, g0.ev, w)
        tgt = rng.permutation(g.n)[:777]
    elif case == "cl12000":
        g = synth.chung_lu(12000, 2.1, 30, 100 + 12000)
    elif case == "cl25000":
        g = synth.chung_lu(25000, 2.1, 20, 100 + 25000)
    else:
        n = 5000
        g = synth.build_graph(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))
    src = synth.random_sources(g, 70, 3000 + g.n)
    src[0] = int(np.argmax(np.diff(g.row_ptr)))  # the longest row is a source too
    src = np.unique(src)
    print(f"[split] {case} n={g.n} nnz={g.nnz} max degree={np.diff(g.row_ptr).max()}", flush=True)
    ppr, dppr, T, resid = ops.ppr_matrix(_csr(ops, g), src, tgt=tgt, tol=1e-6, check_residual=True)
    est, dppr_o, T_o, res_o, d = oracle_ppr(g, src, tol=1e-6)
    assert T == T_o == 86
    if tgt is not None:
        est, dppr_o = est[:, tgt], dppr_o[:, tgt]
    assert_ppr_close(ppr, dppr, est, dppr_o, d[src])
    assert np.abs(resid - res_o).max() <= 2e-6


def _repeated_arc_csr(ops, n, reps):
    # nodes 0 and 1 joined by `reps` parallel arcs each way, all others isolated
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1] = reps
    row_ptr[2:] = 2 * reps
    col = np.concatenate([np.full(reps, 1), np.full(reps, 0)]).astype(np.int32)
    return ops.Csr(n, len(col), torch.as_tensor(row_ptr, device="cuda"), torch.as_tensor(col, device="cuda"), None)


def test_mid_repeated_arcs(ops):
    # rows far longer than n (repeated neighbours) are cut into parts like any
    # long row; the walk is that of a two-node path, with node 5 isolated
    csr = _repeated_arc_csr(ops, 2400, 5000)
    ppr, _, T, resid = ops.ppr_matrix(csr, [0, 5], tol=1e-6, check_residual=True)
    est, _, T_o, _, _ = oracle_ppr(synth.build_graph(2, [0], [1]), [0], T=T)
    p = ppr.double().cpu().numpy()
    assert abs(p[0, 0] - est[0, 0]) <= 1e-6 and abs(p[0, 1] - est[0, 1]) <= 1e-6
    assert np.abs(p[0, 2:]).max() == 0.0
    assert abs(p[1, 5] - (1 - (1 - ALPHA) ** T)) <= 1e-6
    assert np.abs(resid - (1 - ALPHA) ** T).max() <= 2e-6


def test_mid_repeated_arcs_flagged(ops):
    # at n = 10207 the iterate of 4 columns fills the LDS, leaving no room for
    # partial sums, so the rows cannot be cut: the padded arc copy would
    # exceed its workspace bound, which the kernel reports as NaN outputs
    csr = _repeated_arc_csr(ops, 10207, 200000)
    from paper_2112_14944_amd._lib import PPR_ENONFINITE, PprvizError
    with pytest.raises(PprvizError) as ei:
        ops.ppr_matrix(csr, [0, 5], tol=1e-6, check_residual=True)
    assert ei.value.status == PPR_ENONFINITE
    ppr, _, _, _ = ops.ppr_matrix(csr, [0, 5], tol=1e-6)
    assert torch.isnan(ppr).all().item()


def test_resident_repeated_arcs(ops):
    # n = 300 (resident tile, groups of 4 rows): two rows of 2000 repeated arcs
    # pad their group to 2000 arcs per row, which still fits the arc copy's
    # reserved region; the walk is that of a two-node path, node 5 isolated.
    # Each row sums its 2000 equal terms one after another in FP32 (relative
    # error up to 2000 u per push, u = 2^-24), and an error made in one push
    # decays by (1 - alpha) per push: at most 2000 u / alpha relative.
    csr = _repeated_arc_csr(ops, 300, 2000)
    ppr, _, T, resid = ops.ppr_matrix(csr, [0, 5], tol=1e-6, check_residual=True)
    est, _, T_o, _, _ = oracle_ppr(synth.build_graph(2, [0], [1]), [0], T=T)
    p = ppr.double().cpu().numpy()
    rel = 2000 * 2.0 ** -24 / ALPHA
    print(f"[resident repeated arcs] err {abs(p[0, 0] - est[0, 0]):.3e} {abs(p[0, 1] - est[0, 1]):.3e} "
          f"bound {rel * est[0, 0]:.3e}", flush=True)
    assert abs(p[0, 0] - est[0, 0]) <= rel * est[0, 0] and abs(p[0, 1] - est[0, 1]) <= rel * est[0, 1]
    assert np.abs(p[0, 2:]).max() == 0.0
    assert abs(p[1, 5] - (1 - (1 - ALPHA) ** T)) <= 1e-6
    assert np.abs(resid - (1 - ALPHA) ** T).max() <= 2e-6 + rel


def test_resident_repeated_arcs_flagged(ops):
    # with 5000 repeated arcs per row the padded first group would exceed the
    # reserved region: the layout reports it through NaN outputs
    csr = _repeated_arc_csr(ops, 300, 5000)
    from paper_2112_14944_amd._lib import PPR_ENONFINITE, PprvizError
    with pytest.raises(PprvizError) as ei:
        ops.ppr_matrix(csr, [0, 5], tol=1e-6, check_residual=True)
    assert ei.value.status == PPR_ENONFINITE
    ppr, _, _, _ = ops.ppr_matrix(csr, [0, 5], tol=1e-6)
    assert torch.isnan(ppr).all().item()


def test_degenerate_cases(ops):
    # single isolated node; two-node path (closed form 1/(2 - alpha)); T = 0; T = 1; no sources
    g1 = synth.build_graph(1, [], [])
    ppr, dppr, T, _ = ops.ppr_matrix(_csr(ops, g1), [0], tol=1e-6)
    assert abs(ppr.item() - (1 - (1 - ALPHA) ** T)) < 1e-6 and dppr.item() == 0.0
    g2 = synth.build_graph(2, [0], [1])
    ppr, dppr, T, _ = ops.ppr_matrix(_csr(ops, g2), [0, 1], tol=1e-12)
    assert abs(ppr[0, 0].item() - 1 / (2 - ALPHA)) < 1e-6
    assert abs(ppr[1, 0].item() - (1 - ALPHA) / (2 - ALPHA)) < 1e-6
    g = synth.erdos_renyi(40, 4, 9)
    p0, _, T0, _ = ops.ppr_matrix(_csr(ops, g), [1, 2], tol=2.0)
    assert T0 == 0 and p0.abs().max().item() == 0.0
    p1, _, T1, _ = ops.ppr_matrix(_csr(ops, g), [1, 2], tol=0.0, max_iter=1)
    assert T1 == 1 and abs(p1[0, 1].item() - ALPHA) < 1e-7 and abs(p1.sum().item() - 2 * ALPHA) < 1e-6
    pe, _, _, _ = ops.ppr_matrix(_csr(ops, g), np.zeros(0, dtype=np.int32), tol=1e-6)
    assert pe.shape == (0, 40)
    # iteration cap before the tolerance: ENOCONV, outputs still written
    from paper_2112_14944_amd._lib import PprvizError
    with pytest.raises(PprvizError):
        ops.ppr_matrix(_csr(ops, g), [1], tol=1e-9, max_iter=5)
    pc, _, Tc, _ = ops.ppr_matrix(_csr(ops, g), [1], tol=1e-9, max_iter=5, allow_noconv=True)
    est, _, _, _, _ = oracle_ppr(g, [1], T=5)
    assert Tc == 5 and np.abs(pc.double().cpu().numpy() - est).max() <= 1e-6


def test_nonfinite_weights_reported(ops):
    g = synth.sbm(synth.equal_blocks(60, 3), 0.3, 0.05, 3, weighted=(0.5, 2.0, 4))
    csr = _csr(ops, g)
    w = csr.weight.clone()
    w[5] = float("nan")
    from paper_2112_14944_amd._lib import PPR_ENONFINITE, PprvizError
    with pytest.raises(PprvizError) as ei:
        ops.ppr_matrix(csr.with_weight(w), np.arange(60), tol=1e-6, check_residual=True)
    assert ei.value.status == PPR_ENONFINITE


def test_chung_lu_20000_all_pairs_sampled(ops):
    # Chung-Lu n=20000, gamma 2.5, mean degree 20, all 20000 sources to L1
    # residual 1e-7 (T = 100): full FP32 n x n output; the oracle checks 48
    # sources (the 8 of highest degree, where pi_d(s, s) >= alpha d(s) is
    # largest, and 40 seeded others), their PDist block, the first and the
    # 500th Jacobi sweep of those 48 rows of the full-size layout, and the
    # stress trend over the 500 sweeps.
    g = synth.chung_lu(20000, 2.5, 20, synth.BASE_SEED + 2)
    n = g.n
    print(f"[chung-lu n=20000] n={n} nnz={g.nnz}", flush=True)
    csr = _csr(ops, g)
    ppr, dppr, T, resid = ops.ppr_matrix(csr, np.arange(n), tol=1e-7, check_residual=True)
    assert T == 100
    assert np.abs(resid - (1 - ALPHA) ** 100).max() <= 2e-6
    deg = np.diff(g.row_ptr)
    hubs = np.argsort(-deg, kind="stable")[:8]
    rnd = synth.random_sources(g, 48, 31)
    sample = np.concatenate([hubs, rnd[~np.isin(rnd, hubs)][:40]]).astype(np.int32)
    assert len(sample) == 48 and deg[sample[:8]].min() >= deg.max() // 2
    est, dppr_o, _, _, d = oracle_ppr(g, sample, tol=1e-7)
    sidx = torch.as_tensor(sample, device="cuda").long()
    assert_ppr_close(ppr[sidx], dppr[sidx], est, dppr_o, d[sample])
    del ppr
    delta = ops.pdist(dppr, n)
    blk = delta[sidx][:, sidx].double().cpu().numpy()
    D_blk = O.pdist(dppr_o[:, sample], n)
    assert rel_err(blk, D_blk) <= PDIST_REL
    # full-size layout step on sampled rows.  The oracle's Delta row i needs
    # pi_d(j, i) for every j; for an undirected graph it equals pi_d(i, j)
    # (reversibility, pinned in the oracle tests), so row i follows from the
    # oracle's own PPR row of source i.
    x0 = torch.as_tensor(synth.uniform_layout(n, 41), device="cuda")
    x1, st = ops.layout_step(delta, x0, with_stress=True)
    Drows = O.pdist_of_z(2.0 * dppr_o, n)
    Drows[np.arange(len(sample)), sample] = 0.0
    X0 = x0.double().cpu().numpy()
    want = O.jacobi_rows(X0, Drows, sample)
    got = x1[sidx].double().cpu().numpy()
    assert np.abs(got - want).max() <= STEP_REL * np.abs(X0).max()
    assert st.item() > 0 and np.isfinite(st.item())
    # the workload's 500 sweeps: the stress of every 50th layout does not rise,
    # and the 500th sweep, taken from the GPU's 499th layout, matches the
    # oracle's Jacobi step on the sampled rows
    x = x1
    trend = [st.item()]
    for done in range(1, 499, 50):
        x = ops.layout(delta, x, min(50, 499 - done))
        trend.append(ops.stress_eval(delta, x).item())
    x499 = x
    x500 = ops.layout(delta, x499, 1)
    trend.append(ops.stress_eval(delta, x500).item())
    print(f"[chung-lu n=20000] stress every 50 sweeps: {[round(t, 1) for t in trend]}", flush=True)
    assert all(b <= a * (1 + 1e-6) for a, b in zip(trend, trend[1:])), trend
    X499 = x499.double().cpu().numpy()
    want500 = O.jacobi_rows(X499, Drows, sample)
    got500 = x500[sidx].double().cpu().numpy()
    assert np.abs(got500 - want500).max() <= STEP_REL * np.abs(X499).max()
