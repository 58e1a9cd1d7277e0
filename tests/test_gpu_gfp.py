"""GPU parity: level-l DPPR by Group Forward-Push in rounds (gfp_level_dppr),
through the C ABI, against the FP64 oracle.

With r_max = 0 the rounds are the truncated power series, a unique result,
compared element by element.  With r_max > 0 the order of pushes is free
(several results are correct), so the GPU result is checked for what defines
a valid one: the invariant of Lemma lem:fwdpushag with the exact inverse,
the stopping rule, the error bound of Lemma lem:fpsn-correct, and (at any
size) conservation of residue plus estimate."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import ALPHA, get_ops

pytestmark = pytest.mark.gpu

# FP32 rounds against FP64, relative to the largest value.  Every push adds
# nonnegative terms, so each round leaves each entry within about one unit
# roundoff u = 2^-24 of its value on top of the error it carried in; after
# T rounds the entries are within about T u.  The cases here run up to
# T = 86 rounds: 2 T u = 1.0e-5 (the largest ratio measured on MI355X over
# these tests is 4.7e-6).
REL = 1e-5
WORST = [0.0]


def _within_rel(err, scale):
    """err <= REL * scale; keeps the largest ratio err / scale seen."""
    ratio = float(err) / max(float(scale), 1e-300)
    WORST[0] = max(WORST[0], ratio)
    print(f"[gfp rel] {ratio:.3e} (worst so far {WORST[0]:.3e})", flush=True)
    assert ratio <= REL, ratio


@pytest.fixture(scope="module")
def ops():
    return get_ops()


def _blocks(sizes):
    starts = np.concatenate([[0], np.cumsum(sizes)])
    return [np.arange(starts[b], starts[b + 1]) for b in range(len(sizes))]


def _ragged(n, k, seed):
    """k leaf sets of ragged sizes (1 .. 2n/k) over a random part of V."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    sizes = rng.integers(1, max(2, 2 * n // k), size=k)
    sizes = np.minimum(sizes, n // k)
    sizes[0] = 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    return [np.sort(perm[starts[i]:starts[i + 1]]) for i in range(k)]


def _case(n, blocks, weighted, seed):
    wt = (0.5, 2.0, seed + 1) if weighted else None
    sizes = synth.equal_blocks(n, blocks)
    g = synth.sbm(sizes, min(1.0, 12.0 / (n / blocks)), 2.0 / n, seed, weighted=wt)
    return g, _blocks(sizes)


def _exact(g):
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    return W, O.ppr_closed_form(O.transition(W), ALPHA) * d[:, None], d


@pytest.mark.parametrize("n,blocks,k_ragged,weighted", [(600, 6, 0, False), (601, 5, 40, True), (97, 3, 0, False),
                                                      (1203, 4, 70, False)])
def test_zero_threshold_is_the_truncated_series(ops, n, blocks, k_ragged, weighted):
    g, leaves = _case(n, blocks, weighted, synth.BASE_SEED + n)
    if k_ragged:
        leaves = _ragged(n, k_ragged, synth.BASE_SEED + 3)  # two or three slabs of columns
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    P = O.transition(W)
    csr = ops.Csr.from_graph(g, "cuda")
    for T in (1, 2, 17, 86):
        print(f"[gfp zero] n={n} k={len(leaves)} T={T}", flush=True)
        out, est, resid, rounds, st = ops.gfp_level_dppr(csr, leaves, ALPHA, 0.0, T, want_est=True,
                                                          want_resid=True, allow_noconv=True)
        assert rounds == T
        ppr, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        want = O.level_dppr(ppr * d[:, None], leaves)
        got = out.double().cpu().numpy()
        _within_rel(np.abs(got - want).max(), np.abs(want).max())
        e_o, R_o, ne_o, r_o, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, T)
        _within_rel(np.abs(est.double().cpu().numpy() - ne_o).max(), np.abs(ne_o).max())
        _within_rel(np.abs(resid.double().cpu().numpy() - R_o).max(), max(np.abs(R_o).max(), 1e-30))


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("r_max", [1e-3, 1e-5, 1e-7])
def test_threshold_result_is_valid(ops, weighted, r_max):
    g, leaves = _case(1500, 8, weighted, synth.BASE_SEED + 17)
    W, pi_d, d = _exact(g)
    L = O.level_dppr(pi_d, leaves)
    csr = ops.Csr.from_graph(g, "cuda")
    print(f"[gfp valid] weighted={weighted} r_max={r_max}", flush=True)
    out, est, resid, rounds, st = ops.gfp_level_dppr(csr, leaves, ALPHA, r_max, 10000, want_est=True,
                                                      want_resid=True)
    got = out.double().cpu().numpy()
    R = resid.double().cpu().numpy()
    E = est.double().cpu().numpy()
    # stopping rule (the GPU takes it in FP32)
    assert np.all(R <= d[None, :] * r_max * (1 + 1e-5))
    # the k x k output aggregates the per-node estimates
    agg = np.stack([E[:, F].sum(axis=1) / len(F) for F in leaves], axis=1)
    assert np.abs(got - agg).max() <= 1e-6 * np.abs(agg).max()
    # invariant: estimate + error term = exact level-l DPPR
    err = O.gfp_error_term(pi_d, leaves, R, d)
    _within_rel(np.abs(got + err - L).max(), np.abs(L).max())
    # error bound of Lemma lem:fpsn-correct (undirected: r_max * mean degree)
    bound = r_max * np.array([d[F].mean() for F in leaves])
    gap = L - got
    tol = REL * np.abs(L).max()
    assert np.all(gap >= -tol) and np.all(gap <= bound[None, :] + tol)
    # the FP64 rounds oracle lands within the same bound
    e_o, _, _, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, r_max, 10000)
    assert np.all(np.abs(got - e_o) <= bound[None, :] + tol)


@pytest.mark.parametrize("weighted", [False, True])
def test_rows_gathered_by_a_whole_wave(ops, weighted):
    # Chung-Lu n = 4000, exponent 2.0, mean degree 60: 180 rows have more
    # than 256 arcs (up to 456) and take the whole-wave gather; ragged
    # supernodes over a random part of V.
    g0 = synth.chung_lu(4000, 2.0, 60, synth.BASE_SEED + 41)
    w = None
    if weighted:
        w = np.random.default_rng(synth.BASE_SEED + 42).uniform(0.5, 2.0, g0.m_und).astype(np.float32)
    g = synth.build_graph(g0.n, g0.eu, g0.ev, w)
    assert (np.diff(g.row_ptr) > 256).sum() > 100
    leaves = _ragged(g.n, 12, synth.BASE_SEED + 43)
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    csr = ops.Csr.from_graph(g, "cuda")
    P = O.transition(W)
    for T in (1, 7, 30):
        print(f"[gfp wide zero] weighted={weighted} T={T}", flush=True)
        out, est, _, rounds, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, 0.0, T, want_est=True, allow_noconv=True)
        ppr, _, _ = O.ppr_power_iteration(P, np.arange(g.n), ALPHA, fixed_iters=T)
        want = O.level_dppr(ppr * d[:, None], leaves)
        _within_rel(np.abs(out.double().cpu().numpy() - want).max(), np.abs(want).max())
        _, _, ne_o, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, T)
        _within_rel(np.abs(est.double().cpu().numpy() - ne_o).max(), np.abs(ne_o).max())
    r_max = 1e-6
    print(f"[gfp wide valid] weighted={weighted}", flush=True)
    out, _, resid, _, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, r_max, 10000, want_resid=True)
    pi_d = O.ppr_closed_form(P, ALPHA) * d[:, None]
    L = O.level_dppr(pi_d, leaves)
    R = resid.double().cpu().numpy()
    got = out.double().cpu().numpy()
    assert np.all(R <= d[None, :] * r_max * (1 + 1e-5))
    err = O.gfp_error_term(pi_d, leaves, R, d)
    _within_rel(np.abs(got + err - L).max(), np.abs(L).max())
    bound = r_max * np.array([d[F].mean() for F in leaves])
    tol = REL * np.abs(L).max()
    assert np.all(L - got >= -tol) and np.all(L - got <= bound[None, :] + tol)


def test_round_cap_keeps_the_invariant(ops):
    g, leaves = _case(700, 4, False, synth.BASE_SEED + 23)
    W, pi_d, d = _exact(g)
    L = O.level_dppr(pi_d, leaves)
    csr = ops.Csr.from_graph(g, "cuda")
    for cap in (1, 3):
        print(f"[gfp cap] cap={cap}", flush=True)
        out, est, resid, rounds, st = ops.gfp_level_dppr(csr, leaves, ALPHA, 1e-9, cap, want_resid=True,
                                                          allow_noconv=True)
        from paper_2112_14944_amd import _lib
        assert st == _lib.PPR_ENOCONV and rounds == cap
        err = O.gfp_error_term(pi_d, leaves, resid.double().cpu().numpy(), d)
        _within_rel(np.abs(out.double().cpu().numpy() + err - L).max(), np.abs(L).max())
        e_o, R_o, _, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 1e-9, cap)
        _within_rel(np.abs(out.double().cpu().numpy() - e_o).max(), np.abs(e_o).max())


def test_isolated_leaves_and_outside_nodes(ops):
    # isolated nodes in a leaf set start with zero residue; nodes outside S
    # carry residue but contribute no estimate
    n = 300
    g0, _ = _case(n, 3, False, synth.BASE_SEED + 29)
    keep = (g0.eu < n - 5) & (g0.ev < n - 5)
    g = synth.build_graph(n, g0.eu[keep], g0.ev[keep])
    leaves = [np.arange(0, 50), np.arange(100, 140), np.arange(n - 10, n)]
    W, pi_d, d = _exact(g)
    L = O.level_dppr(pi_d, leaves)
    csr = ops.Csr.from_graph(g, "cuda")
    out, est, resid, rounds, st = ops.gfp_level_dppr(csr, leaves, ALPHA, 1e-6, 10000, want_resid=True)
    R = resid.double().cpu().numpy()
    assert np.all(R[:, n - 5:] == 0)
    got = out.double().cpu().numpy()
    err = O.gfp_error_term(pi_d, leaves, R, d)
    _within_rel(np.abs(got + err - L).max(), np.abs(L).max())


def test_invalid_leaf_lists_are_rejected(ops):
    from paper_2112_14944_amd import _lib
    g, _ = _case(200, 2, False, synth.BASE_SEED + 31)
    csr = ops.Csr.from_graph(g, "cuda")
    bad = [
        (np.array([0, 3, 3], np.int32), np.array([1, 2, 3], np.int32)),        # empty set
        (np.array([0, 2, 3], np.int32), np.array([1, 200, 3], np.int32)),      # id out of range
        (np.array([0, 2, 3], np.int32), np.array([1, -1, 3], np.int32)),       # negative id
        (np.array([1, 2, 3], np.int32), np.array([1, 2, 3], np.int32)),        # leaf_ptr[0] != 0
        (np.array([0, 3, 2, 3], np.int32), np.array([1, 2, 3], np.int32)),     # decreasing
    ]
    for ptr, idx in bad:
        with pytest.raises(_lib.PprvizError) as ei:
            ops.gfp_level_dppr(csr, (ptr, idx), ALPHA, 1e-6, 100)
        assert ei.value.status == _lib.PPR_EINVAL


def test_full_size_partition_of_a_million_nodes(ops):
    # Chung-Lu n = 10^6, exponent 2.2, mean degree 30; 25 supernodes that
    # partition V into contiguous id ranges (standing in for the top level of
    # a hierarchy); the paper's defaults eps = 1 - 1/e, delta = 1/(10k),
    # tau = 1/sqrt(kn) give r_max by Eq. eq:rmax, with m = nnz.
    n, k = 1_000_000, 25
    g = synth.chung_lu(n, 2.2, 30, synth.BASE_SEED + 4)
    leaves = _blocks(synth.equal_blocks(n, k))
    r_max = O.rmax_forward(1 - 1 / np.e, 1 / (10 * k), g.nnz, O.tau_default(k, n))
    print(f"[gfp full] n={n} nnz={g.nnz} k={k} r_max={r_max:.3e}", flush=True)
    csr = ops.Csr.from_graph(g, "cuda")
    out, est, resid, rounds, st = ops.gfp_level_dppr(csr, leaves, ALPHA, r_max, 10000, want_est=True,
                                                      want_resid=True)
    torch.cuda.synchronize()
    print(f"[gfp full] rounds={rounds}", flush=True)
    W = O.weight_matrix(n, g.eu, g.ev)
    d = O.degrees(W)
    R = resid.double().cpu().numpy()
    E = est.double().cpu().numpy()
    got = out.double().cpu().numpy()
    # stopping rule and conservation: each push moves alpha r into the
    # estimate and (1 - alpha) r to the neighbours, so residue + estimate
    # keeps the seeds' total mean degree of F(V_i)
    assert np.all(R <= d[None, :] * r_max * (1 + 1e-5))
    mass = R.sum(axis=1) + E.sum(axis=1)
    want_mass = np.array([d[F].mean() for F in leaves])
    assert np.abs(mass - want_mass).max() <= 1e-4 * want_mass.max()
    # against the FP64 rounds oracle: both stop within the error bound
    e_o, R_o, _, rounds_o, _ = O.group_forward_push_rounds(W, leaves, ALPHA, r_max, 10000)
    print(f"[gfp full] oracle rounds={rounds_o}", flush=True)
    bound = r_max * np.array([d[F].mean() for F in leaves])
    tol = 1e-5 * np.abs(e_o).max()
    assert np.all(np.abs(got - e_o) <= bound[None, :] + tol)
    # an undirected graph's exact level-l DPPR is symmetric: the estimate is
    # within the bound of being so
    assert np.all(np.abs(got - got.T) <= np.maximum(bound[None, :], bound[:, None]) + tol)


# ------------------------------------------------ backward push and Tau-Push


def _exact_ppr(g):
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    ppr = O.ppr_closed_form(O.transition(W), ALPHA)
    return W, ppr, ppr * d[:, None], d


@pytest.mark.parametrize("n,blocks,k_ragged,weighted", [(600, 6, 0, False), (601, 5, 40, True)])
def test_backward_zero_threshold_is_the_truncated_series(ops, n, blocks, k_ragged, weighted):
    g, leaves = _case(n, blocks, weighted, synth.BASE_SEED + n + 1)
    if k_ragged:
        leaves = _ragged(n, k_ragged, synth.BASE_SEED + 4)
    k = len(leaves)
    targets = list(range(0, k, 2)) + ([k - 1] if (k - 1) % 2 else [])
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    P = O.transition(W)
    csr = ops.Csr.from_graph(g, "cuda")
    for T in (1, 3, 40):
        print(f"[gbp zero] n={n} k={k} targets={len(targets)} T={T}", flush=True)
        out, est, resid, rounds, _ = ops.gbp_level_dppr(csr, leaves, targets, 0.0, ALPHA, T, want_est=True,
                                                         want_resid=True, allow_noconv=True)
        assert rounds == T
        ppr_T, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        want = O.level_dppr(ppr_T * d[:, None], leaves)[:, targets]
        got = out.double().cpu().numpy()
        _within_rel(np.abs(got[:, targets] - want).max(), np.abs(want).max())
        others = [j for j in range(k) if j not in targets]
        assert np.all(got[:, others] == 0)  # untouched columns of the zeroed output
        e_o, R_o, ne_o, _, _ = O.group_backward_push_rounds(W, leaves, targets, ALPHA, 0.0, T)
        _within_rel(np.abs(est.double().cpu().numpy() - ne_o).max(), np.abs(ne_o).max())
        _within_rel(np.abs(resid.double().cpu().numpy() - R_o).max(), max(np.abs(R_o).max(), 1e-30))


@pytest.mark.parametrize("weighted", [False, True])
def test_backward_result_is_valid(ops, weighted):
    g, leaves = _case(1500, 8, weighted, synth.BASE_SEED + 19)
    W, ppr, pi_d, d = _exact_ppr(g)
    L = O.level_dppr(pi_d, leaves)
    targets = [1, 4, 6]
    th = np.array([1e-3, 1e-5, 1e-7])
    csr = ops.Csr.from_graph(g, "cuda")
    out, _, resid, _, _ = ops.gbp_level_dppr(csr, leaves, targets, th, ALPHA, 10000, want_resid=True)
    got = out.double().cpu().numpy()[:, targets]
    R = resid.double().cpu().numpy()
    assert np.all(R <= th.astype(np.float32).astype(np.float64)[:, None] * (1 + 1e-6))
    err = O.gbp_error_term(ppr, leaves, targets, R, d)
    _within_rel(np.abs(got + err - L[:, targets]).max(), np.abs(L).max())
    means = np.array([d[F].mean() for F in leaves])
    bound = means[:, None] * th[None, :]
    tol = REL * np.abs(L).max()
    gap = L[:, targets] - got
    assert np.all(gap >= -tol) and np.all(gap <= bound + tol)
    e_o, _, _, _, _ = O.group_backward_push_rounds(W, leaves, targets, ALPHA, th, 10000)
    assert np.all(np.abs(got - e_o) <= bound + tol)


def test_invalid_backward_targets_are_rejected(ops):
    from paper_2112_14944_amd import _lib
    g, leaves = _case(200, 2, False, synth.BASE_SEED + 37)
    csr = ops.Csr.from_graph(g, "cuda")
    with pytest.raises(_lib.PprvizError) as ei:
        ops.gbp_level_dppr(csr, leaves, [0, 2], 1e-6, ALPHA, 100)
    assert ei.value.status == _lib.PPR_EINVAL


@pytest.mark.parametrize("forced_tau", [True, False])
def test_tau_push_within_eps_delta(ops, forced_tau):
    # 90-node SBM, 6 blocks: with tau at the median DNPR half the targets are
    # refined backward; with the paper's tau = 1/sqrt(kn) the choice follows
    # the graph.  Every off-diagonal estimate lies within eps*delta below the
    # exact level-l DPPR, and the refined set matches the oracle's.
    g, leaves = _case(90, 6, False, synth.BASE_SEED + 41)
    W, ppr, pi_d, d = _exact_ppr(g)
    L = O.level_dppr(pi_d, leaves)
    k = len(leaves)
    eps, delta = 1 - 1 / np.e, 1 / (10 * k)
    tau_j = np.array([d[F].mean() / g.nnz for F in leaves])
    tau = float(np.median(tau_j)) if forced_tau else 0.0
    csr = ops.Csr.from_graph(g, "cuda")
    out, nb, rounds, _ = ops.tau_push_level_dppr(csr, leaves, ALPHA, eps, delta, tau)
    est_o, targets, tau_o = O.tau_push(W, leaves, ALPHA, eps, delta, tau=tau if forced_tau else None)
    assert nb == len(targets)
    if forced_tau:
        assert 0 < nb < k
    got = out.double().cpu().numpy()
    off = ~np.eye(k, dtype=bool)
    tol = REL * np.abs(L).max()
    gap = (L - got)[off]
    assert np.all(gap >= -tol) and np.all(gap <= eps * delta + tol)
    assert np.all(np.abs(got - est_o)[off] <= eps * delta + tol)


def test_tau_push_refines_hub_supernodes_of_a_power_law_graph(ops):
    # Chung-Lu n = 20000 (exponent 2.5, mean degree 20); 25 singleton
    # supernodes at the 25 largest degrees: with the paper's tau = 1/sqrt(kn)
    # the hubs whose DNPR d/m exceeds tau are refined backward.
    g = synth.chung_lu(20000, 2.5, 20, synth.BASE_SEED + 2)
    d = np.diff(g.row_ptr).astype(np.float64)
    hubs = np.argsort(-d, kind="stable")[:25]
    leaves = [np.array([h]) for h in hubs]
    k = len(leaves)
    tau = 1 / np.sqrt(k * g.n)
    expect = int((d[hubs] / g.nnz > tau).sum())
    csr = ops.Csr.from_graph(g, "cuda")
    eps, delta = 1 - 1 / np.e, 1 / (10 * k)
    out, nb, rounds, _ = ops.tau_push_level_dppr(csr, leaves, ALPHA, eps, delta)
    assert nb == expect
    W = O.weight_matrix(g.n, g.eu, g.ev)
    est_o, targets, _ = O.tau_push(W, leaves, ALPHA, eps, delta)
    assert len(targets) == expect
    got = out.double().cpu().numpy()
    off = ~np.eye(k, dtype=bool)
    # both within eps*delta below the exact values, so within eps*delta of each other
    assert np.all(np.abs(got - est_o)[off] <= eps * delta * (1 + 1e-4) + 1e-6 * np.abs(est_o).max())


def test_degenerate_single_supernode(ops):
    # k = 1: the level-l DPPR of a supernode with itself; forward rounds at
    # r_max = 0 against the truncated series, and Tau-Push keeps the forward
    # value (no other supernode for Eq. eq:brmax)
    g, _ = _case(300, 3, False, synth.BASE_SEED + 43)
    leaves = [np.arange(0, 300)]
    W = O.weight_matrix(g.n, g.eu, g.ev)
    csr = ops.Csr.from_graph(g, "cuda")
    out, _, _, rounds, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, 0.0, 9, allow_noconv=True)
    e_o, _, _, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, 9)
    assert out.shape == (1, 1) and rounds == 9
    assert abs(out.item() - e_o[0, 0]) <= REL * abs(e_o[0, 0])
    tout, nb, _, _ = ops.tau_push_level_dppr(csr, leaves, ALPHA, 0.5, 0.05, tau=1e-12)
    t_o, targets, _ = O.tau_push(W, leaves, ALPHA, 0.5, 0.05, tau=1e-12)
    assert nb == 0 and targets == []
    assert abs(tout.item() - t_o[0, 0]) <= REL * abs(t_o[0, 0])


def test_overlapping_and_repeated_leaves(ops):
    # leaf lists that share a node and list a node twice: every formula reads
    # F(V_i) as the given list, so the repeated node counts twice
    g, _ = _case(200, 2, True, synth.BASE_SEED + 47)
    leaves = [np.array([0, 1, 1, 2, 150]), np.array([2, 3, 4]), np.array([199])]
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    csr = ops.Csr.from_graph(g, "cuda")
    for T in (1, 6):
        out, est, resid, _, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, 0.0, T, want_est=True, want_resid=True,
                                                   allow_noconv=True)
        e_o, R_o, ne_o, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, T)
        _within_rel(np.abs(out.double().cpu().numpy() - e_o).max(), np.abs(e_o).max())
        _within_rel(np.abs(resid.double().cpu().numpy() - R_o).max(), np.abs(R_o).max())
        bo, _, _, _, _ = ops.gbp_level_dppr(csr, leaves, [0, 1, 2], 0.0, ALPHA, T, allow_noconv=True)
        b_o, _, _, _, _ = O.group_backward_push_rounds(W, leaves, [0, 1, 2], ALPHA, 0.0, T)
        _within_rel(np.abs(bo.double().cpu().numpy() - b_o).max(), np.abs(b_o).max())


# ------------------------------------- receive marks (grids of > 8192 blocks)


def _mark_case(weighted=False):
    # SBM n = 10^5 (50 blocks, mean degree ~14, no row over 256 arcs) and
    # k = 70 sets of 2 random leaves: 3 slabs of columns, 9375 blocks per
    # round, so the rounds mark the rows their pushes reach; the pushes
    # spread out from 140 seeds, so rounds 1-3 are under the mark cap.
    n = 100_000
    wt = (0.5, 2.0, synth.BASE_SEED + 73) if weighted else None
    g = synth.sbm(synth.equal_blocks(n, 50), 12.0 / (n / 50), 2.0 / n, synth.BASE_SEED + 71, weighted=wt)
    rng = np.random.default_rng(synth.BASE_SEED + 72)
    leaves = [np.sort(rng.choice(n, 2, replace=False)) for _ in range(70)]
    return g, leaves


@pytest.mark.parametrize("weighted", [False, True])
def test_receive_marks_match_the_truncated_series(ops, weighted):
    # r_max = 0: every round (and the delivery after the round cap) is
    # compared element by element with the FP64 rounds, forward and backward.
    # The same grids switch to flag-free gathers after rounds dense in every
    # block.
    g, leaves = _mark_case(weighted)
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    csr = ops.Csr.from_graph(g, "cuda", weighted=weighted)
    targets = list(range(len(leaves)))
    # from round 4 on every block pushes along nearly all its arcs: rounds 5
    # and up write zeros for the rows that do not push, rounds 6 and up (and
    # the delivery after the cap at T = 8) gather without push flags
    for T in (1, 2, 3, 5, 8):
        print(f"[gfp marks] weighted={weighted} forward T={T}", flush=True)
        out, est, resid, rounds, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, 0.0, T, want_est=True,
                                                         want_resid=True, allow_noconv=True)
        assert rounds == T
        e_o, R_o, ne_o, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, T)
        _within_rel(np.abs(out.double().cpu().numpy() - e_o).max(), np.abs(e_o).max())
        _within_rel(np.abs(est.double().cpu().numpy() - ne_o).max(), np.abs(ne_o).max())
        _within_rel(np.abs(resid.double().cpu().numpy() - R_o).max(), np.abs(R_o).max())
    for T in (2, 4):
        print(f"[gfp marks] weighted={weighted} backward T={T}", flush=True)
        bo, best, bres, rounds, _ = ops.gbp_level_dppr(csr, leaves, targets, 0.0, ALPHA, T, want_est=True,
                                                       want_resid=True, allow_noconv=True)
        assert rounds == T
        b_o, bR_o, bne_o, _, _ = O.group_backward_push_rounds(W, leaves, targets, ALPHA, 0.0, T)
        _within_rel(np.abs(bo.double().cpu().numpy() - b_o).max(), np.abs(b_o).max())
        _within_rel(np.abs(best.double().cpu().numpy() - bne_o).max(), np.abs(bne_o).max())
        _within_rel(np.abs(bres.double().cpu().numpy() - bR_o).max(), np.abs(bR_o).max())


def test_receive_marks_keep_residue_and_stopping_rule(ops):
    # r_max > 0 on the same grid: the late rounds, in which few pairs push,
    # skip the unmarked rows.  A row skipped while it had residue arriving
    # would lose that residue (residue + estimate would fall short of the
    # seeds' mean degree) or leave it above the threshold.
    g, leaves = _mark_case()
    d = O.degrees(O.weight_matrix(g.n, g.eu, g.ev, g.weight))
    csr = ops.Csr.from_graph(g, "cuda")
    for r_max in (1e-5, 1e-7):
        print(f"[gfp marks] r_max={r_max}", flush=True)
        out, est, resid, rounds, _ = ops.gfp_level_dppr(csr, leaves, ALPHA, r_max, 10000, want_est=True,
                                                         want_resid=True)
        R = resid.double().cpu().numpy()
        E = est.double().cpu().numpy()
        assert np.all(R <= d[None, :] * r_max * (1 + 1e-5))
        mass = R.sum(axis=1) + E.sum(axis=1)
        want_mass = np.array([d[F].mean() for F in leaves])
        assert np.abs(mass - want_mass).max() <= 1e-5 * want_mass.max(), rounds
        agg = np.stack([E[:, F].sum(axis=1) / len(F) for F in leaves], axis=1)
        assert np.abs(out.double().cpu().numpy() - agg).max() <= 1e-6 * np.abs(agg).max()
