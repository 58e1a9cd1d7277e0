"""Pins for the level-l DPPR / Group Forward-Push oracle (no GPU).

Each check ties the oracle to something other than itself: a closed form on
the complete graph, symmetry and column sums that reversibility forces on an
undirected graph, the printed first push of the running example, the
invariant of Lemma lem:fwdpushag evaluated with the exact inverse, the
stopping rule and error bound of Lemma lem:fpsn-correct, and the truncated
power series.  A wrong seed (1 / |F| instead of d / |F|), a wrong divisor
(|F(V_i)| instead of |F(V_j)|), a transposed residue product or a dropped
(1 - alpha) fails at least one of them."""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

ALPHA = 0.15


def _pi_d_exact(W):
    P = O.transition(W)
    d = O.degrees(W)
    return O.ppr_closed_form(P, ALPHA) * d[:, None], d


def _sbm_case(seed=11, weighted=False, n=60, blocks=4):
    sizes = synth.equal_blocks(n, blocks)
    wt = (0.5, 2.0, seed + 1) if weighted else None
    g = synth.sbm(sizes, 0.35, 0.04, seed, weighted=wt)
    W = O.weight_matrix(n, g.eu, g.ev, g.weight)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    leaves = [np.arange(starts[b], starts[b + 1]) for b in range(blocks)]
    return W, leaves


def _ragged_leaves(n, seed):
    """Leaf sets of unequal sizes that leave some nodes outside S."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    cuts = [0, 3, 10, 11, 30]
    return [np.sort(perm[cuts[i]:cuts[i + 1]]) for i in range(len(cuts) - 1)]


def _directed_case(seed=21, n=40, p=0.08):
    """A directed graph (the paper's setting) in which every node has an
    out-arc (a cycle through all nodes plus random arcs), so pi_d is not
    symmetric and a transposed operand shows."""
    rng = np.random.default_rng(seed)
    src, dst = np.nonzero(rng.random((n, n)) < p)
    keep = src != dst
    src = np.concatenate([src[keep], np.arange(n)])
    dst = np.concatenate([dst[keep], (np.arange(n) + 1) % n])
    W = O.weight_matrix(n, src, dst, directed=True)
    W.data[:] = 1.0
    return W, _ragged_leaves(n, seed)


def test_level_dppr_complete_graph_closed_form():
    # K_n: pi(s,s) = (alpha+beta)/(1+beta), pi(s,t) = beta/(1+beta), d = n-1.
    n = 9
    eu, ev = np.triu_indices(n, 1)
    W = O.weight_matrix(n, eu, ev)
    pi_d, d = _pi_d_exact(W)
    beta = (1 - ALPHA) / (n - 1)
    a = (ALPHA + beta) / (1 + beta)
    b = beta / (1 + beta)
    leaves = [np.array([0, 1, 2, 3]), np.array([4, 5]), np.array([6])]
    L = O.level_dppr(pi_d, leaves)
    for i, Fi in enumerate(leaves):
        for j, Fj in enumerate(leaves):
            if i == j:
                f = len(Fi)
                want = (n - 1) * (f * a + f * (f - 1) * b) / (f * f)
            else:
                want = (n - 1) * b
            assert abs(L[i, j] - want) < 1e-12


def test_level_dppr_symmetric_and_column_sums():
    # Undirected: pi_d is symmetric, so the level-l matrix is too; and for
    # supernodes partitioning V, sum_i |F_i| L[i, j] = mean of d over F_j.
    for weighted in (False, True):
        W, leaves = _sbm_case(weighted=weighted)
        pi_d, d = _pi_d_exact(W)
        L = O.level_dppr(pi_d, leaves)
        np.testing.assert_allclose(L, L.T, rtol=1e-10, atol=1e-13)
        sizes = np.array([len(F) for F in leaves])
        colsum = (sizes[:, None] * L).sum(axis=0)
        want = np.array([d[F].mean() for F in leaves])
        np.testing.assert_allclose(colsum, want, rtol=1e-10)


def test_level_dppr_singletons_reduce_to_leaf_dppr():
    W, _ = _sbm_case(n=20, blocks=2)
    pi_d, _ = _pi_d_exact(W)
    idx = [3, 7, 12, 19]
    L = O.level_dppr(pi_d, [np.array([v]) for v in idx])
    np.testing.assert_allclose(L, pi_d[np.ix_(idx, idx)], rtol=1e-13)


def test_rmax_and_tau():
    # Eq. eq:rmax with the paper's defaults eps = 1 - 1/e, delta = 1/(10k).
    k, n, m = 25, 10 ** 6, 3 * 10 ** 7
    tau = O.tau_default(k, n)
    assert abs(tau - 2e-4) < 1e-15
    r = O.rmax_forward(1 - 1 / np.e, 1 / (10 * k), m, tau)
    assert abs(r - (1 - 1 / np.e) / (10 * k) / (m * 2e-4)) < 1e-20


def test_first_push_of_the_running_example(golden_dir):
    # Section 3.3's example, with the source as a singleton supernode: the
    # first push turns alpha of d(v0) = 3 into the estimate and sends 0.9 to
    # each out-neighbour.
    ex = json.load(open(os.path.join(golden_dir, "push_example.json")))
    arcs = np.array(ex["second_level"]["arcs"])
    n = ex["second_level"]["n"]
    W = O.weight_matrix(n, arcs[:, 0], arcs[:, 1], directed=True)
    leaves = [np.array([0]), np.array([1]), np.array([2, 3])]
    a = ex["alpha"]
    est, r, pushes = O.group_forward_push(W, leaves, 0, a, 1e-9, max_pushes=1)
    assert pushes == 1
    assert abs(est[0] - ex["after_first_push"]["estimate_source"]) < 1e-12
    for v in (1, 2, 3):
        assert abs(r[v] - ex["after_first_push"]["residue_each_out_neighbour"]) < 1e-12
    assert est[1] == 0 and est[2] == 0 and r[0] == 0


@pytest.mark.parametrize("weighted", [False, True])
def test_group_forward_push_invariant_every_stop(weighted):
    # Eq. eq:fwdpushsn-invariant: level-l DPPR = estimate + error term, after
    # any number of pushes, with pi_d from the exact inverse.
    W, leaves = _sbm_case(weighted=weighted)
    n = W.shape[0]
    leaves = _ragged_leaves(n, 4)
    pi_d, d = _pi_d_exact(W)
    L = O.level_dppr(pi_d, leaves)
    for i in range(len(leaves)):
        for cap in (0, 1, 7, 60, None):
            est, r, _ = O.group_forward_push(W, leaves, i, ALPHA, 1e-4, max_pushes=cap)
            err = O.gfp_error_term(pi_d, leaves, r[None, :], d)[0]
            np.testing.assert_allclose(est + err, L[i], rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("r_max", [1e-2, 1e-4, 1e-7])
def test_group_forward_push_stops_within_bound(r_max):
    # Lemma lem:fpsn-correct: at the stop every r(v) <= d(v) r_max, and the
    # error term is at most r_max / |F_j| sum_{t in F_j} sum_k pi_d(k, t),
    # which is r_max * mean_{t in F_j} d(t) on an undirected graph.
    W, leaves = _sbm_case(seed=12)
    pi_d, d = _pi_d_exact(W)
    L = O.level_dppr(pi_d, leaves)
    bound = r_max * np.array([d[F].mean() for F in leaves])
    for i in range(len(leaves)):
        est, r, _ = O.group_forward_push(W, leaves, i, ALPHA, r_max)
        assert np.all(r <= d * r_max + 1e-18)
        gap = L[i] - est
        assert np.all(gap >= -1e-13)
        assert np.all(gap <= bound * (1 + 1e-9))
    # the bound is not vacuous: a tiny threshold gives the exact values
    for i in range(len(leaves)):
        est, _, _ = O.group_forward_push(W, leaves, i, ALPHA, 1e-15)
        np.testing.assert_allclose(est, L[i], rtol=1e-10)


def test_rounds_with_zero_threshold_are_the_truncated_series():
    # r_max = 0: every node holding residue pushes in every round, so T rounds
    # give alpha sum_{t<T} (1-alpha)^t e P^t, the power iteration at T pushes.
    W, leaves = _sbm_case(seed=13, weighted=True)
    n = W.shape[0]
    leaves = _ragged_leaves(n, 5)
    P = O.transition(W)
    d = O.degrees(W)
    for T in (1, 2, 9, 40):
        ppr, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        want = O.level_dppr(ppr * d[:, None], leaves)
        est, R, node_est, rounds, _ = O.group_forward_push_rounds(W, leaves, ALPHA, 0.0, T)
        assert rounds == T
        np.testing.assert_allclose(est, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("r_max", [1e-3, 1e-6])
def test_rounds_invariant_stop_and_bound(weighted, r_max):
    W, leaves = _sbm_case(seed=14, weighted=weighted, n=80, blocks=5)
    pi_d, d = _pi_d_exact(W)
    L = O.level_dppr(pi_d, leaves)
    est, R, node_est, rounds, active = O.group_forward_push_rounds(W, leaves, ALPHA, r_max, 10 ** 5)
    assert active == 0
    assert np.all(R <= d[None, :] * r_max + 1e-18)
    err = O.gfp_error_term(pi_d, leaves, R, d)
    np.testing.assert_allclose(est + err, L, rtol=1e-11, atol=1e-14)
    bound = r_max * np.array([d[F].mean() for F in leaves])
    gap = L - est
    assert np.all(gap >= -1e-13) and np.all(gap <= bound[None, :] * (1 + 1e-9))
    # one push at a time and in rounds: both within the same bound of each other
    for i in range(len(leaves)):
        seq, _, _ = O.group_forward_push(W, leaves, i, ALPHA, r_max)
        assert np.all(np.abs(seq - est[i]) <= bound * (1 + 1e-9))


def test_rounds_cap_leaves_the_invariant_intact():
    W, leaves = _sbm_case(seed=15)
    pi_d, d = _pi_d_exact(W)
    L = O.level_dppr(pi_d, leaves)
    for cap in (1, 3):
        est, R, _, rounds, active = O.group_forward_push_rounds(W, leaves, ALPHA, 1e-8, cap)
        assert rounds == cap and active > 0
        err = O.gfp_error_term(pi_d, leaves, R, d)
        np.testing.assert_allclose(est + err, L, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("r_max", [1e-3, 1e-12])
def test_directed_graph_invariant_and_limit(r_max):
    # On a directed graph pi_d(s, t) != pi_d(t, s): the invariant and the
    # small-threshold limit check which way every product runs.
    W, leaves = _directed_case()
    pi_d, d = _pi_d_exact(W)
    assert np.abs(pi_d - pi_d.T).max() > 1e-3
    L = O.level_dppr(pi_d, leaves)
    assert np.abs(L - L.T).max() > 1e-4
    est_r, R, _, _, active = O.group_forward_push_rounds(W, leaves, ALPHA, r_max, 10 ** 5)
    assert active == 0
    np.testing.assert_allclose(est_r + O.gfp_error_term(pi_d, leaves, R, d), L, rtol=1e-10, atol=1e-14)
    for i in range(len(leaves)):
        est, r, _ = O.group_forward_push(W, leaves, i, ALPHA, r_max)
        err = O.gfp_error_term(pi_d, leaves, r[None, :], d)[0]
        np.testing.assert_allclose(est + err, L[i], rtol=1e-10, atol=1e-14)
        if r_max < 1e-9:
            np.testing.assert_allclose(est, L[i], rtol=1e-8)


def test_rounds_stop_with_isolated_nodes():
    # An isolated node never holds residue; the strict test r > d r_max (with
    # d = 0) keeps it idle, so the rounds end on their own.
    n = 50
    g = synth.sbm(synth.equal_blocks(n, 2), 0.4, 0.05, 16)
    keep = (g.eu < n - 2) & (g.ev < n - 2)  # nodes n-2, n-1 isolated
    W = O.weight_matrix(n, g.eu[keep], g.ev[keep])
    leaves = [np.arange(0, 20), np.arange(20, n)]  # the second holds both isolated nodes
    est, R, _, rounds, active = O.group_forward_push_rounds(W, leaves, ALPHA, 1e-5, 10 ** 4)
    assert active == 0 and rounds < 10 ** 4
    assert np.all(R[:, n - 2:] == 0)
    pi_d, d = _pi_d_exact(W)
    L = O.level_dppr(pi_d, leaves)
    np.testing.assert_allclose(est + O.gfp_error_term(pi_d, leaves, R, d), L, rtol=1e-10, atol=1e-14)


# ------------------------------------------------- backward push, DNPR, Tau-Push


def _exact_ppr(W):
    P = O.transition(W)
    d = O.degrees(W)
    ppr = O.ppr_closed_form(P, ALPHA)
    return ppr, ppr * d[:, None], d


def test_first_backward_push_of_the_example(golden_dir):
    ex = json.load(open(os.path.join(golden_dir, "backward_push_example.json")))
    arcs = np.array(ex["graph"]["arcs"])
    W = O.weight_matrix(ex["graph"]["n"], arcs[:, 0], arcs[:, 1], directed=True)
    leaves = [np.array([10]), np.array([5]), np.array([6])]
    est, r, pushes = O.group_backward_push(W, leaves, 0, ex["alpha"], 1e-9, max_pushes=1)
    assert pushes == 1 and r[10] == 0
    assert abs(est[0] - ex["after_first_push"]["estimate_target"]) < 1e-12
    for v, want in ex["after_first_push"]["residue"].items():
        assert abs(r[int(v)] - want) < 1e-12
    assert est[1] == 0 and est[2] == 0


@pytest.mark.parametrize("case", ["directed", "weighted"])
def test_backward_push_invariant_every_stop(case):
    # pi_d(V_i, V_j) = estimate + sum_{s in F_i} d(s)/|F_i| sum_k pi(s, k) r(k)
    if case == "directed":
        W, leaves = _directed_case(seed=22)
    else:
        W, leaves = _sbm_case(seed=31, weighted=True)
        leaves = _ragged_leaves(W.shape[0], 6)
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    for j in range(len(leaves)):
        for cap in (0, 1, 9, 80, None):
            est, r, _ = O.group_backward_push(W, leaves, j, ALPHA, 1e-4, max_pushes=cap)
            err = O.gbp_error_term(ppr, leaves, [j], r[None, :], d)[:, 0]
            np.testing.assert_allclose(est + err, L[:, j], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("rb_max", [1e-2, 1e-5])
def test_backward_push_stops_within_bound(rb_max):
    # Lemma lem:bpsn-correct: every r <= rb_max at the stop, and the error of
    # pi_d(V_i, V_j) is at most rb_max * (mean degree of F(V_i))
    W, leaves = _sbm_case(seed=32)
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    bound = rb_max * np.array([d[F].mean() for F in leaves])
    for j in range(len(leaves)):
        est, r, _ = O.group_backward_push(W, leaves, j, ALPHA, rb_max)
        assert np.all(r <= rb_max)
        gap = L[:, j] - est
        assert np.all(gap >= -1e-13) and np.all(gap <= bound * (1 + 1e-9))
    est, _, _ = O.group_backward_push(W, leaves, 1, ALPHA, 1e-15)
    np.testing.assert_allclose(est, L[:, 1], rtol=1e-10)


def test_backward_rounds_zero_threshold_and_invariant():
    W, leaves = _sbm_case(seed=33, weighted=True)
    n = W.shape[0]
    leaves = _ragged_leaves(n, 7)
    P = O.transition(W)
    d = O.degrees(W)
    targets = [0, 2, 3]
    for T in (1, 4, 30):
        ppr_T, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        want = O.level_dppr(ppr_T * d[:, None], leaves)[:, targets]
        est, R, _, rounds, _ = O.group_backward_push_rounds(W, leaves, targets, ALPHA, 0.0, T)
        assert rounds == T
        np.testing.assert_allclose(est, want, rtol=1e-12, atol=1e-15)
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    th = [1e-3, 1e-5, 1e-7]
    est, R, _, _, active = O.group_backward_push_rounds(W, leaves, targets, ALPHA, th, 10 ** 5)
    assert active == 0
    assert np.all(R <= np.array(th)[:, None])
    err = O.gbp_error_term(ppr, leaves, targets, R, d)
    np.testing.assert_allclose(est + err, L[:, targets], rtol=1e-10, atol=1e-14)


def test_backward_rounds_on_a_directed_graph():
    W, leaves = _directed_case(seed=23)
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    targets = [1, 3]
    est, R, _, _, active = O.group_backward_push_rounds(W, leaves, targets, ALPHA, 1e-6, 10 ** 5)
    assert active == 0
    err = O.gbp_error_term(ppr, leaves, targets, R, d)
    np.testing.assert_allclose(est + err, L[:, targets], rtol=1e-10, atol=1e-14)


def test_dnpr_of_an_undirected_graph_is_the_mean_degree_over_m():
    W, leaves = _sbm_case(seed=34, weighted=True)
    leaves = _ragged_leaves(W.shape[0], 8)
    _, pi_d, d = _exact_ppr(W)
    m = W.nnz
    tau = O.dnpr(pi_d, leaves, m)
    np.testing.assert_allclose(tau, [d[F].mean() / m for F in leaves], rtol=1e-10)
    # Eq. eq:brmax: eps delta over the largest mean degree of the other
    # sets (for the set of largest mean degree, the second largest counts)
    means = np.array([d[F].mean() for F in leaves])
    j = int(np.argmax(means))
    rb = O.rmax_backward(0.5, 0.1, d, leaves, j)
    assert abs(rb - 0.05 / np.delete(means, j).max()) < 1e-15
    assert rb > 0.05 / means.max()


def test_tau_push_mixes_both_directions_within_eps_delta():
    W, leaves = _sbm_case(seed=35, n=90, blocks=6)
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    m = W.nnz
    tau_j = np.array([d[F].mean() / m for F in leaves])
    tau = float(np.median(tau_j))  # half the targets refined backward
    eps, delta = 1 - 1 / np.e, 1 / (10 * len(leaves))
    est, targets, _ = O.tau_push(W, leaves, ALPHA, eps, delta, tau=tau)
    assert 0 < len(targets) < len(leaves)
    assert targets == [j for j in range(len(leaves)) if tau_j[j] > tau]
    off = ~np.eye(len(leaves), dtype=bool)
    gap = (L - est)[off]
    assert np.all(gap >= -1e-13) and np.all(gap <= eps * delta)
    # the refined columns are the backward rounds, the rest the forward rounds
    fw, _, _, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, O.rmax_forward(eps, delta, m, tau), 10 ** 5)
    rest = [j for j in range(len(leaves)) if j not in targets]
    np.testing.assert_array_equal(est[:, rest], fw[:, rest])


def test_tau_push_single_supernode_keeps_the_forward_value():
    W, _ = _sbm_case(seed=36, n=40, blocks=2)
    leaves = [np.arange(0, 40)]
    est, targets, _ = O.tau_push(W, leaves, ALPHA, 0.5, 0.05, tau=1e-12)
    assert targets == []
    fw, _, _, _, _ = O.group_forward_push_rounds(W, leaves, ALPHA, O.rmax_forward(0.5, 0.05, W.nnz, 1e-12), 10 ** 5)
    np.testing.assert_array_equal(est, fw)


# ------------------------------------------------------- randomized invariants

from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10 ** 6), n=st.integers(6, 28), k=st.integers(1, 4),
       r_exp=st.integers(2, 9), weighted=st.booleans())
def test_random_graphs_both_directions_keep_their_invariants(seed, n, k, r_exp, weighted):
    # random undirected graphs (possibly with isolated nodes), random leaf
    # lists (possibly overlapping): forward and backward rounds at any
    # threshold satisfy their invariants with the exact inverse
    rng = np.random.default_rng(seed)
    mask = np.triu(rng.random((n, n)) < 0.25, 1)
    eu, ev = np.nonzero(mask)
    w = rng.uniform(0.5, 2.0, eu.size) if weighted else None
    W = O.weight_matrix(n, eu, ev, w)
    leaves = [np.sort(rng.choice(n, size=int(rng.integers(1, n // 2 + 1)), replace=False)) for _ in range(k)]
    ppr, pi_d, d = _exact_ppr(W)
    L = O.level_dppr(pi_d, leaves)
    r_max = 10.0 ** (-r_exp)
    est, R, _, _, active = O.group_forward_push_rounds(W, leaves, ALPHA, r_max, 10 ** 5)
    assert active == 0
    np.testing.assert_allclose(est + O.gfp_error_term(pi_d, leaves, R, d), L, rtol=1e-9, atol=1e-12)
    targets = list(range(k))
    eb, Rb, _, _, active_b = O.group_backward_push_rounds(W, leaves, targets, ALPHA, r_max, 10 ** 5)
    assert active_b == 0
    np.testing.assert_allclose(eb + O.gbp_error_term(ppr, leaves, targets, Rb, d), L, rtol=1e-9, atol=1e-12)
