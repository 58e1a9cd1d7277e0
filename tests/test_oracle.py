"""Pins for the FP64 oracle: closed forms, printed worked values, invariants,
brute force and finite differences.  No GPU.  Each check is chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a wrong log base) fails at least one of them."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

ALPHA = 0.15


def _tiny_weighted(seed=5, n=24, isolated=True):
    g = synth.sbm(synth.equal_blocks(n, 3), 0.5, 0.08, seed, weighted=(0.5, 2.0, seed + 1))
    eu, ev, w = g.eu, g.ev, g.weight
    if isolated:
        keep = (eu != n - 1) & (ev != n - 1)  # make the last node isolated
        eu, ev, w = eu[keep], ev[keep], w[keep]
    return n, eu, ev, w


def _tiny_unit(seed=3, n=30, deg=5.0):
    g = synth.erdos_renyi(n, deg, seed)
    return n, g.eu, g.ev, None


# ----------------------------------------------------------------- PPR

def test_power_iteration_matches_dense_inverse_within_residual():
    for n, eu, ev, w in (_tiny_unit(), _tiny_weighted()):
        W = O.weight_matrix(n, eu, ev, w)
        P = O.transition(W)
        exact = O.ppr_closed_form(P, ALPHA)
        for T in (1, 5, 40, 120):
            est, t, resid = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
            assert t == T
            bound = (1 - ALPHA) ** T
            assert np.abs(est - exact).max() <= bound * (1 + 1e-9)
            # the L1 error of each row is exactly its residue norm
            np.testing.assert_allclose(np.abs(exact - est).sum(1), resid, rtol=1e-9, atol=1e-14)


def test_complete_graph_closed_form():
    # K_n: by symmetry pi(s,s) = a, pi(s,t) = b, a + (n-1) b = 1 and
    # a = alpha + (1-alpha) b  =>  a = (alpha+beta)/(1+beta), beta=(1-alpha)/(n-1)
    n = 6
    eu, ev = np.triu_indices(n, 1)
    P = O.transition(O.weight_matrix(n, eu, ev))
    beta = (1 - ALPHA) / (n - 1)
    a = (ALPHA + beta) / (1 + beta)
    b = beta / (1 + beta)
    assert abs(a - 0.2735042735) < 1e-9 and abs(b - 0.1452991453) < 1e-9
    est, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, tol=1e-15)
    exact = O.ppr_closed_form(P, ALPHA)
    for M in (est, exact):
        np.testing.assert_allclose(np.diag(M), a, atol=1e-13)
        off = M[~np.eye(n, dtype=bool)]
        np.testing.assert_allclose(off, b, atol=1e-13)


def test_two_node_path_closed_form():
    # P_2: a = alpha + (1-alpha)(1-a)  =>  a = 1/(2-alpha)
    P = O.transition(O.weight_matrix(2, [0], [1]))
    est, _, _ = O.ppr_power_iteration(P, [0, 1], ALPHA, tol=1e-15)
    assert abs(est[0, 0] - 1 / (2 - ALPHA)) < 1e-13
    assert abs(est[0, 1] - (1 - ALPHA) / (2 - ALPHA)) < 1e-13
    assert abs(1 / (2 - ALPHA) - 0.5405405405) < 1e-9


def test_random_walk_with_restart_monte_carlo():
    # Section 3.1 definition itself: end point of a walk that stops w.p. alpha
    # at each step and otherwise moves to a random out-neighbour.
    rng = np.random.default_rng(0)
    n = 7
    eu = np.array([0, 0, 1, 2, 2, 3, 4, 5])
    ev = np.array([1, 2, 2, 3, 4, 4, 5, 6])
    w = np.array([1.0, 2.0, 0.5, 1.0, 1.5, 1.0, 1.0, 3.0])
    W = O.weight_matrix(n, eu, ev, w)
    P = O.transition(W)
    est, _, _ = O.ppr_power_iteration(P, [0], ALPHA, tol=1e-14)
    Wd = W.toarray()
    cum = np.cumsum(Wd / Wd.sum(1, keepdims=True), axis=1)
    N = 400_000
    pos = np.zeros(N, dtype=np.int64)
    alive = np.ones(N, dtype=bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        stop = rng.random(idx.size) < ALPHA
        alive[idx[stop]] = False
        mv = idx[~stop]
        u = rng.random(mv.size)
        pos[mv] = (u[:, None] > cum[pos[mv]]).sum(1)
    freq = np.bincount(pos, minlength=n) / N
    sigma = np.sqrt(est[0] * (1 - est[0]) / N)
    assert np.all(np.abs(freq - est[0]) <= 5 * sigma + 1e-12)


def test_mass_conservation_and_residue_norm():
    n, eu, ev, w = _tiny_weighted()
    P = O.transition(O.weight_matrix(n, eu, ev, w))
    for T in (0, 1, 7, 33):
        est, _, resid = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        np.testing.assert_allclose(est.sum(1), 1 - (1 - ALPHA) ** T, atol=1e-13)
        np.testing.assert_allclose(resid, (1 - ALPHA) ** T, rtol=1e-12)


@pytest.mark.parametrize("tol", [1e-6, 1e-7, 1e-10])
def test_stopping_rule_iteration_counts(tol):
    n, eu, ev, w = _tiny_unit()
    P = O.transition(O.weight_matrix(n, eu, ev, w))
    _, T, resid = O.ppr_power_iteration(P, [0, 3], ALPHA, tol=tol)
    # mass conservation: residue after t pushes is (1-alpha)^t exactly
    assert T == math.ceil(math.log(tol) / math.log(1 - ALPHA))
    assert resid.max() <= tol
    assert {1e-6: 86, 1e-7: 100, 1e-10: 142}[tol] == T


def test_dppr_reversible_at_every_truncation():
    # undirected graph: d(s) pi(s,t) = d(t) pi(t,s), at every T
    n, eu, ev, w = _tiny_weighted()
    W = O.weight_matrix(n, eu, ev, w)
    d = O.degrees(W)
    P = O.transition(W)
    for T in (1, 2, 9, 60):
        est, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, fixed_iters=T)
        pid = O.dppr(est, d, np.arange(n))
        np.testing.assert_allclose(pid, pid.T, atol=1e-13)
        # column sums sum_s pi_d(s,t) = d(t) (1 - (1-alpha)^T)
        np.testing.assert_allclose(pid.sum(0), d * (1 - (1 - ALPHA) ** T), atol=1e-12)


def test_total_dppr_mass_is_arc_count():
    # proof of Theorem thm:pprd-nd: sum_{i,j} pi_d(i,j) = sum_i d(i) = m
    n, eu, ev, w = _tiny_unit(seed=11)
    W = O.weight_matrix(n, eu, ev)
    d = O.degrees(W)
    P = O.transition(W)
    est, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, tol=1e-14)
    assert abs(O.dppr(est, d, np.arange(n)).sum() - 2 * len(eu)) < 1e-9


def test_push_worked_example(golden_dir):
    ex = json.load(open(os.path.join(golden_dir, "push_example.json")))
    a = ex["alpha"]
    arcs = np.array(ex["second_level"]["arcs"])
    n = ex["second_level"]["n"]
    W = O.weight_matrix(n, arcs[:, 0], arcs[:, 1], directed=True)
    d = O.degrees(W)
    P = O.transition(W)
    assert d[0] == ex["source_out_degree"]
    est, r = O.forward_push_sync_dppr(P, d, 0, a, 1)
    assert abs(est[0] - ex["after_first_push"]["estimate_source"]) < 1e-12
    np.testing.assert_allclose(r[[1, 2, 3]], ex["after_first_push"]["residue_each_out_neighbour"], atol=1e-12)
    est2, r2 = O.forward_push_sync_dppr(P, d, 0, a, 2)
    for k, v in ex["second_level"]["residue"].items():
        assert abs(r2[int(k)] - v) < 1e-12
    # and the DPPR-unit push agrees with d(s) times the PPR-unit iteration
    e_ppr, _, _ = O.ppr_power_iteration(P, [0], a, fixed_iters=2)
    np.testing.assert_allclose(est2, d[0] * e_ppr[0], atol=1e-14)


def test_forward_push_invariant():
    # Eq. eq:fwd-invariant: pi_d(s,t) = est_d(s,t) + sum_k r(s,k)/d(k) pi_d(k,t)
    n, eu, ev, w = _tiny_weighted(isolated=False)
    W = O.weight_matrix(n, eu, ev, w)
    d = O.degrees(W)
    P = O.transition(W)
    exact_d = O.dppr(O.ppr_closed_form(P, ALPHA), d, np.arange(n))
    for s in (0, 5):
        for T in (0, 1, 4, 25):
            est, r = O.forward_push_sync_dppr(P, d, s, ALPHA, T)
            np.testing.assert_allclose(est + (r / d) @ exact_d, exact_d[s], atol=1e-12)


# ----------------------------------------------------------------- PDist

def test_pdist_special_values_and_range():
    n_clamp = 50
    hi = 2 * math.log(n_clamp)
    # z = e^-2 -> 3 (natural log), z = 1/e -> 2 (lower kink), z = 0 -> 2 ln n
    pid = np.array([[0.0, math.exp(-2) / 2, 0.0, 0.9],
                    [math.exp(-2) / 2, 0.0, math.exp(-1), 0.0],
                    [0.0, 0.0, 0.0, 1e-30],
                    [0.1, 0.0, 0.0, 0.0]])
    D = O.pdist(pid, n_clamp)
    assert abs(D[0, 1] - 3.0) < 1e-12 and abs(D[1, 0] - 3.0) < 1e-12
    assert abs(D[1, 2] - 2.0) < 1e-12           # z = 1/e exactly on the kink
    assert abs(D[0, 2] - hi) < 1e-12            # unreachable
    assert abs(D[2, 3] - hi) < 1e-12            # far below e/n^2
    assert abs(D[0, 3] - 2.0) < 1e-12           # z = 1.0 clamps to 2
    assert np.all(np.diag(D) == 0)
    # asymmetric input: z uses both directions
    pid2 = np.array([[0, 0.02], [0.05, 0]])
    assert abs(O.pdist(pid2, 100)[0, 1] - (1 - math.log(0.07))) < 1e-12


def test_pdist_range_edge_bound_and_nd_bound():
    # proof of Theorem thm:pprd-ulcv: an edge has z >= 2 alpha (1-alpha) w,
    # so Delta_uv <= max(2, 1 - ln(2 alpha (1-alpha) w)); Theorem thm:pprd-nd:
    # ND = sum_{i<j} Delta^-2 <= 0.215 e m + 0.0175 n^2 (needs n >= 15).
    for n, eu, ev, w in (_tiny_unit(n=40, deg=4.0), _tiny_weighted(n=30, isolated=False)):
        W = O.weight_matrix(n, eu, ev, w)
        d = O.degrees(W)
        P = O.transition(W)
        est, _, _ = O.ppr_power_iteration(P, np.arange(n), ALPHA, tol=1e-12)
        D = O.pdist(O.dppr(est, d, np.arange(n)), n)
        off = D[~np.eye(n, dtype=bool)]
        assert off.min() >= 2.0 and off.max() <= 2 * math.log(n) + 1e-12
        np.testing.assert_allclose(D, D.T)
        ww = np.ones(len(eu)) if w is None else w.astype(np.float64)
        bound = np.maximum(2.0, 1.0 - np.log(2 * ALPHA * (1 - ALPHA) * ww))
        assert np.all(D[eu, ev] <= bound + 1e-12)
        m_arcs = 2 * len(eu)
        iu = np.triu_indices(n, 1)
        nd = (1.0 / D[iu] ** 2).sum()
        assert nd <= 0.215 * math.e * m_arcs + 0.0175 * n * n
    # unit weights at alpha = 0.15: every edge within 2.3665
    assert abs(1 - math.log(2 * 0.15 * 0.85) - 2.36649) < 1e-4


def test_pdist_derivative_matches_finite_difference():
    rng = np.random.default_rng(4)
    k, n_clamp = 6, 40
    pid = rng.uniform(0.0005, 0.5, size=(k, k))
    g = O.pdist_dz(pid, n_clamp)
    h = 1e-7
    for i in range(k):
        for j in range(k):
            if i == j:
                continue
            p = pid.copy()
            p[i, j] += h
            m = pid.copy()
            m[i, j] -= h
            fd = (O.pdist(p, n_clamp)[i, j] - O.pdist(m, n_clamp)[i, j]) / (2 * h)
            assert abs(fd - g[i, j]) <= 1e-5 * max(1.0, abs(g[i, j]))


# ----------------------------------------------------------------- stress

def test_stress_vectorised_equals_double_loop_and_planted_zero():
    X = synth.uniform_layout(9, 1).astype(np.float64)
    D = synth.random_distance_matrix(9, 2).astype(np.float64)
    assert abs(O.stress(X, D) - O.stress_bruteforce(X, D)) < 1e-12
    P, Dp = synth.planted_layout_distances(8, 3)
    assert O.stress_bruteforce(P, Dp) < 1e-20
    # scaling the layout by c gives sum (1-c)^2 over pairs
    assert abs(O.stress_bruteforce(2 * P, Dp) - 28) < 1e-9


def _fd_grad(f, X, h=1e-6):
    g = np.zeros_like(X)
    for idx in np.ndindex(*X.shape):
        p = X.copy()
        p[idx] += h
        m = X.copy()
        m[idx] -= h
        g[idx] = (f(p) - f(m)) / (2 * h)
    return g


def test_grad_x_finite_difference_and_invariances():
    X = synth.uniform_layout(10, 5).astype(np.float64)
    D = synth.random_distance_matrix(10, 6).astype(np.float64)
    g = O.grad_x(X, D)
    fd = _fd_grad(lambda Y: O.stress_bruteforce(Y, D), X)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(g.sum(0), 0, atol=1e-12)
    assert abs((X[:, 0] * g[:, 1] - X[:, 1] * g[:, 0]).sum()) < 1e-11
    np.testing.assert_allclose(O.grad_x_rows(X, D[[2, 7]], [2, 7]), g[[2, 7]], atol=1e-12)


def test_grad_delta_finite_difference():
    X = synth.uniform_layout(7, 8).astype(np.float64)
    D = synth.random_distance_matrix(7, 9).astype(np.float64)
    g = O.grad_delta_pair(X, D)
    h = 1e-6
    for i in range(7):
        for j in range(i + 1, 7):
            p = D.copy()
            p[i, j] += h
            p[j, i] += h
            m = D.copy()
            m[i, j] -= h
            m[j, i] -= h
            fd = (O.stress_bruteforce(X, p) - O.stress_bruteforce(X, m)) / (2 * h)
            assert abs(fd - g[i, j]) < 1e-7 and g[i, j] == g[j, i]


def test_jacobi_step_identity_with_fd_gradient():
    # X+ = X - grad L / (2 diag L^w), diag L^w_ii = sum_j Delta_ij^-2
    X = synth.uniform_layout(8, 10).astype(np.float64)
    D = synth.random_distance_matrix(8, 11).astype(np.float64)
    fd = _fd_grad(lambda Y: O.stress_bruteforce(Y, D), X)
    diag = np.array([sum(1.0 / D[i, j] ** 2 for j in range(8) if j != i) for i in range(8)])
    expect = X - fd / (2 * diag[:, None])
    np.testing.assert_allclose(O.jacobi_step(X, D), expect, atol=1e-8)
    np.testing.assert_allclose(O.jacobi_rows(X, D[[0, 5]], [0, 5]), expect[[0, 5]], atol=1e-8)
    sr = O.stress_rows(X, D, list(range(8)))
    assert abs(sr.sum() - O.stress_bruteforce(X, D)) < 1e-12


def test_coincident_points_contribute_no_direction():
    X = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 2.0], [-1.5, 0.5]])
    D = synth.random_distance_matrix(4, 12).astype(np.float64)
    Xp = O.jacobi_step(X, D)
    assert np.all(np.isfinite(Xp))
    np.testing.assert_allclose(O.jacobi_rows(X, D[[0]], [0]), Xp[[0]], atol=1e-12)


def test_layout_fixed_points_and_majorization_monotone():
    P, Dp = synth.planted_layout_distances(7, 13)
    np.testing.assert_allclose(O.jacobi_step(P, Dp), P, atol=1e-10)
    Pc = P - P.mean(0)
    np.testing.assert_allclose(O.majorization_step(Pc, Dp), Pc, atol=1e-9)
    np.testing.assert_allclose(O.grad_x(P, Dp), 0, atol=1e-10)
    # majorization never increases stress, and it solves a realizable target
    X = P + np.random.default_rng(0).normal(scale=0.3, size=P.shape)
    s_prev = O.stress(X, Dp)
    for _ in range(200):
        X = O.majorization_step(X, Dp)
        s = O.stress(X, Dp)
        assert s <= s_prev + 1e-12
        s_prev = s
    assert s_prev < 1e-10
    D = synth.random_distance_matrix(12, 14).astype(np.float64)
    X = synth.uniform_layout(12, 15).astype(np.float64)
    s_prev = O.stress(X, D)
    for _ in range(30):
        X = O.majorization_step(X, D)
        s = O.stress(X, D)
        assert s <= s_prev + 1e-12
        s_prev = s


# ----------------------------------------------------------------- weight gradient

def _weighted_small(seed=21, n=14):
    g = synth.sbm(synth.equal_blocks(n, 2), 0.6, 0.15, seed, weighted=(0.5, 2.0, seed + 1))
    return n, g.eu, g.ev, g.weight.astype(np.float64)


def test_weight_gradient_central_difference():
    n, eu, ev, w = _weighted_small()
    X = synth.uniform_layout(n, 22).astype(np.float64) * 3
    iters = 160
    res = O.grad_weights(n, eu, ev, w, X, ALPHA, iters)

    def loss_w(wv):
        return O.pipeline_forward(n, eu, ev, wv, X, ALPHA, iters)["loss"]

    idx = list(range(len(w)))
    fd = O.central_difference(loss_w, w, idx, 1e-6)
    np.testing.assert_allclose(res["grad_w"], fd, rtol=1e-5, atol=1e-8)
    fdx = O.central_difference(lambda xv: O.pipeline_forward(n, eu, ev, w, xv.reshape(-1, 2), ALPHA, iters)["loss"],
                               X.ravel(), list(range(2 * n)), 1e-6)
    np.testing.assert_allclose(res["grad_x"].ravel(), fdx, rtol=1e-6, atol=1e-8)


def test_weight_gradient_with_kink_pairs_frozen():
    # kink_band takes dDelta/dz = 0 for the pairs near a clamp bound: that is
    # the gradient of the loss whose Delta at those pairs does not follow w.
    # A wide band catches several pairs here; the central differences freeze
    # those Delta entries at their unperturbed values.
    n, eu, ev, w = _weighted_small(seed=25, n=14)
    X = synth.uniform_layout(n, 26).astype(np.float64) * 3
    iters = 160
    base = O.pipeline_forward(n, eu, ev, w, X, ALPHA, iters)
    z = base["pi_d"] + base["pi_d"].T
    off = ~np.eye(n, dtype=bool)
    band = float(np.sort(np.abs(1.0 - np.log(z[off]) - 2.0))[10]) + 1e-9
    res = O.grad_weights(n, eu, ev, w, X, ALPHA, iters, kink_band=band)
    kp = res["kink_pairs"]
    assert 3 <= len(kp) < n * (n - 1) // 2 and np.all(kp[:, 0] < kp[:, 1])
    raw = 1.0 - np.log(z[kp[:, 0], kp[:, 1]])
    assert np.all(np.abs(raw - 2.0) < band)
    D0 = base["Delta"]

    def loss_frozen(wv):
        D = O.pipeline_forward(n, eu, ev, wv, X, ALPHA, iters)["Delta"].copy()
        D[kp[:, 0], kp[:, 1]] = D0[kp[:, 0], kp[:, 1]]
        D[kp[:, 1], kp[:, 0]] = D0[kp[:, 1], kp[:, 0]]
        return O.stress(X, D)

    fd = O.central_difference(loss_frozen, w, list(range(len(w))), 1e-6)
    np.testing.assert_allclose(res["grad_w"], fd, rtol=1e-5, atol=1e-8)
    # and it differs from the plain gradient (the frozen pairs did contribute)
    assert np.abs(res["grad_w"] - O.grad_weights(n, eu, ev, w, X, ALPHA, iters)["grad_w"]).max() > 1e-6


def test_weight_gradient_euler_identity():
    # scaling every weight by c keeps P, multiplies pi_d by c and shifts every
    # unclamped Delta by -ln c: sum_e w_e dL/dw_e = -sum_{i<j unclamped} dL/dDelta_ij
    n, eu, ev, w = _weighted_small(seed=31, n=16)
    X = synth.uniform_layout(n, 32).astype(np.float64) * 4
    res = O.grad_weights(n, eu, ev, w, X, ALPHA, 120)
    gD = O.grad_delta_pair(X, res["Delta"])
    inside = O.pdist_dz(res["pi_d"], n) != 0
    iu = np.triu_indices(n, 1)
    rhs = -(gD * inside)[iu].sum()
    assert abs((w * res["grad_w"]).sum() - rhs) <= 1e-10 * max(1.0, abs(rhs))


def test_adjoint_dot_product_and_truncation():
    n, eu, ev, w = _tiny_weighted(seed=41, n=20)
    P = O.transition(O.weight_matrix(n, eu, ev, w))
    rng = np.random.default_rng(1)
    G = rng.normal(size=(n, 3))
    H = rng.normal(size=(n, 3))
    A = O.adjoint_solve(P, ALPHA, G)
    MinvH = O.ppr_closed_form(P, ALPHA) @ H / ALPHA
    assert abs((A * H).sum() - (G * MinvH).sum()) < 1e-10
    for T in (10, 50, 200):
        At = O.adjoint_solve(P, ALPHA, G, iters=T)
        # the truncated tail is ((1-alpha) P^T)^T A, bounded by (1-alpha)^T in L1 per column
        assert np.abs(At - A).sum(0).max() <= (1 - ALPHA) ** T * np.abs(A).sum(0).max() * 1.000001 + 1e-12
