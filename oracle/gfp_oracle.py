"""FP64 CPU oracle for level-l DPPR and the Group Forward-Push (GFP).

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by the test
suite, the smoke check and the benchmark's CPU-baseline leg, never by the HIP
library, and sharing no code with it.

Paper: "Effective and Efficient PageRank-based Positioning for Graph
Visualization" (arXiv 2112.14944), Section 3.2 (multi-level PPR distance,
Definition def:spprdeg) and Section 4 (Tau-Push: Eq. eq:rmax, Algorithm
alg:fwdpushsn, the invariant Eq. eq:fwdpushsn-invariant of Lemma
lem:fwdpushag).

A supernode V_i is given by its leaf set F(V_i), a list of node ids.  The
leaf sets of the k supernodes of S need not cover V (residue flows through
nodes outside S) and may in principle overlap; every formula below is the
paper's with F(V_i) read as the given list.

It also holds the Group Backward-Push (Algorithm alg:bwdpushsn), the DNPR of
Eq. eq:dnpr-dnppr, the backward threshold of Eq. eq:brmax and Tau-Push
(Algorithm alg:taupush).

Pins (tests/test_oracle_gfp.py): the complete-graph closed form, symmetry and
column sums of the level-l DPPR of an undirected graph, the printed first
pushes of Section 3.3's forward example and Section 4.1's backward example,
the forward and backward invariants against the exact inverse at every
stopping point (also on a directed graph), the termination rules, the error
bounds of Lemmas lem:fpsn-correct and lem:bpsn-correct, the power-iteration
series that the rounds of both directions reduce to when the threshold is
zero, the DNPR of an undirected graph against its definition, and Tau-Push's
eps * delta bound.  No function here is "parity unpinned".
"""
from __future__ import annotations

import collections
import math

import numpy as np
import scipy.sparse as sp

from .pprviz_oracle import degrees


def level_dppr(pi_d, leaves):
    """Level-l DPPR between supernodes (Definition def:spprdeg): the mean of the
    leaf-level DPPR pi_d(v_s, v_t) over v_s in F(V_i) and v_t in F(V_j).

    ``pi_d`` is the n x n leaf-level DPPR matrix (rows = sources), ``leaves``
    a list of k index arrays.  Returns the k x k matrix [i, j]."""
    k = len(leaves)
    out = np.zeros((k, k))
    for i, Fi in enumerate(leaves):
        Fi = np.asarray(Fi, dtype=np.int64)
        for j, Fj in enumerate(leaves):
            Fj = np.asarray(Fj, dtype=np.int64)
            out[i, j] = pi_d[np.ix_(Fi, Fj)].sum() / (Fi.size * Fj.size)
    return out


def tau_default(k, n):
    """DNPR threshold tau = 1 / sqrt(k n) (Algorithm alg:taupush, first step)."""
    return 1.0 / math.sqrt(k * n)


def rmax_forward(eps, delta, m, tau):
    """Forward residue threshold r_max = eps * delta / (m * tau) (Eq. eq:rmax)."""
    return eps * delta / (m * tau)


def _arcs(W):
    W = sp.csr_matrix(W)
    return W.indptr, W.indices, W.data


def _seed(d, Fi):
    """Initial residues of a source supernode: d(v) / |F(V_i)| on each leaf v
    (Algorithm alg:fwdpushsn, initialisation)."""
    r = np.zeros(d.shape[0])
    Fi = np.asarray(Fi, dtype=np.int64)
    np.add.at(r, Fi, d[Fi] / Fi.size)
    return r


def group_forward_push(W, leaves, i, alpha, r_max, max_pushes=None):
    """Algorithm alg:fwdpushsn from source supernode V_i, one push at a time.

    While some node v_k holds more residue r than d(v_k) * r_max: r(v_k) is
    set to 0; if v_k is a leaf of a supernode V_j of S, alpha * r / |F(V_j)|
    is added to the estimate pi_d(V_i, V_j) (to every such V_j when leaf sets
    overlap); the other 1 - alpha of r goes to the out-neighbours of v_k in
    proportion to the arc weights (evenly for unit weights).  Nodes are taken
    in first-in first-out order of crossing the threshold (the paper leaves
    the order open).  ``max_pushes`` stops early (the invariant holds after
    every push).

    Returns (estimate over the k supernodes, residue over the n nodes,
    number of pushes)."""
    indptr, indices, data = _arcs(W)
    d = degrees(W)
    n = d.shape[0]
    k = len(leaves)
    member = [[] for _ in range(n)]
    for j, Fj in enumerate(leaves):
        for v in np.asarray(Fj, dtype=np.int64):
            member[int(v)].append(j)
    size = [len(Fj) for Fj in leaves]
    r = _seed(d, leaves[i])
    est = np.zeros(k)
    queue = collections.deque(v for v in range(n) if r[v] > d[v] * r_max)
    queued = np.zeros(n, dtype=bool)
    queued[list(queue)] = True
    pushes = 0
    while queue:
        if max_pushes is not None and pushes >= max_pushes:
            break
        v = queue.popleft()
        queued[v] = False
        if not r[v] > d[v] * r_max:
            continue
        rv = r[v]
        r[v] = 0.0  # cleared first, so that a self-loop's share is kept
        for j in member[v]:
            est[j] += alpha * rv / size[j]
        for e in range(indptr[v], indptr[v + 1]):
            u = indices[e]
            r[u] += (1.0 - alpha) * rv * data[e] / d[v]
            if not queued[u] and r[u] > d[u] * r_max:
                queue.append(u)
                queued[u] = True
        pushes += 1
    return est, r, pushes


def group_forward_push_rounds(W, leaves, alpha, r_max, max_rounds):
    """The same pushes for all k source supernodes at once, in synchronous
    rounds: in each round every (source, node) pair whose residue exceeds
    d(node) * r_max at the start of the round pushes that residue, and what
    a node receives during the round waits for the next one.  Pushing part
    of a node's residue keeps Eq. eq:fwdpushsn-invariant, so the result
    satisfies the invariant, the stopping rule and the error bound of the
    one-at-a-time algorithm; only the order of the pushes differs.  With
    r_max = 0 every node holding residue pushes each round, and T rounds give
    the power-iteration series truncated at T terms.

    Round 0 pushes the seeds without gathering; round t >= 1 first adds what
    round t - 1 sent, then pushes.  Stops after the first round in which no
    pair pushed, or after ``max_rounds`` rounds; in the second case what the
    last round sent is added to the residues before returning, so that the
    invariant holds there too.

    Returns (estimate k x k [i, j], residue k x n, per-node estimate k x n,
    rounds run, pairs pushed in the last round)."""
    d = degrees(W)
    n = d.shape[0]
    k = len(leaves)
    W = sp.csr_matrix(W)
    inv = np.zeros(n)
    nz = d > 0
    inv[nz] = 1.0 / d[nz]
    R = np.stack([_seed(d, Fi) for Fi in leaves]) if k else np.zeros((0, n))
    node_est = np.zeros((k, n))
    sent = np.zeros((k, n))
    rounds = 0
    active = 0
    while rounds < max_rounds:
        if rounds > 0:
            # residue that arrives over arc v -> u is (1 - alpha) r(v) w_vu / d(v)
            R = R + (1.0 - alpha) * np.asarray(sent @ W)
        mask = R > d[None, :] * r_max
        active = int(mask.sum())
        node_est += alpha * np.where(mask, R, 0.0)
        sent = np.where(mask, R, 0.0) * inv[None, :]
        R = np.where(mask, 0.0, R)
        rounds += 1
        if active == 0:
            break
    if active:
        R = R + (1.0 - alpha) * np.asarray(sent @ W)
    est = np.zeros((k, k))
    for j, Fj in enumerate(leaves):
        Fj = np.asarray(Fj, dtype=np.int64)
        est[:, j] = node_est[:, Fj].sum(axis=1) / Fj.size
    return est, R, node_est, rounds, active


def gfp_error_term(pi_d, leaves, R, d):
    """The error term of Eq. eq:fwdpushsn-invariant for every (i, j):
        sum_{v_t in F(V_j)} sum_{v_k} r(V_i, v_k) / (|F(V_j)| d(v_k)) pi_d(v_k, v_t).
    ``R`` is the k x n residue (row i from source V_i).  Nodes with d = 0 hold
    no residue and are skipped."""
    d = np.asarray(d, dtype=np.float64)
    inv = np.zeros_like(d)
    nz = d > 0
    inv[nz] = 1.0 / d[nz]
    k = len(leaves)
    out = np.zeros((k, k))
    Rs = np.asarray(R) * inv[None, :]
    for j, Fj in enumerate(leaves):
        Fj = np.asarray(Fj, dtype=np.int64)
        out[:, j] = (Rs @ pi_d[:, Fj]).sum(axis=1) / Fj.size
    return out


# --------------------------------------------------------------------------
# Group Backward-Push (Algorithm alg:bwdpushsn), DNPR (Eq. eq:dnpr-dnppr) and
# Tau-Push (Algorithm alg:taupush)
# --------------------------------------------------------------------------


def group_backward_push(W, leaves, j, alpha, rb_max, max_pushes=None):
    """Algorithm alg:bwdpushsn towards target supernode V_j, one push at a time.

    Residues r(v) start at 1 / |F(V_j)| on the leaves of V_j.  While some node
    v_k holds more than rb_max: r(v_k) is set to 0; if v_k is a leaf of a
    supernode V_i of S, alpha d(v_k) r / |F(V_i)| is added to the estimate
    pi_d(V_i, V_j); each in-neighbour v_i of v_k receives (1 - alpha) r
    w_ik / d(v_i) (the walk's step probability from v_i to v_k; 1 / d(v_i)
    with unit weights).  FIFO order, as in group_forward_push.

    Returns (estimate over the k source supernodes, residue over the n nodes,
    number of pushes)."""
    W = sp.csr_matrix(W)
    d = degrees(W)
    Wt = sp.csr_matrix(W.T)  # row v_k lists the in-neighbours v_i and w_ik
    indptr, indices, data = Wt.indptr, Wt.indices, Wt.data
    n = d.shape[0]
    k = len(leaves)
    member = [[] for _ in range(n)]
    for i, Fi in enumerate(leaves):
        for v in np.asarray(Fi, dtype=np.int64):
            member[int(v)].append(i)
    size = [len(Fi) for Fi in leaves]
    r = np.zeros(n)
    Fj = np.asarray(leaves[j], dtype=np.int64)
    np.add.at(r, Fj, 1.0 / Fj.size)
    est = np.zeros(k)
    queue = collections.deque(v for v in range(n) if r[v] > rb_max)
    queued = np.zeros(n, dtype=bool)
    queued[list(queue)] = True
    pushes = 0
    while queue:
        if max_pushes is not None and pushes >= max_pushes:
            break
        v = queue.popleft()
        queued[v] = False
        if not r[v] > rb_max:
            continue
        rv = r[v]
        r[v] = 0.0
        for i in member[v]:
            est[i] += alpha * d[v] * rv / size[i]
        for e in range(indptr[v], indptr[v + 1]):
            u = indices[e]
            r[u] += (1.0 - alpha) * rv * data[e] / d[u]
            if not queued[u] and r[u] > rb_max:
                queue.append(u)
                queued[u] = True
        pushes += 1
    return est, r, pushes


def group_backward_push_rounds(W, leaves, targets, alpha, rb_max, max_rounds):
    """The backward pushes towards every target supernode in `targets` at
    once, in synchronous rounds (as group_forward_push_rounds): each round
    every (node, target) pair whose residue exceeds its target's threshold
    rb_max[j] (a scalar or one value per target) pushes it, and what arrives
    waits for the next round.  Pushing part of a residue keeps the backward
    invariant, so the result satisfies it, the stopping rule and the error
    bound of Lemma lem:bpsn-correct.  With rb_max = 0, T rounds give the
    power series truncated at T terms.

    Returns (estimate k x len(targets) [i, c] for target targets[c],
    residue len(targets) x n, per-node estimate alpha d(v) sum r, rounds,
    pairs pushed in the last round)."""
    W = sp.csr_matrix(W)
    d = degrees(W)
    n = d.shape[0]
    k = len(leaves)
    t = len(targets)
    inv = np.zeros(n)
    nz = d > 0
    inv[nz] = 1.0 / d[nz]
    R = np.zeros((t, n))
    for c, j in enumerate(targets):
        Fj = np.asarray(leaves[j], dtype=np.int64)
        np.add.at(R[c], Fj, 1.0 / Fj.size)
    th = np.broadcast_to(np.asarray(rb_max, dtype=np.float64), (t,))[:, None]
    node_est = np.zeros((t, n))
    sent = np.zeros((t, n))
    rounds = 0
    active = 0
    while rounds < max_rounds:
        if rounds > 0:
            # node v_i receives (1 - alpha) sum_k w_ik r(v_k) / d(v_i)
            R = R + (1.0 - alpha) * np.asarray(W @ sent.T).T * inv[None, :]
        mask = R > th
        active = int(mask.sum())
        node_est += alpha * d[None, :] * np.where(mask, R, 0.0)
        sent = np.where(mask, R, 0.0)
        R = np.where(mask, 0.0, R)
        rounds += 1
        if active == 0:
            break
    if active:
        R = R + (1.0 - alpha) * np.asarray(W @ sent.T).T * inv[None, :]
    est = np.zeros((k, t))
    for i, Fi in enumerate(leaves):
        Fi = np.asarray(Fi, dtype=np.int64)
        est[i, :] = node_est[:, Fi].sum(axis=1) / Fi.size
    return est, R, node_est, rounds, active


def gbp_error_term(ppr, leaves, targets, R, d):
    """The error of the backward estimate for every (i, target c):
        sum_{v_s in F(V_i)} d(v_s) / |F(V_i)| sum_{v_k} pi(v_s, v_k) r(v_k, V_j),
    with ``ppr`` the exact n x n PPR matrix (rows = sources) and R the
    len(targets) x n residue (the backward form of the push invariant)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros((len(leaves), len(targets)))
    PR = ppr @ np.asarray(R).T  # n x t
    for i, Fi in enumerate(leaves):
        Fi = np.asarray(Fi, dtype=np.int64)
        out[i, :] = (d[Fi][:, None] * PR[Fi, :]).sum(axis=0) / Fi.size
    return out


def dnpr(pi_d, leaves, m):
    """Degree-normalized PageRank of each supernode (Eq. eq:dnpr-dnppr):
    tau_j = sum_{v_t in F(V_j)} sum_{v_k} pi_d(v_k, v_t) / (m |F(V_j)|)."""
    return np.array([pi_d[:, np.asarray(F, dtype=np.int64)].sum() / (m * len(F)) for F in leaves])


def rmax_backward(eps, delta, d, leaves, j):
    """Backward residue threshold of target V_j (Eq. eq:brmax):
    eps delta / max over the other supernodes V_i of their mean leaf degree."""
    means = [np.asarray(d)[np.asarray(F, dtype=np.int64)].mean() for i, F in enumerate(leaves) if i != j]
    return eps * delta / max(means) if means else math.inf


def tau_push(W, leaves, alpha, eps, delta, max_rounds=100000, tau=None):
    """Algorithm alg:taupush: tau = 1 / sqrt(k n) (unless given), forward
    threshold by Eq. eq:rmax, the Group Forward-Push from every source
    supernode; then, for each target supernode with DNPR tau_j > tau, the
    Group Backward-Push with its threshold by Eq. eq:brmax replaces the
    column pi_d(., V_j).  The pushes run in synchronous rounds.  m is the arc
    count (nnz of W).  Returns (estimate k x k, the refined targets, tau)."""
    W = sp.csr_matrix(W)
    d = degrees(W)
    n = d.shape[0]
    k = len(leaves)
    m = W.nnz
    if tau is None:
        tau = tau_default(k, n)
    est, _, _, _, _ = group_forward_push_rounds(W, leaves, alpha, rmax_forward(eps, delta, m, tau), max_rounds)
    # Eq. eq:dnpr-dnppr on an undirected graph: sum_k pi_d(k, t) = d(t), so
    # tau_j is the mean leaf degree of V_j over m (the column sums of pi_d
    # are checked against this in the pins)
    tau_j = np.array([d[np.asarray(F, dtype=np.int64)].mean() / m for F in leaves])
    # with one supernode, Eq. eq:brmax has no other supernode to take the
    # maximum over: the column keeps its forward value
    targets = [j for j in range(k) if tau_j[j] > tau] if k > 1 else []
    if targets:
        rb = [rmax_backward(eps, delta, d, leaves, j) for j in targets]
        eb, _, _, _, _ = group_backward_push_rounds(W, leaves, targets, alpha, rb, max_rounds)
        est[:, targets] = eb
    return est, targets, tau
