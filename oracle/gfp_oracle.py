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

Pins (tests/test_oracle_gfp.py): the complete-graph closed form, symmetry and
column sums of the level-l DPPR of an undirected graph, the printed first push
of Section 3.3's running example, the invariant against the exact inverse at
every stopping point, the termination rule, the error bound of Lemma
lem:fpsn-correct, and the power-iteration series that the rounds reduce to
when the threshold is zero.  No function here is "parity unpinned".
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
