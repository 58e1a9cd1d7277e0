"""FP64 CPU oracle for the PPR -> DPPR -> PDist -> stress-layout path.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
HIP library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library: it builds its own transition matrix from
the undirected edge list (not from the CSR the GPU reads), iterates in FP64,
and evaluates every formula in plain NumPy/SciPy in the paper's notation.

Paper: "Effective and Efficient PageRank-based Positioning for Graph
Visualization" (arXiv 2112.14944).  Citations name the section, definition,
equation (by its LaTeX label) or algorithm that each function follows.

Every function here is pinned by the CPU tests against something other than
itself (closed forms, printed worked values, invariants, brute force, finite
differences).  There is no "parity unpinned" function in this file.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# O1  graph -> weight matrix, degrees, transition matrix
# --------------------------------------------------------------------------


def weight_matrix(n, eu, ev, w=None, directed=False):
    """Sparse FP64 weight matrix W (n x n) from an edge list.

    Section 2.1 (graph G=(V,E)); the paper's graphs are directed and
    unweighted.  ``directed=False`` treats each listed edge as the two arcs
    u->v and v->u sharing one weight (every benchmark graph is undirected);
    ``w=None`` means unit weights."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    vals = np.ones(eu.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    if directed:
        rows, cols, data = eu, ev, vals
    else:
        rows = np.concatenate([eu, ev])
        cols = np.concatenate([ev, eu])
        data = np.concatenate([vals, vals])
    W = sp.coo_matrix((data, (rows, cols)), shape=(n, n)).tocsr()
    W.sum_duplicates()
    return W


def degrees(W):
    """Out-degree d(v) = sum of the weights of v's out-arcs (Definition
    def:pprdist uses the out-degree; for unit weights it is the arc count)."""
    return np.asarray(W.sum(axis=1)).ravel()


def transition(W):
    """Random-walk transition matrix P = D^-1 W (Section 3.1: the walk moves to
    a uniform out-neighbour, weighted by arc weight when weights are given).

    A node without out-arcs gets a self-loop, P[v, v] = 1, so every row stays
    stochastic (the paper does not treat dangling nodes; this reading only
    changes pi(v, v) of an isolated v)."""
    n = W.shape[0]
    d = degrees(W)
    inv = np.zeros(n)
    nz = d > 0
    inv[nz] = 1.0 / d[nz]
    P = sp.diags(inv) @ W
    dang = np.nonzero(~nz)[0]
    if dang.size:
        P = P + sp.coo_matrix((np.ones(dang.size), (dang, dang)), shape=(n, n))
    return sp.csr_matrix(P)


# --------------------------------------------------------------------------
# O2  power iteration = synchronous forward push of every node
# --------------------------------------------------------------------------


def ppr_power_iteration(P, sources, alpha, tol=None, max_iter=100000, fixed_iters=None):
    """Multi-source PPR by power iteration in residual (push) form.

    Section 3.1 defines pi(s, t) as the probability that a random walk with
    restart from s stops at t; Section 3.3 uses power iteration for near-exact
    values; the forward-push invariant (Eq. eq:fwd-invariant) is what one push
    preserves.  Every iteration pushes all nodes at once:
        estimate += alpha * residue ;  residue <- (1 - alpha) * residue @ P
    starting from estimate = 0 and residue = e_s (PPR units) for each source s.

    Stops before the first push whose residue L1 norm (max over sources) is
    already <= tol, or after ``fixed_iters`` pushes if given.  Returns
    (estimate [S x n], pushes T, residue L1 norm per source)."""
    sources = np.asarray(sources, dtype=np.int64)
    n = P.shape[0]
    S = sources.shape[0]
    R = np.zeros((S, n))
    R[np.arange(S), sources] = 1.0
    est = np.zeros((S, n))
    t = 0
    while True:
        resid = np.abs(R).sum(axis=1)
        if fixed_iters is not None:
            if t >= fixed_iters:
                break
        else:
            if S == 0 or resid.max() <= tol or t >= max_iter:
                break
        est += alpha * R
        R = (1.0 - alpha) * np.asarray(R @ P)
        t += 1
    return est, t, np.abs(R).sum(axis=1)


def ppr_closed_form(P, alpha):
    """Exact PPR matrix Pi = alpha (I - (1 - alpha) P)^-1, rows = sources: the
    matrix form of the random walk with restart of Section 3.1 (sum over walk
    lengths of alpha (1-alpha)^l P^l).  Dense; tiny graphs only."""
    Pd = P.toarray() if sp.issparse(P) else np.asarray(P)
    n = Pd.shape[0]
    return alpha * np.linalg.inv(np.eye(n) - (1.0 - alpha) * Pd)


def forward_push_sync_dppr(P, d, source, alpha, steps):
    """The paper's push in DPPR units (Section 3.3 running example): the
    residue starts at d(source); one synchronous step turns alpha of every
    residue into the estimate and spreads 1 - alpha over out-neighbours in
    proportion to P.  Returns (estimate_d, residue_d) after ``steps`` steps."""
    n = P.shape[0]
    r = np.zeros(n)
    r[source] = d[source]
    est = np.zeros(n)
    for _ in range(steps):
        est = est + alpha * r
        r = (1.0 - alpha) * np.asarray(r @ P).ravel()
    return est, r


# --------------------------------------------------------------------------
# O4, O5  DPPR and PDist (Definition def:pprdist, Eq. eq:pprdist)
# --------------------------------------------------------------------------


def dppr(ppr_rows, d, sources):
    """pi_d(s, t) = pi(s, t) * d(s)  (Definition def:pprdist)."""
    sources = np.asarray(sources, dtype=np.int64)
    return ppr_rows * np.asarray(d)[sources][:, None]


def pdist_of_z(z, n_clamp):
    """Eq. eq:pprdist applied elementwise to z = pi_d(i,j) + pi_d(j,i):
    min(max(1 - ln z, 2), 2 ln n), natural logarithm (Section 3.1
    rationale); z = 0 (an unreachable pair) maps to the upper bound 2 ln n."""
    z = np.asarray(z, dtype=np.float64)
    hi = 2.0 * math.log(n_clamp)
    with np.errstate(divide="ignore"):
        raw = np.where(z > 0, 1.0 - np.log(np.where(z > 0, z, 1.0)), np.inf)
    return np.minimum(np.maximum(raw, 2.0), hi)


def pdist(pi_d, n_clamp):
    """PDist matrix of Eq. eq:pprdist on a square DPPR block whose rows and
    columns index the same node set, z = pi_d[i, j] + pi_d[j, i].  The
    diagonal is set to 0; the stress of Eq. eq:loss never reads it."""
    pi_d = np.asarray(pi_d, dtype=np.float64)
    D = pdist_of_z(pi_d + pi_d.T, n_clamp)
    np.fill_diagonal(D, 0.0)
    return D


def pdist_dz(pi_d, n_clamp):
    """d Delta_ij / d z_ij: -1/z strictly inside the clamp range, else 0
    (derivative of Eq. eq:pprdist; zero on and beyond the clamp kinks)."""
    pi_d = np.asarray(pi_d, dtype=np.float64)
    z = pi_d + pi_d.T
    hi = 2.0 * math.log(n_clamp)
    out = np.zeros_like(z)
    pos = z > 0
    raw = np.full_like(z, np.inf)
    raw[pos] = 1.0 - np.log(z[pos])
    inside = pos & (raw > 2.0) & (raw < hi)
    out[inside] = -1.0 / z[inside]
    np.fill_diagonal(out, 0.0)
    return out


# --------------------------------------------------------------------------
# O6 - O10  stress (Eq. eq:loss) and stress majorization (appendix)
# --------------------------------------------------------------------------


def stress_bruteforce(X, D):
    """L(X | Delta) = sum_{i<j} (1 - ||X_i - X_j|| / Delta_ij)^2, Eq. eq:loss,
    by a plain double loop.  Small inputs only."""
    X = np.asarray(X, dtype=np.float64)
    k = X.shape[0]
    total = 0.0
    for i in range(k):
        for j in range(i + 1, k):
            dist = math.hypot(X[i, 0] - X[j, 0], X[i, 1] - X[j, 1])
            total += (1.0 - dist / D[i, j]) ** 2
    return total


def pairwise_dist(X):
    X = np.asarray(X, dtype=np.float64)
    diff = X[:, None, :] - X[None, :, :]
    return np.sqrt((diff * diff).sum(-1))


def stress(X, D):
    """Eq. eq:loss over the strict upper triangle, vectorised."""
    dist = pairwise_dist(X)
    D = np.asarray(D, dtype=np.float64)
    iu = np.triu_indices(X.shape[0], 1)
    return float(((1.0 - dist[iu] / D[iu]) ** 2).sum())


def laplacian_w(D):
    """L^w of the appendix (stress majorization): -1/Delta_ij^2 off the
    diagonal, the negated row sum on the diagonal."""
    D = np.asarray(D, dtype=np.float64)
    k = D.shape[0]
    off = np.zeros((k, k))
    mask = ~np.eye(k, dtype=bool)
    off[mask] = -1.0 / (D[mask] ** 2)
    return off - np.diag(off.sum(axis=1))


def laplacian_y(D, Y):
    """L^Y of the appendix: -1/(Delta_ij ||Y_i - Y_j||) off the diagonal when
    Y_i != Y_j, 0 when they coincide, and the negated row sum on the
    diagonal."""
    D = np.asarray(D, dtype=np.float64)
    dist = pairwise_dist(Y)
    k = D.shape[0]
    off = np.zeros((k, k))
    mask = (~np.eye(k, dtype=bool)) & (dist > 0)
    off[mask] = -1.0 / (D[mask] * dist[mask])
    return off - np.diag(off.sum(axis=1))


def majorization_step(Y, D):
    """Exact stress-majorization update X = (L^w)^-1 L^Y Y (appendix).  L^w
    is singular (its rows sum to zero), so the pseudo-inverse is used, which
    returns the minimiser with zero centroid."""
    Lw = laplacian_w(D)
    LY = laplacian_y(D, Y)
    return np.linalg.pinv(Lw) @ (LY @ np.asarray(Y, dtype=np.float64))


def jacobi_step(Y, D):
    """One Jacobi sweep on the majorization system L^w X = L^Y Y of the
    appendix, starting from X = Y:
        X = Y + diag(L^w)^-1 (L^Y Y - L^w Y).
    Same fixed points as the exact update (both vanish where the stress
    gradient vanishes), no linear solve."""
    Y = np.asarray(Y, dtype=np.float64)
    Lw = laplacian_w(D)
    LY = laplacian_y(D, Y)
    return Y + (LY @ Y - Lw @ Y) / np.diag(Lw)[:, None]


def grad_x(X, D):
    """Gradient of Eq. eq:loss with respect to the positions, from the
    appendix expansion: L = const + tr(X^T L^w X) - 2 tr(X^T L^X X) with the
    Cauchy-Schwarz bound tight at Y = X, so dL/dX = 2 (L^w X - L^X X)."""
    X = np.asarray(X, dtype=np.float64)
    return 2.0 * (laplacian_w(D) @ X - laplacian_y(D, X) @ X)


def grad_delta_pair(X, D):
    """dL/dDelta_ij for each unordered pair i<j of Eq. eq:loss:
    d/dDelta (1 - dist/Delta)^2 = 2 (1 - dist/Delta) dist / Delta^2.
    Returned as a symmetric matrix (both (i,j) and (j,i) hold the pair's
    derivative) with a zero diagonal."""
    dist = pairwise_dist(X)
    D = np.asarray(D, dtype=np.float64)
    k = D.shape[0]
    out = np.zeros((k, k))
    mask = ~np.eye(k, dtype=bool)
    out[mask] = 2.0 * (1.0 - dist[mask] / D[mask]) * dist[mask] / (D[mask] ** 2)
    return out


# --------------------------------------------------------------------------
# O11, O12  gradient with respect to edge weights (chain rule through O1-O5)
# --------------------------------------------------------------------------


def adjoint_solve(P, alpha, G, iters=None):
    """A = M^-T G with M = I - (1 - alpha) P.  With ``iters`` given, the
    truncated Neumann series A = sum_{j<iters} ((1-alpha) P^T)^j G, the same
    truncation as ``iters`` pushes of the forward power iteration; otherwise a
    dense solve."""
    Pd = P.toarray() if sp.issparse(P) else np.asarray(P)
    if iters is None:
        n = Pd.shape[0]
        return np.linalg.solve((np.eye(n) - (1.0 - alpha) * Pd).T, G)
    QT = (1.0 - alpha) * Pd.T
    A = np.zeros_like(G)
    term = np.array(G, dtype=np.float64)
    for _ in range(iters):
        A = A + term
        term = QT @ term
    return A


def pipeline_forward(n, eu, ev, w, X, alpha, iters, n_clamp=None):
    """All-pairs loss L(X | Delta(w)) with every stage in FP64:
    W -> P -> Pi_hat (``iters`` pushes) -> pi_d -> Delta -> stress.
    Returns a dict of the intermediates."""
    W = weight_matrix(n, eu, ev, w)
    d = degrees(W)
    P = transition(W)
    src = np.arange(n)
    Pi, T, resid = ppr_power_iteration(P, src, alpha, fixed_iters=iters)
    pid = dppr(Pi, d, src)
    nc = n if n_clamp is None else n_clamp
    D = pdist(pid, nc)
    L = stress(X, D)
    return dict(W=W, d=d, P=P, Pi=Pi, pi_d=pid, Delta=D, loss=L, T=T, resid=resid)


def kink_pairs(pi_d, n_clamp, band):
    """Pairs i < j whose 1 - ln z_ij lies within ``band`` of a clamp bound of
    Eq. eq:pprdist (2 or 2 ln n_clamp).  The loss has a kink there; a path
    that evaluates z in lower precision may take either side of it."""
    pi_d = np.asarray(pi_d, dtype=np.float64)
    z = pi_d + pi_d.T
    hi = 2.0 * math.log(n_clamp)
    raw = np.full_like(z, np.inf)
    pos = z > 0
    raw[pos] = 1.0 - np.log(z[pos])
    near = (np.abs(raw - 2.0) < band) | (np.abs(raw - hi) < band)
    i, j = np.nonzero(np.triu(near, 1))
    return np.stack([i, j], axis=1)


def grad_weights(n, eu, ev, w, X, alpha, iters, n_clamp=None, adjoint_iters="same", kink_band=None):
    """dL/dw_e for every undirected edge e, and dL/dX, FP64.

    Chain rule through the pipeline (all-pairs, rows = sources):
      Gd  = dL/dpi_d           (pair derivative of Delta times dDelta/dz)
      Gb  = D Gd = dL/dPi_hat  (pi_d = D Pi_hat)
      dd  = rowsum(Gd * Pi_hat) = direct dL/dd through pi_d = D Pi_hat
      A   = M^-T Gb, M = I - (1-alpha) P     (adjoint of Pi = alpha M^-1)
      dQ  = A Pi_hat^T = dL/dQ, Q = (1-alpha) P = (1-alpha) D^-1 W
      arc u->v:  (1-alpha)/d_u (dQ_uv - sum_b P_ub dQ_ub) + dd_u
      edge {u,v}: arc u->v + arc v->u  (one weight shared by both arcs).
    The PPR Jacobian used is that of the converged PPR (implicit function)
    evaluated at the truncated estimate and a truncated adjoint; it differs
    from the derivative of the truncated forward by O((1-alpha)^iters).
    With ``kink_band``, the pairs of kink_pairs(pi_d, n_clamp, kink_band) take
    dDelta/dz = 0 (the one-sided derivative of the clamped side); they are
    returned as "kink_pairs"."""
    f = pipeline_forward(n, eu, ev, w, X, alpha, iters, n_clamp)
    nc = n if n_clamp is None else n_clamp
    D, Pi, pid, d, P, W = f["Delta"], f["Pi"], f["pi_d"], f["d"], f["P"], f["W"]
    gD = grad_delta_pair(X, D)
    dz = pdist_dz(pid, nc)
    kinks = np.zeros((0, 2), dtype=np.int64)
    if kink_band is not None:
        kinks = kink_pairs(pid, nc, kink_band)
        dz[kinks[:, 0], kinks[:, 1]] = 0.0
        dz[kinks[:, 1], kinks[:, 0]] = 0.0
    Gd = gD * dz
    Gb = d[:, None] * Gd
    dd = (Gd * Pi).sum(axis=1)
    A = adjoint_solve(P, alpha, Gb, iters=None if adjoint_iters is None else
                      (iters if adjoint_iters == "same" else adjoint_iters))
    dQ = A @ Pi.T
    Pd = P.toarray()
    rowterm = (Pd * dQ).sum(axis=1)
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)

    def arc(u, v):
        return (1.0 - alpha) / d[u] * (dQ[u, v] - rowterm[u]) + dd[u]

    gw = arc(eu, ev) + arc(ev, eu)
    gx = grad_x(X, D)
    return dict(grad_w=gw, grad_x=gx, loss=f["loss"], Delta=D, pi_d=pid, Pi=Pi,
                grad_pi_d=Gd, adjoint=A, dQ=dQ, d=d, kink_pairs=kinks)


def central_difference(fun, x0, idx, h):
    """Central finite differences of a scalar function at selected
    coordinates of a flat FP64 vector."""
    x0 = np.asarray(x0, dtype=np.float64)
    out = np.empty(len(idx))
    for k, i in enumerate(idx):
        xp = x0.copy()
        xm = x0.copy()
        xp[i] += h
        xm[i] -= h
        out[k] = (fun(xp) - fun(xm)) / (2.0 * h)
    return out


# --------------------------------------------------------------------------
# row-restricted evaluations for parity checks at large sizes
# --------------------------------------------------------------------------


def jacobi_rows(X, D_rows, rows):
    """Jacobi update of selected rows i only, given Delta[i, :] for each:
    X_i^+ = sum_{j != i} w_ij (X_j + Delta_ij (X_i - X_j)/||X_i - X_j||)
            / sum_{j != i} w_ij,  w = Delta^-2
    (the same sweep as :func:`jacobi_step`, written per row; a coincident
    pair contributes w_ij X_j and no direction term, as L^Y is zero there)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty((len(rows), 2))
    for k, i in enumerate(rows):
        Di = np.asarray(D_rows[k], dtype=np.float64)
        mask = np.ones(X.shape[0], dtype=bool)
        mask[i] = False
        diff = X[i] - X[mask]
        dist = np.sqrt((diff * diff).sum(-1))
        w = 1.0 / Di[mask] ** 2
        dirn = np.zeros_like(diff)
        pos = dist > 0
        dirn[pos] = diff[pos] / dist[pos, None]
        num = (w[:, None] * (X[mask] + Di[mask][:, None] * dirn)).sum(0)
        out[k] = num / w.sum()
    return out


def stress_rows(X, D_rows, rows):
    """Per-row half stress sum_{j != i} (1 - ||X_i - X_j||/Delta_ij)^2 / 2 for
    selected rows (summing it over all rows gives Eq. eq:loss)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty(len(rows))
    for k, i in enumerate(rows):
        Di = np.asarray(D_rows[k], dtype=np.float64)
        mask = np.ones(X.shape[0], dtype=bool)
        mask[i] = False
        diff = X[i] - X[mask]
        dist = np.sqrt((diff * diff).sum(-1))
        out[k] = 0.5 * ((1.0 - dist / Di[mask]) ** 2).sum()
    return out


def grad_x_rows(X, D_rows, rows):
    """dL/dX_i for selected rows: sum_{j != i} 2 w_ij (dist - Delta)(X_i - X_j)/dist."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty((len(rows), 2))
    for k, i in enumerate(rows):
        Di = np.asarray(D_rows[k], dtype=np.float64)
        mask = np.ones(X.shape[0], dtype=bool)
        mask[i] = False
        diff = X[i] - X[mask]
        dist = np.sqrt((diff * diff).sum(-1))
        pos = dist > 0
        coef = np.zeros_like(dist)
        coef[pos] = 2.0 * (dist[pos] - Di[mask][pos]) / (Di[mask][pos] ** 2 * dist[pos])
        out[k] = (coef[:, None] * diff).sum(0)
    return out


# --------------------------------------------------------------------------
# Aesthetic metrics of a layout (Section 2.1, Definitions def:node-distri and
# def:edge-var)
# --------------------------------------------------------------------------


def node_distribution(X):
    """ND(X) = sum_{i<j} 1 / ||X_i - X_j||^2 (Definition def:node-distri), by
    a plain double loop; a coincident pair makes it infinite."""
    X = np.asarray(X, dtype=np.float64)
    k = X.shape[0]
    total = 0.0
    for i in range(k):
        for j in range(i + 1, k):
            d2 = (X[i, 0] - X[j, 0]) ** 2 + (X[i, 1] - X[j, 1]) ** 2
            total += math.inf if d2 == 0.0 else 1.0 / d2
    return total


def ulcv(X, eu, ev):
    """ULCV(X) = l_sigma / l_mu over the edge lengths ||X_u - X_v|| of the
    listed edges (Definition def:edge-var), with the population standard
    deviation (the paper does not say which; this reading divides by the
    edge count).  NaN when there is no edge or every edge has length 0."""
    X = np.asarray(X, dtype=np.float64)
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    if eu.size == 0:
        return math.nan
    lengths = [math.hypot(X[u, 0] - X[v, 0], X[u, 1] - X[v, 1]) for u, v in zip(eu, ev)]
    mu = sum(lengths) / len(lengths)
    if mu == 0.0:
        return math.nan
    var = sum((l - mu) ** 2 for l in lengths) / len(lengths)
    return math.sqrt(var) / mu
