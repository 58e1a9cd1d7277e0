"""Seeded synthetic graph and layout inputs.

This module is shared by the test suite, the benchmark and both sides of every
parity check (the FP64 oracle and the HIP library).  It holds no arithmetic of
the method itself: it only draws random undirected simple graphs, edge weights,
source sets, initial layouts and distance matrices, and stores graphs as
symmetric CSR.  Degrees, transition probabilities, PPR, PDist and stress are
each computed independently by the oracle and by the HIP library.

The paper's datasets (its dataset table, SNAP/KONECT/LAW graphs) are not
available; the generators below stand in for them with the graph families the
benchmark configurations name: Erdos-Renyi, Chung-Lu power law and stochastic
block models (the last one standing in for the levels of a supernode
hierarchy, whose construction is outside the data-parallel path).

Every generator returns a :class:`Graph` whose edge list ``(eu, ev)`` holds each
undirected edge once with ``eu < ev``; ``weight`` is ``None`` for unit weights.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2112


@dataclasses.dataclass
class Graph:
    n: int
    eu: np.ndarray            # int64[m_und], eu < ev
    ev: np.ndarray            # int64[m_und]
    weight: np.ndarray | None  # float32[m_und] per undirected edge, or None
    row_ptr: np.ndarray       # int32[n+1] symmetric CSR (both arcs of every edge)
    col_idx: np.ndarray       # int32[nnz], sorted within each row
    arc_weight: np.ndarray | None  # float32[nnz], weight of the edge behind each arc
    arc_edge: np.ndarray      # int64[nnz], index of the undirected edge behind each arc

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m_und(self) -> int:
        return int(self.eu.shape[0])


def _pairs_from_tri_index(idx: np.ndarray):
    """Map linear indices over the strict upper triangle (row-major over the
    lower-triangle enumeration r > c, index = r(r-1)/2 + c) to pairs (c, r)."""
    idx = idx.astype(np.float64)
    r = np.floor((1.0 + np.sqrt(1.0 + 8.0 * idx)) / 2.0).astype(np.int64)
    # guard the float rounding at perfect triangle numbers
    tri = r * (r - 1) // 2
    too_big = tri > idx
    r[too_big] -= 1
    tri = r * (r - 1) // 2
    nxt = (r + 1) * r // 2
    too_small = nxt <= idx
    r[too_small] += 1
    tri = r * (r - 1) // 2
    c = idx.astype(np.int64) - tri
    return c, r


def _sample_distinct(rng: np.random.Generator, population: int, k: int) -> np.ndarray:
    """k distinct integers drawn uniformly from [0, population)."""
    if k <= 0 or population <= 0:
        return np.zeros(0, dtype=np.int64)
    if k >= population:
        return np.arange(population, dtype=np.int64)
    if k > population // 4:
        return np.sort(rng.permutation(population)[:k]).astype(np.int64)
    out = np.unique(rng.integers(0, population, size=k, dtype=np.int64))
    while out.shape[0] < k:
        extra = rng.integers(0, population, size=k - out.shape[0], dtype=np.int64)
        out = np.unique(np.concatenate([out, extra]))
    if out.shape[0] > k:
        out = np.sort(rng.choice(out, size=k, replace=False))
    return out


def _bernoulli_pairs(rng: np.random.Generator, n: int, p: float):
    """Each of the n(n-1)/2 unordered pairs independently with probability p.
    Draws the edge count from the binomial law, then a uniform subset of that
    size, which is the same distribution as independent coin flips."""
    total = n * (n - 1) // 2
    if total == 0 or p <= 0.0:
        z = np.zeros(0, dtype=np.int64)
        return z, z
    k = int(rng.binomial(total, min(p, 1.0)))
    idx = _sample_distinct(rng, total, k)
    return _pairs_from_tri_index(idx)


def build_graph(n: int, eu, ev, weight=None) -> Graph:
    """Symmetric CSR from an undirected simple edge list (self-loops and
    duplicates are dropped here; the first weight of a duplicate is kept)."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    a = np.minimum(eu, ev)
    b = np.maximum(eu, ev)
    keep = a != b
    a, b = a[keep], b[keep]
    w = None if weight is None else np.asarray(weight, dtype=np.float32)[keep]
    key = a * n + b
    key, first = np.unique(key, return_index=True)
    a, b = a[first], b[first]
    if w is not None:
        w = w[first]
    m = a.shape[0]
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    eid = np.concatenate([np.arange(m), np.arange(m)])
    order = np.argsort(src * n + dst)  # by (src, dst); the pairs are unique
    src, dst, eid = src[order], dst[order], eid[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    arc_w = None if w is None else w[eid].astype(np.float32)
    return Graph(n=n, eu=a, ev=b, weight=w, row_ptr=row_ptr.astype(np.int32),
                 col_idx=dst.astype(np.int32), arc_weight=arc_w, arc_edge=eid.astype(np.int64))


def erdos_renyi(n: int, avg_degree: float, seed: int) -> Graph:
    """G(n, p) with p = avg_degree / (n - 1), unit weights."""
    rng = np.random.default_rng(seed)
    p = avg_degree / max(n - 1, 1)
    u, v = _bernoulli_pairs(rng, n, p)
    return build_graph(n, u, v)


def chung_lu_weights(n: int, gamma: float, avg_degree: float) -> np.ndarray:
    """Expected-degree sequence w_i proportional to (i+1)^(-1/(gamma-1)),
    scaled to mean avg_degree and capped at sqrt(sum w) (then rescaled, a few
    rounds), in non-increasing order so node ids follow expected degree."""
    i = np.arange(n, dtype=np.float64)
    w = (i + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= avg_degree / w.mean()
    for _ in range(50):
        cap = math.sqrt(w.sum())
        w = np.minimum(w, cap)
        w *= avg_degree / w.mean()
        if w.max() <= math.sqrt(w.sum()) * (1 + 1e-9):
            break
    return np.minimum(w, math.sqrt(w.sum()))


def chung_lu(n: int, gamma: float, avg_degree: float, seed: int) -> Graph:
    """Power-law graph with expected degrees from :func:`chung_lu_weights`.

    Fast multigraph-collapse sampler: draw Poisson(sum(w)/2) edges whose two
    endpoints are independent with probability w_i / sum(w), then drop
    self-loops and collapse duplicates.  A pair is joined with probability
    1 - exp(-w_i w_j / sum(w)), the usual large-n stand-in for the Chung-Lu
    probability w_i w_j / sum(w)."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, gamma, avg_degree)
    total = w.sum()
    m = int(rng.poisson(total / 2.0))
    cdf = np.cumsum(w / total)
    cdf[-1] = 1.0
    u = _inverse_cdf(cdf, rng.random(m))
    v = _inverse_cdf(cdf, rng.random(m))
    return build_graph(n, u, v)


def _inverse_cdf(cdf, r):
    """searchsorted(cdf, r, side="right"), with the queries visited in sorted
    order (same result, far fewer cache misses for millions of queries)."""
    order = np.argsort(r)
    out = np.empty(r.shape[0], dtype=np.int64)
    out[order] = np.searchsorted(cdf, r[order], side="right")
    return out


def sbm(block_sizes, p_in: float, p_out: float, seed: int, weighted=None) -> Graph:
    """Stochastic block model with block-contiguous node ids.

    A pair inside a block is joined with probability p_in, a pair across
    blocks with p_out, independently.  Sampled as the union of an all-pairs
    draw at p_out and a within-block draw at (p_in - p_out) / (1 - p_out).
    ``weighted=(lo, hi, wseed)`` draws one uniform[lo, hi) FP32 weight per
    undirected edge."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(block_sizes, dtype=np.int64)
    n = int(sizes.sum())
    us, vs = [], []
    u, v = _bernoulli_pairs(rng, n, p_out)
    us.append(u)
    vs.append(v)
    p_extra = (p_in - p_out) / (1.0 - p_out) if p_out < 1.0 else 0.0
    start = 0
    for s in sizes:
        s = int(s)
        u, v = _bernoulli_pairs(rng, s, p_extra)
        us.append(u + start)
        vs.append(v + start)
        start += s
    eu = np.concatenate(us)
    ev = np.concatenate(vs)
    g = build_graph(n, eu, ev)
    if weighted is not None:
        lo, hi, wseed = weighted
        wr = np.random.default_rng(wseed)
        w = wr.uniform(lo, hi, size=g.m_und).astype(np.float32)
        g = build_graph(n, g.eu, g.ev, w)
    return g


def equal_blocks(n: int, n_blocks: int) -> np.ndarray:
    """Near-equal block sizes summing to n."""
    base = n // n_blocks
    sizes = np.full(n_blocks, base, dtype=np.int64)
    sizes[: n - base * n_blocks] += 1
    return sizes


# ---------------------------------------------------------------- batches

@dataclasses.dataclass
class GraphBatch:
    """Disjoint union of independent subgraphs, concatenated.

    Graph g owns global nodes [node_off[g], node_off[g+1]); ``col_idx`` holds
    global node ids, so the concatenation is itself one block-diagonal CSR.
    ``mat_off[g]`` is the offset of graph g's n_g x n_g dense block in a pool
    of concatenated row-major matrices."""
    graphs: list
    node_off: np.ndarray   # int64[G+1]
    row_ptr: np.ndarray    # int32[N+1] global CSR
    col_idx: np.ndarray    # int32[nnz] global ids
    mat_off: np.ndarray    # int64[G+1]

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.node_off)


def concat_graphs(graphs) -> GraphBatch:
    sizes = np.array([g.n for g in graphs], dtype=np.int64)
    node_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(sizes, out=node_off[1:])
    nnzs = np.array([g.nnz for g in graphs], dtype=np.int64)
    arc_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(nnzs, out=arc_off[1:])
    if arc_off[-1] >= 2**31:
        raise ValueError("batch too large for int32 CSR")
    row_ptr = np.zeros(int(node_off[-1]) + 1, dtype=np.int64)
    col = np.empty(int(arc_off[-1]), dtype=np.int32)
    for gi, g in enumerate(graphs):
        a, b = int(node_off[gi]), int(node_off[gi + 1])
        row_ptr[a:b] = g.row_ptr[:-1].astype(np.int64) + arc_off[gi]
        col[arc_off[gi]:arc_off[gi + 1]] = g.col_idx + a
    row_ptr[-1] = arc_off[-1]
    mat_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(sizes * sizes, out=mat_off[1:])
    return GraphBatch(graphs=list(graphs), node_off=node_off, row_ptr=row_ptr.astype(np.int32),
                      col_idx=col, mat_off=mat_off)


def sbm_batch_sizes(count: int, n_lo: int, n_hi: int, seed: int) -> np.ndarray:
    """Subgraph sizes, log-uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)


def sbm_batch(count: int, n_lo: int = 32, n_hi: int = 2048, blocks_lo: int = 4, blocks_hi: int = 16,
              p_in: float = 0.2, p_out: float = 0.01, seed: int = BASE_SEED) -> list:
    """Independent SBM subgraphs standing in for the levels of a multilevel
    supernode hierarchy: sizes log-uniform in [n_lo, n_hi], 4-16 near-equal
    blocks each, subgraph i drawn with seed + 1 + i."""
    sizes = sbm_batch_sizes(count, n_lo, n_hi, seed)
    rng = np.random.default_rng(seed + 7919)
    nblocks = rng.integers(blocks_lo, blocks_hi + 1, size=count)
    out = []
    for i in range(count):
        n = int(sizes[i])
        nb = int(min(nblocks[i], n))
        out.append(sbm(equal_blocks(n, nb), p_in, p_out, seed + 1 + i))
    return out


def stratified_subset(sizes: np.ndarray, k: int) -> np.ndarray:
    """Indices of k graphs spread evenly over the size order (for timing the
    oracle on a bounded sample of a batch)."""
    order = np.argsort(sizes, kind="stable")
    pick = np.linspace(0, len(order) - 1, num=min(k, len(order))).round().astype(np.int64)
    return np.unique(order[pick])


# ---------------------------------------------------------------- other inputs

def random_sources(g: Graph, count: int, seed: int, require_degree: bool = True) -> np.ndarray:
    """count distinct source nodes, uniform over nodes with at least one arc."""
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr)
    pool = np.nonzero(deg > 0)[0] if require_degree else np.arange(g.n)
    if count > pool.shape[0]:
        raise ValueError("not enough candidate sources")
    return np.sort(rng.choice(pool, size=count, replace=False)).astype(np.int32)


def uniform_layout(k: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Initial positions uniform in [lo, hi]^2, float32 [k, 2]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(k, 2)).astype(np.float32)


def random_distance_matrix(k: int, seed: int, lo: float = 2.0, hi: float | None = None) -> np.ndarray:
    """Symmetric float32 [k, k] matrix with zero diagonal and off-diagonal
    entries uniform in [lo, hi] (default hi = 2 ln k, the PDist range)."""
    if hi is None:
        hi = max(2.0 * math.log(max(k, 2)), lo + 1.0)
    rng = np.random.default_rng(seed)
    a = rng.uniform(lo, hi, size=(k, k))
    a = np.triu(a, 1)
    a = a + a.T
    return a.astype(np.float32)


def planted_layout_distances(k: int, seed: int, min_sep: float = 2.0):
    """Points in the plane, all pairwise distances >= min_sep, and their exact
    distance matrix (a Euclidean-realizable target)."""
    rng = np.random.default_rng(seed)
    side = math.sqrt(k) * min_sep * 1.5
    pts = []
    while len(pts) < k:
        p = rng.uniform(0, side, size=2)
        if all(math.hypot(p[0] - q[0], p[1] - q[1]) >= min_sep for q in pts):
            pts.append(p)
    P = np.array(pts)
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    return P, D
