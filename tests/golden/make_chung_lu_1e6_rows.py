"""Writes chung_lu_1e6_rows.npz: FP64 oracle PPR rows for the large
multi-source workload (Chung-Lu n = 10^6, exponent 2.2, mean degree 30,
4096 seeded sources with at least one arc, L1 residue 1e-6, T = 86 pushes).

Rows are kept at the targets the GPU accumulates (the 4096 sources) plus the
four highest-degree nodes of the whole graph.  Twenty sources are stored:
the four highest-degree nodes among the 4096 sources, twelve more of the
4096 drawn with a fixed seed, and the four highest-degree nodes of the whole
graph (the hubs, where pi_d(s, s) >= alpha d(s) is largest and FP32 is
tightest).  Power iteration in residual form (Section 3.1 / 3.3) by
``oracle.ppr_power_iteration``; nothing here comes from the HIP library.

Usage: python tests/golden/make_chung_lu_1e6_rows.py   (a few minutes)
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

N = 1_000_000
S = 4096
ALPHA = 0.15
TOL = 1e-6


def inputs():
    g = synth.chung_lu(N, 2.2, 30, synth.BASE_SEED + 4)
    src = synth.random_sources(g, S, synth.BASE_SEED + 5)
    return g, src


def picks(g, src):
    """(rows of src to compare, global hub ids, target ids)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    order = np.argsort(-deg[src], kind="stable")
    top = order[:4]
    rng = np.random.default_rng(synth.BASE_SEED + 7)
    rest = rng.choice(np.setdiff1d(np.arange(S), top), 12, replace=False)
    rows = np.concatenate([top, np.sort(rest)]).astype(np.int64)
    hubs = np.argsort(-deg, kind="stable")[:4].astype(np.int64)
    tgt = np.unique(np.concatenate([src.astype(np.int64), hubs]))
    return rows, hubs, tgt


def digest(g, src):
    h = hashlib.sha256()
    for a in (g.row_ptr.astype(np.int64), g.col_idx.astype(np.int64), src.astype(np.int64)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    g, src = inputs()
    rows, hubs, tgt = picks(g, src)
    print(f"n={g.n} nnz={g.nnz} hubs={hubs.tolist()} hub degrees={np.diff(g.row_ptr)[hubs].tolist()}", flush=True)
    W = O.weight_matrix(g.n, g.eu, g.ev)
    P = O.transition(W)
    sources = np.concatenate([src[rows].astype(np.int64), hubs])
    est, T, resid = O.ppr_power_iteration(P, sources, ALPHA, tol=TOL)
    out = os.path.join(HERE, "chung_lu_1e6_rows.npz")
    np.savez_compressed(out, sources=sources, rows=rows, hubs=hubs, tgt=tgt, ppr_tgt=est[:, tgt],
                        resid=resid, T=np.int64(T), digest=np.array(digest(g, src)), alpha=np.float64(ALPHA))
    print(f"wrote {out} in {time.time() - t0:.0f} s (T = {T})", flush=True)


if __name__ == "__main__":
    main()
