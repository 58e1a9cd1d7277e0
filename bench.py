"""Benchmark: subgraphs laid out per second, batched vs plain, on one MI355X.

Workload (default): 4096 independent stochastic-block-model subgraphs, sizes
log-uniform in [32, 2048], 4-16 blocks each, p_in = 0.2, p_out = 0.01, unit
weights; per subgraph all-pairs PPR (alpha = 0.15, L1 residual 1e-6, T = 86
pushes), DPPR, PDist and 200 Jacobi stress-layout sweeps from U[-1,1]^2.

A step is one pass of the whole path over the batch: one replay of the HIP
graph that holds planning, the persistent PPR kernel, PDist and the 200
layout launches.  The plain path runs the same subgraphs one at a time
through the C ABI (ppr_matrix, pdist, 200 x layout_step per subgraph).

Prints one JSON line.  Inputs are synthetic and seeded; they are generated
and uploaded before the timed region.
"""
import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# Plain FP32 adds: 256 CUs x 64 lanes x 2.4 GHz, one add per lane and clock
# (a CU issues one 64-lane VALU instruction per clock; no packed FP32).
PEAK_FP32_ADDS = 256 * 64 * 2.4e9
ALPHA = 0.15
TOL = 1e-6
STRESS_ITERS = 200


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "batch_ppr_kernel": ["paper_2112_14944_amd/csrc/ppr_core.hpp", "paper_2112_14944_amd/csrc/ppr.hip",
                         "paper_2112_14944_amd/csrc/batch.hip"],
    "batch_pair_kernel": ["paper_2112_14944_amd/csrc/layout_core.hpp", "paper_2112_14944_amd/csrc/batch.hip"],
}


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}@{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def _oracle_subgraph(args):
    """One sampled subgraph through the FP64 oracle (run in a worker process
    with its BLAS pool limited to one thread): all-pairs PPR, PDist and the
    Jacobi sweeps.  Returns the seconds it took."""
    g, seed = args
    import oracle as O
    import synth

    t0 = time.perf_counter()
    W = O.weight_matrix(g.n, g.eu, g.ev)
    d = O.degrees(W)
    src = np.arange(g.n)
    est, _, _ = O.ppr_power_iteration(O.transition(W), src, ALPHA, tol=TOL)
    D = O.pdist(O.dppr(est, d, src), g.n)
    X = synth.uniform_layout(g.n, seed).astype(np.float64)
    for _ in range(STRESS_ITERS):
        X = O.jacobi_step(X, D)
    return time.perf_counter() - t0


def _one_blas_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(graphs, sample_count=32, max_procs=16):
    """The FP64 oracle (unchanged) on a stratified sample of the batch, one
    subgraph per task in a pool of worker processes, one per host core (at
    most 16, the host share of one GPU), each with a one-thread BLAS pool.
    The sample is the subgraphs at evenly spaced size quantiles, each through
    all-pairs PPR, PDist and 200 Jacobi sweeps.  Returns subgraphs/s of the
    whole pool (sample size over wall time); ``balanced_value`` is the rate
    with the worker time spread evenly over the processes, which is what the
    pool would approach on the whole batch."""
    import multiprocessing as mp

    sizes = np.array([g.n for g in graphs])
    order = np.argsort(sizes, kind="stable")
    qs = (np.arange(sample_count) + 0.5) / sample_count
    pick = order[np.minimum((qs * len(order)).astype(int), len(order) - 1)]
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0)), len(pick)))
    # largest first, so that the pool's tail is short
    tasks = [(graphs[gi], int(gi)) for gi in sorted(pick, key=lambda i: -sizes[i])]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs, initializer=_one_blas_thread) as pool:
        per = pool.map(_oracle_subgraph, tasks, chunksize=1)
    dt = time.perf_counter() - t0
    return dict(value=len(pick) / dt, unit="subgraphs/s", cores=procs, kind="oracle",
                balanced_value=procs * len(pick) / float(sum(per)),
                sample=f"{len(pick)} subgraphs at evenly spaced size quantiles (n from {int(sizes[pick].min())} to "
                       f"{int(sizes[pick].max())}), each all-pairs PPR T=86 + PDist + {STRESS_ITERS} FP64 Jacobi "
                       f"sweeps, in {procs} worker processes with one BLAS thread each; {dt:.1f} s wall, "
                       f"{sum(per):.1f} s of worker time",
                seconds=dt, worker_seconds=float(sum(per)), host_cpus=len(os.sched_getaffinity(0)),
                cpu_model=host_cpu_model())


def stage_rooflines(gb, T, ms):
    """Roofline records of the batched stages from the library's stage times.

    PPR (three persistent launches, one per tile class, timed together): the
    tile keeps X in LDS and is bound by VALU issue, so its roofline is FP32
    adds (one per arc, source column and push) against the plain FP32 add
    peak, 256 CUs x 64 lanes x 2.4 GHz (no packed FP32).  The bytes a
    streaming SpMM would move are kept beside it (hbm_model): per push and
    subgraph 8 n^2 (read X_t, write X_t+1, S = n sources) + 4 nnz + 8 n + 4
    (column indices, row pointers, 1/d); T - 1 pushes follow the initial
    iterate.
    Layout (a pair-tile launch plus a combine launch per sweep): Delta is
    symmetric, so a sweep needs one triangle of 1/Delta with its diagonal,
    2 n (n + 1) bytes, plus 20 n of positions in and out and weight sums per
    subgraph; the per-tile partial sums the sweep writes and reads back are
    overhead, not counted.  The layout's FP32 work, by the convention of 15
    FLOP per ordered pair (FMA = 2, rsq = 1; dx, dy 2, d^2 3, rsq 1, c 1, w 1,
    w X_j 4, c (dx, dy) 4), is k (k - 1) * 15 per sweep and subgraph, reported
    against the FP32 vector peak."""
    sizes = gb.sizes.astype(np.float64)
    nnz = np.diff(gb.row_ptr.astype(np.int64))
    arcs = np.add.reduceat(nnz, gb.node_off[:-1].astype(np.int64)).astype(np.float64)
    pushes = max(T - 1, 0)
    ppr_bytes = pushes * float((8.0 * sizes * sizes + 4.0 * arcs + 8.0 * sizes + 4.0).sum())
    ppr_adds = pushes * float((arcs * sizes).sum())
    layout_bytes = float((2.0 * sizes * (sizes + 1.0) + 20.0 * sizes).sum())
    ppr_ms, layout_ms = ms[1], ms[3]
    lay_launch_ms = layout_ms / (STRESS_ITERS + 1)
    adds_per_s = ppr_adds / (ppr_ms * 1e-3)
    hbm_ach = ppr_bytes / (ppr_ms * 1e-3) / 1e9
    st_ppr = dict(kernel="batch_ppr_kernel", ms=ppr_ms, launches=3, bound="alu", unit="TFLOP/s",
                  achieved=adds_per_s / 1e12, peak=PEAK_FP32_ADDS / 1e12, frac=adds_per_s / PEAK_FP32_ADDS,
                  work=f"{ppr_adds:.4g} FP32 adds over {pushes} pushes (one per arc, source column and push)",
                  adds_per_s=adds_per_s, adds=ppr_adds,
                  hbm_model=dict(unit="GB/s", achieved=hbm_ach, peak=PEAK_HBM_GBS, frac=hbm_ach / PEAK_HBM_GBS,
                                 work=f"{ppr_bytes:.4g} B over {pushes} pushes (X read and written once per "
                                      f"push, plus CSR), the bytes a streaming SpMM would move"))
    st_lay = dict(kernel="batch_pair_kernel", ms=layout_ms, launches=2 * (STRESS_ITERS + 1), bound="hbm",
                  unit="GB/s", achieved=layout_bytes / (lay_launch_ms * 1e-3) / 1e9, peak=PEAK_HBM_GBS,
                  work=f"{layout_bytes:.4g} B per sweep (one triangle of 1/Delta, X in and out, weight sums)")
    st_lay["frac"] = st_lay["achieved"] / PEAK_HBM_GBS
    lay_flops = STRESS_ITERS * 15.0 * float((sizes * (sizes - 1.0)).sum())
    st_lay["flops"] = lay_flops
    st_lay["tflops"] = lay_flops / (layout_ms * 1e-3) / 1e12
    st_lay["flop_frac"] = st_lay["tflops"] / PEAK_FP32_TFLOPS
    return dict(plan_ms=ms[0], ppr=st_ppr, pdist_ms=ms[2], layout=st_lay)


def spmm_all_pairs(ops, dev, n=20000, gamma=2.5, avg_degree=20, tol=1e-7, reps=2, sweeps=500):
    """The single large graph end to end: all-pairs PPR on a Chung-Lu graph,
    n = 20000, exponent 2.5, mean degree 20, to L1 1e-7 (one whole
    ppr_matrix call: row order, arc deal, T pushes, DPPR written; at this size
    the library keeps 2 source columns of every node in LDS, ppr_mid_kernel),
    then PDist and `sweeps` Jacobi sweeps of the 20000-node layout
    (layout_step, one launch per sweep), each stage timed with HIP events on
    the stream the library launches on.  Algorithmic bytes: per push, as for
    any SpMM that keeps X in HBM, 8 n S (X read and written once, S = n
    sources) + 4 nnz + 8 (n + 1); PDist reads and writes n^2 floats; a sweep
    reads Delta (4 n^2 bytes).  Sweep FLOPs by the 15-per-ordered-pair
    convention."""
    import torch
    import synth

    g = synth.chung_lu(n, gamma, avg_degree, synth.BASE_SEED + 2)
    csr = ops.Csr.from_graph(g, dev)
    src = torch.arange(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    best = None
    dppr = None
    T = 0
    for _ in range(reps):
        dppr = None
        (_, dppr, T, _), t = timed(lambda: ops.ppr_matrix(csr, src, None, alpha=ALPHA, tol=tol, want_ppr=False,
                                                         want_dppr=True))
        best = t if best is None else min(best, t)
    delta, t_pd = timed(lambda: ops.pdist(dppr, n))
    del dppr
    x0 = torch.as_tensor(synth.uniform_layout(n, 41), device=dev)
    s0 = ops.stress_eval(delta, x0).item()
    x, t_lay = timed(lambda: ops.layout(delta, x0, sweeps))
    s1 = ops.stress_eval(delta, x).item()
    del delta
    nnz = int(g.col_idx.shape[0])
    alg = (T - 1) * (8.0 * n * n + 4.0 * nnz + 8.0 * (n + 1))
    pd_bytes = 8.0 * n * n
    lay_bytes = sweeps * 4.0 * n * n
    lay_flops = sweeps * 15.0 * n * (n - 1.0)
    return dict(workload=f"chung_lu n={n} gamma={gamma} mean degree {avg_degree}, all {n} sources, "
                         f"L1 {tol:g} (T={T}), PDist, {sweeps} Jacobi sweeps from U[-1,1]^2",
                kernel="ppr_mid_kernel", ms=best, bound="hbm", unit="GB/s", achieved=alg / (best * 1e-3) / 1e9,
                peak=PEAK_HBM_GBS, frac=alg / (best * 1e-3) / 1e9 / PEAK_HBM_GBS,
                work=f"{alg:.4g} B over {T - 1} pushes", nnz=nnz,
                pdist=dict(kernel="pdist_kernel", ms=t_pd, bound="hbm", unit="GB/s",
                           achieved=pd_bytes / (t_pd * 1e-3) / 1e9, frac=pd_bytes / (t_pd * 1e-3) / 1e9 / PEAK_HBM_GBS),
                layout=dict(kernel="layout_rows_kernel", sweeps=sweeps, ms=t_lay, ms_per_sweep=t_lay / sweeps,
                            bound="hbm", unit="GB/s", achieved=lay_bytes / (t_lay * 1e-3) / 1e9,
                            frac=lay_bytes / (t_lay * 1e-3) / 1e9 / PEAK_HBM_GBS,
                            tflops=lay_flops / (t_lay * 1e-3) / 1e12, stress_before=s0, stress_after=s1),
                total_ms=best + t_pd + t_lay)


def spmm_large(ops, dev, n=1_000_000, gamma=2.2, avg_degree=30, n_src=4096, tol=1e-6, reps=2):
    """The multi-source SpMM above the LDS sizes: Chung-Lu n = 10^6, exponent
    2.2, mean degree 30 (about 3e7 arcs), PPR from 4096 seeded sources to L1
    1e-6, accumulated at the 4096 sources as targets, one whole ppr_matrix call.
    The iterate (4096 columns of 10^6 nodes, 16.4 GB per buffer) lives in HBM
    (stream_step_kernel, one launch per push).  Algorithmic bytes per push:
    8 n S + 4 nnz + 8 (n + 1)."""
    import torch
    import synth

    g = synth.chung_lu(n, gamma, avg_degree, synth.BASE_SEED + 4)
    src = synth.random_sources(g, n_src, synth.BASE_SEED + 5)
    csr = ops.Csr.from_graph(g, dev)
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, dppr, T, _ = ops.ppr_matrix(csr, src, tgt=src, alpha=ALPHA, tol=tol, want_ppr=False, want_dppr=True)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    delta = ops.pdist(dppr, n)  # PDist among the sources, n_clamp = |V|
    del dppr
    nnz = int(g.col_idx.shape[0])
    alg = (T - 1) * (8.0 * n * n_src + 4.0 * nnz + 8.0 * (n + 1))
    return dict(workload=f"chung_lu n={n} gamma={gamma} mean degree {avg_degree}, {n_src} sources, "
                         f"L1 {tol:g} (T={T}), DPPR among the sources, whole ppr_matrix call",
                kernel="stream_step_kernel", ms=best, bound="hbm", unit="GB/s",
                achieved=alg / (best * 1e-3) / 1e9, peak=PEAK_HBM_GBS,
                frac=alg / (best * 1e-3) / 1e9 / PEAK_HBM_GBS, work=f"{alg:.4g} B over {T - 1} pushes",
                nnz=nnz), (g, csr, delta, src)


def layout_metrics_leg(ops, dev, x, g, src, reps=3):
    """ND and ULCV (Section 2.1) of the 4096-node layout: ND over all pairs,
    ULCV over the edges of the graph induced on the 4096 sources.  Timed
    whole calls (each synchronizes to return its two numbers)."""
    import torch
    import synth

    pos = np.full(g.n, -1, dtype=np.int64)
    pos[np.asarray(src)] = np.arange(len(src))
    keep = (pos[g.eu] >= 0) & (pos[g.ev] >= 0)
    sub = synth.build_graph(len(src), pos[g.eu[keep]], pos[g.ev[keep]])
    csr = ops.Csr.from_graph(sub, dev)
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nd, ul = ops.layout_metrics(x, csr)
        t = (time.perf_counter() - t0) * 1e3
        best = t if best is None else min(best, t)
    k = x.shape[0]
    return dict(workload=f"ND over the {k * (k - 1) // 2} pairs of the 4096-node layout after the exact step; "
                         f"ULCV over the {sub.m_und} edges induced on its nodes", nd=nd, ulcv=ul, ms=best,
                kernel="nd_kernel", pairs=k * (k - 1) // 2)


def batch_exact_leg(ops, b, bufs, sizes, reps=3):
    """The exact stress-majorization step for every subgraph of the batch in
    one launch (pprviz_batch_step_exact, one block per subgraph), from the
    batch's layout after its Jacobi sweeps, with the batch's PDist pool, CG to
    1e-6.  Algorithmic bytes: 4 n_g^2 per pass over Delta_g (the right-hand
    side, then one L^w apply per CG iteration of that subgraph)."""
    import torch

    best = None
    iters = conv = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, iters, conv = ops.batch_step_exact(b, bufs["delta"], bufs["x_out"], cg_tol=1e-6)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    it = iters.cpu().numpy().astype(np.int64)
    nbytes = float((4 * sizes.astype(np.float64) ** 2 * (it + 1)).sum())
    achieved = nbytes / (best * 1e-3) / 1e9
    return dict(workload=f"exact majorization step of all {b.n_graphs} subgraphs of the batch (sizes 32..2048) "
                         f"from their layouts after the Jacobi sweeps, CG to 1e-6, one launch",
                kernel="cg_batch_kernel", ms=best, subgraphs_per_s=b.n_graphs / (best * 1e-3),
                cg_iters_mean=float(it.mean()), cg_iters_max=int(it.max()),
                converged=int(conv.cpu().numpy().sum()), bound="hbm", unit="GB/s", achieved=achieved,
                peak=PEAK_HBM_GBS, frac=achieved / PEAK_HBM_GBS,
                work=f"{nbytes:.3e} B: the right-hand side and one L^w apply per CG iteration, per subgraph")


def layout_exact_leg(ops, dev, delta, sweeps=200, reps=3, cpu=False):
    """The exact stress-majorization step (layout_step_exact, conjugate
    gradients on L^w X = L^Y(Y) Y) on the 4096-node layout of the 10^6-node
    graph: Delta is the PDist among its 4096 sources, Y the layout after 200
    Jacobi sweeps from U[-1,1]^2.  Algorithmic bytes: 4 k^2 per pass over
    Delta (the right-hand side, then one L^w apply per CG iteration)."""
    import torch
    import synth

    k = delta.shape[0]
    x0 = torch.as_tensor(synth.uniform_layout(k, synth.BASE_SEED + 6), device=dev)
    y = ops.layout(delta, x0, sweeps)
    s_y = ops.stress_eval(delta, y).item()
    best = None
    iters = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        x, iters = ops.layout_step_exact(delta, y, cg_tol=1e-6)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    s_x = ops.stress_eval(delta, x).item()
    alg = (iters + 1) * 4.0 * k * k
    cpu_o = None
    if cpu:
        import oracle as O
        kc = 2048  # the oracle's pseudo-inverse costs O(k^3): timed at k/2, scaled by 8
        D = delta[:kc, :kc].double().cpu().numpy()
        Y = y[:kc].double().cpu().numpy()
        t0 = time.perf_counter()
        O.majorization_step(Y, D)
        dt = time.perf_counter() - t0
        cpu_o = dict(ms=dt * 8e3, kind="oracle", sample=f"one step at k={kc} (the leading block of Delta), "
                     f"{dt:.1f} s, scaled by (k/{kc})^3 = 8 for the pseudo-inverse")
    exact_x = x
    return exact_x, dict(workload=f"exact stress-majorization step, k={k} (PDist among the 4096 sources of the "
                         f"10^6-node graph), from the layout after {sweeps} Jacobi sweeps, CG to 1e-6",
                kernel="cg_rows_kernel", ms=best, cg_iters=iters, stress_before=s_y, stress_after=s_x,
                bound="hbm", unit="GB/s", achieved=alg / (best * 1e-3) / 1e9, peak=PEAK_HBM_GBS,
                frac=alg / (best * 1e-3) / 1e9 / PEAK_HBM_GBS,
                work=f"{alg:.4g} B: {iters + 1} passes over Delta", cpu_oracle=cpu_o)


def gfp_cpu_oracle(g, k, r_max, sample=4):
    """The FP64 oracle's rounds (oracle.group_forward_push_rounds, unchanged)
    on the same graph and threshold for `sample` of the k source supernodes
    (evenly spaced), timed on the host and scaled by k / sample: the source
    columns are independent, so the work is linear in their number."""
    import oracle as O
    import synth

    W = O.weight_matrix(g.n, g.eu, g.ev)
    leaves = []
    start = 0
    for sz in synth.equal_blocks(g.n, k):
        leaves.append(np.arange(start, start + sz))
        start += sz
    pick = [leaves[i] for i in np.linspace(0, k - 1, sample).round().astype(int)]
    t0 = time.perf_counter()
    _, _, _, rounds, _ = O.group_forward_push_rounds(W, pick, ALPHA, r_max, 10000)
    dt = (time.perf_counter() - t0) * k / sample
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = 1
    return dict(ms=dt * 1e3, rounds=rounds, cores=int(threads), kind="oracle",
                sample=f"{sample} of the {k} source supernodes (and the same {sample} as targets), every round, "
                       f"{dt * sample / k:.1f} s, extrapolated linearly to {k}")


def gbp_level(ops, dev, g, csr, k=25, reps=3):
    """Level-l DPPR towards all 25 target supernodes of the top supernode of
    the 10^6-node graph by the Group Backward-Push in rounds (one
    gbp_level_dppr call), each target with its threshold of Eq. eq:brmax
    (eps delta over the largest mean leaf degree of the other supernodes;
    eps = 1 - 1/e, delta = 1/(10k)).  Same byte model per round as the
    forward pushes."""
    import torch
    import synth

    n = g.n
    nnz = int(g.col_idx.shape[0])
    sizes = synth.equal_blocks(n, k)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    ptr = torch.as_tensor(starts.astype(np.int32), device=dev)
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    deg = np.diff(g.row_ptr).astype(np.float64)
    means = np.array([deg[starts[i]:starts[i + 1]].mean() for i in range(k)])
    ed = (1.0 - 1.0 / math.e) / (10 * k)
    th = np.array([ed / np.delete(means, j).max() for j in range(k)], dtype=np.float32)
    best = None
    rounds = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, _, rounds, _ = ops.gbp_level_dppr(csr, (ptr, idx), np.arange(k), th, ALPHA, 10000)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    ld = 32 * ((k + 31) // 32)
    alg = rounds * (16.0 * n * ld + 4.0 * nnz + 24.0 * n)
    return dict(workload=f"chung_lu n={n} gamma=2.2 mean degree 30, k={k} target supernodes partitioning V, "
                         f"thresholds by Eq. eq:brmax ({th.min():.3e} .. {th.max():.3e}), whole gbp_level_dppr call",
                kernel="gfp_round_kernel (backward)", ms=best, rounds=rounds, bound="hbm", unit="GB/s",
                achieved=alg / (best * 1e-3) / 1e9, peak=PEAK_HBM_GBS, frac=alg / (best * 1e-3) / 1e9 / PEAK_HBM_GBS,
                work=f"{alg:.4g} B over {rounds} rounds")


def tau_push_hubs(ops, dev, reps=3):
    """Tau-Push (Algorithm alg:taupush) on a supernode of 25 singleton
    children at the 25 largest degrees of a Chung-Lu graph (n = 20000,
    exponent 2.5, mean degree 20), with the paper's tau = 1/sqrt(kn),
    eps = 1 - 1/e, delta = 1/(10k): the hubs whose DNPR exceeds tau are
    refined by the backward pushes."""
    import torch
    import synth

    g = synth.chung_lu(20000, 2.5, 20, synth.BASE_SEED + 2)
    d = np.diff(g.row_ptr)
    hubs = np.argsort(-d, kind="stable")[:25]
    leaves = [np.array([h]) for h in hubs]
    csr = ops.Csr.from_graph(g, dev)
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, nb, rounds, _ = ops.tau_push_level_dppr(csr, leaves, ALPHA)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    return dict(workload="chung_lu n=20000 gamma=2.5 mean degree 20; 25 singleton supernodes at the largest "
                         "degrees; tau = 1/sqrt(kn), eps 1-1/e, delta 1/(10k); whole tau_push_level_dppr call",
                ms=best, backward_targets=nb, forward_rounds=rounds[0], backward_rounds=rounds[1])


def gfp_level(ops, dev, g, csr, k=25, reps=3, cpu=False):
    """Level-l DPPR among the k = 25 children of the top supernode of the
    10^6-node Chung-Lu graph above, by Group Forward-Push in rounds (one
    gfp_level_dppr call from all 25 source supernodes).  The children
    partition V into contiguous id ranges (the hierarchy itself is not built
    here).  Threshold by Eq. eq:rmax with the paper's defaults
    eps = 1 - 1/e, delta = 1/(10k), tau = 1/sqrt(kn), m = nnz.
    Algorithmic bytes per round (gfp_round_kernel): 16 n ld (what the last
    round sent, read once; the residue read and written; what this round
    sends, written; ld = 32 columns) + 4 nnz + 24 n (arcs, row table,
    degrees)."""
    import torch
    import synth

    n = g.n
    nnz = int(g.col_idx.shape[0])
    sizes = synth.equal_blocks(n, k)
    ptr = torch.as_tensor(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32), device=dev)
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    eps, delta, tau = 1.0 - 1.0 / math.e, 1.0 / (10 * k), 1.0 / math.sqrt(k * n)
    r_max = eps * delta / (nnz * tau)
    best = None
    rounds = None
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out, _, _, rounds, _ = ops.gfp_level_dppr(csr, (ptr, idx), ALPHA, r_max, 10000)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    ld = 32 * ((k + 31) // 32)
    alg = rounds * (16.0 * n * ld + 4.0 * nnz + 24.0 * n)
    cpu_o = gfp_cpu_oracle(g, k, r_max) if cpu else None
    return dict(workload=f"chung_lu n={n} gamma=2.2 mean degree 30, k={k} supernodes partitioning V, "
                         f"r_max={r_max:.3e} (eps 1-1/e, delta 1/(10k), tau 1/sqrt(kn)), whole gfp_level_dppr call",
                kernel="gfp_round_kernel", ms=best, rounds=rounds, bound="hbm", unit="GB/s",
                achieved=alg / (best * 1e-3) / 1e9, peak=PEAK_HBM_GBS,
                frac=alg / (best * 1e-3) / 1e9 / PEAK_HBM_GBS, work=f"{alg:.4g} B over {rounds} rounds",
                cpu_oracle=cpu_o)


def counters_pass(ops, b, x0, dev):
    """One eager batched pass, one all-pairs SpMM run (n = 20000), then a plain 1 GiB
    device copy, for rocprofv3 --pmc runs: the copy's FETCH_SIZE / WRITE_SIZE
    calibrate the counters."""
    import torch

    bufs = b.buffers(x0)
    ms = ops.pprviz_batch_profile(b, bufs, alpha=ALPHA, tol=TOL, stress_iters=STRESS_ITERS)
    log(f"eager pass stage ms {ms}")
    _, iters, _ = ops.batch_step_exact(b, bufs["delta"], bufs["x_out"], cg_tol=1e-6)
    torch.cuda.synchronize()
    log(f"batched exact step, CG iterations mean {float(iters.float().mean()):.2f}")
    del bufs
    sp = spmm_all_pairs(ops, dev, reps=1, sweeps=1)
    log(f"all-pairs SpMM (n = 20000) {sp['ms']:.1f} ms")
    calibration_copy()


def calibration_copy():
    """A plain 1 GiB device-to-device copy: its FETCH_SIZE / WRITE_SIZE give
    the counters' scale."""
    import torch

    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    c.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: 1 GiB read, 1 GiB written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--graphs", type=int, default=4096)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the stage-timing pass")
    ap.add_argument("--no-spmm", action="store_true", help="skip the all-pairs SpMM measurement (n = 20000)")
    ap.add_argument("--no-gfp", action="store_true",
                    help="skip the level-l DPPR (group forward push) leg on the 10^6-node graph")
    ap.add_argument("--no-spmm-large", action="store_true",
                    help="skip the 4096-source SpMM on the n = 10^6 graph")
    ap.add_argument("--only-gfp", action="store_true",
                    help="run only the level-l DPPR leg (10^6-node graph) and print its JSON object")
    ap.add_argument("--counters", action="store_true",
                    help="one eager batched pass plus a 1 GiB calibration copy (for rocprofv3 --pmc), no timing")
    ap.add_argument("--counters-large", action="store_true",
                    help="one 4096-source ppr_matrix call on the 10^6-node graph plus the 1 GiB calibration copy "
                         "(for rocprofv3 --pmc), no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1 "
                                   "(the multi-GPU sharding is a design, not a build)"}))
        sys.exit(2)

    import torch

    import synth
    from paper_2112_14944_amd import _lib as L
    from paper_2112_14944_amd import ops

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    if args.counters_large:
        sp, _ = spmm_large(ops, dev, reps=1)
        log(f"4096-source SpMM (n = 10^6): {sp['ms']:.1f} ms")
        calibration_copy()
        return
    if args.only_gfp:
        g_big = synth.chung_lu(1_000_000, 2.2, 30, synth.BASE_SEED + 4)
        gfp = gfp_level(ops, dev, g_big, ops.Csr.from_graph(g_big, dev), cpu=not args.no_cpu_baseline)
        log(f"level-l DPPR by group forward push (n = 10^6, k = 25): {gfp['ms']:.2f} ms, "
            f"{gfp['rounds']} rounds, {gfp['achieved']:.0f} GB/s algorithmic")
        print(json.dumps({"level_dppr_gfp": gfp}), flush=True)
        return
    G = args.graphs
    t0 = time.perf_counter()
    graphs = synth.sbm_batch(G, seed=synth.BASE_SEED)
    gb = synth.concat_graphs(graphs)
    sizes = gb.sizes
    log(f"generated {G} subgraphs in {time.perf_counter() - t0:.1f}s: nodes={int(sizes.sum())} "
        f"arcs={gb.col_idx.shape[0]} sum n^2={int((sizes ** 2).sum())}")
    b = ops.Batch(gb, dev)
    x0 = torch.as_tensor(synth.uniform_layout(b.n_nodes, synth.BASE_SEED + 99), device=dev)
    bufs = b.buffers(x0)
    T, _ = ops.pushes_for_tolerance(ALPHA, TOL, 100000)
    if args.counters:
        counters_pass(ops, b, x0, dev)
        return
    plan = ops.BatchPlan(b, bufs, alpha=ALPHA, tol=TOL, stress_iters=STRESS_ITERS)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        plan.launch()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = G / (ms_step / 1e3)
    log(f"batched: {ms_step:.2f} ms/step -> {value:.1f} subgraphs/s (wall {wall:.2f}s for {args.steps} steps)")
    stress = bufs["stress"].cpu().numpy()
    assert np.all(np.isfinite(stress)), "non-finite stress in the batched result"

    # ---- per-stage timing (HIP events recorded by the library on this stream)
    stages = None
    roof = None
    if not args.no_profile:
        bufs_p = b.buffers(x0)
        ms = ops.pprviz_batch_profile(b, bufs_p, alpha=ALPHA, tol=TOL, stress_iters=STRESS_ITERS)
        assert torch.equal(bufs_p["x_out"], bufs["x_out"]), "profiled run differs from the graph replay"
        del bufs_p
        stages = stage_rooflines(gb, T, ms)
        dom = stages["ppr"] if stages["ppr"]["ms"] >= stages["layout"]["ms"] else stages["layout"]
        traffic = traffic_from_profiles(dom["kernel"], f"sbm_batch_{G}")
        roof = dict(kernel=dom["kernel"], bound=dom["bound"], achieved=dom["achieved"], peak=dom["peak"],
                    unit=dom["unit"], frac=dom["frac"], traffic=traffic)
        log(f"stages ms: plan {ms[0]:.2f} ppr {ms[1]:.2f} pdist {ms[2]:.2f} layout {ms[3]:.2f}; "
            f"ppr {stages['ppr']['adds_per_s'] / 1e12:.2f} T adds/s ({100 * stages['ppr']['frac']:.0f}% of the "
            f"FP32 add peak; {stages['ppr']['hbm_model']['achieved']:.0f} GB/s by the SpMM byte model), "
            f"layout {stages['layout']['achieved']:.0f} GB/s, {stages['layout']['tflops']:.1f} TFLOP/s FP32 "
            f"({100 * stages['layout']['flop_frac']:.0f}% of the vector peak)")

    batch_exact = batch_exact_leg(ops, b, bufs, sizes)
    log(f"batched exact step ({G} subgraphs): {batch_exact['ms']:.2f} ms, CG iterations mean "
        f"{batch_exact['cg_iters_mean']:.1f} max {batch_exact['cg_iters_max']}, {batch_exact['converged']} converged, "
        f"{batch_exact['achieved']:.0f} GB/s algorithmic")

    # ---- plain path: one subgraph at a time through the C ABI
    plain = None
    if not args.no_plain:
        lib = L.lib()
        sp = C.c_void_p(stream.cuda_stream)
        per = []
        max_n = int(sizes.max())
        ws_layout = torch.empty(lib.layout_workspace(max_n), dtype=torch.uint8, device=dev)
        csrs = []
        for g in graphs:
            csr = ops.Csr.from_graph(g, dev)
            cg = csr.c()
            src = torch.arange(g.n, dtype=torch.int32, device=dev)
            wsz = lib.ppr_matrix_workspace(C.byref(cg), g.n, g.n)
            ws = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
            dppr = torch.empty((g.n, g.n), dtype=torch.float32, device=dev)
            delta = torch.empty_like(dppr)
            xa = torch.empty((g.n, 2), dtype=torch.float32, device=dev)
            xb = torch.empty_like(xa)
            csrs.append((csr, cg, src, ws, dppr, delta, xa, xb))
        a0 = gb.node_off
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        pe0 = torch.cuda.Event(enable_timing=True)
        pe1 = torch.cuda.Event(enable_timing=True)
        pe0.record(stream)
        it = C.c_int32()
        for gi, (csr, cg, src, ws, dppr, delta, xa, xb) in enumerate(csrs):
            n = graphs[gi].n
            st = lib.ppr_matrix(C.byref(cg), C.c_void_p(src.data_ptr()), n, None, n, ALPHA, TOL, 100000, None,
                                C.c_void_p(dppr.data_ptr()), None, C.byref(it), C.c_void_p(ws.data_ptr()),
                                ws.numel(), sp)
            assert st == 0
            assert lib.pdist(C.c_void_p(dppr.data_ptr()), n, n, C.c_void_p(delta.data_ptr()), sp) == 0
            xa.copy_(x0[int(a0[gi]):int(a0[gi + 1])])
            pd, pa, pb = C.c_void_p(delta.data_ptr()), C.c_void_p(xa.data_ptr()), C.c_void_p(xb.data_ptr())
            wsl = C.c_void_p(ws_layout.data_ptr())
            for s in range(STRESS_ITERS):
                lib.layout_step(pd, n, pa, pb, None, wsl, ws_layout.numel(), sp)
                pa, pb = pb, pa
        pe1.record(stream)
        torch.cuda.synchronize()
        plain_wall = time.perf_counter() - p0
        plain_ms = pe0.elapsed_time(pe1)
        # same results as the batched path on the largest subgraph: DPPR and
        # Delta bit for bit (same kernels), the layout to rounding (the batch
        # sums each unordered pair once over tiles, the plain step sweeps rows)
        gi = int(np.argmax(sizes))
        lo, hi_ = int(a0[gi]), int(a0[gi + 1])
        res = csrs[gi][6] if STRESS_ITERS % 2 == 0 else csrs[gi][7]
        same_bits = bool(torch.equal(csrs[gi][4], ops.graph_block(gb, bufs["dppr"], gi)) and
                         torch.equal(csrs[gi][5], ops.graph_block(gb, bufs["delta"], gi)))
        xb = bufs["x_out"][lo:hi_]
        lay_diff = float((res - xb).abs().max().item() / max(1.0, res.abs().max().item()))
        assert same_bits and lay_diff <= 1e-2, (same_bits, lay_diff)
        plain = dict(value=G / (plain_ms / 1e3), unit="subgraphs/s", ms=plain_ms, wall_s=plain_wall,
                     abi_calls_per_subgraph=2 + STRESS_ITERS, dppr_delta_identical=same_bits,
                     layout_rel_diff_vs_batched=lay_diff)
        log(f"plain: {plain_ms:.1f} ms -> {plain['value']:.1f} subgraphs/s; batched/plain = "
            f"{value / plain['value']:.2f}x; dppr/delta identical={same_bits}, layout rel diff {lay_diff:.2e}")
        del csrs

    spmm = None
    if not args.no_spmm:
        spmm = spmm_all_pairs(ops, dev)
        log(f"all-pairs SpMM (n = 20000): {spmm['ms']:.1f} ms, {spmm['achieved']:.0f} GB/s algorithmic; PDist "
            f"{spmm['pdist']['ms']:.2f} ms; {spmm['layout']['sweeps']} sweeps {spmm['layout']['ms']:.1f} ms "
            f"({spmm['layout']['achieved']:.0f} GB/s), stress {spmm['layout']['stress_before']:.4g} -> "
            f"{spmm['layout']['stress_after']:.4g}")

    spmm_big = None
    gfp = None
    gbp = None
    tau = None
    exact = None
    metrics = None
    if not args.no_spmm_large:
        del bufs
        plan.close()
        plan = None
        torch.cuda.empty_cache()
        spmm_big, (g_big, csr_big, delta_big, src_big) = spmm_large(ops, dev)
        log(f"4096-source SpMM (n = 10^6): {spmm_big['ms']:.1f} ms, {spmm_big['achieved']:.0f} GB/s algorithmic")
        x_exact, exact = layout_exact_leg(ops, dev, delta_big, cpu=not args.no_cpu_baseline)
        log(f"exact majorization step (k = 4096): {exact['ms']:.2f} ms, {exact['cg_iters']} CG iterations, "
            f"{exact['achieved']:.0f} GB/s algorithmic; stress {exact['stress_before']:.10g} -> {exact['stress_after']:.10g}")
        metrics = layout_metrics_leg(ops, dev, x_exact, g_big, src_big)
        log(f"layout metrics (k = 4096): ND {metrics['nd']:.6g}, ULCV {metrics['ulcv']:.4f}, {metrics['ms']:.2f} ms")
        del delta_big
        if not args.no_gfp:
            torch.cuda.empty_cache()
            gfp = gfp_level(ops, dev, g_big, csr_big, cpu=not args.no_cpu_baseline)
            log(f"level-l DPPR by group forward push (n = 10^6, k = 25): {gfp['ms']:.2f} ms, "
                f"{gfp['rounds']} rounds, {gfp['achieved']:.0f} GB/s algorithmic")
            gbp = gbp_level(ops, dev, g_big, csr_big)
            log(f"level-l DPPR by group backward push (n = 10^6, 25 targets): {gbp['ms']:.2f} ms, "
                f"{gbp['rounds']} rounds, {gbp['achieved']:.0f} GB/s algorithmic")
            tau = tau_push_hubs(ops, dev)
            log(f"Tau-Push, 25 hub supernodes (n = 20000): {tau['ms']:.2f} ms, {tau['backward_targets']} refined "
                f"backward, rounds {tau['forward_rounds']} + {tau['backward_rounds']}")
        del g_big, csr_big

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample ...")
        cpu = cpu_baseline(graphs)
        log(f"oracle: {cpu['value']:.4f} subgraphs/s ({cpu['seconds']:.1f}s wall, {cpu['cores']} processes, "
            f"{cpu['cpu_model']})")

    out = {
        "metric": "subgraphs laid out/sec (batched vs plain, same GPU) at PPR err<=1e-6; SpMM HBM GB/s",
        "value": value,
        "unit": "subgraphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SBM subgraphs; no dataset)",
        "config": {"workload": f"sbm_batch_{G}: {G} SBM subgraphs, n log-uniform [32,2048], 4-16 blocks, "
                               f"p_in 0.2, p_out 0.01; all-pairs PPR alpha 0.15 to L1 1e-6 (T={T}), PDist, "
                               f"{STRESS_ITERS} Jacobi stress sweeps; one HIP-graph replay per step",
                   "subgraphs": G, "nodes": int(sizes.sum()), "pairs": int((sizes ** 2).sum()),
                   "pushes": T, "stress_iters": STRESS_ITERS},
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "roofline": roof,
        "stages": stages,
        "spmm": spmm,
        "spmm_large": spmm_big,
        "level_dppr_gfp": gfp,
        "level_dppr_gbp": gbp,
        "tau_push": tau,
        "layout_exact": exact,
        "layout_exact_batch": batch_exact,
        "layout_metrics": metrics,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if plan is not None:
        plan.close()


if __name__ == "__main__":
    main()
