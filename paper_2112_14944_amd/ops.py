"""Python binding of the C ABI: argument marshalling only.

PyTorch supplies device memory and the current stream; every step of the
computation runs in libpprviz.so.  Function names follow include/pprviz.h.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("pprviz ops take device tensors")


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Csr:
    """Symmetric CSR on the device (int32 row_ptr/col_idx, optional FP32
    arc weights)."""
    n: int
    nnz: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    weight: torch.Tensor | None = None

    @staticmethod
    def from_graph(g, device="cuda", weighted=None):
        use_w = (g.arc_weight is not None) if weighted is None else weighted
        rp = torch.as_tensor(np.ascontiguousarray(g.row_ptr), device=device)
        ci = torch.as_tensor(np.ascontiguousarray(g.col_idx), device=device)
        w = torch.as_tensor(np.ascontiguousarray(g.arc_weight), device=device) if use_w else None
        return Csr(g.n, g.nnz, rp, ci, w)

    def with_weight(self, w):
        return Csr(self.n, self.nnz, self.row_ptr, self.col_idx, w)

    def c(self):
        return L.ppr_csr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.weight))


def pushes_for_tolerance(alpha, tol, max_iter):
    T = C.c_int32()
    conv = C.c_int32()
    L.check("pprviz_pushes_for_tolerance",
            L.lib().pprviz_pushes_for_tolerance(alpha, tol, max_iter, C.byref(T), C.byref(conv)))
    return T.value, bool(conv.value)


def ppr_matrix(g: Csr, src, tgt=None, alpha=0.15, tol=1e-6, max_iter=100000, want_ppr=True, want_dppr=True,
               check_residual=False, allow_noconv=False):
    """pi_hat(src[i], tgt[j]) (and d(src[i]) times it), FP32 [n_src, n_tgt].
    Returns (ppr, dppr, pushes, resid) with resid an FP64 numpy array when
    check_residual is set (that synchronizes)."""
    dev = g.row_ptr.device
    src = torch.as_tensor(src, dtype=torch.int32, device=dev).contiguous()
    n_src = int(src.numel())
    if tgt is not None:
        tgt = torch.as_tensor(tgt, dtype=torch.int32, device=dev).contiguous()
        n_tgt = int(tgt.numel())
    else:
        n_tgt = g.n
    cg = g.c()
    ws = _ws(L.lib().ppr_matrix_workspace(C.byref(cg), n_src, n_tgt), dev)
    ppr = torch.empty((n_src, n_tgt), dtype=torch.float32, device=dev) if want_ppr else None
    dppr = torch.empty((n_src, n_tgt), dtype=torch.float32, device=dev) if want_dppr else None
    resid = np.zeros(max(n_src, 1), dtype=np.float64) if check_residual else None
    iters = C.c_int32()
    st = L.lib().ppr_matrix(C.byref(cg), _ptr(src), n_src, _ptr(tgt), n_tgt, alpha, tol, max_iter, _ptr(ppr),
                            _ptr(dppr), resid.ctypes.data_as(C.POINTER(C.c_double)) if resid is not None else None,
                            C.byref(iters), _ptr(ws), ws.numel(), _stream(dev))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("ppr_matrix", st, allow)
    return ppr, dppr, iters.value, (resid[:n_src] if resid is not None else None)


def ppr_matrix_noalloc(g: Csr, src, tgt=None, alpha=0.15, tol=1e-6, max_iter=100000, ppr=None, dppr=None,
                       check_residual=False, allow_noconv=False):
    """ppr_matrix through the entry point that allocates nothing: the library
    takes its workspace from its own per-GPU scratch array.  ``ppr`` and
    ``dppr`` are caller-owned [n_src, n_tgt] FP32 outputs (either may be
    None).  Returns (pushes, resid)."""
    dev = g.row_ptr.device
    src = torch.as_tensor(src, dtype=torch.int32, device=dev).contiguous()
    n_src = int(src.numel())
    if tgt is not None:
        tgt = torch.as_tensor(tgt, dtype=torch.int32, device=dev).contiguous()
        n_tgt = int(tgt.numel())
    else:
        n_tgt = g.n
    for o in (ppr, dppr):
        if o is not None:
            assert o.shape == (n_src, n_tgt) and o.dtype == torch.float32 and o.is_contiguous() and o.is_cuda
    cg = g.c()
    resid = np.zeros(max(n_src, 1), dtype=np.float64) if check_residual else None
    iters = C.c_int32()
    st = L.lib().ppr_matrix_noalloc(C.byref(cg), _ptr(src), n_src, _ptr(tgt), n_tgt, alpha, tol, max_iter,
                                    _ptr(ppr), _ptr(dppr),
                                    resid.ctypes.data_as(C.POINTER(C.c_double)) if resid is not None else None,
                                    C.byref(iters), _stream(dev))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("ppr_matrix_noalloc", st, allow)
    return iters.value, (resid[:n_src] if resid is not None else None)


def gfp_level_dppr(g: Csr, leaves, alpha=0.15, r_max=0.0, max_rounds=10000, want_est=False, want_resid=False,
                   allow_noconv=False):
    """Level-l DPPR between supernodes by Group Forward-Push in rounds.
    ``leaves`` is a list of k node-id arrays (the leaf sets) or a pair
    (leaf_ptr, leaf_idx).  Returns (dppr [k, k], est [k, n] or None,
    resid [k, n] or None, rounds, status)."""
    dev = g.row_ptr.device
    if isinstance(leaves, tuple):
        ptr, idx = leaves
    else:
        sizes = [len(F) for F in leaves]
        ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        idx = np.concatenate([np.asarray(F, dtype=np.int32) for F in leaves]) if leaves else np.zeros(0, np.int32)
    ptr = torch.as_tensor(ptr, dtype=torch.int32, device=dev).contiguous()
    idx = torch.as_tensor(idx, dtype=torch.int32, device=dev).contiguous()
    k = int(ptr.numel()) - 1
    cg = g.c()
    ws = _ws(L.lib().gfp_workspace(C.byref(cg), k, max_rounds), dev)
    out = torch.empty((k, k), dtype=torch.float32, device=dev)
    est = torch.empty((k, g.n), dtype=torch.float32, device=dev) if want_est else None
    resid = torch.empty((k, g.n), dtype=torch.float32, device=dev) if want_resid else None
    rounds = C.c_int32()
    st = L.lib().gfp_level_dppr(C.byref(cg), _ptr(ptr), _ptr(idx), k, int(idx.numel()), alpha, r_max, max_rounds,
                                _ptr(out), _ptr(est), _ptr(resid), C.byref(rounds), _ptr(ws), ws.numel(),
                                _stream(dev))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("gfp_level_dppr", st, allow)
    return out, est, resid, rounds.value, st


def _leaf_lists(leaves, dev):
    if isinstance(leaves, tuple):
        ptr, idx = leaves
    else:
        sizes = [len(F) for F in leaves]
        ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        idx = np.concatenate([np.asarray(F, dtype=np.int32) for F in leaves]) if leaves else np.zeros(0, np.int32)
    ptr = torch.as_tensor(ptr, dtype=torch.int32, device=dev).contiguous()
    idx = torch.as_tensor(idx, dtype=torch.int32, device=dev).contiguous()
    return ptr, idx


def gbp_level_dppr(g: Csr, leaves, targets, rb_max, alpha=0.15, max_rounds=10000, out=None, want_est=False,
                   want_resid=False, allow_noconv=False):
    """Group Backward-Push in rounds towards the target supernodes `targets`
    with per-target thresholds `rb_max`.  Writes the target columns of `out`
    (a [k, k] tensor, zeros when not given).  Returns (out, est [t, n] or None,
    resid [t, n] or None, rounds, status)."""
    dev = g.row_ptr.device
    ptr, idx = _leaf_lists(leaves, dev)
    k = int(ptr.numel()) - 1
    tg = torch.as_tensor(targets, dtype=torch.int32, device=dev).contiguous()
    th = torch.as_tensor(rb_max, dtype=torch.float32, device=dev).reshape(-1).expand(tg.numel()).contiguous()
    t = int(tg.numel())
    cg = g.c()
    ws = _ws(L.lib().gfp_workspace(C.byref(cg), k, max_rounds), dev)
    out = torch.zeros((k, k), dtype=torch.float32, device=dev) if out is None else out
    est = torch.empty((t, g.n), dtype=torch.float32, device=dev) if want_est else None
    resid = torch.empty((t, g.n), dtype=torch.float32, device=dev) if want_resid else None
    rounds = C.c_int32()
    st = L.lib().gbp_level_dppr(C.byref(cg), _ptr(ptr), _ptr(idx), k, int(idx.numel()), _ptr(tg), t, _ptr(th),
                                alpha, max_rounds, _ptr(out), _ptr(est), _ptr(resid), C.byref(rounds), _ptr(ws),
                                ws.numel(), _stream(dev))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("gbp_level_dppr", st, allow)
    return out, est, resid, rounds.value, st


def tau_push_level_dppr(g: Csr, leaves, alpha=0.15, eps=1 - 1 / math.e, delta=None, tau=0.0, max_rounds=10000,
                        allow_noconv=False):
    """Tau-Push: forward pushes from every supernode, backward refinement of
    the targets whose DNPR exceeds tau (1/sqrt(kn) when tau <= 0).  delta
    defaults to 1/(10k).  Returns (dppr [k, k], targets refined, (forward
    rounds, backward rounds), status)."""
    dev = g.row_ptr.device
    ptr, idx = _leaf_lists(leaves, dev)
    k = int(ptr.numel()) - 1
    delta = 1.0 / (10 * k) if delta is None else delta
    cg = g.c()
    ws = _ws(L.lib().gfp_workspace(C.byref(cg), k, max_rounds), dev)
    out = torch.empty((k, k), dtype=torch.float32, device=dev)
    nb = C.c_int32()
    rounds = (C.c_int32 * 2)()
    st = L.lib().tau_push_level_dppr(C.byref(cg), _ptr(ptr), _ptr(idx), k, int(idx.numel()), alpha, eps, delta,
                                     tau, max_rounds, _ptr(out), C.byref(nb), rounds, _ptr(ws), ws.numel(),
                                     _stream(dev))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("tau_push_level_dppr", st, allow)
    return out, nb.value, (rounds[0], rounds[1]), st


def pdist(dppr: torch.Tensor, n_clamp: int):
    _require_cuda(dppr)
    k = dppr.shape[0]
    assert dppr.shape == (k, k) and dppr.dtype == torch.float32 and dppr.is_contiguous()
    out = torch.empty_like(dppr)
    L.check("pdist", L.lib().pdist(_ptr(dppr), k, int(n_clamp), _ptr(out), _stream(dppr.device)))
    return out


def pdist_backward(dppr, grad_delta, n_clamp):
    _require_cuda(dppr, grad_delta)
    k = dppr.shape[0]
    out = torch.empty_like(dppr)
    L.check("pdist_backward", L.lib().pdist_backward(_ptr(dppr), _ptr(grad_delta.contiguous()), k, int(n_clamp),
                                                      _ptr(out), _stream(dppr.device)))
    return out


def _check_layout(delta, x):
    _require_cuda(delta, x)
    k = x.shape[0]
    assert x.shape == (k, 2) and x.dtype == torch.float32 and x.is_contiguous()
    assert delta.shape == (k, k) and delta.dtype == torch.float32 and delta.is_contiguous()
    return k


def stress_eval(delta, x):
    """Eq. eq:loss as a device FP64 scalar tensor."""
    k = _check_layout(delta, x)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    ws = _ws(L.lib().layout_workspace(k), x.device)
    L.check("stress_eval", L.lib().stress_eval(_ptr(delta), k, _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                                                _stream(x.device)))
    return out


def layout_step(delta, x, with_stress=False, out=None, ws=None):
    """One Jacobi majorization sweep; returns (x_next, stress_of_x or None)."""
    k = _check_layout(delta, x)
    xo = torch.empty_like(x) if out is None else out
    st_out = torch.empty(1, dtype=torch.float64, device=x.device) if with_stress else None
    if ws is None:
        ws = _ws(L.lib().layout_workspace(k), x.device)
    L.check("layout_step", L.lib().layout_step(_ptr(delta), k, _ptr(x), _ptr(xo), _ptr(st_out), _ptr(ws),
                                                ws.numel(), _stream(x.device)))
    return xo, st_out


def layout(delta, x0, steps):
    """`steps` Jacobi sweeps from x0 (one launch per sweep)."""
    k = _check_layout(delta, x0)
    ws = _ws(L.lib().layout_workspace(k), x0.device)
    a = x0.clone()
    b = torch.empty_like(x0)
    for _ in range(steps):
        layout_step(delta, a, out=b, ws=ws)
        a, b = b, a
    return a


def layout_metrics(x, g: Csr | None = None):
    """(ND, ULCV) of a layout; ULCV is None without a graph."""
    _require_cuda(x)
    k = x.shape[0]
    assert x.shape == (k, 2) and x.dtype == torch.float32 and x.is_contiguous()
    ws = _ws(L.lib().layout_metrics_workspace(k), x.device)
    nd = C.c_double()
    ul = C.c_double()
    cg = g.c() if g is not None else None
    st = L.lib().layout_metrics(_ptr(x), k, C.byref(cg) if cg is not None else None, C.byref(nd),
                                C.byref(ul) if g is not None else None, _ptr(ws), ws.numel(), _stream(x.device))
    L.check("layout_metrics", st)
    return nd.value, (ul.value if g is not None else None)


def layout_step_exact(delta, x, cg_tol=1e-6, cg_max_iter=1000, out=None, allow_noconv=False):
    """The exact (Guttman) stress-majorization step by conjugate gradients.
    Returns (x_out [k, 2], CG iterations)."""
    _check_layout(delta, x)
    k = delta.shape[0]
    out = torch.empty_like(x) if out is None else out
    ws = _ws(L.lib().layout_exact_workspace(k), delta.device)
    iters = C.c_int32()
    st = L.lib().layout_step_exact(_ptr(delta), k, _ptr(x), _ptr(out), cg_tol, cg_max_iter, C.byref(iters),
                                   _ptr(ws), ws.numel(), _stream(delta.device))
    allow = (L.PPR_OK, L.PPR_ENOCONV) if allow_noconv else (L.PPR_OK,)
    L.check("layout_step_exact", st, allow)
    return out, iters.value


def stress_backward(delta, x, grad_scale=1.0, want_grad_x=True, want_grad_delta=True):
    k = _check_layout(delta, x)
    gx = torch.empty_like(x) if want_grad_x else None
    gd = torch.empty_like(delta) if want_grad_delta else None
    L.check("stress_backward", L.lib().stress_backward(_ptr(delta), k, _ptr(x), float(grad_scale), _ptr(gx),
                                                        _ptr(gd), _stream(x.device)))
    return gx, gd


def ppr_matrix_backward(g: Csr, alpha, T, ppr, grad_dppr):
    """dLoss/dw per arc (each arc carries the gradient of its undirected
    edge's shared weight)."""
    dev = g.row_ptr.device
    cg = g.c()
    ws = _ws(L.lib().ppr_backward_workspace(C.byref(cg), 1 if ppr is None else 0), dev)
    out = torch.empty(g.nnz, dtype=torch.float32, device=dev)
    L.check("ppr_matrix_backward", L.lib().ppr_matrix_backward(C.byref(cg), alpha, int(T), _ptr(ppr),
                                                                _ptr(grad_dppr.contiguous()), _ptr(out), _ptr(ws),
                                                                ws.numel(), _stream(dev)))
    return out


# ------------------------------------------------------------------ batch

class Batch:
    """Device copy of a disjoint union of subgraphs (unit weights)."""

    def __init__(self, gb, device="cuda"):
        self.gb = gb
        self.device = device
        self.node_off = torch.as_tensor(gb.node_off, device=device)
        self.row_ptr = torch.as_tensor(gb.row_ptr, device=device)
        self.col_idx = torch.as_tensor(gb.col_idx, device=device)
        self.mat_off = torch.as_tensor(gb.mat_off, device=device)
        self.n_graphs = len(gb.graphs)
        self.n_nodes = int(gb.node_off[-1])
        self.nnz = int(gb.col_idx.shape[0])
        self.max_n = int(gb.sizes.max())
        self.pool = int(gb.mat_off[-1])

    def c(self):
        return L.ppr_batch(self.n_graphs, self.n_nodes, self.nnz, self.max_n, self.pool, _ptr(self.node_off),
                           _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.mat_off))

    def buffers(self, x0):
        dev = self.device
        cb = self.c()
        return dict(
            x0=x0.contiguous(),
            x_out=torch.empty_like(x0),
            dppr=torch.empty(self.pool, dtype=torch.float32, device=dev),
            delta=torch.empty(self.pool, dtype=torch.float32, device=dev),
            stress=torch.empty(self.n_graphs, dtype=torch.float64, device=dev),
            ws=_ws(L.lib().pprviz_batch_workspace(C.byref(cb)), dev),
        )


def batch_max_n():
    return int(L.lib().pprviz_batch_max_n())


def batch_step_exact(batch: "Batch", delta_pool, x, cg_tol=1e-6, cg_max_iter=1000, out=None):
    """The exact (Guttman) step of every subgraph of a batch, one block per
    subgraph.  ``delta_pool`` is the PDist pool pprviz_batch writes, ``x``
    the positions [n_nodes, 2].  Returns (x_out, iterations [n_graphs],
    converged [n_graphs]) as device int32 tensors."""
    dev = batch.device
    x = x.contiguous()
    out = torch.empty_like(x) if out is None else out
    iters = torch.empty(batch.n_graphs, dtype=torch.int32, device=dev)
    conv = torch.empty(batch.n_graphs, dtype=torch.int32, device=dev)
    cb = batch.c()
    L.check("pprviz_batch_step_exact",
            L.lib().pprviz_batch_step_exact(C.byref(cb), _ptr(delta_pool), _ptr(x), _ptr(out), cg_tol,
                                            cg_max_iter, _ptr(iters), _ptr(conv), _stream(dev)))
    return out, iters, conv


def pprviz_batch(b: Batch, bufs, alpha=0.15, tol=1e-6, max_iter=100000, stress_iters=200):
    cb = b.c()
    st = L.lib().pprviz_batch(C.byref(cb), alpha, tol, max_iter, stress_iters, _ptr(bufs["x0"]), _ptr(bufs["x_out"]),
                              _ptr(bufs["dppr"]), _ptr(bufs["delta"]), _ptr(bufs["stress"]), _ptr(bufs["ws"]),
                              bufs["ws"].numel(), _stream(b.device))
    L.check("pprviz_batch", st)
    return bufs


def pprviz_batch_profile(b: Batch, bufs, alpha=0.15, tol=1e-6, max_iter=100000, stress_iters=200):
    """Eager batched run with HIP events between stages; returns the stage
    times in ms: (planning, ppr, pdist, layout)."""
    cb = b.c()
    ms = (C.c_double * 4)()
    st = L.lib().pprviz_batch_profile(C.byref(cb), alpha, tol, max_iter, stress_iters, _ptr(bufs["x0"]),
                                      _ptr(bufs["x_out"]), _ptr(bufs["dppr"]), _ptr(bufs["delta"]),
                                      _ptr(bufs["stress"]), _ptr(bufs["ws"]), bufs["ws"].numel(), _stream(b.device),
                                      ms)
    L.check("pprviz_batch_profile", st)
    return tuple(ms)


class BatchPlan:
    """The batched pipeline captured once into a HIP graph; launch() replays it."""

    def __init__(self, b: Batch, bufs, alpha=0.15, tol=1e-6, max_iter=100000, stress_iters=200):
        self.b = b
        self.bufs = bufs
        self._cb = b.c()
        h = C.c_void_p()
        st = L.lib().pprviz_batch_plan_create(C.byref(self._cb), alpha, tol, max_iter, stress_iters,
                                              _ptr(bufs["x0"]), _ptr(bufs["x_out"]), _ptr(bufs["dppr"]),
                                              _ptr(bufs["delta"]), _ptr(bufs["stress"]), _ptr(bufs["ws"]),
                                              bufs["ws"].numel(), _stream(b.device), C.byref(h))
        L.check("pprviz_batch_plan_create", st)
        self.handle = h

    def launch(self):
        L.check("pprviz_batch_plan_launch", L.lib().pprviz_batch_plan_launch(self.handle, _stream(self.b.device)))

    def close(self):
        if self.handle:
            L.lib().pprviz_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_block(gb, pool, g):
    """Graph g's n_g x n_g block of a flat pool tensor."""
    n = int(gb.node_off[g + 1] - gb.node_off[g])
    a = int(gb.mat_off[g])
    return pool[a:a + n * n].view(n, n)

