"""torch.autograd.Function over the C ABI: stress of the PDist layout as a
function of the edge weights and the node coordinates.

forward:  ppr_matrix (all pairs, fixed T) -> pdist -> stress_eval
backward: stress_backward -> pdist_backward -> ppr_matrix_backward
The two n x n PPR matrices are kept for backward when they fit the given
byte budget; otherwise backward recomputes them (activation checkpointing).
"""
from __future__ import annotations

import torch

from . import ops


class PPRLayoutLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, edge_weight, x, csr, arc_edge, edge_arc, alpha, T, n_clamp, save_budget_bytes):
        w_arc = edge_weight[arc_edge].contiguous()
        g = csr.with_weight(w_arc)
        n = g.n
        ppr, dppr, _, _ = ops.ppr_matrix(g, torch.arange(n, dtype=torch.int32, device=x.device), alpha=alpha,
                                         tol=0.0, max_iter=T)
        delta = ops.pdist(dppr, n_clamp)
        loss = ops.stress_eval(delta, x)
        keep = 2 * n * n * 4 <= save_budget_bytes
        ctx.g = g
        ctx.alpha, ctx.T, ctx.n_clamp = alpha, T, n_clamp
        ctx.edge_arc = edge_arc
        ctx.recomputed = not keep
        if keep:
            ctx.save_for_backward(x, delta, ppr, dppr)
        else:
            del ppr, dppr
            ctx.save_for_backward(x, delta)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_loss):
        saved = ctx.saved_tensors
        x, delta = saved[0], saved[1]
        g = ctx.g
        if len(saved) == 4:
            ppr, dppr = saved[2], saved[3]
        else:
            n = g.n
            ppr, dppr, _, _ = ops.ppr_matrix(g, torch.arange(n, dtype=torch.int32, device=x.device),
                                             alpha=ctx.alpha, tol=0.0, max_iter=ctx.T)
        scale = float(grad_loss)
        gx, gd = ops.stress_backward(delta, x, grad_scale=scale)
        gpid = ops.pdist_backward(dppr, gd, ctx.n_clamp)
        garc = ops.ppr_matrix_backward(g, ctx.alpha, ctx.T, ppr, gpid)
        gw = garc[ctx.edge_arc]
        return gw, gx, None, None, None, None, None, None, None


def edge_maps(graph, device):
    """arc -> undirected edge index, and one arc per edge (the u < v arc)."""
    arc_edge = torch.as_tensor(graph.arc_edge, device=device)
    rows = torch.repeat_interleave(torch.arange(graph.n), torch.as_tensor(graph.row_ptr[1:] - graph.row_ptr[:-1]).long())
    cols = torch.as_tensor(graph.col_idx).long()
    fwd = torch.nonzero(rows < cols).flatten()
    edge_arc = torch.empty(graph.m_und, dtype=torch.long)
    edge_arc[torch.as_tensor(graph.arc_edge)[fwd]] = fwd
    return arc_edge, edge_arc.to(device)


def pprviz_loss(edge_weight, x, csr, arc_edge, edge_arc, alpha=0.15, T=100, n_clamp=None,
                save_budget_bytes=8 << 30):
    n_clamp = csr.n if n_clamp is None else n_clamp
    return PPRLayoutLoss.apply(edge_weight, x, csr, arc_edge, edge_arc, alpha, T, n_clamp, save_budget_bytes)
