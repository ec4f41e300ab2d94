"""torch.autograd.Function over the Flowtree cost of explicit pairs with the
tree and the flow pattern frozen (ft_flowtree_cost_grad FT_FWD / FT_BWD)."""
from __future__ import annotations

import torch

from . import FT_BWD, FT_FWD, Index, flowtree_cost_grad


def _mass_f64(m):
    """uint32 masses (carried in int32 tensors) as float64."""
    return (m.to(torch.int64) & 0xFFFFFFFF).to(torch.float64)


class FlowtreeCost(torch.autograd.Function):
    """cost[p] = Flowtree(query pair_q[p], doc pair_d[p]), differentiable in
    the coordinates X (V x d) and in the weights w = mass / 2^Q of the query
    CSR (q_w, one per query item) and of the dataset (d_w, one per dataset
    item, in the order the index was built with).  The flow comes from the
    integer masses; q_w and d_w must equal them divided by 2^Q exactly.

    The backward pass repeats the forward launch that saves the flow pattern
    before the gradient launch, so any number of forward calls (on this or
    other pairs) may come between a forward and its backward."""

    @staticmethod
    def forward(ctx, X, q_w, d_w, index: Index, q_off, q_id, q_mass, pair_q, pair_d):
        scale = float(2 ** -index.Q)
        if q_w.numel() != q_mass.numel() or not torch.equal(
                q_w.detach().to(torch.float64), _mass_f64(q_mass) * scale):
            raise ValueError("q_w must equal q_mass / 2^Q")
        if d_w.numel() != index.doc_mass.numel() or not torch.equal(
                d_w.detach().to(torch.float64), _mass_f64(index.doc_mass) * scale):
            raise ValueError("d_w must equal the index's dataset masses / 2^Q")
        cost = torch.empty(pair_q.numel(), dtype=torch.float32, device=X.device)
        flowtree_cost_grad(index, X.detach(), q_off, q_id, q_mass, pair_q, pair_d, FT_FWD, cost=cost)
        ctx.index = index
        ctx.args = (q_off, q_id, q_mass, pair_q, pair_d)
        ctx.save_for_backward(X)
        ctx.q_dtype, ctx.d_dtype = q_w.dtype, d_w.dtype
        ctx.nq = q_w.numel()
        ctx.nd = d_w.numel()
        return cost

    @staticmethod
    def backward(ctx, g):
        (X,) = ctx.saved_tensors
        q_off, q_id, q_mass, pair_q, pair_d = ctx.args
        need = ctx.needs_input_grad
        Xd = X.detach()
        # the index keeps the flow pattern of its latest FT_FWD call only
        scratch = torch.empty(pair_q.numel(), dtype=torch.float32, device=X.device)
        flowtree_cost_grad(ctx.index, Xd, q_off, q_id, q_mass, pair_q, pair_d, FT_FWD, cost=scratch)
        gX = torch.zeros_like(Xd, dtype=torch.float32) if need[0] else None
        gq = torch.zeros(ctx.nq, dtype=torch.float32, device=X.device) if need[1] else None
        gd = torch.zeros(ctx.nd, dtype=torch.float32, device=X.device) if need[2] else None
        flowtree_cost_grad(ctx.index, Xd, q_off, q_id, q_mass, pair_q, pair_d, FT_BWD,
                           grad_out=g.to(torch.float32).contiguous(), grad_X=gX, grad_qmass=gq,
                           grad_dmass=gd)
        if gq is not None:
            gq = gq.to(ctx.q_dtype)
        if gd is not None:
            gd = gd.to(ctx.d_dtype)
        return gX, gq, gd, None, None, None, None, None, None


def flowtree_cost(X, q_w, d_w, index, q_off, q_id, q_mass, pair_q, pair_d):
    return FlowtreeCost.apply(X, q_w, d_w, index, q_off, q_id, q_mass, pair_q, pair_d)
