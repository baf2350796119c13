"""Differentiable solve map (b, tau) -> x* behind torch.autograd.Function.

forward runs the HIP solver and keeps its final interior point (z, s);
backward runs the HIP adjoint: one PCG solve of
(Theta^{-1} + F F^T) w = [g; -g] at that point (Theta, P frozen), then
dL/db = A (w_u - w_v) and dL/dtau = -1^T w.  tau is treated as an
independent input.
"""
from __future__ import annotations

import numpy as np
import torch

from .mfipm import Solver


class SolveStatusError(RuntimeError):
    """An instance of a forward or adjoint solve did not end with status 0."""

    def __init__(self, where, bad):
        super().__init__(f"{where}: instances not converged: {bad}")
        self.where = where
        self.bad = bad


def _raise_on_status(where, infos):
    bad = [(j, i["status_name"]) for j, i in enumerate(infos) if i["status"] != 0]
    if bad:
        raise SolveStatusError(where, bad)


class MfipmSolve(torch.autograd.Function):
    """x = MfipmSolve.apply(b, tau, solver, A, rows, n) for a single instance,
    or a batch when b is 2-D (B x m) and tau is 1-D (B): all instances share
    the operator (dense A or rows of the partial DCT)."""

    @staticmethod
    def forward(ctx, b, tau, solver: Solver, A=None, rows=None, n=None):
        batched = b.dim() == 2
        bb = b if batched else b.unsqueeze(0)
        B, m = bb.shape
        nn = A.shape[1] if A is not None else int(n)
        n_off = np.arange(B + 1, dtype=np.int64) * nn
        m_off = np.arange(B + 1, dtype=np.int64) * m
        taus = tau.detach().reshape(-1).double().cpu().numpy()
        if taus.size == 1 and B > 1:
            taus = np.full(B, float(taus[0]))
        res = solver.solve_batched(bb.detach().reshape(-1), taus, n_off, m_off, A_packed=A, rows=rows,
                                   shared_op=True)
        _raise_on_status("forward", res.infos)
        ctx.solver = solver
        ctx.A, ctx.rows = A, rows
        ctx.n_off, ctx.m_off = n_off, m_off
        ctx.batched = batched
        ctx.tau_shape = tau.shape
        ctx.save_for_backward(res.state)
        ctx.infos = res.infos
        x = res.x.view(B, nn)
        return x if batched else x[0]

    @staticmethod
    def backward(ctx, grad_x):
        (state,) = ctx.saved_tensors
        g = grad_x if ctx.batched else grad_x.unsqueeze(0)
        gb, gt, binf = ctx.solver.backward(state, g.contiguous().reshape(-1), ctx.n_off, ctx.m_off,
                                           A_packed=ctx.A, rows=ctx.rows, shared_op=True)
        _raise_on_status("backward", binf)
        B = g.shape[0]
        gb = gb.view(B, -1)
        if not ctx.batched:
            gb = gb[0]
            gt = gt.reshape(ctx.tau_shape)
        else:
            gt = gt.reshape(ctx.tau_shape) if len(ctx.tau_shape) else gt.sum()
        return gb, gt, None, None, None, None


def solve(b, tau, solver: Solver, A=None, rows=None, n=None):
    return MfipmSolve.apply(b, tau, solver, A, rows, n)
