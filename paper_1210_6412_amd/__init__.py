"""Reachability probabilities of discrete-time Markov chains on AMD MI355X.

A HIP library (librp.so, C ABI in include/rp.h) implements the method of
Cormie-Bowins, "A Comparison of Sequential and GPU Implementations of
Iterative Methods to Compute Reachability Probabilities" (GRAPHITE 2012):
the state partition of Section 2.2, the reduced system (I - A) x = b of
Section 2.3, and the Jacobi (Section 3.1) and BiCGStab (Section 3.2)
iterations, with FP32 sweeps inside FP64 iterative refinement, block-diagonal
batching of many chains, and an adjoint gradient.

``binding`` holds the ctypes entry points (same names as the C ABI);
``ReachProb`` wraps a forward solve and its adjoint as a torch autograd
function.  PyTorch supplies device memory and streams only.
"""
from __future__ import annotations

import torch

from . import binding
from .binding import (RP_FP32_REFINED, RP_FP64, RP_PROB0_ONLY, RP_S0, RP_S1, RP_SCHEDULE_SEGSCAN, RP_SQ,
                      RP_STOP_CERTIFIED, RP_STOP_DELTA, RP_STOP_RESIDUAL, RP_TILING_AUTO, RP_TILING_OFF,
                      RP_UPDATE_IN_PLACE, RP_UPDATE_TWO_BUFFER, RpError, rp_adjoint,
                      rp_bicgstab, rp_solve_rhs, rp_matrix_system, rp_context_create, rp_context_destroy, rp_jacobi, rp_last_error, rp_opts_default, rp_precompute,
                      rp_system_destroy, rp_system_export, rp_system_instance_sizes, rp_system_sizes, rp_scc,
                      rp_scc_solve)

__all__ = ["binding", "ReachProb", "reach_prob", "RpError", "rp_adjoint", "rp_bicgstab", "rp_solve_rhs",
           "rp_scc", "rp_scc_solve",
           "rp_matrix_system",
           "rp_context_create",
           "rp_context_destroy", "rp_jacobi", "rp_last_error", "rp_opts_default", "rp_precompute",
           "rp_system_destroy", "rp_system_export", "rp_system_instance_sizes", "rp_system_sizes",
           "RP_FP32_REFINED", "RP_FP64", "RP_PROB0_ONLY", "RP_S0", "RP_S1", "RP_SQ", "RP_STOP_CERTIFIED",
           "RP_STOP_DELTA", "RP_STOP_RESIDUAL", "RP_TILING_AUTO", "RP_TILING_OFF", "RP_SCHEDULE_SEGSCAN",
           "RP_UPDATE_TWO_BUFFER", "RP_UPDATE_IN_PLACE"]


class ReachProb(torch.autograd.Function):
    """x = reachability probabilities of a chain whose stored transition
    probabilities are `values` (structure fixed).  backward() returns
    dL/dP(s, s') = lambda_s x_{s'} on the stored entries, from the adjoint
    solve (I - A)^T lambda = dL/dx."""

    @staticmethod
    def forward(fctx, values, ctx, row_ptr, col, goal_mask, inst_state_offset, method, flags, opts_kw):
        sys = rp_precompute(ctx, row_ptr, col, values.detach().contiguous(), goal_mask, inst_state_offset, flags)
        solve = rp_jacobi if method == 0 else rp_bicgstab
        x, info, code = solve(ctx, sys, **opts_kw)
        if code != binding.RP_OK:
            raise RpError(code, rp_last_error(ctx))
        fctx.sys = sys
        fctx.ctx = ctx
        fctx.method = method
        fctx.opts_kw = opts_kw
        fctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(fctx, grad_x):
        (x,) = fctx.saved_tensors
        kw = dict(fctx.opts_kw)
        kw.pop("x0", None)
        _, g, _, code = rp_adjoint(fctx.ctx, fctx.sys, x, grad_x.contiguous().to(torch.float64), fctx.method, **kw)
        if code != binding.RP_OK:
            raise RpError(code, rp_last_error(fctx.ctx))
        return g, None, None, None, None, None, None, None, None


def reach_prob(values, ctx, row_ptr, col, goal_mask, inst_state_offset=None, method=0, flags=0, **opts):
    """Differentiable reachability probabilities (see ReachProb)."""
    return ReachProb.apply(values, ctx, row_ptr, col, goal_mask, inst_state_offset, method, flags, opts)
