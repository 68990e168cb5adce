"""torch.autograd.Function over K unrolled iterations of the lifted solver.

The forward pass creates a problem on the GPU from (f, lambda, w), runs K iterations of
the primal-dual method (Sec. 4) with a checkpoint every C iterations and returns the
read-out u. The backward pass is the hand-written adjoint of those iterations
(sl_unrolled_backward): gradients with respect to the data image f, the TV weight lambda
and the per-label additive values w of the data term, for learning data terms. Only
argument marshalling happens here.
"""
from __future__ import annotations

import numpy as np

from . import RHO_TRUNC_QUAD, Problem


def _torch():
    import torch
    return torch


def _make_function():
    torch = _torch()

    class UnrolledSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f, lam, w, gamma, rho, a, nu, K, C, normalize):
            gamma = np.asarray(gamma, dtype=np.float64)
            H, W = f.shape
            prob = Problem(H, W, gamma, rho, float(lam), f=f.detach(), a=a, nu=nu,
                           tau=gamma if w is not None else None,
                           samples=w.detach() if w is not None else None,
                           normalize=normalize, device=f.device)
            prob.unrolled_forward(K, C)
            _, u = prob.read_u()
            ctx.prob = prob
            ctx.lam_meta = (lam.dtype, lam.device, lam.shape) if torch.is_tensor(lam) else None
            ctx.has_w = w is not None
            return u

        @staticmethod
        def backward(ctx, gu):
            prob = ctx.prob
            if prob is None:
                raise RuntimeError("unrolled_solve supports one backward pass per forward pass "
                                   "(its checkpoints are released after it); run the forward "
                                   "again instead of retain_graph=True")
            need_f, need_lam, need_w = ctx.needs_input_grad[:3]
            gf, gl, gw = prob.unrolled_backward(gu.contiguous(), want_f=need_f,
                                                want_w=need_w and ctx.has_w)
            prob.close()
            ctx.prob = None
            glam = None
            if need_lam and ctx.lam_meta is not None:
                dt, dev, shape = ctx.lam_meta
                glam = torch.full(shape, gl, dtype=dt, device=dev)
            return gf, glam, gw, None, None, None, None, None, None, None

    return UnrolledSolve


_FN = None


def unrolled_solve(f, lam, w=None, gamma=None, rho: int = RHO_TRUNC_QUAD, a: float = 2.0,
                   nu: float = 0.025, K: int = 200, C: int = 20, normalize: bool = True):
    """Read-out u [H, W] after K unrolled iterations; differentiable in f [H, W] (float32,
    on the GPU), lam (0-dim tensor or float) and w [L, H, W] (additive values, optional).
    ``gamma`` are the L labels (default: 8 equispaced on [0, 1])."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    if gamma is None:
        gamma = np.linspace(0.0, 1.0, 8)
    return _FN.apply(f, lam, w, gamma, rho, a, nu, K, C, normalize)
