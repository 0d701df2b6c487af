"""Differentiable projector and unrolled SPGM on top of the C ABI.

* :class:`ProjectorFn` -- ``y = A_B s`` (Sec. II, Eq. 1 on the minibatch rows); its backward is
  the adjoint ``A_B^H ybar`` (``spgm_adjoint``).
* :class:`AdjointFn`   -- ``g = A_B^H r``; its backward is ``A_B gbar`` (``spgm_forward``).
* :class:`UnrolledSPGMFn` -- K iterations of Eq. 5 with the minibatch gradient of Eq. 6 and
  per-iteration step sizes ``eta_k`` and thresholds ``tau_k`` as differentiable parameters:
      s_{k+1} = S_{tau_k}( s_k - (eta_k/B) A_k^H (A_k s_k - y_k) ).
  The forward pass keeps only checkpoints of the iterate (every ``checkpoint_every``
  iterations, default ceil(sqrt(K))); the backward pass recomputes one segment at a time with
  ``spgm_step_grad`` (the iterate and the gradient A_k^H (A_k s_k - y_k) at it) and runs the
  native backward step ``spgm_unrolled_vjp_step_g``, which forms entries only for
  A_k^H A_k zbar: four entry passes per iteration, and O(sqrt(K) N) memory instead of O(K N).

Complex gradients follow PyTorch's convention for real losses (dL/dRe + j dL/dIm).  Tensors
are complex64 / int32 on the plan's device; every arithmetic step runs in the library.
"""
from __future__ import annotations

import math

import torch


class ProjectorFn(torch.autograd.Function):
    """y = A_B s for minibatch ``rows``."""

    @staticmethod
    def forward(ctx, s, plan, rows):
        ctx.plan, ctx.rows = plan, rows
        return plan.spgm_forward(rows, s.contiguous())

    @staticmethod
    def backward(ctx, ybar):
        return ctx.plan.spgm_adjoint(ctx.rows, ybar.contiguous()), None, None


class AdjointFn(torch.autograd.Function):
    """g = A_B^H r for minibatch ``rows``."""

    @staticmethod
    def forward(ctx, r, plan, rows):
        ctx.plan, ctx.rows = plan, rows
        return plan.spgm_adjoint(rows, r.contiguous())

    @staticmethod
    def backward(ctx, gbar):
        return ctx.plan.spgm_forward(ctx.rows, gbar.contiguous()), None, None


def projector(plan, rows, s):
    return ProjectorFn.apply(s, plan, rows)


def adjoint(plan, rows, r):
    return AdjointFn.apply(r, plan, rows)


class UnrolledSPGMFn(torch.autograd.Function):
    """s_K of K unrolled SPGM iterations; differentiable in s0, eta (K,) and tau (K,)."""

    @staticmethod
    def forward(ctx, y, s0, eta, tau, plan, rows_table, checkpoint_every=None):
        K = rows_table.shape[0]
        if eta.numel() != K or tau.numel() != K:
            raise ValueError("eta and tau need one value per iteration")
        c = checkpoint_every or max(1, int(math.ceil(math.sqrt(K))))
        eta_h = [float(v) for v in eta.detach().cpu().tolist()]
        tau_h = [float(v) for v in tau.detach().cpu().tolist()]
        y = y.contiguous()
        s = s0.detach().contiguous().clone()
        ckpts = {0: s.clone()}
        for k in range(K):
            plan.spgm_step(rows_table[k], y, s, eta_h[k], tau_h[k])
            if (k + 1) % c == 0 and k + 1 < K:
                ckpts[k + 1] = s.clone()
        ctx.plan, ctx.rows, ctx.c = plan, rows_table, c
        ctx.eta_h, ctx.tau_h = eta_h, tau_h
        ctx.ckpts = ckpts
        ctx.save_for_backward(y)
        ctx.param_meta = (eta.dtype, eta.device, tau.dtype, tau.device)
        return s

    @staticmethod
    def backward(ctx, sbar_out):
        (y,) = ctx.saved_tensors
        plan, rows, c = ctx.plan, ctx.rows, ctx.c
        K = rows.shape[0]
        dev = y.device
        sbar = sbar_out.contiguous().clone()
        eta_bar = torch.zeros(K, dtype=torch.float64, device=dev)
        tau_bar = torch.zeros(K, dtype=torch.float64, device=dev)
        for start in sorted(ctx.ckpts, reverse=True):
            end = min(K, start + c)
            # recompute the iterates s_start .. s_{end-1} of this segment and the gradient
            # A_k^H (A_k s_k - y_k) at each of them (the last step's new iterate is not needed)
            states, grads = [ctx.ckpts[start]], []
            for k in range(start, end):
                nxt = states[-1].clone()
                g = torch.empty_like(nxt)
                plan.spgm_step_grad(rows[k], y, nxt, ctx.eta_h[k], ctx.tau_h[k], g)
                grads.append(g)
                if k + 1 < end:
                    states.append(nxt)
            for k in range(end - 1, start - 1, -1):
                plan.spgm_unrolled_vjp_step_g(rows[k], states[k - start], grads[k - start], ctx.eta_h[k],
                                              ctx.tau_h[k], sbar, sbar, eta_bar[k:k + 1], tau_bar[k:k + 1])
        edt, edev, tdt, tdev = ctx.param_meta
        return None, sbar, eta_bar.to(dtype=edt, device=edev), tau_bar.to(dtype=tdt, device=tdev), None, None, None


def unrolled_spgm(plan, rows_table, y, s0, eta, tau, checkpoint_every=None):
    return UnrolledSPGMFn.apply(y, s0, eta, tau, plan, rows_table, checkpoint_every)
