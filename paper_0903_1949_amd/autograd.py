"""torch.autograd binding of the emergent intensity and its hand-written
adjoint (pprt_emergent_intensity / pprt_formal_solution_vjp; with in-layer
scattering pprt_formal_solution_scattering / pprt_formal_solution_scattering_vjp).

Both directions run in libpprt's kernels; this module only marshals tensors.
The forward keeps layer checkpoints in a workspace tensor saved for the
backward pass, which recomputes each segment of layers from them.
"""
from __future__ import annotations

import torch

from . import pprt


class EmergentIntensity(torch.autograd.Function):
    """Iemerg[b, k, i] = I+(tau_1, mu_i, nu_k) of the omega = 0 formal
    solution, differentiable in q, Sg, Bbot and Bbot_prev (diffusion lower
    boundary) or q, Sg and Ibot (given lower boundary)."""

    @staticmethod
    def forward(ctx, plan: pprt.Plan, checkpoint_interval: int, tau, q, Sg, Bbot, Bbot_prev, Ibot):
        diff = plan.lower_bc == pprt.BC_DIFFUSION
        q, Sg = q.contiguous(), Sg.contiguous()
        Bbot = Bbot.contiguous() if Bbot is not None else None
        Bbot_prev = Bbot_prev.contiguous() if Bbot_prev is not None else None
        Ibot = Ibot.contiguous() if Ibot is not None else None
        Iem, ws = plan.emergent_intensity(tau, q, Sg, Bbot if diff else None,
                                          Bbot_prev if diff else None, None if diff else Ibot,
                                          checkpoint_interval=checkpoint_interval)
        ctx.plan = plan
        ctx.K = checkpoint_interval
        ctx.save_for_backward(tau, q, Sg, Bbot, Bbot_prev, Ibot, ws)
        return Iem

    @staticmethod
    def backward(ctx, gI):
        tau, q, Sg, Bbot, Bbot_prev, Ibot, ws = ctx.saved_tensors
        plan = ctx.plan
        diff = plan.lower_bc == pprt.BC_DIFFUSION
        g = plan.formal_solution_vjp(tau, q, Sg, gI.contiguous(), ws,
                                     Bbot if diff else None, Bbot_prev if diff else None,
                                     None if diff else Ibot, checkpoint_interval=ctx.K)
        return (None, None, None, g["dq"], g["dSg"], g.get("dBbot"), g.get("dBbot_prev"),
                g.get("dIbot"))


def emergent_intensity(plan: pprt.Plan, tau, q, Sg, Bbot=None, Bbot_prev=None, Ibot=None,
                       checkpoint_interval: int = 16):
    """Differentiable emergent intensity [nb, nf, na]."""
    return EmergentIntensity.apply(plan, checkpoint_interval, tau, q, Sg, Bbot, Bbot_prev, Ibot)


class EmergentIntensityScattering(torch.autograd.Function):
    """Iemerg[b, k, i] of the formal solution with in-layer scattering (FP64
    plans that request PPRT_OUT_IEMERG, na <= 16), differentiable in q, Sg,
    Bbot and Bbot_prev (diffusion lower boundary) or q, Sg and Ibot; omega and
    Itop are held fixed.  The backward pass reruns the bottom-up recursion
    inside pprt_formal_solution_scattering_vjp, so nothing but the inputs is
    saved."""

    @staticmethod
    def forward(ctx, plan: pprt.Plan, tau, q, Sg, omega, Bbot, Bbot_prev, Ibot, Itop):
        if not plan.outputs & pprt.OUT_IEMERG:
            raise ValueError("the plan must request OUT_IEMERG")
        diff = plan.lower_bc == pprt.BC_DIFFUSION
        q, Sg, omega = q.contiguous(), Sg.contiguous(), omega.contiguous()
        out = plan.formal_solution_scattering(tau, q, Sg, omega, Bbot=Bbot if diff else None,
                                              Bbot_prev=Bbot_prev if diff else None, Itop=Itop,
                                              Ibot=None if diff else Ibot)
        ctx.plan = plan
        ctx.save_for_backward(tau, q, Sg, omega, Bbot, Bbot_prev, Ibot, Itop)
        return out["Iemerg"]

    @staticmethod
    def backward(ctx, gI):
        tau, q, Sg, omega, Bbot, Bbot_prev, Ibot, Itop = ctx.saved_tensors
        plan = ctx.plan
        diff = plan.lower_bc == pprt.BC_DIFFUSION
        g = plan.formal_solution_scattering_vjp(tau, q, Sg, omega, gI.contiguous(),
                                                Bbot=Bbot if diff else None,
                                                Bbot_prev=Bbot_prev if diff else None, Itop=Itop,
                                                Ibot=None if diff else Ibot)
        return (None, None, g["dq"], g["dSg"], None, g.get("dBbot"), g.get("dBbot_prev"),
                g.get("dIbot"), None)


def emergent_intensity_scattering(plan: pprt.Plan, tau, q, Sg, omega, Bbot=None, Bbot_prev=None,
                                  Ibot=None, Itop=None):
    """Differentiable emergent intensity [nb, nf, na] with in-layer scattering."""
    return EmergentIntensityScattering.apply(plan, tau, q, Sg, omega, Bbot, Bbot_prev, Ibot, Itop)
