"""Differentiable projection: c = P(R) psi with hand-written backward.

Forward:   c[a][n][b] = h^3 sum_{i in S_a} P_an(i; R_a) psi_b(i)   (sho_plan_project)
Backward:  dL/dpsi    = h^3 sum_a sum_n (dL/dc)[a][n][b] P_an          (sho_plan_expand_scaled
                        with alpha = h^3 into a zeroed buffer: the expansion is the
                        adjoint of the projection up to the grid-volume factor)
           dL/dR_a    = sum_{n,b} (dL/dc)[a][n][b] dc[a][n][b]/dR_a    (sho_plan_force)

Derivatives with respect to the atom centres are taken with every support S_a
frozen at the points the plan was built with (the sampled functions move, the
set of grid points does not), which makes c a smooth function of R.

All work runs in the library's kernels on the current stream; the Python layer
only moves arguments.
"""
import numpy as np
import torch

from . import binding as bd


def _use_centres(plan, p):
    """Make p the plan's function centres (supports stay as built)."""
    if not np.array_equal(p, plan.centres()):
        plan.set_centres(p)


class SHOProject(torch.autograd.Function):
    """c = SHOProject.apply(psi, pos, plan).

    psi: float64 GPU tensor (nz, ny, nx, B); pos: float64 tensor (natoms, 3)
    (any device; its values become the plan's function centres); plan: a
    binding.Plan built for this geometry.
    """

    @staticmethod
    def forward(ctx, psi, pos, plan):
        p = pos.detach().to("cpu", torch.float64).numpy().reshape(-1, 3).copy()
        _use_centres(plan, p)
        c = plan.project(psi.contiguous())
        ctx.save_for_backward(psi)
        ctx.plan = plan
        ctx.centres = p
        ctx.pos_device = pos.device
        return c

    @staticmethod
    def backward(ctx, grad_c):
        (psi,) = ctx.saved_tensors
        plan = ctx.plan
        # the plan may have been moved by later forward calls
        _use_centres(plan, ctx.centres)
        g = grad_c.contiguous()
        grad_psi = grad_pos = None
        if ctx.needs_input_grad[0]:
            grad_psi = torch.zeros_like(psi)
            plan.expand(g, grad_psi, alpha=plan.h ** 3)
        if ctx.needs_input_grad[1]:
            grad_pos = plan.force(psi.contiguous(), g).to(ctx.pos_device)
        return grad_psi, grad_pos, None


def project(psi, pos, plan):
    """Differentiable projection; see SHOProject."""
    return SHOProject.apply(psi, pos, plan)
