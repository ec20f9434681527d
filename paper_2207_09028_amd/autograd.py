"""torch.autograd.Function over the library's build and adjoint entry points.

Forward: occrik_build_device gives E_x (and K_{mu j}).  Backward: occrik_grad
gives dL/dC = g (2/N_k) K_{mu j} and dL/domega = g dE_x/domega; the potentials
are recomputed in the omega sweep, never stored.  The adjoint reads the plan's last
build, so backward raises if the plan has been built again (or its omega changed)
since this forward: keep one plan per live graph, or run backward first.
"""
from __future__ import annotations

import torch

from .plan import Plan


class ExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, omega, plan: Plan):
        if omega is not None and plan.spec.kernel != 0:
            plan.set_omega(float(omega.detach().cpu()) if isinstance(omega, torch.Tensor) else float(omega))
        Ex = torch.empty((1,), dtype=torch.float64, device=C.device)
        plan.build_device(C.detach().contiguous(), None, None, Ex)
        plan.status()
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.omega_is_tensor = isinstance(omega, torch.Tensor)
        return Ex[0]

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("exchange_energy backward: the plan was built again (or its omega changed) after "
                               "this forward, so it no longer holds the K_{mu j} and orbitals of this forward; "
                               "use one plan per live graph or call backward before the next build")
        want_w = ctx.omega_is_tensor and ctx.needs_input_grad[1]
        gC, gw = plan.grad(float(g.detach().cpu()), want_C=ctx.needs_input_grad[0], want_omega=want_w)
        gw_t = torch.tensor(gw, dtype=torch.float64) if want_w else None
        return gC, gw_t, None


def exchange_energy(plan: Plan, C, omega=None):
    """E_x(C, omega) with gradients through the HIP adjoint."""
    return ExchangeEnergy.apply(C, omega, plan)
