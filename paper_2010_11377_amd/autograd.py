"""Differentiable IRK time stepping for ``u_t = div(kappa grad u)``.

``IRKDiffusionFn.apply(kappa_nodes, u0, solver, nsteps, h_x)`` returns
``u_T`` after ``nsteps`` IRK steps with the stiffness matrix built from the
nodal coefficient field ``kappa_nodes`` ((ny+2) x (nx+2), boundary nodes
included).  Its backward pass runs the discrete adjoint of every step in
reverse (``irk_adjoint_step``: the transposed stage system, preconditioned by
the transposed block preconditioner) from the checkpointed ``u_n`` and
accumulates ``dJ/dkappa`` on the GPU (``irk_grad_diffusion_nodes``).

The solver is shared: another forward (a different kappa) may run between this
forward and its backward.  The forward keeps its stiffness matrix and the
solver's operator version; the backward reinstalls that matrix when the
version has moved on, so the adjoint always uses the K of its own forward.

The stiffness matrix is assembled on the host from ``kappa_nodes`` (problem
set-up, like any CSR handed to ``irk_setup``); every solve, adjoint solve and
the gradient accumulation run in the HIP library.
"""
import numpy as np
import torch

from . import problems


class IRKDiffusionFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa_nodes, u0, solver, nsteps, h_x):
        kn = kappa_nodes.detach().to("cpu", torch.float64).numpy()
        K = problems.kappa_diffusion(kn, length=h_x * (kn.shape[0] - 1))
        ctx.op_version = solver.update_operator(K)
        ctx.K = K
        u = u0.detach().contiguous()
        checkpoints = []
        for _ in range(nsteps):
            checkpoints.append(u)
            u = solver.step(u)
        ctx.solver = solver
        ctx.h_x = float(h_x)
        ctx.kshape = tuple(kappa_nodes.shape)
        ctx.kdevice = kappa_nodes.device
        ctx.save_for_backward(*checkpoints)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        solver = ctx.solver
        if solver.op_version != ctx.op_version:
            ctx.op_version = solver.update_operator(ctx.K)
        lam = grad_u.detach().to(torch.float64).contiguous()
        gnode = torch.zeros(ctx.kshape, dtype=torch.float64, device=lam.device)
        for u_n in reversed(ctx.saved_tensors):
            lam, psi, U = solver.adjoint_step(u_n, lam)
            solver.grad_diffusion_nodes(psi, U, ctx.h_x, gnode)
        return gnode.to(ctx.kdevice), lam, None, None, None
