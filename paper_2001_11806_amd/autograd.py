"""``torch.autograd.Function`` over the HIP forward sweep and its adjoint.

``LBMFunction.apply(u0, F, lbm, nsteps, rho_init)`` initialises the lattice
at equilibrium with velocity ``u0`` (3, nz, ny, nx), applies the uniform body
force ``F`` (3,), runs ``nsteps`` fused stream-collide steps and returns the
velocity readout u_T.  The backward pass seeds the adjoint with dL/du_T,
runs the hand-written adjoint sweep back to t = 0 (recomputing each
checkpoint segment) and returns dL/du0 and dL/dF.  The lattice must have been
created with ``checkpoint_every > 0`` and ``max_tape_steps >= nsteps``.

A lattice holds one trajectory at a time: if the lattice is initialised,
stepped or given a new force between this forward and its backward (for
example by a second ``apply``), the backward raises instead of returning the
gradients of the other run.
"""

import torch


class LBMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, F, lbm, nsteps, rho_init=None):
        lbm.set_force(F.detach().to("cpu", torch.float64).numpy())
        lbm.init_equilibrium(rho_init, u0.detach())
        lbm.step(nsteps)
        _, u = lbm.macroscopic(dtype=u0.dtype)
        ctx.lbm = lbm
        ctx.generation = lbm.generation
        ctx.nsteps = int(nsteps)
        ctx.F_meta = (F.dtype, F.device)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lbm = ctx.lbm
        if lbm.generation != ctx.generation:
            raise RuntimeError("the lattice no longer holds the trajectory of this forward pass "
                               "(it was initialised, stepped or given a new force since); "
                               "run backward before reusing the lattice")
        lbm.adjoint_seed(grad_u.contiguous())
        lbm.adjoint_step(ctx.nsteps)
        du0, _, dF = lbm.adjoint_grads(dtype=grad_u.dtype)
        dtype, device = ctx.F_meta
        return du0, torch.tensor(dF, dtype=dtype, device=device), None, None, None


def lbm_forward(u0, F, lbm, nsteps, rho_init=None):
    return LBMFunction.apply(u0, F, lbm, nsteps, rho_init)
