"""Differentiable far-field map q -> u_far for PyTorch.

forward: hps_factor + hps_solve + hps_far_field (Section 1 data, operator F
of eq. farfielddef); backward: the adjoint solve hps_vjp on the stored
factors (Theorem 2 in discrete form), which for a real input and a complex
output returns Re(J^H g) -- PyTorch's convention for real-to-complex maps.
The solver keeps one factorisation; if it has been refactored since this
forward (e.g. by another forward), backward first restores the forward's
state (factor + solve again); it always re-selects the forward's measurement
set (theta, R) before the adjoint solve."""
import torch


class FarField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, solver, k, dirs, thetas, R):
        solver.factor(q.detach().contiguous(), k)
        solver.solve(dirs)
        u = solver.far_field(thetas, R)
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.args = (q.detach().contiguous(), k, dirs, thetas, R)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        s = ctx.solver
        q, k, dirs, thetas, R = ctx.args
        if s.generation != ctx.generation:
            s.factor(q, k)
            s.solve(dirs)
        # the adjoint uses the measurement set of the last far-field call:
        # re-select this forward's (theta, R) in case another call changed it
        # (no host work when it is unchanged)
        s.far_field(thetas, R)
        g = s.vjp(grad_u.contiguous())
        return g, None, None, None, None, None


def far_field(q, solver, k, dirs, thetas, R):
    """u_far [ndir, ntheta] as a differentiable function of q (PDE nodes)."""
    return FarField.apply(q, solver, k, dirs, thetas, R)
