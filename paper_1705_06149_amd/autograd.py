"""torch.autograd wrappers of the fine solve and its hand-written adjoint.

    J = kinetic_energy(handle, u0, v0, w0, lid, nsteps, dt)
    J.backward()          # u0.grad, v0.grad, w0.grad, lid.grad

The forward pass runs the fine propagator (nsteps projection steps, Sec. 2
of Croce, Ruprecht & Krause), returns J = 1/2 hx hy hz sum u_T^2 and leaves
its checkpoints on the handle (nsp_fine_solve_record); the backward pass
reverses that record (nsp_fine_solve_reverse: segments recomputed from the
checkpoints, adjoint projection and adjoint momentum kernels), so the
forward sweep runs once.  If the record went stale in between (another
record on the handle, or a new lid), backward records again first.  Lid
profiles parameterised by sine modes go through LidFromModes.  All
arithmetic runs in libnsp's kernels.
"""
from __future__ import annotations

import torch

from . import nsp


class LidFromModes(torch.autograd.Function):
    """lid = 1 + sum_{m,n} c[m,n] sin(m pi x) sin(n pi z) at the top u-faces."""

    @staticmethod
    def forward(ctx, coef, handle):
        ctx.handle = handle
        ctx.nmodes = int(coef.shape[0])
        return handle.lid_from_modes(coef.detach().contiguous())

    @staticmethod
    def backward(ctx, g_lid):
        return ctx.handle.lid_modes_grad(g_lid.contiguous(), ctx.nmodes), None


class NSFineSolve(torch.autograd.Function):
    """J(u0, v0, w0, lid) = kinetic energy after nsteps fine steps."""

    @staticmethod
    def forward(ctx, u0, v0, w0, lid, handle, nsteps, dt, ckpt_every, opts):
        handle.set_lid(lid.detach().contiguous())
        keep = any(ctx.needs_input_grad[:4])  # no record when no gradient can be asked for
        J, tape = handle.fine_solve_record(_y0(handle, u0, v0, w0), nsteps, dt, ckpt_every, opts, keep=keep)
        ctx.save_for_backward(u0, v0, w0, lid)
        ctx.args = (handle, nsteps, dt, ckpt_every, opts)
        ctx.tape = tape
        return torch.tensor(J, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, gJ):
        u0, v0, w0, lid = ctx.saved_tensors
        handle, nsteps, dt, ckpt_every, opts = ctx.args
        tape = ctx.tape
        if not handle.tape_valid(tape):
            handle.set_lid(lid.detach().contiguous())
            _, tape = handle.fine_solve_record(_y0(handle, u0, v0, w0), nsteps, dt, ckpt_every, opts, keep=True)
        g, gl = handle.fine_solve_reverse(tape, device=u0.device)
        return gJ * g[0][0], gJ * g[1][0], gJ * g[2][0], gJ * gl, None, None, None, None, None


def _y0(handle, u0, v0, w0):
    p0 = torch.zeros((1, handle.nz, handle.ny, handle.nx), dtype=torch.float64, device=u0.device)
    return (u0.detach().contiguous()[None], v0.detach().contiguous()[None], w0.detach().contiguous()[None], p0)


def kinetic_energy(handle, u0, v0, w0, lid, nsteps, dt, ckpt_every=10, opts=None):
    """Differentiable J = 1/2 hx hy hz sum over open faces of the velocity after
    nsteps steps; u0, v0, w0 are one slice (no batch dimension)."""
    return NSFineSolve.apply(u0, v0, w0, lid, handle, int(nsteps), float(dt), int(ckpt_every),
                             opts or nsp.PoissonOpts(rtol=1e-12))
