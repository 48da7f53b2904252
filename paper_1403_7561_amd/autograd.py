"""Electron count in a dot region as a differentiable function of the gate
voltages and the per-element permittivity.

``DotCharge.apply(dir_val, eps_r, problem, box, opts)`` solves the device on
the GPU (qe_solve), returns the electron count Q in ``box`` (qe_count_electrons)
and, in backward, calls the adjoint entry point (qe_adjoint) for dQ/dV and
dQ/deps.  The capacitance of Sec. III follows as C_g = q dQ/dV_g.
"""
from __future__ import annotations

import copy

import torch

from . import qe

Q_E = 1.602176634e-19  # C


def with_params(problem, dir_val, eps_r):
    """A shallow copy of ``problem`` that reads the given device tensors for
    the Dirichlet values and the permittivity."""
    p = copy.copy(problem)
    dv = dir_val.detach().to(device=problem.device, dtype=torch.float64).contiguous()
    ep = eps_r.detach().to(device=problem.device, dtype=torch.float64).contiguous()
    if dv.numel() != problem.n_dir or ep.numel() != problem.E:
        raise ValueError("dir_val / eps_r have the wrong length")
    p.dir_val = dv
    p.eps_r = ep
    return p


class DotCharge(torch.autograd.Function):
    """Q(dir_val, eps_r) = electrons in ``box`` at the converged potential."""

    @staticmethod
    def forward(ctx, dir_val, eps_r, problem, box, opts=None):
        P = with_params(problem, dir_val, eps_r)
        o = opts if opts is not None else qe.qe_default_options()
        phi, _, _ = qe.qe_solve(P, opts=o, want_density=False)
        Q = qe.qe_count_electrons(P, phi, [box])[0]
        ctx.P, ctx.box, ctx.opts = P, box, o
        ctx.save_for_backward(phi)
        return torch.tensor(Q, dtype=torch.float64, device=dir_val.device)

    @staticmethod
    def backward(ctx, gQ):
        (phi,) = ctx.saved_tensors
        want_eps = ctx.needs_input_grad[1]
        _, dV, deps, _, _ = qe.qe_adjoint(ctx.P, phi, ctx.box, opts=ctx.opts, want_eps=want_eps)
        g = gQ.to(torch.float64)
        gV = g * torch.as_tensor(dV, dtype=torch.float64, device=gQ.device) if ctx.needs_input_grad[0] else None
        ge = g * deps.to(gQ.device) if want_eps else None
        return gV, ge, None, None, None


def dot_charge(problem, box, dir_val=None, eps_r=None, opts=None):
    """Convenience wrapper: Q with autograd through the adjoint."""
    dv = problem.dir_val[: problem.n_dir] if dir_val is None else dir_val
    ep = problem.eps_r if eps_r is None else eps_r
    return DotCharge.apply(dv, ep, problem, box, opts)


def capacitance_aF(dQ_dV):
    """Dot-to-gate capacitance C = q dQ/dV in attofarads."""
    return Q_E * dQ_dV * 1e18
