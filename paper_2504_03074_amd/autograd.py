"""torch.autograd front end of the discrete adjoint.

``helmholtz_solve(solver, c2, f, ...)`` returns the WaveHoltz fixed point
v* = W_h(v*, f) for the speed field c^2 and source f as a differentiable
function of both: the backward pass solves the adjoint fixed-point problem
(I - S_h)^T lam = dL/dv* and evaluates lam . dW_h(v*, f)/d(c^2, f) with the
library's reverse-time leapfrog (checkpointed).  All arithmetic runs in the
library's HIP kernels; this module only marshals tensors.

The time parameters are held fixed: N_t is taken from the first call (or
given) and passed as an override, so perturbing c^2 does not change the
discretisation in time.
"""
from __future__ import annotations

import torch


class _HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c2, f, solver, omega, periods, nt, method, rtol, maxit):
        solver.set_c2(c2.detach().contiguous())
        solver.set_source(f.detach().contiguous())
        solver.set_frequency(omega, periods=periods, nt=nt)
        v, info = solver.solve(method=method, rtol=rtol, maxit=maxit)
        if not info["converged"]:
            raise RuntimeError(f"forward WaveHoltz solve did not converge: {info}")
        ctx.solver = solver
        ctx.args = (omega, periods, nt, method, rtol, maxit)
        ctx.save_for_backward(c2, f, v)
        ctx.forward_info = info
        return v

    @staticmethod
    def backward(ctx, grad_v):
        c2, f, v = ctx.saved_tensors
        solver = ctx.solver
        omega, periods, nt, method, rtol, maxit = ctx.args
        # the solver may have been reconfigured since the forward pass
        solver.set_c2(c2.detach().contiguous())
        solver.set_source(f.detach().contiguous())
        solver.set_frequency(omega, periods=periods, nt=nt)
        lam, info = solver.solve_adjoint(grad_v.detach().contiguous(), method=method, rtol=rtol, maxit=maxit)
        if not info["converged"]:
            raise RuntimeError(f"adjoint WaveHoltz solve did not converge: {info}")
        grads = solver.gradient(v, lam, c2=ctx.needs_input_grad[0], f=ctx.needs_input_grad[1])
        return grads.get("c2"), grads.get("f"), None, None, None, None, None, None, None


def helmholtz_solve(solver, c2, f, omega, periods=1, nt=None, method="cg", rtol=1e-10, maxit=20000):
    """Differentiable v*(c^2, f) on `solver`'s grid (FP64 state; restart >= 2
    for CG).  nt = None fixes N_t from the time-step recipe for this c^2."""
    if nt is None:
        solver.set_c2(c2.detach().contiguous())
        nt = solver.set_frequency(omega, periods=periods)["nt"]
    return _HelmholtzSolve.apply(c2, f, solver, float(omega), int(periods), int(nt), method, float(rtol),
                                 int(maxit))
