"""Differentiable all-at-once solve for PyTorch (argument marshalling only).

``heat_solve(f, u0, problem)`` returns x = A^{-1} [b; f] with b_0 = u0 (the
all-at-once system of the paper's eq. (2.4), solved by the library's FGMRES),
and its backward pass applies the adjoint: with lam = A^{-T} dL/dx (the
library's transposed solve), dL/df = lam_V and dL/du0 = lam_{v,0}.  With
``theta`` (log of the nodal diffusivity) the library takes theta itself
(``aao_set_kappa`` with is_log, on the same handle) and dL/dtheta comes from
``aao_grad_logkappa``.

All arithmetic runs in the HIP library; this module only routes tensors.
"""
import torch


def _split_rhs_grad(problem, lam):
    """(dL/df, dL/du0) from lam = A^{-T} dL/dx for rhs = [u0; 0; f]."""
    N, nt, s = problem.N, problem.nt, problem.s
    gu0 = lam[:N]
    gf = lam[(nt + 1) * N:].reshape(nt, s, N)
    return gf, gu0


class _HeatSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, u0, theta, problem):
        if theta is not None:
            problem.set_kappa(theta.detach().to(torch.float64).contiguous().view(-1), log=True)
        rhs = problem.assemble_rhs(f.detach().contiguous().view(-1), u0.detach().contiguous().view(-1))
        x, st = problem.solve(rhs)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.problem = problem
        ctx.has_theta = theta is not None
        ctx.f_shape = f.shape
        ctx.save_for_backward(x, theta.detach().clone() if theta is not None else None)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, theta = ctx.saved_tensors
        problem = ctx.problem
        if theta is not None:
            # another forward call may have moved the handle to another theta
            problem.set_kappa(theta.to(torch.float64).contiguous().view(-1), log=True)
        lam, st = problem.solve_adjoint(gx.contiguous().to(torch.float64))
        if not st["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        gf, gu0 = _split_rhs_grad(problem, lam)
        gtheta = problem.grad_logkappa(x, lam) if ctx.has_theta else None
        return gf.reshape(ctx.f_shape), gu0, gtheta, None


def heat_solve(f, u0, problem, theta=None):
    """Differentiable x = A^{-1} [u0; 0; f].

    f: (nt, s, N) float64 CUDA tensor sampled at the stage times; u0: (N,).
    problem: a HeatProblem fixing dim, n, s, nt, T and the solver options;
    theta: optional (N,) log-diffusivity; the problem must then have been
    created with a kappa array (its value is replaced by exp(theta) inside
    the library on each call), and theta receives a gradient.
    Returns x of length U in the paper's layout (Sec. 2).
    """
    if theta is not None and problem._kappa is None:
        raise ValueError("differentiating in log kappa needs a problem created with a kappa array")
    return _HeatSolve.apply(f, u0, theta, problem)
