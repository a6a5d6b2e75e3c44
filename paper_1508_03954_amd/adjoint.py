"""Gradient of an outer-shell functional with respect to a potential V(x).

The channel Helmholtz problem of the paper's Section 2 with a spatially
varying potential,  -Lap u + (V - phi0) u = chi,  i.e. nodal phi = phi0 - V.
The stand-in for the far-field post-processing is J(V) = sum_{j in S} |u_j|^2
over a shell S of vertices.  Its gradient needs one extra solve with the
adjoint operator:

    lambda = H^-H (1_S u)        (H is complex symmetric, so H^H = conj(H)),
    dJ/dV_j = -2 Re sum_{cells c containing j} 2^-d eta^d lambda_c^H M u_c .

Both solves and the gradient run in the HIP library (mg_solve with a
conjugate-mode context, mg_grad_potential); this module only wires them into
torch.autograd.
"""

from __future__ import annotations

import torch

from . import mg


class ShellFunctional(torch.autograd.Function):
    """J = sum over `shell` of |u|^2, u = H(V)^-1 b.

    forward(V, b, shell, cfg) with V real (n,)*d float64 on the GPU, b complex128
    (n,)*d, shell a bool (n,)*d mask, cfg a dict: dim, level_max, theta, phi0,
    variant, rtol, maxit.  Returns a 0-d float64 tensor.
    """

    @staticmethod
    def forward(ctx, V, b, shell, cfg):
        phi = (cfg["phi0"] - V.to(torch.complex128)).contiguous()
        fwd = mg.Solver(cfg["dim"], cfg["level_max"], theta=cfg.get("theta", 0.0), phi=0.0, phi_field=phi,
                        variant=cfg.get("variant", "bpx"), omega=cfg.get("omega", 0.6))
        u, its, rel, rc = fwd.solve(b, rtol=cfg.get("rtol", 1e-12), maxit=cfg.get("maxit", 2000),
                                    driver="bicgstab")
        if rc != 0:
            raise mg.MGError(rc, f"forward solve stopped at relative residual {rel:.3e} after {its} iterations")
        J = (u.abs() ** 2)[shell].sum()
        ctx.save_for_backward(u, phi, shell)
        ctx.cfg = cfg
        ctx.fwd = fwd
        ctx.stats = {"forward_iterations": its, "forward_relres": rel}
        return J

    @staticmethod
    def backward(ctx, gJ):
        u, phi, shell = ctx.saved_tensors
        cfg = ctx.cfg
        g = torch.where(shell, u, torch.zeros_like(u))
        adj = mg.Solver(cfg["dim"], cfg["level_max"], theta=cfg.get("theta", 0.0), phi=0.0, phi_field=phi,
                        variant=cfg.get("variant", "bpx"), omega=cfg.get("omega", 0.6), conjugate=True)
        lam, its, rel, rc = adj.solve(g, rtol=cfg.get("rtol", 1e-12), maxit=cfg.get("maxit", 2000),
                                      driver="bicgstab")
        if rc != 0:
            raise mg.MGError(rc, f"adjoint solve stopped at relative residual {rel:.3e} after {its} iterations")
        dJdV = ctx.fwd.grad_potential(u, lam)
        return gJ * dJdV, None, None, None


def shell_functional(V, b, shell, cfg):
    return ShellFunctional.apply(V, b, shell, cfg)
