"""Oracle: solve drivers around the cycle.

Test infrastructure only (see the package header).

* `stationary_solve` -- repeated pipelined cycles (the paper's iteration:
  one traversal per cycle) until the finest h-norm residual has dropped by
  rtol relative to the start, then a flush;
* `bicgstab`         -- BiCGStab with the additive cycle from a zero start as
  right preconditioner (the paper uses its solver as a preconditioner,
  Sections 2 and 4); an addition beyond the paper, needed because the
  stationary cycle diverges on indefinite 3D problems;
* `dense_solve`      -- LU on the dense interior matrix (tiny grids only), the
  fixed point both drivers must reach;
* `nested_initial_guess` -- the finest level's starting point of a nested
  solve: the level below solved with the load sampled there, prolonged;
* `max_norm_reduction` -- the measure of the Section 7.4 study: the maximum
  norm of the residual after a number of iterations from u = 0, relative to
  that of the start.
"""

from __future__ import annotations

import numpy as np

import dataclasses

from .cycle import Params, Pipelined, zero_start_cycle
from .discretisation import dense_H, interior_mask, lumped_rhs, zero_boundary
from .transfer import prolong


def stationary_solve(p: Params, b: np.ndarray, rtol: float, maxit: int, u0=None):
    """Returns (u, cycles, history of h-norm residuals, converged?)."""
    pipe = Pipelined(p, b, u0)
    hist = []
    converged = False
    for _ in range(maxit):
        rh, _ = pipe.cycle()
        hist.append(rh)
        if rh <= rtol * hist[0]:
            converged = True
            break
        if not np.isfinite(rh) or rh > 1e8 * hist[0]:
            break
    u = pipe.flush()
    return u, len(hist), hist, converged


def bicgstab(p: Params, b: np.ndarray, rtol: float, maxit: int, x0=None, precondition=True):
    """Right-preconditioned BiCGStab on interior vertices (van der Vorst 1992).
    Inner products are conjugating (np.vdot).  Returns (x, iterations,
    relative-residual history, converged?)."""
    L = p.level_max
    A = lambda v: p.H(v, L)
    M = (lambda v: zero_start_cycle(p, v)) if precondition else (lambda v: v)
    b = zero_boundary(b)
    x = np.zeros_like(b) if x0 is None else zero_boundary(x0)
    r = zero_boundary(b - A(x))
    bnorm = np.linalg.norm(b)
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    pv = np.zeros_like(b)
    hist = [np.linalg.norm(r) / bnorm]
    for it in range(1, maxit + 1):
        rho_new = np.vdot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        pv = r + beta * (pv - omega * v)
        y = M(pv)
        v = A(y)
        alpha = rho_new / np.vdot(rh, v)
        s = r - alpha * v
        if np.linalg.norm(s) / bnorm <= rtol:
            x = x + alpha * y
            hist.append(np.linalg.norm(s) / bnorm)
            return x, it, hist, True
        z = M(s)
        t = A(z)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * y + omega * z
        r = s - omega * t
        rho = rho_new
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rtol:
            return x, it, hist, True
    return x, maxit, hist, False


def dense_solve(p: Params, b: np.ndarray) -> np.ndarray:
    """u with H u = b on interior vertices, zero boundary (np.linalg.solve)."""
    L = p.level_max
    n = p.n(L)
    A = dense_H(n, p.dim, L, p.theta_at(L), p.phi_at(L), p.conjugate)
    m = interior_mask(n, p.dim)
    u = np.zeros((n,) * p.dim, dtype=np.complex128)
    u[m] = np.linalg.solve(A, np.asarray(b)[m])
    return u


def nested_initial_guess(p: Params, chi: np.ndarray) -> np.ndarray:
    """Initial guess of the finest level L in a nested solve, the regular-grid
    form of the remark on FMG-like cycles (Section 5): coarse solutions act as
    initial guesses on finer grids.  The load chi (nodal, finest grid) is
    sampled at the vertices of level L - 1, that level is solved exactly
    (dense_solve) and its solution prolonged d-linearly to level L.

    Pinned: for a Poisson problem with a smooth manufactured solution the
    guess converges to it at O(h^2) (tests/test_oracle_solve.py)."""
    L = p.level_max
    q = dataclasses.replace(p, level_max=L - 1, level_min=min(p.level_min, L - 1))
    chic = np.asarray(chi)[(slice(None, None, 3),) * p.dim]
    uc = dense_solve(q, lumped_rhs(chic, L - 1, p.theta_at(L - 1)))
    return prolong(uc)


def max_norm_reduction(p: Params, b: np.ndarray, iterations: int):
    """max|b - H u_n| / max|b| after n pipelined cycles from u_0 = 0 and a
    flush (u_n the n-th iterate), with the flushed iterate (Section 7.4,
    Table 08gaussian measures this after 50 iterations)."""
    pipe = Pipelined(p, b)
    for _ in range(iterations):
        pipe.cycle()
    u = pipe.flush()
    L = p.level_max
    r = zero_boundary(np.asarray(b) - p.H(u, L))
    m = interior_mask(p.n(L), p.dim)
    return float(np.abs(r[m]).max() / np.abs(np.asarray(b)[m]).max()), u
