"""Pins of the oracle's adjoint gradient.

* H^-H g = conj(H^-1 conj g) for the complex-symmetric operator (dense LU)
* dJ/dV from the cell formula == central finite differences of J(V) with
  dense solves (tiny grids)
"""

import numpy as np
import pytest

import oracle as O
from oracle.cycle import Params
from oracle.discretisation import interior_mask
from paper_1508_03954_amd.inputs import shell_mask


def solve_dense(level, dim, theta, phi_nodal, b, conjugate=False):
    p = Params(dim=dim, level_max=level, theta=theta, phi=0, phi_nodal=phi_nodal,
               conjugate=conjugate)
    return O.dense_solve(p, b)


def test_adjoint_conjugate_identity(rng):
    dim, L, theta = 2, 3, 0.2
    n = 3 ** L + 1
    phi = (120 + 40 * rng.standard_normal((n,) * dim)) * (1 + 0.3j)
    g = O.zero_boundary(rng.standard_normal((n,) * dim) + 1j * rng.standard_normal((n,) * dim))
    lam = solve_dense(L, dim, theta, phi, g, conjugate=True)
    alt = np.conj(solve_dense(L, dim, theta, phi, np.conj(g)))
    np.testing.assert_allclose(lam, alt, atol=1e-12 * np.abs(alt).max())


@pytest.mark.parametrize("dim,L", [(2, 3), (3, 2)])
def test_gradient_matches_finite_differences(dim, L, rng):
    n = 3 ** L + 1
    theta = 0.0
    phi0 = 60 * (1 + 0.3j)
    V = 30 * rng.standard_normal((n,) * dim)
    b = O.zero_boundary(rng.standard_normal((n,) * dim) + 1j * rng.standard_normal((n,) * dim))
    S = shell_mask(L, dim, 0.5, 0.9)
    assert S.sum() > 3

    def J(Vv):
        u = solve_dense(L, dim, theta, phi0 - Vv, b)
        return O.shell_functional(u, S), u

    J0, u = J(V)
    g = np.where(S, u, 0)
    lam = solve_dense(L, dim, theta, phi0 - V, g, conjugate=True)
    grad = O.potential_gradient(u, lam, L, theta)
    idx = list(np.argwhere(interior_mask(n, dim))[rng.choice(int(interior_mask(n, dim).sum()), 6, replace=False)])
    idx.append(np.zeros(dim, int))          # a boundary vertex still enters the cell averages
    eps = 1e-4
    for j in idx:
        j = tuple(j)
        Vp, Vm = V.copy(), V.copy()
        Vp[j] += eps
        Vm[j] -= eps
        fd = (J(Vp)[0] - J(Vm)[0]) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-6 * abs(fd) + 1e-7 * np.abs(grad).max(), (j, fd, grad[j])
