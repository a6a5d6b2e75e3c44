"""Pins of the oracle's solve drivers and of the discretisation's accuracy.

* fixed point   <- LU solve of the dense interior matrix
* Poisson MMS   <- analytic prod sin(pi x) solution of the paper's Poisson load
                   (phi = 0, theta = 0): second-order convergence, error / 9 per level
* Helmholtz MMS <- the same with chi = (d pi^2 - phi) prod sin(pi x)
* stationary Poisson cycle converges (Section 7.1: mesh-independent-ish rates)
"""

import numpy as np
import pytest

import oracle as O
from oracle.cycle import Params
from paper_1508_03954_amd.inputs import sine_load, sine_solution


def rand_c(shape, rng):
    return O.zero_boundary(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


@pytest.mark.parametrize("dim,L", [(2, 3), (3, 2)])
@pytest.mark.parametrize("variant", ["add", "bpx"])
def test_bicgstab_reaches_dense_solution(dim, L, variant, rng):
    p = Params(dim=dim, level_max=L, theta=np.pi / 6, phi=400.0, variant=variant, omega=0.6)
    n = 3 ** L + 1
    b = rand_c((n,) * dim, rng)
    ref = O.dense_solve(p, b)
    x, its, hist, ok = O.bicgstab(p, b, 1e-12, 200)
    assert ok
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_stationary_poisson_converges():
    L, dim = 4, 2
    p = Params(dim=dim, level_max=L, theta=0.0, phi=0.0, variant="add", omega=0.6,
               omega_scheme="exp")
    b = O.lumped_rhs(sine_load(L, dim), L, 0.0)
    u, its, hist, ok = O.stationary_solve(p, b, 1e-8, 400)
    assert ok
    ref = O.dense_solve(p, b)
    assert np.linalg.norm(u - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("dim,levels", [(2, (3, 4, 5)), (3, (2, 3))])
@pytest.mark.parametrize("phi", [0.0, 20.0])
def test_manufactured_solution_second_order(dim, levels, phi):
    errs = []
    for L in levels:
        p = Params(dim=dim, level_max=L, theta=0.0, phi=phi, variant="bpx", omega=0.6)
        chi = sine_load(L, dim) * (1.0 - phi / (dim * np.pi ** 2))
        b = O.lumped_rhs(chi, L, 0.0)
        u, its, hist, ok = O.bicgstab(p, b, 1e-13, 300)
        assert ok
        errs.append(np.abs(u - sine_solution(L, dim)).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 7.0 < r < 11.0, (errs, ratios)


def test_nested_initial_guess_converges_at_second_order():
    """The nested guess (level L - 1 solved with the sampled load, prolonged)
    approaches the manufactured Poisson solution prod sin(pi x) at O(h^2):
    its max error drops by about 9 from L = 3 to L = 4 (2D), and it beats the
    zero guess by far."""
    errs = []
    for L in (3, 4):
        p = Params(dim=2, level_max=L, theta=0.0, phi=0.0)
        guess = O.nested_initial_guess(p, sine_load(L, 2))
        exact = sine_solution(L, 2)
        # the guess is zero on the boundary, where the solution vanishes too
        assert np.all(guess[0, :] == 0) and np.all(guess[:, -1] == 0)
        errs.append(np.abs(guess - exact).max())
        assert errs[-1] < 0.1 * np.abs(exact).max()
    assert 6.0 < errs[0] / errs[1] < 12.0, errs


def test_nested_initial_guess_on_coarse_vertices_is_the_coarse_solution():
    """At the vertices the two levels share, the guess equals the level L - 1
    discrete solution (P reproduces coarse values at c-points)."""
    p = Params(dim=2, level_max=3, theta=np.pi / 6, phi=90 * (1 + 0.5j))
    rng = np.random.default_rng(11)
    chi = rng.standard_normal((28, 28)) + 1j * rng.standard_normal((28, 28))
    guess = O.nested_initial_guess(p, chi)
    q = Params(dim=2, level_max=2, theta=np.pi / 6, phi=90 * (1 + 0.5j))
    uc = O.dense_solve(q, O.lumped_rhs(chi[::3, ::3], 2, np.pi / 6))
    np.testing.assert_allclose(guess[::3, ::3], uc, rtol=0, atol=1e-13 * np.abs(uc).max())


def _rotated_mms_error(dim, L, theta, phi, weight_theta):
    """Max error of the discrete solution against prod sin(pi x) for the load
    chi = (d pi^2 e^(-2 i theta) - phi) prod sin(pi x), lumped with the weight
    of `weight_theta` (the correct weight is eta_L^d = (3^-L e^(i theta))^d)."""
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi, variant="bpx", omega=0.6)
    exact = sine_solution(L, dim)
    chi = (dim * np.pi ** 2 * np.exp(-2j * theta) - phi) * exact
    b = O.lumped_rhs(chi, L, weight_theta)
    if (3 ** L - 1) ** dim <= 700:
        u = O.dense_solve(p, b)
    else:
        u, its, hist, ok = O.bicgstab(p, b, 1e-13, 400)
        assert ok
    return np.abs(u - exact).max()


@pytest.mark.parametrize("dim,levels", [(2, (2, 3, 4)), (3, (2, 3))])
def test_rotated_grid_manufactured_solution(dim, levels):
    """Complex grid rotation (Section 2, CSG) with the lumped load weight
    eta_L^d: on the grid x -> x e^(i theta) the discrete operator approximates
    e^(-2 i theta) (-Lap) - phi, so the load (d pi^2 e^(-2 i theta) - phi)
    prod sin(pi x) has the solution prod sin(pi x), reached at O(h^2).  The
    weights h^d or eta^(d-2) in place of eta^d leave an O(1) error."""
    theta, phi = np.pi / 6, 30 * (1 + 0.2j)
    errs = [_rotated_mms_error(dim, L, theta, phi, theta) for L in levels]
    for a, c in zip(errs, errs[1:]):
        assert 7.0 < a / c < 11.0, errs
    # a planted mistake in the weight (h^d: the unrotated weight) fails the pin
    assert _rotated_mms_error(dim, levels[-1], theta, phi, 0.0) > 0.3
