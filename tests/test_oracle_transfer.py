"""Pins of the oracle's grid transfers.

* P reproduces d-linear functions exactly (the definition of d-linear
  interpolation, checked on sampled functions, not on the weights)
* R = P^T as the bilinear identity <R x, y> = <x, P y> on interior vectors
* I P = id (coarse vertices are copied)
* Galerkin identity R H_l P = H_(l-1) for constant phi and uniform rotation
  (Section 4), and its failure for varying phi
* FAS right-hand side, Lemma 2: R rhat = R r + H_(l-1) I u
"""

import itertools

import numpy as np
import pytest

import oracle as O
from oracle.discretisation import interior_mask
from paper_1508_03954_amd.inputs import vertex_coords


def rand_c(shape, rng, zero_bnd=True):
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return O.zero_boundary(v) if zero_bnd else v


@pytest.mark.parametrize("dim,level", [(1, 2), (2, 2), (3, 2)])
def test_prolong_reproduces_dlinear_functions(dim, level, rng):
    coef = rng.standard_normal(2 ** dim) + 1j * rng.standard_normal(2 ** dim)

    def f(lev):
        xs = vertex_coords(lev, dim)
        out = 0
        for i, k in enumerate(itertools.product((0, 1), repeat=dim)):
            term = coef[i]
            for a in range(dim):
                term = term * (xs[a] if k[a] else 1.0)
            out = out + term * np.ones((3 ** lev + 1,) * dim)
        return out

    np.testing.assert_allclose(O.prolong(f(level - 1)), f(level), atol=1e-13)


@pytest.mark.parametrize("dim,level", [(1, 3), (2, 2), (3, 2)])
def test_restrict_is_transpose_of_prolong(dim, level, rng):
    nf, nc = 3 ** level + 1, 3 ** (level - 1) + 1
    x = rand_c((nf,) * dim, rng)
    y = rand_c((nc,) * dim, rng)
    lhs = np.sum(O.restrict(x) * y)
    rhs = np.sum(x * O.prolong(y))
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


@pytest.mark.parametrize("dim,level", [(2, 3), (3, 2)])
def test_inject_after_prolong_is_identity(dim, level, rng):
    nc = 3 ** (level - 1) + 1
    y = rand_c((nc,) * dim, rng, zero_bnd=False)
    np.testing.assert_array_equal(O.inject(O.prolong(y)), y)


@pytest.mark.parametrize("dim,level", [(2, 3), (3, 2)])
@pytest.mark.parametrize("theta,phi", [(0.0, 0.0), (np.pi / 6, 400.0), (0.2, 100 * (1 + 0.5j))])
def test_galerkin_identity(dim, level, theta, phi, rng):
    nc = 3 ** (level - 1) + 1
    v = rand_c((nc,) * dim, rng)
    lhs = O.restrict(O.apply_H(O.prolong(v), level, theta, phi))
    rhs = O.apply_H(v, level - 1, theta, phi)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_galerkin_identity_fails_for_varying_phi(rng):
    dim, level = 2, 3
    nf, nc = 3 ** level + 1, 3 ** (level - 1) + 1
    phi = 200 + 150 * rng.standard_normal((nf,) * dim)
    v = rand_c((nc,) * dim, rng)
    lhs = O.restrict(O.apply_H(O.prolong(v), level, 0.1, phi))
    rhs = O.apply_H(v, level - 1, 0.1, phi[::3, ::3])
    assert np.abs(lhs - rhs).max() > 1e-6 * np.abs(rhs).max()


@pytest.mark.parametrize("dim,level", [(2, 3), (3, 2)])
def test_fas_rhs_lemma2(dim, level, rng):
    theta, phi = 0.3, 60 * (1 + 0.4j)
    nf = 3 ** level + 1
    u = rand_c((nf,) * dim, rng)
    b = rand_c((nf,) * dim, rng)
    uc = O.inject(u)
    uhat = u - O.prolong(uc)
    rhat = b - O.apply_H(uhat, level, theta, phi)
    r = b - O.apply_H(u, level, theta, phi)
    lhs = O.restrict(rhat)
    rhs = O.restrict(r) + O.apply_H(uc, level - 1, theta, phi)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()


def test_cpoints():
    m = O.cpoint_mask(10, 2, 2, 1)
    assert m.sum() == 16 and m[0, 0] and m[3, 6] and not m[1, 0]
    assert not O.cpoint_mask(10, 2, 1, 1).any()
