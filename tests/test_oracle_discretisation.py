"""Pins of the oracle's discretisation against facts fixed independently of it.

* element matrices        <- Gauss quadrature of the d-linear shape functions
* operator on sine modes  <- closed-form symbol of the tensor-product stencil
* assembled operator      <- Kronecker products of the textbook 1D FE matrices
* varying-phi mass term   <- brute-force cell loops with quadrature
* diagonal                <- closed form (Section 4: known explicitly from phi)
"""

import itertools
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle.cycle import Params
from oracle.discretisation import element_matrices, interior_mask

GAUSS_X, GAUSS_W = np.polynomial.legendre.leggauss(3)
GX = 0.5 * (GAUSS_X + 1.0)
GW = 0.5 * GAUSS_W


def hat(k, x):
    return x if k == 1 else 1.0 - x


def dhat(k, x):
    return 1.0 if k == 1 else -1.0


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_element_matrices_by_quadrature(dim):
    K, M = element_matrices(dim)
    cs = list(itertools.product((0, 1), repeat=dim))
    Kq = np.zeros_like(K)
    Mq = np.zeros_like(M)
    for pt in itertools.product(range(3), repeat=dim):
        x = [GX[i] for i in pt]
        w = np.prod([GW[i] for i in pt])
        for i, ki in enumerate(cs):
            Ni = np.prod([hat(ki[a], x[a]) for a in range(dim)])
            gi = [dhat(ki[a], x[a]) * np.prod([hat(ki[b], x[b]) for b in range(dim) if b != a])
                  for a in range(dim)]
            for j, kj in enumerate(cs):
                Nj = np.prod([hat(kj[a], x[a]) for a in range(dim)])
                gj = [dhat(kj[a], x[a]) * np.prod([hat(kj[b], x[b]) for b in range(dim) if b != a])
                      for a in range(dim)]
                Mq[i, j] += w * Ni * Nj
                Kq[i, j] += w * sum(gi[a] * gj[a] for a in range(dim))
    np.testing.assert_allclose(K, Kq, atol=1e-14)
    np.testing.assert_allclose(M, Mq, atol=1e-14)


def symbol(dim, level, theta, phi, ks):
    """Eigenvalue of H on the sine mode prod_a sin(pi k_a j_a / N):
    eta^(d-2) sum_a 2(1-c_a) prod_(b!=a) (2+c_b)/3 - phi eta^d prod_a (2+c_a)/3."""
    N = 3 ** level
    eta = 3.0 ** (-level) * np.exp(1j * theta)
    c = [math.cos(math.pi * k / N) for k in ks]
    stiff = sum(2 * (1 - c[a]) * np.prod([(2 + c[b]) / 3 for b in range(dim) if b != a])
                for a in range(dim))
    mass = np.prod([(2 + ca) / 3 for ca in c])
    return eta ** (dim - 2) * stiff - phi * eta ** dim * mass


def sine_mode(dim, level, ks):
    N = 3 ** level
    j = np.arange(N + 1)
    v = np.ones((N + 1,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = N + 1
        v = v * np.sin(np.pi * ks[a] * j / N).reshape(shape)
    return v.astype(np.complex128)


@pytest.mark.parametrize("dim,level", [(2, 2), (2, 3), (3, 2)])
@pytest.mark.parametrize("theta,phi", [(0.0, 0.0), (math.pi / 6, 400.0), (0.3, 100 * (1 + 0.5j)),
                                       (0.0, -50.0)])
def test_sine_modes_are_eigenvectors(dim, level, theta, phi):
    N = 3 ** level
    rng = np.random.default_rng(level * 7 + dim)
    for _ in range(6):
        ks = [int(k) for k in rng.integers(1, N, dim)]
        s = sine_mode(dim, level, ks)
        Hs = O.apply_H(s, level, theta, phi)
        lam = symbol(dim, level, theta, phi, ks)
        scale = max(abs(lam), 1e-300) * np.abs(s).max()
        assert np.abs(Hs - lam * s).max() <= 1e-13 * scale


def fe_1d(n):
    """Textbook 1D interior FE matrices on unit spacing: tridiag(-1,2,-1) and
    tridiag(1/6, 2/3, 1/6)."""
    m = n - 2
    K = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    M = (4 * np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1)) / 6.0
    return K, M


@pytest.mark.parametrize("dim,level", [(2, 2), (3, 1), (3, 2)])
def test_dense_operator_is_kronecker_of_1d(dim, level):
    theta, phi = 0.4, 70 * (1 + 0.25j)
    n = 3 ** level + 1
    K1, M1 = fe_1d(n)
    eta = 3.0 ** (-level) * np.exp(1j * theta)
    stiff = 0
    for a in range(dim):
        m = np.ones((1, 1))
        for b in range(dim):
            m = np.kron(m, K1 if a == b else M1)
        stiff = stiff + m
    mass = np.ones((1, 1))
    for _ in range(dim):
        mass = np.kron(mass, M1)
    ref = eta ** (dim - 2) * stiff - phi * eta ** dim * mass
    A = O.dense_H(n, dim, level, theta, phi)
    np.testing.assert_allclose(A, ref, atol=1e-14 * np.abs(ref).max())
    # complex symmetric; conjugate mode is the Hermitian adjoint
    np.testing.assert_allclose(A, A.T, atol=1e-15 * np.abs(ref).max())
    Ac = O.dense_H(n, dim, level, theta, phi, conjugate=True)
    np.testing.assert_allclose(Ac, A.conj().T, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("dim,level", [(2, 1), (2, 2), (3, 1)])
def test_varying_phi_brute_force(dim, level):
    """Cell loops: H = sum_c [ eta^(d-2) int grad N_i grad N_j - phibar_c eta^d int N_i N_j ],
    phibar_c the mean of phi over the cell's vertices, integrals by quadrature on
    the physical cell (side h, Jacobian factors written out)."""
    rng = np.random.default_rng(3)
    n = 3 ** level + 1
    h = 3.0 ** (-level)
    theta = 0.35
    eta = h * np.exp(1j * theta)
    phi = (rng.uniform(-40, 90, (n,) * dim) + 1j * rng.uniform(0, 30, (n,) * dim))
    N = n ** dim
    A = np.zeros((N, N), dtype=np.complex128)
    cs = list(itertools.product((0, 1), repeat=dim))
    for cell in itertools.product(range(n - 1), repeat=dim):
        verts = [tuple(cell[a] + k[a] for a in range(dim)) for k in cs]
        pbar = np.mean([phi[v] for v in verts])
        for pt in itertools.product(range(3), repeat=dim):
            x = [GX[i] for i in pt]
            w = np.prod([GW[i] for i in pt])
            for i, ki in enumerate(cs):
                Ni = np.prod([hat(ki[a], x[a]) for a in range(dim)])
                # physical gradient on side eta: d/dx = (1/eta) d/dxi, volume eta^d
                gi = [dhat(ki[a], x[a]) / eta * np.prod([hat(ki[b], x[b]) for b in range(dim) if b != a])
                      for a in range(dim)]
                for j, kj in enumerate(cs):
                    Nj = np.prod([hat(kj[a], x[a]) for a in range(dim)])
                    gj = [dhat(kj[a], x[a]) / eta * np.prod([hat(kj[b], x[b]) for b in range(dim) if b != a])
                          for a in range(dim)]
                    val = w * eta ** dim * (sum(gi[a] * gj[a] for a in range(dim)) - pbar * Ni * Nj)
                    A[np.ravel_multi_index(verts[i], (n,) * dim),
                      np.ravel_multi_index(verts[j], (n,) * dim)] += val
    m = interior_mask(n, dim).ravel()
    ref = A[np.ix_(m, m)]
    got = O.dense_H(n, dim, level, theta, phi)
    np.testing.assert_allclose(got, ref, atol=1e-13 * np.abs(ref).max())
    # the diagonal accumulated cell by cell agrees with the assembled one
    D = O.diag_H(n, dim, level, theta, phi)
    np.testing.assert_allclose(D[interior_mask(n, dim)], np.diag(ref), atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_diag_closed_form(dim):
    level, theta, phi = 2, 0.5, 33 * (1 - 0.2j)
    n = 3 ** level + 1
    eta = 3.0 ** (-level) * np.exp(1j * theta)
    closed = eta ** (dim - 2) * 2 * dim * (2 / 3) ** (dim - 1) - phi * eta ** dim * (2 / 3) ** dim
    D = O.diag_H(n, dim, level, theta, phi)
    np.testing.assert_allclose(D[interior_mask(n, dim)], closed, rtol=1e-14)


def test_norms():
    level, dim = 2, 3
    n = 3 ** level + 1
    r = np.ones((n,) * dim, dtype=np.complex128) * (3 + 4j)
    # |r|_h = (h^d * (n-2)^d * 25)^(1/2); max norm 5
    assert abs(O.norm_h(r, level) - math.sqrt((1 / 9) ** 3 * 8 ** 3 * 25)) < 1e-13
    assert O.norm_max(r) == 5.0


def test_paper_regular_grid_vertex_count():
    """The regular h = 1/81 grid of the p = 2 application study has 6,400
    (interior) vertices (Section 7.4); fixture under tests/golden."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    for dim, level, count in ((int(a), int(b), int(c)) for a, b, c in rows):
        n = 3 ** level + 1
        assert interior_mask(n, dim).sum() == count


@pytest.mark.parametrize("dim,L,lmin", [(2, 4, 1), (2, 4, 3), (3, 3, 1)])
def test_coarse_fields_sample_the_analytic_field(dim, L, lmin):
    """Rediscretisation (Section 4): the nodal phi of every coarse level is the
    function phi(x) itself at that level's vertices x_j = j 3^-l.  The field
    is smooth, complex, nonlinear and not symmetric in the axes, so a wrong
    stride, an offset, a transposed axis or an average instead of a sample
    would all change it."""
    from paper_1508_03954_amd.inputs import vertex_coords

    def phi_fn(xs):
        a = xs[0]
        c = xs[-1]
        mid = xs[1] if len(xs) == 3 else 0.25
        return (50 + 30 * np.sin(2.1 * a + 0.7 * c) + 17 * a * c ** 2 + 5 * mid) * (1 + 0.3j) + 3j * c

    shape = lambda l: (3 ** l + 1,) * dim
    fine = np.broadcast_to(phi_fn(vertex_coords(L, dim)), shape(L)).astype(np.complex128)
    fields = O.coarse_fields(fine, L, lmin)
    assert sorted(fields) == list(range(lmin, L + 1))
    p = Params(dim=dim, level_max=L, level_min=lmin, phi=0, phi_nodal=fine)
    for lev in range(lmin, L + 1):
        ref = np.broadcast_to(phi_fn(vertex_coords(lev, dim)), shape(lev))
        np.testing.assert_allclose(fields[lev], ref, rtol=1e-14, atol=0)
        np.testing.assert_allclose(p.phi_at(lev), ref, rtol=1e-14, atol=0)


def _layer_cells(level, dim, layer_theta, width, faces, theta):
    """The test's own classification of the absorbing layer (Section 7.4):
    cell angle by its centre's distance to the selected faces, coordinate a
    counted from the fastest-varying axis (numpy axis dim - 1 - a)."""
    m = 3 ** level
    ang = np.full((m,) * dim, float(theta))
    for cell in itertools.product(range(m), repeat=dim):
        for a in range(dim):
            c = (cell[dim - 1 - a] + 0.5) / m
            if (faces >> (2 * a) & 1 and c < width) or (faces >> (2 * a + 1) & 1 and 1 - c < width):
                ang[cell] = layer_theta
    return ang


@pytest.mark.parametrize("dim,level,faces", [(2, 2, 0b0110), (2, 3, 0b1001), (3, 1, 0b100010)])
def test_layer_cells_brute_force(dim, level, faces):
    """Per-cell rotation: each cell's element integrals by quadrature on its
    own complex side eta_c = h exp(i theta_c) (gradients 1/eta_c, volume
    eta_c^d), theta_c from the test's own layer classification; the varying
    phi is averaged per cell.  The faces chosen are asymmetric, so a swapped
    axis or face bit changes the matrix."""
    rng = np.random.default_rng(11 + level)
    n = 3 ** level + 1
    h = 3.0 ** (-level)
    theta, lt, width = 0.15, math.radians(30), 1.0 / 3.0
    ang = _layer_cells(level, dim, lt, width, faces, theta)
    assert 0 < np.count_nonzero(ang == lt) < ang.size
    np.testing.assert_array_equal(O.cell_theta(level, dim, theta, (lt, width, faces)), ang)
    phi = rng.uniform(-40, 90, (n,) * dim) + 1j * rng.uniform(0, 30, (n,) * dim)
    N = n ** dim
    A = np.zeros((N, N), dtype=np.complex128)
    cs = list(itertools.product((0, 1), repeat=dim))
    for cell in itertools.product(range(n - 1), repeat=dim):
        eta = h * np.exp(1j * ang[cell])
        verts = [tuple(cell[a] + k[a] for a in range(dim)) for k in cs]
        pbar = np.mean([phi[v] for v in verts])
        for pt in itertools.product(range(3), repeat=dim):
            x = [GX[i] for i in pt]
            w = np.prod([GW[i] for i in pt])
            for i, ki in enumerate(cs):
                Ni = np.prod([hat(ki[a], x[a]) for a in range(dim)])
                gi = [dhat(ki[a], x[a]) / eta * np.prod([hat(ki[b], x[b]) for b in range(dim) if b != a])
                      for a in range(dim)]
                for j, kj in enumerate(cs):
                    Nj = np.prod([hat(kj[a], x[a]) for a in range(dim)])
                    gj = [dhat(kj[a], x[a]) / eta * np.prod([hat(kj[b], x[b]) for b in range(dim) if b != a])
                          for a in range(dim)]
                    val = w * eta ** dim * (sum(gi[a] * gj[a] for a in range(dim)) - pbar * Ni * Nj)
                    A[np.ravel_multi_index(verts[i], (n,) * dim),
                      np.ravel_multi_index(verts[j], (n,) * dim)] += val
    m = interior_mask(n, dim).ravel()
    ref = A[np.ix_(m, m)]
    tc = O.cell_theta(level, dim, theta, (lt, width, faces))
    got = O.dense_H(n, dim, level, tc, phi)
    np.testing.assert_allclose(got, ref, atol=1e-13 * np.abs(ref).max())
    D = O.diag_H(n, dim, level, tc, phi)
    np.testing.assert_allclose(D[interior_mask(n, dim)], np.diag(ref), atol=1e-13 * np.abs(ref).max())
    # the lumped load weight is the row sum of the lumped (per-cell) mass: the
    # mean of eta_c^d over the vertex's cells, here from the assembled masses
    Mrow = np.zeros(N, dtype=np.complex128)
    for cell in itertools.product(range(n - 1), repeat=dim):
        eta = h * np.exp(1j * ang[cell])
        for k in cs:
            Mrow[np.ravel_multi_index(tuple(cell[a] + k[a] for a in range(dim)), (n,) * dim)] += eta ** dim / 2 ** dim
    chi = rng.uniform(-1, 1, (n,) * dim) + 1j * rng.uniform(-1, 1, (n,) * dim)
    b = O.lumped_rhs(chi, level, tc)
    np.testing.assert_allclose(b[interior_mask(n, dim)], (Mrow * chi.ravel())[m], rtol=1e-14)


def test_layer_manufactured_solution_2d():
    """Absorbing layer on the faces x = 1 and y = 0 (angle 30 degrees, width
    1/3) around cells rotated by 0.2, constant phi.  In 2D the stiffness
    scale eta^(d-2) = 1 is the same in every cell, so the discrete problem is
    consistent with  -Lap u - phi e^(2 i theta(x)) u = e^(2 i theta(x)) chi;
    u* = sin(3 pi x) sin(3 pi y) vanishes on the layer's interfaces and solves
    it for chi = (18 pi^2 e^(-2 i theta(x)) - phi) u*.  The discrete solution
    (dense LU) converges at O(h^2): error ratios of about 9 per level.  A
    mass term rotated by e^(i theta) instead of e^(2 i theta), the layer on
    the wrong faces, or the load weighted with the global eta^d would each
    leave an O(1) error."""
    from paper_1508_03954_amd.inputs import vertex_coords
    theta, lt, faces = 0.2, math.radians(30), 0b0110
    phi = 30 + 10j
    errs = []
    for L in (2, 3, 4):
        y, x = vertex_coords(L, 2)
        us = np.sin(3 * np.pi * x) * np.sin(3 * np.pi * y) * np.ones((3 ** L + 1,) * 2)
        in_layer = (x > 2 / 3) | (y < 1 / 3)
        th = np.where(in_layer, lt, theta)
        chi = (18 * np.pi ** 2 * np.exp(-2j * th) - phi) * us
        p = Params(dim=2, level_max=L, theta=theta, phi=phi, layer=(lt, 1 / 3, faces))
        b = O.lumped_rhs(chi, L, p.theta_at(L))
        u = O.dense_solve(p, b)
        errs.append(np.abs(u - us).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 7 < r1 < 11 and 7 < r2 < 11, errs
    assert errs[2] < 1e-2
