"""Oracle: Ritz-Galerkin d-linear discretisation of  -Lap u - phi u = chi.

Test infrastructure only (see the package header).

The paper's Section 4 discretises the channel Helmholtz equation with d-linear
nodal shape functions on the hypercube cells of each spacetree level, keeps
only precomputed local element matrices and evaluates the operator cell by
cell (Appendix B).  On level l the cells have side h_l = 3^-l; the complex
grid scaling of Section 2 (CSG) replaces the side by eta_l = h_l exp(i theta).

Readings of points the paper leaves open (each listed in the design notes):
  * the complex side enters both element scalings, stiffness eta^(d-2) and mass
    eta^d (the Jacobian of the map x -> x exp(i theta));
  * a spatially varying phi weighs each cell's consistent mass matrix with the
    average of phi over the cell's 2^d vertices; coarse levels sample phi at
    their own vertices (rediscretisation, not Galerkin);
  * the discrete load is lumped: b_j = eta_L^d chi(x_j) at interior vertices;
  * rows of boundary vertices are dropped (zero Dirichlet): operator results
    are zero on the boundary and boundary input entries are ignored;
  * the absorbing layer of Section 7.4 rotates single cells: a cell whose
    centre lies within the layer width of one of the layer's faces takes the
    layer's angle, every other cell the global theta.  Rotation angles may
    therefore be given per cell; the lumped load weight of a vertex is then the
    mean of eta_c^d over its 2^d cells (the row sum of the lumped mass matrix).
"""

from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

# Unit-cell 1D element matrices of linear hat functions on [0, 1]:
#   stiffness  int phi_i' phi_j'   and   mass  int phi_i phi_j .
K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


@lru_cache(maxsize=None)
def element_matrices(dim: int):
    """Reference-cell d-linear element matrices (2^d x 2^d).

    Stiffness  K = sum_a  (x)_b (K1 if b == a else M1)   (grad.grad splits per axis)
    Mass       M = (x)_b M1.
    Local vertex index = ravel of its corner offsets (k_0, ..., k_{d-1}) in numpy
    axis order.  Pinned by quadrature of the shape functions in the tests.
    """
    K = np.zeros((2 ** dim, 2 ** dim))
    for a in range(dim):
        m = np.ones((1, 1))
        for b in range(dim):
            m = np.kron(m, K1 if b == a else M1)
        K += m
    M = np.ones((1, 1))
    for _ in range(dim):
        M = np.kron(M, M1)
    return K, M


def level_eta(level: int, theta: float, conjugate: bool = False) -> complex:
    """Complex cell side eta_l = 3^-l exp(i theta) (conjugated for H^H)."""
    eta = 3.0 ** (-level) * np.exp(1j * theta)
    return np.conj(eta) if conjugate else eta


def cell_theta(level: int, dim: int, theta: float, layer=None):
    """Rotation angle of every cell of a level (Section 7.4 absorbing layer).

    layer = None gives the uniform angle theta (a scalar).  Otherwise layer is
    (layer_theta, width, faces): faces is a bit set, bit 2a for the face
    x_a = 0 and bit 2a + 1 for the face x_a = 1, coordinate x_0 being the
    fastest-varying one (numpy's last axis); a cell whose centre lies closer
    than `width` to a selected face is rotated by layer_theta, every other cell
    by theta.  Returns an array of shape (3^level,)*dim.
    """
    if layer is None:
        return theta
    lt, width, faces = layer
    m = 3 ** level
    centre = (np.arange(m) + 0.5) / m
    inside = np.zeros((m,) * dim, dtype=bool)
    for a in range(dim):
        shape = [1] * dim
        shape[dim - 1 - a] = m
        if faces & (1 << (2 * a)):
            inside |= (centre < width).reshape(shape)
        if faces & (1 << (2 * a + 1)):
            inside |= (1.0 - centre < width).reshape(shape)
    return np.where(inside, float(lt), float(theta))


def cell_eta(level: int, theta, conjugate: bool = False):
    """Complex cell sides 3^-l exp(i theta_c) for a scalar or per-cell theta."""
    eta = 3.0 ** (-level) * np.exp(1j * np.asarray(theta, dtype=np.float64))
    eta = np.conj(eta) if conjugate else eta
    return complex(eta) if np.ndim(eta) == 0 else eta


def corners(dim: int):
    return list(itertools.product((0, 1), repeat=dim))


def _cell_view(a: np.ndarray, k) -> tuple:
    """Slice selecting, for every cell c, the vertex c + k."""
    n = a.shape[0]
    return tuple(slice(kk, kk + n - 1) for kk in k)


def zero_boundary(v: np.ndarray) -> np.ndarray:
    out = np.array(v, dtype=np.complex128, copy=True)
    for a in range(out.ndim):
        idx = [slice(None)] * out.ndim
        idx[a] = 0
        out[tuple(idx)] = 0
        idx[a] = -1
        out[tuple(idx)] = 0
    return out


def interior_mask(n: int, dim: int) -> np.ndarray:
    m = np.zeros((n,) * dim, dtype=bool)
    m[(slice(1, -1),) * dim] = True
    return m


def cell_average(phi_nodal: np.ndarray) -> np.ndarray:
    """Average of a nodal field over the 2^d vertices of every cell."""
    dim = phi_nodal.ndim
    acc = np.zeros(tuple(s - 1 for s in phi_nodal.shape), dtype=np.complex128)
    for k in corners(dim):
        acc += phi_nodal[_cell_view(phi_nodal, k)]
    return acc / 2 ** dim


def coarse_fields(phi_nodal_fine: np.ndarray, level_max: int, level_min: int) -> dict:
    """Nodal phi on every level by sampling (injection) of the finest field."""
    out = {level_max: np.asarray(phi_nodal_fine, dtype=np.complex128)}
    for lev in range(level_max, level_min, -1):
        out[lev - 1] = out[lev][(slice(None, None, 3),) * out[lev].ndim]
    return out


def apply_H(u: np.ndarray, level: int, theta: float, phi, conjugate: bool = False) -> np.ndarray:
    """(H_l u)_j = sum over cells c containing j of (H_c u_c)_loc(j),
    H_c = eta^(d-2) K - phibar_c eta^d M, evaluated element by element.

    `phi` is a complex scalar or a nodal array of shape (n,)*d (cell-averaged);
    `theta` a scalar or one angle per cell (shape (n-1,)*d, see cell_theta).
    Boundary entries of u are ignored; boundary rows of the result are zero.
    Conjugate mode builds conj(H) = H^H (H is complex symmetric).
    Pinned by: the sine-mode symbol, the Kronecker assembly of 1D FE matrices,
    and brute-force quadrature for varying phi.
    """
    dim = u.ndim
    K, M = element_matrices(dim)
    eta = cell_eta(level, theta, conjugate)
    if np.ndim(phi) == 0:
        phibar = complex(phi)
    else:
        phibar = cell_average(np.asarray(phi))
    if conjugate:
        phibar = np.conj(phibar)
    u = zero_boundary(u)
    cs = corners(dim)
    U = np.stack([u[_cell_view(u, k)] for k in cs])                 # (2^d, cells...)
    KU = np.tensordot(K, U, axes=(1, 0))
    MU = np.tensordot(M, U, axes=(1, 0))
    HU = eta ** (dim - 2) * KU - (eta ** dim) * phibar * MU
    out = np.zeros_like(u)
    for i, k in enumerate(cs):
        out[_cell_view(out, k)] += HU[i]
    return zero_boundary(out)


def diag_H(n: int, dim: int, level: int, theta: float, phi, conjugate: bool = False) -> np.ndarray:
    """diag(H_l) accumulated cell by cell (the paper's Section 4 explicit
    accumulation, needed for varying phi).  Boundary entries are set to 1 so
    that a division leaves the (zero) boundary residual untouched.
    Pinned by the closed form  eta^(d-2) 2d (2/3)^(d-1) - phi eta^d (2/3)^d."""
    K, M = element_matrices(dim)
    eta = cell_eta(level, theta, conjugate)
    if np.ndim(phi) == 0:
        phibar = complex(phi) * np.ones((n - 1,) * dim)
    else:
        phibar = cell_average(np.asarray(phi))
    if conjugate:
        phibar = np.conj(phibar)
    out = np.zeros((n,) * dim, dtype=np.complex128)
    for i, k in enumerate(corners(dim)):
        out[_cell_view(out, k)] += eta ** (dim - 2) * K[i, i] - eta ** dim * phibar * M[i, i]
    out[~interior_mask(n, dim)] = 1.0
    return out


def lumped_rhs(chi: np.ndarray, level: int, theta) -> np.ndarray:
    """b_j = eta_L^d chi(x_j) on interior vertices, zero on the boundary.  With
    one angle per cell the weight is the mean of eta_c^d over the vertex's 2^d
    cells."""
    chi = np.asarray(chi)
    dim = chi.ndim
    if np.ndim(theta) == 0:
        return zero_boundary(level_eta(level, theta) ** dim * chi)
    etad = cell_eta(level, theta) ** dim
    wgt = np.zeros(chi.shape, dtype=np.complex128)
    for k in corners(dim):
        wgt[_cell_view(wgt, k)] += etad
    return zero_boundary(wgt / 2 ** dim * chi)


def dense_H(n: int, dim: int, level: int, theta: float, phi, conjugate: bool = False) -> np.ndarray:
    """Dense matrix of H_l restricted to interior vertices (tiny grids only),
    obtained column by column from apply_H."""
    mask = interior_mask(n, dim)
    idx = np.flatnonzero(mask.ravel())
    A = np.zeros((idx.size, idx.size), dtype=np.complex128)
    e = np.zeros(n ** dim, dtype=np.complex128)
    for col, j in enumerate(idx):
        e[:] = 0
        e[j] = 1
        A[:, col] = apply_H(e.reshape((n,) * dim), level, theta, phi, conjugate).ravel()[idx]
    return A


def norm_h(r: np.ndarray, level: int) -> float:
    """|r|_h = (sum_i |h|^d |r_i|^2)^(1/2) over interior vertices (Section 7),
    |h| the real cell width of the level."""
    dim = r.ndim
    n = r.shape[0]
    m = interior_mask(n, dim)
    h = 3.0 ** (-level)
    return float(np.sqrt(h ** dim * np.sum(np.abs(r[m]) ** 2)))


def norm_max(r: np.ndarray) -> float:
    m = interior_mask(r.shape[0], r.ndim)
    return float(np.max(np.abs(r[m]))) if m.any() else 0.0
