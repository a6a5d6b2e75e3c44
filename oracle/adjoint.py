"""Oracle: shell functional and its gradient with respect to the potential.

Test infrastructure only (see the package header).

Not in the paper: the stand-in for its far-field post-processing (Section 2)
is J(u) = sum_{j in S} |u_j|^2 over a spherical shell S of vertices, with u
solving H(V) u = b for  -Lap u + (V - phi0) u = chi,  i.e. nodal
phi = phi0 - V.  V enters H only through the cell averages of phi, so

    dH_c / dV_j = +2^-d eta^d M   for each cell c containing vertex j,

and with the adjoint lambda = H^-H (1_S u):

    dJ/dV_j = -2 Re sum_{c containing j} 2^-d eta^d  lambda_c^H M u_c .

Pinned by central finite differences with dense solves on tiny grids.
"""

from __future__ import annotations

import numpy as np

from .discretisation import _cell_view, corners, element_matrices, level_eta


def shell_functional(u: np.ndarray, shell: np.ndarray) -> float:
    return float(np.sum(np.abs(u[shell]) ** 2))


def potential_gradient(u: np.ndarray, lam: np.ndarray, level: int, theta: float) -> np.ndarray:
    """dJ/dV at every vertex from the forward solution u and the adjoint lam
    (both zero on the boundary), by the cell-wise formula above."""
    dim = u.ndim
    _, M = element_matrices(dim)
    eta = level_eta(level, theta)
    cs = corners(dim)
    U = np.stack([u[_cell_view(u, k)] for k in cs])
    Lm = np.stack([lam[_cell_view(lam, k)] for k in cs])
    MU = np.tensordot(M, U, axes=(1, 0))
    cellval = np.sum(np.conj(Lm) * MU, axis=0)           # lambda_c^H M u_c per cell
    contrib = -2.0 * np.real(eta ** dim * cellval) / 2 ** dim
    g = np.zeros(u.shape)
    for k in cs:
        g[_cell_view(g, k)] += contrib
    return g
