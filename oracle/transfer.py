"""Oracle: geometric grid transfers between 3-partitioned levels.

Test infrastructure only (see the package header).

Section 4 of the paper: P is d-linear interpolation from level l-1 to level l
(each coarse cell splits into 3 per axis), R = P^T, and I is injection (plain
copy of the coinciding vertex).  The factor-3 linear weights are not printed in
the paper; they follow from linear interpolation: a fine vertex at offset
o = j - 3m from coarse vertex m gets weight 1 - |o|/3.

P is the tensor product of a 1D interpolation matrix, applied axis by axis.
Pinned by: exact reproduction of d-linear functions, R = P^T as a bilinear
identity, I P = id, and the Galerkin identity R H_l P = H_(l-1).
"""

from __future__ import annotations

import numpy as np

from .discretisation import zero_boundary


def prolong_matrix_1d(n_coarse: int) -> np.ndarray:
    """1D linear interpolation, shape (3 (n_coarse - 1) + 1, n_coarse)."""
    n_fine = 3 * (n_coarse - 1) + 1
    P = np.zeros((n_fine, n_coarse))
    for m in range(n_coarse):
        for o in range(-2, 3):
            j = 3 * m + o
            if 0 <= j < n_fine:
                P[j, m] = 1.0 - abs(o) / 3.0
    return P


def _along_axes(mat: np.ndarray, v: np.ndarray) -> np.ndarray:
    out = np.asarray(v, dtype=np.complex128)
    for a in range(out.ndim):
        out = np.moveaxis(np.tensordot(mat, out, axes=(1, a)), 0, a)
    return out


def prolong(vc: np.ndarray) -> np.ndarray:
    """P v: d-linear interpolation of a coarse vertex field to the next finer level."""
    return _along_axes(prolong_matrix_1d(vc.shape[0]), vc)


def restrict(vf: np.ndarray) -> np.ndarray:
    """R v = P^T v, boundary entries of the coarse result set to zero (they carry
    no unknowns under zero Dirichlet conditions)."""
    nc = (vf.shape[0] - 1) // 3 + 1
    return zero_boundary(_along_axes(prolong_matrix_1d(nc).T, vf))


def inject(vf: np.ndarray) -> np.ndarray:
    """I v: the value at the fine vertex that coincides with each coarse vertex."""
    return np.array(vf[(slice(None, None, 3),) * vf.ndim], dtype=np.complex128)


def cpoint_mask(n: int, dim: int, level: int, level_min: int) -> np.ndarray:
    """cPoint(v): the vertex coincides with a vertex of the next coarser level
    (Section 5.1).  On the coarsest compute level no coarser compute level
    exists and the predicate is false."""
    m = np.zeros((n,) * dim, dtype=bool)
    if level > level_min:
        m[(slice(None, None, 3),) * dim] = True
    return m
