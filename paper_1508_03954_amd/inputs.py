"""Seeded synthetic inputs for the complex Helmholtz multilevel workloads.

This module only draws random numbers and samples analytic source/potential
functions at grid vertices.  It holds none of the solver's arithmetic (no
operator, transfer, smoother or cycle), so both the FP64 oracle and the HIP
path take their inputs from here.

Geometry: the unit hypercube (0,1)^d, level l has 3^l cells per axis and
n_l = 3^l + 1 vertices per axis, boundary included (the regular spacetree of
the paper's Section 3).  Arrays are C-ordered numpy arrays of shape (n_l,)*d;
the last axis is x (fastest).  Vertex j sits at the real position j * 3^-l.

The right-hand sides follow the paper's benchmark families: Gaussian loads
(the application problem of Section 7.4 uses a Gaussian chi) and the
manufactured product-of-sines load of the Poisson study (Section 7.1).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def n_vertices(level: int) -> int:
    """Vertices per axis on a level of the regular 3-partitioned tree."""
    return 3 ** level + 1


def vertex_coords(level: int, dim: int) -> List[np.ndarray]:
    """Real vertex coordinates per numpy axis, broadcastable to (n,)*dim."""
    n = n_vertices(level)
    x = np.arange(n, dtype=np.float64) / 3 ** level
    out = []
    for a in range(dim):
        shape = [1] * dim
        shape[a] = n
        out.append(x.reshape(shape))
    return out


def gaussian(level: int, dim: int, centre: Sequence[float], sigma: float) -> np.ndarray:
    """exp(-|x - centre|^2 / (2 sigma^2)) sampled at the vertices of a level."""
    xs = vertex_coords(level, dim)
    r2 = sum((xs[a] - centre[a]) ** 2 for a in range(dim))
    return np.exp(-r2 / (2.0 * sigma * sigma))


def sine_load(level: int, dim: int) -> np.ndarray:
    """d pi^2 prod_i sin(pi x_i): the manufactured load whose Poisson solution is
    prod_i sin(pi x_i) (the paper's Poisson benchmark, index i running over the d
    coordinates)."""
    xs = vertex_coords(level, dim)
    v = np.ones((n_vertices(level),) * dim)
    for a in range(dim):
        v = v * np.sin(np.pi * xs[a])
    return dim * np.pi ** 2 * v


def sine_solution(level: int, dim: int) -> np.ndarray:
    xs = vertex_coords(level, dim)
    v = np.ones((n_vertices(level),) * dim)
    for a in range(dim):
        v = v * np.sin(np.pi * xs[a])
    return v


def random_complex(shape, seed) -> np.ndarray:
    """Uniform complex entries, real and imaginary parts in [-1, 1)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


@dataclasses.dataclass
class Problem:
    """One Helmholtz problem  -Lap u - phi u = chi  on (0,1)^dim, zero Dirichlet.

    phi is either the constant `phi` or, when `potential` is given, the nodal
    field phi(x) = phi - V(x) on the finest level.  theta is the complex grid
    rotation h -> h exp(i theta).
    """

    name: str
    dim: int
    level_max: int
    level_min: int
    theta: float
    phi: complex
    chi: np.ndarray                     # nodal load on the finest level, complex128
    potential: Optional[np.ndarray] = None   # nodal real V(x) on the finest level
    variant: str = "bpx"
    omega: complex = 0.6
    cycles: int = 30
    phi_nodal: Optional[np.ndarray] = None   # nodal phi(x) on the finest level (replaces phi)
    layer: Optional[Tuple[float, float, int]] = None   # absorbing layer: angle, width, face bits

    @property
    def n(self) -> int:
        return n_vertices(self.level_max)

    def phi_field(self) -> Optional[np.ndarray]:
        if self.phi_nodal is not None:
            return np.asarray(self.phi_nodal, dtype=np.complex128)
        if self.potential is None:
            return None
        return (self.phi - self.potential).astype(np.complex128)


def config_2d_bpx(level_max: int = 5, seed: int = 1) -> Problem:
    """2D, k = 10, CSL shift phi = k^2 (1 + 0.5i), theta = 0, one Gaussian load
    (sigma 0.05, centre uniform in [0.3, 0.7]^2), BPX, omega 0.6, 30 cycles."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, 2)
    chi = gaussian(level_max, 2, c, 0.05).astype(np.complex128)
    return Problem("2d_bpx_k10", 2, level_max, 1, 0.0, 100.0 * (1 + 0.5j), chi,
                   variant="bpx", omega=0.6, cycles=30)


def config_3d_csg(level_max: int = 5, seed: int = 2, variant: str = "bpx") -> Problem:
    """3D, k = 20, real phi = k^2, complex grid rotation theta = pi/6.  Load: sum
    of four Gaussians (sigma 0.05, centres uniform in [0.2, 0.8]^3) plus uniform
    complex noise of amplitude 1e-3 at every vertex.  50 cycles."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, (4, 3))
    chi = np.zeros((n_vertices(level_max),) * 3, dtype=np.complex128)
    for m in range(4):
        chi += gaussian(level_max, 3, centres[m], 0.05)
    shape = chi.shape
    chi += 1e-3 * (rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape))
    return Problem("3d_csg_k20_" + variant, 3, level_max, 1, math.pi / 6, 400.0 + 0j, chi,
                   variant=variant, omega=0.6, cycles=50)


def config_3d_large(level_max: int = 6, seed: int = 3) -> Problem:
    """3D, k = 40, CSL shift phi = k^2 (1 + 0.5i), theta = 0, one Gaussian load
    (sigma 0.05, centre uniform in [0.3, 0.7]^3)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, 3)
    chi = gaussian(level_max, 3, c, 0.05).astype(np.complex128)
    return Problem("3d_csl_k40", 3, level_max, 1, 0.0, 1600.0 * (1 + 0.5j), chi,
                   variant="bpx", omega=0.6, cycles=50)


def config_batched(seed: int = 4, n2d: int = 64, n3d: int = 32,
                   levels2d: Tuple[int, int] = (3, 6),
                   levels3d: Tuple[int, int] = (3, 5)) -> List[Problem]:
    """Many independent problems of uneven depth: finest levels uniform in the
    given inclusive ranges, k uniform in [5, 60], phi = k^2 (1 + 0.5i), one
    seeded Gaussian load each.  Problem i draws from seed (seed, i)."""
    out = []
    for i in range(n2d + n3d):
        rng = np.random.default_rng([seed, i])
        dim = 2 if i < n2d else 3
        lo, hi = levels2d if dim == 2 else levels3d
        L = int(rng.integers(lo, hi + 1))
        k = float(rng.uniform(5.0, 60.0))
        c = rng.uniform(0.3, 0.7, dim)
        chi = gaussian(L, dim, c, 0.05).astype(np.complex128)
        out.append(Problem(f"batch{i}_{dim}d_L{L}", dim, L, 1, 0.0, k * k * (1 + 0.5j), chi,
                           variant="bpx", omega=0.6, cycles=50))
    return out


def config_potential(level_max: int = 5, seed: int = 5) -> Problem:
    """3D, k = 15, potential V = sum of 8 Gaussians (amplitude in [-50, 50], sigma
    in [0.03, 0.1], centres in [0.1, 0.9]^3); phi(x) = k^2 (1 + 0.3i) - V(x);
    one Gaussian load (sigma 0.05, centre in [0.3, 0.7]^3)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-50, 50, 8)
    sig = rng.uniform(0.03, 0.1, 8)
    cen = rng.uniform(0.1, 0.9, (8, 3))
    V = np.zeros((n_vertices(level_max),) * 3)
    for m in range(8):
        V += amp[m] * gaussian(level_max, 3, cen[m], sig[m])
    c = rng.uniform(0.3, 0.7, 3)
    chi = gaussian(level_max, 3, c, 0.05).astype(np.complex128)
    return Problem("3d_potential_k15", 3, level_max, 1, 0.0, 225.0 * (1 + 0.3j), chi,
                   potential=V, variant="bpx", omega=0.6, cycles=50)


def config_gaussian08(theta_deg: float, level_max: int = 4) -> Problem:
    """The p = 2 application problem of Section 7.4 (eq. 08-gaussian) on the
    regular grid h = 3^-level_max (1/81 by default):
        chi(x, y) = exp(-(125 x)^2 - (125 y)^2),
        phi(x, y) = 45^2 + 135^2 (exp(-(15 x)^2) + exp(-(15 y)^2)),
    x and y measured from the corner at the origin (the centre of mass).  The
    faces x = 1 and y = 1 are open: the cells within 1/3 of them form an
    absorbing layer rotated by 30 degrees; every other cell is rotated by
    theta_deg.  The faces are bits 1 (x = 1) and 3 (y = 1) of the layer's
    face set, x being the fastest-varying coordinate."""
    xs = vertex_coords(level_max, 2)
    y, x = xs[0], xs[1]
    chi = np.exp(-(125.0 * x) ** 2 - (125.0 * y) ** 2) * np.ones((n_vertices(level_max),) * 2)
    phi = 45.0 ** 2 + 135.0 ** 2 * (np.exp(-(15.0 * x) ** 2) + np.exp(-(15.0 * y) ** 2))
    phi = np.broadcast_to(phi, chi.shape)
    return Problem(f"gaussian08_theta{theta_deg:g}", 2, level_max, 1, math.radians(theta_deg), 0j,
                   chi.astype(np.complex128), variant="bpx", omega=0.4, cycles=50,
                   phi_nodal=phi.astype(np.complex128),
                   layer=(math.radians(30.0), 1.0 / 3.0, (1 << 1) | (1 << 3)))


def shell_mask(level: int, dim: int, r_in: float = 0.9, r_out: float = 0.95) -> np.ndarray:
    """Vertices of the shell r_in < |x| < r_out around the origin (the corner
    of the domain where the paper's axes measure distance from the centre of
    mass)."""
    xs = vertex_coords(level, dim)
    r = np.sqrt(sum(x ** 2 for x in xs))
    return (r > r_in) & (r < r_out)


def sample_vertices(level: int, dim: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct interior vertex multi-indices, shape (count, dim)."""
    rng = np.random.default_rng(seed)
    n = n_vertices(level)
    seen = set()
    out = []
    while len(out) < count:
        j = tuple(int(v) for v in rng.integers(1, n - 1, dim))
        if j not in seen:
            seen.add(j)
            out.append(j)
    return np.array(out, dtype=np.int64)
