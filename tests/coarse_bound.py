"""Tolerance of the coarse-level fields in the Galerkin form.

With a constant phi the coarse residual is r_l = R^(L-l) r_L (Lemmas 1 and
2), and the coarse smoothing fields are pointwise functions of it.  R has
nonnegative weights, so an entrywise deviation |delta| <= eps |r_L| of the
finest residual reaches level l as |R^k delta| <= eps R^k |r_L| (k = L - l).
Relative to the field's own norm the bound is eps c_l with

    c_l = |R^k |r_L|| / |R^k r_L|  >= 1,

the cancellation factor of the restriction chain on this residual: as the
iteration converges the coarse residuals become small differences of large
fine contributions and c_l grows (about 1.3e3 on level 1 of the 2D k = 10
workload after 30 cycles).  A field on level l is held to eps max(c_m, m >= l),
the largest factor among the levels whose residuals it is built from (sf
collects the injected corrections of every finer level).
"""

import numpy as np

import oracle as O


def chain_factors(pipe) -> dict:
    """{level: max over m >= level (m < L) of c_m} for the pipeline's last
    finest residual; 1 on the finest level."""
    p = pipe.p
    L, lmin = p.level_max, p.level_min
    r = O.zero_boundary(pipe.residual)
    a = np.abs(r).astype(np.complex128)
    c = {L: 1.0}
    for lev in range(L - 1, lmin - 1, -1):
        r, a = O.restrict(r), O.restrict(a)
        nr = np.linalg.norm(r)
        c[lev] = max(c[lev + 1], np.linalg.norm(a) / nr if nr > 0 else 1.0)
    return c
