"""Oracle: the additive multilevel cycles of the paper, level by level.

Test infrastructure only (see the package header).

Four formulations of one cycle, kept separate so that each cross-checks the
others:

* `textbook_additive`  -- Algorithm 1 ("add"), the correction scheme with zero
  coarse start, coarse weight omega_cg = 1 (constant phi only: for varying phi
  its rediscretised coarse correction differs from FAS by design);
* `bottom_up_fas`      -- the appendix algorithm "buFAS" (recursive, unpipelined
  FAS) with its BPX prolongation of u_(l-1) - I(u_l + du_l);
* `semantic_cycle`     -- the same map unrolled: FAS right-hand sides top-down
  (eq. HTMG), one damped Jacobi step per level, corrections summed bottom-up
  with the variant's level operator (identity for add, c-point mask for hb,
  s - P I s for BPX);
* `Pipelined`          -- the single-sweep Algorithms tdAdd / tdBPX with helpers
  sc, sf, si, linearised level by level: parents before children on the way
  down (pre-phase) and children before parents on the way back (post-phase).

Contract: n pipelined cycles followed by a flush equal n semantic cycles; the
residual reported by pipelined cycle n is that of iterate n-1 (Section 5: the
update is shifted by half an iteration).
"""

from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

from .discretisation import (apply_H, cell_theta, coarse_fields, diag_H, interior_mask,
                             norm_h, norm_max, zero_boundary)
from .transfer import cpoint_mask, inject, prolong, restrict

VARIANTS = ("add", "hb", "bpx")
OMEGA_SCHEMES = ("const", "jacobi", "lgrid", "exp", "transition", "two_phase")


@dataclasses.dataclass
class Params:
    dim: int
    level_max: int
    level_min: int = 1
    theta: float = 0.0
    phi: complex = 0.0
    phi_nodal: Optional[np.ndarray] = None   # finest-level nodal phi (varying case)
    variant: str = "add"
    omega_scheme: str = "const"
    omega: complex = 0.6
    omega_L: int = 1                          # grid count bound of the L-grid scheme
    conjugate: bool = False
    layer: Optional[tuple] = None             # absorbing layer (angle, width, faces), Section 7.4

    def __post_init__(self):
        assert self.variant in VARIANTS
        assert self.omega_scheme in OMEGA_SCHEMES
        assert 1 <= self.level_min <= self.level_max
        self._phi = None
        self._diag = {}

    @property
    def levels(self):
        return range(self.level_min, self.level_max + 1)

    def n(self, level: int) -> int:
        return 3 ** level + 1

    def phi_at(self, level: int):
        """phi on a level: the constant, or the injected nodal field."""
        if self.phi_nodal is None:
            return self.phi
        if self._phi is None:
            self._phi = coarse_fields(self.phi_nodal, self.level_max, self.level_min)
        return self._phi[level]

    def theta_at(self, level: int):
        """Rotation of the level's cells: theta, or per cell with the layer
        (each level's cells are classified by their own centres)."""
        return cell_theta(level, self.dim, self.theta, self.layer)

    def H(self, v: np.ndarray, level: int) -> np.ndarray:
        return apply_H(v, level, self.theta_at(level), self.phi_at(level), self.conjugate)

    def D(self, level: int) -> np.ndarray:
        if level not in self._diag:
            self._diag[level] = diag_H(self.n(level), self.dim, level, self.theta_at(level),
                                       self.phi_at(level), self.conjugate)
        return self._diag[level]

    def cpoints(self, level: int) -> np.ndarray:
        return cpoint_mask(self.n(level), self.dim, level, self.level_min)


def omega_levels(p: Params, iteration: int = 1) -> Dict[int, complex]:
    """Per-level relaxation omega_l (the table of Section 5.1) on a regular
    grid, where succ(v) = l_max - l for every interior vertex of level l.

    const       omega on every level ("undamped coarse grid correction")
    jacobi      omega on the finest level only, 0 elsewhere
    lgrid       omega where succ <= omega_L, 0 elsewhere
    exp         omega^(succ + 1)                      (exponential damping)
    transition  omega^((1 - 1/n)(succ + 1)), n the iteration counter (n >= 1)
    two_phase   omega on odd n, -conj(omega) on even n, every level (the
                two-phase relaxation of Section 7.4; pinned against explicit
                Jacobi steps with a dense matrix in tests/test_oracle_cycle.py)
    """
    out = {}
    for lev in p.levels:
        succ = p.level_max - lev
        w = complex(p.omega)
        if p.omega_scheme == "const":
            out[lev] = w
        elif p.omega_scheme == "jacobi":
            out[lev] = w if succ == 0 else 0j
        elif p.omega_scheme == "lgrid":
            out[lev] = w if succ <= p.omega_L else 0j
        elif p.omega_scheme == "exp":
            out[lev] = w ** (succ + 1)
        elif p.omega_scheme == "two_phase":
            out[lev] = w if iteration % 2 == 1 else -np.conj(w)
        else:
            out[lev] = w ** ((1.0 - 1.0 / iteration) * (succ + 1))
    return out


def _smooth(p: Params, level: int, r: np.ndarray, omega: complex) -> np.ndarray:
    """omega S = omega diag(H)^-1 r, zero on the boundary."""
    return zero_boundary(omega * r / p.D(level))


def _level_operator(p: Params, level: int, s: np.ndarray) -> np.ndarray:
    """What a level adds of its own smoothing update in each variant."""
    if level == p.level_min or p.variant == "add":
        return s
    if p.variant == "hb":
        return np.where(p.cpoints(level), 0, s)
    return s - prolong(inject(s))      # BPX: s - P I s


def semantic_cycle(p: Params, u: np.ndarray, b: np.ndarray, iteration: int = 1):
    """One additive FAS cycle as a map u -> u + Delta_L.  Returns the new finest
    iterate and the h- and max-norms of the finest residual of the input u."""
    L, lmin = p.level_max, p.level_min
    om = omega_levels(p, iteration)
    us = {L: zero_boundary(u)}
    bs = {L: zero_boundary(b)}
    for lev in range(L, lmin, -1):
        us[lev - 1] = inject(us[lev])
        uhat = us[lev] - prolong(us[lev - 1])
        bs[lev - 1] = restrict(bs[lev] - p.H(uhat, lev))
    s = {}
    rL = None
    for lev in p.levels:
        r = zero_boundary(bs[lev] - p.H(us[lev], lev))
        if lev == L:
            rL = r
        s[lev] = _smooth(p, lev, r, om[lev])
    delta = s[lmin]
    for lev in range(lmin + 1, L + 1):
        delta = _level_operator(p, lev, s[lev]) + prolong(delta)
    return us[L] + delta, norm_h(rL, L), norm_max(rL)


def zero_start_cycle(p: Params, v: np.ndarray, iteration: int = 1) -> np.ndarray:
    """One cycle from u = 0 with right-hand side v: the additive preconditioner
    B v (no operator application survives because every u_l is zero)."""
    out, _, _ = semantic_cycle(p, np.zeros_like(v, dtype=np.complex128), v, iteration)
    return out


def textbook_additive(p: Params, u: np.ndarray, chi: np.ndarray, iteration: int = 1,
                      omega_S=None, omega_cg: complex = 1.0) -> np.ndarray:
    """Algorithm 1 (add variant, correction scheme).  With omega_S = None the
    smoother weight is the level's omega_l from the scheme table; otherwise the
    constant omega_S, and omega_cg damps every coarse-grid contribution."""
    om = omega_levels(p, iteration)

    def add(lev, u_l, chi_l):
        r = zero_boundary(chi_l - p.H(u_l, lev))
        u_l = u_l + _smooth(p, lev, r, om[lev] if omega_S is None else omega_S)
        if lev > p.level_min:
            u_c = add(lev - 1, np.zeros((p.n(lev - 1),) * p.dim, dtype=np.complex128), restrict(r))
            u_l = u_l + omega_cg * prolong(u_c)
        return u_l

    return add(p.level_max, zero_boundary(u), zero_boundary(chi))


def bottom_up_fas(p: Params, u: np.ndarray, b: np.ndarray, iteration: int = 1) -> np.ndarray:
    """The appendix's recursive bottom-up FAS ("buFAS"), invoked on l_max."""
    om = omega_levels(p, iteration)
    us = {p.level_max: zero_boundary(u)}
    bs = {p.level_max: zero_boundary(b)}

    def rec(lev):
        du = _smooth(p, lev, zero_boundary(bs[lev] - p.H(us[lev], lev)), om[lev])
        if p.variant == "hb" and lev > p.level_min:
            du = np.where(p.cpoints(lev), 0, du)
        if lev == p.level_min:
            us[lev] = us[lev] + du
            return
        us[lev - 1] = inject(us[lev])
        uhat = us[lev] - prolong(us[lev - 1])
        bs[lev - 1] = restrict(bs[lev] - p.H(uhat, lev))
        rec(lev - 1)
        if p.variant == "bpx":
            us[lev] = us[lev] + du + prolong(us[lev - 1] - inject(us[lev] + du))
        else:
            us[lev] = us[lev] + du + prolong(us[lev - 1] - inject(us[lev]))

    rec(p.level_max)
    return us[p.level_max]


class Pipelined:
    """Single-sweep pipelined FAS (Algorithms tdAdd and tdBPX; hb is tdAdd with
    the c-point mask of eq. hb-omega), level-ordered.

    State per level: u, b (coarse b is written by the finer level's
    post-phase), sc, sf, si.  At start-up sc = sf = si = 0 and coarse u is the
    injection of the finest u.
    """

    def __init__(self, p: Params, b: np.ndarray, u0: Optional[np.ndarray] = None):
        self.p = p
        L, lmin = p.level_max, p.level_min
        shape = lambda lev: (p.n(lev),) * p.dim
        uL = zero_boundary(np.zeros(shape(L)) if u0 is None else u0)
        self.u = {L: uL}
        for lev in range(L, lmin, -1):
            self.u[lev - 1] = inject(self.u[lev])
        self.b = {lev: np.zeros(shape(lev), dtype=np.complex128) for lev in p.levels}
        self.b[L] = zero_boundary(b)
        self.sc = {lev: np.zeros(shape(lev), dtype=np.complex128) for lev in p.levels}
        self.sf = {lev: np.zeros(shape(lev), dtype=np.complex128) for lev in p.levels}
        self.si = {lev: np.zeros(shape(lev), dtype=np.complex128) for lev in p.levels}
        self.iteration = 0
        self.uhat = {}
        self.residual = None

    def pre(self, lev: int) -> None:
        """Descent part of tdAdd / tdBPX on one level."""
        p = self.p
        if lev > p.level_min:
            self.sc[lev] = self.sc[lev] + prolong(self.sc[lev - 1])
            if p.variant == "bpx":
                self.sc[lev] = self.sc[lev] - np.where(p.cpoints(lev), 0, prolong(self.si[lev - 1]))
        self.u[lev] = self.u[lev] + self.sc[lev] + self.sf[lev]
        if lev > p.level_min:
            self.uhat[lev] = self.u[lev] - prolong(self.u[lev - 1])

    def post(self, lev: int, omega: complex) -> None:
        """Backtracking part of tdAdd / tdBPX on one level."""
        p = self.p
        r = zero_boundary(self.b[lev] - p.H(self.u[lev], lev))
        if lev == p.level_max:
            self.residual = r
        s = _smooth(p, lev, r, omega)
        if p.variant in ("hb", "bpx"):
            self.sc[lev] = np.where(p.cpoints(lev), 0, s)
        else:
            self.sc[lev] = s
        if lev > p.level_min:
            rhat = zero_boundary(self.b[lev] - p.H(self.uhat[lev], lev))
            if p.variant == "bpx":
                self.si[lev - 1] = inject(s)
            self.b[lev - 1] = restrict(rhat)
            self.sf[lev - 1] = inject(self.sf[lev] + self.sc[lev])

    def cycle(self):
        """One traversal; returns (|r|_h, |r|_max) of the iterate it started from."""
        self.iteration += 1
        om = omega_levels(self.p, self.iteration)
        for lev in self.p.levels:
            self.pre(lev)
        for lev in reversed(list(self.p.levels)):
            self.post(lev, om[lev])
        L = self.p.level_max
        return norm_h(self.residual, L), norm_max(self.residual)

    def flush(self) -> np.ndarray:
        """Apply the pending update (pre-phase only), clear the helpers, and
        return the finest iterate."""
        for lev in self.p.levels:
            self.pre(lev)
        for lev in self.p.levels:
            self.sc[lev][...] = 0
            self.sf[lev][...] = 0
            self.si[lev][...] = 0
        return self.u[self.p.level_max].copy()

    def restricted_residual_state(self) -> dict:
        """The coarse fields the last cycle's post-phase wrote, formed from the
        finest residual instead of from each level's own FAS residual.

        With constant phi and a uniform rotation, Lemma 2 and the Galerkin
        identity R H_l P = H_(l-1) give b_(l-1) - H_(l-1) I u_l = R r_l, and
        Lemma 1 (u_(l-1) = I u_l when residuals are evaluated) turns this into
        r_(l-1) = R r_l on every coarse level, so r_l = R^(L-l) r_L.  The
        post-phase then forms s_l = omega_l r_l / D_l, sc_l (s_l, or 0 on
        c-points for hb / BPX), si_(l-1) = I s_l (BPX) and sf_(l-1) =
        I(sf_l + sc_l), from the finest level down.

        Returns {level: {"b": r_l, "sc", "sf", "si"}} for the coarse levels l < L
        ("b" holds the residual r_l = b_l - H_l u_l).  Unlike b_l - H_l u_l,
        whose two terms grow with the iterate while their difference shrinks,
        nothing here is formed by cancellation: the values carry rounding
        relative to their own size.  Valid for the Galerkin case only; pinned
        against the pipeline's own post-phase in tests/test_oracle_cycle.py.
        """
        p = self.p
        L, lmin = p.level_max, p.level_min
        assert p.phi_nodal is None and p.layer is None, \
            "the restricted-residual form needs a constant phi and a uniform rotation"
        om = omega_levels(p, self.iteration)
        r = {L: zero_boundary(self.residual)}
        for lev in range(L, lmin, -1):
            r[lev - 1] = restrict(r[lev])
        out = {lev: {"b": r[lev]} for lev in p.levels if lev < L}
        sf_l = self.sf[L]
        for lev in range(L, lmin - 1, -1):
            s = _smooth(p, lev, r[lev], om[lev])
            sc = np.where(p.cpoints(lev), 0, s) if p.variant in ("hb", "bpx") else s
            if lev < L:
                out[lev]["sc"] = sc
            if lev > lmin:
                out[lev - 1]["si"] = inject(s) if p.variant == "bpx" else self.si[lev - 1].copy()
                out[lev - 1]["sf"] = inject(sf_l + sc)
                sf_l = out[lev - 1]["sf"]
        for lev in range(lmin, L):
            out[lev].setdefault("sf", self.sf[lev].copy())
            out[lev].setdefault("si", self.si[lev].copy())
        return out

    def state(self) -> dict:
        return {"u": {k: v.copy() for k, v in self.u.items()},
                "b": {k: v.copy() for k, v in self.b.items()},
                "sc": {k: v.copy() for k, v in self.sc.items()},
                "sf": {k: v.copy() for k, v in self.sf.items()},
                "si": {k: v.copy() for k, v in self.si.items()}}
