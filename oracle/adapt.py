"""Oracle: feature-based dynamic adaptivity on a dense envelope of levels.

Test infrastructure only (see the package header).

Section 5.3 of the paper: per vertex and level the criterion
s = max over axes a of |Delta_a u|; the span of s is cut into 20 equal
subranges, the vertices of the top bins (as many bins as bring the count
closest to 10 %) are refined, those of the bottom bins (closest to 2 %) are
erased; both are vetoed where the mesh-size limits would be broken or where
|r| / |diag| exceeds 1e-2.  Section 4: a hanging vertex takes its value from
the next coarser level through P, and so does a vertex a refinement creates
(its hierarchical surplus starts at zero).

The grid is a spacetree whose every level is held as a full regular array
(the envelope): level l has 3^l + 1 vertices per axis, and its state is one
flag per cell ("this cell is refined into 3^d cells of level l+1").  A cell of
level l exists when l is the coarsest level or its parent cell is refined.

Readings (where the paper leaves a choice open; the HIP path takes the same):
  * Delta_a u is the undivided second difference along axis a,
    u(j + e_a) - 2 u(j) + u(j - e_a), evaluated in FP64 as
    (u(j + e_a) + u(j - e_a)) - (u(j) + u(j)) per component, |.|^2 as
    re*re + im*im with no fused multiply-add, s as the square root of the
    largest |.|^2 over the axes.
  * The candidates of a level are its persistent vertices (interior, every
    adjacent cell present); bins and the 10 % / 2 % targets count only them,
    and are taken per level.  Bin b of value s is
    floor(nbins (s - s_min) / (s_max - s_min)), the top value going to the top
    bin; with s_max = s_min every candidate sits in bin 0.
  * The number k of top bins minimises |100 count(top k) - pct N| over
    k = 0..nbins, the smaller k on ties; the number e of bottom bins does the
    same over e = 0..nbins - k for the erase percentage.
  * Refining vertex v of level l refines its 2^d adjacent cells of level l
    (vetoed on the finest level of the envelope); erasing it returns those cells
    to leaves (vetoed below the coarsest-mesh level level_keep, and per cell if
    a refine mark of the same step also touches it or one of the cell's
    children is refined after the step, so that no refined cell is orphaned).
  * The residual veto compares |r|^2 > veto^2 |diag|^2 (same rounding as
    |r| / |diag| > veto up to ties) with the level's constant diagonal.
  * Vertex classes after a step: absent (no adjacent cell present), persistent
    (interior, all 2^d adjacent cells present), hanging (interior, some but not
    all present), boundary (on the domain boundary, some adjacent cell present).
    A hanging vertex, and one that becomes persistent, takes P u_(l-1); one
    that becomes absent or boundary is set to zero (homogeneous Dirichlet
    data); every other vertex keeps its value (Section 5.3 gives values only
    to the vertices a step creates).

Pinned by: the closed form of s for quadratic and d-linear fields, hand-counted
bins and bin choices, hand-built refinement patterns in 2D and the closed-form
vertex classes of a refined block, exact interpolation of d-linear fields.
"""

from __future__ import annotations

import itertools

import numpy as np

from .transfer import prolong

ABSENT, PERSISTENT, HANGING, BOUNDARY = 0, 1, 2, 3
KEEP, REFINE, ERASE = 0, 1, 2


def _shift(a: np.ndarray, axis: int, off: int) -> np.ndarray:
    """a at j + off e_axis for every interior index j (interior-shaped view)."""
    idx = [slice(1, -1)] * a.ndim
    idx[axis] = slice(1 + off, a.shape[axis] - 1 + off)
    return a[tuple(idx)]


def criterion(u: np.ndarray) -> np.ndarray:
    """s = max_a |Delta_a u| on interior vertices, zero on the boundary."""
    u = np.asarray(u, dtype=np.complex128)
    c = u[(slice(1, -1),) * u.ndim]
    best = np.zeros(c.shape)
    for a in range(u.ndim):
        p, m = _shift(u, a, 1), _shift(u, a, -1)
        dre = (p.real + m.real) - (c.real + c.real)
        dim_ = (p.imag + m.imag) - (c.imag + c.imag)
        m2 = np.add(np.multiply(dre, dre), np.multiply(dim_, dim_))
        best = np.maximum(best, m2)
    s = np.zeros(u.shape)
    s[(slice(1, -1),) * u.ndim] = np.sqrt(best)
    return s


def bin_index(s: np.ndarray, s_min: float, s_max: float, nbins: int) -> np.ndarray:
    """Equal subranges of [s_min, s_max]; the top value falls into the top bin."""
    if not s_max > s_min:
        return np.zeros(s.shape, dtype=np.int64)
    q = np.floor(((s - s_min) / (s_max - s_min)) * float(nbins)).astype(np.int64)
    return np.minimum(q, nbins - 1)


def choose_bins(counts: np.ndarray, n: int, refine_pct: int, erase_pct: int):
    """(k, e): numbers of top and bottom bins whose counts come closest to the
    refine and erase percentages of n; ties go to fewer bins."""
    nb = len(counts)
    best_k, best_d = 0, None
    for k in range(nb + 1):
        c = int(sum(counts[nb - k:])) if k else 0
        d = abs(100 * c - refine_pct * n)
        if best_d is None or d < best_d:
            best_k, best_d = k, d
    best_e, best_d = 0, None
    for e in range(nb - best_k + 1):
        c = int(sum(counts[:e]))
        d = abs(100 * c - erase_pct * n)
        if best_d is None or d < best_d:
            best_e, best_d = e, d
    return best_k, best_e


def mark_level(u, r, diag, cls, level, level_keep, level_max, nbins=20, refine_pct=10, erase_pct=2,
               veto=1e-2):
    """Marks of one level: KEEP / REFINE / ERASE per vertex, and the statistics
    (bin counts, k, e, candidates, s_min, s_max)."""
    u = np.asarray(u, dtype=np.complex128)
    cand = cls == PERSISTENT
    s = criterion(u)
    n = int(cand.sum())
    if n == 0:
        return np.zeros(u.shape, dtype=np.uint8), dict(counts=np.zeros(nbins, np.int64), k=0, e=0, n=0,
                                                      s_min=0.0, s_max=0.0)
    s_min, s_max = float(s[cand].min()), float(s[cand].max())
    b = bin_index(s, s_min, s_max, nbins)
    counts = np.bincount(b[cand], minlength=nbins).astype(np.int64)
    k, e = choose_bins(counts, n, refine_pct, erase_pct)
    vetoed = np.zeros(u.shape, dtype=bool)
    if r is not None:
        r = np.asarray(r, dtype=np.complex128)
        r2 = np.add(np.multiply(r.real, r.real), np.multiply(r.imag, r.imag))
        d2 = np.add(np.multiply(diag.real, diag.real), np.multiply(diag.imag, diag.imag))
        vetoed = r2 > np.multiply(veto * veto, d2)
    marks = np.zeros(u.shape, dtype=np.uint8)
    if level < level_max:
        marks[cand & ~vetoed & (b >= nbins - k)] = REFINE
    if level >= level_keep:
        marks[cand & ~vetoed & (b < e)] = ERASE
    return marks, dict(counts=counts, k=k, e=e, n=n, s_min=s_min, s_max=s_max)


def regular_cells(dim: int, level_min: int, level_keep: int, level_max: int) -> dict:
    """Refined-cell flags of the regular grid of level level_keep."""
    return {l: np.full((3 ** l,) * dim, 1 if l < level_keep else 0, dtype=np.uint8)
            for l in range(level_min, level_max)}


def cell_exists(cells: dict, level: int, level_min: int, dim: int) -> np.ndarray:
    """Presence of every cell of a level: the coarsest level is whole; below it
    a cell is present where its parent is refined."""
    if level == level_min:
        return np.ones((3 ** level,) * dim, dtype=bool)
    par = cells[level - 1].astype(bool)
    for a in range(dim):
        par = np.repeat(par, 3, axis=a)
    return par


def _any_corner(marks: np.ndarray, value: int) -> np.ndarray:
    """For every cell, whether one of its 2^d vertices carries the mark."""
    dim = marks.ndim
    nc = marks.shape[0] - 1
    out = np.zeros((nc,) * dim, dtype=bool)
    for k in itertools.product((0, 1), repeat=dim):
        out |= marks[tuple(slice(kk, kk + nc) for kk in k)] == value
    return out


def _any_child(cells_fine: np.ndarray) -> np.ndarray:
    """For every cell of the coarser level, whether one of its 3^d children is refined."""
    dim = cells_fine.ndim
    nc = cells_fine.shape[0] // 3
    return cells_fine.reshape(sum(((nc, 3) for _ in range(dim)), ())).astype(bool).any(
        axis=tuple(range(1, 2 * dim, 2)))


def adapt(cells: dict, marks: dict, dim: int, level_min: int, level_max: int) -> dict:
    """One adaptation step: the refined-cell flags of every level after the
    marks of every level are applied (marks[l] may be missing: no marks)."""
    new = {}
    for l in range(level_max - 1, level_min - 1, -1):
        old = cells[l].astype(bool)
        exists = cell_exists(cells, l, level_min, dim)
        m = marks.get(l)
        any_r = _any_corner(m, REFINE) if m is not None else np.zeros_like(old)
        any_e = _any_corner(m, ERASE) if m is not None else np.zeros_like(old)
        child = _any_child(new[l + 1]) if l + 1 < level_max else np.zeros_like(old)
        keep = old & ~(any_e & ~child)
        new[l] = (exists & (any_r | keep)).astype(np.uint8)
    return new


def classify(cells: dict, dim: int, level_min: int, level: int) -> np.ndarray:
    """Vertex classes of one level from the refined-cell flags."""
    n = 3 ** level + 1
    ex = cell_exists(cells, level, level_min, dim)
    cnt = np.zeros((n,) * dim, dtype=np.int64)
    for k in itertools.product((0, 1), repeat=dim):
        # the cell at v - k holds vertex v as its corner k
        cnt[tuple(slice(kk, kk + n - 1) for kk in k)] += ex
    cls = np.full((n,) * dim, ABSENT, dtype=np.uint8)
    inner = np.zeros((n,) * dim, dtype=bool)
    inner[(slice(1, -1),) * dim] = True
    cls[inner & (cnt == 2 ** dim)] = PERSISTENT
    cls[inner & (cnt > 0) & (cnt < 2 ** dim)] = HANGING
    cls[~inner & (cnt > 0)] = BOUNDARY
    return cls


def interpolate(cls_old: np.ndarray, cls_new: np.ndarray, u_coarse: np.ndarray, u_fine: np.ndarray) -> np.ndarray:
    """Level values after a step: hanging and newly persistent vertices take
    P u_coarse, vertices that became absent or boundary are set to zero, the
    rest keep theirs."""
    out = np.array(u_fine, dtype=np.complex128, copy=True)
    pu = prolong(u_coarse)
    take = (cls_new == HANGING) | ((cls_new == PERSISTENT) & (cls_old != PERSISTENT))
    out[take] = pu[take]
    gone = ((cls_new == ABSENT) | (cls_new == BOUNDARY)) & (cls_new != cls_old)
    out[gone] = 0
    return out
