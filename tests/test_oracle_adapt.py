"""Pins of the adaptivity oracle (Section 5.3 criterion and bins, Section 4
hanging vertices) against closed forms and hand-counted cases."""

import numpy as np
import pytest

from oracle import adapt as A
from paper_1508_03954_amd.inputs import vertex_coords


def _coords(level, dim):
    return np.meshgrid(*vertex_coords(level, dim), indexing="ij")


@pytest.mark.parametrize("dim,level", [(2, 3), (3, 2)])
def test_criterion_of_a_quadratic_is_its_second_difference(dim, level):
    # u = sum_a c_a x_a^2 + linear + const: the undivided second difference
    # along axis a is 2 c_a h^2 at every interior vertex, so s = 2 h^2 max |c_a|
    h = 3.0 ** -level
    c = np.array([0.7 - 0.2j, -1.3 + 0.4j, 0.5 + 1.1j][:dim])
    X = _coords(level, dim)
    u = 0.3 + 0.1j + sum(c[a] * X[a] ** 2 + (0.2 * a - 0.5j) * X[a] for a in range(dim))
    s = A.criterion(u)
    inner = (slice(1, -1),) * dim
    want = 2 * h * h * np.abs(c).max()
    np.testing.assert_allclose(s[inner], want, rtol=0, atol=1e-13)
    assert np.all(s[~np.pad(np.ones((3 ** level - 1,) * dim, bool), 1)] == 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_criterion_vanishes_on_d_linear_fields(dim):
    X = _coords(3, dim)
    u = np.ones_like(X[0], dtype=np.complex128)
    for a in range(dim):
        u = u * ((0.4 + 0.3j) + (1.0 - 0.6j * a) * X[a])
    assert np.abs(A.criterion(u)).max() < 1e-14


def test_criterion_of_a_spike():
    # a unit spike at (4, 6) on a 10 x 10 grid: s = 2 there, 1 at the four
    # axis neighbours (one of their differences sees the spike), 0 elsewhere
    u = np.zeros((10, 10), np.complex128)
    u[4, 6] = 1j
    s = A.criterion(u)
    want = np.zeros((10, 10))
    want[4, 6] = 2
    for j in [(3, 6), (5, 6), (4, 5), (4, 7)]:
        want[j] = 1
    np.testing.assert_array_equal(s, want)


def test_bins_and_choice_by_hand():
    # 0, 20 and ten values in the middle of each of the 20 unit subranges of
    # [0, 20]: bins 0 and 19 hold 11, the others 10, N = 202
    s = np.concatenate([[0.0, 20.0], np.repeat(np.arange(20) + 0.5, 10)])
    b = A.bin_index(s, 0.0, 20.0, 20)
    counts = np.bincount(b, minlength=20)
    assert counts[0] == 11 and counts[19] == 11 and np.all(counts[1:19] == 10)
    # 10 % of 202 = 20.2: top 2 bins (21) beat 1 (11) and 3 (31);
    # 2 % = 4.04: no bin (0) beats bin 0 alone (11)
    assert A.choose_bins(counts, 202, 10, 2) == (2, 0)
    # 5 % = 10.1: bin 0 (11) is closer than nothing
    assert A.choose_bins(counts, 202, 10, 5) == (2, 1)
    # ties go to fewer bins: 75 % of 20 lies 5 from both 10 and 20
    assert A.choose_bins(np.array([10, 10]), 20, 75, 0) == (1, 0)


def test_mark_level_on_a_spike_with_and_without_veto():
    # level 2 in 2D (10 x 10), regular: 64 candidates; s = 2 at the spike, 1 at
    # its four neighbours, 0 at 59 vertices -> bins 19, 10 and 0.  Top 10 bins
    # hold 5 (|500 - 640| = 140, the least; k = 10..19 tie, fewer bins win);
    # erasing bin 0 (59) is farther from 2 % than erasing none.
    dim, level = 2, 2
    cells = A.regular_cells(dim, 1, 2, 3)
    cls = A.classify(cells, dim, 1, level)
    u = np.zeros((10, 10), np.complex128)
    u[4, 6] = 1
    diag = np.complex128(4.0 + 1.0j)
    marks, st = A.mark_level(u, None, diag, cls, level, level_keep=2, level_max=3)
    assert st["n"] == 64 and st["k"] == 10 and st["e"] == 0
    want = np.zeros((10, 10), np.uint8)
    for j in [(4, 6), (3, 6), (5, 6), (4, 5), (4, 7)]:
        want[j] = A.REFINE
    np.testing.assert_array_equal(marks, want)
    # |r| / |diag| above 1e-2 at the spike vetoes it
    r = np.zeros_like(u)
    r[4, 6] = 0.05
    r[3, 6] = 0.04
    marks, _ = A.mark_level(u, r, diag, cls, level, level_keep=2, level_max=3)
    want[4, 6] = 0
    np.testing.assert_array_equal(marks, want)
    # the finest level of the envelope refines nothing
    marks, _ = A.mark_level(u, None, diag, cls, level, level_keep=2, level_max=2)
    assert not marks.any()


def test_mark_level_on_a_constant_field_marks_nothing():
    cells = A.regular_cells(3, 1, 2, 3)
    cls = A.classify(cells, 3, 1, 2)
    marks, st = A.mark_level(np.full((10,) * 3, 2 - 1j), None, 1.0, cls, 2, 1, 3)
    assert st["k"] == 0 and st["e"] == 0 and not marks.any()


def _marks_at(dim, level, points, value):
    m = np.zeros((3 ** level + 1,) * dim, np.uint8)
    for p in points:
        m[p] = value
    return m


def test_refine_and_erase_by_hand_2d():
    dim, lmin, lkeep, lmax = 2, 1, 1, 3
    cells = A.regular_cells(dim, lmin, lkeep, lmax)
    assert not cells[1].any() and not cells[2].any()
    # refining level-1 vertex (1, 1) refines its four cells
    cells = A.adapt(cells, {1: _marks_at(dim, 1, [(1, 1)], A.REFINE)}, dim, lmin, lmax)
    want = np.zeros((3, 3), np.uint8)
    want[:2, :2] = 1
    np.testing.assert_array_equal(cells[1], want)
    # level 2: the 7 x 7 vertices over those cells; 13 on the domain boundary,
    # 25 inside the patch, 11 on its inner edges hanging, 51 absent
    cls = A.classify(cells, dim, lmin, 2)
    got = [int((cls == c).sum()) for c in (A.ABSENT, A.PERSISTENT, A.HANGING, A.BOUNDARY)]
    assert got == [51, 25, 11, 13]
    assert cls[6, 3] == A.HANGING and cls[3, 3] == A.PERSISTENT and cls[0, 3] == A.BOUNDARY
    assert cls[7, 3] == A.ABSENT
    # refine level-2 vertex (3, 3); an erase of (1, 1) in the next step is
    # vetoed on every cell: each has a refined child
    cells = A.adapt(cells, {2: _marks_at(dim, 2, [(3, 3)], A.REFINE)}, dim, lmin, lmax)
    assert cells[2].sum() == 4 and cells[2][2:4, 2:4].all()
    after = A.adapt(cells, {1: _marks_at(dim, 1, [(1, 1)], A.ERASE)}, dim, lmin, lmax)
    np.testing.assert_array_equal(after[1], want)
    np.testing.assert_array_equal(after[2], cells[2])
    # erasing both in one step returns to the regular grid (finer level first)
    back = A.adapt(cells, {1: _marks_at(dim, 1, [(1, 1)], A.ERASE),
                           2: _marks_at(dim, 2, [(3, 3)], A.ERASE)}, dim, lmin, lmax)
    assert not back[1].any() and not back[2].any()
    # a refine and an erase touching the same cell: the refine wins
    both = A.adapt(cells, {1: _marks_at(dim, 1, [(1, 1)], A.ERASE) + _marks_at(dim, 1, [(2, 2)], A.REFINE),
                           2: _marks_at(dim, 2, [(3, 3)], A.ERASE)}, dim, lmin, lmax)
    want2 = np.zeros((3, 3), np.uint8)
    want2[1:3, 1:3] = 1
    np.testing.assert_array_equal(both[1], want2)


@pytest.mark.parametrize("m", [1, 2])
def test_classes_of_a_refined_block_3d(m):
    # an m^3 block of refined level-1 cells away from the boundary (level 1 has
    # 3 cells per axis, so the block sits at cell 1 when m = 1; use level 2 for
    # m = 2): (3m + 1)^3 vertices on level l + 1, (3m - 1)^3 of them persistent
    dim, lmin, lmax = 3, 1, 3
    cells = A.regular_cells(dim, lmin, 2, lmax)          # level 1 fully refined
    cells[2][2:2 + m, 2:2 + m, 2:2 + m] = 1
    cls = A.classify(cells, dim, lmin, 3)
    assert int((cls == A.PERSISTENT).sum()) == (3 * m - 1) ** 3
    assert int((cls == A.HANGING).sum()) == (3 * m + 1) ** 3 - (3 * m - 1) ** 3
    assert int((cls == A.BOUNDARY).sum()) == 0
    # the regular levels: level 2 is whole, persistent inside, boundary outside
    cls2 = A.classify(cells, dim, lmin, 2)
    assert int((cls2 == A.PERSISTENT).sum()) == 8 ** 3 and int((cls2 == A.BOUNDARY).sum()) == 10 ** 3 - 8 ** 3


def test_interpolation_is_exact_on_linear_fields():
    # a linear coarse field: hanging and new vertices of the finer level take
    # its values at their own coordinates; old persistent vertices keep theirs
    dim, lmin, lmax = 2, 1, 2
    cells0 = A.regular_cells(dim, lmin, 1, lmax)
    cells1 = A.adapt(cells0, {1: _marks_at(dim, 1, [(1, 1)], A.REFINE)}, dim, lmin, lmax)
    cls_old, cls_new = A.classify(cells0, dim, lmin, 2), A.classify(cells1, dim, lmin, 2)
    Xc, Xf = _coords(1, dim), _coords(2, dim)
    f = lambda X: (0.2 - 0.7j) + (1.5 + 0.25j) * X[0] - 0.5j * X[1]
    u_fine = np.full((10, 10), 9.0 + 9.0j)
    out = A.interpolate(cls_old, cls_new, f(Xc), u_fine)
    take = (cls_new == A.HANGING) | (cls_new == A.PERSISTENT)
    np.testing.assert_allclose(out[take], f(Xf)[take], rtol=0, atol=1e-15)
    # level 2 was absent before: the new boundary vertices are set to zero,
    # the vertices that stay absent keep what they held
    became = (cls_new == A.BOUNDARY) & (cls_old == A.ABSENT)
    assert became.any() and np.all(out[became] == 0)
    stay = (cls_new == A.ABSENT) & (cls_old == A.ABSENT)
    assert np.all(out[stay] == 9.0 + 9.0j)
    # a second call with nothing new keeps the persistent values
    out2 = A.interpolate(cls_new, cls_new, 0 * f(Xc), out)
    np.testing.assert_array_equal(out2[cls_new == A.PERSISTENT], out[cls_new == A.PERSISTENT])
    assert np.all(out2[cls_new == A.HANGING] == 0)
