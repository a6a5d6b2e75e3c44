"""Parity of the adaptivity entry points (mg_amr_*) with the oracle: marks,
statistics, refined-cell flags and vertex classes bit for bit, hanging-vertex
values to 1e-14 (Section 5.3 criterion and bins, Section 4 hanging vertices)."""

import numpy as np
import pytest

from oracle import adapt as A
from paper_1508_03954_amd.inputs import gaussian, random_complex

pytestmark = pytest.mark.gpu


def _mg():
    from paper_1508_03954_amd import mg
    return mg


def feature_field(dim, level, seed, bumps=3):
    """Gaussian bumps of complex amplitude and small noise: s is large around
    the bumps and small elsewhere, as for a localised solution."""
    rng = np.random.default_rng(seed)
    u = 1e-3 * random_complex((3 ** level + 1,) * dim, seed)
    for _ in range(bumps):
        c = rng.uniform(0.2, 0.8, dim)
        amp = complex(rng.uniform(-1, 1), rng.uniform(-1, 1))
        u = u + amp * gaussian(level, dim, c, rng.uniform(0.03, 0.08))
    return u


def _check_mark(a, level, u, r, diag, cls, lkeep, lmax, **kw):
    mg = _mg()
    st = a.mark(level, u, r, diag, **kw)
    got = a.get(level, "marks").cpu().numpy()
    want, ost = A.mark_level(u, r, np.asarray(diag, dtype=np.complex128), cls, level, lkeep, lmax,
                             **{k: v for k, v in kw.items()})
    assert st["n"] == ost["n"]
    if ost["n"]:
        # s range: max/min are exact and the square root is correctly rounded
        assert st["s_min"] == ost["s_min"] and st["s_max"] == ost["s_max"]
    np.testing.assert_array_equal(st["counts"], ost["counts"])
    assert (st["k"], st["e"]) == (ost["k"], ost["e"])
    np.testing.assert_array_equal(got, want)
    assert st["refined"] == int((want == A.REFINE).sum()) and st["erased"] == int((want == A.ERASE).sum())
    assert mg.AMR_MARKS["refine"] == A.REFINE
    return want, st


@pytest.mark.parametrize("dim,level,seed", [(2, 5, 11), (2, 3, 12), (3, 4, 13), (3, 2, 14)])
def test_mark_of_a_regular_level_matches_oracle(dim, level, seed):
    mg = _mg()
    a = mg.Adapt(dim, 1, level, level + 1)
    cls = a.get(level, "classes").cpu().numpy()
    np.testing.assert_array_equal(cls, A.classify(A.regular_cells(dim, 1, level, level + 1), dim, 1, level))
    u = feature_field(dim, level, seed)
    r = 1e-4 * random_complex(u.shape, seed + 100)
    r[tuple(np.array(u.shape) // 2)] = 1.0      # one vetoed vertex in the middle
    diag = complex(4.0 * 3 ** (level * (dim - 2)), 0.3)
    marks, st = _check_mark(a, level, u, r, diag, cls, level, level + 1)
    assert st["refined"] > 0 and st["k"] > 0
    # without a residual: no veto; an erase percentage large enough to erase
    _check_mark(a, level, u, None, diag, cls, level, level + 1, erase_pct=30)
    # odd bin counts and percentages
    _check_mark(a, level, u, r, diag, cls, level, level + 1, nbins=7, refine_pct=33, erase_pct=5)
    _check_mark(a, level, u, r, diag, cls, level, level + 1, nbins=1, refine_pct=100, erase_pct=0)
    # a per-vertex diagonal (varying phi): the veto threshold moves with it
    dfield = diag * (1.0 + 0.5 * random_complex(u.shape, seed + 200))
    r2 = 1e-2 * abs(diag) * random_complex(u.shape, seed + 300)
    marks_f, _ = _check_mark(a, level, u, r2, dfield, cls, level, level + 1)
    marks_c, _ = _check_mark(a, level, u, r2, diag, cls, level, level + 1)
    assert not np.array_equal(marks_f, marks_c)
    a.close()


def test_mark_edge_cases():
    mg = _mg()
    dim = 2
    a = mg.Adapt(dim, 1, 2, 4)
    # a level with no persistent vertex (level 4 is absent): nothing marked
    u = feature_field(dim, 4, 3)
    st = a.mark(4, u)
    assert st["n"] == 0 and st["refined"] == 0 and st["erased"] == 0 and not st["counts"].any()
    assert not a.get(4, "marks").cpu().numpy().any()
    # a constant field: s = 0 everywhere, one bin holds every candidate, no marks
    st = a.mark(2, np.full((10, 10), 1 + 1j))
    assert st["n"] == 64 and st["counts"][0] == 64 and st["k"] == 0 and st["e"] == 0
    assert st["s_min"] == 0 and st["s_max"] == 0
    # the finest level refines nothing
    cells = A.regular_cells(dim, 1, 4, 4)
    a2 = mg.Adapt(dim, 1, 4, 4)
    u4 = feature_field(dim, 4, 5)
    _check_mark(a2, 4, u4, None, 1.0, A.classify(cells, dim, 1, 4), 4, 4)
    with pytest.raises(mg.MGError):
        a.mark(2, u[:10, :10].copy(), nbins=65)
    with pytest.raises(mg.MGError):
        mg.Adapt(3, 2, 1, 3)
    a.close()
    a2.close()


def _run_steps(dim, lmin, lkeep, lmax, plan, seed):
    """Marks and adapts on the GPU and in the oracle, step by step; checks the
    marks, cells and classes of every level after every step.  plan: a list of
    steps, each a list of (level, kwargs) marks."""
    mg = _mg()
    a = mg.Adapt(dim, lmin, lkeep, lmax)
    cells = A.regular_cells(dim, lmin, lkeep, lmax)
    cls = {l: A.classify(cells, dim, lmin, l) for l in range(lmin, lmax + 1)}
    for step, marks_plan in enumerate(plan):
        marks = {}
        for level, kw in marks_plan:
            u = feature_field(dim, level, seed + 7 * step + level)
            marks[level], _ = _check_mark(a, level, u, None, 1.0, cls[level], lkeep, lmax, **kw)
        counts = a.adapt()
        cells = A.adapt(cells, marks, dim, lmin, lmax)
        for l in range(lmin, lmax):
            np.testing.assert_array_equal(a.get(l, "cells").cpu().numpy(), cells[l], err_msg=f"step {step} level {l}")
        old = cls
        cls = {l: A.classify(cells, dim, lmin, l) for l in range(lmin, lmax + 1)}
        for l in range(lmin, lmax + 1):
            np.testing.assert_array_equal(a.get(l, "classes").cpu().numpy(), cls[l], err_msg=f"step {step} level {l}")
            np.testing.assert_array_equal(a.get(l, "classes_old").cpu().numpy(), old[l])
            assert counts[l] == tuple(int((cls[l] == c).sum()) for c in range(4))
    return a, cells, cls, old


@pytest.mark.parametrize("dim,lmin,lkeep,lmax", [(2, 1, 3, 6), (3, 1, 2, 4)])
def test_refine_erase_sequence_matches_oracle(dim, lmin, lkeep, lmax):
    plan = [
        [(lkeep, {})],                                               # refine around the bumps
        [(lkeep, {}), (lkeep + 1, {})],                              # refine again, one level deeper
        [(lkeep + 1, dict(erase_pct=40)), (lkeep + 2, {})],          # erase on a partial level
        [(lkeep, dict(refine_pct=0, erase_pct=60)), (lkeep + 1, dict(refine_pct=0, erase_pct=60))],
    ]
    a, cells, cls, _ = _run_steps(dim, lmin, lkeep, lmax, plan, seed=40 + dim)
    # the hierarchy got deeper than the base grid and some of it was erased again
    assert cells[lkeep].any()
    assert (cls[lkeep + 1] == A.HANGING).any()
    a.close()


@pytest.mark.parametrize("dim,lmin,lkeep,lmax", [(2, 1, 3, 5), (3, 1, 2, 4)])
def test_interpolation_matches_oracle(dim, lmin, lkeep, lmax):
    import torch
    plan = [[(lkeep, {})], [(lkeep, {}), (lkeep + 1, {})]]
    a, cells, cls, old = _run_steps(dim, lmin, lkeep, lmax, plan, seed=70 + dim)
    for level in range(lkeep + 1, lmax + 1):
        uc = random_complex((3 ** (level - 1) + 1,) * dim, 900 + level)
        uf = random_complex((3 ** level + 1,) * dim, 950 + level)
        dev = torch.from_numpy(uf).cuda()
        a.interpolate(level, uc, dev)
        got = dev.cpu().numpy()
        want = A.interpolate(old[level], cls[level], uc, uf)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14 * np.abs(uc).max())
        # vertices that keep their values keep them bit for bit
        keep = (cls[level] == A.PERSISTENT) & (old[level] == A.PERSISTENT)
        np.testing.assert_array_equal(got[keep], uf[keep])
    a.close()


def device_feature_field(level, seed, bumps=4):
    """3D feature field built on the device (the 730^3 level is too large to
    generate on the host in a test): uniform noise of size 1e-3 and separable
    Gaussian bumps of complex amplitude."""
    import torch
    n = 3 ** level + 1
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    re = torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64)
    im = torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64)
    u = torch.complex(2e-3 * re - 1e-3, 2e-3 * im - 1e-3)
    del re, im
    rng = np.random.default_rng(seed)
    x = torch.arange(n, device="cuda", dtype=torch.float64) / 3 ** level
    for _ in range(bumps):
        c = rng.uniform(0.2, 0.8, 3)
        sig = rng.uniform(0.03, 0.08)
        amp = complex(rng.uniform(-1, 1), rng.uniform(-1, 1))
        gz, gy, gx = (torch.exp(-(x - c[a]) ** 2 / (2 * sig * sig)) for a in range(3))
        u += amp * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return u


def test_full_size_mark_and_adapt_level6():
    """730^3 envelope (levels 1..6, base 244^3): marks of level 5 bit for bit
    with the oracle, one step (cells of level 5 and the classes of level 6 bit
    for bit), then the marks of the partial level 6 checked by counts and on
    sampled vertices, and the hanging values on sampled vertices."""
    import torch
    mg = _mg()
    dim, lmin, lkeep, lmax = 3, 1, 5, 6
    a = mg.Adapt(dim, lmin, lkeep, lmax)
    u5 = feature_field(dim, 5, 61, bumps=4)
    cells = A.regular_cells(dim, lmin, lkeep, lmax)
    cls5 = A.classify(cells, dim, lmin, 5)
    marks5, st5 = _check_mark(a, 5, u5, None, 1.0, cls5, lkeep, lmax)
    assert st5["refined"] > 0
    counts = a.adapt()
    cells = A.adapt(cells, {5: marks5}, dim, lmin, lmax)
    np.testing.assert_array_equal(a.get(5, "cells").cpu().numpy(), cells[5])
    cls6 = A.classify(cells, dim, lmin, 6)
    assert counts[6] == tuple(int((cls6 == c).sum()) for c in range(4))
    cls6_dev = a.get(6, "classes")
    assert np.array_equal(cls6_dev.cpu().numpy(), cls6)
    # marks of level 6 (its persistent vertices only)
    rng = np.random.default_rng(62)
    u6 = device_feature_field(6, 63)
    st6 = a.mark(6, u6)
    assert st6["n"] == int((cls6 == A.PERSISTENT).sum()) == int(st6["counts"].sum())
    assert (st6["k"], st6["e"]) == A.choose_bins(st6["counts"], st6["n"], 10, 2)
    assert st6["refined"] == 0                       # the finest level refines nothing
    marks6 = a.get(6, "marks")
    assert st6["erased"] == int((marks6 == A.ERASE).sum().item())
    assert int((marks6[cls6_dev != A.PERSISTENT] != 0).sum().item()) == 0
    # sampled persistent vertices: s from their 3^3 window, the bin against
    # the GPU's range, and the erase decision
    pts = np.argwhere(cls6 == A.PERSISTENT)
    pts = pts[rng.choice(len(pts), 2000, replace=False)]
    off = np.array(np.meshgrid(*([np.arange(-1, 2)] * 3), indexing="ij")).reshape(3, -1).T
    idx = torch.from_numpy((pts[:, None, :] + off[None]).reshape(-1, 3)).cuda()
    wins = u6[idx[:, 0], idx[:, 1], idx[:, 2]].reshape(-1, 3, 3, 3).cpu().numpy()
    mk = marks6[tuple(torch.from_numpy(pts).cuda().T)].cpu().numpy()
    for w, m in zip(wins, mk):
        s = A.criterion(w)[1, 1, 1]
        assert st6["s_min"] <= s <= st6["s_max"]
        b = int(A.bin_index(np.array([s]), st6["s_min"], st6["s_max"], 20)[0])
        assert m == (A.ERASE if b < st6["e"] else A.KEEP)
    del u6, marks6
    # hanging vertices of level 6 take P u_5 (checked on sampled vertices
    # against the oracle's P on the coarse cell around them); absent ones 0
    uc = random_complex((244,) * 3, 64)
    uf = torch.full((3 ** 6 + 1,) * 3, 7.0 + 7.0j, dtype=torch.complex128, device="cuda")
    a.interpolate(6, uc, uf)
    hang = np.argwhere(cls6 == A.HANGING)
    hang = hang[rng.choice(len(hang), 500, replace=False)]
    vals = uf[tuple(torch.from_numpy(hang).cuda().T)].cpu().numpy()
    for p, v in zip(hang, vals):
        m = np.minimum(p // 3, 242)
        fine = A.prolong(uc[m[0]:m[0] + 2, m[1]:m[1] + 2, m[2]:m[2] + 2])
        q = p - 3 * m
        np.testing.assert_allclose(v, fine[tuple(q)], rtol=0, atol=1e-14)
    # level 6 was absent before the step: vertices that stay absent keep their
    # values; none became absent or boundary (the step only refined)
    assert bool((uf[cls6_dev == A.ABSENT] == 7.0 + 7.0j).all().item())
    assert bool((uf[cls6_dev == A.PERSISTENT] != 7.0 + 7.0j).all().item())
    a.close()


@pytest.mark.parametrize("dim,lmin,lmax", [(2, 1, 5), (3, 1, 4)])
def test_set_cells_matches_oracle(dim, lmin, lmax):
    """Refined-cell flags set directly (random, each refined cell under a
    refined parent): every level's classes bit for bit, then one marked step
    from that state."""
    mg = _mg()
    rng = np.random.default_rng(90 + dim)
    a = mg.Adapt(dim, lmin, lmin, lmax)
    cells = A.regular_cells(dim, lmin, lmin, lmax)
    for l in range(lmin, lmax):
        flags = (rng.random((3 ** l,) * dim) < 0.35).astype(np.uint8)
        if l > lmin:
            flags &= A.cell_exists(cells, l, lmin, dim).astype(np.uint8)
        cells[l] = flags
        a.set_cells(l, flags)
    for l in range(lmin, lmax):
        np.testing.assert_array_equal(a.get(l, "cells").cpu().numpy(), cells[l])
    cls = {}
    for l in range(lmin, lmax + 1):
        cls[l] = A.classify(cells, dim, lmin, l)
        np.testing.assert_array_equal(a.get(l, "classes").cpu().numpy(), cls[l], err_msg=f"level {l}")
        np.testing.assert_array_equal(a.get(l, "classes_old").cpu().numpy(), cls[l])
    # one step from the set state: marks on two levels, cells and classes
    marks = {}
    for level in (lmin + 1, lmin + 2):
        u = feature_field(dim, level, 95 + level)
        marks[level], _ = _check_mark(a, level, u, None, 1.0, cls[level], lmin, lmax, erase_pct=20)
    a.adapt()
    cells = A.adapt(cells, marks, dim, lmin, lmax)
    for l in range(lmin, lmax):
        np.testing.assert_array_equal(a.get(l, "cells").cpu().numpy(), cells[l], err_msg=f"level {l}")
    for l in range(lmin, lmax + 1):
        np.testing.assert_array_equal(a.get(l, "classes").cpu().numpy(), A.classify(cells, dim, lmin, l))
    a.close()
