"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Every comparison is element by element on seeded inputs; the FP64 bar is
relative 2-norm error <= 1e-12 (the summation order differs between the two
sides, nothing else).  Sizes span several thread blocks and the fused sweep's
tiles with ragged tails.
"""

import math
import time

import numpy as np
import pytest

import oracle as O
from coarse_bound import chain_factors
from oracle.cycle import Params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_03954_amd import mg
    mg.load_library()


def mgmod():
    from paper_1508_03954_amd import mg
    return mg


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(got, ref):
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def rand_c(shape, seed, zero_bnd=True):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return O.zero_boundary(v) if zero_bnd else v


def nodal_phi(dim, L, seed):
    rng = np.random.default_rng(seed)
    n = 3 ** L + 1
    return (120 + 80 * rng.standard_normal((n,) * dim)) * (1 + 0.3j)


APPLY_CASES = [(2, 3), (2, 5), (3, 2), (3, 3), (3, 4)]


@pytest.mark.parametrize("dim,L", APPLY_CASES)
@pytest.mark.parametrize("phi_case", ["const", "varying"])
@pytest.mark.parametrize("conj", [False, True])
def test_apply_matches_oracle(dim, L, phi_case, conj):
    print(f"\n[case] apply dim={dim} L={L} phi={phi_case} conj={conj}", flush=True)
    mg = mgmod()
    theta, phi = 0.37, 150 * (1 + 0.4j)
    pn = nodal_phi(dim, L, 11) if phi_case == "varying" else None
    s = mg.Solver(dim, L, theta=theta, phi=phi, conjugate=conj,
                  phi_field=None if pn is None else torch.from_numpy(pn))
    x = rand_c((3 ** L + 1,) * dim, 5, zero_bnd=False)       # boundary entries must be ignored
    y = to_np(s.apply(x))
    ref = O.apply_H(x, L, theta, phi if pn is None else pn, conjugate=conj)
    assert relerr(y, ref) <= TOL


def test_rhs_from_nodal():
    mg = mgmod()
    dim, L, theta = 3, 3, math.pi / 6
    s = mg.Solver(dim, L, theta=theta, phi=400.0)
    chi = rand_c((3 ** L + 1,) * dim, 3, zero_bnd=False)
    b = to_np(s.rhs_from_nodal(chi))
    assert relerr(b, O.lumped_rhs(chi, L, theta)) <= 1e-15


def level_ref(pipe, p, lev, field, galerkin, chain=None):
    """Oracle counterpart of a GPU level field.  The finest level stores the
    folded iterate u + sc.  With the Galerkin form a coarse b slot holds the
    restricted residual b_l - H_l u_l, and the coarse smoothing fields derive
    from it: their reference is the oracle's restricted-residual form
    (R^(L-l) r_L, Lemmas 1 and 2), which has no cancellation, rather than the
    FAS form b_l - H_l u_l, whose rounding grows with the iterate while the
    residual shrinks."""
    L = p.level_max
    if lev == L:
        if field == "u":
            return pipe.u[L] + pipe.sc[L]
        if field == "b":
            return pipe.b[L]
        return np.zeros_like(pipe.u[L])
    if galerkin and field in ("b", "sc", "sf", "si"):
        return chain[lev][field]
    return getattr(pipe, field)[lev]


CYCLE_CASES = [
    # dim, L, lmin, variant, restrict, sweep, phi_case, scheme
    (2, 4, 1, "add", "galerkin", "generic", "const", "const"),
    (2, 4, 1, "hb", "galerkin", "generic", "const", "exp"),
    (2, 4, 1, "bpx", "galerkin", "generic", "const", "const"),
    (2, 4, 2, "bpx", "fas", "generic", "const", "transition"),
    (2, 4, 1, "add", "fas", "generic", "varying", "const"),
    (2, 4, 1, "bpx", "fas", "generic", "varying", "exp"),
    (3, 3, 1, "add", "galerkin", "generic", "const", "const"),
    (3, 3, 1, "hb", "fas", "generic", "const", "const"),
    (3, 3, 1, "bpx", "galerkin", "generic", "const", "const"),
    (3, 3, 1, "bpx", "fas", "generic", "varying", "const"),
    (3, 3, 3, "bpx", "galerkin", "generic", "const", "const"),
    # 82^3: the finest descent and the surplus as z marches
    (3, 4, 1, "bpx", "fas", "generic", "varying", "const"),
    (3, 4, 2, "hb", "galerkin", "generic", "const", "exp"),
    # fused finest sweep: grids of several tiles with ragged tails in every axis
    (2, 4, 1, "add", "galerkin", "fused", "const", "const"),
    (2, 5, 1, "hb", "galerkin", "fused", "const", "exp"),
    (2, 5, 2, "bpx", "galerkin", "fused", "const", "const"),
    (3, 3, 1, "add", "galerkin", "fused", "const", "const"),
    (3, 3, 1, "hb", "galerkin", "fused", "const", "transition"),
    (3, 3, 2, "bpx", "galerkin", "fused", "const", "const"),
    (3, 4, 1, "bpx", "galerkin", "fused", "const", "const"),
    (3, 4, 1, "add", "galerkin", "fused", "const", "exp"),
    (3, 2, 1, "bpx", "galerkin", "fused", "const", "const"),
    # two-phase relaxation: plain Jacobi (one level) and multilevel, fused and not
    (2, 3, 3, "add", "galerkin", "generic", "const", "two_phase"),
    (2, 4, 1, "hb", "galerkin", "generic", "const", "two_phase"),
    (3, 3, 1, "bpx", "galerkin", "fused", "const", "two_phase"),
]


def run_cycle_parity(dim, L, lmin, variant, restrict, sweep, phi_case, scheme, ncycles=3, tol=TOL, tile=None,
                     layer=None, conj=False):
    mg = mgmod()
    theta, phi = 0.4, 90 * (1 + 0.5j)
    n = 3 ** L + 1
    pn = nodal_phi(dim, L, 7) if phi_case == "varying" else None
    p = Params(dim=dim, level_max=L, level_min=lmin, theta=theta, phi=phi, phi_nodal=pn,
               variant=variant, omega_scheme=scheme, omega=0.6, layer=layer, conjugate=conj)
    b = rand_c((n,) * dim, 1)
    u0 = rand_c((n,) * dim, 2)
    s = mg.Solver(dim, L, level_min=lmin, theta=theta, phi=phi, variant=variant, omega_scheme=scheme,
                  omega=0.6, restrict_form=restrict, sweep=sweep, layer=layer, conjugate=conj,
                  phi_field=None if pn is None else torch.from_numpy(pn))
    if tile is not None:
        s.set_tile(tile)
    s.set_rhs(b)
    s.set_solution(u0)
    pipe = O.Pipelined(p, b, u0)
    galerkin = restrict == "galerkin"
    for k in range(ncycles):
        rh_ref, rm_ref = pipe.cycle()
        rh, rm = s.cycle(1)
        assert abs(rh[0] - rh_ref) <= tol * rh_ref, (k, rh[0], rh_ref)
        assert abs(rm[0] - rm_ref) <= tol * rm_ref
        chain = pipe.restricted_residual_state() if galerkin and lmin < L else None
        cf = chain_factors(pipe) if chain is not None else None
        for lev in range(lmin, L + 1):
            for field in ("u", "b", "sc", "sf", "si"):
                got = to_np(s.get_level(lev, field))
                if galerkin and lev < L and field == "u":
                    # the Galerkin form does not form coarse iterates (zeros)
                    assert not np.any(got), (k, lev)
                    continue
                ref = level_ref(pipe, p, lev, field, galerkin, chain)
                if not np.any(ref):
                    assert not np.any(got), (k, lev, field)
                    continue
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                bound = tol * (cf[lev] if cf is not None and field != "u" else 1.0)
                assert err <= bound, (k, lev, field, err, bound)
    u_ref = pipe.flush()
    u = to_np(s.flush())
    assert relerr(u, u_ref) <= tol


@pytest.mark.parametrize("case", CYCLE_CASES, ids=lambda c: "-".join(map(str, c)))
def test_cycle_state_matches_pipelined_oracle(case):
    print(f"\n[case] cycle {case}", flush=True)
    run_cycle_parity(*case)


# absorbing layer (Section 7.4): per-cell rotation on every level; faces are
# asymmetric (bit 2a: x_a = 0, bit 2a + 1: x_a = 1, x_0 fastest) so that a
# swapped axis or face would show
LAYER_CASES = [
    # dim, L, lmin, variant, phi_case, scheme, faces, conj
    (2, 4, 1, "bpx", "const", "const", 0b1010, False),
    (2, 4, 1, "add", "varying", "transition", 0b0110, False),
    (2, 4, 4, "add", "varying", "two_phase", 0b1010, False),
    (3, 3, 1, "bpx", "const", "const", 0b100010, False),
    (3, 3, 1, "hb", "varying", "exp", 0b010001, False),
    (3, 3, 1, "bpx", "varying", "const", 0b001010, True),
]


@pytest.mark.parametrize("case", LAYER_CASES, ids=lambda c: "-".join(map(str, c)))
def test_layer_cycle_matches_pipelined_oracle(case):
    dim, L, lmin, variant, phi_case, scheme, faces, conj = case
    print(f"\n[case] layer cycle {case}", flush=True)
    run_cycle_parity(dim, L, lmin, variant, "fas", "generic", phi_case, scheme, ncycles=3,
                     layer=(math.radians(30), 1.0 / 3.0, faces), conj=conj)


@pytest.mark.parametrize("dim,L,faces", [(2, 4, 0b0110), (3, 3, 0b100010)])
def test_layer_apply_and_rhs_match_oracle(dim, L, faces):
    mg = mgmod()
    theta, phi, lt = 0.25, 70 * (1 + 0.3j), math.radians(30)
    layer = (lt, 1.0 / 3.0, faces)
    pn = nodal_phi(dim, L, 13)
    tc = O.cell_theta(L, dim, theta, layer)
    for conj in (False, True):
        print(f"\n[case] layer apply dim={dim} L={L} faces={faces:b} conj={conj}", flush=True)
        s = mg.Solver(dim, L, theta=theta, phi=phi, layer=layer, conjugate=conj, phi_field=torch.from_numpy(pn))
        x = rand_c((3 ** L + 1,) * dim, 5, zero_bnd=False)
        assert relerr(to_np(s.apply(x)), O.apply_H(x, L, tc, pn, conjugate=conj)) <= TOL
        chi = rand_c((3 ** L + 1,) * dim, 6, zero_bnd=False)
        assert relerr(to_np(s.rhs_from_nodal(chi)), O.lumped_rhs(chi, L, tc)) <= 1e-15
    # a constant phi with a layer takes the per-cell path too
    s = mg.Solver(dim, L, theta=theta, phi=phi, layer=layer)
    x = rand_c((3 ** L + 1,) * dim, 7, zero_bnd=False)
    assert relerr(to_np(s.apply(x)), O.apply_H(x, L, tc, phi)) <= TOL
    with pytest.raises(mg.MGError):
        mg.Solver(dim, L, theta=theta, phi=phi, layer=(lt, 1.0 / 3.0, 1 << (2 * dim)))
    with pytest.raises(mg.MGError):
        mg.Solver(dim, L, theta=theta, phi=phi, layer=layer, restrict_form="galerkin")


@pytest.mark.parametrize("dim,L", [(3, 4), (3, 3), (2, 5)])
@pytest.mark.parametrize("variant", ["add", "bpx"])
def test_every_fused_tile_matches_oracle(dim, L, variant):
    """Each tile variant of the fused sweep (the autotuner may choose any).  3D
    L = 4 has 28 coarse rows (ragged z tails for z extents 9 and 21), L = 3 has
    10 (ragged y tails for 4 coarse rows a tile, one z tile)."""
    mg = mgmod()
    ntiles = mg.Solver(dim, L, level_min=1, theta=0.4, phi=90 * (1 + 0.5j), variant=variant,
                       sweep="fused").tiles()[1]
    for tile in range(ntiles):
        print(f"\n[case] fused tile {tile} dim={dim} L={L} {variant}", flush=True)
        run_cycle_parity(dim, L, 1, variant, "galerkin", "fused", "const", "const", ncycles=2, tile=tile)


def test_autotune_keeps_state():
    mg = mgmod()
    dim, L = 3, 4
    s = mg.Solver(dim, L, theta=0.3, phi=200.0, variant="bpx", sweep="fused")
    b = rand_c((3 ** L + 1,) * dim, 1)
    s.set_rhs(b)
    s.set_solution(rand_c((3 ** L + 1,) * dim, 2))
    s.cycle(2)
    before = {f: to_np(s.get_level(L - 1, f)) for f in ("u", "b", "sc", "si")}
    before["w"] = to_np(s.get_level(L, "u"))
    best, us, times = s.autotune(reps=2)
    assert s.tiles()[0] == best and len(times) == s.tiles()[1] and min(times) == us
    after = {f: to_np(s.get_level(L - 1, f)) for f in ("u", "b", "sc", "si")}
    after["w"] = to_np(s.get_level(L, "u"))
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])


@pytest.mark.parametrize("dim,L,variant,sweep", [(3, 4, "bpx", "fused"), (3, 3, "bpx", "fused"),
                                                  (2, 5, "hb", "fused"), (3, 3, "add", "generic")])
def test_cycles_in_one_call_match_single_calls(dim, L, variant, sweep):
    """mg_cycle(ctx, 4) runs the next cycle's small-level pre-phase inside the
    previous cycle's last launch; the state and the residual history equal
    those of four mg_cycle(ctx, 1) calls bit for bit."""
    print(f"\n[case] cycles in one call dim={dim} L={L} {variant} {sweep}", flush=True)
    mg = mgmod()
    n = 3 ** L + 1
    b, u0 = rand_c((n,) * dim, 1), rand_c((n,) * dim, 2)
    solvers, hist = [], []
    for one_call in (True, False):
        s = mg.Solver(dim, L, theta=0.4, phi=90 * (1 + 0.5j), variant=variant, sweep=sweep, omega=0.6)
        s.set_rhs(b)
        s.set_solution(u0)
        if one_call:
            rh, rm = s.cycle(4)
        else:
            rh, rm = [], []
            for _ in range(4):
                a, m = s.cycle(1)
                rh += list(a)
                rm += list(m)
        solvers.append(s)
        hist.append((list(rh), list(rm)))
    assert hist[0] == hist[1]
    for lev in range(1, L + 1):
        for field in ("u", "b", "sc", "sf", "si"):
            np.testing.assert_array_equal(to_np(solvers[0].get_level(lev, field)),
                                          to_np(solvers[1].get_level(lev, field)), err_msg=f"{lev} {field}")
    np.testing.assert_array_equal(to_np(solvers[0].flush()), to_np(solvers[1].flush()))


@pytest.mark.parametrize("dim,L,sweep", [(3, 4, "fused"), (2, 4, "fused"), (3, 3, "generic")])
def test_sweep_timing_hook(dim, L, sweep):
    """mg_time_sweeps records one event pair per finest sweep (the fused
    sweep's pair takes the kernel's own start and end); the recorded time is
    positive and below the cycles' wall time, recording stops when disabled,
    and the cycles' results do not depend on whether timing is on."""
    mg = mgmod()
    n = 3 ** L + 1
    b, u0 = rand_c((n,) * dim, 1), rand_c((n,) * dim, 2)
    finals = []
    for timed in (False, True):
        print(f"\n[case] sweep timing dim={dim} L={L} {sweep} timed={timed}", flush=True)
        s = mg.Solver(dim, L, theta=0.3, phi=200.0, variant="bpx", sweep=sweep)
        s.set_rhs(b)
        s.set_solution(u0)
        if timed:
            s.time_sweeps(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.cycle(5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        finals.append(to_np(s.get_level(L, "u")))
        if timed:
            ms, cnt = s.sweep_time()
            assert cnt == 5
            assert 0 < ms < 1e3 * wall, (ms, wall)
            s.time_sweeps(False)
            s.cycle(1)
            assert s.sweep_time()[1] == 5
    np.testing.assert_array_equal(finals[0], finals[1])


@pytest.mark.parametrize("dim,L,variant", [(2, 4, "bpx"), (3, 3, "hb"), (3, 3, "add")])
@pytest.mark.parametrize("phi_case", ["const", "varying"])
def test_precondition_matches_zero_start_cycle(dim, L, variant, phi_case):
    print(f"\n[case] precondition dim={dim} L={L} {variant} {phi_case}", flush=True)
    mg = mgmod()
    theta, phi = 0.3, 200.0
    pn = nodal_phi(dim, L, 3) if phi_case == "varying" else None
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi, phi_nodal=pn, variant=variant,
               omega_scheme="exp", omega=0.7)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant=variant, omega_scheme="exp", omega=0.7,
                  phi_field=None if pn is None else torch.from_numpy(pn))
    v = rand_c((3 ** L + 1,) * dim, 9, zero_bnd=False)
    z = to_np(s.precondition(v))
    ref = O.zero_start_cycle(p, O.zero_boundary(v))
    assert relerr(z, ref) <= TOL


@pytest.mark.parametrize("dim,L,variant", [(3, 3, "bpx"), (3, 3, "hb"), (3, 4, "add"), (3, 4, "bpx"), (2, 4, "hb")])
def test_precondition_apply_matches_oracle(dim, L, variant):
    """The Krylov step z = B v, y = H z: in 3D one pass over the finest grid
    (L = 4 spans several x, y and z tiles of the march; L = 3 a single one)."""
    print(f"\n[case] precondition_apply dim={dim} L={L} {variant}", flush=True)
    mg = mgmod()
    theta, phi = 0.3, 200.0 * (1 + 0.5j)
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi, variant=variant, omega_scheme="exp", omega=0.7)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant=variant, omega_scheme="exp", omega=0.7)
    v = rand_c((3 ** L + 1,) * dim, 19, zero_bnd=False)
    z, y = s.precondition_apply(v)
    zref = O.zero_start_cycle(p, O.zero_boundary(v))
    assert relerr(to_np(z), zref) <= TOL
    assert relerr(to_np(y), O.apply_H(zref, L, theta, phi)) <= TOL


@pytest.mark.parametrize("dim,L", [(2, 3), (3, 2)])
def test_bicgstab_reaches_dense_solution(dim, L):
    mg = mgmod()
    theta, phi = math.pi / 6, 400.0
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi, variant="bpx")
    b = rand_c((3 ** L + 1,) * dim, 4)
    ref = O.dense_solve(p, b)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant="bpx")
    u, its, rel, rc = s.solve(b, rtol=1e-12, maxit=300, driver="bicgstab")
    assert rc == 0 and rel <= 1e-12
    assert relerr(to_np(u), ref) <= 1e-9


@pytest.mark.parametrize("dim,level", [(2, 2), (2, 4), (3, 3), (3, 4)])
def test_prolong_matches_oracle(dim, level):
    """mg_prolong against the oracle's tensor-product P (interior; zero boundary)."""
    print(f"\n[case] prolong dim={dim} level={level}", flush=True)
    mg = mgmod()
    s = mg.Solver(dim, level, theta=0.3, phi=100.0)
    uc = rand_c((3 ** (level - 1) + 1,) * dim, 21, zero_bnd=False)
    got = to_np(s.prolong(torch.from_numpy(uc), level))
    ref = O.zero_boundary(O.prolong(uc))
    assert relerr(got, ref) <= 1e-14


NESTED_CASES = [(2, 4, 90 * (1 + 0.5j), 0.3), (3, 3, 400.0, math.pi / 6)]


@pytest.mark.parametrize("dim,L,phi,theta", NESTED_CASES)
def test_nested_initial_guess_matches_oracle(dim, L, phi, theta):
    """With a finest-level target the start already meets (rtol 10), the
    nested solve returns its initial guess: level L - 1 solved (to 1e-13 here)
    with the sampled load and prolonged.  Oracle: the dense solution of level
    L - 1, prolonged."""
    print(f"\n[case] nested guess dim={dim} L={L}", flush=True)
    mg = mgmod()
    n = 3 ** L + 1
    chi = rand_c((n,) * dim, 31, zero_bnd=False)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant="bpx")
    u, its, rel, rc = s.solve_nested(torch.from_numpy(chi), level_start=1, coarse_rtol=1e-13, rtol=10.0,
                                     maxit=500, driver="bicgstab")
    assert rc == 0 and its == 0
    ref = O.nested_initial_guess(Params(dim=dim, level_max=L, theta=theta, phi=phi), chi)
    assert relerr(to_np(u), ref) <= 1e-9


@pytest.mark.parametrize("dim,L,phi,driver,precision", [(2, 3, 400.0, "bicgstab", "fp64"),
                                                        (3, 2, 400.0, "bicgstab", "fp64"),
                                                        (2, 3, -100.0, "stationary", "fp64"),
                                                        (2, 3, 400.0, "bicgstab", "fp32_refine")])
def test_nested_solve_reaches_dense_solution(dim, L, phi, driver, precision):
    print(f"\n[case] nested solve dim={dim} L={L} {driver} {precision}", flush=True)
    mg = mgmod()
    theta = math.pi / 6 if phi > 0 else 0.0
    n = 3 ** L + 1
    chi = rand_c((n,) * dim, 41, zero_bnd=False)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant="bpx", omega=0.6, precision=precision)
    u, its, rel, rc = s.solve_nested(torch.from_numpy(chi), level_start=1, coarse_rtol=1e-6, rtol=1e-12,
                                     maxit=500, driver=driver)
    assert rc == 0 and rel <= 1e-12
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi)
    ref = O.dense_solve(p, O.lumped_rhs(chi, L, theta))
    assert relerr(to_np(u), ref) <= 1e-9


def test_stationary_solve_poisson():
    mg = mgmod()
    from paper_1508_03954_amd.inputs import sine_load
    dim, L = 2, 4
    p = Params(dim=dim, level_max=L, theta=0.0, phi=0.0, variant="add", omega_scheme="exp", omega=0.6)
    b = O.lumped_rhs(sine_load(L, dim), L, 0.0)
    s = mg.Solver(dim, L, theta=0.0, phi=0.0, variant="add", omega_scheme="exp", omega=0.6)
    u, its, rel, rc = s.solve(b, rtol=1e-8, maxit=400, driver="stationary")
    assert rc == 0 and rel <= 1e-8
    ref, its_ref, _, ok = O.stationary_solve(p, b, 1e-8, 400)
    assert ok and abs(its - its_ref) <= 4
    assert relerr(to_np(u), O.dense_solve(p, b)) <= 1e-6


@pytest.mark.parametrize("dim,L", [(2, 4), (3, 3)])
def test_fp32_refinement_reaches_fp64_accuracy(dim, L):
    mg = mgmod()
    theta, phi = 0.0, 100 * (1 + 0.5j)
    p = Params(dim=dim, level_max=L, theta=theta, phi=phi, variant="bpx")
    b = rand_c((3 ** L + 1,) * dim, 6)
    s = mg.Solver(dim, L, theta=theta, phi=phi, variant="bpx", precision="fp32_refine")
    u, its, rel, rc = s.solve(b, rtol=1e-10, maxit=2000, driver="bicgstab")
    assert rc == 0 and rel <= 1e-10
    ref, _, _, ok = O.bicgstab(p, b, 1e-13, 400)
    assert ok
    err = relerr(to_np(u), ref)
    print(f"\n[fp32-refine] dim={dim} L={L} inner iterations={its} relres={rel:.2e} error vs FP64={err:.2e}")
    assert err <= 1e-8


@pytest.mark.parametrize("dim,L", [(2, 4), (3, 3)])
def test_fp32_refinement_with_stationary_cycles(dim, L):
    """Inner complex64 solves by pipelined cycles (fused sweep in FP32)."""
    mg = mgmod()
    p = Params(dim=dim, level_max=L, theta=0.0, phi=-30.0, variant="bpx", omega_scheme="const", omega=0.6)
    b = rand_c((3 ** L + 1,) * dim, 8)
    s = mg.Solver(dim, L, theta=0.0, phi=-30.0, variant="bpx", omega=0.6, precision="fp32_refine")
    u, its, rel, rc = s.solve(b, rtol=1e-10, maxit=3000, driver="stationary")
    assert rc == 0 and rel <= 1e-10, (rc, rel, its)
    ref, _, _, ok = O.bicgstab(p, b, 1e-13, 400)
    err = relerr(to_np(u), ref)
    print(f"\n[fp32-refine stationary] dim={dim} L={L} cycles={its} relres={rel:.2e} error vs FP64={err:.2e}")
    assert err <= 1e-8


@pytest.mark.parametrize("dim,L", [(2, 4), (3, 3)])
def test_grad_potential_matches_oracle(dim, L):
    mg = mgmod()
    theta = 0.2
    s = mg.Solver(dim, L, theta=theta, phi=50.0)
    u = rand_c((3 ** L + 1,) * dim, 21)
    lam = rand_c((3 ** L + 1,) * dim, 22)
    g = to_np(s.grad_potential(u, lam))
    ref = O.potential_gradient(u, lam, L, theta)
    assert relerr(g, ref) <= TOL


def test_invalid_arguments_raise():
    mg = mgmod()
    with pytest.raises(mg.MGError):
        mg.Solver(3, 2, sweep="fused", phi_field=torch.zeros((10, 10, 10), dtype=torch.complex128))
    s = mg.Solver(2, 2)
    with pytest.raises(ValueError):
        s.apply(np.zeros((5, 5), dtype=np.complex128))


@pytest.mark.parametrize("dim,L,lmin,variant,sweep,scheme", [(2, 4, 1, "add", "generic", "transition"),
                                                             (2, 3, 3, "add", "generic", "two_phase"),
                                                             (3, 3, 1, "bpx", "fused", "two_phase")])
def test_cycle_flush_cycle_keeps_the_cycle_counter(dim, L, lmin, variant, sweep, scheme):
    """A flush applies the pending update without restarting the cycle count:
    the transition scheme (Section 5.1) and the two-phase relaxation (Section
    7.4) continue with the next cycle number, as the oracle's pipeline does."""
    print(f"\n[case] cycle-flush-cycle dim={dim} L={L} {variant} {scheme}", flush=True)
    mg = mgmod()
    theta, phi = 0.4, 90 * (1 + 0.5j)
    n = 3 ** L + 1
    w = 0.6 if scheme == "transition" else 0.3 * (math.sqrt(3) - 1j)
    p = Params(dim=dim, level_max=L, level_min=lmin, theta=theta, phi=phi, variant=variant, omega_scheme=scheme,
               omega=w)
    b, u0 = rand_c((n,) * dim, 1), rand_c((n,) * dim, 2)
    s = mg.Solver(dim, L, level_min=lmin, theta=theta, phi=phi, variant=variant, omega_scheme=scheme, omega=w,
                  sweep=sweep)
    s.set_rhs(b)
    s.set_solution(u0)
    pipe = O.Pipelined(p, b, u0)
    for ncyc in (3, 2):
        rh, _ = s.cycle(ncyc)
        ref = [pipe.cycle()[0] for _ in range(ncyc)]
        for a, c in zip(rh, ref):
            assert abs(a - c) <= TOL * c, (a, c)
        u = to_np(s.flush())
        assert relerr(u, pipe.flush()) <= TOL


def test_stationary_driver_status_and_count():
    """The stationary driver against the oracle's: the cycle count at which it
    stops, MG_EDIVERGED for the indefinite 3D cycle with omega 0.6 on every
    level (it grows by 1e8 within 14 cycles), MG_ENOTCONV at maxit with the
    iterate of that many cycles, MG_OK and the returned iterate's residual
    when it converges."""
    mg = mgmod()
    rng = np.random.default_rng(3)
    # diverging: k = 30 without shift or rotation
    p = Params(dim=3, level_max=3, theta=0.0, phi=900.0, variant="bpx", omega=0.6)
    b = O.zero_boundary(rng.standard_normal((28,) * 3) + 0j)
    _, its_ref, hist, ok = O.stationary_solve(p, b, 1e-10, 300)
    assert not ok and hist[-1] > 1e8 * hist[0]
    s = mg.Solver(3, 3, theta=0.0, phi=900.0, variant="bpx", omega=0.6)
    u, its, rel, rc = s.solve(b, rtol=1e-10, maxit=300, driver="stationary")
    print(f"\n[stationary] diverging: rc={rc}, cycles {its} (oracle {its_ref})", flush=True)
    assert rc == mg.MG_EDIVERGED and its == its_ref
    # Poisson: converges; stopped after maxit = 5 first
    from paper_1508_03954_amd.inputs import sine_load
    q = Params(dim=2, level_max=4, theta=0.0, phi=0.0, variant="add", omega_scheme="exp", omega=0.6)
    bq = O.lumped_rhs(sine_load(4, 2), 4, 0.0)
    sq = mg.Solver(2, 4, theta=0.0, phi=0.0, variant="add", omega_scheme="exp", omega=0.6)
    u5, its5, rel5, rc5 = sq.solve(bq, rtol=1e-12, maxit=5, driver="stationary")
    u5_ref, its5_ref, _, ok5 = O.stationary_solve(q, bq, 1e-12, 5)
    assert rc5 == mg.MG_ENOTCONV and its5 == 5 == its5_ref and not ok5
    assert relerr(to_np(u5), u5_ref) <= TOL
    true5 = np.linalg.norm(O.zero_boundary(bq - O.apply_H(u5_ref, 4, 0.0, 0.0))) / np.linalg.norm(bq)
    assert abs(rel5 - true5) <= 1e-10 * true5
    uc, itsc, relc, rcc = sq.solve(bq, rtol=1e-8, maxit=400, driver="stationary")
    uc_ref, itsc_ref, _, okc = O.stationary_solve(q, bq, 1e-8, 400)
    assert okc and rcc == mg.MG_OK and itsc == itsc_ref and relc <= 1e-8
    assert relerr(to_np(uc), uc_ref) <= 1e-10
