"""Parity at the full workload sizes, in the launch configuration the benchmark
times (fused finest sweep, tile chosen by the autotuner).

* 3D, levels 1..5 (244^3 vertices), k = 20, theta = pi/6, hb and BPX: every
  level field against the pipelined FP64 oracle after each of 2 cycles.
* 2D, levels 1..5 (244^2), k = 10, CSL shift (1 + 0.5i), BPX: 30 cycles.
* 3D, levels 1..6 (730^3): the operator at 2000 seeded vertices against the
  oracle applied on a local window (the full oracle does not fit this size).
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.cycle import Params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_03954_amd import mg
    mg.load_library()


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def compare_state(s, pipe, p, k, tol=1e-12):
    """Every level field against the oracle at tol relative to the field's own
    norm.  Coarse b slots and smoothing fields (Galerkin form) against the
    oracle's restricted-residual form R^(L-l) r_L (no cancellation)."""
    L = p.level_max
    chain = pipe.restricted_residual_state()
    for lev in range(p.level_min, L + 1):
        for field in ("u", "b", "sc", "sf", "si"):
            got = to_np(s.get_level(lev, field))
            if lev == L:
                ref = {"u": pipe.u[L] + pipe.sc[L], "b": pipe.b[L]}.get(field, np.zeros_like(got))
            elif field == "u":
                ref = pipe.u[lev]
            else:
                ref = chain[lev][field]
            if not np.any(ref):
                assert not np.any(got), (k, lev, field)
                continue
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= tol, (k, lev, field, err)


def run_workload(prob, ncycles, tol=1e-12):
    from paper_1508_03954_amd import mg
    L, dim = prob.level_max, prob.dim
    s = mg.Solver(dim, L, theta=prob.theta, phi=prob.phi, variant=prob.variant, omega=prob.omega)
    tile, us, _ = s.autotune(reps=2)
    print(f"\n[case] {prob.name}: tile {tile} ({us:.1f} us)", flush=True)
    b = s.rhs_from_nodal(torch.from_numpy(prob.chi).cuda())
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    p = Params(dim=dim, level_max=L, theta=prob.theta, phi=prob.phi, variant=prob.variant, omega=prob.omega)
    bo = O.lumped_rhs(prob.chi, L, prob.theta)
    assert np.linalg.norm(to_np(b) - bo) <= 1e-15 * np.linalg.norm(bo)
    pipe = O.Pipelined(p, bo)
    for k in range(ncycles):
        rh_ref, rm_ref = pipe.cycle()
        rh, rm = s.cycle(1)
        assert abs(rh[0] - rh_ref) <= tol * rh_ref and abs(rm[0] - rm_ref) <= tol * rm_ref, (k, rh, rh_ref)
        if k < 3 or k == ncycles - 1:
            compare_state(s, pipe, p, k, tol)
    u_ref = pipe.flush()
    u = to_np(s.flush())
    assert np.linalg.norm(u - u_ref) <= tol * np.linalg.norm(u_ref)


@pytest.mark.parametrize("variant", ["bpx", "hb"])
def test_3d_k20_csg_full_size(variant):
    from paper_1508_03954_amd.inputs import config_3d_csg
    run_workload(config_3d_csg(level_max=5, variant=variant), ncycles=2)


def test_2d_k10_csl_full_size_30_cycles():
    from paper_1508_03954_amd.inputs import config_2d_bpx
    run_workload(config_2d_bpx(level_max=5), ncycles=30)


def test_3d_level6_operator_sampled():
    """mg_apply at 730^3 on 2000 seeded vertices against the oracle applied to a
    5^3 window around each vertex (its centre row is exact)."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_3d_large, sample_vertices
    prob = config_3d_large(level_max=6)
    L, dim = 6, 3
    s = mg.Solver(dim, L, theta=prob.theta, phi=prob.phi, variant="bpx", sweep="generic")
    x = torch.from_numpy(prob.chi).cuda()
    y = s.apply(x)
    verts = sample_vertices(L, dim, 2000, seed=66)
    idx = torch.from_numpy(verts).cuda()
    yv = y[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    chi = prob.chi
    n = chi.shape[0]
    worst = 0.0
    for t, j in enumerate(verts):
        lo = [max(int(c) - 2, 0) for c in j]
        win = np.zeros((5, 5, 5), dtype=np.complex128)
        sl = tuple(slice(l, min(l + 5, n)) for l in lo)
        sub = chi[sl]
        win[tuple(slice(0, m) for m in sub.shape)] = sub
        # the window's own boundary plays the role of zeros; vertices on the
        # true domain boundary are zeroed as the operator ignores them
        for a in range(3):
            for off in range(5):
                g = lo[a] + off
                if g <= 0 or g >= n - 1:
                    sl2 = [slice(None)] * 3
                    sl2[a] = off
                    win[tuple(sl2)] = 0
        # the oracle operator on the window (level L cell width); the row of
        # the sampled vertex only touches window entries inside the window
        c = tuple(int(j[a]) - lo[a] for a in range(3))
        ref = O.apply_H(win, L, prob.theta, prob.phi)[c]
        worst = max(worst, abs(yv[t] - ref) / max(abs(ref), 1e-300))
    print(f"\n[level 6 apply] worst relative deviation over 2000 vertices: {worst:.2e}")
    assert worst <= 1e-11
