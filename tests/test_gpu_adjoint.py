"""Adjoint form: gradient of the outer-shell functional J = sum_S |u|^2 with
respect to the potential V, through torch.autograd, against

* the oracle's cell formula evaluated on dense oracle solves (small grid), and
* central finite differences of J at 32 seeded interior vertices on the full
  3D L = 5, k = 15 potential workload (GPU solves, relative residual 1e-13).
"""

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


def test_autograd_gradient_matches_oracle_small():
    from paper_1508_03954_amd.adjoint import shell_functional
    from paper_1508_03954_amd.inputs import shell_mask
    dim, L = 3, 3
    n = 3 ** L + 1
    rng = np.random.default_rng(17)
    V = 40 * rng.standard_normal((n,) * dim)
    phi0 = 225 * (1 + 0.3j)
    b = O.zero_boundary(rng.standard_normal((n,) * dim) + 1j * rng.standard_normal((n,) * dim))
    shell = shell_mask(L, dim, 0.5, 0.9)
    cfg = {"dim": dim, "level_max": L, "theta": 0.0, "phi0": phi0, "variant": "bpx", "rtol": 1e-13}
    Vt = torch.tensor(V, dtype=torch.float64, device="cuda", requires_grad=True)
    J = shell_functional(Vt, torch.from_numpy(b).cuda(), torch.from_numpy(shell).cuda(), cfg)
    J.backward()
    g = Vt.grad.cpu().numpy()
    p = Params(dim=dim, level_max=L, theta=0.0, phi=0, phi_nodal=phi0 - V)
    u = O.dense_solve(p, b)
    pc = Params(dim=dim, level_max=L, theta=0.0, phi=0, phi_nodal=phi0 - V, conjugate=True)
    lam = O.dense_solve(pc, np.where(shell, u, 0))
    ref = O.potential_gradient(u, lam, L, 0.0)
    Jref = O.shell_functional(u, shell)
    assert abs(J.item() - Jref) <= 1e-11 * Jref
    assert np.linalg.norm(g - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.timeout(600)
def test_gradient_finite_differences_full_potential_workload():
    """Central differences with steps 1e-1 and 1e-2 and their Richardson
    extrapolation (the central difference's error is c eps^2 + O(eps^4), so
    (100 FD(1e-2) - FD(1e-1)) / 99 removes the eps^2 term), at 16 seeded
    interior vertices and 16 seeded vertices next to the shell
    (0.85 < |x| < 1), where the gradient is largest.  Per vertex j:
        |FD_R(j) - dJ/dV_j| <= 1e-3 |dJ/dV_j| + 100 u64 |J| / 1e-2,
    the second term the rounding floor of a difference quotient whose two
    values of J (from solves to 1e-13) each carry up to ~50 ulps (u64 = 2^-53);
    it is about 1e-4 of the largest sampled gradient here.  At least 8
    vertices must have gradients 100 times above that floor, so the relative
    term is what bites there."""
    from paper_1508_03954_amd.adjoint import shell_functional
    from paper_1508_03954_amd.inputs import config_potential, sample_vertices, shell_mask, vertex_coords
    from paper_1508_03954_amd import mg
    prob = config_potential(level_max=5)
    L, dim = prob.level_max, prob.dim
    shell = torch.from_numpy(shell_mask(L, dim, 0.9, 0.95)).cuda()
    cfg = {"dim": dim, "level_max": L, "theta": prob.theta, "phi0": prob.phi, "variant": "bpx", "rtol": 1e-13,
           "maxit": 3000}
    V = torch.from_numpy(prob.potential).cuda()
    helper = mg.Solver(dim, L, theta=prob.theta, phi=prob.phi)
    b = helper.rhs_from_nodal(torch.from_numpy(prob.chi).cuda())
    Vt = V.clone().requires_grad_(True)
    J = shell_functional(Vt, b, shell, cfg)
    J.backward()
    grad = Vt.grad
    n = 3 ** L + 1
    xs = vertex_coords(L, dim)
    rad = np.sqrt(sum(x ** 2 for x in xs))
    near = np.argwhere((rad > 0.85) & (rad < 1.0) & np.pad(np.ones((n - 2,) * dim, bool), 1))
    pick = np.random.default_rng(56).choice(len(near), 16, replace=False)
    verts = [tuple(int(t) for t in j) for j in sample_vertices(L, dim, 16, seed=55)]
    verts += [tuple(int(t) for t in near[k]) for k in pick]

    def fd(idx, eps):
        with torch.no_grad():
            Vp = V.clone()
            Vp[idx] += eps
            Vm = V.clone()
            Vm[idx] -= eps
            return (shell_functional(Vp, b, shell, cfg).item() - shell_functional(Vm, b, shell, cfg).item()) / (2 * eps)

    f1 = np.array([fd(j, 1e-1) for j in verts])
    f2 = np.array([fd(j, 1e-2) for j in verts])
    ad = np.array([grad[j].item() for j in verts])
    rich = (100 * f2 - f1) / 99
    big = np.abs(ad).max()
    floor = 100 * 2.0 ** -53 * abs(J.item()) / 1e-2
    dev = np.abs(rich - ad)
    bound = 1e-3 * np.abs(ad) + floor
    strong = np.abs(ad) >= 100 * floor
    print(f"\n[adjoint FD] J={J.item():.6e}; 32 vertices, max|dJ/dV|={big:.3e}, rounding floor {floor:.2e}; "
          f"worst deviation / bound {np.max(dev / bound):.2f}; {strong.sum()} vertices above 100 floors, worst "
          f"relative deviation there {np.max(dev[strong] / np.abs(ad[strong])):.2e}; step pair spread "
          f"{np.abs(f1 - f2).max() / big:.2e} of max", flush=True)
    assert big > 0 and strong.sum() >= 8
    assert np.all(dev <= bound), (dev / bound, ad, rich)
