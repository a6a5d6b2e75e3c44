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


def test_gradient_finite_differences_full_potential_workload():
    from paper_1508_03954_amd.adjoint import shell_functional
    from paper_1508_03954_amd.inputs import config_potential, sample_vertices, shell_mask
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
    verts = sample_vertices(L, dim, 32, seed=55)
    eps = 1e-2
    fd, ad = [], []
    with torch.no_grad():
        for j in verts:
            idx = tuple(int(t) for t in j)
            Vp = V.clone()
            Vp[idx] += eps
            Vm = V.clone()
            Vm[idx] -= eps
            Jp = shell_functional(Vp, b, shell, cfg).item()
            Jm = shell_functional(Vm, b, shell, cfg).item()
            fd.append((Jp - Jm) / (2 * eps))
            ad.append(grad[idx].item())
    fd, ad = np.array(fd), np.array(ad)
    scale = np.abs(fd).max()
    err = np.abs(fd - ad).max() / scale
    print(f"\n[adjoint FD] J={J.item():.6e}, 32 vertices, max|dJ/dV|={scale:.3e}, max rel. deviation={err:.2e}")
    assert scale > 0
    assert err <= 1e-3, (fd, ad)
