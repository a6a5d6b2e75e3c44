"""GPU: the Section 7.4 application problem (eq. 08-gaussian, regular grid
h = 1/81, absorbing layer) through the C ABI, against the FP64 oracle and the
regular-grid columns of Table 08gaussian.

For every rotation and solver of the table: 50 cycles from u = 0 and a flush;
the flushed iterate must match the oracle's to 1e-12 relative, and the
maximum-norm residual reduction (residual from the library's own operator)
both the oracle's value (1e-10 relative) and the paper's entry under the
soft criterion of tests/test_oracle_gaussian08.py.
"""

import math

import numpy as np
import pytest

import oracle as O
from paper_1508_03954_amd.inputs import config_gaussian08
from test_oracle_gaussian08 import OMEGA_2PHASE, SOLVERS, agrees, paper_table, solver_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def gpu_kwargs(prob, solver):
    kw = dict(theta=prob.theta, phi=0.0, layer=prob.layer, phi_field=torch.from_numpy(prob.phi_field()))
    if solver == "jacobi":
        if prob.theta == 0:
            return dict(level_min=prob.level_max, variant="add", omega_scheme="two_phase", omega=OMEGA_2PHASE, **kw)
        return dict(level_min=prob.level_max, variant="add", omega_scheme="const", omega=0.4, **kw)
    if solver == "transition":
        return dict(level_min=1, variant="add", omega_scheme="transition", omega=0.4, **kw)
    return dict(level_min=1, variant="bpx", omega_scheme="const", omega=0.4, **kw)


@pytest.mark.parametrize("theta", [0, 18, 25, 35, 45])
def test_table_08gaussian_on_gpu(theta):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_03954_amd import mg
    table = paper_table()
    prob = config_gaussian08(theta)
    L = prob.level_max
    for solver in SOLVERS:
        print(f"\n[case] gaussian08 theta={theta} {solver}", flush=True)
        p = solver_params(prob, solver)
        b_ref = O.lumped_rhs(prob.chi, L, p.theta_at(L))
        red_ref, u_ref = O.max_norm_reduction(p, b_ref, 50)
        s = mg.Solver(2, L, **gpu_kwargs(prob, solver))
        b = s.rhs_from_nodal(torch.from_numpy(prob.chi))
        assert np.linalg.norm(b.cpu().numpy() - b_ref) <= 1e-15 * np.linalg.norm(b_ref)
        s.set_rhs(b)
        s.set_solution(torch.zeros_like(b))
        s.cycle(50, norms=False)
        u = s.flush()
        r = (b - s.apply(u)).cpu().numpy()
        bn = b.cpu().numpy()
        red = np.abs(r[1:-1, 1:-1]).max() / np.abs(bn[1:-1, 1:-1]).max()
        un = u.cpu().numpy()
        err = np.linalg.norm(un - u_ref) / np.linalg.norm(u_ref)
        print(f"theta {theta:2d} {solver:10s} gpu {red:.3e} oracle {red_ref:.3e} paper {table[theta][solver]}"
              f"  |u - u_oracle|/|u_oracle| {err:.1e}", flush=True)
        assert err <= 1e-12, (theta, solver, err)
        assert abs(red - red_ref) <= 1e-10 * red_ref, (theta, solver, red, red_ref)
        assert agrees(solver, red, table[theta][solver]), (theta, solver, red)
