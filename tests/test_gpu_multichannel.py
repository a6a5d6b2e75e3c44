"""Same-grid multichannel form (Section 7.5) through the C ABI: nchan channels
with their own phi on one grid (array-of-structures), against nchan
independent runs of the FP64 oracle's pipelined cycle -- residual norms of
every channel after every cycle and the flushed iterates (1e-12) -- and the
operator of every channel against the oracle's."""

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


def channel_phis(nchan, seed):
    rng = np.random.default_rng(seed)
    k = rng.uniform(3.0, 25.0, nchan)
    return [float(kk) ** 2 * (1 + 0.5j) for kk in k]


CASES = [
    # dim, L, lmin, nchan, variant, scheme
    (2, 4, 1, 1, "bpx", "const"),
    (2, 4, 1, 4, "add", "const"),
    (2, 5, 2, 8, "hb", "exp"),
    (2, 3, 1, 16, "bpx", "transition"),
    (3, 3, 1, 2, "bpx", "const"),
    (3, 3, 1, 4, "hb", "const"),
    (3, 4, 1, 8, "add", "const"),
    (3, 2, 1, 16, "bpx", "two_phase"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_multichannel_matches_independent_oracle_runs(case):
    from paper_1508_03954_amd import mg
    dim, L, lmin, nchan, variant, scheme = case
    print(f"\n[case] multichannel {case}", flush=True)
    theta = 0.3
    phis = channel_phis(nchan, seed=31 + nchan)
    n = 3 ** L + 1
    rng = np.random.default_rng(7 + nchan)
    b = rng.standard_normal((n,) * dim + (nchan,)) + 1j * rng.standard_normal((n,) * dim + (nchan,))
    u0 = rng.standard_normal((n,) * dim + (nchan,)) + 1j * rng.standard_normal((n,) * dim + (nchan,))
    m = mg.MultiChannel(dim, L, phis, level_min=lmin, theta=theta, variant=variant, omega_scheme=scheme, omega=0.6)
    m.set_rhs(b)
    m.set_solution(u0)
    pipes = []
    for c in range(nchan):
        p = Params(dim=dim, level_max=L, level_min=lmin, theta=theta, phi=phis[c], variant=variant,
                   omega_scheme=scheme, omega=0.6)
        pipes.append(O.Pipelined(p, O.zero_boundary(b[..., c]), O.zero_boundary(u0[..., c])))
    ncyc = 4
    res = m.cycle(ncyc)
    for k in range(ncyc):
        for c in range(nchan):
            ref, _ = pipes[c].cycle()
            assert abs(res[k, c] - ref) <= 1e-12 * ref, (k, c, res[k, c], ref)
    u = m.flush().cpu().numpy()
    for c in range(nchan):
        ur = pipes[c].flush()
        err = np.linalg.norm(u[..., c] - ur) / np.linalg.norm(ur)
        assert err <= 1e-12, (c, err)
    # the operator of every channel
    x = rng.standard_normal((n,) * dim + (nchan,)) + 1j * rng.standard_normal((n,) * dim + (nchan,))
    y = m.apply(x).cpu().numpy()
    for c in range(nchan):
        yr = O.apply_H(x[..., c], L, theta, phis[c])
        assert np.linalg.norm(y[..., c] - yr) <= 1e-12 * np.linalg.norm(yr), c
    m.close()


def test_multichannel_rejects_bad_arguments():
    from paper_1508_03954_amd import mg
    with pytest.raises(mg.MGError):
        mg.MultiChannel(2, 3, [1.0, 2.0, 3.0])          # 3 channels
    with pytest.raises(mg.MGError):
        mg.MultiChannel(2, 3, [1.0], level_min=3)        # one level
