"""GPU: the allocation-free residual norm (mg_residual_norm_noalloc) against
mg_residual_norm, through the C ABI, on two calls in a row -- the second on a
smaller problem -- so the shared fixed scratch is reused with fewer blocks."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rand(shape, seed):
    g = torch.Generator().manual_seed(seed)
    re = torch.randn(shape, generator=g, dtype=torch.float64)
    im = torch.randn(shape, generator=g, dtype=torch.float64)
    return torch.complex(re, im).cuda().contiguous()


@pytest.mark.parametrize("first,second", [((3, 4, 0.3, 200.0, None), (2, 3, 0.0, 100 * (1 + 0.5j), None)),
                                          ((2, 6, 0.2, 50.0, "varying"), (3, 3, 0.4, 90.0, "layer"))])
def test_noalloc_residual_norm_matches_allocating_entry(first, second):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_03954_amd import mg
    for dim, L, theta, phi, kind in (first, second):
        print(f"\n[case] noalloc residual dim={dim} L={L} {kind}", flush=True)
        n = 3 ** L + 1
        kw = dict(theta=theta, phi=phi)
        if kind == "varying":
            kw["phi_field"] = (phi * (1 + 0.2 * _rand((n,) * dim, 9).real)).cpu()
        if kind == "layer":
            kw["layer"] = (0.5, 1.0 / 3.0, 0b000110)
        s = mg.Solver(dim, L, **kw)
        u, b = _rand((n,) * dim, 1), _rand((n,) * dim, 2)
        ref_h = s.residual_norm(u, b)
        torch.cuda.synchronize()
        got_h, got_max = s.residual_norm_noalloc(u, b)
        r = (b - s.apply(u)).cpu().numpy()
        inner = (slice(1, -1),) * dim
        ref_max = np.abs(r[inner]).max()
        assert abs(got_h - ref_h) <= 1e-12 * ref_h, (got_h, ref_h)
        assert abs(got_max - ref_max) <= 1e-12 * ref_max, (got_max, ref_max)
        # a second call on the same inputs reuses the scratch and gives the same bits
        assert s.residual_norm_noalloc(u, b) == (got_h, got_max)
        s.close()
