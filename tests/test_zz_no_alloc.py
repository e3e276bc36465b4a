"""amrto_oc_update_noalloc (static per-GPU scratch, no allocation) against
amrto_oc_update on the same inputs: bit-identical densities, change and
multiplier, on two calls in a row, the second on a smaller mesh (the scratch
keeps the first call's contents), and the device's free memory unchanged by
the no-allocation calls."""
import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(p, seed):
    rng = np.random.default_rng(seed)
    ne = p.orc.n_elems
    rho = torch.tensor(rng.uniform(0.05, 1.0, ne), dtype=torch.float64, device="cuda")
    dc = torch.tensor(-rng.uniform(0.01, 2.0, ne), dtype=torch.float64, device="cuda")
    want = torch.empty_like(rho)
    got = torch.full_like(rho, np.nan)
    return rho, dc, want, got


def test_oc_noalloc_matches_oc_update(lib):
    from paper_1009_4975_amd import binding
    big = cases.octree_pair((4, 2, 2), 2, width=0.2)
    small = cases.uniform_pair((6, 3, 3))
    assert small.orc.n_elems < big.orc.n_elems
    for p, seed, volfrac in ((big, 11, 0.4), (small, 12, 0.45)):
        ctx = binding.Context(0)
        ctx.upload_mesh(p.lib_mesh)
        rho, dc, want, got = _inputs(p, seed)
        ch0, lam0 = ctx.oc_update(rho, dc, want, volfrac)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        ch1, lam1 = ctx.oc_update_noalloc(rho, dc, got, volfrac)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
        assert torch.equal(got, want), "no-allocation OC differs from amrto_oc_update"
        assert ch1 == ch0 and lam1 == lam0
        vol = p.orc.volumes[p.eperm]
        assert float(got.cpu().numpy() @ vol) == pytest.approx(volfrac * vol.sum(), rel=1e-11)
