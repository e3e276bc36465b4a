"""The design difference of Eq. (10) through the C ABI against the oracle's
finest-lattice statement, on an octree against a uniform brick of the same
lattice box, octree against octree (different leaf sets) and a design
against itself."""
import numpy as np
import pytest

import cases
from oracle import design

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(p):
    from paper_1009_4975_amd import binding
    ctx = binding.Context(0)
    ctx.upload_mesh(p.lib_mesh)
    return ctx


def _m(p):
    o = p.orc
    return (o.level, o.anchor, o.max_level, o.dims)


def test_design_difference_matches_oracle(lib):
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    oa = cases.octree_pair((4, 2, 2), 2, width=0.2)
    ob = cases.octree_pair((4, 2, 2), 2, width=0.35)
    un = cases.uniform_pair(oa.orc.dims)
    assert len(oa.orc.level) != len(ob.orc.level)
    rng = np.random.default_rng(3)
    ra = rng.uniform(0.001, 1, oa.orc.n_elems)
    rb = rng.uniform(0.001, 1, ob.orc.n_elems)
    ru = rng.uniform(0.001, 1, un.orc.n_elems)
    ca, cb, cu = _ctx(oa), _ctx(ob), _ctx(un)
    da, db, du = dev(oa.to_lib_elems(ra)), dev(ob.to_lib_elems(rb)), dev(un.to_lib_elems(ru))
    for (c1, d1, p1, r1), (c2, d2, p2, r2) in (((ca, da, oa, ra), (cu, du, un, ru)),
                                               ((cu, du, un, ru), (ca, da, oa, ra)),
                                               ((ca, da, oa, ra), (cb, db, ob, rb))):
        got = c1.design_difference(d1, c2, d2)
        want = design.design_difference(_m(p1), r1, _m(p2), r2)
        assert got == pytest.approx(want, rel=1e-13)
    assert ca.design_difference(da, ca, da) == 0.0
    # the uniform refinement of a design differs from it by zero
    cells = design.finest_cells(*_m(oa), ra).ravel()
    assert ca.design_difference(da, cu, dev(cells)) == pytest.approx(0.0, abs=1e-15)


def test_design_difference_rejects_other_box(lib):
    from paper_1009_4975_amd import binding
    a = cases.uniform_pair((4, 3, 2))
    b = cases.uniform_pair((4, 3, 3))
    ca, cb = _ctx(a), _ctx(b)
    ra = torch.ones(a.orc.n_elems, dtype=torch.float64, device="cuda")
    rb = torch.ones(b.orc.n_elems, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.AmrtoError):
        ca.design_difference(ra, cb, rb)
