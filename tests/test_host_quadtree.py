"""The library's host quadtree (C++, no GPU needed) against the 2-D oracle's
independent quadtree: identical leaves after refinement and closure, identical
meshes (nodes, connectivity, hanging interpolation, supports, the point load),
identical adaptations (marking, both sweeps, closure, density transfer) and a
nodal transfer that reproduces bilinear fields exactly."""
import numpy as np
import pytest

from oracle import plane
from paper_1009_4975_amd import binding

FIXED = [{"x": 0}]


def leafset(level, anchor):
    return {(int(l), int(a[0]), int(a[1])) for l, a in zip(level, anchor)}


def grow(base, L, seed, rounds=None, p=0.3):
    """Refine the same leaves (by position) on both sides, then close."""
    rng = np.random.default_rng(seed)
    t = binding.Quadtree(base, L)
    lv, an = plane.base_leaves(base, L)
    for _ in range(L if rounds is None else rounds):
        tl, ta = t.leaves()
        pick = {k for k in sorted(leafset(tl, ta)) if rng.random() < p}
        t.refine(np.array([(int(l), int(a[0]), int(a[1])) in pick for l, a in zip(tl, ta)]))
        lv, an, _ = plane.refine(lv, an, L, np.array([(int(l), int(a[0]), int(a[1])) in pick
                                                      for l, a in zip(lv, an)]))
    t.balance()
    lv, an, _ = plane.balance(lv, an, L)
    return t, lv, an


@pytest.mark.parametrize("base,L,seed", [((4, 2), 2, 0), ((4, 2), 3, 1), ((6, 3), 3, 2), ((2, 2), 4, 3)])
def test_refine_and_closure_match_oracle(base, L, seed):
    t, lv, an = grow(base, L, seed)
    tl, ta = t.leaves()
    assert leafset(tl, ta) == leafset(lv, an)
    assert plane.is_balanced(tl, ta, L)
    # Morton order: every family of four siblings is contiguous
    sizes = plane.leaf_sizes(tl, L)
    for i in range(len(tl)):
        if tl[i] > 0 and ta[i][0] % (2 * sizes[i]) == 0 and ta[i][1] % (2 * sizes[i]) == 0:
            fam = leafset(tl[i:i + 4], ta[i:i + 4])
            if all(l == tl[i] for l in tl[i:i + 4]):
                assert len(fam) == 4


def _mesh_pair(base, L, seed, load_at=None):
    t, lv, an = grow(base, L, seed)
    dims = tuple(b << L for b in base)
    at = load_at or (dims[0], dims[1] // 2)
    load = {"at": at, "comp": 1, "total": -1.0}
    m = t.build_mesh(FIXED, load)
    o = plane.build_mesh(lv, an, L, dims)
    return t, m, o, load


@pytest.mark.parametrize("base,L,seed", [((4, 2), 2, 0), ((6, 3), 3, 2)])
def test_mesh_matches_oracle(base, L, seed):
    t, m, o, load = _mesh_pair(base, L, seed)
    assert m.n_nodes == o.n_nodes and m.n_elems == o.n_elems
    key = {tuple(c): i for i, c in enumerate(o.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in m.node_xy.tolist()])
    assert len(set(perm.tolist())) == m.n_nodes
    # nodes numbered with x fastest: y, then x non-decreasing
    assert (np.lexsort((m.node_xy[:, 0], m.node_xy[:, 1])) == np.arange(m.n_nodes)).all()
    tl, ta = t.leaves()
    okey = {(int(l), int(a[0]), int(a[1])): e for e, (l, a) in enumerate(zip(o.level, o.anchor))}
    for e in range(m.n_elems):
        oe = okey[(int(tl[e]), int(ta[e][0]), int(ta[e][1]))]
        assert (perm[m.elem_nodes[e]] == o.elem_nodes[oe]).all()
        assert m.elem_level[e] == o.level[oe]
    # hanging rows: same nodes, same masters and weights
    assert m.hang_node.size > 0
    hang = np.zeros(m.n_nodes, bool)
    hang[m.hang_node] = True
    assert (o.hanging[perm] == hang).all()
    Tn = o.Tn.tocsr()
    for h, v in enumerate(m.hang_node):
        got = {int(perm[mm]): w for mm, w in zip(m.hang_master[m.hang_ptr[h]:m.hang_ptr[h + 1]],
                                                 m.hang_w[m.hang_ptr[h]:m.hang_ptr[h + 1]])}
        row = Tn.getrow(perm[v])
        want = {int(c): float(w) for c, w in zip(row.indices, row.data)}
        assert got.keys() == want.keys()
        for c in got:
            assert got[c] == pytest.approx(want[c], abs=1e-15)
    fixed = plane.fixed_dofs(o, FIXED)
    assert (m.dof_fixed.astype(bool) == fixed.reshape(-1, 2)[perm].ravel()).all()
    f = plane.load_vector(o, load)
    assert np.array_equal(m.f_load, f.reshape(-1, 2)[perm].ravel())


@pytest.mark.parametrize("seed,r_amr", [(0, 1.5), (1, 2.5), (2, 4.0)])
def test_adapt_matches_oracle(seed, r_amr):
    base, L = (6, 3), 3
    t, lv, an = grow(base, L, seed, rounds=2)
    rng = np.random.default_rng(100 + seed)
    tl, ta = t.leaves()
    # a smooth solid blob plus noise, on the library's leaf order; the
    # oracle gets the same values through the leaf keys
    cen = ta + 0.5 * plane.leaf_sizes(tl, L)[:, None]
    rho = np.clip(np.exp(-((cen[:, 0] - 20.0) ** 2 + (cen[:, 1] - 12.0) ** 2) / 60.0)
                  + 0.1 * rng.random(len(tl)), 1e-3, 1.0)
    idx = {(int(l), int(a[0]), int(a[1])): i for i, (l, a) in enumerate(zip(tl, ta))}
    rho_o = np.array([rho[idx[(int(l), int(a[0]), int(a[1]))]] for l, a in zip(lv, an)])
    rnew = t.adapt(rho, 0.5, r_amr)
    l2, a2, r2 = plane.adapt(lv, an, L, rho_o, 0.5, r_amr)
    nl, na = t.leaves()
    assert leafset(nl, na) == leafset(l2, a2)
    okey = {(int(l), int(a[0]), int(a[1])): r for l, a, r in zip(l2, a2, r2)}
    got = {(int(l), int(a[0]), int(a[1])): r for l, a, r in zip(nl, na, rnew)}
    for k in okey:
        assert got[k] == pytest.approx(okey[k], rel=1e-14, abs=1e-15)
    assert plane.is_balanced(nl, na, L)


def test_transfer_reproduces_bilinear_fields():
    base, L = (4, 2), 3
    t, _, _ = grow(base, L, 5, rounds=2)
    dims = tuple(b << L for b in base)
    load = {"at": (dims[0], dims[1] // 2), "comp": 1, "total": -1.0}
    m0 = t.build_mesh(FIXED, load)
    tl, ta = t.leaves()
    cen = ta + 0.5 * plane.leaf_sizes(tl, L)[:, None]
    rho = np.where(np.abs(cen[:, 1] - dims[1] / 2) < 3, 1.0, 0.05)
    t.adapt(rho, 0.5, 1.5)
    m1 = t.build_mesh(FIXED, load)

    def field(xy):
        x, y = xy[:, 0].astype(float), xy[:, 1].astype(float)
        return np.stack([0.3 + 0.02 * x - 0.05 * y, -0.1 + 0.04 * x + 0.01 * y], 1).ravel()

    u1 = t.transfer_nodal(field(m0.node_xy), m1.n_nodes)
    assert np.allclose(u1, field(m1.node_xy), atol=1e-13)
