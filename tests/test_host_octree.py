"""The library's host octree (C++, no GPU needed) against the oracle's
independent octree: identical leaves after refinement and closure, identical
meshes (nodes, hanging interpolation, supports, loads) and identical
adaptations (marking, both sweeps, closure, transfer)."""
import numpy as np
import pytest

import synth
from oracle import amr, mesh as om
from paper_1009_4975_amd import binding


def leafset(level, anchor):
    return {(int(l), *map(int, a)) for l, a in zip(level, anchor)}


def grow_band(base, L, width=synth.C2_WIDTH):
    """C2 recipe on both sides: refine where the band meets a leaf, then close."""
    case = synth.c2(base=base, max_level=L, width=width)
    fld = case.extra["field"]
    t = binding.Octree(base, L)
    b = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])]) << L
    lv, an = np.zeros(len(b), np.int64), b
    for _ in range(L):
        tl, ta = t.leaves()
        t.refine(synth.band_marks(fld, tl, ta, L))
        lv, an, _ = amr.refine(lv, an, L, synth.band_marks(fld, lv, an, L))
    t.balance()
    lv, an, _ = amr.balance(lv, an, L)
    return case, t, lv, an


@pytest.mark.parametrize("base,L", [((4, 2, 2), 2), ((6, 3, 3), 3)])
def test_refine_and_closure_match_oracle(base, L):
    case, t, lv, an = grow_band(base, L, width=0.2)
    tl, ta = t.leaves()
    assert leafset(tl, ta) == leafset(lv, an)
    # Morton order keeps families contiguous: anchors non-decreasing in Morton key
    assert amr.is_balanced(tl, ta, L)


@pytest.mark.parametrize("seed", range(4))
def test_random_closure_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    L = 3
    t = binding.Octree((2, 2, 2), L)
    b = np.array([[i, j, k] for k in range(2) for j in range(2) for i in range(2)]) << L
    lv, an = np.zeros(8, np.int64), b
    for _ in range(3):
        tl, ta = t.leaves()
        # mark the same leaves on both sides (by position)
        pick = {(int(l), *map(int, a)) for l, a in zip(tl, ta) if rng.random() < 0.3}
        t.refine(np.array([(int(l), *map(int, a)) in pick for l, a in zip(tl, ta)]))
        lv, an, _ = amr.refine(lv, an, L, np.array([(int(l), *map(int, a)) in pick for l, a in zip(lv, an)]))
    t.balance()
    lv, an, _ = amr.balance(lv, an, L)
    tl, ta = t.leaves()
    assert leafset(tl, ta) == leafset(lv, an)


def _oracle_mesh_from(t, case):
    tl, ta = t.leaves()
    return om.build_mesh(tl, ta, case.max_level, case.dims)


def test_mesh_hanging_supports_loads_match_oracle():
    case, t, lv, an = grow_band((4, 2, 2), 2, width=0.2)
    m = t.build_mesh(case.fixed, case.load)
    o = _oracle_mesh_from(t, case)
    assert m.n_nodes == o.n_nodes and m.n_elems == o.n_elems
    # node correspondence by coordinates
    key = {tuple(c): i for i, c in enumerate(o.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in m.node_xyz.tolist()])
    assert len(set(perm.tolist())) == m.n_nodes
    # connectivity (local vertex order i + 2j + 4k) identical per leaf
    tl, ta = t.leaves()
    okey = {(int(l), *map(int, a)): e for e, (l, a) in enumerate(zip(o.level, o.anchor))}
    for e in range(m.n_elems):
        oe = okey[(int(tl[e]), *map(int, ta[e]))]
        assert (perm[m.elem_nodes[e]] == o.elem_nodes[oe]).all()
    # hanging set and weights
    assert m.hang_node.size > 0
    assert set(perm[m.hang_node].tolist()) == set(np.nonzero(o.hanging)[0].tolist())
    T = o.Tn.tocsr()
    for i, h in enumerate(m.hang_node):
        ms = m.hang_master[m.hang_ptr[i]:m.hang_ptr[i + 1]]
        ws = m.hang_w[m.hang_ptr[i]:m.hang_ptr[i + 1]]
        row = T[perm[h]]
        want = dict(zip(row.indices.tolist(), row.data.tolist()))
        got = {int(perm[a]): float(w) for a, w in zip(ms, ws)}
        assert set(got) == set(want)
        for k in got:
            assert got[k] == pytest.approx(want[k], abs=1e-15)
    # supports and consistent loads
    fx = om.fixed_dofs(o, case.fixed)
    f = om.load_vector(o, case.load)
    P3 = (3 * perm[:, None] + np.arange(3)).ravel()
    assert (m.dof_fixed.astype(bool) == fx[P3]).all()
    assert np.allclose(m.f_load, f[P3], rtol=1e-14, atol=1e-15)


def test_bridge_face_load_matches_oracle():
    L = 2
    t = binding.Octree((4, 2, 2), L)
    fld = synth.c2(base=(4, 2, 2), max_level=L, width=0.2).extra["field"]
    tl, ta = t.leaves()
    t.refine(synth.band_marks(fld, tl, ta, L))
    t.balance()
    dims = t.dims
    fixed, load = synth.bridge_bc(*dims)
    m = t.build_mesh(fixed, load)
    tl, ta = t.leaves()
    o = om.build_mesh(tl, ta, L, dims)
    key = {tuple(c): i for i, c in enumerate(o.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in m.node_xyz.tolist()])
    P3 = (3 * perm[:, None] + np.arange(3)).ravel()
    assert np.allclose(m.f_load, om.load_vector(o, load)[P3], rtol=1e-14, atol=1e-16)
    assert (m.dof_fixed.astype(bool) == om.fixed_dofs(o, fixed)[P3]).all()
    assert m.f_load.sum() == pytest.approx(-1.0)


def test_uniform_mesh_lexicographic():
    fixed, load = synth.cantilever_bc(5, 3, 2)
    m = binding.uniform_mesh((5, 3, 2), fixed, load)
    o = om.uniform_mesh((5, 3, 2))
    assert (m.node_xyz == o.coords).all()
    assert m.hang_node.size == 0
    assert np.allclose(m.f_load, om.load_vector(o, load), rtol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adapt_matches_oracle(seed):
    L = 3
    case, t, lv, an = grow_band((4, 2, 2), L, width=0.3)
    rng = np.random.default_rng(seed)
    tl, ta = t.leaves()
    # a density that is solid in a blob and void elsewhere
    cen = ta + 0.5 * (1 << (L - tl))[:, None]
    c0 = rng.uniform([0, 0, 0], case.dims)
    rho = np.where(np.linalg.norm(cen - c0, axis=1) < 8.0, 0.9, 0.05) + 0.01 * rng.random(len(tl))
    new_rho = t.adapt(rho, 0.5, 1.5)
    nl, na = t.leaves()
    ol, oa, orho, _ = amr.adapt(tl, ta, L, rho, 0.5, 1.5)
    assert leafset(nl, na) == leafset(ol, oa)
    okey = {(int(l), *map(int, a)): r for l, a, r in zip(ol, oa, orho)}
    for l, a, r in zip(nl, na, new_rho):
        assert r == pytest.approx(okey[(int(l), *map(int, a))], rel=1e-14)
    assert amr.is_balanced(nl, na, L)


def test_transfer_nodal_matches_oracle():
    L = 2
    case, t, lv, an = grow_band((4, 2, 2), L, width=0.3)
    m_old = t.build_mesh(case.fixed, case.load)
    tl, ta = t.leaves()
    o_old = om.build_mesh(tl, ta, L, case.dims)
    rng = np.random.default_rng(3)
    # a continuous field: values on unconstrained nodes, hanging ones interpolated
    key = {tuple(c): i for i, c in enumerate(o_old.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in m_old.node_xyz.tolist()])
    from oracle import system as osys
    ut = rng.normal(size=3 * o_old.n_nodes)
    u_o = osys.dof_interp(o_old) @ np.where(np.repeat(o_old.hanging, 3), 0.0, ut)
    u_p = u_o.reshape(-1, 3)[perm].ravel()
    rho = np.full(len(tl), 0.02)
    rho[: len(tl) // 3] = 0.9
    t.adapt(rho, 0.5, 1.5)
    m_new = t.build_mesh(case.fixed, case.load)
    got = t.transfer_nodal(u_p, m_new.n_nodes)
    want = amr.transfer_displacement(o_old, u_o, m_new.node_xyz.astype(np.int64))
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_library_exports_every_declared_symbol():
    import ctypes
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(binding.PKG), "include", "amrto.h")).read()
    declared = set(re.findall(r"\b(amrto_[a-z0-9_]+)\s*\(", hdr))
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [s for s in sorted(declared) if not hasattr(lib, s)]
    assert not missing, missing
    assert declared >= set(binding.exported_symbols())


@pytest.mark.parametrize("seed", range(3))
def test_rebuild_tree_from_leaf_set(seed):
    """Checkpoint restore: the tree rebuilt from a saved leaf set has the same
    leaves in the same order and builds the same mesh, node for node."""
    from paper_1009_4975_amd.simp import rebuild_tree
    rng = np.random.default_rng(seed)
    base, L = (4, 2, 2), 3
    t = binding.Octree(base, L)
    for _ in range(3):
        n = len(t.leaves()[0])
        t.refine((rng.random(n) < 0.25).astype(np.uint8))
        t.balance()
    lv, an = t.leaves()
    r = rebuild_tree(base, L, lv, an)
    lv2, an2 = r.leaves()
    assert np.array_equal(lv, lv2) and np.array_equal(an, an2)
    fixed, load = synth.cantilever_bc(*t.dims)
    m1, m2 = t.build_mesh(fixed, load), r.build_mesh(fixed, load)
    for f in ("node_xyz", "elem_nodes", "hang_node", "hang_ptr", "hang_master", "hang_w", "dof_fixed", "f_load"):
        assert np.array_equal(getattr(m1, f), getattr(m2, f)), f
    # a leaf set that is no tree of this base grid is refused
    with pytest.raises(ValueError):
        rebuild_tree(base, L, lv[1:], an[1:])
    with pytest.raises(ValueError):
        rebuild_tree((4, 2, 1), L, lv, an)


def test_sweep2_case_matches_oracle():
    """The hand-built sweep-2 tree (a complete void family whose derefinement
    would put an edge-4 leaf next to edge-1 leaves): the library's adaptation
    drops it exactly as the oracle's does and leaves the tree unchanged."""
    from test_oracle_amr import sweep2_tree
    level, anchor, L = sweep2_tree()
    t = binding.Octree((2, 1, 1), L)
    want = leafset(level, anchor)
    for _ in range(L):
        tl, ta = t.leaves()
        # split every library leaf that is an ancestor of (strictly contains) a target leaf
        s = 1 << (L - tl)
        marks = [any(lv > l and (a >= an).all() and (a < an + sz).all() for lv, a in zip(level, anchor))
                 for l, an, sz in zip(tl, ta, s)]
        t.refine(np.array(marks, np.uint8))
    tl, ta = t.leaves()
    assert leafset(tl, ta) == want
    rho = np.where(tl == 3, 1.0, 0.1)
    t.adapt(rho, 0.5, 1.5)
    nl, na = t.leaves()
    assert leafset(nl, na) == want
