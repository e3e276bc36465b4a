"""Pins for the oracle's octree operations (paper Sec. 4 marking and sweeps,
Sec. 6 level-one compatibility), checked against pairwise brute force."""
import itertools

import numpy as np
import pytest

import synth
from oracle import amr, mesh as om


def brute_incompatible(level, anchor, L):
    """Pairs sharing a face or edge (closed boxes meet in >= 1 dimension) with
    gap >= 2, by comparing every pair of leaves."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    s = (1 << (L - level)).astype(np.int64)
    hi_ = anchor + s[:, None]
    lo = np.maximum(anchor[:, None, :], anchor[None, :, :])
    hi = np.minimum(hi_[:, None, :], hi_[None, :, :])
    touch = (hi >= lo).all(-1)
    dim = (hi > lo).sum(-1)
    gap = np.abs(level[:, None] - level[None, :])
    i, j = np.nonzero(np.triu(touch & (dim >= 1) & (gap >= 2), 1))
    return list(zip(i.tolist(), j.tolist()))


def random_tree(seed, base=(2, 2, 2), L=3, rounds=3, p=0.3):
    rng = np.random.default_rng(seed)
    b = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])])
    level = np.zeros(len(b), np.int64)
    anchor = b * (1 << L)
    for _ in range(rounds):
        marks = rng.random(len(level)) < p
        level, anchor, _ = amr.refine(level, anchor, L, marks)
    return level, anchor, L


@pytest.mark.parametrize("seed", range(6))
def test_incompatibility_detection_matches_brute_force(seed):
    level, anchor, L = random_tree(seed)
    f, c = amr.incompatible_pairs(level, anchor, L)
    got = {tuple(sorted(p)) for p in zip(f.tolist(), c.tolist())}
    want = {tuple(sorted(p)) for p in brute_incompatible(level, anchor, L)}
    assert got == want


def family_parent(level, anchor, L):
    """(level - 1, parent anchor) of every leaf of level >= 1."""
    ps = (1 << (L - (level - 1))).astype(np.int64)
    pa = (anchor // ps[:, None]) * ps[:, None]
    return [(int(l) - 1, *map(int, a)) for l, a in zip(level, pa)]


def covered_by_original(key, level0, anchor0, L):
    """True if an original leaf contains the box of node `key` (level, anchor)."""
    l, *a = key
    a = np.array(a, np.int64)
    s0 = (1 << (L - level0)).astype(np.int64)
    return bool(np.any((level0 <= l) & (anchor0 <= a).all(1) & (a < anchor0 + s0[:, None]).all(1)))


@pytest.mark.parametrize("seed", range(6))
def test_balance_is_minimal_closure(seed):
    """Sec. 6 closure: the balanced refinement is the smallest one.  Brute
    force: every complete family of leaves that the closure created (its
    parent lies inside an original leaf) is put back as its parent, one at a
    time; each such undo must bring back a level-two incompatibility.  An
    over-refining closure (refining the fine partner, refining across corners,
    one level too many) leaves a family whose undo stays compatible."""
    level, anchor, L = random_tree(seed)
    l2, a2, src = amr.balance(level, anchor, L)
    assert brute_incompatible(l2, a2, L) == []
    # leaves tile the domain
    s = (1 << (L - l2)).astype(np.int64)
    assert np.sum(s ** 3) == 8 * (1 << L) ** 3
    keys = family_parent(l2, a2, L)
    fams = {}
    for i, k in enumerate(keys):
        if l2[i] > 0:
            fams.setdefault(k, []).append(i)
    checked = 0
    for k, members in fams.items():
        if len(members) != 8 or not covered_by_original(k, level, anchor, L):
            continue
        keep = np.ones(len(l2), bool)
        keep[members] = False
        lu = np.concatenate([l2[keep], [k[0]]])
        au = np.concatenate([a2[keep], [k[1:]]])
        assert brute_incompatible(lu, au, L) != [], f"closure family {k} was not needed"
        checked += 1
    assert checked >= (0 if len(l2) == len(level) else 1)


def test_balance_minimality_check_catches_over_refinement():
    """The minimality check above fails for a closure that refines one leaf too
    many (planted on the oracle's output, on the CPU)."""
    level, anchor, L = random_tree(2)
    l2, a2, _ = amr.balance(level, anchor, L)
    # refine one original coarse leaf that the closure left alone and whose
    # children stay compatible
    for i in np.nonzero(l2 < L)[0]:
        m = np.zeros(len(l2), bool)
        m[i] = True
        l3, a3, _ = amr.refine(l2, a2, L, m)
        if brute_incompatible(l3, a3, L) == []:
            break
    else:
        pytest.skip("no compatible over-refinement in this tree")
    k = family_parent(l3[-8:], a3[-8:], L)[0]
    keep = np.ones(len(l3), bool)
    keep[-8:] = False
    lu = np.concatenate([l3[keep], [k[0]]])
    au = np.concatenate([a3[keep], [k[1:]]])
    assert brute_incompatible(lu, au, L) == []   # the undo stays compatible: detected


def test_marking_rule():
    L = 1
    a = np.array([[i, j, 0] for j in range(4) for i in range(4)])
    level = np.ones(16, np.int64)
    rho = np.full(16, 0.1)
    rho[5] = 0.9                                  # solid at (1,1)
    m = amr.mark(level, a, L, rho, rho_s=0.5, r_amr=1.5)
    cen = a + 0.5
    for e in range(16):
        d = np.linalg.norm(cen[e] - cen[5])
        if e == 5:
            assert m[e] == 0                      # solid but already finest: no-op
        elif d <= 1.5:
            assert m[e] == 0                      # near solid, finest level
        else:
            assert m[e] == -1


def test_sweeps_and_adapt_preserve_volume_and_balance():
    level, anchor, L = random_tree(4, rounds=2, p=0.4)
    level, anchor, _ = amr.balance(level, anchor, L)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.0, 1.0, len(level)) ** 3
    V = (1 << (L - level)).astype(float) ** 3
    l2, a2, r2, cover = amr.adapt(level, anchor, L, rho)
    V2 = (1 << (L - l2)).astype(float) ** 3
    assert V2.sum() == V.sum()
    assert brute_incompatible(l2, a2, L) == []
    assert r2 @ V2 == pytest.approx(rho @ V, rel=1e-12)
    # every derefined family had all eight members marked for derefinement
    m = amr.mark(level, anchor, L, rho)
    for cv in cover:
        if len(cv) == 8:
            assert (m[cv] == -1).all()


def test_c2_band_refinement_runs_and_balances():
    case = synth.c2(base=(4, 2, 2), max_level=2)
    fld = case.extra["field"]
    b = np.array([[i, j, k] for k in range(2) for j in range(2) for i in range(4)]) * 4
    level, anchor = np.zeros(len(b), np.int64), b
    for _ in range(case.max_level):
        marks = synth.band_marks(fld, level, anchor, case.max_level)
        level, anchor, _ = amr.refine(level, anchor, case.max_level, marks)
    level, anchor, _ = amr.balance(level, anchor, case.max_level)
    assert brute_incompatible(level, anchor, case.max_level) == []
    m = om.build_mesh(level, anchor, case.max_level, case.dims)
    assert m.n_elems == len(level)


def two_level_leaves():
    """L = 2 over a 2x1x1 base: the left cell split into level-1 leaves (edge 2),
    its leaf at (2, 0, 0) split again into level-2 leaves (edge 1), the right
    cell left at level 0 (edge 4)."""
    L = 2
    level = np.zeros(2, np.int64)
    anchor = np.array([[0, 0, 0], [4, 0, 0]], np.int64)
    level, anchor, _ = amr.refine(level, anchor, L, np.array([True, False]))
    pick = (level == 1) & (anchor == [2, 0, 0]).all(1)
    level, anchor, _ = amr.refine(level, anchor, L, pick)
    return level, anchor, L


def test_marking_refines_coarse_leaves_near_solid():
    """Sec. 4 marking on a mesh with three levels: a coarse void leaf is marked
    for refinement when a solid centre lies within r_AMR of its centre and for
    derefinement otherwise; a coarse solid leaf is refined; level-0 voids and
    finest-level solids stay.  Distances are computed here by hand."""
    level, anchor, L = two_level_leaves()
    s = 1 << (L - level)
    cen = anchor + 0.5 * s[:, None]
    solid = int(np.nonzero((level == 2) & (anchor == [3, 0, 0]).all(1))[0][0])   # centre (3.5, .5, .5)
    rho = np.full(len(level), 0.1)
    rho[solid] = 0.8
    coarse_near = int(np.nonzero((level == 1) & (anchor == [0, 0, 0]).all(1))[0][0])  # centre (1, 1, 1)
    d2 = float(((cen[coarse_near] - cen[solid]) ** 2).sum())
    assert d2 == 2.5 ** 2 + 0.25 + 0.25                     # 6.75: |d| = 2.598
    m = amr.mark(level, anchor, L, rho, rho_s=0.5, r_amr=2.6)
    assert m[coarse_near] == +1                             # coarse void within r_AMR: refine
    m = amr.mark(level, anchor, L, rho, rho_s=0.5, r_amr=2.5)
    assert m[coarse_near] == -1                             # beyond r_AMR: derefine
    right = int(np.nonzero(level == 0)[0][0])               # level 0, centre (6, 2, 2)
    assert m[right] == 0                                    # void at level 0: cannot derefine
    assert m[solid] == 0                                    # solid at the finest level: stays
    rho2 = rho.copy()
    rho2[coarse_near] = 0.6                                 # a coarse solid leaf
    m = amr.mark(level, anchor, L, rho2, rho_s=0.5, r_amr=1.5)
    assert m[coarse_near] == +1
    # every mark against a direct evaluation of the rule
    for r_amr in (1.0, 1.5, 2.6, 3.0):
        m = amr.mark(level, anchor, L, rho, rho_s=0.5, r_amr=r_amr)
        for e in range(len(level)):
            near = rho[e] >= 0.5 or np.linalg.norm(cen[e] - cen[solid]) <= r_amr
            want = (+1 if level[e] < L else 0) if near else (-1 if level[e] > 0 else 0)
            assert m[e] == want, (r_amr, e)


def test_marking_distance_tie_is_inclusive():
    """A leaf whose centre lies exactly r_AMR from a solid centre is marked for
    refinement (the inclusive reading of 'within r_AMR').  Ties arise between
    leaves of one level (squared centre distances are integers times the edge
    squared); between a leaf and one a level finer the squared distance is a
    sum of three odd squares over 4 (3/4 modulo 2), which never equals r_AMR^2
    for r_AMR = 1.5.  Leaves of edge 2 at distance exactly 2 and 4 here."""
    L = 1
    a = np.array([[2 * i, 2 * j, 0] for j in range(3) for i in range(3)], np.int64)
    level = np.zeros(len(a), np.int64)
    rho = np.full(len(a), 0.1)
    rho[4] = 0.9                                            # centre leaf
    for r_amr, want_near in ((2.0, {1, 3, 5, 7}), (4.0, set(range(9)))):
        m = amr.mark(level, a, L, rho, rho_s=0.5, r_amr=r_amr)
        got = {e for e in range(9) if m[e] == 1} - {4}
        assert got == want_near - {4}, (r_amr, got)
    m = amr.mark(level, a, L, rho, rho_s=0.5, r_amr=np.nextafter(2.0, 0.0))
    assert {e for e in range(9) if m[e] == 1} == {4}


def sweep2_tree():
    """2x1x1 base cells of edge 8 (L = 3).  Both cells are split; the left
    cell's child P at (4, 0, 0) is split into a family F of edge-2 leaves; the
    right cell's child Q at (8, 0, 0) is split, and Q's child R at (8, 0, 0)
    is split into edge-1 leaves that touch F across the plane x = 8."""
    L = 3
    level = np.zeros(2, np.int64)
    anchor = np.array([[0, 0, 0], [8, 0, 0]], np.int64)
    level, anchor, _ = amr.refine(level, anchor, L, np.array([True, True]))
    for lev, at in ((1, ([4, 0, 0], [8, 0, 0])), (2, ([8, 0, 0],))):
        pick = (level == lev) & np.any([(anchor == a).all(1) for a in at], axis=0)
        level, anchor, _ = amr.refine(level, anchor, L, pick)
    return level, anchor, L


def test_sweep2_drops_a_complete_family():
    """Sec. 4 sweep 2: every leaf is void except the edge-1 leaves of R, so
    sweep 1 keeps exactly one derefinement (the complete family F); putting F
    back as its parent P (edge 4) would leave P next to edge-1 leaves, a
    level-two incompatibility, so sweep 2 must drop it and the adaptation
    changes nothing."""
    level, anchor, L = sweep2_tree()
    assert brute_incompatible(level, anchor, L) == []
    fine = level == 3
    assert fine.sum() == 8
    rho = np.where(fine, 1.0, 0.1)
    m = amr.mark(level, anchor, L, rho)
    d1 = amr.sweep_families(level, anchor, L, m == -1)
    fam = (level == 2) & (anchor[:, 0] >= 4) & (anchor[:, 0] < 8)
    assert fam.sum() == 8 and (d1 == fam).all()             # sweep 1 keeps F only
    l2, a2, _ = amr.coarsen(level, anchor, L, d1)
    assert brute_incompatible(l2, a2, L) != []              # without sweep 2: incompatible
    nl, na, nrho, cover = amr.adapt(level, anchor, L, rho)
    assert {(int(l), *map(int, a)) for l, a in zip(nl, na)} == {(int(l), *map(int, a)) for l, a in zip(level, anchor)}
    assert all(len(cv) == 1 for cv in cover)


def linear_field(coords, A, b):
    return (coords.astype(np.float64) @ A.T + b).ravel()


def test_transfer_reproduces_linear_fields():
    """The transferred displacement is the old trilinear field evaluated at the
    new nodes; a linear field lies in every mesh's space, so after an
    adaptation that both refines and derefines (hanging nodes on both meshes)
    it must come out exactly (to rounding) at every new node.  Catches wrong
    shape-function weights, node order, leaf edge or anchor."""
    rng = np.random.default_rng(4)
    level, anchor, L = random_tree(7, rounds=2, p=0.4)
    level, anchor, _ = amr.balance(level, anchor, L)
    dims = (2 << L, 2 << L, 2 << L)
    m_old = om.build_mesh(level, anchor, L, dims)
    assert m_old.hanging.any()
    A, b = rng.normal(size=(3, 3)), rng.normal(size=3)
    u_old = linear_field(m_old.coords, A, b)
    cen = anchor + 0.5 * (1 << (L - level))[:, None]
    rho = np.where(cen[:, 0] < 3.0, 0.9, 0.05)              # solid slab at x < 3, void elsewhere
    nl, na, _, cover = amr.adapt(level, anchor, L, rho)
    n_deref = sum(len(cv) == 8 for cv in cover)
    n_ref = sum(1 for l, cv in zip(nl, cover) if len(cv) == 1 and l > level[cv[0]])
    assert n_deref > 0 and n_ref > 0
    m_new = om.build_mesh(nl, na, L, dims)
    assert m_new.hanging.any()
    got = amr.transfer_displacement(m_old, u_old, m_new.coords)
    want = linear_field(m_new.coords, A, b)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def brute_eval(level, anchor, L, coords, elem_nodes, u, pts):
    """Finite-element field at points: the leaf is found by testing every leaf's
    closed box, the value by trilinear interpolation of its eight vertices."""
    s = (1 << (L - np.asarray(level))).astype(np.float64)
    U = u.reshape(-1, 3)
    out = np.zeros((len(pts), 3))
    for i, p in enumerate(pts):
        inside = ((p >= anchor) & (p <= anchor + s[:, None])).all(1)
        e = int(np.nonzero(inside)[0][0])
        t = (p - anchor[e]) / s[e]
        w = np.array([(t[0] if a & 1 else 1 - t[0]) * (t[1] if a & 2 else 1 - t[1]) * (t[2] if a & 4 else 1 - t[2])
                      for a in range(8)])
        out[i] = w @ U[elem_nodes[e]]
    return out


def test_transfer_keeps_the_field_under_refinement():
    """Refinement nests the finite-element spaces, so the field rebuilt from the
    transferred nodal values must equal the old field everywhere.  The old
    field is a random continuous one (hanging values interpolated from their
    masters); both fields are evaluated at random points by a brute-force leaf
    search.  Catches a transfer that picks a leaf not containing the node."""
    from oracle import system as osys
    rng = np.random.default_rng(5)
    level, anchor, L = random_tree(3, rounds=2, p=0.35)
    level, anchor, _ = amr.balance(level, anchor, L)
    dims = (2 << L, 2 << L, 2 << L)
    m_old = om.build_mesh(level, anchor, L, dims)
    ut = rng.normal(size=3 * m_old.n_nodes)
    u_old = osys.dof_interp(m_old) @ np.where(np.repeat(m_old.hanging, 3), 0.0, ut)
    marks = rng.random(len(level)) < 0.3
    nl, na, _ = amr.refine(level, anchor, L, marks)
    nl, na, _ = amr.balance(nl, na, L)
    m_new = om.build_mesh(nl, na, L, dims)
    u_new = amr.transfer_displacement(m_old, u_old, m_new.coords)
    pts = rng.uniform(0, dims[0], size=(300, 3))
    pts[:40] = m_new.coords[rng.choice(m_new.n_nodes, 40)]      # nodes too (faces, edges)
    old = brute_eval(m_old.level, m_old.anchor, L, m_old.coords, m_old.elem_nodes, u_old, pts)
    new = brute_eval(m_new.level, m_new.anchor, L, m_new.coords, m_new.elem_nodes, u_new, pts)
    assert np.abs(old - new).max() <= 1e-12 * np.abs(old).max()
