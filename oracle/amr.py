"""Octree adaptation, written from the rule text of paper Sec. 4 and Sec. 6.

Leaves: ``level`` (n,), ``anchor`` (n, 3) on the finest lattice, ``max_level``.

* Level-one compatibility (Sec. 6, Fig. 3): two leaves whose closed boxes share
  a segment (a face or an edge) differ by at most one level.  It is checked
  segment by segment: every unit lattice segment on an edge of a leaf is looked
  up in the leaves whose closed boxes contain it.
* Closure (Sec. 6): coarse ("gray") leaves next to leaves two or more levels
  finer are refined until no such pair remains.
* Marking (Sec. 4): a leaf is solid if rho >= rho_s; it is marked for
  refinement if it is solid or some solid leaf's centre lies within r_amr of
  its centre, otherwise for derefinement.
* Sweep 1 (Sec. 4): a derefinement is dropped unless all eight siblings are
  leaves marked for derefinement.
* Sweep 2 (Sec. 4): a derefinement is dropped if the mesh that would result
  has a level-two (or worse) incompatibility at the new parent.
* Field transfer (not described in the paper): children inherit their parent's
  density, a derefined parent gets the mean of its children (volume is kept),
  and displacements are the old finite-element field evaluated at new nodes.
"""
from __future__ import annotations

import numpy as np

from .element import shape_values
from .mesh import LeafIndex, leaf_sizes

_CHILD = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=np.int64)


def refine(level, anchor, max_level, marks):
    """Split every marked leaf (below max_level) into its eight children.
    Returns new (level, anchor, parent_index) with parent_index mapping each new
    leaf to the old leaf it came from."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    marks = np.asarray(marks, bool) & (level < max_level)
    keep = np.nonzero(~marks)[0]
    split = np.nonzero(marks)[0]
    half = leaf_sizes(level[split] + 1, max_level)
    ch_anchor = (anchor[split][:, None, :] + half[:, None, None] * _CHILD[None]).reshape(-1, 3)
    ch_level = np.repeat(level[split] + 1, 8)
    new_level = np.concatenate([level[keep], ch_level])
    new_anchor = np.concatenate([anchor[keep], ch_anchor])
    src = np.concatenate([keep, np.repeat(split, 8)])
    return new_level, new_anchor, src


def _edge_segments(level, anchor, max_level):
    """Midpoints of all unit segments on the 12 edges of each leaf: (m, 3)
    float midpoints, the axis of each segment, and the owning leaf."""
    s = leaf_sizes(level, max_level)
    mids, axes, owner = [], [], []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        for c1 in (0, 1):
            for c2 in (0, 1):
                for e in np.unique(s):
                    sel = np.nonzero(s == e)[0]
                    t = np.arange(e) + 0.5
                    base = anchor[sel].astype(np.float64)
                    pts = np.repeat(base[:, None, :], e, axis=1)
                    pts[:, :, ax] += t[None, :]
                    pts[:, :, o1] += c1 * e
                    pts[:, :, o2] += c2 * e
                    mids.append(pts.reshape(-1, 3))
                    axes.append(np.full(len(sel) * e, ax))
                    owner.append(np.repeat(sel, e))
    return np.concatenate(mids), np.concatenate(axes), np.concatenate(owner)


def incompatible_pairs(level, anchor, max_level):
    """(fine, coarse) leaf index pairs sharing a segment with level gap >= 2."""
    level = np.asarray(level, np.int64)
    idx = LeafIndex(level, anchor, max_level)
    mids, axes, owner = _edge_segments(level, anchor, max_level)
    fine_list, coarse_list = [], []
    for ax in range(3):
        sel = axes == ax
        m, ow = mids[sel], owner[sel]
        o1, o2 = [a for a in range(3) if a != ax]
        for d1 in (-0.5, 0.5):
            for d2 in (-0.5, 0.5):
                q = m.copy()
                q[:, o1] += d1
                q[:, o2] += d2
                lf = idx.find(q)
                ok = lf >= 0
                gap = level[ow[ok]] - level[lf[ok]]
                bad = gap >= 2
                fine_list.append(ow[ok][bad])
                coarse_list.append(lf[ok][bad])
    f = np.concatenate(fine_list) if fine_list else np.zeros(0, np.int64)
    c = np.concatenate(coarse_list) if coarse_list else np.zeros(0, np.int64)
    return f, c


def is_balanced(level, anchor, max_level) -> bool:
    f, _ = incompatible_pairs(level, anchor, max_level)
    return len(f) == 0


def balance(level, anchor, max_level, src=None):
    """Refinement closure: refine coarse partners of incompatible pairs until none."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    src = np.arange(len(level)) if src is None else np.asarray(src)
    while True:
        _, coarse = incompatible_pairs(level, anchor, max_level)
        if len(coarse) == 0:
            return level, anchor, src
        marks = np.zeros(len(level), bool)
        marks[coarse] = True
        level, anchor, s2 = refine(level, anchor, max_level, marks)
        src = src[s2]


def mark(level, anchor, max_level, rho, rho_s=0.5, r_amr=1.5):
    """+1 refine, -1 derefine (Sec. 4 marking); brute force over solid leaves."""
    level = np.asarray(level, np.int64)
    s = leaf_sizes(level, max_level).astype(np.float64)
    cen = anchor + 0.5 * s[:, None]
    solid = np.asarray(rho) >= rho_s
    near = solid.copy()
    sc = cen[solid]
    if len(sc):
        r2 = r_amr * r_amr
        for i in range(0, len(cen), 4096):
            d2 = ((cen[i:i + 4096, None, :] - sc[None]) ** 2).sum(-1)
            near[i:i + 4096] |= (d2 <= r2).any(axis=1)
    out = np.where(near, 1, -1)
    out[(out == 1) & (level >= max_level)] = 0
    out[(out == -1) & (level == 0)] = 0
    return out


def _parent_key(level, anchor, max_level):
    ps = leaf_sizes(level - 1, max_level)
    pa = (anchor // ps[:, None]) * ps[:, None]
    return [(int(l) - 1, int(a[0]), int(a[1]), int(a[2])) for l, a in zip(level, pa)]


def sweep_families(level, anchor, max_level, dmarks):
    """Sweep 1: keep a derefinement only if all 8 siblings are leaves marked."""
    level = np.asarray(level, np.int64)
    dmarks = np.asarray(dmarks, bool) & (level > 0)
    keys = _parent_key(level, anchor, max_level)
    count = {}
    for i in np.nonzero(dmarks)[0]:
        count[keys[i]] = count.get(keys[i], 0) + 1
    out = dmarks.copy()
    for i in np.nonzero(dmarks)[0]:
        if count[keys[i]] != 8:
            out[i] = False
    return out


def coarsen(level, anchor, max_level, dmarks):
    """Replace every complete marked family by its parent.  Returns new leaves,
    and for each new leaf the list of old leaves it covers."""
    level = np.asarray(level, np.int64)
    keys = _parent_key(level, anchor, max_level)
    fam = {}
    for i in np.nonzero(dmarks)[0]:
        fam.setdefault(keys[i], []).append(int(i))
    keep = np.nonzero(~np.asarray(dmarks, bool))[0]
    nl = list(level[keep])
    na = [tuple(a) for a in anchor[keep]]
    cover = [[int(i)] for i in keep]
    for (l, ax, ay, az), members in fam.items():
        assert len(members) == 8
        nl.append(l)
        na.append((ax, ay, az))
        cover.append(members)
    return np.array(nl, np.int64), np.array(na, np.int64).reshape(-1, 3), cover


def adapt(level, anchor, max_level, rho, rho_s=0.5, r_amr=1.5):
    """One adaptation: mark, sweep 1, refine + closure, sweep 2, derefine.

    Returns (level, anchor, rho_new, cover) where cover[i] lists the old leaves
    whose union or parent is new leaf i (for transfers)."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    rho = np.asarray(rho, np.float64)
    m = mark(level, anchor, max_level, rho, rho_s, r_amr)
    dmark = sweep_families(level, anchor, max_level, m == -1)
    # refinement of the marked leaves, then closure
    l1, a1, src = refine(level, anchor, max_level, m == 1)
    l1, a1, src = balance(l1, a1, max_level, src)
    # derefinement candidates that are still untouched leaves after closure
    unsplit = np.bincount(src, minlength=len(level)) == 1
    d1 = dmark[src] & unsplit[src]
    d1 = sweep_families(l1, a1, max_level, d1)
    # sweep 2: drop families whose parent would be level-two incompatible
    while True:
        l2, a2, cover = coarsen(l1, a1, max_level, d1)
        f, c = incompatible_pairs(l2, a2, max_level)
        is_parent = np.array([len(cv) == 8 for cv in cover])
        bad = set()
        for x in np.concatenate([f, c]):
            if is_parent[x]:
                bad.update(cover[x])
        if not bad:
            break
        d1 = d1.copy()
        d1[list(bad)] = False
    cover_old = [[int(src[i]) for i in cv] for cv in cover]
    new_rho = np.array([rho[cv].mean() if len(cv) == 8 else rho[cv[0]] for cv in cover_old])
    # a refined leaf's children all map to that same old leaf: mean = inherit
    return l2, a2, new_rho, cover_old


def transfer_displacement(old_mesh, u_old, new_coords):
    """Evaluate the old trilinear field (all nodes, hanging recovered) at new nodes."""
    idx = LeafIndex(old_mesh.level, old_mesh.anchor, old_mesh.max_level)
    pts = new_coords.astype(np.float64)
    dims = np.asarray(old_mesh.dims)
    # a point a quarter cell away (towards the interior) lies in a leaf whose
    # closed box contains the node
    probe = np.where(pts >= dims, pts - 0.25, pts + 0.25)
    leaf = idx.find(probe)
    assert (leaf >= 0).all()
    out = np.zeros((len(pts), 3))
    U = u_old.reshape(-1, 3)
    for i, (p, l) in enumerate(zip(pts, leaf)):
        s = float(old_mesh.size[l])
        w = shape_values((p - old_mesh.anchor[l]) / s)
        out[i] = w @ U[old_mesh.elem_nodes[l]]
    return out.ravel()
