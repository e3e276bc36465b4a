"""Octree leaves -> finite-element mesh: nodes, connectivity, hanging-node
interpolation P (paper Sec. 6, Eq. (6)), supports and consistent loads.

Leaves are given as ``level`` (n,) and ``anchor`` (n, 3) on the finest integer
lattice of a tree with ``max_level`` levels: a leaf of level l has edge
2**(max_level - l).  A uniform brick is the special case max_level = 0.

Hanging nodes are found from geometry alone: a node is hanging when it lies in
the closed box of some leaf without being one of that leaf's eight vertices.
Its interpolation weights are that leaf's trilinear shape functions evaluated
at the node (the paper's "linear interpolation from unconstrained DOFs"); when
a master is itself hanging it is replaced by its own masters until every
master is unconstrained.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .element import shape_values

_B = 18  # bits per coordinate in a packed key


def pack(level, ax, ay, az):
    level = np.asarray(level, dtype=np.int64)
    return (((level << _B | np.asarray(az, np.int64)) << _B | np.asarray(ay, np.int64)) << _B
            | np.asarray(ax, np.int64))


def pack_point(p):
    p = np.asarray(p, dtype=np.int64)
    return ((p[..., 2] << _B) | p[..., 1]) << _B | p[..., 0]


def uniform_leaves(dims):
    nx, ny, nz = dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    anchor = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.int64)
    return np.zeros(len(anchor), dtype=np.int64), anchor, 0


def leaf_sizes(level, max_level):
    return (np.int64(1) << (max_level - np.asarray(level, dtype=np.int64)))


class LeafIndex:
    """Find the leaf containing a (non-lattice) point by trying every level."""

    def __init__(self, level, anchor, max_level):
        self.level = np.asarray(level, dtype=np.int64)
        self.anchor = np.asarray(anchor, dtype=np.int64)
        self.L = int(max_level)
        keys = pack(self.level, *self.anchor.T)
        self.order = np.argsort(keys)
        self.keys = keys[self.order]

    def find(self, pts):
        """pts (m, 3) float strictly inside leaves -> leaf index (m,), -1 if outside."""
        pts = np.asarray(pts, dtype=np.float64)
        out = np.full(len(pts), -1, dtype=np.int64)
        for lev in range(self.L + 1):
            s = 1 << (self.L - lev)
            a = (np.floor(pts / s).astype(np.int64)) * s
            ok = (a >= 0).all(axis=1)
            k = pack(np.full(len(pts), lev), a[:, 0].clip(0), a[:, 1].clip(0), a[:, 2].clip(0))
            pos = np.searchsorted(self.keys, k)
            pos = np.minimum(pos, len(self.keys) - 1)
            hit = ok & (self.keys[pos] == k) & (out < 0)
            out[hit] = self.order[pos[hit]]
        return out


@dataclass
class Mesh:
    level: np.ndarray        # (ne,)
    anchor: np.ndarray       # (ne, 3)
    max_level: int
    dims: tuple              # finest-lattice extents
    coords: np.ndarray       # (nn, 3) int64 lattice coordinates, sorted z, y, x
    elem_nodes: np.ndarray   # (ne, 8) local order i + 2j + 4k
    size: np.ndarray         # (ne,) element edge length h_e
    hanging: np.ndarray      # (nn,) bool
    Tn: sp.csr_matrix        # (nn, nn) node interpolation: u = Tn @ u_unconstrained

    @property
    def n_nodes(self):
        return len(self.coords)

    @property
    def n_elems(self):
        return len(self.level)

    @property
    def volumes(self):
        return self.size.astype(np.float64) ** 3

    @property
    def centres(self):
        return self.anchor + 0.5 * self.size[:, None]


def build_mesh(level, anchor, max_level, dims) -> Mesh:
    level = np.asarray(level, dtype=np.int64)
    anchor = np.asarray(anchor, dtype=np.int64)
    size = leaf_sizes(level, max_level)
    loc = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)
    verts = anchor[:, None, :] + size[:, None, None] * loc[None]          # (ne, 8, 3)
    # node numbering: lexicographic with x fastest (sort on z, then y, then x)
    vk = pack_point(verts.reshape(-1, 3))
    uk, inv = np.unique(vk, return_inverse=True)
    mask = (1 << _B) - 1
    coords = np.stack([uk & mask, (uk >> _B) & mask, (uk >> (2 * _B)) & mask], axis=1)
    elem_nodes = inv.reshape(-1, 8).astype(np.int64)

    # hanging detection from geometry: probe the eight octants around each node
    idx = LeafIndex(level, anchor, max_level)
    nn = len(coords)
    octs = np.array([[sx, sy, sz] for sz in (-0.5, 0.5) for sy in (-0.5, 0.5) for sx in (-0.5, 0.5)])
    masters = {}
    for o in octs:
        q = coords + o
        leaf = idx.find(q)
        have = leaf >= 0
        nodes_h = np.nonzero(have)[0]
        L = leaf[have]
        s = size[L]
        rel = coords[nodes_h] - anchor[L]
        is_vertex = ((rel == 0) | (rel == s[:, None])).all(axis=1)
        for n, l, r, sz in zip(nodes_h[~is_vertex], L[~is_vertex], rel[~is_vertex], s[~is_vertex]):
            w = shape_values(r / float(sz))
            ent = {int(elem_nodes[l, a]): float(w[a]) for a in range(8) if abs(w[a]) > 0.0}
            prev = masters.get(int(n))
            if prev is None:
                masters[int(n)] = ent
            else:
                # the same node seen from two leaves must interpolate identically
                # on the shared boundary (continuity of the coarse field)
                assert set(prev) == set(ent) and all(abs(prev[k] - ent[k]) < 1e-14 for k in ent), \
                    f"inconsistent hanging interpolation at node {n}"
    hanging = np.zeros(nn, dtype=bool)
    hanging[list(masters.keys())] = True
    # transitive closure: replace hanging masters by their own masters
    changed = True
    while changed:
        changed = False
        for h, ent in masters.items():
            if any(hanging[m] for m in ent):
                new = {}
                for m, w in ent.items():
                    if hanging[m]:
                        for m2, w2 in masters[m].items():
                            new[m2] = new.get(m2, 0.0) + w * w2
                    else:
                        new[m] = new.get(m, 0.0) + w
                masters[h] = new
                changed = True
    rows, cols, vals = [], [], []
    free_nodes = np.nonzero(~hanging)[0]
    rows.extend(free_nodes.tolist())
    cols.extend(free_nodes.tolist())
    vals.extend([1.0] * len(free_nodes))
    for h, ent in masters.items():
        for m, w in ent.items():
            rows.append(h)
            cols.append(m)
            vals.append(w)
    Tn = sp.csr_matrix((vals, (rows, cols)), shape=(nn, nn))
    return Mesh(level, anchor, int(max_level), tuple(dims), coords, elem_nodes, size, hanging, Tn)


def uniform_mesh(dims) -> Mesh:
    lv, an, L = uniform_leaves(dims)
    return build_mesh(lv, an, L, dims)


# ---------------------------------------------------------------- supports
def _where_mask(coords, where):
    axes = {"x": 0, "y": 1, "z": 2}
    m = np.ones(len(coords), dtype=bool)
    for k, v in where.items():
        m &= coords[:, axes[k]] == v
    return m


def fixed_dofs(mesh: Mesh, fixed_spec) -> np.ndarray:
    """(3 nn,) bool: every DOF of every node on a listed plane/line is fixed."""
    node = np.zeros(mesh.n_nodes, dtype=bool)
    for w in fixed_spec:
        node |= _where_mask(mesh.coords, w)
    return np.repeat(node, 3)


# ---------------------------------------------------------------- loads
def load_vector(mesh: Mesh, spec) -> np.ndarray:
    """Consistent nodal loads (3 nn,) on all nodes (hanging ones included).

    "line": each leaf edge lying on the line carries length/2 at each end;
    "face": each leaf face lying in the plane carries area/4 at each corner.
    The result is scaled so that its sum equals ``spec["total"]``."""
    axes = {"x": 0, "y": 1, "z": 2}
    where = {axes[k]: v for k, v in spec["where"].items()}
    f = np.zeros(mesh.n_nodes)
    key_of = {tuple(c): i for i, c in enumerate(mesh.coords.tolist())}
    seen = set()
    total = 0.0
    for e in range(mesh.n_elems):
        a = mesh.anchor[e]
        s = int(mesh.size[e])
        loc = [(i, j, k) for k in (0, 1) for j in (0, 1) for i in (0, 1)]
        corners = [tuple(int(a[d] + s * off[d]) for d in range(3)) for off in loc]
        on = [c for c in corners if all(c[ax] == v for ax, v in where.items())]
        if spec["kind"] == "line" and len(on) == 2:
            seg = tuple(sorted(on))
            if seg in seen:
                continue
            seen.add(seg)
            for c in on:
                f[key_of[c]] += 0.5 * s
            total += s
        elif spec["kind"] == "face" and len(on) == 4:
            face = tuple(sorted(on))
            if face in seen:
                continue
            seen.add(face)
            for c in on:
                f[key_of[c]] += 0.25 * s * s
            total += s * s
    out = np.zeros(3 * mesh.n_nodes)
    out[spec["comp"]::3] = f * (spec["total"] / total)
    return out
