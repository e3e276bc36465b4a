"""The 2-D variant of the method (paper Sec. 6 and 7, Test 1: a 2-D cantilever on
a quadtree mesh refined and derefined during the optimisation).

Test infrastructure: a plain FP64 CPU statement of every step, used only by
the tests to judge the library.

* Element (Sec. 3 in 2-D): bilinear Q4 on squares, plane stress with unit
  thickness.  K0 is the unit square's matrix (E = 1), 2x2 Gauss (exact);
  an element of edge h has the same matrix (stiffness of a square is
  size-free in 2-D), so K_e = E(rho_e) K0 with E = Emin + rho^p (E0 - Emin).
  Local node a = i + 2 j at (i, j); local DOF 2 a + c.
* Mesh (Sec. 6, Eq. (6)): nodes are leaf corners on the finest lattice; a node
  strictly inside an edge of a leaf of which it is not a corner hangs, with the
  bilinear shape functions of that leaf as weights (1/2, 1/2 on the edge);
  chains are resolved so masters are never hanging.
* Constrained operator A~ = F T^T K T F + (I - F) (Eq. (7)-(8)); supported DOFs
  are identity rows with zero right-hand side.
* Compliance, sensitivity dc_e = -p rho^(p-1) (E0 - Emin) u_e^T K0 u_e, the
  Eq. (5) filter with V_d = h_d^2 (areas), OC as in 3-D.
* Quadtree adaptation (Sec. 4, Sec. 6): level-one compatibility across edges
  (leaves sharing an edge segment differ by at most one level; corner
  contact is unconstrained); marking, sweep 1 over families of four siblings,
  refinement and closure, sweep 2, derefinement; densities transfer as in
  3-D (children inherit, parents average).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import cKDTree

_LOC = np.array([[a & 1, (a >> 1) & 1] for a in range(4)], dtype=np.int64)
_B = 24


# ---------------------------------------------------------------- element
def plane_stress(E=1.0, nu=0.3):
    return E / (1.0 - nu * nu) * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]])


def shape_values(xi):
    return np.array([(xi[0] if i else 1 - xi[0]) * (xi[1] if j else 1 - xi[1]) for i, j in _LOC])


def shape_grad(xi):
    g = np.zeros((4, 2))
    for a, (i, j) in enumerate(_LOC):
        fx, fy = (xi[0] if i else 1 - xi[0]), (xi[1] if j else 1 - xi[1])
        g[a] = ((1.0 if i else -1.0) * fy, fx * (1.0 if j else -1.0))
    return g


def k0(nu=0.3, E=1.0):
    """Unit-square Q4 plane-stress matrix (8 x 8) by 2x2 Gauss."""
    D = plane_stress(E, nu)
    x, w = np.polynomial.legendre.leggauss(2)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    K = np.zeros((8, 8))
    for i in range(2):
        for j in range(2):
            g = shape_grad(np.array([x[i], x[j]]))
            B = np.zeros((3, 8))
            B[0, 0::2] = g[:, 0]
            B[1, 1::2] = g[:, 1]
            B[2, 0::2] = g[:, 1]
            B[2, 1::2] = g[:, 0]
            K += B.T @ D @ B * (w[i] * w[j])
    return 0.5 * (K + K.T)


def rigid_modes():
    """(8, 3): two translations and the infinitesimal rotation (-y, x)."""
    X = _LOC.astype(np.float64) - 0.5
    R = np.zeros((8, 3))
    R[0::2, 0] = 1.0
    R[1::2, 1] = 1.0
    R[0::2, 2] = -X[:, 1]
    R[1::2, 2] = X[:, 0]
    return R


# ---------------------------------------------------------------- mesh
def leaf_sizes(level, max_level):
    return np.int64(1) << (max_level - np.asarray(level, dtype=np.int64))


def uniform_leaves(dims):
    nx, ny = dims
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.zeros(nx * ny, np.int64), np.stack([ix.ravel(), iy.ravel()], 1).astype(np.int64), 0


def base_leaves(base, max_level):
    bx, by = base
    iy, ix = np.meshgrid(np.arange(by), np.arange(bx), indexing="ij")
    return np.zeros(bx * by, np.int64), np.stack([ix.ravel(), iy.ravel()], 1).astype(np.int64) << max_level


class LeafIndex:
    """The leaf containing a (non-lattice) point, by trying every level."""

    def __init__(self, level, anchor, max_level):
        self.level = np.asarray(level, np.int64)
        self.anchor = np.asarray(anchor, np.int64)
        self.L = int(max_level)
        self.map = {(int(l), int(a[0]), int(a[1])): i for i, (l, a) in enumerate(zip(self.level, self.anchor))}

    def find(self, pts):
        out = np.full(len(pts), -1, np.int64)
        for k, p in enumerate(np.asarray(pts, np.float64)):
            for lev in range(self.L + 1):
                s = 1 << (self.L - lev)
                a = np.floor(p / s).astype(np.int64) * s
                i = self.map.get((lev, int(a[0]), int(a[1])))
                if i is not None:
                    out[k] = i
                    break
        return out


@dataclass
class Mesh:
    level: np.ndarray
    anchor: np.ndarray      # (ne, 2)
    max_level: int
    dims: tuple
    coords: np.ndarray      # (nn, 2) sorted y, then x
    elem_nodes: np.ndarray  # (ne, 4), local a = i + 2 j
    size: np.ndarray
    hanging: np.ndarray
    Tn: sp.csr_matrix

    @property
    def n_nodes(self):
        return len(self.coords)

    @property
    def n_elems(self):
        return len(self.level)

    @property
    def areas(self):
        return self.size.astype(np.float64) ** 2

    @property
    def centres(self):
        return self.anchor + 0.5 * self.size[:, None]


def build_mesh(level, anchor, max_level, dims) -> Mesh:
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    size = leaf_sizes(level, max_level)
    verts = anchor[:, None, :] + size[:, None, None] * _LOC[None]
    vk = (verts[..., 1] << _B) | verts[..., 0]
    uk, inv = np.unique(vk.ravel(), return_inverse=True)
    coords = np.stack([uk & ((1 << _B) - 1), uk >> _B], 1)
    elem_nodes = inv.reshape(-1, 4).astype(np.int64)
    idx = LeafIndex(level, anchor, max_level)
    masters = {}
    for o in ((-0.5, -0.5), (0.5, -0.5), (-0.5, 0.5), (0.5, 0.5)):
        leaf = idx.find(coords + np.array(o))
        for n in np.nonzero(leaf >= 0)[0]:
            l = leaf[n]
            rel = coords[n] - anchor[l]
            s = size[l]
            if ((rel == 0) | (rel == s)).all():
                continue
            w = shape_values(rel / float(s))
            ent = {int(elem_nodes[l, a]): float(w[a]) for a in range(4) if w[a] != 0.0}
            prev = masters.get(int(n))
            assert prev is None or prev == ent, f"inconsistent hanging interpolation at node {n}"
            masters[int(n)] = ent
    hanging = np.zeros(len(coords), bool)
    hanging[list(masters)] = True
    changed = True
    while changed:
        changed = False
        for h, ent in list(masters.items()):
            if any(hanging[m] for m in ent):
                new = {}
                for m, w in ent.items():
                    for m2, w2 in (masters[m].items() if hanging[m] else [(m, 1.0)]):
                        new[m2] = new.get(m2, 0.0) + w * w2
                masters[h] = new
                changed = True
    rows, cols, vals = list(np.nonzero(~hanging)[0]), list(np.nonzero(~hanging)[0]), [1.0] * int((~hanging).sum())
    for h, ent in masters.items():
        for m, w in ent.items():
            rows.append(h)
            cols.append(m)
            vals.append(w)
    Tn = sp.csr_matrix((vals, (rows, cols)), shape=(len(coords), len(coords)))
    return Mesh(level, anchor, int(max_level), tuple(dims), coords, elem_nodes, size, hanging, Tn)


def fixed_dofs(mesh: Mesh, fixed_spec):
    """(2 nn,) bool: both DOFs of every node on a listed line or point."""
    node = np.zeros(mesh.n_nodes, bool)
    for w in fixed_spec:
        m = np.ones(mesh.n_nodes, bool)
        for k, v in w.items():
            m &= mesh.coords[:, {"x": 0, "y": 1}[k]] == v
        node |= m
    return np.repeat(node, 2)


def load_vector(mesh: Mesh, spec):
    """A point load of `total` on component `comp` at the node spec['at']."""
    f = np.zeros(2 * mesh.n_nodes)
    at = spec["at"]
    n = np.nonzero((mesh.coords[:, 0] == at[0]) & (mesh.coords[:, 1] == at[1]))[0]
    assert len(n) == 1
    f[2 * n[0] + spec["comp"]] = spec["total"]
    return f


# ---------------------------------------------------------------- system
def young(rho, E0=1.0, Emin=1e-9, p=3.0):
    return Emin + np.asarray(rho, np.float64) ** p * (E0 - Emin)


def elem_dofs(mesh: Mesh):
    return (2 * mesh.elem_nodes[:, :, None] + np.arange(2)[None, None, :]).reshape(-1, 8)


def assemble(mesh: Mesh, coeff, nu=0.3):
    K0 = k0(nu)
    d = elem_dofs(mesh)
    rows = np.repeat(d, 8, axis=1).ravel()
    cols = np.tile(d, (1, 8)).ravel()
    vals = (np.asarray(coeff, np.float64)[:, None, None] * K0[None]).ravel()
    n = 2 * mesh.n_nodes
    K = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    return K


@dataclass
class System:
    A: sp.csr_matrix
    b: np.ndarray
    T: sp.csr_matrix
    free: np.ndarray
    f: np.ndarray


def build_system(mesh: Mesh, coeff, fixed, f, nu=0.3) -> System:
    K = assemble(mesh, coeff, nu)
    T = sp.kron(mesh.Tn, sp.identity(2), format="csr")
    free = ~(np.repeat(mesh.hanging, 2) | fixed)
    F = sp.diags(free.astype(np.float64))
    A = (F @ (T.T @ (K @ (T @ F)))).tocsr() + sp.diags((~free).astype(np.float64))
    A = A.tocsr()
    A.sum_duplicates()
    return System(A, F @ (T.T @ f), T, free, f)


def apply_constrained(mesh: Mesh, coeff, fixed, x, nu=0.3):
    """A~ x by an element loop: mask, interpolate hanging values, K, condense, identity rows."""
    T = sp.kron(mesh.Tn, sp.identity(2), format="csr")
    free = ~(np.repeat(mesh.hanging, 2) | fixed)
    u = T @ np.where(free, x, 0.0)
    K0 = k0(nu)
    d = elem_dofs(mesh)
    ye = (u[d] @ K0.T) * np.asarray(coeff)[:, None]
    y = np.bincount(d.ravel(), weights=ye.ravel(), minlength=len(u))
    return np.where(free, T.T @ y, x)


def solve_direct(s: System):
    idx = np.nonzero(s.free)[0]
    ut = np.zeros(len(s.b))
    ut[idx] = spla.spsolve(s.A[idx][:, idx].tocsc(), s.b[idx])
    return s.T @ ut


def sensitivities(mesh: Mesh, rho, u, E0=1.0, Emin=1e-9, p=3.0, nu=0.3):
    ue = u[elem_dofs(mesh)]
    w = np.einsum("ei,ij,ej->e", ue, k0(nu), ue)
    return -p * np.asarray(rho, np.float64) ** (p - 1.0) * (E0 - Emin) * w


def filter_weights(mesh: Mesh, rmin):
    cen = mesh.centres
    tree = cKDTree(cen)
    pairs = tree.sparse_distance_matrix(tree, rmin, output_type="ndarray")
    i, j, dist = pairs["i"], pairs["j"], pairs["v"]
    keep = i != j
    n = mesh.n_elems
    i = np.concatenate([i[keep], np.arange(n)])
    j = np.concatenate([j[keep], np.arange(n)])
    dist = np.concatenate([dist[keep], np.zeros(n)])
    H = np.maximum(rmin - dist, 0.0)
    ok = H > 0
    return sp.csr_matrix((H[ok] * mesh.areas[j[ok]], (i[ok], j[ok])), shape=(n, n))


def filter_sensitivity(mesh: Mesh, rmin, rho, dc, rho_min=1e-3):
    W = filter_weights(mesh, rmin)
    return (W @ (np.asarray(rho) * np.asarray(dc))) / (np.maximum(rho, rho_min) * np.asarray(W.sum(1)).ravel())


# ---------------------------------------------------------------- quadtree adaptation
def refine(level, anchor, max_level, marks):
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    marks = np.asarray(marks, bool) & (level < max_level)
    keep, split = np.nonzero(~marks)[0], np.nonzero(marks)[0]
    half = leaf_sizes(level[split] + 1, max_level)
    ch = (anchor[split][:, None, :] + half[:, None, None] * _LOC[None]).reshape(-1, 2)
    return (np.concatenate([level[keep], np.repeat(level[split] + 1, 4)]), np.concatenate([anchor[keep], ch]),
            np.concatenate([keep, np.repeat(split, 4)]))


def incompatible_pairs(level, anchor, max_level):
    """(fine, coarse) leaves sharing an edge segment with a level gap >= 2: every
    unit segment on a leaf's edges is probed on both sides."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    idx = LeafIndex(level, anchor, max_level)
    s = leaf_sizes(level, max_level)
    fine, coarse = [], []
    for e in range(len(level)):
        a, h = anchor[e], int(s[e])
        for ax in (0, 1):
            o = 1 - ax
            for side in (0, h):
                for t in range(h):
                    mid = np.zeros(2)
                    mid[ax] = a[ax] + t + 0.5
                    mid[o] = a[o] + side
                    for d in (-0.5, 0.5):
                        q = mid.copy()
                        q[o] += d
                        l = idx.find([q])[0]
                        if l >= 0 and level[e] - level[l] >= 2:
                            fine.append(e)
                            coarse.append(int(l))
    return np.array(fine, np.int64), np.array(coarse, np.int64)


def is_balanced(level, anchor, max_level):
    return len(incompatible_pairs(level, anchor, max_level)[0]) == 0


def balance(level, anchor, max_level, src=None):
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    src = np.arange(len(level)) if src is None else np.asarray(src)
    while True:
        _, coarse = incompatible_pairs(level, anchor, max_level)
        if len(coarse) == 0:
            return level, anchor, src
        m = np.zeros(len(level), bool)
        m[coarse] = True
        level, anchor, s2 = refine(level, anchor, max_level, m)
        src = src[s2]


def mark(level, anchor, max_level, rho, rho_s=0.5, r_amr=1.5):
    """+1 refine (solid, or a solid centre within r_amr), -1 derefine, 0 capped."""
    level = np.asarray(level, np.int64)
    s = leaf_sizes(level, max_level).astype(np.float64)
    cen = anchor + 0.5 * s[:, None]
    solid = np.asarray(rho) >= rho_s
    near = solid.copy()
    if solid.any():
        d2 = ((cen[:, None, :] - cen[solid][None]) ** 2).sum(-1)
        near |= (d2 <= r_amr * r_amr).any(1)
    out = np.where(near, 1, -1)
    out[(out == 1) & (level >= max_level)] = 0
    out[(out == -1) & (level == 0)] = 0
    return out


def _parent(level, anchor, max_level):
    ps = leaf_sizes(level - 1, max_level)
    pa = (anchor // ps[:, None]) * ps[:, None]
    return [(int(l) - 1, int(a[0]), int(a[1])) for l, a in zip(level, pa)]


def sweep_families(level, anchor, max_level, dmarks):
    level = np.asarray(level, np.int64)
    dmarks = np.asarray(dmarks, bool) & (level > 0)
    keys = _parent(level, anchor, max_level)
    count = {}
    for i in np.nonzero(dmarks)[0]:
        count[keys[i]] = count.get(keys[i], 0) + 1
    out = dmarks.copy()
    for i in np.nonzero(dmarks)[0]:
        out[i] = count[keys[i]] == 4
    return out


def coarsen(level, anchor, max_level, dmarks):
    level = np.asarray(level, np.int64)
    keys = _parent(level, anchor, max_level)
    fam = {}
    for i in np.nonzero(dmarks)[0]:
        fam.setdefault(keys[i], []).append(int(i))
    keep = np.nonzero(~np.asarray(dmarks, bool))[0]
    nl, na, cover = list(level[keep]), [tuple(a) for a in anchor[keep]], [[int(i)] for i in keep]
    for (l, ax, ay), mem in fam.items():
        assert len(mem) == 4
        nl.append(l)
        na.append((ax, ay))
        cover.append(mem)
    return np.array(nl, np.int64), np.array(na, np.int64).reshape(-1, 2), cover


def adapt(level, anchor, max_level, rho, rho_s=0.5, r_amr=1.5):
    """Mark, sweep 1, refine + closure, sweep 2, derefine; (level, anchor, rho_new)."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    rho = np.asarray(rho, np.float64)
    m = mark(level, anchor, max_level, rho, rho_s, r_amr)
    dm = sweep_families(level, anchor, max_level, m == -1)
    l1, a1, src = refine(level, anchor, max_level, m == 1)
    l1, a1, src = balance(l1, a1, max_level, src)
    untouched = np.bincount(src, minlength=len(level)) == 1
    d1 = sweep_families(l1, a1, max_level, dm[src] & untouched[src])
    while True:
        l2, a2, cover = coarsen(l1, a1, max_level, d1)
        f, c = incompatible_pairs(l2, a2, max_level)
        parent = np.array([len(cv) == 4 for cv in cover])
        bad = set()
        for x in np.concatenate([f, c]):
            if parent[x]:
                bad.update(cover[x])
        if not bad:
            break
        d1 = d1.copy()
        d1[list(bad)] = False
    cover_old = [[int(src[i]) for i in cv] for cv in cover]
    return l2, a2, np.array([rho[cv].mean() for cv in cover_old])
