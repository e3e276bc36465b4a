"""Test-side builders: the same seeded synthetic case turned into (a) the
library's mesh through its own octree and (b) the oracle's mesh through the
oracle's own octree.  Each side grows its leaves independently; the builders
assert that both arrive at the same leaves and return the node permutation
(library node -> oracle node) that matches coordinates."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth
from oracle import amr, mesh as om, system as osys, topopt


@dataclass
class Pair:
    lib_mesh: object        # binding.MeshArrays
    orc: om.Mesh            # oracle mesh
    perm: np.ndarray        # library node i -> oracle node perm[i]
    eperm: np.ndarray       # library element e -> oracle element eperm[e]
    fixed: np.ndarray       # oracle DOF mask
    f: np.ndarray           # oracle consistent load
    case: object

    @property
    def dof_perm(self):
        return (3 * self.perm[:, None] + np.arange(3)).ravel()

    def to_lib_nodes(self, v_oracle):
        return np.asarray(v_oracle).reshape(-1, 3)[self.perm].ravel()

    def to_lib_elems(self, v_oracle):
        return np.asarray(v_oracle)[self.eperm]


def uniform_pair(dims, bc="cantilever"):
    from paper_1009_4975_amd import binding
    fixed, load = (synth.cantilever_bc if bc == "cantilever" else synth.bridge_bc)(*dims)
    t = binding.Octree(dims, 0)
    lm = binding.uniform_mesh(dims, fixed, load, tree=t)
    o = om.uniform_mesh(dims)
    n = o.n_nodes
    return Pair(lm, o, np.arange(n), np.arange(o.n_elems), om.fixed_dofs(o, fixed), om.load_vector(o, load),
                dict(fixed=fixed, load=load, dims=dims, tree=t))


def octree_pair(base, L, width=synth.C2_WIDTH, bc="cantilever"):
    """The C2 recipe at any size: band refinement then closure, on both sides."""
    from paper_1009_4975_amd import binding
    case = synth.c2(base=base, max_level=L, width=width)
    fld = case.extra["field"]
    dims = case.dims
    fixed, load = (synth.cantilever_bc if bc == "cantilever" else synth.bridge_bc)(*dims)
    t = binding.Octree(base, L)
    b = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])]) << L
    lv, an = np.zeros(len(b), np.int64), b
    for _ in range(L):
        tl, ta = t.leaves()
        t.refine(synth.band_marks(fld, tl, ta, L))
        lv, an, _ = amr.refine(lv, an, L, synth.band_marks(fld, lv, an, L))
    t.balance()
    lv, an, _ = amr.balance(lv, an, L)
    tl, ta = t.leaves()
    got = {(int(l), *map(int, a)) for l, a in zip(tl, ta)}
    want = {(int(l), *map(int, a)) for l, a in zip(lv, an)}
    assert got == want, "library and oracle octrees differ"
    lm = t.build_mesh(fixed, load)
    o = om.build_mesh(lv, an, L, dims)
    key = {tuple(c): i for i, c in enumerate(o.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in lm.node_xyz.tolist()])
    okey = {(int(l), *map(int, a)): e for e, (l, a) in enumerate(zip(o.level, o.anchor))}
    eperm = np.array([okey[(int(l), *map(int, a))] for l, a in zip(tl, ta)])
    return Pair(lm, o, perm, eperm, om.fixed_dofs(o, fixed), om.load_vector(o, load),
                dict(fixed=fixed, load=load, dims=dims, field=fld, tree=t))


def centre_density(pair, fld):
    """rho_e = field at element centre (C2 recipe), in oracle element order."""
    return fld(pair.orc.centres)


def c1_density(dims=(24, 12, 12)):
    """C1: U[0.05, 1] iid smoothed once by the cone density filter (oracle)."""
    case = synth.c1(dims)
    m = om.uniform_mesh(dims)
    return topopt.filter_density(m, case.smooth_radius, case.rho)


def oracle_system(pair, rho_oracle):
    return osys.build_system(pair.orc, osys.elem_coeff(pair.orc, rho_oracle), pair.fixed, pair.f)
