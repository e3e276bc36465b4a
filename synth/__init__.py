"""Seeded synthetic inputs for the AMR topology-optimisation hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
*only* input definitions: random draws, the synthetic density fields, and
declarative descriptions of the supports and loads.  It performs none of the
method's arithmetic (no element matrices, no filters, no solves, no mesh
balancing); each consumer turns these descriptions into its own data.

Conventions
-----------
* Axes: x = length (axis 0), y = depth (axis 1), z = up (axis 2).
* All coordinates are on the finest integer lattice (finest element size 1).
* Uniform element order is x-fastest: ``e = ix + nx*(iy + ny*iz)``.
* Material (SIMP, paper Sec. 3 Eq. (2) with the modified floor
  E = Emin + rho^p (E0 - Emin)): E0 = 1, Emin = 1e-9, nu = 0.3, p = 3.

Problem families (cantilever: Sec. 7 Test 2 geometry class; bridge: a beam on
two bottom line supports under a distributed top load):

* ``cantilever(nx, ny, nz)``: every DOF on the face x = 0 is fixed; a total
  load of -1 in z is spread along the line x = nx, z = 0 (all y).
* ``bridge(nx, ny, nz)``: every DOF on the two lines (x = 0, z = 0) and
  (x = nx, z = 0) is fixed; a total load of -1 in z is spread uniformly over
  the top face z = nz.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MATERIAL = dict(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)

# Support / load descriptors.  A "where" dict fixes lattice coordinates:
# {"x": 0} is the plane x = 0, {"x": 0, "z": 0} is a line.
# kind "line": the load is spread along a line with its total given;
# kind "face": the load is spread over a plane region with its total given.


def cantilever_bc(nx: int, ny: int, nz: int):
    fixed = [{"x": 0}]
    load = {"kind": "line", "where": {"x": nx, "z": 0}, "comp": 2, "total": -1.0}
    return fixed, load


def bridge_bc(nx: int, ny: int, nz: int):
    fixed = [{"x": 0, "z": 0}, {"x": nx, "z": 0}]
    load = {"kind": "face", "where": {"z": nz}, "comp": 2, "total": -1.0}
    return fixed, load


@dataclass
class UniformCase:
    """A uniform Q1 hex brick of ``dims`` elements (finest h = 1)."""
    name: str
    dims: tuple
    rho: np.ndarray            # element densities, x-fastest
    fixed: list
    load: dict
    smooth_radius: float = 0.0  # >0: the inputs expect one density-filter pass
    filter_radius: float = 1.5
    extra: dict = field(default_factory=dict)

    @property
    def n_elems(self):
        nx, ny, nz = self.dims
        return nx * ny * nz

    @property
    def n_nodes(self):
        nx, ny, nz = self.dims
        return (nx + 1) * (ny + 1) * (nz + 1)


@dataclass
class OctreeCase:
    """An octree mesh grown from ``base`` leaves up to ``max_level`` levels."""
    name: str
    base: tuple                # leaves at level 0 along x, y, z
    max_level: int
    fixed: list
    load: dict
    extra: dict = field(default_factory=dict)

    @property
    def dims(self):
        s = 1 << self.max_level
        return tuple(b * s for b in self.base)


def uniform_random(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


# --------------------------------------------------------------------------
# C1: 24x12x12 cantilever, rho0 ~ U[0.05, 1] iid (seed 0), smoothed once by
# the cone density filter of radius 1.5 (done by each consumer).
# --------------------------------------------------------------------------
def c1(dims=(24, 12, 12), seed: int = 0) -> UniformCase:
    nx, ny, nz = dims
    fixed, load = cantilever_bc(nx, ny, nz)
    rho0 = uniform_random(nx * ny * nz, 0.05, 1.0, seed)
    return UniformCase("cantilever_uniform", tuple(dims), rho0, fixed, load,
                       smooth_radius=1.5, filter_radius=1.5)


# --------------------------------------------------------------------------
# C2: smooth banded field on a 16x8x8 base refined up to 3 levels.
#   s(x) = 1/2 + 1/2 tanh(phi(x)/w),  phi = sum_m a_m sin(2 pi k_m . xhat + th_m)
#   rho(x) = 0.05 + 0.95 s(x),   xhat = x / domain size (per axis)
# --------------------------------------------------------------------------
C2_WIDTH = 0.058


@dataclass
class SmoothField:
    k: np.ndarray      # (6, 3) integer wave vectors
    a: np.ndarray      # (6,)
    th: np.ndarray     # (6,)
    width: float
    domain: tuple      # finest-lattice extents

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        xh = pts / np.asarray(self.domain, dtype=np.float64)
        phase = 2.0 * math.pi * (xh @ self.k.T.astype(np.float64)) + self.th
        phi = np.sin(phase) @ self.a
        s = 0.5 + 0.5 * np.tanh(phi / self.width)
        return 0.05 + 0.95 * s


def smooth_field(domain, seed: int = 0, width: float = C2_WIDTH) -> SmoothField:
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < 6:
        k = rng.integers(0, 3, size=3)
        if k.any():
            ks.append(k)
    a = rng.uniform(0.5, 1.0, size=6)
    th = rng.uniform(0.0, 2.0 * math.pi, size=6)
    return SmoothField(np.array(ks, dtype=np.int64), a, th, float(width), tuple(domain))


def c2(base=(16, 8, 8), max_level: int = 3, seed: int = 0, width: float = C2_WIDTH) -> OctreeCase:
    s = 1 << max_level
    dims = tuple(b * s for b in base)
    fixed, load = cantilever_bc(*dims)
    fld = smooth_field(dims, seed, width)
    return OctreeCase("cantilever_octree", tuple(base), max_level, fixed, load,
                      extra=dict(field=fld, band=(0.1, 0.9)))


def leaf_probe_points(level: np.ndarray, anchor: np.ndarray, max_level: int) -> np.ndarray:
    """Eight corners and the centre of each leaf (n, 9, 3): where the C2 band
    criterion samples the field.  Pure geometry of the input recipe."""
    size = (1 << (max_level - level.astype(np.int64)))[:, None, None]
    offs = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)] + [[0.5, 0.5, 0.5]],
                    dtype=np.float64)[None]
    return anchor[:, None, :].astype(np.float64) + size * offs


def band_marks(fld: SmoothField, level, anchor, max_level, band=(0.1, 0.9)) -> np.ndarray:
    """C2 input recipe: a leaf below ``max_level`` is marked when the field at
    any of its corners or its centre lies strictly inside ``band``."""
    pts = leaf_probe_points(level, anchor, max_level)
    v = fld(pts.reshape(-1, 3)).reshape(pts.shape[0], 9)
    inside = ((v > band[0]) & (v < band[1])).any(axis=1)
    return inside & (level < max_level)


# --------------------------------------------------------------------------
# C3: 192x96x96 value noise (3 octaves) thresholded to 30 % solid.
# --------------------------------------------------------------------------
def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise(dims, lattices, amps, seed: int, pts: np.ndarray) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.zeros(pts.shape[0])
    D = np.asarray(dims, dtype=np.float64)
    for lat, amp in zip(lattices, amps):
        lat = np.asarray(lat)
        vals = rng.uniform(-1.0, 1.0, size=tuple(lat + 1))
        g = pts / D * lat                          # lattice coordinates
        i0 = np.minimum(np.floor(g).astype(np.int64), lat - 1)
        t = _smoothstep(g - i0)
        acc = np.zeros(pts.shape[0])
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    w = ((t[:, 0] if di else 1 - t[:, 0]) * (t[:, 1] if dj else 1 - t[:, 1])
                         * (t[:, 2] if dk else 1 - t[:, 2]))
                    acc += w * vals[i0[:, 0] + di, i0[:, 1] + dj, i0[:, 2] + dk]
        out += amp * acc
    return out


def element_centres(dims) -> np.ndarray:
    nx, ny, nz = dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([ix.ravel() + 0.5, iy.ravel() + 0.5, iz.ravel() + 0.5], axis=1)


def c3(dims=(192, 96, 96), seed: int = 0, vec_seed: int = 1) -> UniformCase:
    nx, ny, nz = dims
    fixed, load = cantilever_bc(nx, ny, nz)
    lat = [(max(1, nx // 24), max(1, ny // 24), max(1, nz // 24))]
    lat = [lat[0], tuple(2 * v for v in lat[0]), tuple(4 * v for v in lat[0])]
    noise = value_noise(dims, lat, (1.0, 0.5, 0.25), seed, element_centres(dims))
    thr = np.quantile(noise, 0.70)
    rho = (noise > thr).astype(np.float64)
    return UniformCase("cantilever_noise_uniform", tuple(dims), rho, fixed, load,
                       extra=dict(vec_seed=vec_seed, lattices=lat))


# --------------------------------------------------------------------------
# C4: bridge, base 32x16x16, finest 128x64x64 (2 refinements), rho = 0.25.
# --------------------------------------------------------------------------
def c4(base=(32, 16, 16), max_level: int = 2, volfrac: float = 0.25, iters: int = 50,
       adapt_every: int = 5, train_iters: int = 10) -> OctreeCase:
    s = 1 << max_level
    dims = tuple(b * s for b in base)
    fixed, load = bridge_bc(*dims)
    return OctreeCase("bridge_octree_simp", tuple(base), max_level, fixed, load,
                      extra=dict(rho_init=0.25, volfrac=volfrac, rmin=1.5, r_amr=1.5,
                                 rho_solid=0.5, iters=iters, adapt_every=adapt_every,
                                 train_iters=train_iters, net_seed=0))


# --------------------------------------------------------------------------
# AMR against the uniform fine mesh (the shape of the paper's 3-D cantilever
# test: uniform 128x32x32 against an adaptive run whose initial mesh is
# 64x16x16, one refinement level, volume fraction 0.25).  The test's loads and
# supports exist only in a figure: the synthetic cantilever BCs stand in.  The
# filter radius equals the refinement radius r (Sec. 6), in finest cells: 1.5,
# or 3, with which the filter acts on the initial mesh too (its elements are 2
# cells wide; a radius at or below that gives every neighbour weight zero).
# --------------------------------------------------------------------------
def amr_vs_uniform(base=(64, 16, 16), max_level: int = 1, steps: int = 300, r: float = 1.5) -> OctreeCase:
    s = 1 << max_level
    dims = tuple(b * s for b in base)
    fixed, load = cantilever_bc(*dims)
    return OctreeCase("cantilever_amr_vs_uniform", tuple(base), max_level, fixed, load,
                      extra=dict(rho_init=0.25, volfrac=0.25, rmin=r, r_amr=r, rho_solid=0.5, steps=steps,
                                 min_steps=5, max_steps=10, change_tol=0.01))


# --------------------------------------------------------------------------
# C5: bridge 128x64x64, rho ~ U[0.01, 1] iid (seed 0); FD on 64 elements (seed 1).
# --------------------------------------------------------------------------
def c5(dims=(128, 64, 64), seed: int = 0, fd_seed: int = 1, n_fd: int = 64) -> UniformCase:
    nx, ny, nz = dims
    fixed, load = bridge_bc(nx, ny, nz)
    rho = uniform_random(nx * ny * nz, 0.01, 1.0, seed)
    fd = np.random.default_rng(fd_seed).choice(nx * ny * nz, size=min(n_fd, nx * ny * nz), replace=False)
    return UniformCase("bridge_uniform", tuple(dims), rho, fixed, load,
                       extra=dict(fd_elems=np.sort(fd), fd_step=1e-6))
