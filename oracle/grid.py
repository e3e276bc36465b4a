"""Reference mesh <-> grid transfers of the learned warm start (test
infrastructure; nothing in the product path imports this module).

Not in the paper; these are plain definitions on the finest lattice:

* grid nodes sit every ``cell`` lattice units, arrays are node-major (z, y, x);
* density at a grid node = mean of the element density over the node's dual
  cell (the box of edge ``cell`` centred at the node, clipped to the domain),
  computed on a voxel image of the design at half-lattice resolution so that
  half-cell offsets land on voxel faces;
* displacement at a grid node = the finite-element field there: trilinear
  interpolation over a leaf whose closed box holds the point (the field is
  continuous once hanging values follow Eq. (6), so any such leaf gives it);
* mesh node value from grid values = trilinear interpolation on the grid cell
  holding the node.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


def voxel_image(mesh: Mesh, rho, up=2):
    """rho on the lattice refined ``up`` times, indexed [z, y, x]."""
    nx, ny, nz = mesh.dims
    img = np.zeros((nz * up, ny * up, nx * up))
    for e in range(mesh.n_elems):
        a = mesh.anchor[e] * up
        h = int(mesh.size[e]) * up
        img[a[2]:a[2] + h, a[1]:a[1] + h, a[0]:a[0] + h] = rho[e]
    return img


def grid_density(mesh: Mesh, rho, cell):
    nx, ny, nz = mesh.dims
    gx, gy, gz = nx // cell, ny // cell, nz // cell
    img = voxel_image(mesh, rho, 2)
    out = np.zeros((gz + 1, gy + 1, gx + 1))
    for k in range(gz + 1):
        z0, z1 = max(0, 2 * k * cell - cell), min(2 * nz, 2 * k * cell + cell)
        for j in range(gy + 1):
            y0, y1 = max(0, 2 * j * cell - cell), min(2 * ny, 2 * j * cell + cell)
            for i in range(gx + 1):
                x0, x1 = max(0, 2 * i * cell - cell), min(2 * nx, 2 * i * cell + cell)
                out[k, j, i] = img[z0:z1, y0:y1, x0:x1].mean()
    return out


def fe_eval(mesh: Mesh, u, pts):
    """u (3 nn) evaluated at lattice points pts (m, 3) -> (m, 3)."""
    u = np.asarray(u).reshape(-1, 3)
    out = np.zeros((len(pts), 3))
    lo = mesh.anchor
    hi = mesh.anchor + mesh.size[:, None]
    for q, p in enumerate(np.asarray(pts, dtype=np.float64)):
        e = int(np.flatnonzero(((lo <= p) & (p <= hi)).all(axis=1))[0])
        t = (p - lo[e]) / mesh.size[e]
        for a in range(8):
            bits = np.array([a & 1, (a >> 1) & 1, a >> 2])
            w = np.prod(np.where(bits == 1, t, 1.0 - t))
            out[q] += w * u[mesh.elem_nodes[e, a]]
    return out


def grid_points(dims, cell):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz // cell + 1), np.arange(ny // cell + 1), np.arange(nx // cell + 1),
                          indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) * cell


def grid_sample(mesh: Mesh, u, cell, scale=1.0):
    """(3, gz+1, gy+1, gx+1): scale times the FE displacement at the grid nodes."""
    nx, ny, nz = mesh.dims
    vals = fe_eval(mesh, u, grid_points(mesh.dims, cell))
    return scale * vals.T.reshape(3, nz // cell + 1, ny // cell + 1, nx // cell + 1)


def grid_interp(ugrid, cell, coords, scale=1.0):
    """Mesh-node values (3 nn) from grid values (3, gz+1, gy+1, gx+1)."""
    _, GZ, GY, GX = ugrid.shape
    out = np.zeros((len(coords), 3))
    for n, p in enumerate(np.asarray(coords)):
        ix = min(int(p[0]) // cell, GX - 2)
        iy = min(int(p[1]) // cell, GY - 2)
        iz = min(int(p[2]) // cell, GZ - 2)
        t = (np.asarray(p, dtype=np.float64) - np.array([ix, iy, iz]) * cell) / cell
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
            w = (t[0] if ax else 1 - t[0]) * (t[1] if ay else 1 - t[1]) * (t[2] if az else 1 - t[2])
            out[n] += w * ugrid[:, iz + az, iy + ay, ix + ax]
    return scale * out.ravel()
