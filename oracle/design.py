"""Design-level rules of the paper that sit around one SIMP iteration.

Test infrastructure: a plain CPU statement of each rule, used only by the
tests to judge the library.

* Design difference D (Sec. 7, Eq. (10)): the L1 norm of rho1 - rho2 over the
  domain divided by the integral of rho1.  Both designs are first carried to
  the finest level everywhere without changing them (each finest-lattice cell
  takes the density of the leaf that covers it), so every cell has unit volume
  and the integrals are plain sums over cells.
* Adaptation trigger (Sec. 4): adapt when CASE (i) the design has settled --
  the largest change of a design variable in the last step is below a
  tolerance (0.01 in the paper) -- and at least a minimum number of steps (5)
  have passed since the last adaptation; or CASE (ii) a maximum number of
  steps (10) has passed without CASE (i).  The paper's first condition speaks
  of the relative change of the compliance and then explains it as the largest
  design change; the latter is taken.
* p-continuation (Sec. 3): the penalty starts at p = 1 and grows slowly as the
  design converges.  The paper gives no schedule; the one stated here raises p
  by dp whenever the design has settled (largest change below a tolerance) or
  a number of steps has passed at the current p, up to p_max.
"""
from __future__ import annotations

import numpy as np

from .mesh import leaf_sizes


def finest_cells(level, anchor, max_level, dims, values):
    """Values of the leaves on the finest lattice: array (nz, ny, nx) whose
    cell (k, j, i) holds the value of the leaf covering it.  Every cell must
    be covered exactly once (leaves tile the box)."""
    nx, ny, nz = (int(d) for d in dims)
    out = np.full((nz, ny, nx), np.nan)
    cover = np.zeros((nz, ny, nx), np.int64)
    h = leaf_sizes(level, max_level)
    for (ax, ay, az), s, v in zip(np.asarray(anchor, np.int64), h, np.asarray(values, np.float64)):
        out[az:az + s, ay:ay + s, ax:ax + s] = v
        cover[az:az + s, ay:ay + s, ax:ax + s] += 1
    if not (cover == 1).all():
        raise ValueError("leaves do not tile the lattice box exactly once")
    return out


def design_difference(mesh1, rho1, mesh2, rho2):
    """Eq. (10): D = sum |rho1 - rho2| / sum rho1 over finest-lattice cells.
    mesh = (level, anchor, max_level, dims) of the leaves the densities live on."""
    c1 = finest_cells(*mesh1, rho1)
    c2 = finest_cells(*mesh2, rho2)
    if c1.shape != c2.shape:
        raise ValueError("designs live on different lattice boxes")
    return float(np.abs(c1 - c2).sum() / c1.sum())


def adapt_due(steps_since, change, min_steps=5, max_steps=10, tol=0.01):
    """Sec. 4: CASE (i) change < tol and steps_since >= min_steps, or CASE (ii)
    steps_since >= max_steps.  steps_since counts the design steps taken on the
    current mesh; change is the largest |rho_new - rho| of the last one."""
    return (change < tol and steps_since >= min_steps) or steps_since >= max_steps


def p_next(p, steps_at_p, change, dp=0.5, p_max=3.0, tol=0.01, max_steps=20):
    """Continuation on the penalty (Sec. 3): p + dp (capped at p_max) once the
    design has settled (change < tol) or max_steps steps were taken at p."""
    if p >= p_max:
        return p_max
    if change < tol or steps_at_p >= max_steps:
        return min(p_max, p + dp)
    return p
