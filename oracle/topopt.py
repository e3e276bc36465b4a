"""Compliance, sensitivities, filters and the Optimality Criteria update.

* Compliance c = f^T u (paper Sec. 3, Eq. (1)).
* Sensitivity (Sec. 3, "sensitivity analysis"; the text gives no formula):
  compliance is self-adjoint, so dc/drho_e = -u_e^T (dK_e/drho_e) u_e =
  -p rho_e^(p-1) (E0 - Emin) h_e u_e^T K0 u_e.
* Filters (Sec. 6, Eq. (3)-(5)): H_de = max(r_min - dist(d, e), 0) with dist
  the distance between element centres.  The sensitivity filter uses the
  volume-weighted form of Eq. (5); the same weights in "density" mode give the
  cone density filter used to smooth seeded densities.
* OC (Sec. 3 names Optimality Criteria without a formula): the standard
  heuristic rho_new = clamp(rho * (-dc / (lam V_e))^eta, max(rho_min, rho - m),
  min(1, rho + m)) with lam fixed by sum rho_new V_e = V0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .element import k0 as element_k0
from .mesh import Mesh
from .system import elem_dofs


def compliance(f, u) -> float:
    return float(np.dot(f, u))


def element_energy(mesh: Mesh, u, K0=None, nu=0.3) -> np.ndarray:
    """w_e = u_e^T K0 u_e for every element."""
    if K0 is None:
        K0 = element_k0(nu)
    ue = u[elem_dofs(mesh)]
    return np.einsum("ei,ij,ej->e", ue, K0, ue)


def sensitivities(mesh: Mesh, rho, u, E0=1.0, Emin=1e-9, p=3.0, K0=None, nu=0.3):
    w = element_energy(mesh, u, K0, nu)
    rho = np.asarray(rho, dtype=np.float64)
    return -p * rho ** (p - 1.0) * (E0 - Emin) * mesh.size.astype(np.float64) * w


def filter_weights(mesh: Mesh, rmin: float) -> sp.csr_matrix:
    """W[e, d] = H_de V_d (Eq. (4)-(5)); pairs with H_de = 0 are absent."""
    cen = mesh.centres
    tree = cKDTree(cen)
    pairs = tree.sparse_distance_matrix(tree, rmin, output_type="ndarray")
    i, j, dist = pairs["i"], pairs["j"], pairs["v"]
    keep = i != j
    i, j, dist = i[keep], j[keep], dist[keep]
    n = mesh.n_elems
    i = np.concatenate([i, np.arange(n)])
    j = np.concatenate([j, np.arange(n)])
    dist = np.concatenate([dist, np.zeros(n)])
    H = np.maximum(rmin - dist, 0.0)
    ok = H > 0
    V = mesh.volumes
    return sp.csr_matrix((H[ok] * V[j[ok]], (i[ok], j[ok])), shape=(n, n))


def filter_sensitivity(mesh: Mesh, rmin, rho, dc, rho_min=1e-3, W=None):
    """Eq. (5): sum_d rho_d H_de V_d dc_d / (rho_e sum_d H_de V_d); the
    denominator density is floored at rho_min (the paper's rho_o)."""
    if W is None:
        W = filter_weights(mesh, rmin)
    num = W @ (np.asarray(rho) * np.asarray(dc))
    den = np.maximum(np.asarray(rho), rho_min) * np.asarray(W.sum(axis=1)).ravel()
    return num / den


def filter_density(mesh: Mesh, rmin, x, W=None):
    """Cone density filter with the same weights: sum_d H_de V_d x_d / sum_d H_de V_d."""
    if W is None:
        W = filter_weights(mesh, rmin)
    return (W @ np.asarray(x)) / np.asarray(W.sum(axis=1)).ravel()


def oc_update(rho, dc, vol, v0, move=0.2, eta=0.5, rho_min=1e-3, rtol=1e-13):
    """Optimality Criteria step with lam found by bisection in log(lam)."""
    rho = np.asarray(rho, dtype=np.float64)
    g = np.maximum(-np.asarray(dc, dtype=np.float64), 0.0) / vol
    lo_b = np.maximum(rho_min, rho - move)
    hi_b = np.minimum(1.0, rho + move)

    def step(lam):
        return np.clip(rho * (g / lam) ** eta, lo_b, hi_b)

    def volume(lam):
        return float(np.dot(step(lam), vol))

    lo, hi = 1e-300, 1e300
    # volume is non-increasing in lam: bracket, then bisect geometrically
    for _ in range(4000):
        mid = np.sqrt(lo) * np.sqrt(hi)
        if volume(mid) > v0:
            lo = mid
        else:
            hi = mid
        if (hi - lo) <= rtol * hi:
            break
    lam = np.sqrt(lo) * np.sqrt(hi)
    new = step(lam)
    return new, lam, float(np.max(np.abs(new - rho)))
