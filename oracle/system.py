"""Assembly and solution of K(rho) u = f with hanging-node and support
constraints (paper Sec. 3 Eq. (1)-(2), Sec. 5, Sec. 6 Eq. (6)-(9)).

Element stiffness: K_e = E_e * h_e * K0 with E_e = Emin + rho_e^p (E0 - Emin)
(Eq. (2) with the floor stiffness written as Emin; rho_o^p = Emin for
rho_o = 1e-3, p = 3).

Constrained operator used throughout (Eq. (8) plus identity rows and columns
for supported DOFs).  With T the DOF-level interpolation (unconstrained ->
all DOFs, hanging columns removed) and F the diagonal 0/1 mask of DOFs that are
neither hanging nor supported:

    A~ = F T^T K T F + (I - F),      b~ = F T^T f,

and the displacement is recovered as u = T u~ (Eq. (9)).  A~ is symmetric
positive definite; on the free unconstrained DOFs it equals the projected
system of Eq. (7) with the supported DOFs eliminated.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import k0 as element_k0
from .mesh import Mesh


def young(rho, E0=1.0, Emin=1e-9, p=3.0):
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho ** p * (E0 - Emin)


def elem_coeff(mesh: Mesh, rho, E0=1.0, Emin=1e-9, p=3.0):
    """c_e = E(rho_e) * h_e."""
    return young(rho, E0, Emin, p) * mesh.size.astype(np.float64)


def elem_dofs(mesh: Mesh) -> np.ndarray:
    return (3 * mesh.elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)


def assemble(mesh: Mesh, coeff, K0=None, nu=0.3, chunk=200_000) -> sp.csr_matrix:
    """Global K = sum_e c_e G_e^T K0 G_e over all nodes (hanging included)."""
    if K0 is None:
        K0 = element_k0(nu)
    dofs = elem_dofs(mesh)
    n = 3 * mesh.n_nodes
    K = sp.csr_matrix((n, n))
    for s in range(0, mesh.n_elems, chunk):
        d = dofs[s:s + chunk]
        c = np.asarray(coeff[s:s + chunk], dtype=np.float64)
        rows = np.repeat(d, 24, axis=1).ravel()
        cols = np.tile(d, (1, 24)).ravel()
        vals = (c[:, None, None] * K0[None]).ravel()
        K = K + sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    return K


def apply_elementwise(mesh: Mesh, coeff, x, K0=None, nu=0.3, chunk=100_000):
    """y = K x by looping over elements (no assembled matrix); plain definition."""
    if K0 is None:
        K0 = element_k0(nu)
    dofs = elem_dofs(mesh)
    y = np.zeros(3 * mesh.n_nodes)
    for s in range(0, mesh.n_elems, chunk):
        d = dofs[s:s + chunk]
        ue = x[d]                                   # (m, 24)
        ye = (ue @ K0.T) * np.asarray(coeff[s:s + chunk])[:, None]
        y += np.bincount(d.ravel(), weights=ye.ravel(), minlength=len(y))
    return y


def dof_interp(mesh: Mesh) -> sp.csr_matrix:
    """DOF-level T (3nn x 3nn): columns of hanging nodes are zero."""
    Tn = mesh.Tn.tocsc().copy()
    Tn = Tn.tocsr()
    return sp.kron(Tn, sp.identity(3), format="csr")


def free_mask(mesh: Mesh, fixed: np.ndarray) -> np.ndarray:
    return ~(np.repeat(mesh.hanging, 3) | fixed)


@dataclass
class System:
    A: sp.csr_matrix       # A~ (3nn x 3nn), SPD
    b: np.ndarray          # b~
    T: sp.csr_matrix
    free: np.ndarray       # bool (3nn,)
    f: np.ndarray          # consistent load on all nodes


def build_system(mesh: Mesh, coeff, fixed, f, K0=None, nu=0.3) -> System:
    K = assemble(mesh, coeff, K0, nu)
    T = dof_interp(mesh)
    free = free_mask(mesh, fixed)
    F = sp.diags(free.astype(np.float64))
    A = (F @ (T.T @ (K @ (T @ F)))).tocsr()
    A = A + sp.diags((~free).astype(np.float64))
    A = A.tocsr()
    A.sum_duplicates()
    b = F @ (T.T @ f)
    return System(A, b, T, free, f)


def apply_constrained(mesh: Mesh, coeff, fixed, x, K0=None, nu=0.3):
    """A~ x without assembling: mask, interpolate, element loop, condense, identity rows."""
    free = free_mask(mesh, fixed)
    T = dof_interp(mesh)
    xf = np.where(free, x, 0.0)
    u = T @ xf
    Ku = apply_elementwise(mesh, coeff, u, K0, nu)
    y = T.T @ Ku
    return np.where(free, y, x)


def solve_direct(sysm: System) -> np.ndarray:
    """u~ by sparse LU on the free DOFs, then u = T u~ (Eq. (9))."""
    idx = np.nonzero(sysm.free)[0]
    A = sysm.A[idx][:, idx].tocsc()
    ut = np.zeros(len(sysm.b))
    ut[idx] = spla.spsolve(A, sysm.b[idx])
    return ut


def recover(sysm: System, ut: np.ndarray) -> np.ndarray:
    return sysm.T @ ut


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    rel_res: float          # true ||b - A x|| / ||b||
    seconds: float


def pcg_jacobi(A: sp.csr_matrix, b: np.ndarray, x0=None, rtol=1e-8, max_it=100_000,
               diag=None) -> PCGResult:
    """Textbook conjugate gradients with the Jacobi preconditioner M = diag(A).

    Jacobi preconditioning is the symmetric diagonal rescaling
    D^-1/2 A D^-1/2 of the paper's Sec. 5; stopping uses the recurrence residual
    ||r_k|| <= rtol ||b|| and the true residual is reported at exit."""
    t0 = time.perf_counter()
    d = A.diagonal() if diag is None else diag
    dinv = 1.0 / d
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return PCGResult(np.zeros_like(b), 0, 0.0, time.perf_counter() - t0)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < max_it:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    rel = np.linalg.norm(b - A @ x) / nb
    return PCGResult(x, it, rel, time.perf_counter() - t0)
