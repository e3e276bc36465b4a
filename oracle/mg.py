"""Geometric multigrid on the octree hierarchy as the preconditioner of CG.

Test infrastructure: a plain FP64 CPU statement of the multigrid the library
runs, used only by the tests to judge it.

The paper (Sec. 5) finds the rescaled system unusable without a good
preconditioner at the p = 3 stiffness contrast and uses IC(0); the method here
is a stronger, parallel alternative built from textbook definitions:

* Level meshes.  Level 0 is the analysis mesh with leaves of levels 0..L.  For
  1 <= k <= L, every leaf finer than level L - k is replaced by its ancestor
  at that level (all siblings of a finest leaf are leaves, so merging keeps the
  one-level rule between neighbours).  For k > L the uniform base grid is
  coarsened by two per axis, k - L times, as long as every base extent stays
  divisible.  The first coarse level may take ``first`` > 1 such steps at
  once (level depths first, first + 1, ...).  Levels are added until one is
  a uniform grid (depth >= L, no hanging nodes) with at most ``coarse_dofs``
  DOFs, or no further level can be built.  Supports are the same lattice
  planes or lines on every level.
* Prolongation P_k from level k to level k - 1 (vectors in the constrained
  form: zero at hanging and supported DOFs): the level-k field T_k F_k x is
  continuous and trilinear on each level-k leaf; its values at the level
  k - 1 nodes, masked by F_{k-1}, are P_k x.  Every level k - 1 leaf lies in
  one level-k leaf, so the coarse space is contained in the fine one.
* Galerkin operators A_k = P_k^T A_{k-1} P_k + (I - F_k) (identity rows for
  the constrained DOFs, as A~ has on level 0).
* Smoother: the Chebyshev iteration for M^-1 A on the interval
  [hi / ratio, hi], hi = 1.1 lambda_max(M^-1 A), degree m on level 0 and
  optionally another degree on the coarse levels (Golub and Varga's
  three-term recurrence as in Saad, Iterative Methods for Sparse Linear
  Systems, Alg. 12.1).  M is D = diag A, or on level 0 optionally the block
  diagonal of A's 3 x 3 node blocks (point-block Jacobi: the three
  displacement components of a node are coupled in A).  The same polynomial
  smooths before and after the coarse correction, so one V-cycle is a
  symmetric operator.
* V-cycle: pre-smooth from zero, restrict the residual with P^T, recurse,
  prolong and add the coarse correction, recompute the residual, post-smooth;
  the coarsest level is solved exactly.
* CG preconditioned by one V-cycle per iteration.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import shape_values
from .mesh import LeafIndex, Mesh, build_mesh, fixed_dofs
from .system import PCGResult, dof_interp, free_mask


# ---------------------------------------------------------------- levels
def coarsen_leaves(level, anchor, max_level, base, k):
    """Leaves of level mesh k: (level, anchor, max_level) of a tree on the same
    finest lattice, or None when level k cannot be built."""
    level = np.asarray(level, np.int64)
    anchor = np.asarray(anchor, np.int64)
    L = int(max_level)
    if k <= L:
        lv = np.minimum(level, L - k)
        ml = L
    else:
        j = k - L
        if any(int(b) % (1 << j) for b in base):
            return None
        lv = np.zeros_like(level)
        ml = k
    s = np.int64(1) << (ml - lv)
    an = (anchor // s[:, None]) * s[:, None]
    key = np.unique(np.concatenate([lv[:, None], an], 1), axis=0)
    return key[:, 0], key[:, 1:], ml


@dataclass
class Level:
    mesh: Mesh
    fixed: np.ndarray          # (3 nn,) supported DOFs
    free: np.ndarray           # (3 nn,) neither hanging nor supported
    A: sp.csr_matrix = None
    dinv: np.ndarray = None
    minv: object = None        # smoother's M^-1: dinv, or the sparse node-block inverse
    P: sp.csr_matrix = None    # from the next coarser level to this one
    lo: float = 0.0
    hi: float = 0.0


def hierarchy(mesh0: Mesh, base, fixed_spec, coarse_dofs=1000, first=1):
    """Level meshes of depths 0, first, first + 1, ... (depth 0 is mesh0)."""
    levels = [Level(mesh0, fixed_dofs(mesh0, fixed_spec), None)]
    levels[0].free = free_mask(mesh0, levels[0].fixed)
    k, prev = first, 0
    while prev < mesh0.max_level or 3 * levels[-1].mesh.n_nodes > coarse_dofs:
        c = coarsen_leaves(mesh0.level, mesh0.anchor, mesh0.max_level, base, k)
        if c is None:
            break
        m = build_mesh(c[0], c[1], c[2], mesh0.dims)
        fx = fixed_dofs(m, fixed_spec)
        levels.append(Level(m, fx, free_mask(m, fx)))
        prev, k = k, k + 1
    return levels


def interp_nodes(coarse: Mesh, fine_coords) -> sp.csr_matrix:
    """(n_fine x n_coarse) trilinear weights: the continuous coarse field (all
    coarse nodes, hanging ones included) evaluated at the fine nodes."""
    idx = LeafIndex(coarse.level, coarse.anchor, coarse.max_level)
    pts = np.asarray(fine_coords, np.float64)
    dims = np.asarray(coarse.dims)
    # a point a quarter cell towards the interior lies in a leaf whose closed box holds the node
    leaf = idx.find(np.where(pts >= dims, pts - 0.25, pts + 0.25))
    assert (leaf >= 0).all()
    rows, cols, vals = [], [], []
    for i, (p, l) in enumerate(zip(pts, leaf)):
        w = shape_values((p - coarse.anchor[l]) / float(coarse.size[l]))
        for a in range(8):
            if w[a] != 0.0:
                rows.append(i)
                cols.append(int(coarse.elem_nodes[l, a]))
                vals.append(float(w[a]))
    I = sp.csr_matrix((vals, (rows, cols)), shape=(len(pts), coarse.n_nodes))
    I.sum_duplicates()
    return I


def prolongation(fine: Level, coarse: Level) -> sp.csr_matrix:
    """P = F_f (I (x) I3) T_c F_c  (3 n_f x 3 n_c)."""
    I3 = sp.kron(interp_nodes(coarse.mesh, fine.mesh.coords), sp.identity(3), format="csr")
    Ff = sp.diags(fine.free.astype(np.float64))
    Fc = sp.diags(coarse.free.astype(np.float64))
    P = (Ff @ I3 @ dof_interp(coarse.mesh) @ Fc).tocsr()
    P.eliminate_zeros()
    return P


def galerkin(A_f: sp.csr_matrix, P: sp.csr_matrix, free_c) -> sp.csr_matrix:
    Ac = (P.T @ A_f @ P).tocsr() + sp.diags((~np.asarray(free_c)).astype(np.float64))
    Ac = Ac.tocsr()
    Ac.sum_duplicates()
    return Ac


def node_blocks(A: sp.csr_matrix) -> np.ndarray:
    """The 3 x 3 diagonal blocks of A, one per node (n, 3, 3)."""
    n = A.shape[0] // 3
    A = A.tocsr()
    return np.stack([A[3 * v:3 * v + 3, 3 * v:3 * v + 3].toarray() for v in range(n)])


def block_diag_matrix(blocks) -> sp.csr_matrix:
    """Sparse block-diagonal matrix from (n, 3, 3) blocks."""
    n = len(blocks)
    rows = np.repeat(np.arange(3 * n).reshape(n, 3), 3, axis=1).ravel()
    cols = np.tile(np.arange(3 * n).reshape(n, 3), (1, 3)).ravel()
    return sp.csr_matrix((np.asarray(blocks).ravel(), (rows, cols)), shape=(3 * n, 3 * n))


def lambda_max(A: sp.csr_matrix, minv) -> float:
    """Largest eigenvalue of M^-1 A, through the symmetric form L^T A L with
    M^-1 = L L^T: L = diag(sqrt(dinv)) for a diagonal M (minv the vector of
    1 / D), else the node-block Cholesky factors of M^-1 (minv sparse)."""
    if sp.issparse(minv):
        n = minv.shape[0] // 3
        b = np.stack([minv[3 * v:3 * v + 3, 3 * v:3 * v + 3].toarray() for v in range(n)])
        s = block_diag_matrix(np.linalg.cholesky(b))
    else:
        s = sp.diags(np.sqrt(minv))
    S = (s.T @ A @ s).tocsr()
    if S.shape[0] <= 400:
        return float(np.linalg.eigvalsh(S.toarray())[-1])
    return float(spla.eigsh(S, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])


# ---------------------------------------------------------------- smoothing and cycles
def chebyshev(A, minv, b, x, lo, hi, m, need_residual=True):
    """m steps of the Chebyshev iteration for M^-1 A on [lo, hi] from x
    (minv: the vector 1 / diag A, or the sparse matrix M^-1); returns (x, r)
    with r = b - A x (None when not needed after the last step)."""
    apply_m = (lambda v: minv @ v) if sp.issparse(minv) else (lambda v: minv * v)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    x = np.array(x, dtype=np.float64)
    r = b - A @ x if np.any(x) else np.array(b, dtype=np.float64)
    rho = 1.0 / sigma
    d = apply_m(r) / theta
    for k in range(m):
        x = x + d
        if k == m - 1 and not need_residual:
            return x, None
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * apply_m(r)
        rho = rho_new
    return x, r


@dataclass
class MG:
    levels: list
    degree: int = 2
    ratio: float = 10.0
    coarse_inv: np.ndarray = field(default=None)
    coarse_degree: int = 0      # degree on levels k >= 1 (0: the same as degree)

    def vcycle(self, b, k=0):
        lv = self.levels[k]
        if k == len(self.levels) - 1:
            return self.coarse_inv @ b
        m = self.degree if k == 0 or self.coarse_degree <= 0 else self.coarse_degree
        x, r = chebyshev(lv.A, lv.minv, b, np.zeros_like(b), lv.lo, lv.hi, m)
        P = self.levels[k + 1].P
        x = x + P @ self.vcycle(P.T @ r, k + 1)
        r = b - lv.A @ x
        e, _ = chebyshev(lv.A, lv.minv, r, np.zeros_like(b), lv.lo, lv.hi, m, need_residual=False)
        return x + e


def setup(levels, A0, degree=2, ratio=10.0, bounds=None, coarse_degree=0, blocks0=False) -> MG:
    """Galerkin operators, diagonals, smoothing intervals (``bounds``: optional
    list of lambda_max per smoothed level) and the coarsest inverse; with
    ``blocks0`` level 0 smooths with its inverse 3 x 3 node blocks."""
    levels[0].A = A0.tocsr()
    for k in range(1, len(levels)):
        levels[k].P = prolongation(levels[k - 1], levels[k])
        levels[k].A = galerkin(levels[k - 1].A, levels[k].P, levels[k].free)
    for k, lv in enumerate(levels):
        lv.dinv = 1.0 / lv.A.diagonal()
        lv.minv = lv.dinv
        if k == 0 and blocks0:
            lv.minv = block_diag_matrix(np.linalg.inv(node_blocks(lv.A)))
        if k < len(levels) - 1:
            lam = lambda_max(lv.A, lv.minv) if bounds is None else bounds[k]
            lv.hi = 1.1 * lam
            lv.lo = lv.hi / ratio
    Ac = levels[-1].A.toarray()
    inv = sla.cho_solve(sla.cho_factor(Ac), np.identity(len(Ac)))
    return MG(levels, degree, ratio, 0.5 * (inv + inv.T), coarse_degree)


def mg_pcg(A: sp.csr_matrix, b, mg: MG, x0=None, rtol=1e-8, max_it=10_000) -> PCGResult:
    """Textbook CG with z = V-cycle(r); stops on ||r_k|| <= rtol ||b||."""
    t0 = time.perf_counter()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return PCGResult(np.zeros_like(b), 0, 0.0, time.perf_counter() - t0)
    z = mg.vcycle(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < max_it:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = mg.vcycle(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return PCGResult(x, it, float(np.linalg.norm(b - A @ x) / nb), time.perf_counter() - t0)
