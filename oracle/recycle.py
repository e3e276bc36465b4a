"""Krylov subspace recycling for a sequence of SPD systems (paper Sec. 5: an
approximate invariant subspace for the smallest eigenvalues, taken from the
Krylov space of one solve, is carried to the next system of the design
sequence).

Test infrastructure: a plain CPU statement of each step.

* Recorded PCG: textbook preconditioned CG (preconditioner given as a
  function z = M^-1 r) that also keeps the first m preconditioned residuals
  z_j, the products r_j^T z_j and p_j^T A p_j.
* Lanczos matrix from the CG coefficients (the CG/Lanczos correspondence,
  e.g. Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7):
  alpha_j = r_j^T z_j / p_j^T A p_j, beta_j = r_{j+1}^T z_{j+1} / r_j^T z_j,
  T[j, j] = 1/alpha_j + beta_{j-1}/alpha_{j-1} (the second term absent for
  j = 0), T[j, j+1] = T[j+1, j] = sqrt(beta_j) / alpha_j, with the
  M-orthonormal Lanczos vectors v_j = (-1)^j z_j / sqrt(r_j^T z_j).
* Ritz pairs: eigenpairs (theta, y) of T_m; Ritz vector u = V_m y
  approximates an eigenvector of the pencil (A, M) with eigenvalue theta.
* Rayleigh-Ritz on a subspace span(S) for the pencil (A, D), D the diagonal
  of A: the generalized eigenproblem S^T A S y = theta S^T D S y; the k
  smallest pairs give W = S Y.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pcg_record(A, b, minv, m, x0=None, max_it=None):
    """Preconditioned CG from x0 for max_it iterations (default m), recording
    z_0..z_{m-1} as columns of Z, rz[j] = r_j^T z_j and pq[j] = p_j^T A p_j.
    minv(r) applies M^-1.  Returns (x, Z, rz, pq)."""
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64)
    r = b - A @ x
    z = minv(r)
    p = z.copy()
    Z, rz, pq = [], [], []
    its = m if max_it is None else max_it
    for j in range(its):
        rzj = float(r @ z)
        if j < m:
            Z.append(z.copy())
            rz.append(rzj)
        q = A @ p
        pqj = float(p @ q)
        if j < m:
            pq.append(pqj)
        alpha = rzj / pqj
        x = x + alpha * p
        r = r - alpha * q
        z = minv(r)
        beta = float(r @ z) / rzj
        p = z + beta * p
    return x, np.array(Z).T, np.array(rz), np.array(pq)


def lanczos_from_cg(rz, pq):
    """T_m (m = len(pq)) from the CG coefficients; rz needs m entries."""
    m = len(pq)
    alpha = np.asarray(rz[:m]) / np.asarray(pq)
    beta = np.asarray(rz[1:m]) / np.asarray(rz[:m - 1])
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return T


def lanczos_vectors(Z, rz):
    """V with columns (-1)^j z_j / sqrt(r_j^T z_j)."""
    m = Z.shape[1]
    sign = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    return Z * (sign / np.sqrt(np.asarray(rz[:m])))[None, :]


def ritz_pairs(Z, rz, pq, k):
    """The k smallest Ritz values and their Ritz vectors (columns) of the
    recorded solve's preconditioned operator, and the Lanczos residual norms
    |T[m-1, m] y_{m-1}| (needs rz of m + 1 steps for the last off-diagonal;
    when only m are given the residual bound is returned as NaN)."""
    m = len(pq)
    T = lanczos_from_cg(rz, pq)
    theta, Y = np.linalg.eigh(T)
    U = lanczos_vectors(Z[:, :m], rz) @ Y[:, :k]
    if len(rz) > m:
        off = np.sqrt(rz[m] / rz[m - 1]) / (rz[m - 1] / pq[m - 1])
        res = np.abs(off * Y[m - 1, :k])
    else:
        res = np.full(k, np.nan)
    return theta[:k], U, res


def rayleigh_ritz(A, d, S, k):
    """The k smallest pairs of S^T A S y = theta S^T diag(d) S y; returns
    (theta, W = S Y) with W^T diag(d) W = I."""
    G = S.T @ (A @ S)
    B = S.T @ (d[:, None] * S)
    theta, Y = sla.eigh(0.5 * (G + G.T), 0.5 * (B + B.T))
    return theta[:k], S @ Y[:, :k]
