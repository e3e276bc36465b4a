"""Pins of oracle/recycle.py against facts fixed by the mathematics: on a
small SPD pencil, (1) the Lanczos matrix built from CG coefficients equals
the one an explicit M-inner-product Lanczos run (a different algorithm)
builds from the same start; (2) after n steps its eigenvalues are those of
the pencil (A, M); (3) every Ritz pair satisfies the Lanczos residual
identity ||A u - theta M u||_{M^-1} = |T[m-1, m] y_{m-1}|; (4) the Lanczos
vectors are M-orthonormal; (5) Rayleigh-Ritz on a subspace that contains the
pencil's k lowest eigenvectors returns them exactly."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import recycle


def _spd(n, seed, lo=1e-3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(lo, 10.0, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    s = rng.uniform(0.5, 3.0, n)  # rescale rows/cols so the diagonal is not constant
    return s[:, None] * A * s[None, :]


def _explicit_lanczos(A, d, r0, m):
    """Lanczos for M^-1 A (M = diag(d)) with M-inner products, start M^-1 r0."""
    minv = lambda v: v / d
    v = minv(r0)
    v = v / np.sqrt(v @ (d * v))
    V, a, b = [v], [], []
    w_prev = np.zeros_like(v)
    beta = 0.0
    for j in range(m):
        w = minv(A @ V[-1]) - beta * w_prev
        al = w @ (d * V[-1])
        w = w - al * V[-1]
        a.append(al)
        beta = np.sqrt(w @ (d * w))
        b.append(beta)
        w_prev = V[-1]
        V.append(w / beta)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    return T


def test_cg_lanczos_matrix_equals_explicit_lanczos():
    A = _spd(12, 0)
    d = np.diag(A).copy()
    b = np.random.default_rng(1).standard_normal(12)
    _, Z, rz, pq = recycle.pcg_record(A, b, lambda r: r / d, 6)
    T_cg = recycle.lanczos_from_cg(rz, pq)
    T_ex = _explicit_lanczos(A, d, b, 6)
    assert np.allclose(T_cg, T_ex, rtol=1e-10, atol=1e-12 * np.abs(T_ex).max())


def test_full_krylov_space_gives_pencil_eigenvalues():
    # well conditioned, so that n Lanczos steps keep their vectors orthogonal
    A = _spd(10, 2, lo=0.5)
    d = np.diag(A).copy()
    b = np.random.default_rng(3).standard_normal(10)
    _, Z, rz, pq = recycle.pcg_record(A, b, lambda r: r / d, 10)
    theta = np.linalg.eigvalsh(recycle.lanczos_from_cg(rz, pq))
    want = sla.eigh(A, np.diag(d), eigvals_only=True)
    assert np.allclose(theta, want, rtol=1e-10)


def test_ritz_residual_identity_and_orthonormality():
    A = _spd(40, 4)
    d = np.diag(A).copy()
    b = np.random.default_rng(5).standard_normal(40)
    m, k = 15, 4
    _, Z, rz, pq = recycle.pcg_record(A, b, lambda r: r / d, m + 1)
    theta, U, res = recycle.ritz_pairs(Z, rz, pq[:m], k)
    V = recycle.lanczos_vectors(Z[:, :m], rz)
    assert np.allclose(V.T @ (d[:, None] * V), np.eye(m), atol=1e-8)
    for i in range(k):
        r = A @ U[:, i] - theta[i] * d * U[:, i]
        assert np.sqrt(r @ (r / d)) == pytest.approx(res[i], rel=1e-6, abs=1e-12)
    # the smallest Ritz value bounds the smallest eigenvalue from above
    lam_min = sla.eigh(A, np.diag(d), eigvals_only=True)[0]
    assert theta[0] >= lam_min * (1 - 1e-12)


def test_rayleigh_ritz_recovers_contained_eigenvectors():
    A = _spd(30, 6)
    d = np.diag(A).copy()
    lam, X = sla.eigh(A, np.diag(d))
    rng = np.random.default_rng(7)
    S = np.concatenate([X[:, :3] @ rng.standard_normal((3, 3)), rng.standard_normal((30, 4))], axis=1)
    theta, W = recycle.rayleigh_ritz(A, d, S, 3)
    assert np.allclose(theta, lam[:3], rtol=1e-9)
    for i in range(3):
        c = abs(W[:, i] @ (d * X[:, i]))
        assert c == pytest.approx(1.0, abs=1e-8)
