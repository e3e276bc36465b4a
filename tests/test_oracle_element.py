"""Pins for the oracle's Q1 element stiffness K0 (paper Sec. 3: trilinear
displacement, B8 bricks).  Every check here is independent of the oracle's
B^T D B quadrature code path."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import element

NU = 0.3


def lame(nu):
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    return lam, mu


def k0_index_form_exact(nu):
    """K[(a,c),(b,d)] = int lam N_a,c N_b,d + mu N_a,d N_b,c + mu delta_cd grad N_a . grad N_b,
    with every integral factorised into exact 1-D integrals of linear hat functions."""
    nu = Fraction(nu).limit_denominator(1000)
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    F = Fraction

    def i1(ia, ib, da, db):
        # int_0^1 phi_ia^(da) phi_ib^(db) dt, phi_0 = 1 - t, phi_1 = t
        if da and db:
            return F(1) if ia == ib else F(-1)
        if da:
            return F(1, 2) * (1 if ia else -1)
        if db:
            return F(1, 2) * (1 if ib else -1)
        return F(1, 3) if ia == ib else F(1, 6)

    def g(a, b, p, q):
        # int dN_a/dx_p * dN_b/dx_q over the unit cube
        ia = [(a >> s) & 1 for s in range(3)]
        ib = [(b >> s) & 1 for s in range(3)]
        out = F(1)
        for ax in range(3):
            out *= i1(ia[ax], ib[ax], ax == p, ax == q)
        return out

    K = [[F(0)] * 24 for _ in range(24)]
    for a, b, c, d in itertools.product(range(8), range(8), range(3), range(3)):
        v = lam * g(a, b, c, d) + mu * g(a, b, d, c)
        if c == d:
            v += mu * sum(g(a, b, k, k) for k in range(3))
        K[3 * a + c][3 * b + d] = v
    return np.array([[float(x) for x in row] for row in K])


def test_k0_matches_exact_index_form():
    K = element.k0(NU)
    Kx = k0_index_form_exact(NU)
    assert np.max(np.abs(K - Kx)) < 1e-15 * np.max(np.abs(Kx)) * 10


def test_k0_closed_form_entries():
    lam, mu = lame(NU)
    K = element.k0(NU)
    for a in range(8):
        for c in range(3):
            assert K[3 * a + c, 3 * a + c] == pytest.approx((lam + 4 * mu) / 9, abs=1e-15)
    assert K[0, 3] == pytest.approx(-(lam + mu) / 9, abs=1e-15)   # ux_000, ux_100
    assert K[0, 1] == pytest.approx((lam + mu) / 12, abs=1e-15)   # ux_000, uy_000
    assert np.trace(K) == pytest.approx(24 * (lam + 4 * mu) / 9, rel=1e-14)
    assert K[0, 0] == pytest.approx(0.235043, abs=1e-6)
    assert K[0, 3] == pytest.approx(-0.106838, abs=1e-6)
    assert K[0, 1] == pytest.approx(0.080128, abs=1e-6)


def test_k0_symmetric_psd_rank18_rigid_null_space():
    K = element.k0(NU)
    assert np.allclose(K, K.T, atol=0, rtol=0)
    ev = np.linalg.eigvalsh(K)
    assert ev[:6].max() < 1e-14 and ev[:6].min() > -1e-14
    assert ev[6] > 1e-2
    # rigid-body modes built here, not taken from the oracle
    X = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    modes = []
    for c in range(3):
        v = np.zeros(24)
        v[c::3] = 1.0
        modes.append(v)
    for w in np.eye(3):
        v = np.cross(np.broadcast_to(w, X.shape), X).ravel()
        modes.append(v)
    R = np.stack(modes, 1)
    assert np.linalg.matrix_rank(R) == 6
    assert np.max(np.abs(K @ R)) < 1e-14
    # a pure stretch is not in the null space
    s = np.zeros(24)
    s[0::3] = X[:, 0]
    assert s @ K @ s > 1e-2


def test_gauss_orders_agree():
    assert np.max(np.abs(element.k0(NU, order=2) - element.k0(NU, order=3))) < 1e-15


def test_k0_reflection_symmetry():
    """K0 commutes with the cube's mirror maps (node flip x component sign)."""
    K = element.k0(NU)
    for ax in range(3):
        P = np.zeros((24, 24))
        for a in range(8):
            b = a ^ (1 << ax)
            for c in range(3):
                P[3 * b + c, 3 * a + c] = -1.0 if c == ax else 1.0
        assert np.max(np.abs(P @ K @ P.T - K)) < 1e-15


def test_k0_scales_linearly_with_E():
    assert np.allclose(element.k0(NU, E=2.5), 2.5 * element.k0(NU), rtol=1e-15, atol=1e-16)
