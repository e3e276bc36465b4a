"""Pins for compliance, sensitivities (self-adjoint compliance), the filters of
paper Eq. (3)-(5) and the OC update."""
import math

import numpy as np
import pytest

import synth
from oracle import amr, mesh as om, system as osys, topopt


def _small_problem(dims=(4, 2, 2), seed=0):
    m = om.uniform_mesh(dims)
    rho = np.random.default_rng(seed).uniform(0.2, 1.0, m.n_elems)
    fx, ld = synth.cantilever_bc(*dims)
    return m, rho, om.fixed_dofs(m, fx), om.load_vector(m, ld)


def _compliance(m, rho, fixed, f):
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, f)
    return f @ osys.recover(s, osys.solve_direct(s))


def test_sensitivity_matches_central_differences():
    m, rho, fixed, f = _small_problem()
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, f)
    u = osys.recover(s, osys.solve_direct(s))
    dc = topopt.sensitivities(m, rho, u)
    assert (dc <= 0).all()
    h = 1e-5
    for e in [0, 3, 7, 12, 15]:
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (_compliance(m, rp, fixed, f) - _compliance(m, rm, fixed, f)) / (2 * h)
        assert dc[e] == pytest.approx(fd, rel=1e-6)


def test_sensitivity_on_amr_mesh_matches_fd():
    l, a = np.array([0, 0]), np.array([[0, 0, 0], [2, 0, 0]])
    l, a, _ = amr.refine(l, a, 1, np.array([True, False]))
    m = om.build_mesh(l, a, 1, (4, 2, 2))
    rho = np.random.default_rng(1).uniform(0.2, 1.0, m.n_elems)
    fx, ld = synth.cantilever_bc(4, 2, 2)
    fixed, f = om.fixed_dofs(m, fx), om.load_vector(m, ld)
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, f)
    u = osys.recover(s, osys.solve_direct(s))
    dc = topopt.sensitivities(m, rho, u)
    for e in range(m.n_elems):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += 1e-5
        rm[e] -= 1e-5
        fd = (_compliance(m, rp, fixed, f) - _compliance(m, rm, fixed, f)) / 2e-5
        assert dc[e] == pytest.approx(fd, rel=1e-6)


def test_compliance_equals_sum_of_element_energies():
    m, rho, fixed, f = _small_problem(seed=2)
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, f)
    u = osys.recover(s, osys.solve_direct(s))
    w = topopt.element_energy(m, u)
    assert topopt.compliance(f, u) == pytest.approx(np.sum(osys.elem_coeff(m, rho) * w), rel=1e-12)


def test_filter_interior_weights_19_point_stencil():
    m = om.uniform_mesh((5, 5, 5))
    W = topopt.filter_weights(m, 1.5)
    e = 2 + 5 * (2 + 5 * 2)
    row = W[e].toarray().ravel()
    assert np.count_nonzero(row) == 19
    assert row.sum() == pytest.approx(22.5 - 12 * math.sqrt(2), rel=1e-14)
    assert row[e] == pytest.approx(1.5)
    assert sorted(set(np.round(row[row > 0], 12))) == sorted({1.5, 0.5, round(1.5 - math.sqrt(2), 12)})


def test_filter_fixed_points():
    m = om.uniform_mesh((6, 3, 3))
    x = np.full(m.n_elems, 0.37)
    assert np.allclose(topopt.filter_density(m, 1.5, x), x, rtol=1e-14)
    dc = np.full(m.n_elems, -2.0)
    assert np.allclose(topopt.filter_sensitivity(m, 1.5, x, dc), dc, rtol=1e-14)


def test_filter_inactive_for_coarse_elements():
    """Eq. (5) with r_min smaller than the element size leaves dc unchanged."""
    l = np.zeros(8, int)
    a = np.array([[i, j, k] for k in (0, 2) for j in (0, 2) for i in (0, 2)])
    m = om.build_mesh(l, a, 1, (4, 4, 4))
    rho = np.random.default_rng(0).uniform(0.1, 1, 8)
    dc = -np.random.default_rng(1).uniform(0.1, 1, 8)
    assert np.allclose(topopt.filter_sensitivity(m, 1.5, rho, dc), dc, rtol=1e-14)


def test_filter_volume_weighting_against_brute_force():
    l, a = np.array([0, 0]), np.array([[0, 0, 0], [2, 0, 0]])
    l, a, _ = amr.refine(l, a, 1, np.array([True, False]))
    m = om.build_mesh(l, a, 1, (4, 2, 2))
    rng = np.random.default_rng(5)
    rho, dc = rng.uniform(0.1, 1, m.n_elems), -rng.uniform(0.1, 1, m.n_elems)
    out = topopt.filter_sensitivity(m, 2.2, rho, dc)
    cen, V = m.centres, m.volumes
    for e in range(m.n_elems):
        num = den = 0.0
        for d in range(m.n_elems):
            H = max(2.2 - math.dist(cen[e], cen[d]), 0.0)
            num += rho[d] * H * V[d] * dc[d]
            den += H * V[d]
        assert out[e] == pytest.approx(num / (rho[e] * den), rel=1e-13)


def test_oc_volume_bounds_and_closed_form():
    rng = np.random.default_rng(0)
    n = 500
    rho = rng.uniform(0.2, 0.8, n)
    dc = -rng.uniform(0.5, 2.0, n)
    vol = np.ones(n)
    v0 = 0.5 * n
    new, lam, ch = topopt.oc_update(rho, dc, vol, v0)
    assert new @ vol == pytest.approx(v0, rel=1e-12)
    assert (new >= np.maximum(1e-3, rho - 0.2) - 1e-15).all()
    assert (new <= np.minimum(1.0, rho + 0.2) + 1e-15).all()
    # with no active bound the multiplier has a closed form
    new2, lam2, _ = topopt.oc_update(rho, dc, vol, v0, move=10.0, rho_min=1e-12)
    g = -dc
    if (new2 < 1.0).all():
        lam_exact = (np.sum(rho * np.sqrt(g) * vol) / v0) ** 2
        assert lam2 == pytest.approx(lam_exact, rel=1e-11)
        assert np.allclose(new2, rho * np.sqrt(g / lam_exact), rtol=1e-11)
    # monotone in -dc for equal rho
    r = np.full(n, 0.5)
    out, _, _ = topopt.oc_update(r, dc, vol, 0.5 * n)
    order = np.argsort(-dc)
    assert (np.diff(out[order]) >= -1e-15).all()
