"""Pins for the reference mesh <-> grid transfers: constants and linear
fields are reproduced exactly, and the dual cells partition the domain so the
grid density conserves mass."""
import numpy as np
import pytest

from oracle import amr, grid, mesh as om


def small_octree(base=(4, 2, 2), L=2, seed=0):
    rng = np.random.default_rng(seed)
    b = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])]) << L
    lv, an = np.zeros(len(b), np.int64), b
    for _ in range(L):
        lv, an, _ = amr.refine(lv, an, L, rng.random(len(lv)) < 0.3)
    lv, an, _ = amr.balance(lv, an, L)
    dims = tuple(x << L for x in base)
    return om.build_mesh(lv, an, L, dims)


@pytest.mark.parametrize("cell", [1, 2, 4, 3])
def test_density_constant_and_mass(cell):
    m = small_octree() if cell != 3 else om.uniform_mesh((6, 3, 9))
    assert all(d % cell == 0 for d in m.dims)
    g = grid.grid_density(m, np.full(m.n_elems, 0.37), cell)
    assert np.allclose(g, 0.37, atol=1e-15)
    rho = np.random.default_rng(1).random(m.n_elems)
    g = grid.grid_density(m, rho, cell)
    # dual cell volumes: half cells at the domain faces
    vol = np.ones_like(g)
    for ax, n in zip((2, 1, 0), m.dims):
        w = np.full(n // cell + 1, float(cell))
        w[0] = w[-1] = cell / 2
        shape = [1, 1, 1]
        shape[ax] = -1
        vol = vol * w.reshape(shape)
    assert np.isclose(vol.sum(), np.prod(m.dims))
    assert np.isclose((g * vol).sum(), (rho * m.volumes).sum(), rtol=1e-13)


def test_density_single_element():
    m = om.uniform_mesh((4, 4, 4))
    rho = np.zeros(m.n_elems)
    rho[(1 * 4 + 1) * 4 + 1] = 1.0          # element [1,2)^3
    g = grid.grid_density(m, rho, 2)        # node (1,1,1) at 2: dual box [1,3)^3
    assert g[1, 1, 1] == pytest.approx(1.0 / 8)
    assert g[0, 0, 0] == pytest.approx(0.0)  # box [0,1)^3 does not reach it
    assert g.sum() == pytest.approx(1.0 / 8)


@pytest.mark.parametrize("cell", [1, 2, 4])
def test_linear_fields_exact(cell):
    m = small_octree(seed=3)
    A = np.array([[0.3, -1.0, 0.2], [0.5, 0.1, -0.7], [-0.2, 0.4, 0.9]])
    c = np.array([0.1, -0.2, 0.3])
    u = (m.coords @ A.T + c).ravel()
    ug = grid.grid_sample(m, u, cell, scale=2.0)
    pts = grid.grid_points(m.dims, cell)
    want = 2.0 * (pts @ A.T + c)
    assert np.allclose(ug.reshape(3, -1).T, want, atol=1e-12)
    back = grid.grid_interp(ug, cell, m.coords, scale=0.5)
    assert np.allclose(back, u, atol=1e-12)
