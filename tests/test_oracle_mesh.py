"""Pins for the oracle's mesh, hanging-node interpolation (paper Sec. 6,
Eq. (6)-(9)), supports, loads and solves."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amr, element, mesh as om, system as osys


def two_level_leaves():
    """2x1x1 base of edge-2 leaves; the first is split into 8 unit leaves."""
    level = np.array([0, 0])
    anchor = np.array([[0, 0, 0], [2, 0, 0]])
    l, a, _ = amr.refine(level, anchor, 1, np.array([True, False]))
    return l, a, 1, (4, 2, 2)


def test_uniform_numbering_is_lexicographic():
    m = om.uniform_mesh((3, 2, 2))
    nx, ny = 4, 3
    for n, (x, y, z) in enumerate(m.coords):
        assert n == x + nx * (y + ny * z)
    e = 1 + 3 * (1 + 2 * 1)
    assert list(m.elem_nodes[e]) == [x + nx * (y + ny * z) for z in (1, 2) for y in (1, 2) for x in (1, 2)]
    assert not m.hanging.any()


def test_hanging_nodes_of_one_refined_leaf():
    l, a, L, dims = two_level_leaves()
    m = om.build_mesh(l, a, L, dims)
    h = np.nonzero(m.hanging)[0]
    assert len(h) == 5                      # 4 edge midpoints + 1 face centre on x = 2
    T = m.Tn.toarray()
    for n in h:
        x, y, z = m.coords[n]
        assert x == 2
        w = T[n][T[n] != 0]
        if y == 1 and z == 1:
            assert np.allclose(sorted(w), [0.25] * 4)
        else:
            assert np.allclose(sorted(w), [0.5, 0.5])
        assert w.sum() == pytest.approx(1.0)
        # masters are corners of the coarse face
        for mm in np.nonzero(T[n])[0]:
            assert m.coords[mm][0] == 2 and m.coords[mm][1] in (0, 2) and m.coords[mm][2] in (0, 2)


def test_chained_hanging_nodes_resolve_to_unconstrained():
    # 3 levels: refine leaf 0 of a 2x1x1 base twice at the corner touching leaf 1
    level = np.array([0, 0])
    anchor = np.array([[0, 0, 0], [4, 0, 0]])
    l, a, _ = amr.refine(level, anchor, 2, np.array([True, False]))
    sel = np.zeros(len(l), bool)
    sel[np.nonzero((a[:, 0] == 2) & (a[:, 1] == 2) & (a[:, 2] == 2) & (l == 1))[0]] = True
    l, a, _ = amr.refine(l, a, 2, sel)
    l, a, _ = amr.balance(l, a, 2)
    m = om.build_mesh(l, a, 2, (8, 4, 4))
    T = m.Tn.tocsr()
    for hnode in np.nonzero(m.hanging)[0]:
        cols = T.indices[T.indptr[hnode]:T.indptr[hnode + 1]]
        assert not m.hanging[cols].any()
        assert T[hnode].sum() == pytest.approx(1.0)


def test_all_same_level_octree_equals_uniform_grid():
    base = np.array([[i, j, k] for k in range(2) for j in range(1) for i in range(2)]) * 2
    l, a, _ = amr.refine(np.zeros(len(base), int), base, 1, np.ones(len(base), bool))
    m1 = om.build_mesh(l, a, 1, (4, 2, 4))
    m2 = om.uniform_mesh((4, 2, 4))
    assert (m1.coords == m2.coords).all()
    assert not m1.hanging.any()
    # same elements (up to element order): compare node sets keyed by anchor
    k1 = {tuple(x): tuple(n) for x, n in zip(m1.anchor, m1.elem_nodes)}
    k2 = {tuple(x): tuple(n) for x, n in zip(m2.anchor, m2.elem_nodes)}
    assert k1 == k2


def _linear_field(coords, A, b):
    return (coords @ A.T + b).ravel()


@pytest.mark.parametrize("amr_mesh", [False, True])
def test_patch_test_linear_field(amr_mesh):
    """Linear displacement fields are reproduced exactly: P interpolates them,
    the interior equilibrium residual vanishes, and a Dirichlet solve with the
    linear field on the boundary returns it everywhere (across hanging nodes)."""
    if amr_mesh:
        l, a, L, dims = two_level_leaves()
        l, a, _ = amr.refine(l, a, L, np.zeros(len(l), bool))
        m = om.build_mesh(l, a, L, dims)
        assert m.hanging.any()
    else:
        m = om.uniform_mesh((3, 2, 2))
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    u = _linear_field(m.coords.astype(float), A, b)
    T = osys.dof_interp(m)
    unc = ~np.repeat(m.hanging, 3)
    assert np.max(np.abs(T @ np.where(unc, u, 0.0) - u)) < 1e-12
    c = np.ones(m.n_elems) * m.size
    K = osys.assemble(m, c)
    r = T.T @ (K @ u)
    dims = np.array(m.dims)
    interior = ((m.coords > 0) & (m.coords < dims)).all(axis=1)
    rows = np.repeat(interior & ~m.hanging, 3)
    assert np.max(np.abs(r[rows])) < 1e-12
    # Dirichlet solve: boundary nodes prescribed, interior unknown
    bnd = np.repeat(~interior, 3)
    A_ = (T.T @ K @ T).tocsr()
    free = unc & ~bnd
    fi = np.nonzero(free)[0]
    bi = np.nonzero(unc & bnd)[0]
    ub = np.where(unc & bnd, u, 0.0)
    if len(fi):
        sol = sp.linalg.spsolve(A_[fi][:, fi].tocsc(), -(A_[fi][:, bi] @ ub[bi]))
        ut = ub.copy()
        ut[fi] = sol
        assert np.max(np.abs(T @ ut - u)) < 1e-10


@pytest.mark.parametrize("amr_mesh", [False, True])
def test_uniaxial_stress_exact_solution(amr_mesh):
    """Roller supports on x=0 (u_x), y=0 (u_y), z=0 (u_z) and a unit traction
    on x = L: the exact solution u = (x, -nu y, -nu z) * sigma / E is linear,
    so Q1 elements reproduce it exactly - including across hanging nodes."""
    if amr_mesh:
        l, a, L, dims = two_level_leaves()
        m = om.build_mesh(l, a, L, dims)
    else:
        m = om.uniform_mesh((4, 2, 2))
    nu, E = 0.3, 2.0
    X = m.coords.astype(float)
    fixed = np.zeros(3 * m.n_nodes, bool)
    fixed[0::3] = X[:, 0] == 0
    fixed[1::3] = X[:, 1] == 0
    fixed[2::3] = X[:, 2] == 0
    ny, nz = m.dims[1], m.dims[2]
    f = om.load_vector(m, {"kind": "face", "where": {"x": m.dims[0]}, "comp": 0,
                           "total": float(ny * nz)})            # traction sigma = 1
    coeff = E * m.size.astype(float)
    s = osys.build_system(m, coeff, fixed, f, nu=nu)
    u = osys.recover(s, osys.solve_direct(s))
    exact = np.stack([X[:, 0], -nu * X[:, 1], -nu * X[:, 2]], 1).ravel() / E
    assert np.max(np.abs(u - exact)) < 1e-11
    # compliance identities: f.u = u^T K u
    K = osys.assemble(m, coeff, nu=nu)
    assert f @ u == pytest.approx(u @ (K @ u), rel=1e-12)


def test_cantilever_direct_vs_pcg_and_mirror_symmetry():
    case = synth.c1(dims=(8, 4, 4))
    m = om.uniform_mesh(case.dims)
    # a density symmetric about the mid-plane y = W/2
    rho = case.rho.reshape(4, 4, 8)
    rho = 0.5 * (rho + rho[:, ::-1, :])
    rho = rho.ravel()
    fixed = om.fixed_dofs(m, case.fixed)
    f = om.load_vector(m, case.load)
    assert f.sum() == pytest.approx(-1.0)
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, f)
    ud = osys.solve_direct(s)
    r = osys.pcg_jacobi(s.A, s.b, rtol=1e-13)
    assert np.linalg.norm(r.x - ud) <= 1e-10 * np.linalg.norm(ud)
    u = osys.recover(s, ud).reshape(-1, 3)
    X = m.coords
    mirror = np.array([np.nonzero((X[:, 0] == x) & (X[:, 1] == 4 - y) & (X[:, 2] == z))[0][0]
                       for x, y, z in X])
    assert np.allclose(u[mirror, 0], u[:, 0], atol=1e-12 * np.abs(u).max())
    assert np.allclose(u[mirror, 2], u[:, 2], atol=1e-12 * np.abs(u).max())
    assert np.allclose(u[mirror, 1], -u[:, 1], atol=1e-12 * np.abs(u).max())
    # the tip moves down
    assert u[:, 2].min() < 0


def test_dense_cholesky_agrees_with_sparse_lu():
    m = om.uniform_mesh((3, 2, 2))
    rho = np.linspace(0.2, 1.0, m.n_elems)
    fx, ld = synth.cantilever_bc(3, 2, 2)
    s = osys.build_system(m, osys.elem_coeff(m, rho), om.fixed_dofs(m, fx), om.load_vector(m, ld))
    A = s.A.toarray()
    L = np.linalg.cholesky(A)
    x = np.linalg.solve(L.T, np.linalg.solve(L, s.b))
    assert np.allclose(x, osys.solve_direct(s), rtol=1e-12, atol=1e-14)


def test_apply_constrained_equals_assembled_operator():
    l, a, L, dims = two_level_leaves()
    m = om.build_mesh(l, a, L, dims)
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.1, 1, m.n_elems)
    fx, ld = synth.cantilever_bc(*dims)
    fixed = om.fixed_dofs(m, fx)
    s = osys.build_system(m, osys.elem_coeff(m, rho), fixed, om.load_vector(m, ld))
    x = rng.normal(size=3 * m.n_nodes)
    y1 = s.A @ x
    y2 = osys.apply_constrained(m, osys.elem_coeff(m, rho), fixed, x)
    assert np.allclose(y1, y2, rtol=1e-13, atol=1e-13)
    assert abs(s.A - s.A.T).max() < 1e-15


def test_line_and_face_loads_on_amr_mesh():
    l, a, L, dims = two_level_leaves()
    m = om.build_mesh(l, a, L, dims)
    f = om.load_vector(m, {"kind": "face", "where": {"z": 2}, "comp": 2, "total": -1.0})
    assert f.sum() == pytest.approx(-1.0)
    # total top area 8; the nodes with x < 2 collect 3 of the 4 fine faces'
    # area units (the column x in [1, 2] hands half of its area to x = 2)
    top_fine = (m.coords[:, 2] == 2) & (m.coords[:, 0] < 2)
    assert f[2::3][top_fine].sum() == pytest.approx(-3.0 / 8.0, rel=1e-14)
    # the face centre hanging node (2, 1, 2) gets 4 fine quarter-faces / 8
    hc = np.nonzero((m.coords == [2, 1, 2]).all(1))[0][0]
    assert m.hanging[hc] and f[3 * hc + 2] == pytest.approx(-2 * 0.25 / 8.0, rel=1e-14)
    g = om.load_vector(m, {"kind": "line", "where": {"x": 4, "z": 0}, "comp": 2, "total": -1.0})
    assert g.sum() == pytest.approx(-1.0)
    assert np.count_nonzero(g) == 2
