"""Pins of the multigrid oracle (oracle/mg.py) against what the mathematics
fixes: merged leaf sets tile the domain and keep the one-level rule; the
prolongation reproduces linear displacement fields exactly (nested spaces);
the Galerkin operator equals the coarse mesh's own stiffness matrix when the
density is constant on every coarse leaf; m Chebyshev steps damp each
eigencomponent by the scaled Chebyshev polynomial; one V-cycle is a symmetric
positive definite operator whose two-grid error propagation contracts in the
energy norm; and CG preconditioned by it reaches the direct solution.  The
node-block smoother (level 0 smoothing with the inverse 3 x 3 node blocks)
is pinned by its layout on random non-symmetric blocks, by reducing exactly
to the diagonal smoother when every node block is diagonal, by keeping the
V-cycle symmetric and contracting, and by reaching the direct solution in
fewer iterations than the diagonal smoother."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amr, mg
from oracle import mesh as om
from oracle import system as osys


def band_tree(base, L, seed=0, p=0.35):
    """A cantilever octree refined at seeded random leaves, then closed."""
    case = synth.c2(base=base, max_level=L, seed=seed)
    rng = np.random.default_rng(seed)
    lv = np.zeros(int(np.prod(base)), np.int64)
    an = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])]) << L
    for _ in range(L):
        lv, an, _ = amr.refine(lv, an, L, rng.random(len(lv)) < p)
    lv, an, _ = amr.balance(lv, an, L)
    return case, lv, an


@pytest.fixture(scope="module")
def small():
    case, lv, an = band_tree((4, 2, 2), 2)
    m0 = om.build_mesh(lv, an, 2, case.dims)
    assert m0.hanging.any()
    return case, m0


def test_coarsened_leaves_tile_the_domain_and_stay_balanced(small):
    case, m0 = small
    vol = float(np.prod(case.dims))
    for k in range(1, 4):
        c = mg.coarsen_leaves(m0.level, m0.anchor, m0.max_level, case.base, k)
        assert c is not None
        lv, an, ml = c
        s = om.leaf_sizes(lv, ml)
        assert float((s.astype(float) ** 3).sum()) == vol
        if k <= m0.max_level:
            assert amr.is_balanced(lv, an, ml)
            assert lv.max() <= m0.max_level - k
        else:
            assert (s == 1 << k).all()
    # (4, 2, 2) cannot be halved three times beyond the base grid
    assert mg.coarsen_leaves(m0.level, m0.anchor, m0.max_level, case.base, 2 + 3) is None


def test_hierarchy_stops_at_a_small_uniform_level(small):
    case, m0 = small
    levels = mg.hierarchy(m0, case.base, case.fixed, coarse_dofs=100)
    assert not levels[-1].mesh.hanging.any()
    assert 3 * levels[-1].mesh.n_nodes <= 100 or mg.coarsen_leaves(
        m0.level, m0.anchor, m0.max_level, case.base, len(levels)) is None
    assert all(3 * a.mesh.n_nodes > 3 * b.mesh.n_nodes for a, b in zip(levels, levels[1:]))


@pytest.mark.parametrize("first", [1, 2])
def test_prolongation_reproduces_linear_fields(small, first):
    case, m0 = small
    levels = mg.hierarchy(m0, case.base, [], coarse_dofs=100, first=first)   # no supports: any field
    rng = np.random.default_rng(3)
    G = rng.standard_normal((3, 3))
    c0 = rng.standard_normal(3)
    for f, c in zip(levels, levels[1:]):
        P = mg.prolongation(f, c)
        uc = (c.mesh.coords @ G.T + c0).ravel() * c.free       # constrained form: zero at hanging DOFs
        uf = (f.mesh.coords @ G.T + c0).ravel() * f.free
        assert np.abs(P @ uc - uf).max() <= 1e-12 * np.abs(uf).max()


@pytest.mark.parametrize("first", [1, 2])
def test_galerkin_equals_coarse_stiffness_for_coarse_constant_density(small, first):
    case, m0 = small
    levels = mg.hierarchy(m0, case.base, case.fixed, coarse_dofs=100, first=first)
    f, c = levels[0], levels[1]
    rng = np.random.default_rng(4)
    rho_c = rng.uniform(0.1, 1.0, c.mesh.n_elems)
    # every fine leaf takes the density of the coarse leaf containing it
    idx = om.LeafIndex(c.mesh.level, c.mesh.anchor, c.mesh.max_level)
    rho_f = rho_c[idx.find(f.mesh.centres)]
    A0 = osys.build_system(f.mesh, osys.elem_coeff(f.mesh, rho_f), f.fixed, np.zeros(3 * f.mesh.n_nodes)).A
    Ac = mg.galerkin(A0, mg.prolongation(f, c), c.free)
    A1 = osys.build_system(c.mesh, osys.elem_coeff(c.mesh, rho_c), c.fixed, np.zeros(3 * c.mesh.n_nodes)).A
    assert abs(Ac - A1).max() <= 1e-12 * abs(A1).max()
    # a dropped interpolation weight or a transposed P breaks it
    P_bad = mg.prolongation(f, c).copy()
    r0 = int(np.argmax(np.diff(P_bad.indptr)))
    P_bad.data[P_bad.indptr[r0]] *= 0.5
    assert abs(mg.galerkin(A0, P_bad, c.free) - A1).max() > 1e-6 * abs(A1).max()


def test_chebyshev_damping_is_the_scaled_chebyshev_polynomial():
    rng = np.random.default_rng(5)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(0.05, 2.0, n)
    A = sp.csr_matrix(Q @ np.diag(lam) @ Q.T)
    lo, hi, m = 0.2, 2.1, 3
    x_true = rng.standard_normal(n)
    b = A @ x_true
    x, r = mg.chebyshev(A, np.ones(n), b, np.zeros(n), lo, hi, m)
    assert np.allclose(r, b - A @ x, atol=1e-12)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tm = np.polynomial.chebyshev.Chebyshev.basis(m)
    damp = Tm((theta - lam) / delta) / Tm(theta / delta)
    e0 = Q.T @ x_true
    assert np.allclose(Q.T @ (x_true - x), damp * e0, atol=1e-12)


def _vcycle_matrix(M, n):
    return np.stack([M.vcycle(np.eye(n)[i]) for i in range(n)], 1)


def test_node_block_layout():
    rng = np.random.default_rng(3)
    blocks = rng.standard_normal((5, 3, 3))
    x = rng.standard_normal(15)
    want = np.einsum("nij,nj->ni", blocks, x.reshape(5, 3)).ravel()
    assert np.allclose(mg.block_diag_matrix(blocks) @ x, want, rtol=1e-15, atol=1e-15)
    A = mg.block_diag_matrix(blocks) + sp.identity(15)
    assert np.array_equal(mg.node_blocks(A), blocks + np.eye(3))


def test_block_smoothing_reduces_to_diagonal_for_diagonal_node_blocks():
    # SPD matrix whose node blocks are diagonal: a 1-D Laplacian coupling
    # nodes, acting on each component separately, plus a diagonal shift
    n = 12
    T = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    shift = np.random.default_rng(4).uniform(0.5, 2.0, 3 * n)
    A = (sp.kron(T, sp.identity(3)) + sp.diags(shift)).tocsr()
    dinv = 1.0 / A.diagonal()
    binv = mg.block_diag_matrix(np.linalg.inv(mg.node_blocks(A)))
    assert mg.lambda_max(A, binv) == pytest.approx(mg.lambda_max(A, dinv), rel=1e-12)
    b = np.random.default_rng(5).standard_normal(3 * n)
    hi = 1.1 * mg.lambda_max(A, dinv)
    xd, rd = mg.chebyshev(A, dinv, b, np.zeros(3 * n), hi / 10, hi, 3)
    xb, rb = mg.chebyshev(A, binv, b, np.zeros(3 * n), hi / 10, hi, 3)
    assert np.allclose(xb, xd, rtol=1e-13, atol=1e-13) and np.allclose(rb, rd, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("blocks0", [False, True])
def test_vcycle_is_spd_and_two_grid_contracts(blocks0):
    case, lv, an = band_tree((2, 2, 2), 1)
    m0 = om.build_mesh(lv, an, 1, case.dims)
    rho = np.random.default_rng(6).uniform(0.05, 1.0, m0.n_elems)
    fx = om.fixed_dofs(m0, case.fixed)
    A = osys.build_system(m0, osys.elem_coeff(m0, rho), fx, np.zeros(3 * m0.n_nodes)).A
    levels = mg.hierarchy(m0, case.base, case.fixed, coarse_dofs=30)
    assert len(levels) >= 2
    M = mg.setup(levels, A, degree=2, blocks0=blocks0)
    n = A.shape[0]
    V = _vcycle_matrix(M, n)
    assert np.abs(V - V.T).max() <= 1e-10 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    # error propagation I - V A contracts in the A-norm: eigenvalues of V A in (0, 2)
    w = np.linalg.eigvals(V @ A.toarray()).real
    assert w.min() > 0 and w.max() < 2


def test_mg_pcg_reaches_the_direct_solution(small):
    case, m0 = small
    rho = np.maximum(np.clip(case.extra["field"](m0.centres), 0, 1), 1e-3)
    fx = om.fixed_dofs(m0, case.fixed)
    f = om.load_vector(m0, case.load)
    s = osys.build_system(m0, osys.elem_coeff(m0, rho), fx, f)
    levels = mg.hierarchy(m0, case.base, case.fixed, coarse_dofs=100)
    M = mg.setup(levels, s.A)
    r = mg.mg_pcg(s.A, s.b, M, rtol=1e-10)
    u = osys.solve_direct(s)
    assert np.abs(r.x - u).max() <= 1e-8 * np.abs(u).max()
    assert r.iters < osys.pcg_jacobi(s.A, s.b, rtol=1e-10).iters / 3
    # node-block smoothing on level 0: the same solution in fewer iterations
    levels_b = mg.hierarchy(m0, case.base, case.fixed, coarse_dofs=100)
    rb = mg.mg_pcg(s.A, s.b, mg.setup(levels_b, s.A, blocks0=True), rtol=1e-10)
    assert np.abs(rb.x - u).max() <= 1e-8 * np.abs(u).max()
    assert rb.iters < r.iters
