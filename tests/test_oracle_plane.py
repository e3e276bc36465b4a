"""Pins of the 2-D oracle (oracle/plane.py) against what the mathematics fixes:
K0 against hand-computed entries and an exact index-form integration (not the
Gauss rule), its rank and rigid modes; a linear displacement field reproduced
across hanging nodes (patch test); a quadtree refined everywhere equal to the
uniform grid; the Eq. (5) filter stencil sum; the compliance identity; the
quadtree closure (balanced, minimal) and the marking rule by brute force; the
density transfer conserving the material area."""
import itertools

import numpy as np
import pytest

from oracle import plane
from oracle.topopt import oc_update


def _index_form_k0(nu):
    """K[(a,c),(b,d)] = int D-weighted products of exact 1-D integrals of linear
    shape functions and their derivatives on [0, 1]."""
    lam_ps = nu / (1 - nu * nu)            # plane-stress D12
    d11 = 1.0 / (1 - nu * nu)
    g = (1 - nu) / (2 * (1 - nu * nu))     # D33

    def one_d(ia, ib, da, db):
        if da and db:
            return 1.0 if ia == ib else -1.0
        if da:
            return 0.5 if ia else -0.5
        if db:
            return 0.5 if ib else -0.5
        return 1 / 3 if ia == ib else 1 / 6

    def I(a, b, p, q):  # int dN_a/dx_p dN_b/dx_q
        ia, ja, ib, jb = a & 1, a >> 1, b & 1, b >> 1
        return one_d(ia, ib, p == 0, q == 0) * one_d(ja, jb, p == 1, q == 1)

    K = np.zeros((8, 8))
    for a in range(4):
        for b in range(4):
            K[2 * a, 2 * b] = d11 * I(a, b, 0, 0) + g * I(a, b, 1, 1)
            K[2 * a + 1, 2 * b + 1] = d11 * I(a, b, 1, 1) + g * I(a, b, 0, 0)
            K[2 * a, 2 * b + 1] = lam_ps * I(a, b, 0, 1) + g * I(a, b, 1, 0)
            K[2 * a + 1, 2 * b] = lam_ps * I(a, b, 1, 0) + g * I(a, b, 0, 1)
    return K


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_k0_index_form_rank_and_rigid_modes(nu):
    K = plane.k0(nu)
    assert np.allclose(K, _index_form_k0(nu), atol=1e-15)
    assert np.allclose(K, K.T)
    w = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(w) < 1e-12) == 3 and w.min() > -1e-14
    assert np.abs(K @ plane.rigid_modes()).max() < 1e-14


def test_k0_hand_entries():
    # nu = 0.3: K[ux0,ux0] = (1/2 - nu/6)/(1 - nu^2), K[ux0,uy0] = (1 + nu)/8/(1 - nu^2)
    K = plane.k0(0.3)
    assert K[0, 0] == pytest.approx((0.5 - 0.05) / 0.91, abs=1e-15)
    assert K[0, 1] == pytest.approx(1.3 / 8 / 0.91, abs=1e-15)
    # node 0 -> node 3 (the opposite corner), ux-ux: (-1/6 - (1 - nu)/12) / (1 - nu^2) = (-1/4 + nu/12) / (1 - nu^2)
    assert K[0, 6] == pytest.approx((-0.25 + 0.3 / 12) / 0.91, abs=1e-15)


def _tree(base, L, marks_per_round):
    lv, an = plane.base_leaves(base, L)
    for m in marks_per_round:
        lv, an, _ = plane.refine(lv, an, L, m(lv, an))
    return plane.balance(lv, an, L)[:2]


def test_patch_test_across_hanging_nodes():
    L = 2
    lv, an = _tree((3, 2), L, [lambda lv, an: (an[:, 0] == 4) & (an[:, 1] == 0),
                                 lambda lv, an: (lv == 1) & (an[:, 0] == 4)])
    m = plane.build_mesh(lv, an, L, (12, 8))
    assert m.hanging.any()
    G = np.array([[0.01, -0.02], [0.03, 0.005]])
    u = (m.coords @ G.T + np.array([0.1, -0.2])).ravel()
    # one material (constant strain gives constant stress only then)
    K = plane.assemble(m, plane.young(np.full(m.n_elems, 0.6)))
    T = __import__("scipy.sparse", fromlist=["kron"]).kron(m.Tn, np.eye(2), format="csr")
    # the linear field is exactly representable: u = T u~ with u~ = u on unconstrained nodes
    ut = np.where(np.repeat(m.hanging, 2), 0.0, u)
    assert np.allclose(T @ ut, u, atol=1e-14)
    r = T.T @ (K @ u)
    boundary = np.repeat((m.coords[:, 0] == 0) | (m.coords[:, 0] == 12) | (m.coords[:, 1] == 0)
                         | (m.coords[:, 1] == 8), 2)
    interior = ~boundary & ~np.repeat(m.hanging, 2)
    assert np.abs(r[interior]).max() < 1e-13


def test_refined_everywhere_equals_uniform():
    L = 1
    lv, an = plane.base_leaves((3, 2), L)
    lv, an, _ = plane.refine(lv, an, L, np.ones(len(lv), bool))
    m = plane.build_mesh(lv, an, L, (6, 4))
    u = plane.build_mesh(*plane.uniform_leaves((6, 4))[:2], 0, (6, 4))
    assert not m.hanging.any()
    key = {tuple(c): i for i, c in enumerate(u.coords.tolist())}
    perm = np.array([key[tuple(c)] for c in m.coords.tolist()])
    rho_u = np.random.default_rng(1).uniform(0.1, 1, u.n_elems)
    ekey = {tuple(a): e for e, a in enumerate(u.anchor.tolist())}
    rho_m = rho_u[[ekey[tuple(a)] for a in m.anchor.tolist()]]
    Km = plane.assemble(m, plane.young(rho_m)).toarray()
    Ku = plane.assemble(u, plane.young(rho_u)).toarray()
    dp = (2 * perm[:, None] + np.arange(2)).ravel()
    assert np.allclose(Km, Ku[np.ix_(dp, dp)], atol=1e-14)


def test_filter_stencil_sum_and_constants():
    m = plane.build_mesh(*plane.uniform_leaves((9, 9))[:2], 0, (9, 9))
    W = plane.filter_weights(m, 1.5)
    centre = 4 + 9 * 4
    assert W[centre].sum() == pytest.approx(9.5 - 4 * np.sqrt(2), abs=1e-14)
    rho = np.full(m.n_elems, 0.7)
    dc = np.full(m.n_elems, -2.0)
    assert np.allclose(plane.filter_sensitivity(m, 1.5, rho, dc), -2.0, atol=1e-14)


def test_direct_solve_and_compliance_identity():
    lv, an = _tree((4, 2), 1, [lambda lv, an: an[:, 0] >= 4])
    m = plane.build_mesh(lv, an, 1, (8, 4))
    fixed = plane.fixed_dofs(m, [{"x": 0}])
    f = plane.load_vector(m, {"at": (8, 0), "comp": 1, "total": -1.0})
    rho = np.random.default_rng(2).uniform(0.2, 1.0, m.n_elems)
    s = plane.build_system(m, plane.young(rho), fixed, f)
    u = plane.solve_direct(s)
    K = plane.assemble(m, plane.young(rho))
    assert f @ u == pytest.approx(u @ (K @ u), rel=1e-10)
    dc = plane.sensitivities(m, rho, u)
    assert np.all(dc <= 0)
    # Euler identity: sum rho dc = -p sum rho^p (E0 - Emin) w_e
    ue = u[plane.elem_dofs(m)]
    w = np.einsum("ei,ij,ej->e", ue, plane.k0(), ue)
    assert rho @ dc == pytest.approx(-3 * (rho ** 3 * (1 - 1e-9)) @ w, rel=1e-12)


def test_balance_is_balanced_and_minimal():
    L = 3
    rng = np.random.default_rng(3)
    for _ in range(3):
        lv, an = plane.base_leaves((2, 2), L)
        for _ in range(L):
            lv, an, _ = plane.refine(lv, an, L, rng.random(len(lv)) < 0.3)
        orig = {(int(l), int(a[0]), int(a[1])) for l, a in zip(lv, an)}
        bl, ba, _ = plane.balance(lv, an, L)
        assert plane.is_balanced(bl, ba, L)
        # minimal: merging any family the closure created breaks balance
        new = {(int(l), int(a[0]), int(a[1])) for l, a in zip(bl, ba)} - orig
        fams = {}
        for (l, x, y) in new:
            ps = 1 << (L - l + 1)
            fams.setdefault((l - 1, x // ps * ps, y // ps * ps), []).append((l, x, y))
        leaves = {(int(l), int(a[0]), int(a[1])) for l, a in zip(bl, ba)}
        for (pl, px, py), kids in fams.items():
            if len(kids) != 4:
                continue
            undone = (leaves - set(kids)) | {(pl, px, py)}
            ul = np.array([k[0] for k in undone])
            ua = np.array([[k[1], k[2]] for k in undone])
            assert not plane.is_balanced(ul, ua, L)


def test_marking_brute_force():
    L = 1
    lv, an = plane.base_leaves((3, 1), L)
    lv, an, _ = plane.refine(lv, an, L, np.array([True, False, False]))
    # fine leaves at anchors (0,0),(1,0),(0,1),(1,1); coarse leaves at (2,0),(4,0)
    rho = np.zeros(len(lv))
    solid = np.nonzero((an[:, 0] == 1) & (an[:, 1] == 0) & (lv == 1))[0]
    rho[solid] = 0.9
    m = plane.mark(lv, an, L, rho, 0.5, 1.5)
    cen = an + 0.5 * plane.leaf_sizes(lv, L)[:, None]
    for i in range(len(lv)):
        d = np.linalg.norm(cen[i] - cen[solid[0]])
        want = 1 if d <= 1.5 else -1
        if want == 1 and lv[i] == L:
            want = 0
        if want == -1 and lv[i] == 0:
            want = 0
        assert m[i] == want


def test_adapt_conserves_material_and_balances():
    L = 2
    lv, an = plane.base_leaves((4, 2), L)
    lv, an, _ = plane.refine(lv, an, L, np.ones(len(lv), bool))
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.0, 0.4, len(lv))
    rho[:3] = 0.9
    nl, na, nr = plane.adapt(lv, an, L, rho)
    assert plane.is_balanced(nl, na, L)
    area = lambda l: (plane.leaf_sizes(l, L) ** 2).astype(float)
    assert nr @ area(nl) == pytest.approx(rho @ area(lv), rel=1e-14)
    assert area(nl).sum() == area(lv).sum()
    assert len(nl) < len(lv)  # the void families were derefined
