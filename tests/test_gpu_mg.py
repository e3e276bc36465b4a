"""The multigrid preconditioner on the GPU (amrto_mg_*) against the multigrid
oracle (oracle/mg.py) on the same meshes: level sizes, prolongation and
restriction, the Galerkin operators and their diagonals, one V-cycle with
the oracle's exact smoothing intervals, the power-iteration estimate of
lambda_max, and multigrid-preconditioned CG against the direct solve, on an
octree with hanging nodes and on a uniform brick.  Level-0 vectors are
matched by node coordinates; coarse levels number their nodes with x fastest
on both sides."""
import numpy as np
import pytest
import torch

from cases import centre_density, octree_pair, oracle_system, uniform_pair
from oracle import mg
from oracle import system as osys
from paper_1009_4975_amd import binding

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
COARSE = 200


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


class MgCase:
    def __init__(self, kind, first):
        if kind == "octree":
            self.pair = octree_pair((8, 4, 4), 2)
            self.base = (8, 4, 4)
            rho = np.clip(centre_density(self.pair, self.pair.case["field"]), 0.05, 1.0)
        else:
            self.pair = uniform_pair((24, 12, 12))
            self.base = (24, 12, 12)
            rho = np.random.default_rng(11).uniform(0.05, 1.0, self.pair.orc.n_elems)
        p = self.pair
        self.rho = rho
        self.ctx = binding.Context(0)
        self.ctx.upload_mesh(p.lib_mesh)
        self.ctx.set_density(_t(p.to_lib_elems(rho)))
        self.first = first
        self.ctx.mg_setup(p.case["tree"], coarse_dofs=COARSE, first=first)
        self.sys = oracle_system(p, rho)
        self.levels = mg.hierarchy(p.orc, self.base, p.case["fixed"], coarse_dofs=COARSE, first=first)
        self.M = mg.setup(self.levels, self.sys.A)
        self.dp = p.dof_perm  # library level-0 DOF -> oracle DOF

    def to_lib(self, k, v):
        return _t(np.asarray(v)[self.dp]) if k == 0 else _t(v)

    def to_orc(self, k, t):
        v = t.cpu().numpy()
        if k != 0:
            return v
        out = np.zeros_like(v)
        out[self.dp] = v
        return out


@pytest.fixture(scope="module", params=[("octree", 1), ("octree", 2), ("uniform", 1), ("uniform", 2)],
                ids=lambda p: f"{p[0]}-first{p[1]}")
def case(request):
    return MgCase(*request.param)


def test_hierarchy_matches_oracle(case):
    info = case.ctx.mg_info()
    assert info["dofs"] == [3 * lv.mesh.n_nodes for lv in case.levels]
    assert info["levels"] >= 2
    if case.levels[1].mesh.hanging.any():
        assert info["dense"][1] > 0


def test_prolong_and_restrict_match_oracle(case):
    rng = np.random.default_rng(1)
    for k in range(1, len(case.levels)):
        f, c = case.levels[k - 1], case.levels[k]
        P = c.P
        xc = rng.standard_normal(3 * c.mesh.n_nodes) * c.free
        xf = torch.empty(3 * f.mesh.n_nodes, dtype=torch.float64, device=DEV)
        case.ctx.mg_prolong(k, _t(xc), xf)
        want = P @ xc
        assert np.abs(case.to_orc(k - 1, xf) - want).max() <= 1e-14 * np.abs(want).max()
        rf = rng.standard_normal(3 * f.mesh.n_nodes) * f.free
        rc = torch.empty(3 * c.mesh.n_nodes, dtype=torch.float64, device=DEV)
        case.ctx.mg_restrict(k, case.to_lib(k - 1, rf), rc)
        want = P.T @ rf
        assert np.abs(rc.cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()


def test_level_operators_and_diagonals_match_galerkin(case):
    rng = np.random.default_rng(2)
    for k in range(1, len(case.levels)):
        lv = case.levels[k]
        x = rng.standard_normal(3 * lv.mesh.n_nodes)
        y = torch.empty_like(_t(x))
        case.ctx.mg_level_apply(k, _t(x), y)
        want = lv.A @ x
        assert np.abs(y.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max(), k
        d = torch.empty_like(y)
        case.ctx.mg_level_diag(k, d)
        assert np.allclose(d.cpu().numpy(), lv.dinv, rtol=1e-12, atol=0), k


def test_vcycle_matches_oracle_with_the_same_intervals(case):
    lam = [lv.hi / 1.1 for lv in case.levels[:-1]]
    case.ctx.mg_set_bounds(lam)
    try:
        rng = np.random.default_rng(3)
        r = rng.standard_normal(3 * case.pair.orc.n_nodes) * case.levels[0].free
        z = torch.empty_like(_t(r))
        case.ctx.mg_vcycle(case.to_lib(0, r), z)
        want = case.M.vcycle(r)
        got = case.to_orc(0, z)
        assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
        assert np.allclose(case.ctx.mg_get_bounds(), lam, rtol=1e-15)
    finally:
        case.ctx.mg_set_bounds(None)


def test_vcycle_with_another_coarse_degree(case):
    """Degree 3 on level 0 and 1 on the coarse levels, against the oracle."""
    tree = case.pair.case["tree"]
    case.ctx.mg_setup(tree, coarse_dofs=COARSE, first=case.first, degree=3, coarse_degree=1)
    try:
        M = mg.setup(case.levels, case.sys.A, degree=3, coarse_degree=1)
        case.ctx.mg_set_bounds([lv.hi / 1.1 for lv in M.levels[:-1]])
        r = np.random.default_rng(4).standard_normal(3 * case.pair.orc.n_nodes) * case.levels[0].free
        z = torch.empty_like(_t(r))
        case.ctx.mg_vcycle(case.to_lib(0, r), z)
        want = M.vcycle(r)
        assert np.abs(case.to_orc(0, z) - want).max() <= 1e-9 * np.abs(want).max()
    finally:
        case.ctx.mg_setup(tree, coarse_dofs=COARSE, first=case.first)
        case.M = mg.setup(case.levels, case.sys.A)


def test_vcycle_with_node_block_smoothing(case):
    """Level 0 smooths with the inverse 3 x 3 node blocks (degree 1 there,
    2 on the coarse levels): the V-cycle against the oracle's at the oracle's
    exact intervals, the power estimate of lambda_max(B^-1 A) within 10 %
    below it, and the solve to the direct solution in fewer iterations than
    with the diagonal smoother."""
    tree = case.pair.case["tree"]
    case.ctx.mg_setup(tree, coarse_dofs=COARSE, first=case.first, degree=1, coarse_degree=2, blocks0=True)
    try:
        M = mg.setup(case.levels, case.sys.A, degree=1, coarse_degree=2, blocks0=True)
        exact = np.array([lv.hi / 1.1 for lv in M.levels[:-1]])
        est = case.ctx.mg_get_bounds()
        assert (est <= exact * (1 + 1e-9)).all() and (est >= 0.9 * exact).all(), (est, exact)
        case.ctx.mg_set_bounds(list(exact))
        r = np.random.default_rng(8).standard_normal(3 * case.pair.orc.n_nodes) * case.levels[0].free
        z = torch.empty_like(_t(r))
        case.ctx.mg_vcycle(case.to_lib(0, r), z)
        want = M.vcycle(r)
        assert np.abs(case.to_orc(0, z) - want).max() <= 1e-9 * np.abs(want).max()
        case.ctx.mg_set_bounds(None)
        f = _t(case.pair.to_lib_nodes(case.pair.f))
        b = torch.empty_like(f)
        case.ctx.project_rhs(f, b)
        u = torch.zeros_like(f)
        st = case.ctx.mg_pcg(b, u, rtol=1e-10, max_it=500, check_every=1)
        assert st["status"] == "OK" and st["rel_res"] <= 1e-10, st
        want_u = osys.recover(case.sys, osys.solve_direct(case.sys))
        assert np.abs(case.to_orc(0, u) - want_u).max() <= 1e-8 * np.abs(want_u).max()
        case.ctx.mg_setup(tree, coarse_dofs=COARSE, first=case.first, degree=1, coarse_degree=2)
        u.zero_()
        st_d = case.ctx.mg_pcg(b, u, rtol=1e-10, max_it=500, check_every=1)
        assert st["iters"] <= st_d["iters"], (st, st_d)
    finally:
        case.ctx.mg_setup(tree, coarse_dofs=COARSE, first=case.first)
        case.M = mg.setup(case.levels, case.sys.A)


def test_power_estimate_of_lambda_max(case):
    exact = np.array([lv.hi / 1.1 for lv in case.levels[:-1]])
    est = case.ctx.mg_get_bounds()
    assert (est <= exact * (1 + 1e-9)).all() and (est >= 0.9 * exact).all(), (est, exact)


def test_mg_pcg_matches_direct_solve(case):
    u_ref = osys.solve_direct(case.sys)
    f = _t(case.pair.to_lib_nodes(case.pair.f))
    b = torch.empty_like(f)
    case.ctx.project_rhs(f, b)
    u = torch.zeros_like(f)
    st = case.ctx.mg_pcg(b, u, rtol=1e-10, max_it=500, check_every=1)
    assert st["status"] == "OK" and st["rel_res"] <= 1e-10, st
    # u comes back as T u~: hanging DOFs interpolated from their masters
    got = case.to_orc(0, u)
    want = osys.recover(case.sys, u_ref)
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    jac = osys.pcg_jacobi(case.sys.A, case.sys.b, rtol=1e-10)
    assert st["iters"] * 5 < jac.iters, (st["iters"], jac.iters)
    # warm start from the solution's neighbourhood takes fewer iterations
    u2 = (u * (1.0 + 1e-4 * torch.randn_like(u))).contiguous()
    st2 = case.ctx.mg_pcg(b, u2, rtol=1e-10, max_it=500, check_every=1)
    assert st2["status"] == "OK" and st2["iters"] < st["iters"]


def test_mg_errors():
    p = uniform_pair((8, 4, 4))
    ctx = binding.Context(0)
    ctx.upload_mesh(p.lib_mesh)
    ctx.set_density(_t(np.full(p.orc.n_elems, 0.5)))
    b = torch.zeros(3 * p.orc.n_nodes, dtype=torch.float64, device=DEV)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.mg_pcg(b, b.clone())
    assert e.value.code == -5
    other = binding.Octree((4, 4, 4), 0)
    other.build_mesh(p.case["fixed"], p.case["load"], lexicographic=True)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.mg_setup(other)
    assert e.value.code == -1
    ctx.mg_setup(p.case["tree"], coarse_dofs=COARSE)
    with pytest.raises(binding.AmrtoError):
        ctx.mg_level_apply(0, b, b.clone())


def _c2_library_only():
    """The full-size octree cantilever (16 x 8 x 8 base, 3 levels, band refined),
    built by the library's own octree; densities from the seeded field."""
    import synth
    case = synth.c2()
    fld = case.extra["field"]
    L = case.max_level
    t = binding.Octree(case.base, L)
    for _ in range(L):
        lv, an = t.leaves()
        t.refine(synth.band_marks(fld, lv, an, L))
    t.balance()
    mesh = t.build_mesh(case.fixed, case.load)
    lv, an = t.leaves()
    rho = fld((an + 0.5 * (1 << (L - lv))[:, None]).astype(np.float64))
    return t, mesh, rho


@pytest.mark.parametrize("first,coarse", [(1, 200), (2, 200), (2, 700)])
def test_vcycle_deterministic_symmetric_at_full_size(first, coarse):
    """At the full octree size (255,636 DOFs, many concurrent workgroups per
    level): the same residual gives the same z to rounding (the level-0
    octree pass sums element contributions with LDS atomics, so only the last
    bits may differ; a pass reading values another thread of it rewrites
    would differ far more), r1 . V r2 equals r2 . V r1 to rounding, V is
    positive, and the solve converges within the iteration count the oracle
    multigrid takes on this mesh (79 with two levels merged first) plus a
    margin.  With coarse = 700 the coarsest level has 675 DOFs, so its inverse
    takes eleven blocked Gauss-Jordan steps (the last block 35 rows): an
    inexact or unsymmetric inverse would break the symmetry check."""
    t, mesh, rho = _c2_library_only()
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    ctx.set_density(_t(rho))
    ctx.mg_setup(t, first=first, coarse_dofs=coarse)
    if coarse == 700:
        assert ctx.mg_info()["dofs"][-1] == 675
    f = _t(mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    g = torch.Generator(device=DEV).manual_seed(7)
    r1 = torch.randn(b.numel(), dtype=torch.float64, device=DEV, generator=g)
    r2 = torch.randn(b.numel(), dtype=torch.float64, device=DEV, generator=g)
    # constrained form (zero at hanging and supported DOFs): project through A~'s mask
    ctx.project_rhs(r1.clone(), r1)
    ctx.project_rhs(r2.clone(), r2)
    z1, z1b, z2 = (torch.empty_like(b) for _ in range(3))
    ctx.mg_vcycle(r1, z1)
    ctx.mg_vcycle(r1, z1b)
    ctx.mg_vcycle(r2, z2)
    assert float((z1 - z1b).abs().max()) <= 1e-12 * float(z1.abs().max())
    s12, s21 = float((r2 * z1).sum()), float((r1 * z2).sum())
    assert abs(s12 - s21) <= 1e-10 * abs(s12)
    assert float((r1 * z1).sum()) > 0 and float((r2 * z2).sum()) > 0
    u = torch.zeros_like(b)
    st = ctx.mg_pcg(b, u, rtol=1e-8, max_it=400, check_every=4)
    assert st["status"] == "OK" and st["iters"] <= 110, st


def test_mg_pcg_result_independent_of_check_interval():
    """How often the host reads the convergence state (runs of iterations
    sized from the residual's rate, between check_every and 8 check_every)
    changes only how many iterations are queued past convergence, and those
    leave u and the CG state as they were: on the full-size octree, in
    deterministic mode, every interval gives the same iteration count and the
    same solution bit for bit."""
    t, mesh, rho = _c2_library_only()
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    ctx.set_deterministic(True)
    ctx.set_density(_t(rho))
    ctx.mg_setup(t, first=2, ratio=50.0, degree=1, coarse_degree=2, coarse_dofs=700)
    f = _t(mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    runs = {}
    for ce in (1, 2, 5, 64):
        u = torch.zeros_like(b)
        st = ctx.mg_pcg(b, u, rtol=1e-8, max_it=400, check_every=ce)
        assert st["status"] == "OK" and st["rel_res"] <= 1e-8, (ce, st)
        runs[ce] = (st["iters"], u)
    its = {ce: r[0] for ce, r in runs.items()}
    assert len(set(its.values())) == 1, its
    for ce in (2, 5, 64):
        assert torch.equal(runs[ce][1], runs[1][1]), ce


def test_level_operators_follow_a_material_change():
    """The Galerkin set-up takes a leaf's product from a table of P^T K0 P per
    placement, and K0 depends on the Poisson ratio: after set_material the
    coarse operators must be those of the new ratio (equal, bit for bit, to a
    context built with it from the start), not the old table's."""
    p = octree_pair((8, 4, 4), 2)
    rho = _t(p.to_lib_elems(np.clip(centre_density(p, p.case["field"]), 0.05, 1.0)))

    def build(nu_first, nu_then=None):
        ctx = binding.Context(0)
        ctx.set_material(nu=nu_first)
        ctx.upload_mesh(p.lib_mesh)
        ctx.set_density(rho)
        ctx.mg_setup(p.case["tree"], coarse_dofs=COARSE, first=2)
        if nu_then is not None:
            x = _t(np.random.default_rng(4).standard_normal(ctx.mg_info()["dofs"][1]))
            y_old = torch.empty_like(x)
            ctx.mg_level_apply(1, x, y_old)
            ctx.set_material(nu=nu_then)
            ctx.set_density(rho)
            return ctx, y_old
        return ctx, None

    changed, y_old = build(0.3, 0.25)
    fresh, _ = build(0.25)
    for k in range(1, len(fresh.mg_info()["dofs"]) - 1):
        x = _t(np.random.default_rng(4 + k).standard_normal(fresh.mg_info()["dofs"][k]))
        ya, yb = torch.empty_like(x), torch.empty_like(x)
        changed.mg_level_apply(k, x, ya)
        fresh.mg_level_apply(k, x, yb)
        assert torch.equal(ya, yb), k
        if k == 1:
            assert not torch.equal(ya, y_old)
