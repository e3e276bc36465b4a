"""The 2-D variant on the GPU (amrto_plane_*) against the 2-D oracle on the
same quadtree meshes, element by element: the constrained operator, the
projected right-hand side, PCG against the direct solve (hanging values
recovered), compliance and sensitivities, both filter modes, the OC step,
and a short adaptive SIMP sequence against the oracle's loop.  Library and
oracle build their meshes independently from the same leaves; nodes are
matched by coordinates and elements by (level, anchor)."""
import numpy as np
import pytest
import torch

from oracle import plane
from oracle.topopt import oc_update
from paper_1009_4975_amd import binding
from paper_1009_4975_amd.plane_simp import PlaneSIMP, cantilever_2d

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _key(l, a):
    return (int(l), int(a[0]), int(a[1]))


def grow(base, L, seed, p=0.3, uniform=False):
    rng = np.random.default_rng(seed)
    t = binding.Quadtree(base, L)
    lv, an = plane.base_leaves(base, L)
    for _ in range(L):
        tl, ta = t.leaves()
        if uniform:
            pick = {_key(l, a) for l, a in zip(tl, ta)}
        else:
            pick = {k for k in sorted(_key(l, a) for l, a in zip(tl, ta)) if rng.random() < p}
        t.refine(np.array([_key(l, a) in pick for l, a in zip(tl, ta)]))
        lv, an, _ = plane.refine(lv, an, L, np.array([_key(l, a) in pick for l, a in zip(lv, an)]))
    t.balance()
    lv, an, _ = plane.balance(lv, an, L)
    return t, lv, an


class Case:
    def __init__(self, base, L, seed, uniform=False):
        t, lv, an = grow(base, L, seed, uniform=uniform)
        self.dims = tuple(b << L for b in base)
        self.fixed, self.load = cantilever_2d(self.dims)
        self.m = t.build_mesh(self.fixed, self.load)
        self.o = plane.build_mesh(lv, an, L, self.dims)
        key = {tuple(c): i for i, c in enumerate(self.o.coords.tolist())}
        self.perm = np.array([key[tuple(c)] for c in self.m.node_xy.tolist()])
        self.dperm = (2 * self.perm[:, None] + np.arange(2)).ravel()   # library DOF -> oracle DOF
        tl, ta = t.leaves()
        okey = {_key(l, a): e for e, (l, a) in enumerate(zip(self.o.level, self.o.anchor))}
        self.eperm = np.array([okey[_key(l, a)] for l, a in zip(tl, ta)])  # library elem -> oracle elem
        self.fixed_o = plane.fixed_dofs(self.o, self.fixed)
        self.f_o = plane.load_vector(self.o, self.load)
        self.ctx = binding.PlaneContext(0)
        self.ctx.set_material()
        self.ctx.upload_mesh(self.m)

    def dofs(self, v_o):
        return torch.tensor(np.asarray(v_o)[self.dperm], dtype=torch.float64, device=DEV)

    def elems(self, v_o):
        return torch.tensor(np.asarray(v_o)[self.eperm], dtype=torch.float64, device=DEV)

    def to_o_dofs(self, t):
        out = np.zeros(2 * self.m.n_nodes)
        out[self.dperm] = t.cpu().numpy()
        return out

    def to_o_elems(self, t):
        out = np.zeros(self.m.n_elems)
        out[self.eperm] = t.cpu().numpy()
        return out


CASES = {"small": ((8, 4), 2, 0, False), "tiles": ((16, 8), 3, 1, False), "uniform": ((8, 4), 2, 2, True)}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    c = Case(*CASES[request.param])
    if request.param != "uniform":
        assert c.m.hang_node.size > 0
    return c


def _rho(case, seed, lo=1e-3):
    return np.random.default_rng(seed).uniform(lo, 1.0, case.o.n_elems)


def test_apply_matches_oracle(case):
    rho = _rho(case, 1)
    x = np.random.default_rng(2).standard_normal(2 * case.o.n_nodes)
    case.ctx.set_density(case.elems(rho))
    y = torch.empty(2 * case.m.n_nodes, dtype=torch.float64, device=DEV)
    case.ctx.apply(case.dofs(x), y)
    want = plane.apply_constrained(case.o, plane.young(rho), case.fixed_o, x)
    got = case.to_o_dofs(y)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # the assembled matrix agrees with the operator
    s = plane.build_system(case.o, plane.young(rho), case.fixed_o, case.f_o)
    assert np.abs(s.A @ x - want).max() <= 1e-12 * np.abs(want).max()


def test_project_rhs_matches_oracle(case):
    f = np.random.default_rng(3).standard_normal(2 * case.o.n_nodes)
    b = torch.empty(2 * case.m.n_nodes, dtype=torch.float64, device=DEV)
    case.ctx.project_rhs(case.dofs(f), b)
    s = plane.build_system(case.o, np.ones(case.o.n_elems), case.fixed_o, f)
    assert np.abs(case.to_o_dofs(b) - s.b).max() <= 1e-14 * np.abs(s.b).max()


@pytest.mark.parametrize("warm", [False, True])
def test_pcg_matches_direct_solve(case, warm):
    rho = _rho(case, 4, lo=0.05)
    s = plane.build_system(case.o, plane.young(rho), case.fixed_o, case.f_o)
    u_ref = plane.solve_direct(s)
    case.ctx.set_density(case.elems(rho))
    f = case.dofs(case.f_o)
    b = torch.empty_like(f)
    case.ctx.project_rhs(f, b)
    rng = np.random.default_rng(5)
    if warm:
        # a perturbed solution, with garbage at supported and hanging entries (ignored)
        u0 = u_ref * (1.0 + 1e-3 * rng.standard_normal(u_ref.size)) + 1e-2 * (~s.free)
    else:
        u0 = np.zeros_like(u_ref)
    u = case.dofs(u0)
    st = case.ctx.pcg(b, u, rtol=1e-11, max_it=20000, check_every=8)
    assert st["status"] == "OK" and st["rel_res"] <= 1e-11, st
    got = case.to_o_dofs(u)
    assert np.abs(got - u_ref).max() <= 1e-8 * np.abs(u_ref).max()
    c = case.ctx.compliance(u, f)
    assert c == pytest.approx(float(case.f_o @ u_ref), rel=1e-9)
    if warm:
        cold = case.dofs(np.zeros_like(u_ref))
        st0 = case.ctx.pcg(b, cold, rtol=1e-11, max_it=20000, check_every=8)
        assert st["iters"] < st0["iters"]


def test_compliance_and_sensitivities_match_oracle(case):
    rho = _rho(case, 6)
    u = np.random.default_rng(7).standard_normal(2 * case.o.n_nodes)
    dc = torch.empty(case.m.n_elems, dtype=torch.float64, device=DEV)
    c = case.ctx.compliance(case.dofs(u), case.dofs(case.f_o), case.elems(rho), dc)
    assert c == pytest.approx(float(case.f_o @ u), rel=1e-13, abs=1e-15)
    want = plane.sensitivities(case.o, rho, u)
    assert np.abs(case.to_o_elems(dc) - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("rmin", [1.5, 2.6, 4.3])
def test_filters_match_oracle(case, rmin):
    rng = np.random.default_rng(8)
    rho = rng.uniform(1e-3, 1.0, case.o.n_elems)
    x = rng.standard_normal(case.o.n_elems)
    out = torch.empty(case.m.n_elems, dtype=torch.float64, device=DEV)
    case.ctx.filter(binding.FILTER_SENSITIVITY, rmin, case.elems(x), out, rho=case.elems(rho))
    want = plane.filter_sensitivity(case.o, rmin, rho, x)
    assert np.abs(case.to_o_elems(out) - want).max() <= 1e-12 * np.abs(want).max()
    case.ctx.filter(binding.FILTER_DENSITY, rmin, case.elems(x), out)
    W = plane.filter_weights(case.o, rmin)
    want = (W @ x) / np.asarray(W.sum(1)).ravel()
    assert np.abs(case.to_o_elems(out) - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("volfrac", [0.55, 0.4])
def test_oc_matches_oracle(case, volfrac):
    rng = np.random.default_rng(9)
    rho = rng.uniform(1e-3, 1.0, case.o.n_elems)
    dc = -rng.uniform(0.0, 2.0, case.o.n_elems) * case.o.areas
    out = torch.empty(case.m.n_elems, dtype=torch.float64, device=DEV)
    ch, lam = case.ctx.oc_update(case.elems(rho), case.elems(dc), out, volfrac)
    a = case.o.areas
    want, lam_o, ch_o = oc_update(rho, dc, a, volfrac * a.sum())
    got = case.to_o_elems(out)
    assert np.abs(got - want).max() <= 1e-9
    assert lam == pytest.approx(lam_o, rel=1e-9)
    assert ch == pytest.approx(ch_o, abs=1e-9)
    assert float(got @ a) == pytest.approx(volfrac * a.sum(), rel=1e-9)


def test_errors_and_states():
    ctx = binding.PlaneContext(0)
    x = torch.zeros(8, dtype=torch.float64, device=DEV)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.set_density(x)
    assert e.value.code == -5
    with pytest.raises(binding.AmrtoError):
        ctx.set_material(E0=1.0, Emin=2.0)
    empty = binding.Mesh2DArrays((4, 4), 0, np.zeros((0, 2), np.int32), np.zeros((0, 4), np.int32),
                                 np.zeros(0, np.int8), np.zeros(0, np.int32), np.zeros(1, np.int32),
                                 np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.uint8), np.zeros(0))
    with pytest.raises(binding.AmrtoError) as e:
        ctx.upload_mesh(empty)
    assert e.value.code == -1


def _oracle_loop(base, L, steps, adapt_every, volfrac, rmin, r_amr):
    dims = tuple(b << L for b in base)
    fixed, load = cantilever_2d(dims)
    lv, an = plane.base_leaves(base, L)
    rho = np.full(len(lv), volfrac)
    hist, leaves = [], []
    for it in range(steps):
        if it > 0 and it % adapt_every == 0:
            lv, an, rho = plane.adapt(lv, an, L, rho, 0.5, r_amr)
            leaves.append({_key(l, a) for l, a in zip(lv, an)})
        mesh = plane.build_mesh(lv, an, L, dims)
        fx, f = plane.fixed_dofs(mesh, fixed), plane.load_vector(mesh, load)
        s = plane.build_system(mesh, plane.young(rho), fx, f)
        u = plane.solve_direct(s)
        hist.append(float(f @ u))
        dc = plane.sensitivities(mesh, rho, u)
        dcf = plane.filter_sensitivity(mesh, rmin, rho, dc)
        rho, _, _ = oc_update(rho, dcf, mesh.areas, volfrac * mesh.areas.sum())
    return hist, leaves, {_key(l, a): r for l, a, r in zip(lv, an, rho)}


def test_simp_sequence_with_adaptation_matches_oracle():
    base, L, steps, k, volfrac, rmin, r_amr = (8, 4), 2, 8, 3, 0.5, 1.5, 1.5
    sim = PlaneSIMP(base, L, volfrac=volfrac, rmin=rmin, r_amr=r_amr, adapt_every=k, rtol=1e-11)
    hist, leaves = [], []
    for it in range(steps):
        rec = sim.step()
        if rec["adapted"]:
            lv, an = sim.leaves()
            leaves.append({_key(l, a) for l, a in zip(lv, an)})
        hist.append(rec["compliance"])
    h_o, leaves_o, rho_o = _oracle_loop(base, L, steps, k, volfrac, rmin, r_amr)
    assert len(leaves) == len(leaves_o) == 2
    for a, b in zip(leaves, leaves_o):
        assert a == b
    assert np.allclose(hist, h_o, rtol=1e-7)
    lv, an = sim.leaves()
    rho = sim.rho.cpu().numpy()
    got = {_key(l, a): r for l, a, r in zip(lv, an, rho)}
    assert got.keys() == rho_o.keys()
    assert max(abs(got[k] - rho_o[k]) for k in got) <= 1e-6
