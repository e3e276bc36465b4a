"""Adjoint sensitivity path (compliance backward through torch.autograd)
against the oracle gradient, central finite differences and an exact
cancellation-free difference form.

Difference form: with K(rho+) u+ = f and K(rho-) u- = f, rho+- differing only
in element e, c(rho+) - c(rho-) = f^T (u+ - u-) = -(c_e(rho+) - c_e(rho-))
(u+_e)^T K0 u-_e exactly (no linearisation, no cancellation between two
compliances, and no use of the adjoint formula)."""
import numpy as np
import pytest

import cases
import synth
from oracle import element, system as osys, topopt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def coeff(rho, E0=1.0, Emin=1e-9, p=3.0):
    return Emin + rho ** p * (E0 - Emin)


@pytest.fixture(scope="module")
def bridge(lib):
    from paper_1009_4975_amd import autograd
    dims = (16, 8, 8)
    p = cases.uniform_pair(dims, bc="bridge")
    rho = synth.uniform_random(p.orc.n_elems, 0.01, 1.0, 0)
    prob = autograd.ComplianceProblem(p.lib_mesh, rtol=1e-13)
    return p, rho, prob


def test_backward_matches_oracle_gradient(bridge):
    from paper_1009_4975_amd import autograd
    p, rho, prob = bridge
    r = dev(rho).requires_grad_(True)
    c = autograd.compliance(r, prob)
    c.backward()
    s = cases.oracle_system(p, rho)
    u = osys.recover(s, osys.solve_direct(s))
    assert c.item() == pytest.approx(float(s.f @ u), rel=1e-10)
    g_or = topopt.sensitivities(p.orc, rho, u)
    g = r.grad.cpu().numpy()
    assert np.linalg.norm(g - g_or) <= 1e-8 * np.linalg.norm(g_or)


def test_central_differences_and_difference_form(bridge):
    from paper_1009_4975_amd import autograd
    p, rho, prob = bridge
    r = dev(rho).requires_grad_(True)
    autograd.compliance(r, prob).backward()
    g = r.grad.cpu().numpy()
    K0 = element.k0(0.3)
    edofs = osys.elem_dofs(p.orc)
    delta = 1e-6
    picks = np.random.default_rng(1).choice(len(rho), 8, replace=False)
    for e in picks:
        rp, rm = rho.copy(), rho.copy()
        rp[e] += delta
        rm[e] -= delta
        cp = autograd.compliance(dev(rp), prob).item()
        up = prob.u.cpu().numpy()
        cm = autograd.compliance(dev(rm), prob).item()
        um = prob.u.cpu().numpy()
        fd = (cp - cm) / (2 * delta)
        # plain central differences: limited by cancellation in cp - cm
        assert fd == pytest.approx(g[e], rel=1e-4)
        exact = -(coeff(rp[e]) - coeff(rm[e])) * (up[edofs[e]] @ K0 @ um[edofs[e]]) / (2 * delta)
        assert exact == pytest.approx(g[e], rel=1e-7)
