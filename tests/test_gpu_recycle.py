"""Krylov recycling through the C ABI against the oracle (oracle/recycle.py):
Rayleigh-Ritz on the same vectors for the pencil (A~, diag A~) of the
oracle's assembled operator; Ritz pairs harvested from a recorded FP64
Jacobi-PCG solve, checked by the Lanczos residual identity with the oracle's
operator and against the oracle's own recorded CG; solves with the recycled
vectors in the coarse space against the oracle's direct solution."""
import numpy as np
import pytest

import cases
from oracle import recycle, system as osys

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def setup(lib):
    from paper_1009_4975_amd import binding
    p = cases.octree_pair((4, 2, 2), 2, width=0.2)
    rho = cases.centre_density(p, p.case["field"])
    s = cases.oracle_system(p, rho)
    ctx = binding.Context(0)
    ctx.upload_mesh(p.lib_mesh)
    ctx.set_density(dev(p.to_lib_elems(rho)))
    ctx.recycle_setup(40)
    return p, s, ctx


def _to_oracle(p, v_lib):
    out = np.empty_like(v_lib)
    out.reshape(-1, 3)[p.perm] = v_lib.reshape(-1, 3)
    return out


def test_rayleigh_ritz_matches_oracle(setup):
    p, s, ctx = setup
    rng = np.random.default_rng(9)
    S = rng.standard_normal((len(s.b), 6)) * s.free[:, None]
    outs = [torch.empty(len(s.b), dtype=torch.float64, device="cuda") for _ in range(3)]
    theta, rank = ctx.rayleigh_ritz([dev(p.to_lib_nodes(S[:, j])) for j in range(6)], outs)
    d = s.A.diagonal()
    th_o, W_o = recycle.rayleigh_ritz(s.A, d, S, 3)
    assert rank == 6
    assert np.allclose(theta, th_o, rtol=1e-10)
    for i in range(3):
        w = _to_oracle(p, outs[i].cpu().numpy())
        assert abs(w @ (d * W_o[:, i])) == pytest.approx(1.0, abs=1e-8)
        assert w @ (d * w) == pytest.approx(1.0, rel=1e-10)


def test_harvest_ritz_pairs(setup):
    p, s, ctx = setup
    b = dev(p.to_lib_nodes(s.b))
    u = torch.zeros_like(b)
    st = ctx.pcg(b, u, rtol=1e-12, record=True)
    assert st["status"] == "OK" and st["iters"] > 41
    k = 4
    outs = [torch.empty_like(b) for _ in range(k)]
    theta, resid, m = ctx.recycle_harvest(outs)
    assert m == 39  # 40 vectors stored, 39 steps with known alpha
    d = s.A.diagonal()
    for i in range(k):
        w = _to_oracle(p, outs[i].cpu().numpy())
        assert np.all(w[~s.free] == 0.0)
        r = s.A @ w - theta[i] * d * w
        # the Lanczos residual identity ||A u - theta D u||_{D^-1} = |T[m-1, m] y_{m-1}|
        assert np.sqrt(r @ (r / d)) == pytest.approx(resid[i], rel=1e-6, abs=1e-9 * theta[i])
    # the oracle's own recorded CG on the same system from zero
    _, Z, rz, pq = recycle.pcg_record(s.A, s.b, lambda r: r / d, 40)
    th_o, _, _ = recycle.ritz_pairs(Z, rz, pq[:39], k)
    assert np.allclose(theta[:2], th_o[:2], rtol=1e-6)
    assert np.all(np.diff(theta) >= 0)


@pytest.mark.parametrize("affine", [False, True])
def test_recycled_coarse_space_solve(setup, affine):
    p, s, ctx = setup
    u_ref = p.to_lib_nodes(osys.recover(s, osys.solve_direct(s)))
    b = dev(p.to_lib_nodes(s.b))
    u = torch.zeros_like(b)
    ctx.pcg(b, u, rtol=1e-10, record=True)
    U = [torch.empty_like(b) for _ in range(4)]
    ctx.recycle_harvest(U)
    W = [torch.empty_like(b) for _ in range(4)]
    ctx.rayleigh_ritz(U, W)
    ctx.coarse_setup(W, 2, 1, 1, affine=affine)
    for record in (False, True):
        u = torch.zeros_like(b)
        st = ctx.pcg(b, u, rtol=1e-12, record=record)
        assert st["status"] == "OK"
        err = np.linalg.norm(u.cpu().numpy() - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-8
    ctx.coarse_clear()
