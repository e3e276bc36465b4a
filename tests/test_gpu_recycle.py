"""Krylov recycling through the C ABI against the oracle (oracle/recycle.py):
Rayleigh-Ritz on the same vectors for the pencil (A~, diag A~) of the
oracle's assembled operator; Ritz pairs harvested from a recorded FP64
Jacobi-PCG solve, checked by the Lanczos residual identity with the oracle's
operator and against the oracle's own recorded CG; Ritz values harvested from
solves that run the fused coarse-space pass (block-Jacobi + affine coarse
space, FP64 and the first cycle of a mixed solve) against the oracle's CG
with the same two-level preconditioner written from its definition; solves
started from the recycled vectors or with them in the coarse space against
the oracle's direct solution."""
import numpy as np
import pytest

import cases
from oracle import recycle, system as osys
from test_gpu_parity import _affine_z

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


def _two_level_minv(p, s, regions):
    """M^-1 r = B^-1 r + Z (Z^T A~ Z)^-1 Z^T r, B the 3x3 node blocks of the
    oracle's A~ (oracle node order), Z the affine fields (library order,
    permuted here)."""
    import scipy.sparse as sp
    A = s.A.tocsr()
    n = A.shape[0] // 3
    blocks = np.zeros((n, 3, 3))
    for c in range(3):
        for d in range(3):
            blocks[:, c, d] = A[3 * np.arange(n) + c, 3 * np.arange(n) + d].A1
    binv = np.linalg.inv(blocks)
    Zl = _affine_z(p.lib_mesh, p.lib_mesh.dims, regions).toarray()
    Z = np.empty_like(Zl)
    Z.reshape(-1, 3, Zl.shape[1])[p.perm] = Zl.reshape(-1, 3, Zl.shape[1])
    E = Z.T @ (A @ Z)
    Einv = np.linalg.pinv(E, rcond=1e-12)
    return lambda r: np.einsum("nij,nj->ni", binv, r.reshape(-1, 3)).ravel() + Z @ (Einv @ (Z.T @ r))


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_harvest_from_fused_coarse_block3_solve(setup, inner):
    from paper_1009_4975_amd import binding
    p, s, ctx = setup
    regions = (2, 1, 1)
    b = dev(p.to_lib_nodes(s.b))
    ctx.coarse_setup([], *regions, affine=True)
    u = torch.zeros_like(b)
    prec = binding.FP64 if inner == "fp64" else binding.FP32
    st = ctx.pcg(b, u, rtol=1e-12, record=True, precond=binding.BLOCK3, inner_prec=prec, inner_rtol=1e-3)
    assert st["status"] == "OK"
    outs = [torch.empty_like(b) for _ in range(3)]
    theta, _, m = ctx.recycle_harvest(outs)
    ctx.coarse_clear()
    minv = _two_level_minv(p, s, regions)
    _, Z, rz, pq = recycle.pcg_record(s.A, s.b, minv, m + 1)
    th_o, U_o, _ = recycle.ritz_pairs(Z, rz, pq[:m], 3)
    # FP32 vectors make the recurrence lose orthogonality sooner: its small
    # Ritz values agree to a few parts in a hundred, the FP64 ones to 1e-6
    tol = 1e-6 if inner == "fp64" else 3e-2
    assert np.allclose(theta[:2], th_o[:2], rtol=tol)
    if inner == "fp64":
        # the smallest Ritz vector itself, up to sign, in the A~-norm
        w = _to_oracle(p, outs[0].cpu().numpy())
        a = w @ (s.A @ U_o[:, 0])
        assert abs(a) / np.sqrt((w @ (s.A @ w)) * (U_o[:, 0] @ (s.A @ U_o[:, 0]))) == pytest.approx(1.0, abs=1e-6)


def test_recycled_start_solve(setup):
    """Ritz vectors of one system start the solve of a perturbed one (the
    next design): the start is the Galerkin projection of the initial error
    onto them; the solve reaches the direct solution."""
    from paper_1009_4975_amd import binding
    p, s, ctx = setup
    b = dev(p.to_lib_nodes(s.b))
    u = torch.zeros_like(b)
    ctx.pcg(b, u, rtol=1e-10, record=True)
    U = [torch.empty_like(b) for _ in range(4)]
    ctx.recycle_harvest(U)
    rho = cases.centre_density(p, p.case["field"]) * np.random.default_rng(4).uniform(0.9, 1.1, p.orc.n_elems)
    rho = np.clip(rho, 1e-3, 1.0)
    s2 = cases.oracle_system(p, rho)
    u_ref = p.to_lib_nodes(osys.recover(s2, osys.solve_direct(s2)))
    ctx.set_density(dev(p.to_lib_elems(rho)))
    x0 = torch.empty_like(b)
    coef = ctx.energy_combine(b, U, x0, base=u)
    assert all(np.isfinite(coef))
    st = ctx.pcg(b, x0, rtol=1e-12)
    assert st["status"] == "OK"
    assert np.linalg.norm(x0.cpu().numpy() - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    ctx.set_density(dev(p.to_lib_elems(cases.centre_density(p, p.case["field"]))))
