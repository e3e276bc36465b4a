"""Deterministic mode (amrto_set_deterministic) on the full C2 octree (61,028
elements, 255,636 DOFs, hanging nodes in every refined band, every chunk run
by eight waves):

* y = A~ x in FP64, FP32 and BF16 is the same bit for bit over repeated
  calls, equals the default mode's result to the rounding of the summation
  order, and meets the oracle's element-by-element operator at the same
  bound as the default mode's parity tests;
* the Jacobi diagonal and the 3x3 node blocks formed twice from the same
  density are the same bit for bit;
* whole solves (plain FP64 Jacobi-PCG, mixed FP32 inner with node blocks and
  the affine coarse space in recurrence form as timed, FP64 with the coarse
  space, the one-reduction form, and multigrid-preconditioned CG with the
  hierarchy set up again) repeat with the same iteration count and the same
  solution bit for bit, and agree with the default mode's solution within
  what the 1e-8 residual allows.

Repetition shows run-to-run reproducibility on this device; it does not prove
order independence under every schedule, which is what the fixed turn order
of the waves gives by construction."""
import numpy as np
import pytest

import cases
from oracle import system as osys

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def c2():
    from paper_1009_4975_amd import binding
    pair = cases.octree_pair((16, 8, 8), 3)
    rho = cases.centre_density(pair, pair.case["field"])
    ctx = binding.Context(0)
    ctx.upload_mesh(pair.lib_mesh)
    ctx.set_density(dev(pair.to_lib_elems(rho)))
    assert 3 * pair.orc.n_nodes == 255636
    yield pair, rho, ctx
    ctx.set_deterministic(False)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 5e-6), (2, 1e-4)], ids=["fp64", "fp32", "bf16"])
def test_apply_repeats_bitwise(c2, prec, tol):
    pair, rho, ctx = c2
    dt = torch.float64 if prec == 0 else torch.float32
    x = np.random.default_rng(5).uniform(-1, 1, 3 * pair.orc.n_nodes)
    xd = dev(pair.to_lib_nodes(x), dt)
    ctx.set_deterministic(False)
    y_def = torch.empty_like(xd)
    ctx.apply(xd, y_def, prec=prec)
    ctx.set_deterministic(True)
    ys = []
    for _ in range(4):
        y = torch.empty_like(xd)
        ctx.apply(xd, y, prec=prec)
        ys.append(y)
    for y in ys[1:]:
        assert torch.equal(y, ys[0])
    want = pair.to_lib_nodes(osys.apply_constrained(pair.orc, osys.elem_coeff(pair.orc, rho), pair.fixed, x))
    got = host(ys[0])
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))
    # the two modes differ only in the order of the same sums
    order = {0: 1e-13, 1: 1e-5, 2: 1e-5}[prec]
    assert np.max(np.abs(got - host(y_def))) <= order * np.max(np.abs(want))


def test_diagonals_repeat_bitwise(c2):
    pair, rho, ctx = c2
    ctx.set_deterministic(True)
    n3 = 3 * pair.orc.n_nodes
    d = [torch.empty(n3, dtype=torch.float64, device=DEV) for _ in range(2)]
    blk = [torch.empty(3 * n3, dtype=torch.float64, device=DEV) for _ in range(2)]
    for i in range(2):
        ctx.set_density(dev(pair.to_lib_elems(rho)))
        ctx.diag(d[i])
        ctx.block_diag(blk[i])
    assert torch.equal(d[0], d[1])
    assert torch.equal(blk[0], blk[1])


SOLVES = ["fp64", "fp32+block3+coarse", "fp64+coarse", "fp64+one-reduction", "mg"]


def _solve(binding, pair, ctx, kind):
    f = dev(pair.lib_mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    u = torch.zeros_like(f)
    if kind == "mg":
        ctx.mg_setup(pair.case["tree"], first=2, ratio=50.0, degree=1, coarse_degree=2)
        st = ctx.mg_pcg(b, u, rtol=1e-8, max_it=400)
    elif "+coarse" in kind:
        ctx.coarse_setup([], 3, 2, 2, affine=True)
        st = ctx.pcg(b, u, rtol=1e-8, max_it=50000, inner_rtol=0.1,
                     inner_prec=binding.FP32 if kind.startswith("fp32") else binding.FP64,
                     precond=binding.BLOCK3 if "+block3" in kind else binding.JACOBI)
        ctx.coarse_clear()
    else:
        st = ctx.pcg(b, u, rtol=1e-8, max_it=50000, single_reduction="one-reduction" in kind)
    assert st["status"] == "OK" and st["rel_res"] <= 1e-8, (kind, st)
    return st, u


@pytest.mark.parametrize("kind", SOLVES)
def test_solves_repeat_bitwise(c2, kind):
    from paper_1009_4975_amd import binding
    pair, rho, ctx = c2
    ctx.set_deterministic(False)
    ctx.set_density(dev(pair.to_lib_elems(rho)))
    st_def, u_def = _solve(binding, pair, ctx, kind)
    ctx.set_deterministic(True)
    runs = []
    for _ in range(2):
        ctx.set_density(dev(pair.to_lib_elems(rho)))
        runs.append(_solve(binding, pair, ctx, kind))
    (st1, u1), (st2, u2) = runs
    assert st1["iters"] == st2["iters"], (st1, st2)
    assert torch.equal(u1, u2)
    # both modes solve the same system to a 1e-8 residual; rounding moves the
    # iteration count a little (FP32 inner solves with restarts the most: the
    # default mode's mixed solve on this mesh has taken 803 to 859)
    assert float((u1 - u_def).norm()) <= 1e-4 * float(u_def.norm())
    assert abs(st1["iters"] - st_def["iters"]) <= max(5, st_def["iters"] // 8), (st1, st_def)
