"""The C ABI's contract that hot calls allocate nothing: after one warm-up of
each call (code objects load on first use), repeated filter (several radii,
both modes), apply (every precision), PCG (plain, mixed, block-Jacobi),
compliance and OC calls on an octree mesh leave the device's free memory
unchanged.  Their tensors are allocated before the first reading."""
import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_hot_calls_allocate_nothing(lib):
    from paper_1009_4975_amd import binding
    p = cases.octree_pair((4, 2, 2), 2, width=0.2)
    rho_h = cases.centre_density(p, p.case["field"])
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = binding.Context(0)
    ctx.upload_mesh(p.lib_mesh)
    rho = dev(p.to_lib_elems(rho_h))
    ctx.set_density(rho)
    n3, ne = 3 * p.orc.n_nodes, p.orc.n_elems
    f = dev(p.lib_mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    u = torch.zeros_like(f)
    x64 = torch.randn(n3, dtype=torch.float64, device="cuda")
    y64 = torch.empty_like(x64)
    x32 = x64.float()
    y32 = torch.empty_like(x32)
    dc = torch.empty(ne, dtype=torch.float64, device="cuda")
    dcf = torch.empty_like(dc)
    rho_new = torch.empty_like(dc)

    def calls():
        for r in (1.5, 2.6, 4.3):
            ctx.filter(binding.FILTER_SENSITIVITY, r, dc, dcf, rho=rho)
            ctx.filter(binding.FILTER_DENSITY, r, rho, dcf)
        ctx.apply(x64, y64, binding.FP64)
        ctx.apply(x32, y32, binding.FP32)
        ctx.apply(x32, y32, binding.BF16)
        for prec, pc in ((binding.FP64, binding.JACOBI), (binding.FP32, binding.JACOBI),
                         (binding.FP64, binding.BLOCK3)):
            u.zero_()
            st = ctx.pcg(b, u, rtol=1e-8, inner_prec=prec, precond=pc)
            assert st["status"] == "OK"
        ctx.compliance(u, f, rho, dc)
        ctx.oc_update(rho, dc, rho_new, 0.3)

    calls()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        calls()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, f"device free memory changed by {free0 - free1} bytes across hot calls"


def test_pass_times_leave_solves_intact(lib):
    """amrto_pcg_pass_times on every solver variant of the octree bench
    (plain, mixed, block-Jacobi, with the affine coarse space) returns
    positive per-launch times, and a solve afterwards still reaches the same
    solution as one before it."""
    from paper_1009_4975_amd import binding
    p = cases.octree_pair((4, 2, 2), 2, width=0.2)
    rho_h = cases.centre_density(p, p.case["field"])
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = binding.Context(0)
    ctx.upload_mesh(p.lib_mesh)
    ctx.set_density(dev(p.to_lib_elems(rho_h)))
    f = dev(p.lib_mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    u0 = torch.zeros_like(f)
    ctx.pcg(b, u0, rtol=1e-11)
    for coarse in (False, True):
        if coarse:
            ctx.coarse_setup([], 2, 1, 1, affine=True)
        for prec in (binding.FP64, binding.FP32, binding.BF16):
            for pc in (binding.JACOBI, binding.BLOCK3):
                w = torch.zeros_like(f)
                op, up = ctx.pcg_pass_times(b, w, reps=5, inner_prec=prec, precond=pc)
                assert op > 0 and up > 0
                u = torch.zeros_like(f)
                st = ctx.pcg(b, u, rtol=1e-11, inner_prec=prec, precond=pc)
                assert st["status"] == "OK"
                assert torch.linalg.norm(u - u0) <= 1e-8 * torch.linalg.norm(u0)
