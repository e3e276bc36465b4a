"""Failure handling, forced from the host: iteration caps, non-finite inputs,
calls out of order, bad arguments, corrupt mesh tables, a non-finite network
prediction.  Every case must end in the documented status code (or the
documented fallback); none makes a kernel fault.  Corrupt tables are rejected
on the host before anything reaches the GPU."""
import dataclasses

import numpy as np
import pytest

import cases
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.fixture(scope="module")
def small():
    from paper_1009_4975_amd import binding
    pair = cases.uniform_pair((8, 4, 4))
    rho = cases.c1_density((8, 4, 4))
    ctx = binding.Context(0)
    ctx.upload_mesh(pair.lib_mesh)
    ctx.set_density(dev(rho))
    f = dev(pair.lib_mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    return pair, rho, ctx, b


def code_of(err):
    return str(err.value).split(":")[0]


def test_iteration_cap_reports_not_converged(small):
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    u = torch.zeros_like(b)
    st = ctx.pcg(b, u, rtol=1e-12, max_it=1, allow_not_converged=True)
    assert st["status"] == "NOT_CONVERGED" and st["rel_res"] > 1e-12
    with pytest.raises(binding.AmrtoError) as e:
        ctx.pcg(b, torch.zeros_like(b), rtol=1e-12, max_it=1)
    assert code_of(e) == "NOT_CONVERGED" and "cap" in str(e.value)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_rhs_is_breakdown(small, prec):
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    bad = b.clone()
    bad[7] = float("nan")
    with pytest.raises(binding.AmrtoError) as e:
        ctx.pcg(bad, torch.zeros_like(b), rtol=1e-8,
                inner_prec=binding.FP64 if prec == "fp64" else binding.FP32)
    assert code_of(e) == "EBREAKDOWN"
    # the context stays usable
    st = ctx.pcg(b, torch.zeros_like(b), rtol=1e-8)
    assert st["rel_res"] <= 1e-8


def test_stalled_mixed_solve_falls_back_to_fp64(small):
    """inner_rtol 0.9: every reliable update cuts the true residual by about
    0.9, which the stall rule counts as no progress, so the mixed solve stops
    after three updates; plain FP64 PCG then finishes from its iterate."""
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    ref = torch.zeros_like(b)
    st0 = ctx.pcg(b, ref, rtol=1e-10)
    assert not st0["fell_back"]
    u = torch.zeros_like(b)
    st = ctx.pcg(b, u, rtol=1e-10, inner_prec=binding.FP32, inner_rtol=0.9)
    assert st["status"] == "OK" and st["fell_back"] and st["rel_res"] <= 1e-10
    assert torch.allclose(u, ref, rtol=0, atol=1e-8 * ref.abs().max().item())
    st = ctx.pcg(b, torch.zeros_like(b), rtol=1e-10, inner_prec=binding.FP32, inner_rtol=0.9, fallback_fp64=False,
                 allow_not_converged=True)
    assert st["status"] == "NOT_CONVERGED" and not st["fell_back"] and st["rel_res"] > 1e-10


def test_calls_out_of_order(small):
    from paper_1009_4975_amd import binding
    pair, rho, _, b = small
    ctx = binding.Context(0)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.set_density(dev(rho))
    assert code_of(e) == "ESTATE"
    ctx.upload_mesh(pair.lib_mesh)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.pcg(b, torch.zeros_like(b))
    assert code_of(e) == "ESTATE"
    with pytest.raises(binding.AmrtoError) as e:
        ctx.coarse_setup([], 1, 1, 1, affine=True)
    assert code_of(e) == "ESTATE"


def test_bad_arguments(small):
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    for kw in (dict(rtol=0.0), dict(rtol=-1.0), dict(inner_prec=7), dict(max_it=-1), dict(inner_rtol=1.5)):
        with pytest.raises(binding.AmrtoError) as e:
            ctx.pcg(b, torch.zeros_like(b), **kw)
        assert code_of(e) == "EINVAL", kw
    with pytest.raises(binding.AmrtoError) as e:  # b and u the same buffer
        ctx.pcg(b, b)
    assert code_of(e) == "EINVAL"
    with pytest.raises(binding.AmrtoError) as e:  # 3 * 4 * 128 = 1536 columns
        ctx.coarse_setup([], 8, 8, 2, affine=True)
    assert code_of(e) == "EINVAL"
    with pytest.raises(binding.AmrtoError) as e:  # nine fields
        ctx.coarse_setup([torch.zeros_like(b)] * 5, 1, 1, 1, affine=True)
    assert code_of(e) == "EINVAL"


def test_nonfinite_coarse_field_rejected_and_plain_solve_runs(small):
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    field = torch.ones_like(b)
    field[0] = float("inf")
    ctx.mask(field)
    field[30] = float("nan")
    with pytest.raises(binding.AmrtoError) as e:
        ctx.coarse_setup([field], 1, 1, 1)
    assert code_of(e) == "EINVAL"
    st = ctx.pcg(b, torch.zeros_like(b), rtol=1e-8)  # no coarse space left behind
    assert st["rel_res"] <= 1e-8


def test_nonfinite_start_vector_rejected(small):
    from paper_1009_4975_amd import binding
    pair, rho, ctx, b = small
    v = torch.zeros_like(b)
    v[12] = float("nan")
    x0 = torch.full_like(b, 3.0)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.energy_combine(b, [v], x0)
    assert code_of(e) == "EINVAL"
    assert torch.all(x0 == 3.0)


def _octree_mesh():
    from paper_1009_4975_amd import binding
    t = binding.Octree((4, 2, 2), 2)
    marks = np.zeros(len(t.leaves()[0]), np.uint8)
    marks[5] = 1  # one refined leaf: hanging nodes on its faces and edges
    t.refine(marks)
    t.balance()
    fixed, load = synth.cantilever_bc(*t.dims)
    m = t.build_mesh(fixed, load)
    assert len(m.hang_node) > 3
    return m


@pytest.mark.parametrize("corruption", ["master_range", "master_hanging", "weight_nan", "count", "coord", "node"])
def test_corrupt_mesh_tables_rejected(corruption):
    from paper_1009_4975_amd import binding
    m = _octree_mesh()
    hm, hw, hp = m.hang_master.copy(), m.hang_w.copy(), m.hang_ptr.copy()
    xyz, en = m.node_xyz.copy(), m.elem_nodes.copy()
    if corruption == "master_range":
        hm[0] = m.n_nodes
    elif corruption == "master_hanging":
        hm[0] = m.hang_node[1] if m.hang_node[1] != m.hang_node[0] else m.hang_node[2]
    elif corruption == "weight_nan":
        hw[3] = np.nan
    elif corruption == "count":
        hp[1] = hp[0] - 1
    elif corruption == "coord":
        xyz[5, 1] = m.dims[1] + 4
    elif corruption == "node":
        en[2, 3] = -1
    bad = dataclasses.replace(m, hang_master=hm, hang_w=hw, hang_ptr=hp, node_xyz=xyz, elem_nodes=en)
    ctx = binding.Context(0)
    with pytest.raises(binding.AmrtoError) as e:
        ctx.upload_mesh(bad)
    assert code_of(e) == "EINVAL"
    ctx.upload_mesh(m)  # the same context accepts the intact mesh afterwards
    assert ctx.info()["n_nodes"] == m.n_nodes


def test_nonfinite_network_prediction_falls_back():
    """A network whose weights went non-finite: the learned start is refused
    by the library and the iteration proceeds from u_prev (plain solve)."""
    from paper_1009_4975_amd.learned import LearnedWarmStart
    from paper_1009_4975_amd.simp import AdaptiveSIMP
    base, L = (8, 4, 4), 2
    dims = tuple(x << L for x in base)
    fixed, load = synth.bridge_bc(*dims)
    sim = AdaptiveSIMP(base, L, fixed, load, rtol=1e-8)
    ws = LearnedWarmStart(dims, cell=2, hidden=4, layers=2, epochs=5, coarse=None)
    for _ in range(3):
        sim.step(warm_start=ws.collect_before, after_solve=ws.collect_after)
    ws.train()
    params = ws.net.get_params()
    params[:] = np.nan
    ws.net.set_params(params)
    rec = sim.step(warm_start=ws.warm_start)
    assert ws.last["fallback"] is not None and "not finite" in ws.last["fallback"]
    assert rec["rel_res"] <= 1e-8 and np.isfinite(rec["compliance"])
