"""Checkpoint/resume of the adaptive SIMP run and its learned warm start, and
the per-iteration metrics log.  A resumed run must continue as the
uninterrupted one does: the same designs and compliances (solves agree to
their tolerance; FP64 accumulation order moves iteration counts by a step or
two), the same network and optimiser state."""
import json

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BASE, L = (8, 4, 4), 2


def make_sim(**kw):
    from paper_1009_4975_amd.simp import AdaptiveSIMP
    dims = tuple(x << L for x in BASE)
    fixed, load = synth.bridge_bc(*dims)
    return AdaptiveSIMP(BASE, L, fixed, load, rtol=1e-9, **kw)


def make_learned():
    from paper_1009_4975_amd.learned import LearnedWarmStart
    dims = tuple(x << L for x in BASE)
    return LearnedWarmStart(dims, cell=2, hidden=4, layers=2, epochs=20, coarse=None)


def test_resume_continues_the_run(tmp_path):
    from paper_1009_4975_amd.simp import load_checkpoint, save_checkpoint
    full = make_sim()
    recs = [full.step() for _ in range(8)]
    assert any(r["adapted"] for r in recs)
    part = make_sim()
    for _ in range(6):
        part.step()
    path = tmp_path / "run.npz"
    save_checkpoint(path, part)
    resumed = make_sim()
    load_checkpoint(path, resumed)
    assert resumed.it == 6 and resumed.compliance == part.compliance
    assert torch.equal(resumed.u, part.u) and torch.equal(resumed.rho, part.rho)
    assert resumed.mesh.n_nodes == part.mesh.n_nodes
    assert np.array_equal(resumed.mesh.elem_nodes, part.mesh.elem_nodes)
    for want in recs[6:]:
        got = resumed.step()
        assert got["it"] == want["it"] and got["n_elems"] == want["n_elems"]
        assert got["compliance"] == pytest.approx(want["compliance"], rel=1e-6)
        assert abs(got["iters"] - want["iters"]) <= max(2, want["iters"] // 20)
    assert torch.allclose(resumed.rho, full.rho, rtol=0, atol=1e-6)


def test_resume_restores_learned_state(tmp_path):
    from paper_1009_4975_amd.simp import load_checkpoint, save_checkpoint
    sim, ws = make_sim(), make_learned()
    for _ in range(5):
        sim.step(warm_start=ws.collect_before, after_solve=ws.collect_after)
    ws.train()
    path = tmp_path / "run.npz"
    save_checkpoint(path, sim, ws)
    sim2, ws2 = make_sim(), make_learned()
    load_checkpoint(path, sim2, ws2)
    assert ws2.n_pairs == ws.n_pairs == 4 and ws2.adam_t == ws.adam_t == 20 and ws2.trained
    assert np.array_equal(ws2.net.get_params(), ws.net.get_params())
    for a, b in zip(ws2.net.get_adam(), ws.net.get_adam()):
        assert np.array_equal(a, b)
    assert torch.equal(ws2.X[:4], ws.X[:4]) and torch.equal(ws2.Y[:4], ws.Y[:4])
    # the same further training from the same state
    ws.train(epochs=5)
    ws2.train(epochs=5)
    p, p2 = ws.net.get_params(), ws2.net.get_params()
    assert np.abs(p - p2).max() <= 1e-5 * np.abs(p).max()
    # a checkpoint without learned state is refused for a learned restore
    save_checkpoint(path, sim)
    with pytest.raises(ValueError):
        load_checkpoint(path, make_sim(), make_learned())


def test_checkpoint_for_another_grid_refused(tmp_path):
    from paper_1009_4975_amd.simp import AdaptiveSIMP, load_checkpoint, save_checkpoint
    sim = make_sim()
    sim.step()
    path = tmp_path / "run.npz"
    save_checkpoint(path, sim)
    dims = tuple(x << 1 for x in BASE)
    fixed, load = synth.bridge_bc(*dims)
    with pytest.raises(ValueError):
        load_checkpoint(path, AdaptiveSIMP(BASE, 1, fixed, load))


def test_metrics_log(tmp_path):
    path = tmp_path / "metrics.jsonl"
    sim = make_sim(metrics_path=path)
    for _ in range(6):
        sim.step()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["it"] for x in lines] == list(range(6))
    for x in lines:
        assert x["volume"] == pytest.approx(sim.volfrac, rel=1e-9)
        assert sum(x["elems_per_level"]) == x["n_elems"] and len(x["elems_per_level"]) == L + 1
        assert x["dofs_free"] + x["dofs_fixed"] + x["dofs_hanging"] == x["dofs_all"] == x["dofs"]
        assert x["rel_res"] <= 1e-9 and x["iters"] > 0 and x["solve_ms"] > 0
    assert lines[5]["adapted"] and lines[5]["dofs_hanging"] > 0
