"""Seven SIMP iterations with three adaptations on a small bridge octree (4x2x2
base leaves, two levels, initial density and volume fraction 0.4, adapt
every second iteration: 16 -> 44 -> 296 -> 520 leaves), the library's loop
(AdaptiveSIMP: PCG to 1e-12, sensitivities, Eq. (5) filter, OC, host
adaptation with density and displacement transfer) against a loop built only
from the oracle (direct solve, dc, Eq. (5) filter, OC by bisection, Sec. 4
adaptation, field transfer).  Per iteration: the leaf set, the compliance, the
new densities and the largest design change; at each adaptation the
transferred displacement (the warm start of the next solve)."""
import numpy as np
import pytest

import synth
from oracle import amr, mesh as om, system as osys, topopt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_simp_sequence_with_adapt_matches_oracle_loop(lib):
    from paper_1009_4975_amd.simp import AdaptiveSIMP
    base, L, every, n_it = (4, 2, 2), 2, 2, 7
    dims = tuple(b << L for b in base)
    fixed, load = synth.bridge_bc(*dims)
    volfrac, rmin, rho_s, r_amr = 0.4, 1.5, 0.5, 1.5
    sim = AdaptiveSIMP(base, L, fixed, load, volfrac=volfrac, rho_init=0.4, rmin=rmin, rho_solid=rho_s,
                       r_amr=r_amr, adapt_every=every, rtol=1e-12)
    lv = np.zeros(np.prod(base), np.int64)
    an = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])]) << L
    rho = np.full(len(lv), 0.4)
    seen = {}

    def warm(s):
        seen["u0"] = s.u.cpu().numpy().copy()
        seen["xyz"] = s.mesh.node_xyz.copy()

    m_prev = u_prev = None
    n_adapt = 0
    for it in range(n_it):
        adapted = it > 0 and it % every == 0
        if adapted:
            lv, an, rho, _ = amr.adapt(lv, an, L, rho, rho_s, r_amr)
            n_adapt += 1
        m = om.build_mesh(lv, an, L, dims)
        f = om.load_vector(m, load)
        s = osys.build_system(m, osys.elem_coeff(m, rho), om.fixed_dofs(m, fixed), f)
        u = osys.recover(s, osys.solve_direct(s))
        c = topopt.compliance(f, u)
        dcf = topopt.filter_sensitivity(m, rmin, rho, topopt.sensitivities(m, rho, u))
        rho_new, _, change = topopt.oc_update(rho, dcf, m.volumes, volfrac * m.volumes.sum())

        rec = sim.step(warm_start=warm)
        assert rec["adapted"] == adapted
        tl, ta = sim.tree.leaves()
        key = {(int(l), *map(int, a)): e for e, (l, a) in enumerate(zip(lv, an))}
        assert {(int(l), *map(int, a)) for l, a in zip(tl, ta)} == set(key), f"leaf sets differ at iteration {it}"
        perm = np.array([key[(int(l), *map(int, a))] for l, a in zip(tl, ta)])
        assert rec["compliance"] == pytest.approx(c, rel=1e-9), f"compliance at iteration {it}"
        got = sim.rho.cpu().numpy()
        assert np.max(np.abs(got - rho_new[perm])) <= 1e-8, f"densities at iteration {it}"
        assert rec["change"] == pytest.approx(change, rel=1e-6, abs=1e-10)
        if adapted:
            # warm start after the transfer: the old FE field at the new nodes
            want = amr.transfer_displacement(m_prev, u_prev, seen["xyz"].astype(np.int64))
            assert np.max(np.abs(seen["u0"] - want)) <= 1e-8 * np.max(np.abs(want)), f"transfer at iteration {it}"
        m_prev, u_prev, rho = m, u, rho_new
    assert n_adapt == 3
    assert len(lv) == 520 and lv.max() == L, "the adaptations did not refine to the finest level"
