"""Adaptive SIMP loop of the 2-D variant (paper Sec. 6-7, Test 1) on the
quadtree mesh: Q4 plane-stress elements, FP64 Jacobi-PCG warm-started from the
previous displacement, compliance sensitivities, the Eq. (5) filter with area
weights and the OC step, with a mesh adaptation (Sec. 4) every
``adapt_every`` iterations (``adapt_every=0`` keeps the mesh).

All arithmetic runs in ``libamrto.so``; this module sequences the calls and
moves the per-leaf arrays between the host quadtree and the device when the
mesh changes.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding
from .binding import FILTER_SENSITIVITY


def cantilever_2d(dims):
    """Left edge supported, a unit downward point load at the middle of the
    right edge (lattice units)."""
    return [{"x": 0}], {"at": (dims[0], dims[1] // 2), "comp": 1, "total": -1.0}


class PlaneSIMP:
    def __init__(self, base, max_level, fixed=None, load=None, volfrac=0.5, rho_init=None, rmin=1.5, move=0.2,
                 eta=0.5, rho_min=1e-3, rho_solid=0.5, r_amr=1.5, adapt_every=10, uniform=False, rtol=1e-8,
                 max_it=100000, check_every=32, p=3.0, device=0):
        self.base, self.max_level = tuple(int(b) for b in base), int(max_level)
        self.tree = binding.Quadtree(base, max_level)
        if uniform:  # every leaf at the finest level: the fixed-grid reference
            for _ in range(self.max_level):
                self.tree.refine(np.ones(self.tree.n_leaves, np.uint8))
        self.dims = self.tree.dims
        dfix, dload = cantilever_2d(self.dims)
        self.fixed = dfix if fixed is None else fixed
        self.load = dload if load is None else load
        self.ctx = binding.PlaneContext(device)
        self.dev = torch.device("cuda", device)
        self.volfrac, self.rmin, self.move, self.eta, self.rho_min = volfrac, rmin, move, eta, rho_min
        self.rho_solid, self.r_amr, self.adapt_every = rho_solid, r_amr, adapt_every
        self.rtol, self.max_it, self.check_every = rtol, max_it, check_every
        self.p = float(p)
        self.ctx.set_material(p=self.p)
        self.it = 0
        self.compliance = None
        self._set_mesh(np.full(self.tree.n_leaves, volfrac if rho_init is None else rho_init), None)

    def _set_mesh(self, rho_host, u_host):
        mesh = self.tree.build_mesh(self.fixed, self.load)
        self.ctx.upload_mesh(mesh)
        self.mesh = mesh
        d = self.dev
        self.f = torch.tensor(mesh.f_load, dtype=torch.float64, device=d)
        self.b = torch.empty_like(self.f)
        self.ctx.project_rhs(self.f, self.b)
        self.rho = torch.tensor(rho_host, dtype=torch.float64, device=d)
        self.rho_new = torch.empty_like(self.rho)
        self.dc = torch.empty_like(self.rho)
        self.dcf = torch.empty_like(self.rho)
        self.u = (torch.zeros_like(self.f) if u_host is None
                  else torch.tensor(u_host, dtype=torch.float64, device=d))

    def adapt(self):
        """One mesh adaptation (Sec. 4); rho and u are transferred."""
        rho_new = self.tree.adapt(self.rho.cpu().numpy(), self.rho_solid, self.r_amr)
        u_h = self.u.cpu().numpy()
        mesh = self.tree.build_mesh(self.fixed, self.load)
        self._set_mesh(rho_new, self.tree.transfer_nodal(u_h, mesh.n_nodes))

    def leaves(self):
        return self.tree.leaves()

    def step(self):
        rec = {"it": self.it, "adapted": False}
        t0 = time.perf_counter()
        if self.it > 0 and self.adapt_every > 0 and self.it % self.adapt_every == 0:
            self.adapt()
            rec["adapted"] = True
        t1 = time.perf_counter()
        self.ctx.set_density(self.rho)
        st = self.ctx.pcg(self.b, self.u, rtol=self.rtol, max_it=self.max_it, check_every=self.check_every)
        if st["status"] != "OK":
            raise binding.AmrtoError(1, f"2-D solve: {st}")
        t2 = time.perf_counter()
        c = self.ctx.compliance(self.u, self.f, self.rho, self.dc)
        self.ctx.filter(FILTER_SENSITIVITY, self.rmin, self.dc, self.dcf, rho=self.rho)
        change, lam = self.ctx.oc_update(self.rho, self.dcf, self.rho_new, self.volfrac, move=self.move,
                                         eta=self.eta, rho_min=self.rho_min)
        self.rho, self.rho_new = self.rho_new, self.rho
        self.compliance = c
        self.it += 1
        t3 = time.perf_counter()
        rec.update(n_elems=self.mesh.n_elems, n_nodes=self.mesh.n_nodes, dofs=2 * self.mesh.n_nodes,
                   iters=st["iters"], rel_res=st["rel_res"], solve_ms=st["ms"], adapt_ms=1e3 * (t1 - t0),
                   design_ms=1e3 * (t3 - t2), step_ms=1e3 * (t3 - t0), compliance=c, change=change, lam=lam)
        return rec
