"""Adaptive SIMP loop on the octree mesh (paper Sec. 2-6).

Each iteration solves K(rho) u = f on the current mesh (Eq. (1), (7)-(9)),
forms the compliance sensitivities (Sec. 3), filters them (Eq. (5)) and takes
an optimality-criteria step; every ``adapt_every`` iterations the mesh is
adapted to the current design (Sec. 4) and rho and u are carried over.  The
previous displacement is the initial guess of the next solve (Sec. 5).

All arithmetic runs in ``libamrto.so``; this module only sequences the calls
and moves the per-leaf arrays between the host octree and the device when the
mesh changes.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding
from .binding import FILTER_SENSITIVITY, FP64


class AdaptiveSIMP:
    def __init__(self, base, max_level, fixed, load, volfrac=0.25, rho_init=0.25, rmin=1.5, move=0.2, eta=0.5,
                 rho_min=1e-3, rho_solid=0.5, r_amr=1.5, adapt_every=5, rtol=1e-8, inner_prec=FP64,
                 inner_rtol=1e-2, max_it=100000, device=0):
        self.tree = binding.Octree(base, max_level)
        self.ctx = binding.Context(device)
        self.dev = torch.device("cuda", device)
        self.fixed, self.load = fixed, load
        self.volfrac, self.rmin, self.move, self.eta, self.rho_min = volfrac, rmin, move, eta, rho_min
        self.rho_solid, self.r_amr, self.adapt_every = rho_solid, r_amr, adapt_every
        self.rtol, self.inner_prec, self.inner_rtol, self.max_it = rtol, inner_prec, inner_rtol, max_it
        self.it = 0
        self.compliance = None
        self.mesh_version = 0
        n = self.tree.lib.amrto_octree_n_leaves(self.tree.h)
        self._set_mesh(np.full(n, rho_init), None)

    # ------------------------------------------------------------------ mesh
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
        self.mesh_version += 1

    def adapt(self):
        """One mesh adaptation (Sec. 4); rho and u are transferred."""
        rho_h = self.rho.cpu().numpy()
        u_h = self.u.cpu().numpy()
        rho_new = self.tree.adapt(rho_h, self.rho_solid, self.r_amr)
        mesh = self.tree.build_mesh(self.fixed, self.load)
        u_new = self.tree.transfer_nodal(u_h, mesh.n_nodes)
        self._set_mesh(rho_new, u_new)

    # ------------------------------------------------------------------ step
    def step(self, warm_start=None, after_solve=None):
        """One design iteration.  ``warm_start(sim)`` may replace ``sim.u`` (the
        initial guess) and set a coarse space on ``sim.ctx`` before the solve;
        ``after_solve(sim)`` sees the new displacement before the design update."""
        rec = {"it": self.it, "adapted": False}
        t0 = time.perf_counter()
        if self.it > 0 and self.adapt_every > 0 and self.it % self.adapt_every == 0:
            self.adapt()
            rec["adapted"] = True
        t1 = time.perf_counter()
        self.ctx.set_density(self.rho)
        if warm_start is not None:
            warm_start(self)
        torch.cuda.synchronize(self.dev)
        t2 = time.perf_counter()
        st = self.ctx.pcg(self.b, self.u, rtol=self.rtol, max_it=self.max_it, inner_prec=self.inner_prec,
                          inner_rtol=self.inner_rtol)
        if after_solve is not None:
            after_solve(self)
        t3 = time.perf_counter()
        c = self.ctx.compliance(self.u, self.f, self.rho, self.dc)
        self.ctx.filter(FILTER_SENSITIVITY, self.rmin, self.dc, self.dcf, rho=self.rho)
        change, lam = self.ctx.oc_update(self.rho, self.dcf, self.rho_new, self.volfrac, move=self.move,
                                         eta=self.eta, rho_min=self.rho_min)
        self.rho, self.rho_new = self.rho_new, self.rho
        self.compliance = c
        self.it += 1
        t4 = time.perf_counter()
        info = self.ctx.info()
        rec.update(n_elems=info["n_elems"], n_nodes=info["n_nodes"], dofs=3 * info["n_nodes"],
                   iters=st["iters"], outer=st["outer"], rel_res=st["rel_res"], solve_ms=st["ms"],
                   warm_ms=1e3 * (t2 - t1), adapt_ms=1e3 * (t1 - t0), design_ms=1e3 * (t4 - t3),
                   step_ms=1e3 * (t4 - t0), compliance=c, change=change, lam=lam)
        return rec
