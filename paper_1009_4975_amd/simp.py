"""Adaptive SIMP loop on the octree mesh (paper Sec. 2-6).

Each iteration solves K(rho) u = f on the current mesh (Eq. (1), (7)-(9)),
forms the compliance sensitivities (Sec. 3), filters them (Eq. (5)) and takes
an optimality-criteria step.  The mesh is adapted to the current design
(Sec. 4) and rho and u are carried over either every ``adapt_every``
iterations (``adapt_rule="every"``) or by the paper's rule (``"paper"``):
CASE (i) the largest design change of the last step is below ``change_tol``
(0.01) after at least ``min_steps`` (5) steps on the mesh, CASE (ii) after
``max_steps`` (10) steps without CASE (i).  The previous displacement is the
initial guess of the next solve (Sec. 5).  ``p_continuation`` (Sec. 3) starts
the penalty at p0 and raises it by dp whenever the design has settled (change
below tol) or max_steps steps were taken at the current p, up to p_max.

All arithmetic runs in ``libamrto.so``; this module only sequences the calls
and moves the per-leaf arrays between the host octree and the device when the
mesh changes.
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from . import binding
from .binding import FILTER_SENSITIVITY, FP64


class AdaptiveSIMP:
    def __init__(self, base, max_level, fixed, load, volfrac=0.25, rho_init=0.25, rmin=1.5, move=0.2, eta=0.5,
                 rho_min=1e-3, rho_solid=0.5, r_amr=1.5, adapt_every=5, rtol=1e-8, inner_prec=FP64,
                 inner_rtol=0.1, max_it=100000, device=0, metrics_path=None, precond=binding.JACOBI,
                 adapt_rule="every", min_steps=5, max_steps=10, change_tol=0.01, p_continuation=None,
                 p=3.0, recycle=None, mg=None):
        self.base, self.max_level = tuple(int(b) for b in base), int(max_level)
        self.tree = binding.Octree(base, max_level)
        self.ctx = binding.Context(device)
        self.dev = torch.device("cuda", device)
        self.fixed, self.load = fixed, load
        self.volfrac, self.rmin, self.move, self.eta, self.rho_min = volfrac, rmin, move, eta, rho_min
        self.rho_solid, self.r_amr, self.adapt_every = rho_solid, r_amr, adapt_every
        self.rtol, self.inner_prec, self.inner_rtol, self.max_it = rtol, inner_prec, inner_rtol, max_it
        self.precond = precond
        if adapt_rule not in ("every", "paper", "never"):
            raise ValueError("adapt_rule must be 'every', 'paper' or 'never'")
        self.adapt_rule, self.min_steps, self.max_steps, self.change_tol = adapt_rule, min_steps, max_steps, change_tol
        self.steps_on_mesh = 0
        self.last_change = float("inf")
        # p-continuation: dict(p0=1, dp=0.5, p_max=3, tol=0.01, max_steps=20) or None (fixed p)
        self.p_cont = None if p_continuation is None else dict(dict(p0=1.0, dp=0.5, p_max=3.0, tol=0.01,
                                                                    max_steps=20), **p_continuation)
        self.p = float(self.p_cont["p0"] if self.p_cont else p)
        self.steps_at_p = 0
        # Krylov recycling, or None.  mode "init": each solve starts from the
        # Galerkin projection of its initial error onto the Ritz vectors of
        # the previous solve (k of them, from its first m residuals); mode
        # "coarse": Rayleigh-Ritz keeps the best `keep` of the carried and new
        # Ritz vectors, which join the affine fields (optional) of the coarse
        # space on `regions`
        self.recycle = None if recycle is None else dict(dict(mode="init", m=64, k=4, keep=4, regions=(3, 2, 2),
                                                              affine=True), **recycle)
        self.rec_vecs = []  # carried vectors (kept Rayleigh-Ritz vectors, then the last harvest)
        # multigrid-preconditioned CG (options of Context.mg_setup, e.g.
        # dict(first=2, degree=1, coarse_degree=2, ratio=50)), or None; the
        # hierarchy is rebuilt with every mesh
        self.mg = None if mg is None else dict(mg)
        self.it = 0
        self.compliance = None
        self.mesh_version = 0
        self.metrics_path = metrics_path
        self.ctx.set_material(p=self.p)
        n = self.tree.lib.amrto_octree_n_leaves(self.tree.h)
        self._set_mesh(np.full(n, rho_init), None)

    # ------------------------------------------------------------------ mesh
    def _set_mesh(self, rho_host, u_host):
        mesh = self.tree.build_mesh(self.fixed, self.load)
        self.ctx.upload_mesh(mesh)
        self.mesh = mesh
        if self.mg is not None:
            self.ctx.mg_setup(self.tree, **self.mg)
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
        if self.recycle is not None:
            self.ctx.recycle_setup(self.recycle["m"])
        # per-mesh counts for the metrics log
        lv = mesh.elem_level.astype(np.int64)
        self.elem_volume = np.ldexp(1.0, 3 * (self.max_level - lv))  # leaf edge 2^(L - level) lattice units
        hang = np.zeros(3 * mesh.n_nodes, bool)
        hang[(3 * mesh.hang_node[:, None] + np.arange(3)).ravel()] = True
        fixed = mesh.dof_fixed.astype(bool)
        self.mesh_counts = dict(elems_per_level=np.bincount(lv, minlength=self.max_level + 1).tolist(),
                                dofs_all=3 * mesh.n_nodes, dofs_hanging=int(hang.sum()),
                                dofs_fixed=int((fixed & ~hang).sum()), dofs_free=int((~fixed & ~hang).sum()))

    def adapt(self):
        """One mesh adaptation (Sec. 4); rho and u are transferred."""
        rho_h = self.rho.cpu().numpy()
        u_h = self.u.cpu().numpy()
        rho_new = self.tree.adapt(rho_h, self.rho_solid, self.r_amr)
        mesh = self.tree.build_mesh(self.fixed, self.load)
        u_new = self.tree.transfer_nodal(u_h, mesh.n_nodes)
        # recycled vectors follow the mesh as the displacement does
        rec = [self.tree.transfer_nodal(v.cpu().numpy(), mesh.n_nodes) for v in self.rec_vecs]
        self._set_mesh(rho_new, u_new)
        self.rec_vecs = [torch.tensor(v, dtype=torch.float64, device=self.dev) for v in rec]
        for v in self.rec_vecs:
            self.ctx.mask(v)
        self.steps_on_mesh = 0

    def adapt_due(self):
        """Whether this iteration starts with an adaptation (Sec. 4)."""
        if self.it == 0 or self.adapt_rule == "never":
            return False
        if self.adapt_rule == "every":
            return self.adapt_every > 0 and self.it % self.adapt_every == 0
        settled = self.last_change < self.change_tol and self.steps_on_mesh >= self.min_steps
        return settled or self.steps_on_mesh >= self.max_steps

    # ------------------------------------------------------------------ step
    def step(self, warm_start=None, after_solve=None):
        """One design iteration.  ``warm_start(sim)`` may replace ``sim.u`` (the
        initial guess) and set a coarse space on ``sim.ctx`` before the solve;
        ``after_solve(sim)`` sees the new displacement before the design update."""
        rec = {"it": self.it, "adapted": False}
        t0 = time.perf_counter()
        if self.adapt_due():
            self.adapt()
            rec["adapted"] = True
        t1 = time.perf_counter()
        self.ctx.set_density(self.rho)
        if warm_start is not None:
            warm_start(self)
        if self.recycle is not None:
            self._recycle_coarse()
        torch.cuda.synchronize(self.dev)
        t2 = time.perf_counter()
        if self.mg is not None:
            st = self.ctx.mg_pcg(self.b, self.u, rtol=self.rtol, max_it=min(self.max_it, 5000), check_every=2)
        else:
            st = self.ctx.pcg(self.b, self.u, rtol=self.rtol, max_it=self.max_it, inner_prec=self.inner_prec,
                              inner_rtol=self.inner_rtol, precond=self.precond, record=self.recycle is not None)
        harvest_s = 0.0
        if self.recycle is not None:
            th = time.perf_counter()
            self._recycle_harvest()
            harvest_s = time.perf_counter() - th
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
        self.steps_on_mesh += 1
        self.last_change = change
        rec["p"] = self.p
        self.steps_at_p += 1
        pc = self.p_cont
        if pc is not None and self.p < pc["p_max"] and (change < pc["tol"] or self.steps_at_p >= pc["max_steps"]):
            self.p = min(pc["p_max"], self.p + pc["dp"])
            self.steps_at_p = 0
            self.ctx.set_material(p=self.p)
        t4 = time.perf_counter()
        info = self.ctx.info()
        rec.update(n_elems=info["n_elems"], n_nodes=info["n_nodes"], dofs=3 * info["n_nodes"],
                   iters=st["iters"], outer=st["outer"], rel_res=st["rel_res"], solve_ms=st["ms"],
                   fell_back=st["fell_back"],
                   warm_ms=1e3 * (t2 - t1 + harvest_s), adapt_ms=1e3 * (t1 - t0), design_ms=1e3 * (t4 - t3),
                   step_ms=1e3 * (t4 - t0), compliance=c, change=change, lam=lam)
        if self.metrics_path is not None:
            self.log_metrics(rec)
        return rec

    def _recycle_start(self):
        """Mode "init": u = the warm start plus the combination of the carried
        Ritz vectors minimising the energy (the initial error's Galerkin
        projection onto their span)."""
        if not self.rec_vecs:
            return
        x0 = torch.empty_like(self.u)
        try:
            self.ctx.energy_combine(self.b, self.rec_vecs, x0, base=self.u)
        except binding.AmrtoError:
            return  # a carried vector is not finite: start from the warm start alone
        self.u.copy_(x0)

    def _recycle_coarse(self):
        """Coarse space of this solve: the affine fields (optional) and the
        best `keep` directions, by Rayleigh-Ritz for the current system, of
        the carried vectors."""
        rc = self.recycle
        if rc["mode"] == "init":
            self._recycle_start()
            return
        W = []
        if self.rec_vecs:
            keep = min(rc["keep"], len(self.rec_vecs))
            W = [torch.empty_like(self.u) for _ in range(keep)]
            try:
                self.ctx.rayleigh_ritz(self.rec_vecs, W)
            except binding.AmrtoError:
                W = []  # the carried vectors lost their independent directions
        if W or rc["affine"]:
            self.ctx.coarse_setup(W, *rc["regions"], affine=rc["affine"])
        self.rec_vecs = W

    def _recycle_harvest(self):
        """Ritz vectors of the recorded solve: the next start's vectors (mode
        "init") or joined to the kept vectors (mode "coarse")."""
        U = [torch.empty_like(self.u) for _ in range(self.recycle["k"])]
        try:
            self.ctx.recycle_harvest(U)
        except binding.AmrtoError:
            U = []  # the solve was too short to harvest k vectors
        if self.recycle["mode"] == "init":
            self.rec_vecs = U
        else:
            self.rec_vecs = self.rec_vecs + U
            self.ctx.coarse_clear()

    def log_metrics(self, rec):
        """Append one JSON line: the step record, the volume fraction of the
        new design, elements per level and the DOF counts of the mesh."""
        rho = self.rho.cpu().numpy()
        line = dict(rec, volume=float(rho @ self.elem_volume / self.elem_volume.sum()), **self.mesh_counts)
        with open(self.metrics_path, "a") as fh:
            fh.write(json.dumps(line) + "\n")

    # ------------------------------------------------------------------ checkpoint
    def state_dict(self):
        """Host arrays that restart the run at the next iteration: the leaf set
        (levels and anchors in Morton order), rho per leaf, u on the mesh nodes,
        the iteration counter, the last compliance, and the state of the
        adaptation trigger and of the p-continuation."""
        levels, anchors = self.tree.leaves()
        return {"base": np.array(self.base, np.int32), "max_level": np.int32(self.max_level),
                "leaf_level": levels, "leaf_anchor": anchors, "rho": self.rho.cpu().numpy(),
                "u": self.u.cpu().numpy(), "it": np.int64(self.it),
                "compliance": np.float64(np.nan if self.compliance is None else self.compliance),
                "p": np.float64(self.p), "steps_on_mesh": np.int64(self.steps_on_mesh),
                "last_change": np.float64(self.last_change), "steps_at_p": np.int64(self.steps_at_p)}

    def load_state_dict(self, st):
        """Rebuild the tree from the saved leaf set (refining every leaf that
        is a strict ancestor of a saved leaf, level by level), then the mesh,
        rho and u.  The leaf set was 2:1 balanced when saved, so no closure is
        needed, and the same leaves give the same node numbering."""
        if tuple(int(b) for b in st["base"]) != self.base or int(st["max_level"]) != self.max_level:
            raise ValueError("checkpoint is for another base grid or level count")
        lv_s = np.asarray(st["leaf_level"], np.int64)
        self.tree = rebuild_tree(self.base, self.max_level, lv_s, st["leaf_anchor"])
        rho, u = np.asarray(st["rho"], np.float64), np.asarray(st["u"], np.float64)
        if len(rho) != len(lv_s):
            raise ValueError("checkpoint rho does not match its leaf set")
        self._set_mesh(rho, None)
        if len(u) != self.f.numel():
            raise ValueError("checkpoint u does not match the mesh of its leaf set")
        self.u.copy_(torch.from_numpy(u))
        self.it = int(st["it"])
        c = float(st["compliance"])
        self.compliance = None if np.isnan(c) else c
        if "p" in st:
            self.p = float(st["p"])
            self.steps_on_mesh = int(st["steps_on_mesh"])
            self.last_change = float(st["last_change"])
            self.steps_at_p = int(st["steps_at_p"])
            self.ctx.set_material(p=self.p)


def rebuild_tree(base, max_level, levels, anchors):
    """Octree whose leaves are exactly (levels, anchors) (anchors in units of
    the finest lattice): every leaf that is a strict ancestor of a wanted leaf
    is refined, one level per pass."""
    lv_s = np.asarray(levels, np.int64)
    an_s = np.asarray(anchors, np.int64).reshape(-1, 3)
    L = int(max_level)
    ancestors = set()
    for lev, a in zip(lv_s, an_s):
        for l in range(int(lev)):
            size = 1 << (L - l)
            ancestors.add((l, *(int(x) for x in a // size * size)))
    tree = binding.Octree(base, L)
    for _ in range(L + 1):
        lv, an = tree.leaves()
        marks = np.array([(int(l), *(int(x) for x in a)) in ancestors for l, a in zip(lv, an)], np.uint8)
        if not marks.any():
            break
        tree.refine(marks)
    lv, an = tree.leaves()
    if not (np.array_equal(lv, lv_s) and np.array_equal(an, an_s)):
        raise ValueError("leaf set is not a tree of this base grid")
    return tree


def save_checkpoint(path, sim, learned=None):
    """One .npz (plain arrays, no pickled objects) with the SIMP state and,
    optionally, the learned warm start (weights, Adam moments, training pairs)."""
    arrays = {"sim/" + k: v for k, v in sim.state_dict().items()}
    if learned is not None:
        arrays.update({"net/" + k: v for k, v in learned.state_dict().items()})
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)


def load_checkpoint(path, sim, learned=None):
    """Restore what save_checkpoint wrote into objects built with the same
    configuration."""
    with np.load(path, allow_pickle=False) as z:
        sim.load_state_dict({k[4:]: z[k] for k in z.files if k.startswith("sim/")})
        if learned is not None:
            net = {k[4:]: z[k] for k in z.files if k.startswith("net/")}
            if not net:
                raise ValueError("checkpoint holds no learned state")
            learned.load_state_dict(net)
