"""Learned warm start and coarse correction for the SIMP solves.

Not in the paper, whose solves start from the previous displacement (Sec. 5);
that stays the baseline, and the plain preconditioned solve stays the judge of
every result: the network only proposes vectors.

* Grid: nodes every ``cell`` lattice units over the domain.  Input channels
  [rho, u_prev / c_prev] (density as a dual-cell volume average, displacement
  sampled from the FE field, scaled by the previous compliance so that values
  are O(1) for a unit load); output (u_next - u_prev) / c_prev, the change of
  the displacement between design iterations.  The last layer starts at zero,
  so the untrained network proposes no change.
* Training: pairs (iteration k input, iteration k change) from the first
  iterations of the run, full-batch Adam on the mean squared error, all in the
  library's FP32 kernels.
* Use: the predicted change d is interpolated to the mesh and the initial
  guess is u_prev + a d with the energy-minimising a (a line search, so never
  worse than u_prev in the energy norm; u_prev itself is not rescaled, which
  would bring a global smooth error that Jacobi-PCG removes slowly).
* Coarse space: the affine fields (rigid motions and constant strains) on
  rx x ry x rz boxes, optionally with the predicted change as a further field:
  M^-1 = D^-1 + Z (Z^T A Z)^-1 Z^T, SPD for any Z.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding


class LearnedWarmStart:
    def __init__(self, dims, cell=2, hidden=16, layers=4, seed=0, max_pairs=16, lr=1e-3, epochs=300,
                 regions=(2, 2, 2), coarse="affine", device=0):
        nx, ny, nz = dims
        if nx % cell or ny % cell or nz % cell:
            raise ValueError("cell must divide the lattice extents")
        self.cell = cell
        self.G = (nx // cell + 1, ny // cell + 1, nz // cell + 1)
        gx, gy, gz = self.G
        self.dev = torch.device("cuda", device)
        channels = [4] + [hidden] * (layers - 1) + [3]
        self.net = binding.Net(channels, self.G, max_batch=max_pairs, seed=seed, device=device)
        # last layer starts at zero: the untrained network predicts no change
        params = self.net.get_params()
        n_last = channels[-1] * channels[-2] * 27 + channels[-1]
        params[-n_last:] = 0.0
        self.net.set_params(params)
        self.max_pairs = max_pairs
        self.X = torch.zeros(max_pairs, 4, gz, gy, gx, dtype=torch.float32, device=self.dev)
        self.Y = torch.zeros(max_pairs, 3, gz, gy, gx, dtype=torch.float32, device=self.dev)
        self.Xq = torch.zeros(1, 4, gz, gy, gx, dtype=torch.float32, device=self.dev)  # inference input
        self.out = torch.zeros(max_pairs, 3, gz, gy, gx, dtype=torch.float32, device=self.dev)
        self.dout = torch.zeros_like(self.out)
        self.n_pairs = 0
        self.lr, self.epochs = lr, epochs
        self.regions = tuple(regions)
        if coarse not in (None, "affine", "affine+pred"):
            raise ValueError("coarse must be None, 'affine' or 'affine+pred'")
        self.coarse = coarse
        self._uref = None
        self.trained = False
        self.adam_t = 0  # Adam steps taken (bias correction continues across train calls)
        self.loss_history = []
        self.last = {}
        self._scale = None

    # ------------------------------------------------------------------ data
    def _features(self, sim, x):
        """x (4, gz, gy, gx) = [rho, u_prev / c_prev] of the iteration about to be solved."""
        self._scale = 1.0 / sim.compliance
        sim.ctx.grid_from_mesh(self.cell, rho=sim.rho, u=sim.u, u_scale=self._scale, rho_grid=x[0], u_grid=x[1:4])

    def collect_before(self, sim):
        """warm_start hook of the training iterations: record the input."""
        self._pending = None
        if sim.compliance is None or self.n_pairs >= self.max_pairs:
            return
        self._features(sim, self.X[self.n_pairs])
        if self._uref is None or self._uref.shape != sim.u.shape:
            self._uref = torch.empty_like(sim.u)
        self._uref.copy_(sim.u)
        self._pending = self.n_pairs

    def collect_after(self, sim):
        """after_solve hook of the training iterations: record the target change."""
        if self._pending is None:
            return
        sim.ctx.grid_from_mesh(self.cell, u=sim.u, u_ref=self._uref, u_scale=self._scale,
                               u_grid=self.Y[self._pending])
        self.n_pairs += 1
        self._pending = None

    # ------------------------------------------------------------------ training
    def train(self, epochs=None):
        n = self.n_pairs
        if n == 0:
            raise RuntimeError("no training pairs")
        epochs = self.epochs if epochs is None else epochs
        t0 = time.perf_counter()
        X, Y, out, dout = self.X[:n], self.Y[:n], self.out[:n], self.dout[:n]
        for _ in range(epochs):
            self.net.forward(X, out)
            loss = self.net.mse(out, Y, dout)
            self.net.backward(dout)
            self.adam_t += 1
            self.net.adam(self.lr, self.adam_t)
            self.loss_history.append(loss)
        torch.cuda.synchronize(self.dev)
        self.trained = True
        self.train_ms = 1e3 * (time.perf_counter() - t0)
        return self.loss_history[-1]

    def baseline_loss(self):
        """Loss of the no-change prediction (u_next = u_prev) on the training pairs."""
        n = self.n_pairs
        zero = torch.zeros_like(self.Y[:n])
        return self.net.mse(zero, self.Y[:n], self.dout[:n])

    # ------------------------------------------------------------------ checkpoint
    def state_dict(self):
        n = self.n_pairs
        m, v = self.net.get_adam()
        return {"params": self.net.get_params(), "adam_m": m, "adam_v": v, "adam_t": np.int64(self.adam_t),
                "n_pairs": np.int64(n), "X": self.X[:n].cpu().numpy(), "Y": self.Y[:n].cpu().numpy(),
                "trained": np.int8(self.trained), "loss_history": np.asarray(self.loss_history, np.float64)}

    def load_state_dict(self, st):
        n = int(st["n_pairs"])
        if n > self.max_pairs or tuple(st["X"].shape[1:]) != tuple(self.X.shape[1:]):
            raise ValueError("checkpoint is for another grid or pair capacity")
        self.net.set_params(st["params"])
        self.net.set_adam(st["adam_m"], st["adam_v"])
        self.adam_t = int(st["adam_t"])
        self.n_pairs = n
        self.X[:n].copy_(torch.from_numpy(np.asarray(st["X"], np.float32)))
        self.Y[:n].copy_(torch.from_numpy(np.asarray(st["Y"], np.float32)))
        self.trained = bool(st["trained"])
        self.loss_history = [float(x) for x in st["loss_history"]]

    # ------------------------------------------------------------------ use
    def predict(self, sim):
        """Predicted change of the displacement on the mesh (supported and
        hanging entries zeroed)."""
        self._features(sim, self.Xq[0])
        self.net.forward(self.Xq, self.out[:1])
        d = torch.empty_like(sim.u)
        sim.ctx.grid_to_mesh(self.cell, self.out[0], d, scale=1.0 / self._scale)
        sim.ctx.mask(d)
        return d

    def warm_start(self, sim, use_net=True, coarse=None):
        """warm_start hook of the later iterations: initial guess and coarse space."""
        t0 = time.perf_counter()
        coarse = self.coarse if coarse is None else (None if coarse is False else coarse)
        uprev = sim.u
        sim.ctx.mask(uprev)  # the solve ignores these entries of its initial guess anyway
        coef, kept, d, fallback = [], 0, None, None
        if use_net:
            d = self.predict(sim)
            x0 = torch.empty_like(uprev)
            try:
                coef = sim.ctx.energy_combine(sim.b, [d], x0, base=uprev)
                sim.u = x0
            except binding.AmrtoError as err:  # e.g. a non-finite prediction: keep u_prev
                fallback, d = str(err), None
        if coarse:
            extra = [d] if (coarse == "affine+pred" and d is not None) else []
            try:
                kept = sim.ctx.coarse_setup(extra, *self.regions, affine=True)
            except binding.AmrtoError as err:  # plain Jacobi-PCG then
                sim.ctx.coarse_clear()
                fallback = str(err)
        torch.cuda.synchronize(self.dev)
        self.last = dict(coef=coef, kept=kept, fallback=fallback, ms=1e3 * (time.perf_counter() - t0))
