"""The binding rejects buffers of the wrong length before anything reaches the
library (the C ABI takes bare device pointers, so a short or stale buffer
would be read or written out of bounds by the kernels).  CPU only: the
context below has a mesh but no device, and its library handle fails the
test if any entry point is called."""
import types

import numpy as np
import pytest
import torch

from paper_1009_4975_amd import binding


class NoCalls:
    def __getattr__(self, name):
        def call(*a):
            raise AssertionError(f"library entry point {name} called")
        return call


def fake_context(nn=10, ne=4, dims=(4, 2, 2)):
    ctx = object.__new__(binding.Context)
    ctx.lib = NoCalls()
    ctx.torch = torch
    ctx.h = None
    ctx.mesh = types.SimpleNamespace(n_nodes=nn, n_elems=ne, dims=dims)
    return ctx


def vec(n, dt=torch.float64):
    return torch.zeros(n, dtype=dt)


CALLS = [
    ("set_density", lambda c, n3, ne: c.set_density(vec(ne + 1))),
    ("apply", lambda c, n3, ne: c.apply(vec(n3), vec(n3 - 3))),
    ("apply fp32", lambda c, n3, ne: c.apply(vec(n3 - 1, torch.float32), vec(n3, torch.float32), binding.FP32)),
    ("project_rhs", lambda c, n3, ne: c.project_rhs(vec(n3), vec(2 * n3))),
    ("recover", lambda c, n3, ne: c.recover(vec(n3 + 3), vec(n3))),
    ("diag", lambda c, n3, ne: c.diag(vec(n3 - 3))),
    ("block_diag", lambda c, n3, ne: c.block_diag(vec(n3))),
    ("pcg", lambda c, n3, ne: c.pcg(vec(n3), vec(n3 - 3))),
    ("compliance", lambda c, n3, ne: c.compliance(vec(n3), vec(n3), vec(ne), vec(ne - 1))),
    ("sensitivity", lambda c, n3, ne: c.sensitivity(vec(n3 - 3), vec(ne), vec(ne))),
    ("filter", lambda c, n3, ne: c.filter(0, 1.5, vec(ne), vec(ne), rho=vec(ne + 2))),
    ("oc_update", lambda c, n3, ne: c.oc_update(vec(ne), vec(ne), vec(ne - 1), 0.25)),
    ("mask", lambda c, n3, ne: c.mask(vec(n3 + 1))),
    ("coarse_setup", lambda c, n3, ne: c.coarse_setup([vec(n3), vec(n3 - 3)], 1, 1, 1)),
    ("energy_combine", lambda c, n3, ne: c.energy_combine(vec(n3), [vec(n3)], vec(n3), base=vec(n3 + 3))),
    ("grid_from_mesh", lambda c, n3, ne: c.grid_from_mesh(2, rho=vec(ne), rho_grid=vec(17, torch.float32))),
    ("grid_to_mesh", lambda c, n3, ne: c.grid_to_mesh(2, vec(3 * 18 + 1, torch.float32), vec(n3))),
]


@pytest.mark.parametrize("name,call", CALLS, ids=[c[0] for c in CALLS])
def test_wrong_length_rejected_before_launch(name, call):
    ctx = fake_context()
    with pytest.raises(binding.AmrtoError) as ei:
        call(ctx, 30, 4)
    assert ei.value.code == -1 and "expected" in str(ei.value)


def test_right_lengths_pass_the_size_check():
    """Correct lengths get past the size check and stop only at the device
    check (these are host tensors): the size check is not over-strict."""
    ctx = fake_context()
    for call in (lambda: ctx.apply(vec(30), vec(30)), lambda: ctx.oc_update(vec(4), vec(4), vec(4), 0.25),
                 lambda: ctx.block_diag(vec(90)), lambda: ctx.grid_to_mesh(2, vec(3 * 12, torch.float32), vec(30)),
                 lambda: ctx.grid_from_mesh(2, rho=vec(4), rho_grid=vec(12, torch.float32))):
        with pytest.raises(binding.AmrtoError, match="device tensor"):
            call()


def test_net_buffers_checked():
    net = object.__new__(binding.Net)
    net.lib = NoCalls()
    net.torch = torch
    net.h = None
    net.channels = [2, 8, 3]
    net.grid = (4, 3, 2)
    with pytest.raises(binding.AmrtoError, match="expected"):
        net.forward(torch.zeros(1, 2, 2, 3, 5), torch.zeros(1, 3, 2, 3, 4))
    with pytest.raises(binding.AmrtoError, match="expected"):
        net.forward(torch.zeros(1, 2, 2, 3, 4), torch.zeros(2, 3, 2, 3, 4))
    with pytest.raises(binding.AmrtoError, match="expected"):
        net.mse(torch.zeros(10), torch.zeros(10), torch.zeros(9))
