"""The differentiable zone refuses a backward whose forward state is gone.

The adjoint needs the design-volume DFT and permittivity of the forward run
it differentiates; the zone keeps only the last run's.  A second forward (or
a design change) before the backward must raise instead of returning the
gradient of the later state.  The zone here is a host stand-in with the
binding's state-serial contract (every run, design, permittivity or field
write advances it), so the check runs without a GPU; the GPU test in
test_gpu_autograd.py exercises the real zone."""
import pytest
import torch

from paper_2501_07979_amd.autograd import StaleForwardError, zone_fdtd


class HostZone:
    def __init__(self):
        self.state_serial = 0
        self.rho = None
        self.adjoint_calls = 0

    def set_design(self, rho):
        self.state_serial += 1
        self.rho = rho.clone()

    def run(self, **kw):
        self.state_serial += 1

    def dft(self, monitor):
        return (self.rho.sum() * torch.ones(1, 2, 2, 2)).to(torch.complex64)

    def adjoint_grad(self, g):
        self.adjoint_calls += 1
        return torch.ones_like(self.rho)


def test_backward_after_a_second_forward_raises():
    z = HostZone()
    r1 = torch.rand(2, 2, 2, requires_grad=True)
    r2 = torch.rand(2, 2, 2, requires_grad=True)
    p1 = zone_fdtd(r1, z)
    p2 = zone_fdtd(r2, z)
    with pytest.raises(StaleForwardError):
        p1.abs().sum().backward()
    assert z.adjoint_calls == 0
    p2.abs().sum().backward()          # the latest forward is still differentiable
    assert z.adjoint_calls == 1 and r2.grad is not None


def test_backward_after_a_design_change_raises():
    z = HostZone()
    r = torch.rand(2, 2, 2, requires_grad=True)
    p = zone_fdtd(r, z)
    z.set_design(torch.zeros(2, 2, 2))
    with pytest.raises(StaleForwardError):
        p.abs().sum().backward()
