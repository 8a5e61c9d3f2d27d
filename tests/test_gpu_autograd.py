"""torch.autograd through the zone: forward FDTD + DFT, focal objective,
backward = adjoint FDTD + overlap, against the FP64 oracle's adjoint gradient
of the same objective."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-autograd]", *a, flush=True)


def test_autograd_focal_objective_matches_oracle(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import objective, zda
    from paper_2501_07979_amd.autograd import zone_fdtd
    from paper_2501_07979_amd.workloads import c3_small

    wl = c3_small()
    rho0 = wl.rho()
    eps = wl.eps(rho0)
    om = np.array(wl.omegas)
    focal = objective.focal_length(wl.r_in + 0.5 * wl.nr * wl.dr)
    W = objective.focal_weights(wl, om, focal)
    zone = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    rho = torch.tensor(rho0, device="cuda", requires_grad=True)
    _say("forward + backward", wl.name)
    plane = zone_fdtd(rho, zone, nsteps=wl.steps, omegas=wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c,
                      width=wl.width)
    F, a = objective.focal_objective(plane, W)
    F.backward()
    g_gpu = rho.grad.cpu().numpy()

    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=eps)
    fwd = o.forward(wl.steps, om, omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src, volume=True)
    Wn = W.cpu().numpy().astype(np.complex128)
    a_ref = np.einsum("kaij,kaij->k", Wn, fwd["plane"])
    assert np.allclose(a.detach().cpu().numpy(), a_ref, rtol=1e-4)
    dF = np.conj(a_ref)[:, None, None, None] * Wn
    g_ref = o.adjoint_grad(dF)
    err = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    _say("autograd gradient rel L2 vs oracle = %.3e" % err)
    assert err <= 1e-4
    zone.close()


def test_autograd_refuses_a_stale_forward():
    """Two forward runs on one zone, then the first one's backward: the zone
    holds only the second run's state, so the backward must raise."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda
    from paper_2501_07979_amd.autograd import StaleForwardError, zone_fdtd
    from paper_2501_07979_amd.workloads import c3_small

    wl = c3_small()
    zone = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps(wl.rho()))
    kw = dict(nsteps=200, omegas=wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    r1 = torch.tensor(wl.rho(), device="cuda", requires_grad=True)
    r2 = torch.tensor(1.0 - wl.rho(), device="cuda", requires_grad=True)
    _say("two forwards, then the first backward")
    p1 = zone_fdtd(r1, zone, **kw)
    p2 = zone_fdtd(r2, zone, **kw)
    with pytest.raises(StaleForwardError):
        p1.abs().pow(2).sum().backward()
    p2.abs().pow(2).sum().backward()
    assert r2.grad is not None and torch.isfinite(r2.grad).all()
    zone.close()
