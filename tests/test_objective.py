"""The focal-spot objective: the wedge-weighted projection equals a direct
first Rayleigh-Sommerfeld quadrature of the Cartesian field over the whole
ring of n wedge copies (Bloch-tiled), and its gradient convention matches
torch's complex autograd."""
import numpy as np
import torch

from paper_2501_07979_amd import objective
from paper_2501_07979_amd.workloads import Workload


def test_wedge_weights_equal_full_ring_quadrature():
    rng = np.random.default_rng(3)
    wl = Workload("obj", r_in=60.0, nr=20, nphi=12, nz=10, n_fold=9, m=1, pml=(3, 4, 2, 2))
    om = (0.3, 0.41)
    F = 140.0
    W = objective.focal_weights(wl, om, F, device="cpu").numpy()
    Er = rng.standard_normal((2, wl.nr, wl.nphi)) + 1j * rng.standard_normal((2, wl.nr, wl.nphi))
    Ep = rng.standard_normal((2, wl.nr, wl.nphi)) + 1j * rng.standard_normal((2, wl.nr, wl.nphi))
    plane = np.stack([Er, Ep], axis=1)
    a = np.einsum("kaij,kaij->k", W.astype(np.complex128), plane)
    # direct quadrature over the ring: tile with the Bloch phase of m = 1
    n, dphi = wl.n_fold, 2 * np.pi / (wl.n_fold * wl.nphi)
    tau = 2 * np.pi / n
    ri = wl.r_in + np.arange(wl.nr) * wl.dr
    rh = ri + 0.5 * wl.dr
    act = np.zeros(wl.nr)
    act[wl.pml[0]:wl.nr - wl.pml[1]] = 1
    for k, w in enumerate(om):
        ex = ey = 0.0
        for l in range(n):
            ph = np.exp(1j * wl.m * l * tau)
            for (r, comp, off) in ((rh, 0, 0.0), (ri, 1, 0.5)):
                phi = (np.arange(wl.nphi) + off) * dphi + l * tau
                R = np.sqrt(r * r + F * F)
                G = (F / R) * (1j * w - 1 / R) * np.exp(1j * w * R) / R / (2 * np.pi)
                f = ph * plane[k, comp]
                # each staggered component contributes its own Cartesian parts
                if comp == 0:
                    cx, cy = np.cos(phi), np.sin(phi)
                else:
                    cx, cy = -np.sin(phi), np.cos(phi)
                wq = (act * G * r * wl.dr * dphi)[:, None]
                ex = ex + np.sum(wq * f * cx[None, :])
                ey = ey + np.sum(wq * f * cy[None, :])
        direct = 0.5 * (ex - 1j * ey)
        assert abs(direct - a[k]) < 1e-6 * abs(a[k])   # weights are complex64


def test_objective_gradient_convention():
    """backward passes conj(grad)/2 as dF/dEhat: check on the objective."""
    rng = np.random.default_rng(4)
    wl = Workload("obj", r_in=60.0, nr=10, nphi=8, nz=10, n_fold=9, m=1, pml=(2, 2, 2, 2))
    W = objective.focal_weights(wl, (0.3,), 100.0, device="cpu").to(torch.complex128)
    p = torch.tensor(rng.standard_normal((1, 2, 10, 8)) + 1j * rng.standard_normal((1, 2, 10, 8)),
                     requires_grad=True)
    F, a = objective.focal_objective(p, W)
    F.backward()
    holo = (a.conj()[:, None, None, None] * W).detach()
    assert torch.allclose(p.grad.conj() * 0.5, holo, rtol=1e-12, atol=1e-14)


def test_filter_and_projection_are_differentiable_and_periodic():
    rho = torch.rand(4, 9, 16, dtype=torch.float64, requires_grad=True)
    out = objective.tanh_projection(objective.gaussian_filter_phi_periodic(rho, 1.5), 8.0)
    assert out.shape == rho.shape and float(out.min()) >= 0 and float(out.max()) <= 1
    shifted = objective.gaussian_filter_phi_periodic(torch.roll(rho, 5, dims=2), 1.5)
    assert torch.allclose(torch.roll(objective.gaussian_filter_phi_periodic(rho, 1.5), 5, dims=2), shifted)
    assert torch.autograd.gradcheck(lambda r: objective.tanh_projection(
        objective.gaussian_filter_phi_periodic(r, 1.0), 4.0).sum(), (rho,))


def test_continuous_zone_weights_equal_wedge_weights_on_a_pure_mode():
    """A field carrying e^{i phi} exactly (m = 1) gives the same focal phasor
    whether it is held by a continuous zone (one sample at phi = 0) or by
    any n-fold wedge sampling it at its staggered points: the integrand of
    the ring integral is rotation-invariant."""
    rng = np.random.default_rng(5)
    kw = dict(r_in=0.5, nr=16, nz=10, m=1, pml=(0, 3, 2, 2), axis=1)
    cont = Workload("cont", nphi=1, n_fold=0, **kw)
    om = (0.3, 0.41)
    F = 90.0
    Wc = objective.focal_weights(cont, om, F, device="cpu").numpy().astype(np.complex128)
    E0 = rng.standard_normal((2, 2, kw["nr"])) + 1j * rng.standard_normal((2, 2, kw["nr"]))
    a_c = np.einsum("kaij,kaij->k", Wc, E0[..., None])
    for n, nphi in ((5, 7), (16, 3)):
        wedge = Workload("wedge", nphi=nphi, n_fold=n, **kw)
        Ww = objective.focal_weights(wedge, om, F, device="cpu").numpy().astype(np.complex128)
        dphi = 2 * np.pi / (n * nphi)
        phase = np.stack([np.exp(1j * np.arange(nphi) * dphi), np.exp(1j * (np.arange(nphi) + 0.5) * dphi)])
        plane = E0[..., None] * phase[None, :, None, :]
        a_w = np.einsum("kaij,kaij->k", Ww, plane)
        assert np.allclose(a_w, a_c, rtol=1e-6, atol=0), (n, nphi, a_w, a_c)


def test_ring_focal_field_on_axis_is_the_focal_phasor():
    """On the axis the co-polarised amplitude (E_x - i E_y)/2 of the ring
    projection equals the focal objective's phasor a_k (two independent
    routes: full-ring Cartesian quadrature and the wedge weights)."""
    rng = np.random.default_rng(6)
    wl = Workload("obj", r_in=60.0, nr=20, nphi=12, nz=10, n_fold=9, m=1, pml=(3, 4, 2, 2))
    om = (0.3, 0.41)
    F = 140.0
    W = objective.focal_weights(wl, om, F, device="cpu").numpy().astype(np.complex128)
    plane = rng.standard_normal((2, 2, wl.nr, wl.nphi)) + 1j * rng.standard_normal((2, 2, wl.nr, wl.nphi))
    a = np.einsum("kaij,kaij->k", W, plane)
    E = objective.ring_focal_field(torch.tensor(plane), wl, om, F, [0.0], [0.0])
    co = 0.5 * (E[:, 0, 0] - 1j * E[:, 1, 0])
    assert np.allclose(co, a, rtol=1e-6, atol=0)


def test_thin_ring_lens_focuses_to_the_bessel_spot():
    """A narrow ring carrying the ideal converging wave e^{-i k sqrt(r^2 + F^2)}
    (x + i y polarised, the m = +1 preset's field) focuses to the J0^2 spot of
    an annular aperture: FWHM = 2 x 1.1264 / (k sin theta), sin theta =
    r / sqrt(r^2 + F^2), within 3 %; the focusing efficiency against the
    ring's own transmitted power is below 1 and positive."""
    r0, width, n, nphi = 400.0, 8, 24, 6
    wl = Workload("ring", r_in=r0, nr=width, nphi=nphi, nz=10, n_fold=n, m=1, pml=(0, 0, 2, 2))
    w = 2 * np.pi / 20
    F = 400.0
    dphi = 2 * np.pi / (n * nphi)
    ri = r0 + np.arange(width)
    rh = ri + 0.5
    pj, ph = np.arange(nphi) * dphi, (np.arange(nphi) + 0.5) * dphi
    # x + i y = e^{i phi} (r + i phi): E_r = e^{i phi} u, E_phi = i e^{i phi} u
    u_r = np.exp(-1j * w * np.sqrt(rh ** 2 + F ** 2))[:, None]
    u_p = np.exp(-1j * w * np.sqrt(ri ** 2 + F ** 2))[:, None]
    plane = np.stack([u_r * np.exp(1j * pj)[None], 1j * u_p * np.exp(1j * ph)[None]])[None]
    P_t = objective.exit_plane_power(plane, wl)
    eff = objective.focusing_efficiency(torch.tensor(plane), wl, (w,), F, incident_power=P_t, transmitted_power=P_t,
                                        n_rho=160, n_phi=4, rho_max=120.0)
    rm = r0 + width / 2
    sin_t = rm / np.sqrt(rm ** 2 + F ** 2)
    expect = 2 * 1.1264 / (w * sin_t)
    assert abs(eff["fwhm"][0] - expect) < 0.03 * expect, (eff["fwhm"], expect)
    assert 0.0 < eff["relative"][0] < 1.0
