"""Focal-spot objective of a zone's exit-plane DFT and the design-density
chain (filter + projection), as torch operations on the GPU.

The objective maximises far-field intensity at the designated focal spot of
a lens under normal incidence (section "Results and Discussion"); for
several wavelengths the intensities are summed.  The exit-plane field is
projected onto the on-axis point a focal length F above the plane with the
first Rayleigh-Sommerfeld integral, over the whole ring of n wedge copies.
For the m = +1 (x + iy) excitation the co-polarised on-axis amplitude
a = (E_x - i E_y)/2 is invariant under the wedge rotation (its Bloch phase
e^{i m l tau} cancels the e^{-i l tau} of the Cartesian rotation), so the
ring integral is n times the wedge integral:

  a_k = (n / 4 pi) sum_wedge G_k(R) (Ehat_r - i Ehat_phi) e^{-i phi} r dr dphi,
  G_k(R) = (F / R) (i k - 1/R) e^{i k R} / R,  R = sqrt(r^2 + F^2),

E_r and E_phi taken at their own staggered points, PML cells excluded.
F = sum_k |a_k|^2.  A continuous zone (n_fold = 0, the n -> infinity limit,
one phi sample carrying e^{i m phi} exactly) has a rotation-invariant
integrand, so its ring integral is 2 pi times the phi = 0 sample.  A lens
assembled from concentric zones sums the zones' phasors a_k before |.|^2.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def focal_length(r_mid, na=0.3):
    """Focal length giving numerical aperture na at radius r_mid."""
    return r_mid * math.sqrt(1.0 - na * na) / na


def focal_weights(wl, omegas, focal, device="cuda"):
    """Complex weights w[K][2][nr][nphi] with a_k = sum w * Ehat (E_r, E_phi)."""
    if wl.n_fold > 0:
        n = wl.n_fold
        dphi = 2 * np.pi / (n * wl.nphi)
        phi_j = np.arange(wl.nphi) * dphi
        phi_h = phi_j + 0.5 * dphi
    else:                       # continuous zone: one sample at phi = 0 stands for the whole ring
        n, dphi = 1, 2 * np.pi
        phi_j = phi_h = np.zeros(1)
    ri = wl.r_in + np.arange(wl.nr) * wl.dr
    rh = ri + 0.5 * wl.dr
    active = np.zeros(wl.nr)
    active[wl.pml[0]:wl.nr - wl.pml[1]] = 1.0
    W = np.zeros((len(omegas), 2, wl.nr, wl.nphi), np.complex128)
    for k, w in enumerate(omegas):
        def G(r):
            R = np.sqrt(r * r + focal * focal)
            return (focal / R) * (1j * w - 1.0 / R) * np.exp(1j * w * R) / R
        pref = n / (4 * np.pi) * wl.dr * dphi
        W[k, 0] = pref * (active * G(rh) * rh)[:, None] * np.exp(-1j * phi_j)[None, :]
        W[k, 1] = -1j * pref * (active * G(ri) * ri)[:, None] * np.exp(-1j * phi_h)[None, :]
    return torch.as_tensor(W.astype(np.complex64), device=device)


def focal_objective(plane, weights):
    """F = sum_k |a_k|^2 with a_k = sum(w_k * Ehat_k)."""
    a = (plane * weights).sum(dim=(1, 2, 3))
    return (a.abs() ** 2).sum(), a


def gaussian_filter_phi_periodic(rho, sigma):
    """Separable Gaussian smoothing of [nd][nr][nphi] with a periodic phi
    axis and edge-replicating r and z axes (the density filter of topology
    optimisation; linear, so autograd gives its adjoint)."""
    if sigma <= 0:
        return rho
    rad = int(math.ceil(3 * sigma))
    x = torch.arange(-rad, rad + 1, device=rho.device, dtype=rho.dtype)
    ker = torch.exp(-x * x / (2 * sigma * sigma))
    ker = ker / ker.sum()
    out = rho[None, None]
    for dim in (2, 3, 4):
        pad = [0, 0, 0, 0, 0, 0]
        idx = 2 * (4 - dim)
        pad[idx] = pad[idx + 1] = rad
        mode = "circular" if dim == 4 else "replicate"
        o = torch.nn.functional.pad(out, pad, mode=mode)
        shape = [1, 1, 1, 1, 1]
        shape[dim] = 2 * rad + 1
        out = torch.nn.functional.conv3d(o, ker.view(shape))
    return out[0, 0]


def tanh_projection(x, beta, eta=0.5):
    """Smoothed Heaviside (binarisation) projection."""
    num = math.tanh(beta * eta) + torch.tanh(beta * (x - eta))
    den = math.tanh(beta * eta) + math.tanh(beta * (1 - eta))
    return num / den


# ---- focusing efficiency (section "Centimeter-scale metalens at long-wave
# infrared": the fraction of the incident power within 3 FWHMs of the centre
# of the focal spot; relative to the transmitted power, the relative focusing
# efficiency)

def _sample_points(wl):
    """Exit-plane sample positions of E_r (r_{i+1/2}, phi_j) and E_phi (r_i,
    phi_{j+1/2}) of one wedge, the active (non-PML) row mask and the area
    element r dr dphi of each sample."""
    if wl.n_fold > 0:
        n, dphi = wl.n_fold, 2 * np.pi / (wl.n_fold * wl.nphi)
        phi_j = np.arange(wl.nphi) * dphi
        phi_h = phi_j + 0.5 * dphi
    else:
        n, dphi = 1, 2 * np.pi
        phi_j = phi_h = np.zeros(1)
    ri = wl.r_in + np.arange(wl.nr) * wl.dr
    rh = ri + 0.5 * wl.dr
    active = np.zeros(wl.nr)
    active[wl.pml[0]:wl.nr - wl.pml[1]] = 1.0
    return n, dphi, (rh, phi_j), (ri, phi_h), active


def ring_focal_field(plane, wl, omegas, focal, rho, phi, m=None, chunk=32):
    """Cartesian field (E_x, E_y) at focal-plane points (rho[q] cos phi[q],
    rho[q] sin phi[q], focal) above the exit plane: the first Rayleigh-
    Sommerfeld integral of the tangential exit-plane field over the whole
    ring (n wedge copies, copy l carrying the Bloch factor e^{i m l tau}),
    with the kernel of focal_weights.  plane: [K][2][nr][nphi] complex
    (tensor or array); returns complex128 numpy [K][2][Q]."""
    m = wl.m if m is None else m
    dev = torch.device("cuda" if torch.cuda.is_available() else "cpu")
    P = torch.as_tensor(np.asarray(plane.cpu() if isinstance(plane, torch.Tensor) else plane), device=dev)
    P = P.to(torch.complex128)
    n, dphi, (rh, phj), (ri, phh), active = _sample_points(wl)
    tau = 2 * np.pi / n if wl.n_fold > 0 else 2 * np.pi
    dA_r = torch.as_tensor((active * rh * wl.dr * dphi)[:, None] * np.ones(len(phj))[None], device=dev)
    dA_p = torch.as_tensor((active * ri * wl.dr * dphi)[:, None] * np.ones(len(phh))[None], device=dev)
    rho = np.asarray(rho, np.float64)
    phi = np.asarray(phi, np.float64)
    out = np.zeros((len(omegas), 2, len(rho)), np.complex128)
    copies = range(n) if wl.n_fold > 0 else [0]
    for k, w in enumerate(omegas):
        for q0 in range(0, len(rho), chunk):
            px = torch.as_tensor(rho[q0:q0 + chunk] * np.cos(phi[q0:q0 + chunk]), device=dev)[:, None, None]
            py = torch.as_tensor(rho[q0:q0 + chunk] * np.sin(phi[q0:q0 + chunk]), device=dev)[:, None, None]
            ux = torch.zeros(px.shape[0], dtype=torch.complex128, device=dev)
            uy = torch.zeros_like(ux)
            for l in copies:
                bl = complex(np.exp(1j * m * l * tau)) if wl.n_fold > 0 else 1.0
                for comp, (rr, pp, dA) in enumerate(((rh, phj, dA_r), (ri, phh, dA_p))):
                    if wl.n_fold > 0:
                        ph = torch.as_tensor(pp + l * tau, device=dev)[None, None, :]
                        wrap = 1.0
                    else:
                        # continuous zone: integrate e^{i m phi} over the full turn
                        ph = torch.as_tensor(np.linspace(0, 2 * np.pi, 64, endpoint=False), device=dev)[None, None, :]
                        wrap = None
                    r = torch.as_tensor(rr, device=dev)[None, :, None]
                    R = torch.sqrt(r * r + px * px + py * py - 2 * r * (px * torch.cos(ph) + py * torch.sin(ph))
                                   + focal * focal)
                    G = (focal / R) * (1j * w - 1.0 / R) * torch.exp(1j * w * R) / R
                    if wrap is None:
                        e = P[k, comp, :, 0][None, :, None] * torch.exp(1j * m * ph) * bl
                        G = G * (r * wl.dr * (2 * np.pi / 64)) * torch.as_tensor(active, device=dev)[None, :, None]
                    else:
                        e = P[k, comp][None] * bl
                        G = G * dA[None]
                    c, s = torch.cos(ph), torch.sin(ph)
                    if comp == 0:     # E_r -> (cos, sin)
                        ux += (G * e * c).sum(dim=(1, 2))
                        uy += (G * e * s).sum(dim=(1, 2))
                    else:             # E_phi -> (-sin, cos)
                        ux += (G * e * (-s)).sum(dim=(1, 2))
                        uy += (G * e * c).sum(dim=(1, 2))
            out[k, 0, q0:q0 + chunk] = (ux / (2 * np.pi)).cpu().numpy()
            out[k, 1, q0:q0 + chunk] = (uy / (2 * np.pi)).cpu().numpy()
    return out


def exit_plane_power(plane, wl, index=1.0):
    """Power through the exit plane (active rows, whole ring) of a normally
    propagating field in a medium of refractive index `index`:
    (index / 2) sum |E_t|^2 dA per frequency (numpy [K])."""
    P = np.asarray(plane.cpu() if isinstance(plane, torch.Tensor) else plane)
    n, dphi, (rh, _), (ri, _), active = _sample_points(wl)
    wr = (active * rh * wl.dr * dphi)[None, :, None]
    wp = (active * ri * wl.dr * dphi)[None, :, None]
    ring = n if wl.n_fold > 0 else 2 * np.pi / dphi
    p = (np.abs(P[:, 0]) ** 2 * wr).sum(axis=(1, 2)) + (np.abs(P[:, 1]) ** 2 * wp).sum(axis=(1, 2))
    return 0.5 * index * ring * p


def focusing_efficiency(plane, wl, omegas, focal, incident_power, transmitted_power=None, n_rho=96, n_phi=8,
                        rho_max=None):
    """Absolute (and, given the transmitted power, relative) focusing
    efficiency per frequency: the power of the focal-plane intensity
    (1/2)(|E_x|^2 + |E_y|^2) inside a radius of 3 FWHM around the on-axis
    focal spot, over the incident (transmitted) power.  The FWHM is that of
    the azimuthally averaged radial intensity profile.  Returns a dict of
    numpy arrays per frequency: fwhm, spot_power, absolute, relative."""
    K = len(omegas)
    lam = 2 * np.pi / min(omegas)
    if rho_max is None:
        rho_max = 12.0 * lam        # covers 3 FWHM of any spot with NA >= 0.2
    rho = np.linspace(0.0, rho_max, n_rho)
    phis = np.arange(n_phi) * (2 * np.pi / n_phi)
    rr, pp = np.meshgrid(rho, phis, indexing="ij")
    E = ring_focal_field(plane, wl, omegas, focal, rr.ravel(), pp.ravel())
    I = 0.5 * (np.abs(E[:, 0]) ** 2 + np.abs(E[:, 1]) ** 2).reshape(K, n_rho, n_phi).mean(axis=2)
    fwhm = np.zeros(K)
    spot = np.zeros(K)
    for k in range(K):
        prof = I[k]
        half = 0.5 * prof[0]
        below = np.nonzero(prof < half)[0]
        q = int(below[0]) if len(below) else n_rho - 1
        # linear interpolation of the half-maximum radius
        r_half = rho[q - 1] + (half - prof[q - 1]) * (rho[q] - rho[q - 1]) / (prof[q] - prof[q - 1]) if q > 0 else 0.0
        fwhm[k] = 2.0 * r_half
        R3 = min(3.0 * fwhm[k], rho_max)
        fine = np.linspace(0.0, R3, 257)
        spot[k] = np.trapezoid(np.interp(fine, rho, prof) * 2 * np.pi * fine, fine)
    out = {"fwhm": fwhm, "spot_power": spot, "absolute": spot / np.asarray(incident_power)}
    if transmitted_power is not None:
        out["relative"] = spot / np.asarray(transmitted_power)
    return out
