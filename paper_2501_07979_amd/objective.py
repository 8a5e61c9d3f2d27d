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
