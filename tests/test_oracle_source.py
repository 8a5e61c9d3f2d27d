"""Pin of the plane-wave source preset against the plane wave it stands for.

A normally incident plane wave splits into the Bloch orders m = +-1 (section
"Results and Discussion"); the preset sheet of order m = +1 is the circular
polarisation x + i y = e^{i phi} (r + i phi) and m = -1 its mirror x - i y.
In a homogeneous zone at large radius whose r-layers absorb the walls'
scattering, the DFT of the field that such a sheet radiates is, away from the
layers, the plane wave of the one-dimensional Yee line:

* polarisation: E_phi(j + 1/2) / E_r(j) = i sgn(m) e^{i m dphi / 2} (the two
  components sit half a cell apart in phi), and E_r(j) e^{-i m phi_j} is the
  same at every radius and phi cell;
* amplitude: a sheet current K = J dz = -g (x + i sgn(m) y) radiates
  Ehat = A (x + i sgn(m) y) with A = wt ghat dz / (2 sin(kt dz)) e^{i kt d},
  where ghat = dt sum_n g(t_{n+1/2}) e^{i w t_{n+1/2}}, wt = (2/dt) sin(w dt/2),
  2 sin(kt dz / 2) = wt dz (the discrete dispersion of the Yee line) and d the
  distance from the sheet to the monitor: the outgoing solution of
  (-D_z^2 - wt^2) Ehat = i wt Jhat on an infinite line.

The zone has coarse phi cells (dphi / 2 = 0.13 rad) and dz != 1, so a J_phi
sampled at phi_j instead of phi_{j+1/2}, a flipped -i, or a lost 1/dz fails
the check; the negative controls below plant exactly those mistakes in the
pattern and show that they are caught.
"""
import numpy as np
import pytest

OMEGA = 2 * np.pi / 20
WIDTH = 20.0
K_SRC, K_MON, NZ = 20, 60, 80
NR, PR = 56, 16
TOL_RATIO, TOL_AMP = 5e-3, 1e-2


def _zone(O, m):
    return O.OracleZone(r_in=2000.0, nr=NR, nphi=6, nz=NZ, n_fold=4, m=m, dr=1.0, dz=0.8,
                        pml=(PR, PR, 8, 8), k_mon=K_MON)


def _line_amplitude(O, z, T):
    g, _ = O.pulse(T, z.dt, OMEGA, WIDTH)
    ghat = z.dt * np.sum(g * np.exp(1j * OMEGA * (np.arange(T) + 0.5) * z.dt))
    wt = O.wtilde(OMEGA, z.dt)
    kt = 2 * np.arcsin(wt * z.dz / 2) / z.dz
    return wt * ghat * z.dz / (2 * np.sin(kt * z.dz)) * np.exp(1j * kt * (K_MON - K_SRC) * z.dz)


def _errors(O, z, m, pattern=None, T=1500):
    """(polarisation error, amplitude error) of the exit-plane DFT over the
    rows at least 4 cells clear of the r-layers."""
    g, _ = O.pulse(T, z.dt, OMEGA, WIDTH)
    pat = z.preset_pattern("plane_circ", m) if pattern is None else pattern
    out = z.run(T, patterns=pat[None], profiles=g[None], k_src=K_SRC, omegas=[OMEGA], m=m)
    P = out["plane"][0][:, PR + 4:NR - PR - 4]
    ratio = P[1] / P[0]
    want = 1j * np.sign(m) * np.exp(1j * m * z.dphi / 2)
    u = P[0] * np.exp(-1j * m * np.arange(z.nphi) * z.dphi)[None]
    A = _line_amplitude(O, z, T)
    return np.abs(ratio / want - 1).max(), np.abs(u / A - 1).max()


@pytest.mark.parametrize("m", [1, -1])
def test_plane_circ_preset_radiates_the_circular_plane_wave(oracle_mod, m):
    z = _zone(oracle_mod, m)
    e_pol, e_amp = _errors(oracle_mod, z, m)
    assert e_pol < TOL_RATIO, e_pol
    assert e_amp < TOL_AMP, e_amp


def test_preset_pattern_matches_the_cylindrical_components_of_x_plus_iy(oracle_mod):
    """The pattern itself: -(x + i sgn(m) y)/dz resolved on r and phi at the
    E_r (phi_j) and E_phi (phi_{j+1/2}) sample points."""
    for m in (1, -1):
        z = _zone(oracle_mod, m)
        pat = z.preset_pattern("plane_circ", m)
        pj = np.arange(z.nphi) * z.dphi
        ph = pj + 0.5 * z.dphi
        ex, ey = -1.0 / z.dz, -1j * np.sign(m) / z.dz          # J = -(x + i sgn(m) y) / dz
        jr = ex * np.cos(pj) + ey * np.sin(pj)                 # r-hat = cos x + sin y
        jphi = -ex * np.sin(ph) + ey * np.cos(ph)              # phi-hat = -sin x + cos y
        assert np.allclose(pat[0], jr[None], atol=1e-14)
        assert np.allclose(pat[1], jphi[None], atol=1e-14)


@pytest.mark.parametrize("mistake", ["jphi_at_phi_j", "flipped_i", "no_dz"])
def test_negative_controls_are_caught(oracle_mod, mistake):
    m = 1
    z = _zone(oracle_mod, m)
    pat = z.preset_pattern("plane_circ", m).copy()
    pj = np.arange(z.nphi) * z.dphi
    if mistake == "jphi_at_phi_j":
        pat[1] = -1j * np.exp(1j * m * pj)[None] / z.dz
    elif mistake == "flipped_i":
        pat[1] = -pat[1]
    else:
        pat = pat * z.dz
    e_pol, e_amp = _errors(oracle_mod, z, m, pattern=pat)
    assert e_pol > 10 * TOL_RATIO or e_amp > 10 * TOL_AMP, (e_pol, e_amp)
