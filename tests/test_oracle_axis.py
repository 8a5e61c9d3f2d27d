"""Oracle pins of the zones that contain the axis (r_in = dr/2, the axis at
r_{-1/2} = 0) and of the continuous zone (n_fold = 0, nphi = 1: fields carry
exp(i m phi) exactly), which together let the first zone of a lens be
simulated:

* lossless energy identity with the axis row updated (PEC box, no layer);
* TM resonance of a full PEC cylinder at the Bessel zero j_{1,1} / R,
  converging under grid refinement;
* the continuous zone is the n -> infinity limit of one-cell wedges (fields
  at phi_{j+1/2} carry the phase exp(i m tau / 2) of their sample point),
  with an error that falls as 1/n^2;
* adjoint gradient against FP64 central differences on an axis zone with a
  layer, a source and the continuous seams.
"""
import numpy as np
import pytest
from scipy.special import jn_zeros

from test_oracle_physics import E_COMPS, H_COMPS, _objective, _pencil_freqs, _volumes


def _random_axis_fields(z, rng):
    """Random fields obeying the PEC box; the first row is free (it is not a
    wall in an axis zone)."""
    f = {c: rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape) for c in E_COMPS + H_COMPS}
    f["Er"][0] = 0
    f["Ephi"][0] = 0
    f["Hz"][0] = 0
    for c in f:
        z.set_field(c, f[c])


@pytest.mark.parametrize("kind", ["continuous", "wedge"])
def test_axis_zone_energy_identity(oracle_mod, kind):
    rng = np.random.default_rng(40)
    if kind == "continuous":
        z = oracle_mod.OracleZone(r_in=0.5, nr=10, nphi=1, nz=9, n_fold=0, m=1, dr=1.0, dz=0.8, axis=1)
    else:
        z = oracle_mod.OracleZone(r_in=0.5, nr=10, nphi=4, nz=9, n_fold=3, m=1, dr=1.0, dz=0.8, courant=0.2,
                                  axis=1)
    eps = (1 + 5 * rng.random(z.shape)).astype(np.float32)
    z.set_eps(eps)
    _random_axis_fields(z, rng)
    V = _volumes(z)
    energies = []
    for _ in range(20):
        E = {c: z.get_field(c) for c in E_COMPS}
        Hm = {c: z.get_field(c) for c in H_COMPS}
        z.run(1, reset=False)
        Hp = {c: z.get_field(c) for c in H_COMPS}
        en = 0.5 * sum(np.sum(eps * V[c][None, :, None] * np.abs(E[c]) ** 2) for c in E_COMPS)
        en += 0.5 * sum(np.sum(V[c][None, :, None] * np.real(Hm[c] * np.conj(Hp[c]))) for c in H_COMPS)
        energies.append(en)
        z.run(100, reset=False)
    energies = np.array(energies)
    assert np.abs(energies - energies[0]).max() < 1e-12 * energies[0]
    # and the fields did move (the axis row is live)
    assert np.abs(z.get_field("Ez")[:, 0]).max() > 1e-3


def test_full_cylinder_tm_resonance(oracle_mod):
    """Lowest TM_1 resonance (z-invariant, E_z) of a PEC cylinder of radius R
    containing the axis: k = j_{1,1} / R, with R = r_in + nr dr = (nr + 1/2) dr.
    Refinement by 1, 3, 5 keeps R = 7.5 on the grid."""
    R = 7.5
    k_exact = jn_zeros(1, 1)[0] / R
    errs, hs = [], []
    for res in (1, 3, 5):
        dr = 1.0 / res
        nr = int(round(R / dr - 0.5))
        z = oracle_mod.OracleZone(r_in=0.5 * dr, nr=nr, nphi=1, nz=1, n_fold=0, m=1, dr=dr, dz=dr, axis=1)
        ri = 0.5 * dr + np.arange(nr) * dr
        from scipy.special import jv
        z.set_field("Ez", jv(1, k_exact * ri)[None, :, None].astype(complex))
        T = 3000
        x = np.empty(T, complex)
        probe = (0, nr // 2, 0)
        for t in range(T):
            z.run(1, reset=False)
            x[t] = z.get_field("Ez")[probe]
        wd = _pencil_freqs(x, z.dt, 4)
        lam = 2 / z.dt * np.sin(wd * z.dt / 2)      # remove the leap-frog time error
        errs.append(np.min(np.abs(lam - k_exact)) / k_exact)
        hs.append(dr)
    errs = np.array(errs)
    order = np.log(errs[:-1] / errs[1:]) / np.log(np.array(hs[:-1]) / np.array(hs[1:]))
    assert errs[0] < 2e-2, errs
    assert np.all(order > 1.7), (errs, order)


def test_continuous_zone_is_the_wedge_limit(oracle_mod):
    """A one-cell wedge with n -> infinity approaches the continuous zone; the
    wedge stores E_phi, H_r, H_z at phi_{1/2} = tau/2, so their values carry
    exp(i m tau / 2).  The difference falls as tau^2."""
    rng = np.random.default_rng(41)
    kw = dict(r_in=0.5, nr=8, nphi=1, nz=8, m=1, dr=1.0, dz=1.0, courant=0.4, axis=1)
    init = {c: rng.standard_normal((8, 8, 1)) + 1j * rng.standard_normal((8, 8, 1)) for c in E_COMPS + H_COMPS}
    for c in ("Er", "Ephi", "Hz"):
        init[c][0] = 0
    half = {"Er": 0, "Ephi": 1, "Ez": 0, "Hr": 1, "Hphi": 0, "Hz": 1}

    def run(n_fold):
        z = oracle_mod.OracleZone(n_fold=n_fold, **kw)
        tau = z.tau
        for c, f in init.items():
            z.set_field(c, f * (np.exp(0.5j * kw["m"] * tau) if (half[c] and n_fold > 0) else 1.0))
        z.run(60, reset=False)
        out = {}
        for c in init:
            g = z.get_field(c)
            out[c] = g / (np.exp(0.5j * kw["m"] * tau) if (half[c] and n_fold > 0) else 1.0)
        return out

    ref = run(0)
    errs = []
    for n in (400, 800, 1600):
        w = run(n)
        errs.append(max(np.abs(w[c] - ref[c]).max() / np.abs(ref[c]).max() for c in ref))
    errs = np.array(errs)
    assert errs[-1] < 1e-4, errs
    assert np.all(errs[:-1] / errs[1:] > 3.5), errs          # second order in tau


def test_axis_zone_adjoint_gradient_vs_central_fd(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(42)
    z = O.OracleZone(r_in=0.5, nr=12, nphi=1, nz=14, n_fold=0, m=1, pml=(0, 3, 3, 3), k_mon=10, design=(5, 8),
                     axis=1)
    eps = np.ones(z.shape, np.float32)
    eps[:5] = 2.1
    z.set_eps(eps)
    rho = rng.random((3, 12, 1))
    z.set_design(rho, fp64=True)
    T, omegas = 5000, np.array([0.3, 0.36])
    wts = rng.standard_normal((2, 2, 12, 1)) + 1j * rng.standard_normal((2, 2, 12, 1))
    fwd = z.forward(T, omegas, omega_c=0.33, width=8.0, k_src=3, volume=True)
    _, g = _objective(wts, fwd["plane"])
    grad = z.adjoint_grad(g)
    h = 1e-3

    def central(a, b, hh):
        vals = []
        for s in (+1, -1):
            r2 = rho.copy()
            r2[a, b, 0] += s * hh
            z.set_design(r2, fp64=True)
            out = z.run(T, patterns=z.preset_pattern()[None], profiles=O.pulse(T, z.dt, 0.33, 8.0)[0][None],
                        k_src=3, omegas=omegas)
            vals.append(_objective(wts, out["plane"])[0])
        return (vals[0] - vals[1]) / (2 * hh)

    for (a, b) in [(0, 0), (1, 1), (2, 4), (1, 7)]:          # the axis row included
        fd = (4 * central(a, b, h / 2) - central(a, b, h)) / 3
        assert abs(fd - grad[a, b, 0]) < 1e-7 * np.abs(grad).max(), (a, b, fd, grad[a, b, 0])
    z.set_design(rho, fp64=True)
