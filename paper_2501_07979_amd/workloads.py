"""Seeded synthetic workloads (zone geometries and permittivity maps).

Input generation only: sizes, seeds and the recipes that stand in for the
paper's optimised lenses (whose permittivity data is not available).  No
step of the FDTD method lives here; both the oracle and the HIP path read the
same arrays.  Geometry rule: r_in = 200 (n / 16) (nphi / 64) cells keeps
r_in dphi = 1.2272 cells for every zone, so Courant 0.5 is stable.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    r_in: float
    nr: int
    nphi: int
    nz: int
    n_fold: int
    m: int = 1
    dr: float = 1.0
    dz: float = 1.0
    courant: float = 0.5
    pml: tuple = (8, 8, 8, 8)
    k_src: int = 20
    k_mon: int = 80
    design: tuple = (30, 40)
    eps_bg: float = 1.0
    eps_hi: float = 6.25
    eps_sub: float = 2.1
    k_sub: int = 30                  # substrate for k < k_sub
    steps: int = 1000
    omegas: tuple = ()
    omega_c: float = 0.0
    width: float = 20.0
    seed: int = 1
    density: str = "bernoulli"       # or "smoothed"
    axis: int = 0                    # 1: the zone contains the axis (r_in = dr / 2)
    extra: dict = field(default_factory=dict)

    @property
    def cells(self):
        return self.nr * self.nphi * self.nz

    def desc_kwargs(self):
        return dict(r_in=self.r_in, nr=self.nr, nphi=self.nphi, nz=self.nz, n_fold=self.n_fold, m=self.m,
                    dr=self.dr, dz=self.dz, courant=self.courant, pml=self.pml, k_mon=self.k_mon,
                    design=self.design, eps_bg=self.eps_bg, eps_hi=self.eps_hi, axis=self.axis)

    def rho(self):
        """Design density over the design layer, [k1-k0][nr][nphi] float32."""
        k0, k1 = self.design
        rng = np.random.default_rng(self.seed)
        shape = (k1 - k0, self.nr, self.nphi)
        if self.density == "bernoulli":
            return (rng.random(shape) < 0.5).astype(np.float32)
        return smoothed_density(rng, shape)

    def eps(self, rho=None):
        """Per-cell permittivity [nz][nr][nphi] float32: substrate below the
        design layer, eq. (6) inside it, background above."""
        k0, k1 = self.design
        if rho is None:
            rho = self.rho()
        e = np.full((self.nz, self.nr, self.nphi), self.eps_bg, np.float64)
        e[:self.k_sub] = self.eps_sub
        e[k0:k1] = self.eps_bg + rho.astype(np.float64) * (self.eps_hi - self.eps_bg)
        return e.astype(np.float32)


def smoothed_density(rng, shape, sigma=3.0, beta=8.0, eta=0.5):
    """U(0,1) -> 3-D Gaussian filter (sigma cells; wrap in phi, reflect in r
    and z) -> tanh projection (beta, eta): a grey, feature-sized density like
    an intermediate topology-optimisation iterate."""
    from scipy.ndimage import gaussian_filter
    u = rng.random(shape)
    f = gaussian_filter(u, sigma=sigma, mode=("reflect", "reflect", "wrap"))
    # the filtered field has a small spread around 0.5; rescale to [0, 1]
    f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
    num = np.tanh(beta * eta) + np.tanh(beta * (f - eta))
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (num / den).astype(np.float32)


def _omegas(lams):
    return tuple(2 * np.pi / l for l in lams)


def _pulse(omegas):
    """Broadband pulse covering the frequencies: centre and 1/sigma_w width."""
    wmin, wmax = min(omegas), max(omegas)
    return (wmax + wmin) / 2, 2.0 / (wmax - wmin)


def c1():
    """Parity zone: n = 16 wedge, 64 x 64 x 96 cells, lambda = 20 cells,
    Bernoulli(0.5) design layer z in [30, 40), 1000 steps, one frequency."""
    w = 2 * np.pi / 20
    return Workload("c1_parity_64x64x96", r_in=200.0, nr=64, nphi=64, nz=96, n_fold=16, pml=(8, 8, 8, 8),
                    k_src=20, k_mon=80, design=(30, 40), steps=1000, omegas=(w,), omega_c=w, width=20.0, seed=1)


def c2():
    """Production zone: n = 512 wedge, 512 x 1024 x 400 cells (about 210 M),
    dr = lambda_green / 25, smoothed design layer z in [44, 64), 12-cell PML,
    pulse spanning 450/550/650 nm, 20000 steps, 3-frequency exit-plane DFT."""
    om = _omegas((450 / 22.0, 25.0, 650 / 22.0))
    wc, w = _pulse(om)
    return Workload("c2_production_512x1024x400", r_in=102400.0, nr=512, nphi=1024, nz=400, n_fold=512,
                    pml=(12, 12, 12, 12), k_src=24, k_mon=380, design=(44, 64), k_sub=44, steps=20000,
                    omegas=om, omega_c=wc, width=w, seed=2, density="smoothed")


def c3(steps=8000):
    """Gradient zone: n = 16 wedge, 256 x 512 x 300 cells, smoothed design
    layer z in [30, 50) (256 x 512 x 20 pixels), 3 frequencies.  The run
    length lets the fields decay: the adjoint gradient is that of the fully
    decayed DFT, and central differences of the truncated run agree with it
    to 2e-3 of max |dF/drho| after 4000 steps, 9e-4 after 6000 and 9e-5 after
    8000 (the largest field left falls about eightfold per 2000 steps)."""
    om = _omegas((16.36, 20.0, 23.64))
    wc, w = _pulse(om)
    return Workload("c3_gradient_256x512x300", r_in=1600.0, nr=256, nphi=512, nz=300, n_fold=16,
                    pml=(8, 8, 8, 8), k_src=20, k_mon=60, design=(30, 50), steps=steps, omegas=om,
                    omega_c=wc, width=w, seed=3, density="smoothed")


def c3_small(steps=2500):
    """The gradient zone's small copy: the parity geometry with the design
    layer z in [30, 50) and the gradient config's three frequencies (scaled to
    lambda = 20 cells at the centre)."""
    om = _omegas((16.36, 20.0, 23.64))
    wc, w = _pulse(om)
    return Workload("c3_small_64x64x96", r_in=200.0, nr=64, nphi=64, nz=96, n_fold=16, pml=(8, 8, 8, 8),
                    k_src=20, k_mon=70, design=(30, 50), steps=steps, omegas=om, omega_c=wc, width=w, seed=3,
                    density="smoothed")


def c5_zone(steps=2500):
    """Design zone of the surrogate: the gradient zone's small copy widened to
    a 128 x 128 design layer (n = 16 wedge, 128 x 128 x 96 cells, r_in by
    the geometry rule, three frequencies), patterned with a 2-D pattern
    extruded through the layer z in [30, 50)."""
    om = _omegas((16.36, 20.0, 23.64))
    wc, w = _pulse(om)
    return Workload("c5_surrogate_128x128x96", r_in=400.0, nr=128, nphi=128, nz=96, n_fold=16, pml=(8, 8, 8, 8),
                    k_src=20, k_mon=70, design=(30, 50), steps=steps, omegas=om, omega_c=wc, width=w, seed=5,
                    density="smoothed")


def c4_zone(l, steps=4000):
    """Zone l (1..48) of the batched lens: n rises with radius from 64 to
    4096, Nr 64..512 and Nphi 128..1024 (uneven on purpose), Nz = 300,
    smoothed design layer z in [30, 50), seed 4000 + l."""
    t = (l - 1) / 47.0
    n = int(round(64 + 4032 * t))
    nr = 64 + int(round(448 * t))
    nphi = 128 + int(round(896 * t))
    om = _omegas((16.36, 20.0, 23.64))
    wc, w = _pulse(om)
    r_in = 200.0 * (n / 16.0) * (nphi / 64.0)
    return Workload("c4_zone%02d_%dx%dx300" % (l, nr, nphi), r_in=r_in, nr=nr, nphi=nphi, nz=300, n_fold=n,
                    pml=(8, 8, 8, 8), k_src=20, k_mon=60, design=(30, 50), steps=steps, omegas=om, omega_c=wc,
                    width=w, seed=4000 + l, density="smoothed")


def c4(nzones=48, steps=4000):
    """The batched lens: 48 uneven zones (2.89e9 cells in total)."""
    return [c4_zone(l, steps) for l in range(1, nzones + 1)]


def lwir_lens(nz=180, steps=10000):
    """A lens shaped like the paper's 0.8 cm LWIR design (section "Centimeter-
    scale metalens at long-wave infrared"), at dr = dz = lambda / 50: 16 zones
    of 25 lambda (1250 cells) radially; zone 1 continuous and containing the
    axis, zone l >= 2 an n = 720 l wedge with r dphi <= 0.021 lambda at its
    outer edge (11 phi cells); silicon (n = 3.42) substrate and a 0.6 lambda
    design layer, air above; 12-cell PML on every face (outer only next to
    the axis).  The height (180 cells) and the step count are this
    workload's choices: the paper gives neither."""
    lam = 50.0
    om = (2 * np.pi / lam,)
    eps_si = 3.42 ** 2
    common = dict(nz=nz, m=1, courant=0.35, k_src=30, k_mon=nz - 20, design=(60, 90), k_sub=60, steps=steps,
                  omegas=om, omega_c=om[0], width=4 * lam, eps_hi=eps_si, eps_sub=eps_si, density="smoothed")
    zones = [Workload("lwir_zone01_continuous_1250x1x%d" % nz, r_in=0.5, nr=1250, nphi=1, n_fold=0,
                      pml=(0, 12, 12, 12), axis=1, seed=7001, **common)]
    for l in range(2, 17):
        n = 720 * l
        r_in = 1250.0 * (l - 1) + 0.5
        nphi = int(np.ceil((r_in + 1250.0) * 2 * np.pi / n / (0.021 * lam)))
        zones.append(Workload("lwir_zone%02d_1250x%dx%d" % (l, nphi, nz), r_in=r_in, nr=1250, nphi=nphi, n_fold=n,
                              pml=(12, 12, 12, 12), seed=7000 + l, **common))
    return zones


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c3_small": c3_small, "c5": c5_zone}
