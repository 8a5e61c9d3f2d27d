"""A metalens assembled from concentric zones (section "Zoned discrete
axisymmetry (ZDA)"): the first zone contains the axis and is continuously
axisymmetric, the following ones are n-fold wedges with n growing with the
radius (section "Results and Discussion").  Every zone is its own
PML-terminated simulation; the zones are stepped together in one batch, and
the objective is the focal-spot intensity of the whole lens: each zone's
exit-plane field projected onto the common on-axis focal point, the zones'
phasors summed coherently, F = sum_k |sum_zones a_k|^2.  Its gradient with
respect to every zone's design density comes from one batched adjoint run.
"""
from __future__ import annotations

import torch

from . import objective, zda
from .autograd import batch_fdtd


class Lens:
    """Zones (Workload descriptions sharing the time step, source plane,
    pulse, frequencies and step count) of one lens; focal length from the
    numerical aperture at the lens's outer radius."""

    def __init__(self, workloads, na=0.3):
        self.workloads = list(workloads)
        w0 = self.workloads[0]
        for w in self.workloads[1:]:
            for f in ("dr", "dz", "courant", "k_src", "k_mon", "steps", "omegas", "omega_c", "width", "m"):
                if getattr(w, f) != getattr(w0, f):
                    raise ValueError("zones of one lens share %s (%r != %r)" % (f, getattr(w, f), getattr(w0, f)))
        self.radius = max(w.r_in + w.nr * w.dr for w in self.workloads)
        self.focal = objective.focal_length(self.radius, na)
        self.zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), w.eps()) for w in self.workloads]
        self.batch = zda.Batch(self.zones)
        self.weights = [objective.focal_weights(w, w.omegas, self.focal) for w in self.workloads]
        self.run_kw = dict(nsteps=w0.steps, omegas=w0.omegas, k_src=w0.k_src, omega_c=w0.omega_c, width=w0.width)

    def phasors(self, rhos):
        """Focal phasors a_k of the whole lens for design densities rhos
        (one [k1-k0][nr][nphi] float32 CUDA tensor per zone)."""
        planes = batch_fdtd(rhos, self.batch, **self.run_kw)
        return sum((p * w).sum(dim=(1, 2, 3)) for p, w in zip(planes, self.weights))

    def objective(self, rhos):
        a = self.phasors(rhos)
        return (a.abs() ** 2).sum(), a

    def close(self):
        self.batch.close()
        for z in self.zones:
            z.close()
