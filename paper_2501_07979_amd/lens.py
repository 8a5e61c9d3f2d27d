"""A metalens assembled from concentric zones (section "Zoned discrete
axisymmetry (ZDA)"): the first zone contains the axis and is continuously
axisymmetric, the following ones are n-fold wedges with n growing with the
radius (section "Results and Discussion").  Every zone is its own
PML-terminated simulation; the zones are stepped together in batches (or, for
a lens larger than HBM with both buffer sets, in waves of batches), and
the objective is the focal-spot intensity of the whole lens: each zone's
exit-plane field projected onto the common on-axis focal point, the zones'
phasors summed coherently, F = sum_k |sum_zones a_k|^2.  Its gradient with
respect to every zone's design density comes from batched adjoint runs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import objective, zda
from .autograd import batch_fdtd, wave_fdtd


class Lens:
    """Zones (Workload descriptions sharing the time step, source plane,
    pulse, frequencies and step count) of one lens; focal length from the
    numerical aperture at the lens's outer radius.

    waves=True: zones keep both buffer sets (so the batched two-step kernel
    applies) but hold their time-stepping memory only while they step; the
    forward and the adjoint run go through the zones in waves whose
    time-stepping memory fits budget_bytes (default: 80 % of the HBM free
    once every zone is created, less what a design iteration adds for every
    zone: the forward and adjoint design-volume DFTs, the adjoint source and
    the iteration's tensors), one batch per wave.  One buffer of the largest
    wave's size is allocated once; each wave's zones step in slices of it."""

    def __init__(self, workloads, na=0.3, single_buffer=False, waves=False, budget_bytes=None):
        self.workloads = list(workloads)
        w0 = self.workloads[0]
        for w in self.workloads[1:]:
            for f in ("dr", "dz", "courant", "k_src", "k_mon", "steps", "omegas", "omega_c", "width", "m"):
                if getattr(w, f) != getattr(w0, f):
                    raise ValueError("zones of one lens share %s (%r != %r)" % (f, getattr(w, f), getattr(w0, f)))
        self.radius = max(w.r_in + w.nr * w.dr for w in self.workloads)
        self.focal = objective.focal_length(self.radius, na)
        if waves and single_buffer:
            raise ValueError("waves keep both buffer sets")
        sb = 1 if single_buffer else 0
        self.waves = waves
        self.arena = None
        self.zones = []
        for w in self.workloads:
            z = zda.Zone(zda.default_desc(single_buffer=sb, **w.desc_kwargs()), w.eps())
            if waves:
                z.release_fields()
            self.zones.append(z)
        # one batch per kernel family: narrow wedges and the continuous zone on
        # the flat-mapped two-step kernel, the others on the two-step kernel;
        # single-buffer zones (half the field memory, so that a lens larger
        # than half the HBM fits at once) all on the in-place kernels
        self.groups = []
        if waves:
            if budget_bytes is None:
                torch.cuda.empty_cache()
                budget_bytes = int(0.8 * torch.cuda.mem_get_info()[0]) - sum(iteration_bytes(w)
                                                                            for w in self.workloads)
            need = [z.fields_bytes() for z in self.zones]
            plan = plan_waves(self.workloads, budget_bytes, sizes=need)
            self.arena = torch.empty(max(sum(need[q] for q in idx) for _, idx in plan), dtype=torch.uint8,
                                     device="cuda")
            for fam, idx in plan:
                b = zda.Batch([self.zones[q] for q in idx])
                set_family(b, fam, [self.workloads[q] for q in idx])
                offs = np.cumsum([0] + [need[q] for q in idx])
                bufs = [self.arena[int(offs[p]):int(offs[p + 1])] for p in range(len(idx))]
                self.groups.append((idx, b, bufs))
        elif single_buffer:
            b = zda.Batch(self.zones)
            set_family(b, IN_PLACE, self.workloads)
            self.groups.append((list(range(len(self.zones))), b, None))
        else:
            for narrow in (True, False):
                idx = [q for q, w in enumerate(self.workloads) if is_narrow(w) == narrow]
                if idx:
                    b = zda.Batch([self.zones[q] for q in idx])
                    set_family(b, FLAT if narrow else TWO_STEP, [self.workloads[q] for q in idx])
                    self.groups.append((idx, b, None))
        self.weights = [objective.focal_weights(w, w.omegas, self.focal) for w in self.workloads]
        self.run_kw = dict(nsteps=w0.steps, omegas=w0.omegas, k_src=w0.k_src, omega_c=w0.omega_c, width=w0.width)

    def phasors(self, rhos):
        """Focal phasors a_k of the whole lens for design densities rhos
        (one [k1-k0][nr][nphi] float32 CUDA tensor per zone)."""
        a = 0
        for idx, b, bufs in self.groups:
            if self.waves:
                planes = wave_fdtd([rhos[q] for q in idx], b, bufs, **self.run_kw)
            else:
                planes = batch_fdtd([rhos[q] for q in idx], b, **self.run_kw)
            a = a + sum((p * self.weights[q]).sum(dim=(1, 2, 3)) for p, q in zip(planes, idx))
        return a

    def objective(self, rhos):
        a = self.phasors(rhos)
        return (a.abs() ** 2).sum(), a

    def close(self):
        for _, b, _ in self.groups:
            b.close()
        for z in self.zones:
            z.close()
        self.groups = []          # drops the slices of the wave buffer with it
        self.arena = None


# batch launch codes: the two-step kernel (13 rows) and, for narrow zones,
# the two-step kernel with the flat (r, phi) mapping (whole rows per block)
# in 16-plane chunks: on a 16-zone lens of narrow wedges (37 M cells) it
# measured 42.3 Gcell-updates/s against 28.0 for the flat fused step and
# 25.9 for the flat in-place kernels (chunks of 12 to 64 planes: 39-42)
# Zones up to 32 phi cells (the kernel's limit) take it: in batches of eight
# 1250 x nphi x 180 wedges it ran 47.2, 44.7, 46.1 Gcell-updates/s at
# nphi = 16, 22, 32 against 9.8, 22.7, 31.2 on the 13-row kernel
TWO_STEP, FLAT, IN_PLACE = 13, 34, 4
FLAT_KCHUNK = 16
NARROW_PHI = 32


def family_kchunk(fam, w):
    """Chunk depth a zone takes in a batch of launch family fam (None keeps
    the zone's own)."""
    return min(FLAT_KCHUNK, w.nz) if fam == FLAT else None


def set_family(batch, fam, wls):
    """Sets a batch of the zones described by wls to launch family fam."""
    kcs = [family_kchunk(fam, w) for w in wls]
    batch.set_launch(fam, None if any(k is None for k in kcs) else kcs)


def is_narrow(w):
    """Zones of at most 32 phi cells (and the continuous zone) run with the
    flat mapping, whose lanes all work however narrow the wedge."""
    return w.nphi <= NARROW_PHI


def zone_device_bytes(w, both_sets=True, max_freq=8):
    """Device memory of a zone (fields, dt/eps, PML auxiliaries with the
    two-step kernel's intermediate set, exit-plane DFT), in bytes."""
    cells, plane = w.nr * w.nphi * w.nz, w.nr * w.nphi
    d_r, d_z = w.pml[0] + w.pml[1], w.pml[2] + w.pml[3]
    sets = 3 if both_sets else 1
    aux = (10 * w.nz * d_r * w.nphi + 4 * d_z * plane) * 8 * sets
    return cells * (48 * (2 if both_sets else 1) + 4) + aux + max_freq * 2 * plane * 8


def iteration_bytes(w):
    """Device memory a design iteration adds to a zone beyond its creation:
    the forward and adjoint design-volume DFTs (K x 3 components x design
    planes), the adjoint source pattern and the exit-plane tensors of the
    iteration (K x 2 components each, a few of them), the design density and
    its gradient, in bytes."""
    K, plane = len(w.omegas), w.nr * w.nphi
    nd = w.design[1] - w.design[0]
    return 2 * K * 3 * nd * plane * 8 + 6 * K * 2 * plane * 8 + 2 * nd * plane * 4


def plan_waves(workloads, budget_bytes, tile_rows=None, sizes=None):
    """Waves of zone indices [(launch code, [indices])]: zones of one kernel
    family (or all, if tile_rows fixes the launch), in their order, cut where
    the next zone would take the wave past budget_bytes with both buffer sets
    (zone_device_bytes, or sizes[q] bytes for zone q); narrow zones after the
    others."""
    order = sorted(range(len(workloads)), key=lambda q: is_narrow(workloads[q]) if tile_rows is None else 0)
    waves, cur, used, fam = [], [], 0, None
    for q in order:
        w = workloads[q]
        f = tile_rows if tile_rows is not None else (FLAT if is_narrow(w) else TWO_STEP)
        b = zone_device_bytes(w) if sizes is None else sizes[q]
        if cur and (used + b > budget_bytes or f != fam):
            waves.append((fam, cur))
            cur, used = [], 0
        cur.append(q)
        used += b
        fam = f
    if cur:
        waves.append((fam, cur))
    return waves


def run_in_waves(workloads, nsteps, budget_bytes, tile_rows=None, warmup=0, keep_fields=True):
    """Runs every zone for nsteps steps with both buffer sets (so the batched
    two-step kernel applies) in waves: consecutive zones of one kernel family
    whose memory fits budget_bytes form one batch, which is created, run and
    released before the next (narrow wedges and the continuous zone run on the
    flat-mapped two-step kernel, the others on the 13-row one, unless
    tile_rows fixes one launch for all).  Zones are independent, so this
    equals one batch of all of them.  Returns the exit-plane DFTs (complex64
    host arrays, in the order of workloads), the summed stepping time in ms
    (events around each wave's timed run, after `warmup` untimed steps) and
    the number of waves."""
    waves = plan_waves(workloads, budget_bytes, tile_rows)
    planes, total_ms = [None] * len(workloads), 0.0
    st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for fam, idx in waves:
        wave = [workloads[q] for q in idx]
        zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), w.eps()) for w in wave]
        batch = zda.Batch(zones)
        set_family(batch, fam, wave)
        srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wave]
        if warmup:
            batch.run(srcs, warmup, wave[0].omegas)
        torch.cuda.synchronize()
        st.record()
        batch.run(srcs, nsteps, wave[0].omegas)
        en.record()
        torch.cuda.synchronize()
        total_ms += st.elapsed_time(en)
        if keep_fields:
            for q, z in zip(idx, zones):
                planes[q] = np.asarray(z.dft(zda.MON_PLANE).cpu())
        batch.close()
        for z in zones:
            z.close()
        del zones, batch
        torch.cuda.empty_cache()
    return (planes if keep_fields else []), total_ms, len(waves)

