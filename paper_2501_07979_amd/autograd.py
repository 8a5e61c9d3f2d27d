"""Differentiable zone: forward FDTD + DFT monitors as a torch.autograd.Function
whose backward is the adjoint FDTD run and the permittivity-gradient overlap
(hybrid time/frequency adjoint, section on the cylindrical solver of arXiv
2501.07979; eq. 6 for the design interpolation).  No time history is kept:
the backward needs only the forward design-volume DFT held by the zone, so a
backward is refused once the zone has run, or had its design, permittivity
or fields changed, since the forward it belongs to.
"""
from __future__ import annotations

import torch

from . import zda


class StaleForwardError(RuntimeError):
    """The zone no longer holds the forward state this backward needs."""


def _check_fresh(zone, serial):
    if zone.state_serial != serial:
        raise StaleForwardError(
            "backward of a zone forward run after the zone ran or changed again (serial %d, now %d): the adjoint "
            "would use the later run's design-volume DFT and permittivity; recompute the forward first"
            % (serial, zone.state_serial))


class ZoneFDTD(torch.autograd.Function):
    """rho [k1-k0][nr][nphi] (float32, CUDA) -> exit-plane DFT [K][2][nr][nphi]
    (complex64, CUDA) of one forward run with the preset plane-wave source."""

    @staticmethod
    def forward(ctx, rho, zone, run_kw):
        zone.set_design(rho.detach().contiguous())
        zone.run(volume=True, **run_kw)
        plane = zone.dft(zda.MON_PLANE)
        ctx.zone = zone
        ctx.serial = zone.state_serial
        return plane

    @staticmethod
    def backward(ctx, grad_plane):
        _check_fresh(ctx.zone, ctx.serial)
        # torch passes 2 conj(dF/dEhat) for a real loss F; the ABI takes dF/dEhat
        g = (grad_plane.conj() * 0.5).to(torch.complex64).contiguous()
        grad_rho = ctx.zone.adjoint_grad(g)
        return grad_rho, None, None


def zone_fdtd(rho, zone, **run_kw):
    return ZoneFDTD.apply(rho, zone, run_kw)


class BatchFDTD(torch.autograd.Function):
    """Several zones stepped together in one batch (one launch per time step
    over every zone's tiles): rho_z -> exit-plane DFT of each zone; the
    backward is one batched adjoint run (-m) and the overlaps."""

    @staticmethod
    def forward(ctx, batch, run_kw, *rhos):
        for z, r in zip(batch.zones, rhos):
            z.set_design(r.detach().contiguous())
        sources = [zda.preset_source(k_src=run_kw["k_src"], omega_c=run_kw["omega_c"], width=run_kw["width"])
                   for _ in batch.zones]
        batch.run(sources, run_kw["nsteps"], run_kw["omegas"], volume=True)
        ctx.batch = batch
        ctx.serials = [z.state_serial for z in batch.zones]
        return tuple(z.dft(zda.MON_PLANE) for z in batch.zones)

    @staticmethod
    def backward(ctx, *grad_planes):
        for z, s in zip(ctx.batch.zones, ctx.serials):
            _check_fresh(z, s)
        gs = [(g.conj() * 0.5).to(torch.complex64).contiguous() for g in grad_planes]
        return (None, None, *ctx.batch.adjoint_grad(gs))


def batch_fdtd(rhos, batch, **run_kw):
    return BatchFDTD.apply(batch, run_kw, *rhos)


class WaveFDTD(torch.autograd.Function):
    """BatchFDTD for one wave of zones that hold their time-stepping memory
    only while they step (zones of a lens larger than HBM with both buffer
    sets): the forward acquires the zones' field memory (from the slices of
    a caller's buffer in `bufs`, else allocated), runs and releases it; the
    backward acquires it again for the batched adjoint run and releases it
    after the overlaps.  The forward design-volume DFT stays in the zones in
    between."""

    @staticmethod
    def _acquire(batch, bufs):
        for z, b in zip(batch.zones, bufs if bufs is not None else [None] * len(batch.zones)):
            z.acquire_fields(b)

    @staticmethod
    def forward(ctx, batch, run_kw, bufs, *rhos):
        ctx.bufs = bufs
        WaveFDTD._acquire(batch, bufs)
        try:
            planes = BatchFDTD.forward(ctx, batch, run_kw, *rhos)
        finally:
            for z in batch.zones:
                z.release_fields()
        return planes

    @staticmethod
    def backward(ctx, *grad_planes):
        for z, s in zip(ctx.batch.zones, ctx.serials):
            _check_fresh(z, s)
        WaveFDTD._acquire(ctx.batch, ctx.bufs)
        try:
            return (None, *BatchFDTD.backward(ctx, *grad_planes))
        finally:
            for z in ctx.batch.zones:
                z.release_fields()


def wave_fdtd(rhos, batch, bufs=None, **run_kw):
    return WaveFDTD.apply(batch, run_kw, bufs, *rhos)
