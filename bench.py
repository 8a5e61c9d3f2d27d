"""Benchmark of the ZDA zone hot path on one MI355X.

A step is one leap-frog time step of the whole forward hot path over the
production zone (n = 512 wedge, 512 x 1024 x 400 cells): the H half-step, the
E half-step with the soft source sheet and the 3-frequency exit-plane DFT.
A warm-up run of W steps (which resets fields, auxiliaries and monitors)
is followed by the timed run of K more steps that continues from it, so the
per-run reset is outside the timed region and timed separately; every
per-step piece (source profile and twiddle staging, the update launches,
the divergence checks) is inside.  The value is cell-updates per second.
The default kernel advances two steps per launch (one launch over the tiles
without layer cells, one over the rest).  The dominant kernel's roofline
takes its algorithmic bytes per launch -- 100 B per cell-update (six complex
fields read and written once per step, dt/eps read) plus 2 x 8 B per DFT
accumulator per step, times the cell-updates of one launch -- over its
average launch duration, both measured live with HIP events on the run's
stream; the least HBM traffic the launch can have (every field crosses HBM
once per two steps) is reported beside it.  The FP64 oracle is timed on the
host cores on a bounded sample of the same zone and on the small parity and
gradient zones.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cyl-FDTD Gcell-updates/s, % HBM roofline; design iters/s plain vs surrogate"
HBM_PEAK_GBS = 8000.0


def kernel_hash():
    src = os.path.join(ROOT, "paper_2501_07979_amd", "csrc", "zda_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def algorithmic_bytes(wl, K):
    """Bytes each update kernel must move per launch (one time step).

    H kernel: read E (3 x 8 B), read+write H (6 x 8 B) = 72 B/cell; r-layer
    cells +88 B (four stretch auxiliaries read+written, the H_phi integral
    read+written, the E_phi integral read); z-layer cells +32 B.
    E kernel: read H, read+write E, read dt/eps = 76 B/cell; r-layer +88 B,
    z-layer +32 B; exit-plane cells +K x 2 x 16 B (DFT read+write); source
    plane cells +2 x 8 B (pattern).
    Fused minimum (every field read and written once, dt/eps once): 100 B/cell
    + both kernels' layer and DFT terms."""
    cells = wl.cells
    plane = wl.nr * wl.nphi
    r_cells = (wl.pml[0] + wl.pml[1]) * wl.nphi * wl.nz
    z_cells = (wl.pml[2] + wl.pml[3]) * plane
    h = 72 * cells + 88 * r_cells + 32 * z_cells
    e = 76 * cells + 88 * r_cells + 32 * z_cells + K * 2 * 16 * plane + 16 * plane
    fused = 100 * cells + 176 * r_cells + 64 * z_cells + K * 2 * 16 * plane + 16 * plane
    return h, e, fused


def two_step_interior_bytes(tm, K):
    """Bytes a multi-step kernel's launch over interior tiles must move: it
    reads E, H (48 B) and dt/eps (4 B) of every owned cell once and writes E,
    H (48 B) once for the launch's two (three) time steps (no layer cells in
    these tiles); exit plane cells add K x 2 x 16 B (DFT read+write, the
    steps folded into one update), source cells 2 x 8 B (pattern)."""
    return 100 * tm.e_cells + K * 32 * tm.e_mon_cells + 16 * tm.e_src_cells


def interior_b_alg_per_launch(tm, K):
    """Algorithmic bytes of one launch over interior tiles counted per
    cell-update: 100 B per cell-update (read and write the six complex fields,
    read dt/eps), 2 x 8 B per DFT accumulator per step (2 K on an exit-plane
    cell), 2 x 8 B per source cell per step, times the steps of one launch."""
    return tm.steps_per_launch * (100 * tm.e_cells + K * 32 * tm.e_mon_cells + 16 * tm.e_src_cells)


def zone_b_alg_per_step(wl, K):
    """Whole-zone algorithmic bytes per time step counted per cell-update:
    100 B per cell, 2 x 8 B per stretched-coordinate auxiliary (8 terms in an
    r-layer cell, 4 in a z-layer cell), the exit-plane DFT and the source."""
    plane = wl.nr * wl.nphi
    r_cells = (wl.pml[0] + wl.pml[1]) * wl.nphi * wl.nz
    z_cells = (wl.pml[2] + wl.pml[3]) * plane
    return 100 * wl.cells + 128 * r_cells + 64 * z_cells + K * 32 * plane + 16 * plane


def two_step_zone_bytes(wl, K):
    """Whole-zone minimum per two-step launch pair (interior and layer tiles):
    100 B per cell, r-layer cells 10 auxiliaries x 16 B, z-layer cells 4 x 16
    B, plus the DFT and source terms."""
    plane = wl.nr * wl.nphi
    r_cells = (wl.pml[0] + wl.pml[1]) * wl.nphi * wl.nz
    z_cells = (wl.pml[2] + wl.pml[3]) * plane
    return 100 * wl.cells + 160 * r_cells + 64 * z_cells + K * 32 * plane + 16 * plane


def load_traffic(kernel, wl_name, launch=None):
    """HBM traffic per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and (when the summary records it) the same launch shape."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (kernel, wl_name))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha") != kernel_hash():
        return None
    if launch is not None and rec.get("launch") is not None and rec["launch"] != launch:
        return None
    return rec.get("traffic_bytes_per_launch")


def host_info():
    """Host CPU model, logical CPU count and the oracle's thread count."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    from oracle import oracle
    return {"cpu_model": model, "nproc": os.cpu_count(), "oracle_threads": oracle.num_threads()}


def cpu_baseline(wl, eps=None, budget_s=12.0, max_steps=12):
    """The FP64 oracle on a bounded sample of the same zone (whole zone, full
    source and DFT work, a few steps after one untimed step), and in full on
    the parity zone (64 x 64 x 96, 1000 steps) and on the gradient zone's
    small copy (64 x 64 x 96, 2500 steps forward with the design-layer DFT
    plus the adjoint run and overlap)."""
    from oracle import oracle
    if eps is None:
        eps = wl.eps()
    oz = oracle.OracleZone(**wl.desc_kwargs(), eps=eps)
    del eps
    g, n0 = oracle.pulse(max_steps + 1, oz.dt, wl.omega_c, wl.width)
    pat = oz.preset_pattern()[None]
    om = np.array(wl.omegas)
    oz.run(1, patterns=pat, profiles=g[None, :1], k_src=wl.k_src, omegas=om)
    steps, t0 = 0, time.perf_counter()
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        oz.run(1, patterns=pat, profiles=g[None, steps + 1:steps + 2], k_src=wl.k_src, omegas=om, reset=False,
               n_start=steps + 1)
        steps += 1
    dt = time.perf_counter() - t0
    del oz
    out = {"value": round(wl.cells * steps / dt / 1e9, 5), "unit": "Gcell-updates/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "%d time steps of the full %s zone (FP64, whole-zone H+E updates, source, 3-frequency "
                     "exit-plane DFT), after one untimed step, %.1f s" % (steps, wl.name, dt),
           "host": host_info()}
    from paper_2501_07979_amd.workloads import c1, c3_small
    w1 = c1()
    o1 = oracle.OracleZone(**w1.desc_kwargs(), eps=w1.eps())
    t0 = time.perf_counter()
    o1.forward(w1.steps, np.array(w1.omegas), omega_c=w1.omega_c, width=w1.width, k_src=w1.k_src)
    t1 = time.perf_counter() - t0
    out["c1_parity_full"] = {"workload": w1.name, "steps": w1.steps, "s": round(t1, 3),
                             "gcell_updates_per_s": round(w1.cells * w1.steps / t1 / 1e9, 5)}
    w3 = c3_small()
    o3 = oracle.OracleZone(**w3.desc_kwargs(), eps=w3.eps())
    t0 = time.perf_counter()
    fwd = o3.forward(w3.steps, np.array(w3.omegas), omega_c=w3.omega_c, width=w3.width, k_src=w3.k_src,
                     volume=True)
    rng = np.random.default_rng(5)
    wts = rng.standard_normal(fwd["plane"].shape) + 1j * rng.standard_normal(fwd["plane"].shape)
    o3.adjoint_grad(np.conj(np.sum(wts * fwd["plane"])) * wts)
    t3 = time.perf_counter() - t0
    out["c3_small_forward_adjoint"] = {"workload": w3.name, "steps_per_run": w3.steps, "runs": 2, "s": round(t3, 3),
                                       "gcell_updates_per_s": round(2 * w3.cells * w3.steps / t3 / 1e9, 5)}
    return out


def design_iteration(steps=None):
    """One plain FDTD-adjoint design iteration on the gradient zone (256 x 512
    x 300, 3 frequencies): set rho, forward run with the design-volume DFT,
    focal objective, adjoint run and overlap through torch.autograd."""
    import torch
    from paper_2501_07979_amd import objective, zda
    from paper_2501_07979_amd.autograd import zone_fdtd
    from paper_2501_07979_amd.workloads import c3
    wl = c3() if steps is None else c3(steps)
    rho0 = wl.rho()
    zone = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps(rho0))
    focal = objective.focal_length(wl.r_in + 0.5 * wl.nr * wl.dr)
    W = objective.focal_weights(wl, wl.omegas, focal)
    kw = dict(nsteps=wl.steps, omegas=wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    # the first iteration also allocates the zone's design-volume and adjoint
    # buffers; an optimiser's iterations after it are what is timed
    times = []
    for _ in range(2):
        rho = torch.tensor(rho0, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plane = zone_fdtd(rho, zone, **kw)
        F, _ = objective.focal_objective(plane, W)
        F.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = times[-1]
    ok = bool(torch.isfinite(rho.grad).all().item())
    zone.close()
    return {"workload": wl.name, "steps_per_run": wl.steps, "runs_per_iter": 2, "s_per_iter": round(dt, 3),
            "s_first_iter": round(times[0], 3),
            "iters_per_s": round(1.0 / dt, 4), "gcell_updates_per_s": round(2 * wl.cells * wl.steps / dt / 1e9, 3),
            "finite_gradient": ok, "kind": "plain FDTD-adjoint (no surrogate)"}


def surrogate_comparison():
    """Plain FDTD-adjoint design against surrogate-assisted design (the
    network, about 1.85M parameters, trained once on FDTD samples of seeded
    random patterns; FDTD re-check and gradient every 10 iterations) on the
    128 x 128 x 96 surrogate zone, from the same start, both to the plain
    path's final focusing efficiency within 1 %."""
    from paper_2501_07979_amd import surrogate
    from paper_2501_07979_amd.workloads import c5_zone
    return surrogate.equal_efficiency_comparison(c5_zone())


def batch_lens(steps, warmup, autotune=True):
    """The 48-zone lens (2.89e9 cells, n from 64 to 4096): every zone stepped
    by one batched launch per time step, time loop replayed from a graph."""
    import torch
    from paper_2501_07979_amd import zda
    from paper_2501_07979_amd.workloads import c4
    wls = c4()
    zones = []
    for w in wls:
        eps = torch.from_numpy(w.eps()).cuda()
        zones.append(zda.Zone(zda.default_desc(single_buffer=1, **w.desc_kwargs()), eps))
        del eps
    b = zda.Batch(zones)
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    om = wls[0].omegas
    tune = None
    if autotune:
        print("bench: autotuning the batched launch", file=sys.stderr, flush=True)
        res = b.autotune(srcs, 6, om)
        tune = {"tile_rows": res.tile_rows, "ms_per_step": round(res.ms_per_step, 3), "probes": res.probes}
    b.run(srcs, warmup, om)
    torch.cuda.synchronize()
    st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record()
    b.run(srcs, steps, om)
    en.record()
    torch.cuda.synchronize()
    ms = st.elapsed_time(en)
    cells = sum(w.cells for w in wls)
    b.close()
    for z in zones:
        z.close()
    return cells, ms, tune


def lens_iteration(T):
    """One optimizer step of the 48-zone lens (2.89e9 cells) at T steps per
    run: batched forward runs with the design-layer DFT, the lens focal
    objective (all 48 zones' phasors summed), batched adjoint runs and the
    overlaps, through torch.autograd; the zones hold their field memory (both
    buffer sets, so the batched two-step kernel applies) only while they
    step, in waves.  The second of two iterations is timed."""
    import torch
    from paper_2501_07979_amd import lens
    from paper_2501_07979_amd.workloads import c4, c4_zone
    torch.cuda.empty_cache()
    full_steps = c4_zone(1).steps
    wl_it = c4(steps=T)
    cells = sum(w.cells for w in wl_it)
    print("bench: lens forward + adjoint iteration (%d steps per run)" % T, file=sys.stderr, flush=True)
    ln = lens.Lens(wl_it, waves=True)
    n_waves = len(ln.groups)
    rhos = [torch.tensor(w.rho(), device="cuda", requires_grad=True) for w in wl_it]
    secs = []
    for it in range(2):
        for r in rhos:
            r.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, _ = ln.objective(rhos)
        F.backward()
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        print("bench: lens iteration %d: %.2f s" % (it, secs[-1]), file=sys.stderr, flush=True)
    finite = all(bool(torch.isfinite(r.grad).all()) for r in rhos)
    ln.close()
    del ln, rhos
    torch.cuda.empty_cache()
    rate = 2 * cells * T / secs[1] / 1e9
    return {"workload": "c4_batched_lens_48_zones", "cells": cells, "steps_per_run": T, "runs_per_iter": 2,
            "s_per_iter": round(secs[1], 3), "s_first_iter": round(secs[0], 3), "gcell_updates_per_s": round(rate, 3),
            "finite_gradient": finite,
            "kernels": "batched two-step kernels in waves of zones (%d), each zone's field memory held only while "
                       "it steps" % n_waves,
            "s_per_iter_at_%d_steps" % full_steps: round(2 * cells * full_steps / (rate * 1e9), 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "lwir"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-design-iter", action="store_true",
                    help="skip the gradient-zone design iteration reported beside the headline")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-assisted vs plain design comparison on the surrogate zone")
    ap.add_argument("--lens-iter-steps", type=int, default=None,
                    help="steps per run of the timed lens design iterations (the 48-zone lens with the default "
                         "workload and c4, the LWIR-shaped lens with lwir; 0: none; default 200, 2000 for lwir)")
    ap.add_argument("--launch", default=None, metavar="KCHUNK,TILE_ROWS",
                    help="launch shape of the timed zone (zda_zone_set_launch), e.g. 64,11 for the three-step "
                         "kernel; default: the zone's own")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 4 GiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.lens_iter_steps is None:
        args.lens_iter_steps = 2000 if args.workload == "lwir" else 200
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus %d is not supported "
              "(a lens would shard its zones across GPUs, one zone per GPU; not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_07979_amd import zda
    from paper_2501_07979_amd.workloads import WORKLOADS

    torch.cuda.set_device(0)
    if args.workload == "lwir":
        # a lens shaped like the paper's LWIR design: 16 zones, narrow wedges
        from paper_2501_07979_amd import lens
        from paper_2501_07979_amd.workloads import lwir_lens
        wls = lwir_lens()
        cells = sum(w.cells for w in wls)
        if args.copy_calibration:
            a = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        free, _ = torch.cuda.mem_get_info()
        print("bench: LWIR-shaped lens, %d zones, %d cells" % (len(wls), cells), file=sys.stderr, flush=True)
        _, ms, nwaves = lens.run_in_waves(wls, args.steps, int(0.8 * free), warmup=args.warmup, keep_fields=False)
        gc = cells * args.steps / (ms / 1e3) / 1e9
        t_run = wls[0].steps * cells / (gc * 1e9)
        design = None
        if args.lens_iter_steps > 0:
            # whole design iterations of the lens through its autograd path:
            # batched forward runs with the design-layer DFT, the focal
            # objective, batched adjoint runs and the overlap gradients
            wl_it = lwir_lens(steps=args.lens_iter_steps)
            ln = lens.Lens(wl_it)
            rhos = [torch.tensor(w.rho(), device="cuda", requires_grad=True) for w in wl_it]
            secs = []
            for it in range(2):
                print("bench: lens design iteration %d (%d steps per run)" % (it, args.lens_iter_steps),
                      file=sys.stderr, flush=True)
                for r in rhos:
                    r.grad = None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F, _ = ln.objective(rhos)
                F.backward()
                torch.cuda.synchronize()
                secs.append(time.perf_counter() - t0)
            finite = all(bool(torch.isfinite(r.grad).all()) for r in rhos)
            ln.close()
            del ln, rhos
            torch.cuda.empty_cache()
            rate = 2 * cells * args.lens_iter_steps / secs[1] / 1e9
            design = {"steps_per_run": args.lens_iter_steps, "runs_per_iter": 2, "s_per_iter": round(secs[1], 3),
                      "s_first_iter": round(secs[0], 3), "gcell_updates_per_s": round(rate, 3),
                      "finite_gradient": finite,
                      "s_per_iter_at_%d_steps" % wls[0].steps: round(2 * wls[0].steps * cells / (rate * 1e9), 2)}
        print(json.dumps({"metric": METRIC, "value": round(gc, 4), "unit": "Gcell-updates/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic",
                          "config": {"workload": "lwir_shaped_lens_16_zones", "cells": cells, "frequencies": 1,
                                     "zones": [w.name for w in wls], "waves": nwaves,
                                     "s_per_design_iteration_at_%d_steps" % wls[0].steps: round(2 * t_run, 2)},
                          "design_iteration": design}),
              flush=True)
        return
    if args.workload == "c4":
        cells, ms, tune = batch_lens(args.steps, args.warmup)
        gc = cells * args.steps / (ms / 1e3) / 1e9
        # the same lens in waves of zones that fit with both buffer sets (two-step kernel)
        from paper_2501_07979_amd import lens
        from paper_2501_07979_amd.workloads import c4
        free, _ = torch.cuda.mem_get_info()
        print("bench: the lens in waves (two-step kernel)", file=sys.stderr, flush=True)
        _, ms_w, nwaves = lens.run_in_waves(c4(), args.steps, int(0.8 * free), warmup=args.warmup,
                                            keep_fields=False)
        gw = cells * args.steps / (ms_w / 1e3) / 1e9
        best_waves = gw > gc
        fa = lens_iteration(args.lens_iter_steps) if args.lens_iter_steps > 0 else None
        print(json.dumps({"metric": METRIC, "value": round(max(gc, gw), 4), "unit": "Gcell-updates/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": round((ms_w if best_waves else ms) / args.steps, 4),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic",
                          "config": {"workload": "c4_batched_lens_48_zones", "cells": cells, "frequencies": 3,
                                     "schedule": "waves, two-step" if best_waves else "one batch, single buffer",
                                     "one_batch_single_buffer": {"gcell_updates_per_s": round(gc, 4),
                                                                 "autotune": tune},
                                     "waves_two_step": {"gcell_updates_per_s": round(gw, 4), "waves": nwaves,
                                                        "budget_bytes": int(0.8 * free)}},
                          "forward_adjoint_iteration": fa}), flush=True)
        return
    wl = WORKLOADS[args.workload]()
    K = len(wl.omegas)
    print("bench: building %s (%d cells)" % (wl.name, wl.cells), file=sys.stderr, flush=True)
    eps_host = wl.eps()
    eps = torch.from_numpy(eps_host).cuda()
    zone = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    del eps
    if args.launch:
        kc, tr = (int(v) for v in args.launch.split(","))
        zone.set_launch(kc, tr)
    run_kw = dict(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    stream = torch.cuda.current_stream()
    # the run's reset (fills of both buffer sets, auxiliaries, monitors), timed on its own
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    zone.run(0, wl.omegas, **run_kw)
    r1.record(stream)
    torch.cuda.synchronize()
    reset_ms = r0.elapsed_time(r1)
    print("bench: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    zone.run(args.warmup, wl.omegas, **run_kw)
    torch.cuda.synchronize()
    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    # continues the warmed-up run: no reset inside the timed region
    zone.run(args.steps, wl.omegas, timing=True, cont=True, **run_kw)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    tm = zone.last_timing()
    info = zone.info()
    launch = {"tile_rows": info.tile_rows, "kchunk": info.kchunk}
    # sanity: the run produced finite monitors, and no divergence was flagged
    plane = zone.dft(zda.MON_PLANE)
    assert torch.isfinite(torch.view_as_real(plane)).all().item()
    zone.sync()
    zone.close()

    gcells = wl.cells * args.steps / (ms / 1e3) / 1e9
    hb, eb, fused = algorithmic_bytes(wl, K)
    e_avg = tm.e_ms / tm.e_launches
    kernel_ms = {}
    min_bytes = None
    if tm.steps_per_launch >= 2:   # multi-step kernel: interior tiles + tiles with layer cells
        depth = tm.steps_per_launch
        kernel = "eh%d_kernel_interior" % depth
        kbytes = interior_b_alg_per_launch(tm, K)
        min_bytes = two_step_interior_bytes(tm, K)
        kernel_ms = {kernel: round(e_avg, 5),
                     "eh%d_kernel_layer" % depth: round(tm.layer_ms / tm.layer_launches, 5)}
        zone_min = two_step_zone_bytes(wl, K) / depth
        family = "two-step" if depth == 2 else "three-step"
    elif tm.h_launches == 0:      # fused step: one kernel per time step
        kernel, kbytes = "eh_fused_kernel", fused
        kernel_ms = {"eh_fused_kernel": round(e_avg, 5)}
        zone_min = fused
        family = "fused one-step"
    else:
        kernel, kbytes = "e_step_kernel", eb
        kernel_ms = {"h_step_kernel": round(tm.h_ms / tm.h_launches, 5), "e_step_kernel": round(e_avg, 5)}
        zone_min = hb + eb
        family = "split"
    achieved = kbytes / (e_avg / 1e3) / 1e9
    traffic = load_traffic(kernel, wl.name, launch)
    zone_balg = zone_b_alg_per_step(wl, K) / wl.cells
    roof = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algorithmic_bytes_per_launch": kbytes,
            "algorithmic_bytes": "per cell-update: 100 B + 2 x 8 B per DFT accumulator and source sample",
            "cell_updates_per_launch": tm.e_cells * tm.steps_per_launch,
            "cells_per_launch": tm.e_cells, "steps_per_launch": tm.steps_per_launch,
            "avg_launch_ms": round(e_avg, 5)}
    if traffic is not None:
        # the counters' bytes (FETCH_SIZE + WRITE_SIZE, calibrated) over the
        # same launch time: what the memory system moved
        roof["traffic_achieved"] = round(traffic / (e_avg / 1e3) / 1e9, 1)
        roof["traffic_frac"] = round(traffic / (e_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if min_bytes is not None:
        # the least HBM traffic of the launch: each field read and written
        # once per two steps; its rate against peak is what HBM delivers
        roof["min_traffic_bytes_per_launch"] = min_bytes
        roof["min_traffic_achieved"] = round(min_bytes / (e_avg / 1e3) / 1e9, 1)
        roof["min_traffic_frac"] = round(min_bytes / (e_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    out = {
        "metric": METRIC,
        "value": round(gcells, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "cells": wl.cells,
            "zone": {"n_fold": wl.n_fold, "m": wl.m, "nr": wl.nr, "nphi": wl.nphi, "nz": wl.nz,
                     "r_in": wl.r_in, "pml": list(wl.pml)},
            "frequencies": K,
            "run_steps_of_full_job": wl.steps,
            "kernel_family": family,
            "launch": launch,
            "steps_per_launch": tm.steps_per_launch,
            "kernel_ms_per_launch": kernel_ms,
            "timed_region": "continues the warm-up run (no reset inside); per-run reset timed apart",
            "reset_ms_per_run": round(reset_ms, 3),
            "wall_s": round(wall, 3),
            "zone_b_alg_bytes_per_cell_update": round(zone_balg, 2),
            "zone_b_alg_roofline_frac": round(gcells * 1e9 * zone_balg / (HBM_PEAK_GBS * 1e9), 4),
            "min_hbm_bytes_per_cell_update": round(zone_min / wl.cells, 2),
            "zone_min_bytes_roofline_frac": round(gcells * 1e9 * (zone_min / wl.cells) / (HBM_PEAK_GBS * 1e9), 4),
        },
        "roofline": roof,
    }
    if not args.no_design_iter and args.workload == "c2":
        print("bench: one design iteration on the gradient zone", file=sys.stderr, flush=True)
        out["design_iteration"] = design_iteration()
    if not args.no_surrogate and args.workload == "c2":
        print("bench: surrogate-assisted vs plain design at equal efficiency", file=sys.stderr, flush=True)
        out["surrogate_design"] = surrogate_comparison()
    if args.lens_iter_steps > 0 and args.workload == "c2":
        out["lens_forward_adjoint_iteration"] = lens_iteration(args.lens_iter_steps)
    if not args.no_cpu_baseline:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, eps_host)
    del eps_host
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
