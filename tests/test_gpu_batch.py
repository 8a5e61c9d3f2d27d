"""Batched uneven zones: one launch per time step over the tiles of every
zone, the time loop replayed from a captured graph.  Each zone's result must
equal the same zone run alone (the per-cell code is shared, so bitwise) and
the oracle; the batched adjoint must equal the per-zone adjoint."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-batch]", *a, flush=True)


def _zones(seed=61):
    """Four zones whose n, nr and nphi grow with the zone index (ragged)."""
    from paper_2501_07979_amd.workloads import Workload
    out = []
    for l, (n, nr, nphi) in enumerate([(16, 23, 64), (24, 30, 96), (40, 37, 130), (56, 44, 170)]):
        r_in = 200.0 * (n / 16.0) * (nphi / 64.0)
        om = (0.28, 0.33, 0.39)
        out.append(Workload("batch%d" % l, r_in=r_in, nr=nr, nphi=nphi, nz=40, n_fold=n, pml=(5, 5, 5, 5),
                            k_src=8, k_mon=30, design=(12, 16), k_sub=12, steps=150, omegas=om, omega_c=0.33,
                            width=6.0, seed=seed + l, density="smoothed"))
    return out


@pytest.fixture(scope="module")
def zda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda as Z
    Z.load()
    return Z


@pytest.mark.parametrize("mode", ["fused", "split", "flat", "two", "two_odd", "two_nocarry"])
def test_batch_equals_single_zone_runs(zda, oracle_mod, mode):
    """two_nocarry: the batched layer tiles pass step one's auxiliaries
    through the intermediate set (the single-zone runs keep them in
    registers: same bits either way)."""
    wls = _zones()
    if mode in ("two_odd", "two_nocarry"):   # an odd step count ends with one fused step
        for w in wls:
            w.steps = 151
    eps = [w.eps() for w in wls]
    singles = []
    for w, e in zip(wls, eps):
        z = zda.Zone(zda.default_desc(**w.desc_kwargs()), e)
        if mode == "split":
            z.set_launch(w.nz, 4)
        if mode == "flat":
            z.set_launch(w.nz, 32)
        z.run(w.steps, w.omegas, k_src=w.k_src, omega_c=w.omega_c, width=w.width, volume=True)
        singles.append((z.read_field("Ez").cpu().numpy(), z.dft(zda.MON_PLANE).cpu().numpy(),
                        z.dft(zda.MON_VOLUME).cpu().numpy()))
        z.close()
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    if mode == "two_nocarry":
        for z in zones:
            z.set_option(zda.OPT_LAYER_CARRY, 0)
    b = zda.Batch(zones)
    b.set_launch({"fused": 7, "split": 4, "flat": 32, "two": 13, "two_odd": 5, "two_nocarry": 13}[mode])
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    _say("batch run", mode)
    b.run(srcs, wls[0].steps, wls[0].omegas, volume=True)    # graph replays + eager tail
    for w, e, z, (ez, pl, vol) in zip(wls, eps, zones, singles):
        got = z.dft(zda.MON_PLANE).cpu().numpy()
        o = oracle_mod.OracleZone(**w.desc_kwargs(), eps=e)
        ref = o.forward(w.steps, np.array(w.omegas), omega_c=w.omega_c, width=w.width, k_src=w.k_src)["plane"]
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
        for a, c in ((z.read_field("Ez").cpu().numpy(), ez), (got, pl), (z.dft(zda.MON_VOLUME).cpu().numpy(), vol)):
            rel = np.linalg.norm(a - c) / np.linalg.norm(c)
            _say(w.name, mode, "batch vs single rel L2 %.2e" % rel)
            assert np.array_equal(a, c), rel
    b.close()


@pytest.mark.parametrize("carry", [0, 1])
def test_batch_adjoint_equals_single_zone_adjoint(zda, carry):
    import torch
    wls = _zones(seed=71)
    for w in wls:
        w.steps = 400
    eps = [w.eps() for w in wls]
    rng = np.random.default_rng(5)
    dFs = [torch.tensor((rng.standard_normal((3, 2, w.nr, w.nphi)) +
                         1j * rng.standard_normal((3, 2, w.nr, w.nphi))).astype(np.complex64), device="cuda")
           for w in wls]
    single = []
    for w, e, g in zip(wls, eps, dFs):
        z = zda.Zone(zda.default_desc(**w.desc_kwargs()), e)
        z.run(w.steps, w.omegas, k_src=w.k_src, omega_c=w.omega_c, width=w.width, volume=True)
        single.append(z.adjoint_grad(g).cpu().numpy())
        z.close()
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    for z in zones:
        z.set_option(zda.OPT_LAYER_CARRY, carry)
    b = zda.Batch(zones)
    b.set_launch(13)
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    _say("batch forward + adjoint, carry", carry)
    b.run(srcs, wls[0].steps, wls[0].omegas, volume=True)
    grads = b.adjoint_grad(dFs)
    for gb, gs in zip(grads, single):
        assert np.array_equal(gb.cpu().numpy(), gs)
    b.close()


def test_batch_autotune_keeps_results(zda):
    wls = _zones(seed=81)
    eps = [w.eps() for w in wls]
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    b = zda.Batch(zones)
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    b.run(srcs, 120, wls[0].omegas)
    before = [z.dft(zda.MON_PLANE).cpu().numpy() for z in zones]
    _say("autotune")
    res = b.autotune(srcs, 10, wls[0].omegas)
    assert res.probes >= 6 and res.ms_per_step > 0
    b.run(srcs, 120, wls[0].omegas)
    after = [z.dft(zda.MON_PLANE).cpu().numpy() for z in zones]
    for x, y in zip(before, after):
        if res.tile_rows in (3, 5, 7, 13, 15):
            assert np.array_equal(x, y)          # fused and two-step families are shape-independent bitwise
        else:
            assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(x)
    b.close()


def test_autotune_on_narrow_zones_keeps_results(zda, oracle_mod):
    """The autotuner on a batch of narrow wedges (where the flat two-step
    kernel is a candidate, probed with its own chunk depth): whatever it
    keeps, the zones' results match the oracle to 1e-5 afterwards."""
    from paper_2501_07979_amd.workloads import Workload
    om = (0.28, 0.33)
    common = dict(nz=48, k_src=8, k_mon=36, design=(12, 16), k_sub=12, steps=100, omegas=om, omega_c=0.31,
                  width=6.0, density="smoothed", nphi=11, n_fold=360, pml=(6, 6, 6, 6))
    wls = [Workload("w%d" % q, r_in=600.5 + 200.0 * q, nr=200, seed=95 + q, **common) for q in range(4)]
    eps = [w.eps() for w in wls]
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    b = zda.Batch(zones)
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    _say("autotune, narrow zones")
    res = b.autotune(srcs, 8, om)
    _say("autotune kept tile_rows", res.tile_rows, "%.4f ms/step" % res.ms_per_step)
    assert res.probes >= 6 and res.ms_per_step > 0
    b.run(srcs, wls[0].steps, om)
    for w, e, z in zip(wls, eps, zones):
        got = z.dft(zda.MON_PLANE).cpu().numpy()
        o = oracle_mod.OracleZone(**w.desc_kwargs(), eps=e)
        ref = o.forward(w.steps, np.array(om), omega_c=w.omega_c, width=w.width, k_src=w.k_src)["plane"]
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    b.close()


@pytest.mark.parametrize("mode", ["fused", "two", "two_odd", "flatfused"])
def test_batch_with_the_axis_zone(zda, oracle_mod, mode):
    """The first zones of a lens in one batch: the continuous zone that
    contains the axis (nphi = 1) next to two wedges; each equals its own run
    bitwise and the oracle to 1e-5."""
    from paper_2501_07979_amd.workloads import Workload
    steps = 151 if mode == "two_odd" else 150
    om = (0.28, 0.33, 0.39)
    common = dict(nz=40, k_src=8, k_mon=30, design=(12, 16), k_sub=12, steps=steps, omegas=om, omega_c=0.33,
                  width=6.0, density="smoothed")
    wls = [Workload("axis", r_in=0.5, nr=40, nphi=1, n_fold=0, pml=(0, 5, 5, 5), axis=1, seed=81, **common),
           Workload("ring2", r_in=40.5, nr=30, nphi=64, n_fold=4, pml=(5, 5, 5, 5), seed=82, **common),
           Workload("ring3", r_in=70.5, nr=30, nphi=64, n_fold=8, pml=(5, 5, 5, 5), seed=83, **common)]
    eps = [w.eps() for w in wls]
    singles = []
    for w, e in zip(wls, eps):
        z = zda.Zone(zda.default_desc(**w.desc_kwargs()), e)
        if mode == "flatfused":
            z.set_launch(z.info().kchunk, 33)
        z.run(w.steps, w.omegas, k_src=w.k_src, omega_c=w.omega_c, width=w.width)
        singles.append(z.dft(zda.MON_PLANE).cpu().numpy())
        z.close()
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    b = zda.Batch(zones)
    b.set_launch({"fused": 7, "two": 13, "two_odd": 5, "flatfused": 33}[mode])
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    _say("batch with the axis zone", mode)
    b.run(srcs, steps, om)
    for w, e, z, pl in zip(wls, eps, zones, singles):
        got = z.dft(zda.MON_PLANE).cpu().numpy()
        o = oracle_mod.OracleZone(**w.desc_kwargs(), eps=e)
        ref = o.forward(w.steps, np.array(om), omega_c=w.omega_c, width=w.width, k_src=w.k_src)["plane"]
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say(w.name, mode, "batch vs oracle rel L2 %.2e" % rel)
        assert rel <= 1e-5
        assert np.array_equal(got, pl)
    b.close()


@pytest.mark.parametrize("steps", [150, 151])
def test_batch_of_narrow_zones_flat_two_step(zda, oracle_mod, steps):
    """Narrow zones (the continuous axis zone, wedges of 11, 16 and 32 phi
    cells) in one batch on the flat-mapped two-step kernel: each equals its
    own run with the same launch bitwise and the oracle to 1e-5 (an odd step
    count ends with one flat fused step)."""
    from paper_2501_07979_amd.workloads import Workload
    om = (0.28, 0.33, 0.39)
    common = dict(nz=40, k_src=8, k_mon=30, design=(12, 16), k_sub=12, steps=steps, omegas=om, omega_c=0.33,
                  width=6.0, density="smoothed")
    wls = [Workload("axis", r_in=0.5, nr=40, nphi=1, n_fold=0, pml=(0, 5, 5, 5), axis=1, seed=87, **common),
           Workload("ring11", r_in=600.5, nr=45, nphi=11, n_fold=360, pml=(5, 6, 4, 7), seed=88, **common),
           Workload("ring16", r_in=645.5, nr=33, nphi=16, n_fold=270, pml=(5, 5, 5, 5), seed=89, **common),
           Workload("ring32", r_in=678.5, nr=30, nphi=32, n_fold=140, pml=(5, 5, 5, 5), seed=90, **common)]
    kcs = [16, 7, 12, 40]
    eps = [w.eps() for w in wls]
    singles = []
    for w, e, kc in zip(wls, eps, kcs):
        z = zda.Zone(zda.default_desc(**w.desc_kwargs()), e)
        z.set_launch(kc, 34)
        z.run(w.steps, w.omegas, k_src=w.k_src, omega_c=w.omega_c, width=w.width)
        singles.append(z.dft(zda.MON_PLANE).cpu().numpy())
        z.close()
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    b = zda.Batch(zones)
    b.set_launch(34, kcs)
    srcs = [zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls]
    _say("narrow zones, flat two-step batch", steps)
    b.run(srcs, steps, om)
    for w, e, z, pl in zip(wls, eps, zones, singles):
        got = z.dft(zda.MON_PLANE).cpu().numpy()
        o = oracle_mod.OracleZone(**w.desc_kwargs(), eps=e)
        ref = o.forward(w.steps, np.array(om), omega_c=w.omega_c, width=w.width, k_src=w.k_src)["plane"]
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say(w.name, "flat two-step batch vs oracle rel L2 %.2e" % rel)
        assert rel <= 1e-5
        assert np.array_equal(got, pl)
    b.close()
    wide = zda.Zone(zda.default_desc(r_in=100.0, nr=20, nphi=33, nz=20, n_fold=16, m=1, pml=(3, 3, 3, 3),
                                     k_mon=12, design=(8, 10)))
    with pytest.raises(zda.ZdaError) as ex:
        wide.set_launch(8, 34)
    assert ex.value.status == zda.ZDA_ERR_ARG
    wide.close()


def test_lens_in_waves_equals_one_batch(zda):
    """A lens run in waves of zones (each wave one batch, released before the
    next) gives every zone's exit-plane DFT bitwise equal to one batch of all
    zones."""
    from paper_2501_07979_amd import lens
    wls = _zones(seed=75)
    eps = [w.eps() for w in wls]
    zones = [zda.Zone(zda.default_desc(**w.desc_kwargs()), e) for w, e in zip(wls, eps)]
    b = zda.Batch(zones)
    b.set_launch(13)
    b.run([zda.preset_source(k_src=w.k_src, omega_c=w.omega_c, width=w.width) for w in wls], wls[0].steps,
          wls[0].omegas)
    ref = [z.dft(zda.MON_PLANE).cpu().numpy() for z in zones]
    b.close()
    for z in zones:
        z.close()
    budget = lens.zone_device_bytes(wls[0]) + lens.zone_device_bytes(wls[1]) + 1
    _say("lens in waves, budget", budget)
    planes, ms, nwaves = lens.run_in_waves(wls, wls[0].steps, budget)
    assert nwaves >= 2 and ms > 0
    for a, r in zip(planes, ref):
        assert np.array_equal(a, r)


def test_waves_group_zones_by_kernel_family(zda):
    """A lens with the continuous axis zone (flat-mapped two-step kernel) and
    wedges (two-step kernel) in waves: each zone's exit-plane DFT is bitwise
    that of the zone run alone with the same kernel family."""
    from paper_2501_07979_amd import lens
    from paper_2501_07979_amd.workloads import Workload
    om = (0.28, 0.33, 0.39)
    common = dict(nz=40, k_src=8, k_mon=30, design=(12, 16), k_sub=12, steps=150, omegas=om, omega_c=0.33,
                  width=6.0, density="smoothed")
    wls = [Workload("ring2", r_in=40.5, nr=30, nphi=64, n_fold=4, pml=(5, 5, 5, 5), seed=85, **common),
           Workload("axis", r_in=0.5, nr=40, nphi=1, n_fold=0, pml=(0, 5, 5, 5), axis=1, seed=84, **common),
           Workload("ring3", r_in=70.5, nr=30, nphi=64, n_fold=8, pml=(5, 5, 5, 5), seed=86, **common)]
    ref = []
    for w in wls:
        z = zda.Zone(zda.default_desc(**w.desc_kwargs()), w.eps())
        if lens.is_narrow(w):
            z.set_launch(lens.family_kchunk(lens.FLAT, w), lens.FLAT)
        z.run(w.steps, w.omegas, k_src=w.k_src, omega_c=w.omega_c, width=w.width)
        ref.append(z.dft(zda.MON_PLANE).cpu().numpy())
        z.close()
    _say("waves by family")
    planes, ms, nwaves = lens.run_in_waves(wls, wls[0].steps, 1 << 40)
    assert nwaves == 2
    for a, r in zip(planes, ref):
        assert np.array_equal(a, r)
