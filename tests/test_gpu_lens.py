"""A lens of three zones (the continuous zone containing the axis, then two
wedges with growing n; the first two on the flat-mapped kernel, the third
on the 13-row one) stepped in batches: its focal phasors equal the sum
of the zones' phasors from the FP64 oracle, and the gradient of the lens's
focal intensity (one batched adjoint run) matches central finite differences
of the same objective taken with the oracle, at a design pixel of each
zone (to 1e-3 of the gradient's largest entry)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-lens]", *a, flush=True)


def _zones():
    from paper_2501_07979_amd.workloads import Workload
    common = dict(nz=60, m=1, k_src=12, k_mon=50, design=(24, 30), k_sub=24, steps=2000, omegas=(0.3, 0.36),
                  omega_c=0.33, width=8.0, density="smoothed")
    return [Workload("axis", r_in=0.5, nr=24, nphi=1, n_fold=0, pml=(0, 4, 6, 6), axis=1, seed=91, **common),
            Workload("ring2", r_in=24.5, nr=24, nphi=32, n_fold=4, pml=(4, 4, 6, 6), seed=92, **common),
            Workload("ring3", r_in=48.5, nr=24, nphi=40, n_fold=8, pml=(4, 4, 6, 6), seed=93, **common)]


def test_lens_phasors_and_gradient(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd.lens import Lens
    wls = _zones()
    lens = Lens(wls)
    rho0 = [w.rho() for w in wls]
    rhos = [torch.tensor(r, device="cuda", requires_grad=True) for r in rho0]
    _say("lens forward + backward")
    F, a = lens.objective(rhos)
    F.backward()
    grads = [r.grad.cpu().numpy().astype(np.float64) for r in rhos]
    a_gpu = a.detach().cpu().numpy()
    W = [w.cpu().numpy().astype(np.complex128) for w in lens.weights]
    om = np.array(wls[0].omegas)

    oz = [oracle_mod.OracleZone(**w.desc_kwargs(), eps=w.eps()) for w in wls]

    def zone_phasor(z, r):
        oz[z].set_design(r, fp64=True)
        w = wls[z]
        out = oz[z].forward(w.steps, om, omega_c=w.omega_c, width=w.width, k_src=w.k_src)
        return np.einsum("kaij,kaij->k", W[z], out["plane"])

    base = [zone_phasor(z, rho0[z].astype(np.float64)) for z in range(len(wls))]
    a_ref = sum(base)
    err = np.linalg.norm(a_gpu - a_ref) / np.linalg.norm(a_ref)
    _say("lens phasors rel L2 %.2e" % err)
    assert err <= 1e-5
    assert all(np.linalg.norm(b) > 1e-3 * np.linalg.norm(a_ref) for b in base)   # every zone contributes

    scale = max(np.abs(g).max() for g in grads)
    h = 1e-3
    for z, (l, i, j) in [(0, (2, 8, 0)), (1, (3, 10, 5)), (2, (1, 14, 20))]:
        vals = []
        for s in (+1.0, -1.0):
            r2 = rho0[z].astype(np.float64).copy()
            r2[l, i, j] += s * h
            az = zone_phasor(z, r2)
            vals.append(float(np.sum(np.abs(a_ref - base[z] + az) ** 2)))
        fd = (vals[0] - vals[1]) / (2 * h)
        e = abs(fd - grads[z][l, i, j]) / scale
        _say("zone", z, "pixel", (l, i, j), "fd %.6e gpu %.6e |diff|/max|g| %.2e" % (fd, grads[z][l, i, j], e))
        assert e <= 1e-3
    lens.close()


@pytest.mark.parametrize("zone", [0, 1, 15])
def test_lwir_zone_full_size_in_the_lens_launch(oracle_mod, zone):
    """Zones of the LWIR-shaped lens at full size (1250 x 11 x 180 cells; the
    continuous axis zone 1250 x 1 x 180) in the launch that the lens batches
    run (flat-mapped two-step kernel, 16-plane chunks): arbitrary fields on
    every cell, stepped 21 times (an odd count: ten two-step launches and one
    flat fused step), against the FP64 oracle, every field to 1e-5."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import lens, zda
    from paper_2501_07979_amd.workloads import lwir_lens
    w = lwir_lens()[zone]
    eps = w.eps()
    g = zda.Zone(zda.default_desc(**w.desc_kwargs()), eps)
    g.set_launch(lens.family_kchunk(lens.FLAT, w), lens.FLAT)
    o = oracle_mod.OracleZone(**w.desc_kwargs(), eps=eps)
    rng = np.random.default_rng(64 + zone)
    _say("full-size LWIR zone", w.name, "launch", g.info().tile_rows, g.info().kchunk)
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        f = (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)).astype(np.complex64)
        if c in ("Er", "Ephi", "Hz"):
            f[0] = 0
        if w.r_in >= w.dr and c in ("Ephi", "Ez", "Hr"):
            f[:, 0] = 0
        g.write_field(c, f)
        o.set_field(c, f.astype(np.complex128))
    steps = 21
    zero = np.zeros((1, 2, w.nr, w.nphi), np.complex64)
    g.run(steps, (), kind=zda.SRC_CUSTOM, k_src=w.k_src, patterns=zero, profiles=np.zeros((1, steps)), plane=False,
          cont=True)
    o.run(steps, m=w.m, reset=False)
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        got, ref = g.read_field(c).cpu().numpy(), o.get_field(c)
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say(w.name, c, "rel L2 %.2e" % e)
        assert e <= 1e-5, (c, e)
    g.close()


def test_lens_in_waves_gives_the_same_bits():
    """The lens run in waves (each zone holding its field memory only while
    it steps, one zone per wave here) gives the same phasors and gradient
    bits as the lens whose zones stay resident."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd.lens import Lens
    wls = _zones()
    for w in wls:
        w.steps = 600
    out = []
    for waves in (False, True):
        lens = Lens(wls, waves=waves, budget_bytes=1 if waves else None)
        _say("lens, waves", waves, "groups", len(lens.groups))
        rhos = [torch.tensor(w.rho(), device="cuda", requires_grad=True) for w in wls]
        F, a = lens.objective(rhos)
        F.backward()
        out.append((a.detach().cpu().numpy(), [r.grad.cpu().numpy() for r in rhos]))
        if waves:
            assert len(lens.groups) == len(wls)
            assert all(z.info().device_bytes < 0.5 * zone_full for z, zone_full in zip(lens.zones, full_bytes))
        else:
            full_bytes = [z.info().device_bytes for z in lens.zones]
        lens.close()
    assert np.array_equal(out[0][0], out[1][0])
    for g0, g1 in zip(out[0][1], out[1][1]):
        assert np.array_equal(g0, g1)
