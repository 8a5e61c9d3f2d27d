"""The entry point that allocates nothing (zda_fdtd_run_noalloc) against
zda_fdtd_run: the same zones, sources and launch shapes give the same
exit-plane and design-layer DFTs (bitwise: the same kernels read the same
staged values, only from the library's fixed scratch array), on two calls in
a row of which the second is smaller, after which the zone owns no more
device memory than before.  Limits and refusals are checked too."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def zda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda as Z
    Z.load()
    return Z


def _large():
    from paper_2501_07979_amd.workloads import Workload
    return Workload("noalloc_64x192x96", r_in=600.0, nr=64, nphi=192, nz=96, n_fold=16, pml=(8, 8, 8, 8), k_src=20,
                    k_mon=80, design=(30, 40), k_sub=30, steps=300, omegas=(0.28, 0.31, 0.34), omega_c=0.31,
                    width=10.0, seed=21)


def _small():
    from paper_2501_07979_amd.workloads import Workload
    return Workload("noalloc_30x64x40", r_in=200.0, nr=30, nphi=64, nz=40, n_fold=16, pml=(4, 4, 4, 4), k_src=8,
                    k_mon=30, design=(14, 18), k_sub=14, steps=121, omegas=(0.31,), omega_c=0.31, width=8.0, seed=22)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (kchunk, tile_rows): None = the zone's default (two-step kernel), the fused
# one-step kernel, the split pair, the three-step kernel
SHAPES = [None, (12, 3), (7, 4), (9, 11)]


@pytest.mark.parametrize("shape", SHAPES, ids=["default", "fused_r3", "split_r4", "three_r11"])
def test_noalloc_matches_run_on_two_calls(zda, shape):
    calls = [_large(), _small()]          # the second call is smaller (zone, steps, frequencies)
    zones = []
    for wl in calls:
        eps = wl.eps()
        ref = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        new = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        if shape is not None:
            ref.set_launch(*shape)
            new.set_launch(*shape)
        zones.append((wl, ref, new))
    for wl, ref, new in zones:
        _say(wl.name, shape)
        kw = dict(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        ref.run(wl.steps, wl.omegas, **kw)
        a = ref.dft(zda.MON_PLANE).cpu().numpy()
        before = new.info().device_bytes
        new.run(wl.steps, wl.omegas, noalloc=True, **kw)
        b = new.dft(zda.MON_PLANE).cpu().numpy()
        assert new.info().device_bytes == before
        err = _rel(b, a)
        _say("exit-plane DFT: rel L2 %.3e against zda_fdtd_run, bitwise %s" % (err, np.array_equal(a, b)))
        assert err <= 1e-5
        assert np.array_equal(a, b)
    for _, ref, new in zones:
        ref.close()
        new.close()


def test_noalloc_volume_and_continue(zda):
    """A design-layer run (buffer allocated by a first ordinary run) and a
    continued run through the entry point, against the ordinary entry point."""
    wl = _small()
    kw = dict(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    eps = wl.eps()
    ref = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    new = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    with pytest.raises(zda.ZdaError) as e:
        new.run(wl.steps, wl.omegas, volume=True, noalloc=True, **kw)
    assert e.value.status == zda.ZDA_ERR_STATE
    new.run(4, wl.omegas, volume=True, **kw)        # allocates the design-layer buffer
    before = new.info().device_bytes
    for z, na in ((ref, False), (new, True)):
        z.run(60, wl.omegas, volume=True, noalloc=na, **kw)
        z.run(61, wl.omegas, volume=True, cont=True, noalloc=na, **kw)
    assert new.info().device_bytes == before
    for mon in (zda.MON_PLANE, zda.MON_VOLUME):
        a = ref.dft(mon).cpu().numpy()
        b = new.dft(mon).cpu().numpy()
        assert _rel(b, a) <= 1e-5
        assert np.array_equal(a, b)
    ref.close()
    new.close()


def test_noalloc_refuses_beyond_its_limits(zda):
    wl = _small()
    z = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps())
    kw = dict(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    lib = zda.load()
    too_many = (1 << 17) // 3 + 1                       # nsteps * K beyond the twiddle slice
    with pytest.raises(zda.ZdaError) as e:
        z.run(too_many, (0.2, 0.3, 0.4), noalloc=True, **kw)
    assert e.value.status == zda.ZDA_ERR_ARG
    assert b"no-allocation limit" in lib.zda_last_error()
    with pytest.raises(zda.ZdaError) as e:
        z.run(10, wl.omegas, timing=True, noalloc=True, **kw)
    assert e.value.status == zda.ZDA_ERR_ARG
    # the zone still runs normally through the entry point afterwards
    z.run(wl.steps, wl.omegas, noalloc=True, **kw)
    assert np.isfinite(z.dft_host(zda.MON_PLANE)).all()
    z.close()
