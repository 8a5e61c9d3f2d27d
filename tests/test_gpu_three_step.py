"""The three-step kernel (launch code 11: three leap-frog steps per launch)
gives the same bits as the fused one-step kernel and the two-step kernel on
zones with every kind of tile (interior, z-layer planes only, r-layer bands),
on narrow wedges whose 64-lane window wraps around the zone, and on a zone
holding the axis, for several chunk depths, tile orders and step counts that
leave a remainder of one or two steps (taken by the fused step).  Its parity
with the FP64 oracle (forward DFT, adjoint gradient) is in the parity tests'
launch shapes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-three]", *a, flush=True)


@pytest.fixture(scope="module")
def zda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda as Z
    Z.load()
    return Z


def _fields(zda, g):
    return [g.read_field(c).cpu().numpy() for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz")] + \
        [g.dft(zda.MON_PLANE).cpu().numpy()]


@pytest.mark.parametrize("steps", [120, 121, 122])
@pytest.mark.parametrize("zone", ["ragged", "narrow11", "narrow24", "axis_wedge", "axis_continuous"])
def test_three_step_is_bitwise_identical(zda, zone, steps):
    from paper_2501_07979_amd.workloads import Workload
    kw = dict(r_in=360.0, nr=37, nphi=130, nz=41, n_fold=14, m=1, pml=(5, 6, 4, 7), k_src=9, k_mon=30,
              design=(12, 17), k_sub=12, steps=steps, omegas=(0.3, 0.35), omega_c=0.3, width=6.0)
    if zone == "narrow11":
        kw.update(r_in=600.0, nr=45, nphi=11, n_fold=360)
    elif zone == "narrow24":
        kw.update(r_in=600.0, nr=45, nphi=24, n_fold=165)
    elif zone == "axis_wedge":          # discrete symmetry down to the axis (small r dphi: small time step)
        kw.update(r_in=0.5, nr=37, nphi=70, n_fold=2, courant=0.02, pml=(0, 6, 4, 7), axis=1, width=0.5)
    elif zone == "axis_continuous":     # one phi sample carrying e^{i m phi}
        kw.update(r_in=0.5, nr=45, nphi=1, n_fold=0, pml=(0, 6, 4, 7), axis=1)
    wl = Workload("three_step_" + zone, **kw)
    rng = np.random.default_rng(43)
    eps = (1.0 + 4.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    outs = []
    for kc, tr, opt, val in [(5, 3, 0, 0), (9, 13, 0, 0), (9, 11, 0, 0), (41, 11, 0, 0), (4, 11, 0, 0),
                             (1, 11, 0, 0), (2, 11, 0, 0), (9, 11, zda.OPT_XCD_REMAP, 1),
                             (9, 11, zda.OPT_TILE_PATCH, (2 << 8) | 2), (9, 11, zda.OPT_LAYER_STREAM, 1),
                             (24, 11, zda.OPT_LAYER_KCHUNK, 5), (9, 11, zda.OPT_NT_STORES, 0)]:
        _say(zone, steps, "launch", kc, tr, opt, val)
        g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        g.set_launch(kc, tr)
        if opt:
            g.set_option(opt, val)
        g.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        outs.append(_fields(zda, g))
        g.close()
    for q, o in enumerate(outs[1:], 1):
        for c, (a, b) in enumerate(zip(outs[0], o)):
            assert np.array_equal(a, b), (q, c)
