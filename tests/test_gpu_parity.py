"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances: exit-plane DFT relative L2 <= 1e-5 (FP32
fields vs FP64), adjoint gradient relative L2 <= 1e-4."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-parity]", *a, flush=True)


@pytest.fixture(scope="module")
def zda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda as Z
    Z.load()
    return Z


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# launch shapes: (kchunk, tile_rows); tile_rows 3/7/15 select the fused
# double-buffered step, 5/13 the two-step kernel, 1/2/4/8/16 the split
# in-place H and E kernels, 32 the in-place kernels with the flat (r, phi)
# mapping, 33 the fused step with the flat mapping (nphi <= 64), 34 the
# two-step kernel with the flat mapping (nphi <= 32), 11 the three-step
# kernel; None keeps the zone's default
SHAPES = {"default": None, "fused_tr3_kc7": (7, 3), "fused_tr15_kc13": (13, 15), "split_r4_kc7": (7, 4),
          "split_r1": (0, 1), "two_tr13_kc9": (9, 13), "two_tr5_kc6": (6, 5), "two_tr5_kc3": (3, 5),
          "flat_kc5": (5, 32), "flatfused_kc5": (5, 33), "flattwo_kc5": (5, 34), "flattwo_kc16": (16, 34),
          "three_kc9": (9, 11), "three_kc4": (4, 11)}
# widest zone (phi cells) of the flat-mapped fused and two-step kernels
FLAT_MAX_PHI = {33: 64, 34: 32}


def skip_if_too_wide(shape, nphi):
    if shape is not None and nphi > FLAT_MAX_PHI.get(shape[1], nphi):
        pytest.skip("launch code %d takes zones of at most %d phi cells" % (shape[1], FLAT_MAX_PHI[shape[1]]))


def _zone_pair(zda, oracle_mod, wl, eps, shape=None):
    skip_if_too_wide(shape, wl.nphi)
    g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    if shape is not None:
        kc, tr = shape
        g.set_launch(kc if kc > 0 else wl.nz, tr)
    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=eps)
    return g, o


@pytest.mark.parametrize("shape", ["default", "split_r4_kc7", "two_tr13_kc9", "three_kc9"])
def test_c1_parity_exit_plane_dft(zda, oracle_mod, shape):
    from paper_2501_07979_amd.workloads import c1
    wl = c1()
    _say("c1 full parity", wl.name, wl.steps, shape)
    eps = wl.eps()
    g, o = _zone_pair(zda, oracle_mod, wl, eps, SHAPES[shape])
    g.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    gpu = g.dft(zda.MON_PLANE).cpu().numpy()
    ref = o.forward(wl.steps, np.array(wl.omegas), omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src)["plane"]
    err = _rel(gpu, ref)
    _say("c1 exit-plane DFT rel L2 = %.3e" % err)
    assert err <= 1e-5
    # the fields themselves after 1000 steps
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        e = _rel(g.read_field(c).cpu().numpy(), o.get_field(c))
        assert e <= 1e-4, (c, e)


@pytest.mark.parametrize("shape", ["default", "fused_tr3_kc7", "fused_tr15_kc13", "split_r4_kc7", "two_tr13_kc9",
                                   "two_tr5_kc6", "two_tr5_kc3", "flat_kc5", "three_kc9"])
@pytest.mark.parametrize("case", ["ragged_m1", "ragged_m0", "ragged_mneg", "no_pml"])
def test_ragged_shapes_all_fields(zda, oracle_mod, case, shape):
    """Shapes that are not multiples of the tile (nphi 70, nr 37) with uneven
    PML widths and several z-chunks; every field and the DFTs compared."""
    from paper_2501_07979_amd.workloads import Workload
    m = {"ragged_m1": 1, "ragged_m0": 0, "ragged_mneg": -1, "no_pml": 1}[case]
    pml = (0, 0, 0, 0) if case == "no_pml" else (5, 6, 4, 7)
    wl = Workload(case, r_in=90.0, nr=37, nphi=70, nz=50, n_fold=7, m=m, dz=0.9, pml=pml, k_src=9, k_mon=40,
                  design=(12, 17), k_sub=12, steps=300, omegas=(0.28, 0.33), omega_c=0.31, width=7.0, seed=5)
    rng = np.random.default_rng(21)
    eps = (1.0 + 4.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    _say("ragged", case, shape)
    g, o = _zone_pair(zda, oracle_mod, wl, eps, SHAPES[shape])
    kind = zda.SRC_RADIAL if m == 0 else zda.SRC_PLANE_CIRC
    g.run(wl.steps, wl.omegas, kind=kind, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width, volume=True)
    ref = o.forward(wl.steps, np.array(wl.omegas), omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src,
                    kind="radial" if m == 0 else "plane_circ", volume=True)
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        e = _rel(g.read_field(c).cpu().numpy(), o.get_field(c))
        assert e <= 2e-5, (case, c, e)
    assert _rel(g.dft(zda.MON_PLANE).cpu().numpy(), ref["plane"]) <= 1e-5
    assert _rel(g.dft(zda.MON_VOLUME).cpu().numpy(), ref["vol"]) <= 1e-5


@pytest.mark.parametrize("shape", ["default", "fused_tr3_kc7", "split_r4_kc7", "two_tr13_kc9", "two_tr5_kc3",
                                   "flat_kc5", "flatfused_kc5", "three_kc9", "three_kc4"])
def test_random_state_steps_with_pml(zda, oracle_mod, shape):
    """Arbitrary initial fields (written through the ABI) stepped without
    reset: every update term, PML auxiliary and the seam act from step 1
    (an odd step count, so a two-step run ends with one single step)."""
    from paper_2501_07979_amd.workloads import Workload
    wl = Workload("random_state", r_in=60.0, nr=29, nphi=64, nz=33, n_fold=6, m=2, pml=(6, 5, 5, 6), k_src=3,
                  k_mon=20, design=(10, 12), steps=41)
    rng = np.random.default_rng(22)
    eps = (1.0 + 3.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    g, o = _zone_pair(zda, oracle_mod, wl, eps, SHAPES[shape])
    _say("random state", shape)
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        f = (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)).astype(np.complex64)
        if c == "Er":
            f[0] = 0
        if c == "Ephi":
            f[0] = 0
            f[:, 0] = 0
        if c == "Ez":
            f[:, 0] = 0
        if c == "Hr":
            f[:, 0] = 0
        if c == "Hz":
            f[0] = 0
        g.write_field(c, f)
        o.set_field(c, f.astype(np.complex128))
    zero = np.zeros((1, 2, wl.nr, wl.nphi), np.complex64)
    g.run(wl.steps, (), kind=zda.SRC_CUSTOM, k_src=wl.k_src, patterns=zero, profiles=np.zeros((1, wl.steps)),
          plane=False, cont=True)
    o.run(wl.steps, m=wl.m, reset=False)
    for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz"):
        e = _rel(g.read_field(c).cpu().numpy(), o.get_field(c))
        assert e <= 1e-5, (c, e)


def test_custom_source_profiles(zda, oracle_mod):
    """Several complex patterns with complex time profiles (the adjoint's
    source form) match the oracle."""
    from paper_2501_07979_amd.workloads import Workload
    wl = Workload("custom_src", r_in=100.0, nr=30, nphi=64, nz=40, n_fold=8, m=1, pml=(5, 5, 5, 5), k_src=12,
                  k_mon=30, design=(15, 20), steps=250, omegas=(0.3, 0.35, 0.4))
    rng = np.random.default_rng(23)
    eps = (1.0 + 2.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    g, o = _zone_pair(zda, oracle_mod, wl, eps)
    P = 3
    pat = (rng.standard_normal((P, 2, wl.nr, wl.nphi)) + 1j * rng.standard_normal((P, 2, wl.nr, wl.nphi)))
    prof = rng.standard_normal((P, wl.steps)) + 1j * rng.standard_normal((P, wl.steps))
    prof[:, 60:] = 0
    _say("custom source")
    g.run(wl.steps, wl.omegas, kind=zda.SRC_CUSTOM, k_src=wl.k_src, patterns=pat.astype(np.complex64),
          profiles=prof)
    pat32 = pat.astype(np.complex64).astype(np.complex128)
    ref = o.run(wl.steps, patterns=pat32, profiles=prof, k_src=wl.k_src, omegas=wl.omegas)
    assert _rel(g.dft(zda.MON_PLANE).cpu().numpy(), ref["plane"]) <= 1e-5


def _objective(wts, plane):
    s = np.einsum("kaij,kaij->k", wts, plane)
    return np.sum(np.abs(s) ** 2), np.conj(s)[:, None, None, None] * wts


@pytest.mark.parametrize("shape", ["default", "split_r4_kc7", "two_tr5_kc6", "three_kc4"])
def test_gradient_parity_small_copy(zda, oracle_mod, shape):
    """Adjoint gradient over the design layer of the gradient zone's small
    copy (64 x 64 x 96, three frequencies) against the oracle's gradient."""
    from paper_2501_07979_amd.workloads import c3_small
    wl = c3_small()
    rho = wl.rho()
    eps = wl.eps(rho)
    g, o = _zone_pair(zda, oracle_mod, wl, eps, SHAPES[shape])
    om = np.array(wl.omegas)
    _say("gradient small copy forward", wl.name, wl.steps, shape)
    g.run(wl.steps, om, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width, volume=True)
    fwd = o.forward(wl.steps, om, omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src, volume=True)
    gp = g.dft(zda.MON_PLANE).cpu().numpy()
    assert _rel(gp, fwd["plane"]) <= 1e-5
    assert _rel(g.dft(zda.MON_VOLUME).cpu().numpy(), fwd["vol"]) <= 1e-5
    rng = np.random.default_rng(31)
    wts = (rng.standard_normal((3, 2, wl.nr, wl.nphi)) + 1j * rng.standard_normal((3, 2, wl.nr, wl.nphi)))
    _, dF = _objective(wts, fwd["plane"])
    _say("gradient small copy adjoint")
    grad_gpu = g.adjoint_grad(dF.astype(np.complex64)).cpu().numpy()
    grad_ref = o.adjoint_grad(dF.astype(np.complex64).astype(np.complex128))
    err = _rel(grad_gpu, grad_ref)
    _say("gradient rel L2 = %.3e" % err)
    assert err <= 1e-4
    assert np.isfinite(g.dft(zda.MON_ADJOINT_VOLUME).cpu().numpy()).all()


def test_production_zone_full_size_steps(zda, oracle_mod):
    """The production zone (512 x 1024 x 400, n = 512, 12-cell PML, source and
    3-frequency exit-plane DFT) in the launch shape the benchmark times:
    random fields everywhere, a few steps, every field and the DFT plane
    compared with the FP64 oracle on the full zone."""
    from paper_2501_07979_amd.workloads import c2
    wl = c2()
    steps = 3
    rng = np.random.default_rng(51)
    eps = wl.eps()
    _say("production zone: building GPU and oracle zones")
    g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=eps)
    del eps
    masks = {"Er": ("k0",), "Ephi": ("k0", "i0"), "Ez": ("i0",), "Hr": ("i0",), "Hphi": (), "Hz": ("k0",)}
    for c, zero in masks.items():
        f = rng.standard_normal((wl.nz, wl.nr, 2 * wl.nphi), dtype=np.float32).view(np.complex64)
        if "k0" in zero:
            f[0] = 0
        if "i0" in zero:
            f[:, 0] = 0
        g.write_field(c, f)
        o.set_field(c, f)
        del f
    _say("production zone: stepping")
    g.run(steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width, n0=1, cont=True)
    g_, n0 = oracle_mod.pulse(steps, o.dt, wl.omega_c, wl.width, 1)
    assert np.abs(g_).max() > 0
    ref = o.run(steps, patterns=o.preset_pattern()[None], profiles=g_[None], k_src=wl.k_src,
                omegas=np.array(wl.omegas), reset=False)
    _say("production zone: comparing")
    for c in masks:
        a = g.read_field(c).cpu().numpy()
        b = o.get_field(c)
        e = _rel(a, b)
        _say("production zone", c, "rel L2 %.2e" % e)
        assert e <= 1e-5, (c, e)
        del a, b
    assert _rel(g.dft(zda.MON_PLANE).cpu().numpy(), ref["plane"]) <= 1e-5
    g.close()


def test_fused_launch_shapes_are_bitwise_identical(zda):
    """Every cell is computed by the same instruction sequence whatever the
    tile and chunk shape (halo values are recomputed, not approximated), so
    the fused step and the two-step kernel give the same bits for every
    launch shape, whether the layer tiles keep step one's auxiliaries in
    registers (the default; both 7-row r-layer bands of this zone take the
    7-row r-layer-only tiles in the chunks without z-layer planes and 5-row
    tiles in the others) or pass them through the intermediate set."""
    from paper_2501_07979_amd.workloads import Workload
    wl = Workload("determinism", r_in=360.0, nr=37, nphi=130, nz=41, n_fold=14, m=1, pml=(5, 6, 4, 7), k_src=9,
                  k_mon=30, design=(12, 17), k_sub=12, steps=120, omegas=(0.3,), omega_c=0.3, width=6.0)
    rng = np.random.default_rng(41)
    eps = (1.0 + 4.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    outs = []
    for kc, tr, opt, val in [(41, 7, 0, 0), (5, 3, 0, 0), (13, 15, 0, 0), (1, 7, 0, 0), (9, 13, 0, 0), (41, 13, 0, 0),
                             (4, 5, 0, 0), (1, 5, 0, 0), (9, 13, zda.OPT_LAYER_STREAM, 1), (4, 5, zda.OPT_XCD_REMAP, 1),
                             (9, 13, zda.OPT_TILE_PATCH, (2 << 8) | 2), (4, 5, zda.OPT_TILE_PATCH, (3 << 8) | 1),
                             (24, 13, zda.OPT_LAYER_KCHUNK, 0), (24, 13, zda.OPT_LAYER_KCHUNK, 5),
                             (9, 13, zda.OPT_NT_STORES, 1), (5, 3, zda.OPT_NT_STORES, 1),
                             (9, 13, zda.OPT_LAYER_CARRY, 0), (41, 13, zda.OPT_LAYER_CARRY, 0),
                             (4, 5, zda.OPT_LAYER_CARRY, 0), (24, 13, zda.OPT_LAYER_CARRY, 0)]:
        _say("determinism", kc, tr, opt, val)
        g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        g.set_launch(kc, tr)
        if opt:
            g.set_option(opt, val)
        g.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        outs.append([g.read_field(c).cpu().numpy() for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz")] +
                    [g.dft(zda.MON_PLANE).cpu().numpy()])
        g.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("pml", [(8, 8, 8, 8), (12, 12, 12, 12)])
def test_rband_tilings_are_bitwise_identical(zda, pml):
    """The r-layer bands of 10 and 9 rows (8-cell layers: carried tiles of 5
    rows) and of 14 and 13 rows (12-cell layers: carried tiles of 7 rows
    with the r-layer recursions only in the chunks without z-layer planes,
    5 rows in the others): the same bits as the fused step and as the layer
    tiles that pass their auxiliaries through the intermediate set."""
    from paper_2501_07979_amd.workloads import Workload
    wl = Workload("rband_determinism", r_in=480.0, nr=56, nphi=96, nz=48, n_fold=16, m=1, pml=pml, k_src=14,
                  k_mon=32, design=(18, 22), k_sub=18, steps=90, omegas=(0.3,), omega_c=0.3, width=6.0)
    rng = np.random.default_rng(44)
    eps = (1.0 + 4.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    kinds = set(int(k) for k in zda.plan_two_step_tiles(zda.default_desc(**wl.desc_kwargs()), 13, 9, k_src=wl.k_src,
                                                         order=1 << 16)[0][:, 3])
    assert kinds == ({0, 1, 2} if pml[0] == 8 else {0, 1, 2, 4}), kinds
    outs = []
    for kc, tr, carry in [(5, 3, 1), (9, 13, 1), (48, 13, 1), (4, 5, 1), (9, 13, 0)]:
        _say("r-band determinism", pml, kc, tr, carry)
        g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        g.set_launch(kc, tr)
        g.set_option(zda.OPT_LAYER_CARRY, carry)
        g.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        outs.append([g.read_field(c).cpu().numpy() for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz")] +
                    [g.dft(zda.MON_PLANE).cpu().numpy()])
        g.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("nphi", [11, 24])
def test_narrow_zone_launch_shapes_are_bitwise_identical(zda, nphi):
    """A narrow wedge gives the same bits on the 13-row two-step kernel, the
    flat-mapped fused step and the flat-mapped two-step kernel, with any
    chunk depth, with non-temporal stores and with the XCD tile order (an
    odd step count: the two-step runs end with one fused step)."""
    from paper_2501_07979_amd.workloads import Workload
    wl = Workload("narrow_determinism", r_in=600.0, nr=45, nphi=nphi, nz=41,
                  n_fold=360 * 11 // nphi, m=1, pml=(5, 6, 4, 7), k_src=9, k_mon=30, design=(12, 17), k_sub=12,
                  steps=121, omegas=(0.3,), omega_c=0.3, width=6.0)
    rng = np.random.default_rng(42)
    eps = (1.0 + 4.0 * rng.random((wl.nz, wl.nr, wl.nphi))).astype(np.float32)
    outs = []
    for kc, tr, opt, val in [(9, 13, 0, 0), (5, 33, 0, 0), (16, 34, 0, 0), (4, 34, 0, 0), (41, 34, 0, 0),
                             (16, 34, zda.OPT_NT_STORES, 1), (3, 33, zda.OPT_NT_STORES, 1),
                             (8, 34, zda.OPT_XCD_REMAP, 1)]:
        _say("narrow determinism", nphi, kc, tr, opt, val)
        g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
        g.set_launch(kc, tr)
        if opt:
            g.set_option(opt, val)
        g.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        outs.append([g.read_field(c).cpu().numpy() for c in ("Er", "Ephi", "Ez", "Hr", "Hphi", "Hz")] +
                    [g.dft(zda.MON_PLANE).cpu().numpy()])
        g.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_error_paths_on_device(zda):
    from paper_2501_07979_amd.workloads import c1
    wl = c1()
    g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps())
    with pytest.raises(zda.ZdaError) as e:
        g.adjoint_grad(np.zeros((1, 2, wl.nr, wl.nphi), np.complex64))
    assert e.value.status == zda.ZDA_ERR_STATE
    with pytest.raises(zda.ZdaError) as e:
        g.run(10, [0.3], k_src=0, omega_c=0.3, width=5.0)
    assert e.value.status == zda.ZDA_ERR_ARG
    with pytest.raises(zda.ZdaError) as e:
        g.run(10, [0.3] * 9, k_src=5, omega_c=0.3, width=5.0)
    assert e.value.status == zda.ZDA_ERR_ARG
    with pytest.raises(zda.ZdaError) as e:
        g.set_launch(10, 6)
    assert e.value.status == zda.ZDA_ERR_ARG
    g.close()
    g.close()
