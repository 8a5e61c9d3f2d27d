"""Finite-difference check of the adjoint gradient at the gradient zone's full
size (256 x 512 x 300 cells, 256 x 512 x 20 design pixels, three
frequencies, 8000 steps, by which the fields have decayed far enough for
the adjoint of the decayed DFT to be the derivative of the run's own DFT;
section on the cylindrical solver, adjoint paragraph, and eq. 6).

The FP32 path's gradient (forward run with the design-layer DFT, focal
objective, broadband -m adjoint run, overlap) is compared with central
differences (h = 1e-3) of the same objective evaluated by FP64 runs of the
same discretisation (zda_fdtd_run_fp64): a single pixel moves the objective
by about 1e-9 of itself, below FP32 rounding but far above FP64's.  Checked:
eight single pixels (the four with the largest |dF/drho| away from the
radial layers and four random ones) to 1e-3 of max |dF/drho|, and the
derivative along a random +-1 direction over 64 random pixels.

The FP64 run itself is pinned first against the FP64 oracle on the parity
zone (64 x 64 x 96, 1000 steps)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-fd-full]", *a, flush=True)


@pytest.fixture(scope="module")
def zda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import zda as Z
    Z.load()
    return Z


def test_fp64_run_matches_fp64_oracle(zda, oracle_mod):
    from paper_2501_07979_amd.workloads import c1
    wl = c1()
    eps = wl.eps()
    z = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    _say("FP64 run", wl.name)
    got = z.run_fp64(eps.astype(np.float64), wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c,
                     width=wl.width)
    z.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    f32 = z.dft(zda.MON_PLANE).cpu().numpy()
    z.close()
    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=eps)
    ref = o.forward(wl.steps, np.array(wl.omegas), omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src)["plane"]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    err32 = float(np.linalg.norm(f32 - ref) / np.linalg.norm(ref))
    _say("FP64 GPU vs FP64 oracle rel L2 %.3e (FP32 path %.3e)" % (err, err32))
    assert err <= 1e-11
    assert err32 <= 1e-5


def _eps64(wl, rho):
    """Permittivity in FP64: the FP32 map outside the design layer, eq. (6)
    in FP64 inside it."""
    k0, k1 = wl.design
    e = wl.eps(rho.astype(np.float32)).astype(np.float64)
    e[k0:k1] = wl.eps_bg + rho * (wl.eps_hi - wl.eps_bg)
    return e


H = 1e-3


@pytest.fixture(scope="module")
def full_size(zda):
    """The FP32 adjoint gradient at the gradient zone's full size, the FP64
    objective, and the sampled pixels and direction."""
    from paper_2501_07979_amd import objective
    from paper_2501_07979_amd.workloads import c3
    wl = c3()
    rho0 = wl.rho().astype(np.float64)
    om = np.array(wl.omegas)
    W = objective.focal_weights(wl, om, objective.focal_length(wl.r_in + 0.5 * wl.nr * wl.dr),
                                device="cpu").numpy().astype(np.complex128)
    z = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps(rho0.astype(np.float32)))
    kw = dict(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    _say("FP32 forward + adjoint", wl.name, "steps", wl.steps)
    z.run(wl.steps, wl.omegas, volume=True, **kw)
    plane = z.dft(zda.MON_PLANE).cpu().numpy().astype(np.complex128)
    a = np.einsum("kaij,kaij->k", W, plane)
    dF = (np.conj(a)[:, None, None, None] * W).astype(np.complex64)
    g = z.adjoint_grad(dF).cpu().numpy().astype(np.float64)
    assert np.isfinite(g).all()
    _say("F = %.6e, max|dF/drho| = %.3e" % (float(np.sum(np.abs(a) ** 2)), np.abs(g).max()))

    def F64(rho):
        p = z.run_fp64(_eps64(wl, rho), wl.steps, wl.omegas, **kw)
        b = np.einsum("kaij,kaij->k", W, p)
        return float(np.sum(np.abs(b) ** 2))

    inner = np.zeros(g.shape, bool)
    inner[:, wl.pml[0]:wl.nr - wl.pml[1], :] = True
    order = np.argsort(np.where(inner, np.abs(g), -1.0).ravel())[::-1]
    rng = np.random.default_rng(31)
    cand = np.flatnonzero(inner.ravel())
    pix = [np.unravel_index(q, g.shape) for q in list(order[:4]) + list(rng.choice(cand, 4, replace=False))]
    sel = rng.choice(cand, 64, replace=False)
    v = np.zeros(g.size)
    v[sel] = rng.choice([-1.0, 1.0], 64)
    yield {"g": g, "rho0": rho0, "F64": F64, "pix": pix, "v": v.reshape(g.shape)}
    z.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("q", range(8))
def test_full_size_pixel_against_fp64_central_difference(full_size, q):
    """Pixel q of the eight: the four largest |dF/drho| off the radial
    layers, then four random ones; agreement to 1e-3 of max |dF/drho|."""
    g, rho0, F64 = full_size["g"], full_size["rho0"], full_size["F64"]
    idx = full_size["pix"][q]
    vals = []
    for sgn in (+1.0, -1.0):
        r = rho0.copy()
        r[idx] += sgn * H
        vals.append(F64(r))
    fd = (vals[0] - vals[1]) / (2 * H)
    err = abs(fd - g[idx]) / np.abs(g).max()
    _say("pixel", tuple(int(c) for c in idx), "fd %.6e adjoint %.6e |diff|/max|g| = %.2e" % (fd, g[idx], err))
    assert err <= 1e-3, (idx, fd, g[idx])


@pytest.mark.timeout(300)
def test_full_size_direction_against_fp64_central_difference(full_size):
    """The derivative along a random +-1 direction over 64 random pixels,
    to 1e-3 of sum |g_i| over those pixels."""
    g, rho0, F64, v = full_size["g"], full_size["rho0"], full_size["F64"], full_size["v"]
    fd = (F64(rho0 + H * v) - F64(rho0 - H * v)) / (2 * H)
    gv = float(np.sum(g * v))
    err = abs(fd - gv) / float(np.sum(np.abs(g * v)))
    _say("64-pixel direction: fd %.6e adjoint %.6e |diff|/sum|g_i| = %.2e" % (fd, gv, err))
    assert err <= 1e-3
