"""GPU parity at the lengths and sizes the method runs at.

* The parity zone's geometry (64 x 64 x 96, n = 16) stepped 20,000 steps, the
  production zone's job length: the FP32 exit-plane DFT (accumulated once per
  step over the whole run, section on the cylindrical solver, DTFT monitors)
  against the FP64 oracle, relative L2 <= 1e-5.
* The gradient zone at full size (256 x 512 x 300, 256 x 512 x 20 design
  pixels, three frequencies): the adjoint gradient (eq. 6 overlap of the
  forward and -m adjoint design-layer DFTs) against the oracle's, relative L2
  <= 1e-4.  Both codes run the same truncated run length, so they compute the
  same truncated-DFT adjoint; the run is short so that the oracle finishes in
  about a minute on the host cores.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-longrun]", *a, flush=True)


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


LONG_T = 20000


@pytest.fixture(scope="module")
def parity_zone_reference(oracle_mod):
    """The oracle's exit-plane DFT of the parity zone after LONG_T steps."""
    from paper_2501_07979_amd.workloads import c1
    wl = c1()
    _say("oracle: parity zone at %d steps" % LONG_T)
    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=wl.eps())
    return o.forward(LONG_T, np.array(wl.omegas), omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src)["plane"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("shape", ["default", "split_r4_kc7"])
def test_parity_zone_20000_steps(zda, parity_zone_reference, shape):
    from paper_2501_07979_amd.workloads import c1
    wl = c1()
    T = LONG_T
    _say("parity zone at %d steps" % T, wl.name, shape)
    g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps())
    if shape == "split_r4_kc7":
        g.set_launch(7, 4)
    g.run(T, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    gpu = g.dft(zda.MON_PLANE).cpu().numpy()
    g.close()
    ref = parity_zone_reference
    err = _rel(gpu, ref)
    _say("exit-plane DFT after %d steps: rel L2 = %.3e" % (T, err))
    assert err <= 1e-5


@pytest.mark.timeout(900)
def test_gradient_zone_full_size_gradient(zda, oracle_mod):
    import torch
    from paper_2501_07979_amd import objective
    from paper_2501_07979_amd.workloads import c3
    T = 300
    wl = c3(T)
    _say("gradient zone at full size", wl.name, "steps", T)
    rho = wl.rho()
    eps = wl.eps(rho)
    om = np.array(wl.omegas)
    g = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    g.run(T, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width, volume=True)
    plane_gpu = g.dft(zda.MON_PLANE).cpu().numpy()
    o = oracle_mod.OracleZone(**wl.desc_kwargs(), eps=eps)
    _say("oracle forward")
    fwd = o.forward(T, om, omega_c=wl.omega_c, width=wl.width, k_src=wl.k_src, volume=True)
    ref = fwd["plane"]
    err = _rel(plane_gpu, ref)
    _say("exit-plane DFT rel L2 = %.3e" % err)
    assert err <= 1e-5
    # the focal objective's derivative at the oracle's fields, fed to both codes
    focal = objective.focal_length(wl.r_in + 0.5 * wl.nr * wl.dr)
    W = objective.focal_weights(wl, om, focal, device="cpu").numpy().astype(np.complex128)
    a = np.einsum("kaij,kaij->k", W, ref)
    dF = (np.conj(a)[:, None, None, None] * W).astype(np.complex64)
    g_gpu = g.adjoint_grad(dF).cpu().numpy()
    g.close()
    _say("oracle adjoint")
    g_ref = o.adjoint_grad(dF.astype(np.complex128))
    gerr = _rel(g_gpu, g_ref)
    _say("design gradient (%d pixels) rel L2 = %.3e, max|g| = %.3e" % (g_ref.size, gerr, np.abs(g_ref).max()))
    assert np.isfinite(g_gpu).all()
    assert gerr <= 1e-4
    del torch
