"""Oracle pinned against brute-force sparse assembly (tests/brute.py), which is
written from the integral form of Faraday's and Ampere's laws on each face of
the staggered grid, independently of the oracle's difference code.

Pins: one leap-frog step equals the sparse step (no PML); after the fields
have decayed, the oracle's DFT monitors equal the frequency-domain solution of
(C_H C_E - wt^2 eps) E = i wt J with the stretched (PML) operator; the
oracle's adjoint gradient (one -m run, broadband source, stretched-volume
overlap) equals the gradient from a direct sparse solve of A^T lambda = g.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import brute
from brute import E_COMPS, H_COMPS


def _random_state(G, rng):
    F = {c: rng.standard_normal((G.nz, G.nr, G.nphi)) + 1j * rng.standard_normal((G.nz, G.nr, G.nphi))
         for c in E_COMPS + H_COMPS}
    E = G.unvectorize(G.vectorize(F, E_COMPS), E_COMPS)
    H = G.unvectorize(G.vectorize(F, H_COMPS), H_COMPS)
    return E, H


@pytest.mark.parametrize("m,n_fold", [(1, 6), (0, 3), (-2, 5)])
def test_step_matches_brute(oracle_mod, m, n_fold):
    rng = np.random.default_rng(10 + m)
    geo = dict(r_in=7.0, nr=5, nphi=6, nz=4, n_fold=n_fold, m=m)
    z = oracle_mod.OracleZone(**geo)
    G = brute.Grid(**geo)
    eps = (1 + 3 * rng.random(z.shape)).astype(np.float32)
    z.set_eps(eps)
    E, H = _random_state(G, rng)
    for c in E_COMPS:
        z.set_field(c, E[c])
    for c in H_COMPS:
        z.set_field(c, H[c])
    steps = 3
    z.run(steps, reset=False)
    CE, CH = G.curl_e(m), G.curl_h(m)
    e, h = G.vectorize(E, E_COMPS), G.vectorize(H, H_COMPS)
    ev = G.eps_vector(eps)
    for _ in range(steps):
        h = h - z.dt * (CE @ e)
        e = e + z.dt * (CH @ h) / ev
    Eo = G.vectorize({c: z.get_field(c) for c in E_COMPS}, E_COMPS)
    Ho = G.vectorize({c: z.get_field(c) for c in H_COMPS}, H_COMPS)
    assert np.abs(Eo - e).max() < 1e-12 * np.abs(e).max()
    assert np.abs(Ho - h).max() < 1e-12 * np.abs(h).max()
    # PEC and identically-zero samples stay zero
    for c in E_COMPS + H_COMPS:
        f = z.get_field(c)
        mask = np.ones(z.shape, bool)
        for (k, i, j) in G.index[c]:
            mask[k, i, j] = False
        assert np.all(f[mask] == 0)


def test_curl_adjointness_and_symmetry():
    """C_H = W_E^-1 C_E(-m)^T W_H for plain and stretched geometry: the
    structure the energy identity and the -m adjoint rely on."""
    geo = dict(r_in=9.0, nr=8, nphi=5, nz=7, n_fold=7, m=1)
    G = brute.Grid(**geo)
    for sg in (None, brute.StretchedGeometry(G, 0.37, pml=(3, 2, 2, 3))):
        WE, WH = G.e_weights(sg), G.h_weights(sg)
        lhs = G.curl_h(1, sg).toarray()
        rhs = np.diag(1 / WE) @ G.curl_e(-1, sg).toarray().T @ np.diag(WH)
        assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(lhs).max()


def _tiny_pml_zone(O, rng, m=1):
    geo = dict(r_in=12.0, nr=12, nphi=6, nz=14, n_fold=8, m=m)
    z = O.OracleZone(**geo, pml=(3, 3, 3, 3), k_mon=10, design=(5, 9))
    eps = np.ones(z.shape, np.float32)
    eps[:5] = 2.1
    eps[5:9] = np.where(rng.random((4, 12, 6)) < 0.5, 1.0, 6.25)
    z.set_eps(eps)
    return z, geo, eps


def _solve(G, geo_s, eps, m, omega, dt, b):
    wt = 2 / dt * np.sin(omega * dt / 2)
    A = (G.curl_h(m, geo_s) @ G.curl_e(m, geo_s) - wt ** 2 * sp.diags(G.eps_vector(eps))).tocsc()
    return A, wt, spl.spsolve(A, b)


def test_dft_equals_frequency_domain_solve_with_pml(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    z, geo, eps = _tiny_pml_zone(O, rng)
    T = 6000
    pat = rng.standard_normal((2, 12, 6)) + 1j * rng.standard_normal((2, 12, 6))
    prof, _ = O.pulse(T, z.dt, 0.35, 8.0)
    omegas = np.array([0.3, 0.35, 0.42])
    out = z.run(T, patterns=pat[None], profiles=prof[None], k_src=3, omegas=omegas, volume=True)
    # the fields have decayed: the truncated DFT is the full one
    assert max(np.abs(z.get_field(c)).max() for c in E_COMPS) < 1e-9
    G = brute.Grid(**geo)
    th = (np.arange(T) + 0.5) * z.dt
    for kk, w in enumerate(omegas):
        sg = brute.StretchedGeometry(G, w, pml=(3, 3, 3, 3))
        Jhat = z.dt * np.sum(prof * np.exp(1j * w * th))
        J = {c: np.zeros(z.shape, complex) for c in E_COMPS}
        J["Er"][3], J["Ephi"][3] = pat[0] * Jhat, pat[1] * Jhat
        wt = 2 / z.dt * np.sin(w * z.dt / 2)
        _, _, x = _solve(G, sg, eps, 1, w, z.dt, 1j * wt * G.vectorize(J, E_COMPS))
        X = G.unvectorize(x, E_COMPS)
        ref = np.stack([X["Er"][10], X["Ephi"][10]])
        assert np.linalg.norm(out["plane"][kk] - ref) < 1e-8 * np.linalg.norm(ref)
        refv = np.stack([X[c][5:9] for c in E_COMPS])
        assert np.linalg.norm(out["vol"][kk] - refv) < 1e-8 * np.linalg.norm(refv)


def _objective(wts, plane):
    """F = sum_k |sum_x w_k(x) Ehat_k(x)|^2 and its Wirtinger derivative."""
    s = np.einsum("kaij,kaij->k", wts, plane)
    return np.sum(np.abs(s) ** 2), np.conj(s)[:, None, None, None] * wts


def test_adjoint_gradient_matches_direct_adjoint_solve(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    z, geo, eps = _tiny_pml_zone(O, rng)
    T = 6000
    omegas = np.array([0.3, 0.36])
    fwd = z.forward(T, omegas, omega_c=0.33, width=8.0, k_src=3, volume=True)
    wts = rng.standard_normal((2, 2, 12, 6)) + 1j * rng.standard_normal((2, 2, 12, 6))
    _, g = _objective(wts, fwd["plane"])
    grad = z.adjoint_grad(g)
    # direct: lambda = A^{-T} g on the monitor dofs, dF/deps_c = sum 2 Re[wt^2 lambda_c E_c]
    G = brute.Grid(**geo)
    Ehat_pre = fwd["vol"]
    ref = np.zeros_like(grad)
    for kk, w in enumerate(omegas):
        sg = brute.StretchedGeometry(G, w, pml=(3, 3, 3, 3))
        wt = 2 / z.dt * np.sin(w * z.dt / 2)
        A = (G.curl_h(1, sg) @ G.curl_e(1, sg) - wt ** 2 * sp.diags(G.eps_vector(eps))).tocsc()
        gv = {c: np.zeros(z.shape, complex) for c in E_COMPS}
        gv["Er"][10], gv["Ephi"][10] = g[kk, 0], g[kk, 1]
        lam = G.unvectorize(spl.spsolve(A.T.tocsc(), G.vectorize(gv, E_COMPS)), E_COMPS)
        for a, c in enumerate(E_COMPS):
            ref += 2 * np.real(wt ** 2 * lam[c][5:9] * Ehat_pre[kk, a])
    ref *= (z.eps_hi - z.eps_bg)
    assert np.linalg.norm(grad - ref) < 1e-7 * np.linalg.norm(ref)
