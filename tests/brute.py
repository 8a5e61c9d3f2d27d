"""Brute-force sparse assembly of the discrete ZDA Maxwell operators.

Independent of the oracle: every curl row is written from the integral form
of Faraday's and Ampere's laws on one face of the staggered grid (circulation
of the edge fields divided by the exact annular-sector face area), not from
the difference formulas the time-stepping codes use.  The Bloch seam of
eq. (1)-(2) is the factor exp(+-i m tau) on edges read across the wedge
boundary; PEC walls remove the tangential E edges on the box faces.

PML (local-stretch reading of the regularised r-PML): in the H rows, the
terms that come from an r-derivative or an explicit 1/r carry 1/s_r at the
output point, the d/dz terms carry 1/s_z; the whole z-curl carries 1/s_r.
Same rule for the E rows on the dual faces.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

E_COMPS = ("Er", "Ephi", "Ez")
H_COMPS = ("Hr", "Hphi", "Hz")


class Grid:
    def __init__(self, *, r_in, nr, nphi, nz, n_fold, m, dr=1.0, dz=1.0, courant=0.5):
        self.r_in, self.nr, self.nphi, self.nz = r_in, nr, nphi, nz
        self.n_fold, self.m, self.dr, self.dz = n_fold, m, dr, dz
        self.dt = courant * min(dr, dz)
        self.dphi = 2 * np.pi / (n_fold * nphi)
        self.tau = 2 * np.pi / n_fold
        # active (non-PEC, not identically zero) index ranges (i, k) per component
        nr_, nz_ = nr, nz
        self.ranges = {
            "Er": (range(0, nr_), range(1, nz_)),
            "Ephi": (range(1, nr_), range(1, nz_)),
            "Ez": (range(1, nr_), range(0, nz_)),
            "Hr": (range(1, nr_), range(0, nz_)),
            "Hphi": (range(0, nr_), range(0, nz_)),
            "Hz": (range(0, nr_), range(1, nz_)),
        }
        self.index = {}
        self.offset = {}
        for group in (E_COMPS, H_COMPS):
            n = 0
            for c in group:
                self.offset[c] = n
                ir, kr = self.ranges[c]
                self.index[c] = {}
                for k in kr:
                    for i in ir:
                        for j in range(nphi):
                            self.index[c][(k, i, j)] = n
                            n += 1
            if group is E_COMPS:
                self.nE = n
            else:
                self.nH = n

    def r(self, p):
        return self.r_in + p * self.dr

    def dof(self, comp, k, i, j, m):
        """(row/col index, phase) of a component sample, or (None, 0) when the
        sample is a PEC zero; j outside [0, nphi) wraps with the Bloch phase."""
        ph = 1.0 + 0j
        if j >= self.nphi:
            j -= self.nphi
            ph = np.exp(1j * m * self.tau)
        elif j < 0:
            j += self.nphi
            ph = np.exp(-1j * m * self.tau)
        idx = self.index[comp].get((k, i, j))
        return (idx, ph) if idx is not None else (None, 0.0)

    def vectorize(self, fields, comps):
        """Pack [nz][nr][nphi] arrays into the active DOF vector."""
        n = self.nE if comps is E_COMPS else self.nH
        v = np.zeros(n, np.complex128)
        for c in comps:
            for (k, i, j), q in self.index[c].items():
                v[q] = fields[c][k, i, j]
        return v

    def unvectorize(self, v, comps):
        out = {c: np.zeros((self.nz, self.nr, self.nphi), np.complex128) for c in comps}
        for c in comps:
            for (k, i, j), q in self.index[c].items():
                out[c][k, i, j] = v[q]
        return out

    # -- operators ----------------------------------------------------------
    # geo: object with lr(p) radial edge length at radial coordinate p,
    # R(p) radius at p (the phi edge is R dphi), lz(q) axial edge length at q.
    # Every curl row is (circulation over the face's edges) / (face area).
    def _geo(self, geo):
        if geo is None:
            class _G:
                pass
            geo = _G()
            geo.lr = lambda p: self.dr
            geo.R = lambda p: self.r(p)
            geo.lz = lambda q: self.dz
        return geo

    def _assemble(self, m, loops, nrows, ncols):
        rows, cols, vals = [], [], []
        for row, area, terms in loops:
            for comp, k, i, j, w in terms:
                col, ph = self.dof(comp, k, i, j, m)
                if col is not None:
                    rows.append(row)
                    cols.append(col)
                    vals.append(w * ph / area)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nrows, ncols))

    def curl_e(self, m, geo=None):
        """C_E: E dofs -> (curl E) at H dofs, Faraday loops on primal faces."""
        g = self._geo(geo)
        dph = self.dphi
        loops = []
        for (k, i, j), row in self.index["Hr"].items():
            # face (phi x z) at radius i: Ephi at z_k (+), Ez at phi_{j+1} (+), Ephi at z_{k+1} (-), Ez at phi_j (-)
            Lp, Lz = g.R(i) * dph, g.lz(k + 0.5)
            loops.append((row, Lp * Lz, [("Ephi", k, i, j, Lp), ("Ez", k, i, j + 1, Lz),
                                         ("Ephi", k + 1, i, j, -Lp), ("Ez", k, i, j, -Lz)]))
        for (k, i, j), row in self.index["Hphi"].items():
            # face (z x r): Ez at r_i (+), Er at z_{k+1} (+), Ez at r_{i+1} (-), Er at z_k (-)
            Lr, Lz = g.lr(i + 0.5), g.lz(k + 0.5)
            loops.append((row, Lr * Lz, [("Ez", k, i, j, Lz), ("Er", k + 1, i, j, Lr),
                                         ("Ez", k, i + 1, j, -Lz), ("Er", k, i, j, -Lr)]))
        for (k, i, j), row in self.index["Hz"].items():
            # face (r x phi) at z_k: Er at phi_j (+), Ephi at r_{i+1} (+), Er at phi_{j+1} (-), Ephi at r_i (-)
            Lr = g.lr(i + 0.5)
            loops.append((row, Lr * g.R(i + 0.5) * dph,
                          [("Er", k, i, j, Lr), ("Ephi", k, i + 1, j, g.R(i + 1) * dph),
                           ("Er", k, i, j + 1, -Lr), ("Ephi", k, i, j, -g.R(i) * dph)]))
        return self._assemble(m, loops, self.nH, self.nE)

    def curl_h(self, m, geo=None):
        """C_H: H dofs -> (curl H) at E dofs, Ampere loops on dual faces."""
        g = self._geo(geo)
        dph = self.dphi
        loops = []
        for (k, i, j), row in self.index["Er"].items():
            Lp, Lz = g.R(i + 0.5) * dph, g.lz(k)
            loops.append((row, Lp * Lz, [("Hphi", k - 1, i, j, Lp), ("Hz", k, i, j, Lz),
                                         ("Hphi", k, i, j, -Lp), ("Hz", k, i, j - 1, -Lz)]))
        for (k, i, j), row in self.index["Ephi"].items():
            Lr, Lz = g.lr(i), g.lz(k)
            loops.append((row, Lr * Lz, [("Hz", k, i - 1, j, Lz), ("Hr", k, i, j, Lr),
                                         ("Hz", k, i, j, -Lz), ("Hr", k - 1, i, j, -Lr)]))
        for (k, i, j), row in self.index["Ez"].items():
            Lr = g.lr(i)
            loops.append((row, Lr * g.R(i) * dph,
                          [("Hr", k, i, j - 1, Lr), ("Hphi", k, i, j, g.R(i + 0.5) * dph),
                           ("Hr", k, i, j, -Lr), ("Hphi", k, i - 1, j, -g.R(i - 0.5) * dph)]))
        return self._assemble(m, loops, self.nE, self.nH)

    def eps_vector(self, eps):
        v = np.zeros(self.nE)
        for c in E_COMPS:
            for (k, i, j), q in self.index[c].items():
                v[q] = eps[k, i, j]
        return v

    def e_weights(self, geo=None):
        """Cell volume (primal edge x dual face) at every E dof."""
        g = self._geo(geo)
        w = np.zeros(self.nE, np.complex128)
        for (k, i, j), q in self.index["Er"].items():
            w[q] = g.lr(i + 0.5) * g.R(i + 0.5) * self.dphi * g.lz(k)
        for (k, i, j), q in self.index["Ephi"].items():
            w[q] = g.R(i) * self.dphi * g.lr(i) * g.lz(k)
        for (k, i, j), q in self.index["Ez"].items():
            w[q] = g.lz(k + 0.5) * g.lr(i) * g.R(i) * self.dphi
        return w

    def h_weights(self, geo=None):
        """Cell volume (dual edge x primal face) at every H dof."""
        g = self._geo(geo)
        w = np.zeros(self.nH, np.complex128)
        for (k, i, j), q in self.index["Hr"].items():
            w[q] = g.lr(i) * g.R(i) * self.dphi * g.lz(k + 0.5)
        for (k, i, j), q in self.index["Hphi"].items():
            w[q] = g.R(i + 0.5) * self.dphi * g.lr(i + 0.5) * g.lz(k + 0.5)
        for (k, i, j), q in self.index["Hz"].items():
            w[q] = g.lz(k) * g.lr(i + 0.5) * g.R(i + 0.5) * self.dphi
        return w


class StretchedGeometry:
    """Complex edge lengths of the PML at angular frequency w (the discrete
    CFS pole F = dt / (1 - c e^{i w dt}), c = exp(-alpha dt)).

    sigma grading sigma_max rho^order in layers of d0 (inner/low) and d1
    (outer/high) cells; radial lengths dr (1 + sigma F); radius R = r + Sigma F
    with Sigma the running sum of dr * sigma from each interface outwards
    (outer layer) or inwards (inner layer, |Sigma|); axial lengths likewise."""

    def __init__(self, grid, omega, *, pml, order=3.0, sigma_max=None, alpha=0.05):
        self.g = grid
        d0, d1, z0, z1 = pml
        dt = grid.dt
        smr = sigma_max[0] if sigma_max else 0.8 * (order + 1) / grid.dr
        smz = sigma_max[1] if sigma_max else 0.8 * (order + 1) / grid.dz
        e = np.exp(1j * omega * dt)
        self.F = dt / (1.0 - np.exp(-alpha * dt) * e)

        def grade(p, n, a, b, smax):
            if a > 0 and p < a:
                return smax * ((a - p) / a) ** order
            if b > 0 and p > n - b:
                return smax * ((p - (n - b)) / b) ** order
            return 0.0
        self.sr = lambda p: grade(p, grid.nr, d0, d1, smr)
        self.sz = lambda q: grade(q, grid.nz, z0, z1, smz)
        # Sigma on the half-integer lattice p = 0, 1/2, 1, ..., nr
        pts = np.arange(0, 2 * grid.nr + 1) / 2.0
        Sig = {p: 0.0 for p in pts}
        for p in pts:                       # outer: accumulate outwards
            if p > grid.nr - d1 and p - 1 >= 0:
                Sig[p] = Sig[p - 1] + grid.dr * self.sr(p - 0.5)
        for p in pts[::-1]:                 # inner: accumulate inwards
            if p < d0 and p + 1 <= grid.nr:
                Sig[p] = Sig[p + 1] + grid.dr * self.sr(p + 0.5)
        self.Sig = Sig

    def lr(self, p):
        return self.g.dr * (1 + self.sr(p) * self.F)

    def R(self, p):
        return self.g.r(p) + self.Sig.get(p, 0.0) * self.F

    def lz(self, q):
        return self.g.dz * (1 + self.sz(q) * self.F)


