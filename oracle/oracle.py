"""FP64 CPU oracle for the ZDA cylindrical FDTD hot path (arXiv 2501.07979).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this module; the product path never does.  It shares no
code with the HIP library.  The time loop lives in ``zda_oracle.c`` (plain C,
FP64 complex, OpenMP over z-planes); this module builds the source presets,
the broadband adjoint source and the gradient overlap with numpy, each step
written from its definition:

* source (soft pulsed current sheet; a normally incident plane wave is the
  m = +-1 Bloch component, section "Results and Discussion"):
  J_r = -g(t) e^{i m phi_j} / dz,  J_phi = -i sgn(m) g(t) e^{i m phi_{j+1/2}} / dz
  on plane k_src, g(t) = sin(w_c (t - t0)) exp(-(t - t0)^2 / (2 w^2)),
  sampled at t_{n+1/2}, t0 = (N0 + 1/2) dt, N0 = round(6 w / dt), zero
  outside n in [0, 2 N0].
* DTFT monitors (hybrid time/frequency adjoint paragraph):
  Ehat(w) = dt * sum_{n=1..T} E^n e^{i w n dt}.
* adjoint (same paragraph, broadband adjoint sources): with
  A_m = C_H C_E - wt^2 eps (wt = (2/dt) sin(w dt / 2)) the DFT obeys
  A_m Ehat = i wt Jhat and A_m^T = W A_{-m} W^{-1}, W the stretched cell
  volume r s_r s_z dr dphi dz of each E point.  The adjoint run uses -m and
  the current a_k = W^{-1} (dF/dEhat_k) / (i wt_k) with the broadband time
  profiles q_k = sum_l (P^{-1})_{lk} p_l, P_kl = phat_l(w_k).  The gradient is
  dF/deps_c = sum_k sum_alpha 2 Re[wt_k^2 W X Ehat] and dF/drho = (eps_h - eps_0)
  dF/deps (eq. 6).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zda_oracle.c")
_LIB = os.path.join(_HERE, "libzda_oracle.so")

COMP = {"Er": 0, "Ephi": 1, "Ez": 2, "Hr": 3, "Hphi": 4, "Hz": 5}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("r_in", ctypes.c_double), ("dr", ctypes.c_double), ("dz", ctypes.c_double),
                ("courant", ctypes.c_double),
                ("nr", ctypes.c_int), ("nphi", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_fold", ctypes.c_int),
                ("pml_r_in", ctypes.c_int), ("pml_r_out", ctypes.c_int),
                ("pml_z_lo", ctypes.c_int), ("pml_z_hi", ctypes.c_int),
                ("pml_order", ctypes.c_double), ("pml_sigma_max_r", ctypes.c_double),
                ("pml_sigma_max_z", ctypes.c_double), ("pml_alpha", ctypes.c_double),
                ("axis", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.ora_create.restype = P
        lib.ora_create.argtypes = [ctypes.POINTER(_Params)]
        lib.ora_destroy.argtypes = [P]
        lib.ora_dt.restype = ctypes.c_double
        lib.ora_dt.argtypes = [P]
        lib.ora_get_layer.argtypes = [P, ctypes.c_int, P, P, P]
        lib.ora_set_eps.argtypes = [P, P]
        lib.ora_set_eps64.argtypes = [P, P]
        lib.ora_reset.argtypes = [P]
        lib.ora_set_field.argtypes = [P, ctypes.c_int, P]
        lib.ora_get_field.argtypes = [P, ctypes.c_int, P]
        lib.ora_num_threads.restype = ctypes.c_int
        lib.ora_num_threads.argtypes = []
        lib.ora_run.restype = ctypes.c_int
        lib.ora_run.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                ctypes.c_int, P, P, ctypes.c_int,
                                ctypes.c_int, P,
                                ctypes.c_int, P,
                                ctypes.c_int, ctypes.c_int, P]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def num_threads():
    return int(_load().ora_num_threads())


def pulse(nsteps, dt, omega_c, width, n0=None):
    """g(t_{n+1/2}) for n in [0, nsteps): a Gaussian-windowed sine centred on
    t0 = (N0 + 1/2) dt, kept on the window n in [0, 2 N0] so the samples are
    odd about t0 and deposit no net charge."""
    if n0 is None:
        n0 = int(round(6.0 * width / dt))
    n = np.arange(nsteps)
    t = (n - n0) * dt                          # t_{n+1/2} - t0
    g = np.sin(omega_c * t) * np.exp(-t * t / (2.0 * width * width))
    g[n > 2 * n0] = 0.0                        # window [0, 2 N0]: sum g = 0 exactly
    return g, n0


def wtilde(omega, dt):
    """Leap-frog frequency (2/dt) sin(w dt / 2)."""
    return 2.0 / dt * np.sin(np.asarray(omega, dtype=np.float64) * dt / 2.0)


class OracleZone:
    """One ZDA zone on the CPU in FP64 complex arithmetic."""

    def __init__(self, *, r_in, nr, nphi, nz, n_fold, m, dr=1.0, dz=1.0, courant=0.5,
                 pml=(0, 0, 0, 0), pml_order=3.0, pml_sigma_max=(0.0, 0.0), pml_alpha=0.05,
                 k_mon=None, design=None, eps_bg=1.0, eps_hi=6.25, eps=None, axis=0):
        self.r_in, self.nr, self.nphi, self.nz = float(r_in), int(nr), int(nphi), int(nz)
        self.n_fold, self.m = int(n_fold), int(m)
        self.dr, self.dz, self.courant = float(dr), float(dz), float(courant)
        self.pml = tuple(int(x) for x in pml)
        self.k_mon = k_mon
        self.design = design            # (k0, k1) or None
        self.eps_bg, self.eps_hi = float(eps_bg), float(eps_hi)
        self.axis = int(axis)
        p = _Params(self.r_in, self.dr, self.dz, self.courant, self.nr, self.nphi, self.nz,
                    self.n_fold, *self.pml, float(pml_order), float(pml_sigma_max[0]),
                    float(pml_sigma_max[1]), float(pml_alpha), self.axis)
        lib = _load()
        self._h = lib.ora_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle: bad zone parameters")
        self.dt = lib.ora_dt(self._h)
        # continuous zone (n_fold = 0, nphi = 1): dphi = tau = 1, seams 1 +- i m
        self.dphi = 2.0 * np.pi / (self.n_fold * self.nphi) if self.n_fold > 0 else 1.0
        self.tau = 2.0 * np.pi / self.n_fold if self.n_fold > 0 else 1.0
        self.shape = (self.nz, self.nr, self.nphi)
        self.eps = np.ones(self.shape, np.float32)
        if eps is not None:
            self.set_eps(eps)
        self.last = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().ora_destroy(h)
            self._h = None

    # -- state -----------------------------------------------------------
    def set_eps(self, eps, fp64=False):
        """Per-cell permittivity [nz][nr][nphi]; FP32 like the product's
        input unless fp64 (finite-difference checks)."""
        dt = np.float64 if fp64 else np.float32
        eps = np.ascontiguousarray(eps, dtype=dt).reshape(self.shape)
        self.eps = eps.copy()
        if fp64:
            _load().ora_set_eps64(self._h, _ptr(self.eps))
        else:
            _load().ora_set_eps(self._h, _ptr(self.eps))

    def set_design(self, rho, fp64=False):
        """eq. (6): eps = rho (eps_h - eps_0) + eps_0 inside the design layer."""
        k0, k1 = self.design
        eps = self.eps.astype(np.float64)
        rho = np.asarray(rho, dtype=np.float64).reshape(k1 - k0, self.nr, self.nphi)
        eps[k0:k1] = rho * (self.eps_hi - self.eps_bg) + self.eps_bg
        self.set_eps(eps, fp64=fp64)

    def reset(self):
        _load().ora_reset(self._h)

    def get_field(self, name):
        out = np.empty(self.shape, np.complex128)
        _load().ora_get_field(self._h, COMP[name], _ptr(out))
        return out

    def set_field(self, name, value):
        v = np.ascontiguousarray(value, dtype=np.complex128).reshape(self.shape)
        _load().ora_set_field(self._h, COMP[name], _ptr(v))

    def layer_rows(self):
        """(sigma, sigma~, c) at r integer, r half, z integer, z half points."""
        out = []
        for w in range(4):
            n = self.nr if w < 2 else self.nz
            sig = np.empty(n)
            sgt = np.empty(n)
            c = ctypes.c_double()
            _load().ora_get_layer(self._h, w, _ptr(sig), _ptr(sgt), ctypes.byref(c))
            out.append((sig, sgt, c.value))
        return out

    # -- sources ---------------------------------------------------------
    def preset_pattern(self, kind="plane_circ", m=None):
        """[2][nr][nphi] complex current pattern of the normally incident
        plane-wave component (|m| = 1) or of a radial sheet (m = 0)."""
        m = self.m if m is None else m
        phi_j = np.arange(self.nphi) * self.dphi
        phi_h = (np.arange(self.nphi) + 0.5) * self.dphi
        if self.n_fold == 0:            # continuous zone: every component at phi = 0
            phi_j = phi_h = np.zeros(self.nphi)
        pat = np.zeros((2, self.nr, self.nphi), np.complex128)
        if kind == "plane_circ":
            if abs(m) != 1:
                raise ValueError("plane_circ needs |m| = 1")
            pat[0] = -np.exp(1j * m * phi_j)[None, :] / self.dz
            pat[1] = -1j * np.sign(m) * np.exp(1j * m * phi_h)[None, :] / self.dz
        elif kind == "radial":
            if m != 0:
                raise ValueError("radial needs m = 0")
            pat[0] = -1.0 / self.dz
        else:
            raise ValueError(kind)
        return pat

    # -- runs --------------------------------------------------------------
    def run(self, nsteps, *, patterns=None, profiles=None, k_src=1, omegas=(), m=None,
            plane=True, volume=False, reset=True, n_start=0):
        """Time-step; returns dict with 'plane' [K][2][nr][nphi] and 'vol'
        [K][3][k1-k0][nr][nphi] DFTs (complex128)."""
        m = self.m if m is None else m
        if reset:
            self.reset()
        omegas = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, np.float64)))
        K = omegas.size
        P = 0
        pat = prof = None
        if patterns is not None:
            pat = np.ascontiguousarray(patterns, np.complex128).reshape(-1, 2, self.nr, self.nphi)
            P = pat.shape[0]
            prof = np.ascontiguousarray(np.asarray(profiles, np.complex128).reshape(P, nsteps))
        dplane = np.zeros((K, 2, self.nr, self.nphi), np.complex128) if (plane and K and self.k_mon is not None) else None
        dvol = None
        k0 = k1 = 0
        if volume and K:
            k0, k1 = self.design
            dvol = np.zeros((K, 3, k1 - k0, self.nr, self.nphi), np.complex128)
        rc = _load().ora_run(self._h, int(m), int(nsteps), int(n_start), P, _ptr(pat), _ptr(prof),
                             int(k_src), K, _ptr(omegas),
                             int(self.k_mon if self.k_mon is not None else 0), _ptr(dplane),
                             int(k0), int(k1), _ptr(dvol))
        if rc != 0:
            raise ValueError("oracle: bad run arguments")
        return {"plane": dplane, "vol": dvol, "omegas": omegas}

    def forward(self, nsteps, omegas, *, omega_c, width, n0=None, k_src, kind="plane_circ",
                volume=False):
        """Forward run with the preset soft pulsed source; remembers what the
        adjoint needs."""
        g, n0 = pulse(nsteps, self.dt, omega_c, width, n0)
        out = self.run(nsteps, patterns=self.preset_pattern(kind)[None], profiles=g[None],
                       k_src=k_src, omegas=omegas, volume=volume)
        self.last = dict(out, nsteps=nsteps, width=width, n0=n0)
        return out

    # -- adjoint -------------------------------------------------------------
    def stretched_volume(self, omega):
        """W(alpha, .) = R l_r l_z dphi at the three E points: the complex
        cell volume r (1 + sigma~ F)(1 + sigma_r F)(1 + sigma_z F) dr dphi dz,
        F(w) = dt / (1 - c e^{i w dt}).  Returns ([3][nr], [3][nz]) factors."""
        (sri, gri, cr), (srh, grh, _), (szi, _, cz), (szh, _, _) = self.layer_rows()
        e = np.exp(1j * omega * self.dt)
        Fr = self.dt / (1.0 - cr * e)
        Fz = self.dt / (1.0 - cz * e)
        r_int = self.r_in + np.arange(self.nr) * self.dr
        r_half = r_int + 0.5 * self.dr
        w_half = r_half * (1 + grh * Fr) * (1 + srh * Fr)
        w_int = r_int * (1 + gri * Fr) * (1 + sri * Fr)
        wr = np.stack([w_half, w_int, w_int])
        wz = np.stack([1 + szi * Fz, 1 + szi * Fz, 1 + szh * Fz])
        return wr * (self.dr * self.dphi * self.dz), wz

    def adjoint_grad(self, dFdE, *, adj_width=None, adj_n0=None):
        """dF/drho over the design layer from dF/dEhat on the monitor plane
        ([K][2][nr][nphi] Wirtinger derivative).  Needs a forward run with
        the volume DFT."""
        last = self.last
        if last is None or last["vol"] is None:
            raise RuntimeError("oracle: forward run with the volume DFT required")
        T, omegas = last["nsteps"], last["omegas"]
        K = omegas.size
        width = last["width"] if adj_width is None else adj_width
        n0 = last["n0"] if adj_n0 is None else adj_n0
        wt = wtilde(omegas, self.dt)
        g = np.asarray(dFdE, np.complex128).reshape(K, 2, self.nr, self.nphi)
        pats = np.zeros((K, 2, self.nr, self.nphi), np.complex128)
        km = self.k_mon
        for k in range(K):
            wr, wz = self.stretched_volume(omegas[k])
            for a in range(2):
                Wp = wr[a][:, None] * wz[a][km]
                pats[k, a] = g[k, a] / (Wp * 1j * wt[k])
        # broadband profiles: pulses centred on each w_l, then P^{-1} mixing
        p = np.stack([pulse(T, self.dt, omegas[l], width, n0)[0] for l in range(K)])
        th = (np.arange(T) + 0.5) * self.dt
        Pm = np.array([[self.dt * np.sum(p[l] * np.exp(1j * omegas[k] * th)) for l in range(K)]
                       for k in range(K)])
        C = np.linalg.inv(Pm)
        q = np.einsum("lk,ln->kn", C, p)
        adj = self.run(T, patterns=pats, profiles=q, k_src=km, omegas=omegas, m=-self.m,
                       plane=False, volume=True)
        X, E = adj["vol"], last["vol"]
        k0, k1 = self.design
        grad_eps = np.zeros((k1 - k0, self.nr, self.nphi))
        for k in range(K):
            wr, wz = self.stretched_volume(omegas[k])
            for a in range(3):
                Wp = wr[a][None, :, None] * wz[a][k0:k1][:, None, None]
                grad_eps += 2.0 * np.real(wt[k] ** 2 * Wp * X[k, a] * E[k, a])
        return (self.eps_hi - self.eps_bg) * grad_eps
