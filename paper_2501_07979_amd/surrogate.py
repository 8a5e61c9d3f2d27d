"""Design surrogate: a dilated convolutional network that maps a zone's
design-layer pattern to its complex exit-plane DFT fields, so that inner
design iterations can run on it; the FDTD (libzda) generates its training
samples and stays the fallback and the arbiter, re-checking every k-th
iterate (checked_loop).

Every layer runs on the hand-written gfx950 kernels of libzsur.so (BF16 MFMA
GEMM with FP32 accumulation, im2col/col2im, activation gradient, MSE, Adam);
torch tensors only hold device memory.  Activations are channel-major
[C][B][H][W] (H = r rows, W = phi columns).  Convolutions are 3x3 with
dilation d, periodic in phi and zero-padded in r; the targets are the fields
with the Bloch phase removed (u = E e^{-i m phi}), which are phi-periodic, so
the periodic padding matches them.

The pattern is two-dimensional, extruded through the design layer (the
paper's zones are patterned with pillars that run through the layer); the
fields are the exit-plane E_r and E_phi at every DFT frequency.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
EXPORTS = ["zsur_gemm", "zsur_im2col", "zsur_col2im", "zsur_act_grad", "zsur_rowsum", "zsur_mse", "zsur_to_bf16",
           "zsur_adam", "zsur_last_error"]
ACT_NONE, ACT_LEAKY = 0, 1
_lib = None


class ZsurError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("zsur status %d: %s" % (status, msg))
        self.status = status


def load():
    """Load libzsur.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(HERE, "libzsur.so")
    if not os.path.exists(path):
        raise RuntimeError("libzsur.so is not built (run paper_2501_07979_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, I, L, F, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_float, ctypes.c_size_t
    lib.zsur_gemm.argtypes = [I, I, I, P, L, L, P, L, L, P, L, P, P, I, F, I, P, P]
    lib.zsur_im2col.argtypes = [P, I, I, I, I, I, P, P]
    lib.zsur_col2im.argtypes = [P, I, I, I, I, I, P, P]
    lib.zsur_act_grad.argtypes = [P, P, P, P, S, F, P]
    lib.zsur_rowsum.argtypes = [P, I, I, P, P, P]
    lib.zsur_mse.argtypes = [P, P, S, P, P, P, P]
    lib.zsur_to_bf16.argtypes = [P, P, S, P]
    lib.zsur_adam.argtypes = [P, P, P, P, S, F, F, F, F, I, P, P]
    lib.zsur_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ck(st):
    if st != 0:
        raise ZsurError(st, load().zsur_last_error().decode())


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _Layer:
    def __init__(self, cin, cout, k, dil, act, rng, device):
        import torch
        self.cin, self.cout, self.k, self.dil, self.act = cin, cout, k, dil, act
        fan_in = cin * k * k
        bound = np.sqrt(6.0 / fan_in) * (1.0 if act else 0.5)
        w = rng.uniform(-bound, bound, (cout, fan_in)).astype(np.float32)
        self.w = torch.tensor(w, device=device)
        self.b = torch.zeros(cout, dtype=torch.float32, device=device)
        self.wb = torch.empty((cout, fan_in), dtype=torch.int16, device=device)
        _ck(load().zsur_to_bf16(_p(self.w), _p(self.wb), self.w.numel(), _stream()))
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)


class Surrogate:
    """in_ch -> 3x3 conv (act) -> 3x3 dilated convs (act) -> 1x1 conv -> out_ch."""

    def __init__(self, in_ch=2, width=48, out_ch=12, dilations=(1, 2, 4, 8, 1, 2, 4, 8), slope=0.1, seed=0,
                 device="cuda"):
        rng = np.random.default_rng(seed)
        self.slope = float(slope)
        self.device = device
        self.layers = [_Layer(in_ch, width, 3, 1, True, rng, device)]
        for d in dilations:
            self.layers.append(_Layer(width, width, 3, d, True, rng, device))
        self.layers.append(_Layer(width, out_ch, 1, 1, False, rng, device))
        self.in_ch, self.out_ch = in_ch, out_ch
        self.t = 0
        self._cache = None
        self._work = None

    def n_params(self):
        return sum(l.w.numel() + l.b.numel() for l in self.layers)

    # ---- forward / backward
    def forward(self, x, keep=False):
        """x: FP32 [in_ch][B][H][W] on the device -> FP32 [out_ch][B][H][W]."""
        import torch
        lib = load()
        _, B, H, W = x.shape
        N = B * H * W
        s = _stream()
        cache = []
        h = x.contiguous()
        hb = None
        for l in self.layers:
            y = torch.empty((l.cout, B, H, W), dtype=torch.float32, device=x.device)
            yb = torch.empty((l.cout, B, H, W), dtype=torch.int16, device=x.device)
            if l.k == 3:
                cols = torch.empty((l.cin * 9, N), dtype=torch.int16, device=x.device)
                _ck(lib.zsur_im2col(_p(h), l.cin, B, H, W, l.dil, _p(cols), s))
                K = l.cin * 9
            else:
                if hb is None:
                    hb = torch.empty_like(h, dtype=torch.int16)
                    _ck(lib.zsur_to_bf16(_p(h), _p(hb), h.numel(), s))
                cols = hb
                K = l.cin
            _ck(lib.zsur_gemm(l.cout, N, K, _p(l.wb), K, 1, _p(cols), N, 1, _p(y), N, _p(yb), _p(l.b),
                              ACT_LEAKY if l.act else ACT_NONE, self.slope, 1, None, s))
            if keep:
                cache.append((h, cols, y))
            h, hb = y, yb
        self._cache = (cache, (B, H, W)) if keep else None
        return h

    def backward(self, dy, need_dx=False):
        """dy: FP32 d(loss)/d(output); fills every layer's gw, gb and returns
        d(loss)/d(input) when need_dx."""
        import torch
        lib = load()
        assert self._cache is not None, "forward(keep=True) first"
        cache, (B, H, W) = self._cache
        N = B * H * W
        s = _stream()
        g = dy.contiguous()
        dx = None
        for li in range(len(self.layers) - 1, -1, -1):
            l = self.layers[li]
            h, cols, y = cache[li]
            dz = torch.empty_like(g)
            dzb = torch.empty(g.shape, dtype=torch.int16, device=g.device)
            _ck(lib.zsur_act_grad(_p(y), _p(g), _p(dz), _p(dzb), g.numel(), self.slope if l.act else 1.0, s))
            K = l.cin * (9 if l.k == 3 else 1)
            # split-K over pixels: about 1024 blocks, at least 256 pixels per slice
            tiles = ((l.cout + 63) // 64) * ((K + 63) // 64)
            split = int(max(1, min((1024 + tiles - 1) // tiles, N // 256)))
            need = max(split * l.cout * K, 64 * l.cout)
            if self._work is None or self._work.numel() < need:
                self._work = torch.empty(need, dtype=torch.float32, device=g.device)
            _ck(lib.zsur_rowsum(_p(dz), l.cout, N, _p(l.gb), _p(self._work), s))
            # dW[co][kk] = sum_n dZ[co][n] cols[kk][n]
            _ck(lib.zsur_gemm(l.cout, K, N, _p(dzb), N, 1, _p(cols), 1, N, _p(l.gw), K, None, None, ACT_NONE, 1.0,
                              split, _p(self._work), s))
            if li == 0 and not need_dx:
                break
            # dcols[kk][n] = sum_co W[co][kk] dZ[co][n]
            dcols = torch.empty((K, N), dtype=torch.float32, device=g.device)
            _ck(lib.zsur_gemm(K, N, l.cout, _p(l.wb), 1, K, _p(dzb), N, 1, _p(dcols), N, None, None, ACT_NONE, 1.0,
                              1, None, s))
            if l.k == 3:
                gin = torch.empty((l.cin, B, H, W), dtype=torch.float32, device=g.device)
                _ck(lib.zsur_col2im(_p(dcols), l.cin, B, H, W, l.dil, _p(gin), s))
            else:
                gin = dcols.view(l.cin, B, H, W)
            g = gin
            if li == 0:
                dx = gin
        return dx

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        lib = load()
        s = _stream()
        self.t += 1
        for l in self.layers:
            _ck(lib.zsur_adam(_p(l.w), _p(l.gw), _p(l.mw), _p(l.vw), l.w.numel(), lr, b1, b2, eps, self.t,
                              _p(l.wb), s))
            _ck(lib.zsur_adam(_p(l.b), _p(l.gb), _p(l.mb), _p(l.vb), l.b.numel(), lr, b1, b2, eps, self.t, None,
                              s))

    def mse(self, pred, target):
        """(loss tensor [1], d(loss)/d(pred)) for the mean squared error."""
        import torch
        d = torch.empty_like(pred)
        loss = torch.empty(1, dtype=torch.float32, device=pred.device)
        partial = torch.empty(1024, dtype=torch.float32, device=pred.device)
        _ck(load().zsur_mse(_p(pred), _p(target.contiguous()), pred.numel(), _p(d), _p(loss), _p(partial),
                            _stream()))
        return loss, d


# ---- zone <-> network representation

def features(rho2d, nr, device="cuda"):
    """Network input for a batch of 2-D patterns rho2d [B][nr][nphi]: channel 0
    the pattern, channel 1 the normalised radial index."""
    import torch
    rho2d = torch.as_tensor(rho2d, dtype=torch.float32, device=device)
    B, _, nphi = rho2d.shape
    rr = (torch.arange(nr, dtype=torch.float32, device=device) / max(nr - 1, 1) - 0.5)
    x = torch.empty((2, B, nr, nphi), dtype=torch.float32, device=device)
    x[0] = rho2d
    x[1] = rr[None, :, None].expand(B, nr, nphi)
    return x


def bloch_phases(wl):
    """e^{-i m phi} at the E_r (phi_j) and E_phi (phi_{j+1/2}) sample points."""
    tau = 2 * np.pi / wl.n_fold
    dphi = tau / wl.nphi
    j = np.arange(wl.nphi)
    return np.exp(-1j * wl.m * j * dphi), np.exp(-1j * wl.m * (j + 0.5) * dphi)


def plane_to_targets(plane, wl):
    """Exit-plane DFT [K][2][nr][nphi] complex -> 4K real channels
    [Re u_r, Im u_r, Re u_phi, Im u_phi per frequency] with u = E e^{-i m phi}."""
    pr, pp = bloch_phases(wl)
    plane = np.asarray(plane)
    out = []
    for k in range(plane.shape[0]):
        ur, up = plane[k, 0] * pr[None, :], plane[k, 1] * pp[None, :]
        out += [ur.real, ur.imag, up.real, up.imag]
    return np.stack(out).astype(np.float32)


def targets_to_plane(t, wl):
    """Inverse of plane_to_targets (numpy, complex128)."""
    pr, pp = bloch_phases(wl)
    t = np.asarray(t, dtype=np.float64)
    K = t.shape[0] // 4
    plane = np.empty((K, 2, t.shape[1], t.shape[2]), np.complex128)
    for k in range(K):
        plane[k, 0] = (t[4 * k] + 1j * t[4 * k + 1]) / pr[None, :]
        plane[k, 1] = (t[4 * k + 2] + 1j * t[4 * k + 3]) / pp[None, :]
    return plane


def random_patterns(n, nr, nphi, seed, sigma=2.5, beta=6.0):
    """Seeded smoothed 2-D patterns in [0, 1] (periodic in phi), the kind of
    grey density an optimiser passes through."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    out = np.empty((n, nr, nphi), np.float32)
    for q in range(n):
        f = gaussian_filter(rng.random((nr, nphi)), sigma=sigma, mode=("reflect", "wrap"))
        f = (f - f.mean()) / max(f.std(), 1e-12)
        out[q] = (0.5 + 0.5 * np.tanh(beta * 0.25 * f)).astype(np.float32)
    return out


def generate_samples(wl, patterns, zones_per_batch=32, log=None):
    """FDTD exit-plane fields of every pattern (extruded through the design
    layer), run as batches of zones of the workload's geometry on the batched
    two-step kernel."""
    import torch
    from . import lens, zda
    n = len(patterns)
    nd = wl.design[1] - wl.design[0]
    zb = min(zones_per_batch, n)
    zones = [zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps()) for _ in range(zb)]
    batch = zda.Batch(zones)
    lens.set_family(batch, lens.FLAT if lens.is_narrow(wl) else lens.TWO_STEP, [wl] * zb)
    src = zda.preset_source(k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    out = np.empty((n, 4 * len(wl.omegas), wl.nr, wl.nphi), np.float32)
    for q0 in range(0, n, zb):
        qs = list(range(q0, min(n, q0 + zb)))
        for z, q in zip(zones, qs):
            z.set_design(np.repeat(patterns[q][None], nd, axis=0))
        batch.run([src] * len(zones), wl.steps, wl.omegas)
        for z, q in zip(zones, qs):
            out[q] = plane_to_targets(z.dft(zda.MON_PLANE).cpu().numpy(), wl)
        if log:
            log("samples %d/%d" % (qs[-1] + 1, n))
    torch.cuda.synchronize()
    batch.close()
    for z in zones:
        z.close()
    return out


def train(net, X, T, iters, batch=16, lr=2e-3, lr_end=2e-4, seed=0, log=None):
    """Adam on the MSE between net(X) and T (device tensors, samples along
    dimension 1), with a geometric learning-rate decay."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[1]
    losses = []
    for it in range(iters):
        idx = torch.as_tensor(rng.choice(n, size=min(batch, n), replace=False), device=X.device)
        xb = X[:, idx].contiguous()
        tb = T[:, idx].contiguous()
        y = net.forward(xb, keep=True)
        loss, d = net.mse(y, tb)
        net.backward(d)
        net.adam_step(lr * (lr_end / lr) ** (it / max(iters - 1, 1)))
        if it % 50 == 0 or it == iters - 1:
            losses.append((it, float(loss.item())))
            if log:
                log("train it %d loss %.4e" % losses[-1])
    return losses


def field_errors(net, X, T, wl, scale):
    """Relative L2 error of the predicted complex exit-plane fields per sample."""
    errs = []
    for q in range(X.shape[1]):
        y = net.forward(X[:, q:q + 1].contiguous()).cpu().numpy()[:, 0] * scale
        t = T[:, q].cpu().numpy() * scale
        a, b = targets_to_plane(y, wl), targets_to_plane(t, wl)
        errs.append(float(np.linalg.norm(a - b) / np.linalg.norm(b)))
    return np.array(errs)


def bench_train(steps=60, batch=16, width=48, size=64, seed=0):
    """Times training steps of the surrogate on seeded random data of the
    design-zone shape (2 input channels, 12 outputs, size x size)."""
    import torch
    rng = np.random.default_rng(seed)
    X = torch.tensor(rng.standard_normal((2, batch * 4, size, size)).astype(np.float32), device="cuda")
    T = torch.tensor(rng.standard_normal((12, batch * 4, size, size)).astype(np.float32), device="cuda")
    net = Surrogate(in_ch=2, width=width, out_ch=12, seed=1)
    train(net, X, T, 5, batch=batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    train(net, X, T, steps, batch=batch)
    torch.cuda.synchronize()
    return {"params": net.n_params(), "batch": batch, "ms_per_step": 1e3 * (time.perf_counter() - t0) / steps}


# ---- surrogate-assisted design against plain FDTD-adjoint design at equal
# final focusing efficiency

def adam_update(x, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam ascent step on x along g (torch, in place), clipped to [0, 1]."""
    import torch
    m.mul_(b1).add_(g, alpha=1 - b1)
    v.mul_(b2).addcmul_(g, g, value=1 - b2)
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    x.add_(lr * mh / (torch.sqrt(vh) + eps)).clamp_(0.0, 1.0)


def checked_loop(fdtd, sur, rho0, outer, inner, lr, stop=None, log=None):
    """Surrogate-assisted ascent with the FDTD as fallback and arbiter.

    fdtd(rho) -> (F, dF/drho) is the plain FDTD-adjoint evaluation and
    sur(rho) -> dF/drho the surrogate's gradient.  Each outer step re-checks
    the current pattern with the FDTD.  After a block of surrogate steps the
    re-check accepts the pattern only if F did not fall below the last
    accepted one; otherwise the block is rejected: the loop returns to the
    last accepted pattern (and its Adam moments) and falls back to plain
    FDTD-adjoint steps for 1, 2, 4, ... outer steps (doubling while blocks
    keep failing).  A pattern reached by a plain step is always accepted, as
    in plain design.  Every outer step takes one Adam step along the FDTD
    gradient, then (outside the fall-back) `inner` along the surrogate's.
    stop(step, rho, F) is asked after each accepted re-check.  Returns the
    last accepted pattern, its F and the per-outer-step history."""
    import torch
    rho = rho0.clone()
    m, v = torch.zeros_like(rho), torch.zeros_like(rho)
    t = 0
    best = None          # (rho, F, grad, m, v, t) of the last accepted re-check
    hist = []
    block = False        # the steps since the last re-check include surrogate steps
    wait, gap = 0, 1
    for s in range(outer):
        F, g = fdtd(rho)
        accepted = best is None or not block or F >= best[1]
        if accepted:
            best = (rho.clone(), F, g, m.clone(), v.clone(), t)
            if block:
                gap = 1
        else:
            rho, F, g = best[0].clone(), best[1], best[2]
            m, v, t = best[3].clone(), best[4].clone(), best[5]
            wait, gap = gap, gap * 2
        hist.append({"step": s, "F_fdtd": float(F), "surrogate_block": bool(block), "accepted": bool(accepted)})
        if log:
            log("outer %d F %.5e %s" % (s, F, ("accept" if accepted else "reject, back to the last accepted") +
                                           (" (surrogate block)" if block else "")))
        if accepted and stop is not None and stop(s, rho, F):
            break
        t += 1
        adam_update(rho, g, m, v, t, lr)
        if wait > 0 or inner == 0:
            wait = max(wait - 1, 0)
            block = False
        else:
            for _ in range(inner):
                t += 1
                adam_update(rho, sur(rho), m, v, t, lr)
            block = True
    return best[0], best[1], hist


def incident_power(wl):
    """Incident power of the preset source per frequency: the power its plane
    wave carries through the active ring, from a run of the zone filled with
    the substrate everywhere (nothing reflects it)."""
    from . import objective, zda
    eps = np.full((wl.nz, wl.nr, wl.nphi), wl.eps_sub, np.float32)
    z = zda.Zone(zda.default_desc(**wl.desc_kwargs()), eps)
    z.run(wl.steps, wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
    plane = z.dft(zda.MON_PLANE).cpu().numpy()
    z.close()
    return objective.exit_plane_power(plane, wl, index=float(np.sqrt(wl.eps_sub)))


def mean_efficiency(plane, wl, focal, p_inc):
    """Absolute focusing efficiency averaged over the frequencies."""
    from . import objective
    return float(np.mean(objective.focusing_efficiency(plane, wl, wl.omegas, focal, p_inc, n_rho=64,
                                                       n_phi=4)["absolute"]))


def fdtd_value_and_grad(zone, wl, weights):
    """fdtd(rho2d) for checked_loop: forward run, focal objective, adjoint
    run (torch.autograd through the zone) -> (F, dF/drho2d, exit plane)."""
    import torch
    from .autograd import zone_fdtd
    nd = wl.design[1] - wl.design[0]
    Wt = torch.as_tensor(weights, dtype=torch.complex64, device="cuda")

    def f(rho2d):
        r = rho2d.detach().clone().requires_grad_(True)
        plane = zone_fdtd(r[None].expand(nd, wl.nr, wl.nphi).contiguous(), zone, nsteps=wl.steps,
                          omegas=wl.omegas, k_src=wl.k_src, omega_c=wl.omega_c, width=wl.width)
        a = (Wt * plane).sum(dim=(1, 2, 3))
        F = (a.abs() ** 2).sum()
        F.backward()
        f.last_plane = plane.detach()
        return float(F.item()), r.grad.detach()
    f.last_plane = None
    return f


def surrogate_grad(net, wl, weights, scale):
    """sur(rho2d) for checked_loop: dF/drho2d of the focal objective on the
    network's predicted fields (network backward on its own kernels)."""
    import torch
    Wt = torch.as_tensor(weights, dtype=torch.complex64, device="cuda")
    pr, pp = bloch_phases(wl)
    ph = torch.as_tensor(np.stack([1 / pr, 1 / pp]), dtype=torch.complex64, device="cuda")
    K = len(wl.omegas)

    def g(rho2d):
        x = features(rho2d[None], wl.nr)
        y = net.forward(x, keep=True)
        yv = y[:, 0].detach().clone().requires_grad_(True)
        u = torch.complex(yv[0::2], yv[1::2]).view(K, 2, wl.nr, wl.nphi) * scale
        a = (Wt * (u * ph[None, :, None, :])).sum(dim=(1, 2, 3))
        (a.abs() ** 2).sum().backward()
        dx = net.backward(yv.grad.contiguous()[:, None], need_dx=True)
        return dx[0, 0].detach().clone()
    return g


def plain_to_target(fd, wl, rho0, lr, iters, target, focal, p_inc):
    """Plain FDTD-adjoint Adam from rho0 at learning rate lr until an iterate
    is within 1 % of the target efficiency (or iters updates): (FDTD
    evaluations, seconds excluding the efficiency evaluations, reached)."""
    import torch
    rho = torch.tensor(rho0, device="cuda")
    m, v = torch.zeros_like(rho), torch.zeros_like(rho)
    t = 0.0
    for it in range(iters + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, g = fd(rho)
        torch.cuda.synchronize()
        t += time.perf_counter() - t0
        if mean_efficiency(fd.last_plane.cpu(), wl, focal, p_inc) >= 0.99 * target:
            return it + 1, t, True
        t0 = time.perf_counter()
        if it < iters:
            adam_update(rho, g, m, v, it + 1, lr)
        torch.cuda.synchronize()
        t += time.perf_counter() - t0
    return iters + 1, t, False


def equal_efficiency_comparison(wl, plain_iters=24, outer_max=48, inner=9, lr=0.02, n_train=256, train_iters=1500,
                                width=160, batch=8, seed=7, plain_lrs=(0.05, 0.1), log=None):
    """Plain FDTD-adjoint design against surrogate-assisted design from the
    same start, compared at equal final focusing efficiency.

    Plain: `plain_iters` Adam iterations on the 2-D pattern (one forward and
    one adjoint run each); its final absolute focusing efficiency is the
    target, and its own time to the target is that of the first iterate
    within 1 % of it; the plain path also runs at the learning rates of
    plain_lrs to the same target.  Surrogate: the network (about 2M
    parameters at width 160) is trained once on n_train seeded random
    patterns and their FDTD fields, then checked_loop runs from the same
    start (FDTD re-check and gradient every inner + 1 iterations) at the same
    learning rates until an accepted pattern's efficiency reaches the target
    within 1 % or outer_max re-checks pass.  Wall-clock times exclude the
    efficiency evaluations (measurement only).  Returns a dict of all runs
    and of the fastest of each side."""
    import torch
    from . import objective, zda
    focal = objective.focal_length(wl.r_in + 0.5 * wl.nr * wl.dr)
    W = objective.focal_weights(wl, np.array(wl.omegas), focal).cpu().numpy()
    p_inc = incident_power(wl)
    rho0 = random_patterns(1, wl.nr, wl.nphi, seed=seed)[0]
    zone = zda.Zone(zda.default_desc(**wl.desc_kwargs()), wl.eps())
    fd = fdtd_value_and_grad(zone, wl, W)
    # ---- plain: pattern q is evaluated by the q-th FDTD-adjoint call
    # (q = 0 .. plain_iters); cum[q] is the time spent up to and with it
    rho = torch.tensor(rho0, device="cuda")
    m, v = torch.zeros_like(rho), torch.zeros_like(rho)
    planes, cum, t_plain = [], [], 0.0
    for it in range(plain_iters + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, g = fd(rho)
        if it < plain_iters:
            adam_update(rho, g, m, v, it + 1, lr)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        cum.append(t_plain)
        planes.append(fd.last_plane.cpu())
    F_end = F
    effs = [mean_efficiency(p, wl, focal, p_inc) for p in planes]
    eff_start, eff_plain = effs[0], effs[-1]
    target = eff_plain
    q_reach = next(q for q, e in enumerate(effs) if e >= 0.99 * target)
    if log:
        log("plain: %d iterations, %.2f s, efficiency %.4f -> %.4f (within 1 %% after %d, %.2f s)"
            % (plain_iters, t_plain, eff_start, eff_plain, q_reach, cum[q_reach]))
    # the plain path at larger learning rates, to the same target
    sweep = []
    for lr_p in plain_lrs:
        n_ev, t_ev, ok = plain_to_target(fd, wl, rho0, lr_p, plain_iters, target, focal, p_inc)
        sweep.append({"lr": lr_p, "fdtd_evaluations_to_target": n_ev, "s_to_target": round(t_ev, 3),
                      "reached": bool(ok)})
        if log:
            log("plain at lr %.3f: %s after %d evaluations, %.2f s" % (lr_p, "reached" if ok else "not reached",
                                                                       n_ev, t_ev))
    # ---- offline training set and training
    t0 = time.perf_counter()
    pats = random_patterns(n_train, wl.nr, wl.nphi, seed=seed + 1)
    T = generate_samples(wl, pats)
    t_gen = time.perf_counter() - t0
    scale = float(np.abs(T).std())
    nh = max(8, n_train // 8)
    X = features(pats, wl.nr)
    Tt = torch.tensor(np.ascontiguousarray(np.moveaxis(T / scale, 0, 1)), device="cuda")
    net = Surrogate(in_ch=2, width=width, out_ch=4 * len(wl.omegas), seed=seed)
    t0 = time.perf_counter()
    losses = train(net, X[:, :-nh].contiguous(), Tt[:, :-nh].contiguous(), train_iters, batch=batch, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    errs = field_errors(net, X[:, -nh:].contiguous(), Tt[:, -nh:].contiguous(), wl, scale)
    if log:
        log("surrogate: %d params, %d samples (%.1f s), trained %.1f s, held-out field error median %.3f p90 %.3f"
            % (net.n_params(), n_train, t_gen, t_train, np.median(errs), np.percentile(errs, 90)))
    # ---- assisted, at the learning rate of the reference plain run and at
    # the sweep's: the best of each side is compared with the best of the other
    sur = surrogate_grad(net, wl, W, scale)
    runs = [assisted_to_target(fd, sur, wl, rho0, r, outer_max, inner, target, focal, p_inc, log)
            for r in (lr,) + tuple(plain_lrs)]
    zone.close()
    plain_runs = [{"lr": lr, "fdtd_evaluations_to_target": q_reach + 1, "s_to_target": round(cum[q_reach], 3),
                   "reached": True}] + sweep
    best_p = min((e for e in plain_runs if e["reached"]), key=lambda e: e["s_to_target"])
    done = [a for a in runs if a["reached_target_within_1pct"]]
    best_a = min(done, key=lambda a: a["s"]) if done else None
    return {
        "workload": wl.name, "steps_per_run": wl.steps,
        "efficiency_definition": "absolute: focal-plane power within 3 FWHM of the spot centre / incident power",
        "target_efficiency": round(target, 5),
        "plain": {"iterations": plain_iters, "learning_rate": lr, "s": round(t_plain, 3),
                  "iters_per_s": round((plain_iters + 1) / t_plain, 4),
                  "efficiency_start": round(eff_start, 5), "efficiency_end": round(eff_plain, 5),
                  "efficiency_per_iteration": [round(e, 5) for e in effs], "F_end": round(F_end, 5),
                  "to_target": plain_runs, "best": best_p},
        "surrogate": {"params": net.n_params(), "patch": [wl.nr, wl.nphi], "train_samples": n_train - nh,
                      "held_out": nh, "sample_s": round(t_gen, 2), "train_s": round(t_train, 2),
                      "train_loss_end": losses[-1][1],
                      "field_err_median": round(float(np.median(errs)), 4),
                      "field_err_p90": round(float(np.percentile(errs, 90)), 4)},
        "assisted": {"to_target": runs, "best": best_a},
        # the fastest run of each side to the target (the assisted one counted
        # without and with its one-off training set and training)
        "speedup_online_best": round(best_p["s_to_target"] / best_a["s"], 4) if best_a else None,
        "speedup_with_training_best": round(best_p["s_to_target"] / (best_a["s"] + t_gen + t_train), 4)
                                      if best_a else None,
    }


def assisted_to_target(fd, sur, wl, rho0, lr, outer_max, inner, target, focal, p_inc, log=None):
    """checked_loop from rho0 at learning rate lr until an accepted pattern
    is within 1 % of the target efficiency (or outer_max re-checks); the
    time excludes the efficiency evaluations."""
    import torch
    state = {"t": 0.0, "eff": 0.0, "reached": False}
    clock = [time.perf_counter()]

    def stop(step, r, F):
        torch.cuda.synchronize()
        state["t"] += time.perf_counter() - clock[0]
        e = mean_efficiency(fd.last_plane.cpu(), wl, focal, p_inc)
        state["eff"] = e
        done = e >= 0.99 * target
        state["reached"] = state["reached"] or done
        if log:
            log("assisted lr %.3f re-check %d: F %.4e efficiency %.4f (target %.4f)" % (lr, step, F, e, target))
        clock[0] = time.perf_counter()
        return done

    torch.cuda.synchronize()
    clock[0] = time.perf_counter()
    _, F_best, hist = checked_loop(fd, sur, torch.tensor(rho0, device="cuda"), outer_max, inner, lr, stop=stop)
    torch.cuda.synchronize()
    if not state["reached"]:
        state["t"] += time.perf_counter() - clock[0]
    n_sur = sum(inner for h in hist if h["surrogate_block"])
    return {"lr": lr, "fdtd_rechecks": len(hist), "surrogate_iterations": n_sur, "s": round(state["t"], 3),
            "iters_per_s": round((len(hist) + n_sur) / max(state["t"], 1e-9), 4),
            "efficiency_end": round(state["eff"], 5), "F_end": round(F_best, 5),
            "reached_target_within_1pct": bool(state["reached"]),
            "F_accepted": [round(h["F_fdtd"], 4) for h in hist if h["accepted"]],
            "accepted_surrogate_blocks": sum(1 for h in hist if h["surrogate_block"] and h["accepted"]),
            "rejected_surrogate_blocks": sum(1 for h in hist if h["surrogate_block"] and not h["accepted"])}

if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="design-surrogate training benchmark")
    ap.add_argument("--bench-train", type=int, default=60, help="timed training steps")
    ap.add_argument("--batch", type=int, default=16)
    args = ap.parse_args()
    print(json.dumps(bench_train(args.bench_train, args.batch)))
