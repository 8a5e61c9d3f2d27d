"""ctypes binding of libzda.so (include/zda.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch is used for
device buffers and the current stream.  Importing this module loads the
library (which needs no GPU to load); any call that touches the GPU raises
if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzda.so")

ZDA_OK, ZDA_ERR_ARG, ZDA_ERR_CFL, ZDA_ERR_UNSUPPORTED, ZDA_ERR_OOM, ZDA_ERR_STATE, ZDA_ERR_HIP, ZDA_ERR_DIVERGED = range(8)
ZDA_MAX_FREQ = 8
SRC_PLANE_CIRC, SRC_RADIAL, SRC_CUSTOM = 0, 1, 2
DFT_PLANE, DFT_VOLUME, RUN_CONTINUE, RUN_TIMING = 1, 2, 4, 8
MON_PLANE, MON_VOLUME, MON_ADJOINT_VOLUME = 0, 1, 2
OPT_XCD_REMAP, OPT_NT_STORES, OPT_LAYER_STREAM, OPT_TILE_PATCH, OPT_LAYER_KCHUNK, OPT_WATCHDOG = 1, 2, 3, 4, 5, 6
OPT_LAYER_CARRY = 7
COMP_R, COMP_PHI, COMP_Z = 1, 2, 4
COMP = {"Er": 0, "Ephi": 1, "Ez": 2, "Hr": 3, "Hphi": 4, "Hz": 5}

EXPORTS = ["zda_set_allocator", "zda_zone_desc_default", "zda_zone_create", "zda_zone_destroy", "zda_zone_set_eps",
           "zda_zone_set_design", "zda_zone_set_stream", "zda_zone_sync", "zda_fdtd_run", "zda_fdtd_run_noalloc",
           "zda_fdtd_run_fp64", "zda_dft_fields",
           "zda_adjoint_grad",
           "zda_zone_read_field", "zda_zone_write_field", "zda_zone_release_fields", "zda_zone_acquire_fields",
           "zda_zone_fields_bytes",
           "zda_zone_get_info", "zda_zone_set_launch",
           "zda_zone_set_option",
           "zda_zone_last_timing", "zda_plan_two_step_tiles", "zda_batch_create", "zda_batch_destroy", "zda_batch_run",
           "zda_batch_adjoint_grad", "zda_batch_set_launch", "zda_batch_autotune",
           "zda_status_str", "zda_last_error"]


class ZoneDesc(ctypes.Structure):
    _fields_ = [("r_in", ctypes.c_double), ("nr", ctypes.c_int), ("nphi", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_fold", ctypes.c_int), ("m", ctypes.c_int), ("dr", ctypes.c_double), ("dz", ctypes.c_double),
                ("courant", ctypes.c_double), ("pml_r_in", ctypes.c_int), ("pml_r_out", ctypes.c_int),
                ("pml_z_lo", ctypes.c_int), ("pml_z_hi", ctypes.c_int), ("pml_order", ctypes.c_double),
                ("pml_sigma_max_r", ctypes.c_double), ("pml_sigma_max_z", ctypes.c_double),
                ("pml_alpha", ctypes.c_double), ("k_mon", ctypes.c_int), ("design_k0", ctypes.c_int),
                ("design_k1", ctypes.c_int), ("eps_bg", ctypes.c_double), ("eps_hi", ctypes.c_double),
                ("single_buffer", ctypes.c_int), ("axis", ctypes.c_int)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("k_src", ctypes.c_int), ("omega_c", ctypes.c_double),
                ("width", ctypes.c_double), ("n0", ctypes.c_int), ("n_profiles", ctypes.c_int),
                ("patterns", ctypes.c_void_p), ("patterns_on_device", ctypes.c_int),
                ("profiles", ctypes.c_void_p)]


class ZoneInfo(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_size_t), ("device_bytes", ctypes.c_size_t), ("dt", ctypes.c_double),
                ("cfl", ctypes.c_double), ("launch_chunks", ctypes.c_int), ("kchunk", ctypes.c_int),
                ("tile_rows", ctypes.c_int)]


class Timing(ctypes.Structure):
    _fields_ = [("h_launches", ctypes.c_int), ("e_launches", ctypes.c_int), ("h_ms", ctypes.c_double),
                ("e_ms", ctypes.c_double), ("steps_per_launch", ctypes.c_int), ("layer_launches", ctypes.c_int),
                ("layer_ms", ctypes.c_double), ("e_cells", ctypes.c_size_t), ("e_mon_cells", ctypes.c_size_t),
                ("e_src_cells", ctypes.c_size_t)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int), ("ms_per_step", ctypes.c_double), ("probes", ctypes.c_int)]


class ZdaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_status_name(status), status, msg))
        self.status = status


# zda_set_allocator's callback types: alloc(bytes, device, ctx) -> ptr,
# free(ptr, bytes, device, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)

_lib = None
# every callback pair ever registered stays alive: zones created while it was
# registered free their memory through it until they are destroyed
_allocators = []


def load():
    """Load libzda.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libzda.so is not built (run python paper_2501_07979_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.zda_zone_desc_default.argtypes = [ctypes.POINTER(ZoneDesc)]
    lib.zda_zone_desc_default.restype = None
    lib.zda_zone_create.argtypes = [ctypes.POINTER(ZoneDesc), P, I, ctypes.POINTER(P)]
    lib.zda_zone_destroy.argtypes = [P]
    lib.zda_zone_destroy.restype = None
    lib.zda_zone_set_eps.argtypes = [P, P, I]
    lib.zda_zone_set_design.argtypes = [P, P, I]
    lib.zda_zone_set_stream.argtypes = [P, P]
    lib.zda_zone_sync.argtypes = [P]
    lib.zda_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    lib.zda_fdtd_run.argtypes = [P, ctypes.POINTER(Source), I, P, I, I, P]
    lib.zda_fdtd_run_noalloc.argtypes = [P, ctypes.POINTER(Source), I, P, I, I, P]
    lib.zda_fdtd_run_fp64.argtypes = [P, P, I, ctypes.POINTER(Source), I, P, I, P, I, P]
    lib.zda_dft_fields.argtypes = [P, I, I, P, ctypes.c_size_t, I]
    lib.zda_adjoint_grad.argtypes = [P, P, I, P, I, D, P]
    lib.zda_zone_read_field.argtypes = [P, I, P, I]
    lib.zda_zone_write_field.argtypes = [P, I, P, I]
    lib.zda_zone_release_fields.argtypes = [P]
    lib.zda_zone_acquire_fields.argtypes = [P, P, ctypes.c_size_t]
    lib.zda_zone_fields_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.zda_zone_get_info.argtypes = [P, ctypes.POINTER(ZoneInfo)]
    lib.zda_zone_last_timing.argtypes = [P, ctypes.POINTER(Timing)]
    lib.zda_zone_set_launch.argtypes = [P, I, I]
    lib.zda_zone_set_option.argtypes = [P, I, I]
    lib.zda_plan_two_step_tiles.argtypes = [ctypes.POINTER(ZoneDesc), I, I, I, I, P, ctypes.c_size_t,
                                            ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.zda_batch_create.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(P)]
    lib.zda_batch_destroy.argtypes = [P]
    lib.zda_batch_destroy.restype = None
    lib.zda_batch_run.argtypes = [P, ctypes.POINTER(Source), I, P, I, I, P]
    lib.zda_batch_adjoint_grad.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), P]
    lib.zda_batch_set_launch.argtypes = [P, I, P]
    lib.zda_batch_autotune.argtypes = [P, ctypes.POINTER(Source), I, P, I, P, ctypes.POINTER(TuneResult)]
    lib.zda_status_str.argtypes = [I]
    lib.zda_status_str.restype = ctypes.c_char_p
    lib.zda_last_error.argtypes = []
    lib.zda_last_error.restype = ctypes.c_char_p
    for name in ("zda_set_allocator", "zda_zone_create", "zda_zone_set_eps", "zda_zone_set_design",
                 "zda_zone_set_stream", "zda_zone_sync", "zda_fdtd_run", "zda_fdtd_run_noalloc",
                 "zda_fdtd_run_fp64", "zda_dft_fields", "zda_adjoint_grad", "zda_zone_read_field",
                 "zda_zone_write_field", "zda_zone_get_info",
                 "zda_zone_last_timing", "zda_zone_set_launch", "zda_zone_set_option", "zda_batch_create",
                 "zda_batch_run", "zda_batch_adjoint_grad", "zda_batch_set_launch", "zda_batch_autotune"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def use_torch_allocator(on=True):
    """Back the device memory of zones and batches created from now on with
    torch's caching allocator (on=False restores hipMalloc / hipFree)."""
    lib = load()
    if not on:
        _check(lib.zda_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    torch = _torch()

    def _alloc(nbytes, device, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
        except RuntimeError:
            return None

    def _free(ptr, nbytes, device, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
    _check(lib.zda_set_allocator(cbs[0], cbs[1], None))
    _allocators.append(cbs)


def _status_name(st):
    return load().zda_status_str(st).decode() if _lib is not None else str(st)


def _check(st):
    if st != ZDA_OK:
        raise ZdaError(st, load().zda_last_error().decode())


def default_desc(**kw) -> ZoneDesc:
    d = ZoneDesc()
    load().zda_zone_desc_default(ctypes.byref(d))
    for k, v in kw.items():
        if k == "pml":
            d.pml_r_in, d.pml_r_out, d.pml_z_lo, d.pml_z_hi = v
        elif k == "design":
            d.design_k0, d.design_k1 = v
        elif k in {f[0] for f in ZoneDesc._fields_}:
            setattr(d, k, v)
        else:
            raise TypeError("unknown zone descriptor field %r" % k)
    return d


# zones and batches not yet closed, destroyed at interpreter exit while torch
# (whose caching allocator may back their memory) is still whole
_live_zones = weakref.WeakSet()
_live_batches = weakref.WeakSet()
_exit_hook = False


def _close_live():
    for b in list(_live_batches):
        try:
            b.close()
        except Exception:
            pass
    for z in list(_live_zones):
        try:
            z.close()
        except Exception:
            pass


def _track(obj, live):
    """Registers obj for destruction at exit; the hook is registered after
    torch is imported, so that it runs before torch's own exit handlers."""
    global _exit_hook
    live.add(obj)
    if not _exit_hook:
        atexit.register(_close_live)
        _exit_hook = True


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the ZDA library needs a HIP GPU (no CPU fallback)")
    return torch


def _stream_ptr(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Zone:
    """One ZDA zone on the current GPU (owns its device memory)."""

    def __init__(self, desc: ZoneDesc, eps=None):
        torch = _torch()
        self.desc = desc
        self.shape = (desc.nz, desc.nr, desc.nphi)
        lib = load()
        h = ctypes.c_void_p()
        ptr, on_dev, keep = self._in_ptr(torch, eps, torch.float32)
        _check(lib.zda_zone_create(ctypes.byref(desc), ptr, on_dev, ctypes.byref(h)))
        self._h = h
        _track(self, _live_zones)
        # advanced by every call that changes what an adjoint run would use
        # (permittivity, design, fields, forward monitors)
        self.state_serial = 0
        del keep

    def close(self):
        if getattr(self, "_h", None):
            load().zda_zone_destroy(self._h)
            self._h = None
        _live_zones.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _in_ptr(torch, x, dtype):
        """(pointer, on_device, keep-alive) of an input array or tensor."""
        if x is None:
            return None, 0, None
        if isinstance(x, torch.Tensor):
            t = x.detach().to(dtype).contiguous()
            return ctypes.c_void_p(t.data_ptr()), int(t.is_cuda), t
        a = np.ascontiguousarray(np.asarray(x), dtype=np.float32 if dtype == torch.float32 else None)
        return ctypes.c_void_p(a.ctypes.data), 0, a

    def info(self) -> ZoneInfo:
        inf = ZoneInfo()
        _check(load().zda_zone_get_info(self._h, ctypes.byref(inf)))
        return inf

    def set_option(self, option, value):
        _check(load().zda_zone_set_option(self._h, int(option), int(value)))

    def set_launch(self, kchunk, tile_rows):
        _check(load().zda_zone_set_launch(self._h, int(kchunk), int(tile_rows)))

    def release_fields(self):
        """Give back the time-stepping memory (both field sets, PML
        auxiliaries, intermediate sets); the zone keeps its permittivity,
        design, launch settings and monitors (zda_zone_release_fields)."""
        _check(load().zda_zone_release_fields(self._h))

    def acquire_fields(self, buffer=None):
        """Take the time-stepping memory again, zeroed on the zone's stream
        (zda_zone_acquire_fields): allocated, or carved from `buffer` (a CUDA
        tensor of at least fields_bytes() bytes, 256-byte aligned, that the
        caller keeps and leaves alone until release_fields returns)."""
        if buffer is None:
            _check(load().zda_zone_acquire_fields(self._h, None, 0))
        else:
            nbytes = buffer.numel() * buffer.element_size()
            _check(load().zda_zone_acquire_fields(self._h, ctypes.c_void_p(buffer.data_ptr()), nbytes))

    def fields_bytes(self):
        """Bytes of time-stepping memory the zone carves from a caller's buffer."""
        n = ctypes.c_size_t()
        _check(load().zda_zone_fields_bytes(self._h, ctypes.byref(n)))
        return n.value

    @property
    def dt(self):
        return self.info().dt

    def set_eps(self, eps):
        torch = _torch()
        ptr, dev, keep = self._in_ptr(torch, eps, torch.float32)
        self.state_serial += 1
        _check(load().zda_zone_set_eps(self._h, ptr, dev))

    def set_design(self, rho):
        torch = _torch()
        ptr, dev, keep = self._in_ptr(torch, rho, torch.float32)
        self.state_serial += 1
        _check(load().zda_zone_set_design(self._h, ptr, dev))

    def run(self, nsteps, omegas=(), *, kind=SRC_PLANE_CIRC, k_src=1, omega_c=0.0, width=1.0, n0=-1,
            patterns=None, profiles=None, plane=True, volume=False, cont=False, timing=False, stream=None,
            noalloc=False):
        """Time-step (asynchronous on the current torch stream).  noalloc:
        through zda_fdtd_run_noalloc (staging in the library's fixed device
        scratch; waits for the stream before it returns)."""
        torch = _torch()
        s = Source()
        s.kind, s.k_src, s.omega_c, s.width, s.n0 = kind, k_src, omega_c, width, n0
        keep = []
        if kind == SRC_CUSTOM:
            pat = patterns
            if isinstance(pat, torch.Tensor):
                pt = torch.view_as_real(pat.to(torch.complex64).contiguous()).contiguous()
                s.patterns, s.patterns_on_device = pt.data_ptr(), int(pt.is_cuda)
            else:
                pt = np.ascontiguousarray(np.asarray(pat, np.complex64))
                s.patterns, s.patterns_on_device = pt.ctypes.data, 0
            pr = np.ascontiguousarray(np.asarray(profiles, np.complex128))
            s.n_profiles = pr.shape[0]
            s.profiles = pr.ctypes.data
            keep += [pt, pr]
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, np.float64)))
        flags = (DFT_PLANE if plane else 0) | (DFT_VOLUME if volume else 0) | (RUN_CONTINUE if cont else 0) | \
            (RUN_TIMING if timing else 0)
        self.state_serial += 1
        fn = load().zda_fdtd_run_noalloc if noalloc else load().zda_fdtd_run
        _check(fn(self._h, ctypes.byref(s), int(nsteps), ctypes.c_void_p(om.ctypes.data), int(om.size), flags,
                  _stream_ptr(torch, stream)))
        self._K = int(om.size)

    def run_fp64(self, eps, nsteps, omegas, *, kind=SRC_PLANE_CIRC, k_src=1, omega_c=0.0, width=1.0, n0=-1,
                 stream=None):
        """The same forward run in FP64 (zda_fdtd_run_fp64) with the FP64
        permittivity eps [nz][nr][nphi] (numpy or a CUDA float64 tensor);
        returns the exit-plane DFT as complex128 numpy [K][2][nr][nphi]."""
        torch = _torch()
        s = Source()
        s.kind, s.k_src, s.omega_c, s.width, s.n0 = kind, k_src, omega_c, width, n0
        if isinstance(eps, torch.Tensor):
            e = eps.to(torch.float64).contiguous()
            eptr, edev = e.data_ptr(), int(e.is_cuda)
        else:
            e = np.ascontiguousarray(np.asarray(eps, np.float64))
            eptr, edev = e.ctypes.data, 0
        nr, nphi, nz = self.desc.nr, self.desc.nphi, self.desc.nz
        if (e.numel() if isinstance(e, torch.Tensor) else e.size) != nr * nphi * nz:
            raise ValueError("eps must hold nz * nr * nphi values")
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, np.float64)))
        out = np.empty((om.size, 2, nr, nphi), np.complex128)
        _check(load().zda_fdtd_run_fp64(self._h, ctypes.c_void_p(eptr), edev, ctypes.byref(s), int(nsteps),
                                        ctypes.c_void_p(om.ctypes.data), int(om.size),
                                        ctypes.c_void_p(out.ctypes.data), 0, _stream_ptr(torch, stream)))
        del e
        return out

    def last_timing(self) -> Timing:
        t = Timing()
        _check(load().zda_zone_last_timing(self._h, ctypes.byref(t)))
        return t

    def dft(self, monitor=MON_PLANE, K=None, components=0):
        """Monitor as a complex64 CUDA tensor ([K][C][nr][nphi] or
        [K][C][nd][nr][nphi]; C = every component of the monitor, or those
        whose COMP_* bits `components` sets).  Ordered on the zone's stream."""
        torch = _torch()
        K = self._K if K is None else K
        d = self.desc
        ncomp = 2 if monitor == MON_PLANE else 3
        C = ncomp if components == 0 else bin(int(components)).count("1")
        if monitor == MON_PLANE:
            shape = (K, C, d.nr, d.nphi)
        else:
            shape = (K, C, d.design_k1 - d.design_k0, d.nr, d.nphi)
        out = torch.empty(shape, dtype=torch.complex64, device="cuda")
        _check(load().zda_dft_fields(self._h, monitor, int(components), ctypes.c_void_p(out.data_ptr()),
                                     2 * out.numel(), 1))
        return out

    def dft_host(self, monitor=MON_PLANE, K=None, components=0):
        """The monitor copied into host memory (complex64 numpy array); waits
        for the zone and raises ZdaError (ZDA_ERR_DIVERGED) after a divergence."""
        K = self._K if K is None else K
        d = self.desc
        ncomp = 2 if monitor == MON_PLANE else 3
        C = ncomp if components == 0 else bin(int(components)).count("1")
        shape = (K, C, d.nr, d.nphi) if monitor == MON_PLANE else (K, C, d.design_k1 - d.design_k0, d.nr, d.nphi)
        out = np.empty(shape, np.complex64)
        _check(load().zda_dft_fields(self._h, monitor, int(components), ctypes.c_void_p(out.ctypes.data),
                                     2 * out.size, 0))
        return out

    def sync(self):
        """Wait for the zone's stream; raises ZdaError (ZDA_ERR_DIVERGED) if
        the divergence watchdog fired since the last resetting run."""
        _check(load().zda_zone_sync(self._h))

    def set_stream(self, stream):
        _check(load().zda_zone_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def adjoint_grad(self, dF_dE, adj_width=0.0, stream=None):
        torch = _torch()
        g = dF_dE.to(torch.complex64).contiguous() if isinstance(dF_dE, torch.Tensor) else \
            torch.as_tensor(np.asarray(dF_dE, np.complex64)).cuda()
        g = torch.view_as_real(g).contiguous()
        d = self.desc
        out = torch.empty((d.design_k1 - d.design_k0, d.nr, d.nphi), dtype=torch.float32, device="cuda")
        _check(load().zda_adjoint_grad(self._h, ctypes.c_void_p(g.data_ptr()), 1, ctypes.c_void_p(out.data_ptr()),
                                       1, float(adj_width), _stream_ptr(torch, stream)))
        torch.cuda.current_stream().synchronize()
        return out

    def read_field(self, name):
        torch = _torch()
        out = torch.empty(self.shape, dtype=torch.complex64, device="cuda")
        _check(load().zda_zone_read_field(self._h, COMP[name], ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def write_field(self, name, value):
        torch = _torch()
        t = value if isinstance(value, torch.Tensor) else torch.as_tensor(np.asarray(value, np.complex64))
        t = t.to(device="cuda", dtype=torch.complex64).contiguous()
        self.state_serial += 1
        _check(load().zda_zone_write_field(self._h, COMP[name], ctypes.c_void_p(t.data_ptr()), 1))


def preset_source(kind=SRC_PLANE_CIRC, k_src=1, omega_c=0.0, width=1.0, n0=-1):
    s = Source()
    s.kind, s.k_src, s.omega_c, s.width, s.n0 = kind, k_src, omega_c, width, n0
    return s


class Batch:
    """Zones of uneven size stepped together (one launch per time step,
    graph-replayed time loop).  Keeps references to its zones."""

    def __init__(self, zones):
        torch = _torch()
        self.zones = list(zones)
        arr = (ctypes.c_void_p * len(self.zones))(*[z._h.value for z in self.zones])
        h = ctypes.c_void_p()
        _check(load().zda_batch_create(arr, len(self.zones), ctypes.byref(h)))
        self._h = h
        _track(self, _live_batches)

    def close(self):
        if getattr(self, "_h", None):
            load().zda_batch_destroy(self._h)
            self._h = None
        _live_batches.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sources(self, sources):
        arr = (Source * len(self.zones))()
        for i, s in enumerate(sources):
            arr[i] = s
        return arr

    def run(self, sources, nsteps, omegas, *, plane=True, volume=False, stream=None):
        torch = _torch()
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, np.float64)))
        flags = (DFT_PLANE if plane else 0) | (DFT_VOLUME if volume else 0)
        for z in self.zones:
            z.state_serial += 1
        _check(load().zda_batch_run(self._h, self._sources(sources), int(nsteps), ctypes.c_void_p(om.ctypes.data),
                                    int(om.size), flags, _stream_ptr(torch, stream)))
        for z in self.zones:
            z._K = int(om.size)

    def adjoint_grad(self, dF_dE_list, stream=None):
        torch = _torch()
        gs = [torch.view_as_real(g.to(torch.complex64).contiguous()).contiguous() for g in dF_dE_list]
        outs = []
        for z in self.zones:
            d = z.desc
            outs.append(torch.empty((d.design_k1 - d.design_k0, d.nr, d.nphi), dtype=torch.float32, device="cuda"))
        ga = (ctypes.c_void_p * len(gs))(*[g.data_ptr() for g in gs])
        oa = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        _check(load().zda_batch_adjoint_grad(self._h, ga, oa, _stream_ptr(torch, stream)))
        torch.cuda.current_stream().synchronize()
        return outs

    def set_launch(self, tile_rows, kchunk=None):
        kc = None
        if kchunk is not None:
            kc = (ctypes.c_int * len(kchunk))(*[int(k) for k in kchunk])
        _check(load().zda_batch_set_launch(self._h, int(tile_rows), kc))

    def autotune(self, sources, probe_steps, omegas, stream=None):
        torch = _torch()
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, np.float64)))
        res = TuneResult()
        _check(load().zda_batch_autotune(self._h, self._sources(sources), int(probe_steps),
                                         ctypes.c_void_p(om.ctypes.data), int(om.size), _stream_ptr(torch, stream),
                                         ctypes.byref(res)))
        return res


def plan_two_step_tiles(desc: ZoneDesc, tile_rows=13, kchunk=48, k_src=1, order=0):
    """The two-step launch plan (host only): uint32 array [ntiles][4] of
    {phi block, i0 | rows << 16, kb | ke << 16, kind} and the interior count."""
    lib = load()
    n, ni = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.zda_plan_two_step_tiles(ctypes.byref(desc), tile_rows, kchunk, k_src, order, None, 0,
                                       ctypes.byref(n), ctypes.byref(ni)))
    out = np.zeros((n.value, 4), np.uint32)
    _check(lib.zda_plan_two_step_tiles(ctypes.byref(desc), tile_rows, kchunk, k_src, order,
                                       ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n), ctypes.byref(ni)))
    return out, ni.value

