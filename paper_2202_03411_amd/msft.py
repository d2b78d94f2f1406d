"""ctypes binding of libmsft.so -- argument marshalling only.

Every function named ``msft_*`` here forwards to the C function of the same name
declared in ``include/msft.h``; device buffers are torch tensors (only their
data pointers cross the boundary) and the stream is torch's current stream
unless one is given.  All arithmetic runs in the library's HIP kernels: there
is no fallback, and a missing or unloadable library raises at import time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first: the library then shares torch's HIP runtime

from . import build as _build

MSFT_OK, MSFT_ERR_INVALID, MSFT_ERR_UNDERSAMPLED = 0, 1, 2
MSFT_ERR_NOMEM, MSFT_ERR_DEVICE, MSFT_ERR_BUSY, MSFT_ERR_UNSUPPORTED = 3, 4, 5, 6
MSFT_FP32, MSFT_BF16X3, MSFT_BF16 = 0, 1, 2
MSFT_STRENGTH_MSFT, MSFT_STRENGTH_BORN, MSFT_STRENGTH_DENSITY = 0, 1, 2
MSFT_ALLOW_ALIAS = 1
MSFT_DETECTOR_UNIFORM_Q = 2
MSFT_NOALLOC_MAX_BYTES = 64 << 20
DETECTORS = {"flat": 0, "uniform_q": MSFT_DETECTOR_UNIFORM_Q}

PRECISIONS = {"fp32": MSFT_FP32, "bf16x3": MSFT_BF16X3, "bf16": MSFT_BF16}
STRENGTHS = {"msft": MSFT_STRENGTH_MSFT, "born": MSFT_STRENGTH_BORN, "density": MSFT_STRENGTH_DENSITY}


class MSFTError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {msft_status_str(status)} ({status}): {detail}")


class msft_geometry(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("wavelength", ctypes.c_double),
        ("theta_max_deg", ctypes.c_double),
        ("det_n", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dy", ctypes.c_double),
        ("dz", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("strength", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class msft_shape_grid(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dy", ctypes.c_double),
        ("dz", ctypes.c_double),
        ("edge", ctypes.c_double),
        ("delta0", ctypes.c_double),
        ("beta0", ctypes.c_double),
    ]


class msft_request(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("delta", ctypes.c_void_p),
        ("beta", ctypes.c_void_p),
        ("intensity", ctypes.c_void_p),
        ("amplitude", ctypes.c_void_p),
        ("tile_begin", ctypes.c_int32),
        ("tile_end", ctypes.c_int32),
    ]


def _load():
    path = _build.LIB
    if not os.path.exists(path):
        _build.build()
    lib = ctypes.CDLL(path)
    P, S, I32, I64, VP = ctypes.POINTER, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.msft_plan.argtypes = [P(msft_geometry), ctypes.c_int, P(VP)]
    lib.msft_plan_qlist.argtypes = [P(msft_geometry), VP, I64, ctypes.c_int, P(VP)]
    lib.msft_plan_destroy.argtypes = [VP]
    lib.msft_plan_query.argtypes = [VP, P(I64), P(S), P(S), P(S)]
    lib.msft_plan_qmap.argtypes = [VP, VP]
    lib.msft_plan_grid.argtypes = [VP, VP, VP, VP]
    lib.msft_simulate.argtypes = [VP, VP, VP, VP, VP, VP, S, VP]
    lib.msft_simulate_scan.argtypes = [VP, VP, VP, VP, S, VP]
    lib.msft_simulate_contract.argtypes = [VP, VP, S, VP, VP, VP]
    lib.msft_simulate_noalloc.argtypes = [VP, VP, VP, VP, VP, VP]
    lib.msft_pixel_block.argtypes = []
    lib.msft_batch_query.argtypes = [P(msft_request), I32, P(S)]
    lib.msft_simulate_batch.argtypes = [P(msft_request), I32, VP, S, VP]
    lib.msft_backward.argtypes = [VP, VP, VP, VP, VP, VP, VP, VP, S, VP]
    D = ctypes.c_double
    lib.msft_render_sh.argtypes = [P(msft_shape_grid), I32, D, VP, VP, VP, VP]
    lib.msft_render_sh_query.argtypes = [I32, P(S)]
    lib.msft_render_sh_backward.argtypes = [P(msft_shape_grid), I32, D, VP, VP, VP, VP, VP, S, VP]
    lib.msft_render_ellipsoid.argtypes = [P(msft_shape_grid), VP, VP, VP, VP, VP]
    lib.msft_detect_ideal.argtypes = [VP, VP, D, ctypes.c_uint64, VP, VP, VP]
    lib.msft_render_volume.argtypes = [P(msft_shape_grid), I32, I32, I32, D, D, D, VP, VP, VP, VP, VP]
    lib.msft_peak_mfma.argtypes = [I32, I32, I32, VP, P(D), VP]
    lib.msft_copy.argtypes = [VP, VP, S, VP]
    lib.msft_status_str.argtypes = [ctypes.c_int]
    lib.msft_status_str.restype = ctypes.c_char_p
    lib.msft_last_error.argtypes = []
    lib.msft_last_error.restype = ctypes.c_char_p
    for name in ("msft_plan", "msft_plan_qlist", "msft_plan_destroy", "msft_plan_query",
                 "msft_plan_qmap", "msft_plan_grid", "msft_simulate", "msft_simulate_scan",
                 "msft_simulate_contract", "msft_simulate_noalloc", "msft_pixel_block", "msft_batch_query", "msft_simulate_batch",
                 "msft_backward", "msft_render_sh", "msft_render_sh_query", "msft_render_sh_backward",
                 "msft_render_ellipsoid", "msft_render_volume", "msft_detect_ideal", "msft_peak_mfma",
                 "msft_copy"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()
LIBRARY_PATH = _build.LIB

# every symbol the C header declares
EXPORTS = ("msft_plan", "msft_plan_qlist", "msft_plan_destroy", "msft_plan_query", "msft_plan_qmap",
           "msft_plan_grid", "msft_simulate", "msft_simulate_scan", "msft_simulate_contract",
           "msft_simulate_noalloc", "msft_pixel_block",
           "msft_batch_query",
           "msft_simulate_batch", "msft_backward", "msft_render_sh", "msft_render_sh_query",
           "msft_render_sh_backward", "msft_render_ellipsoid", "msft_render_volume",
           "msft_detect_ideal", "msft_peak_mfma", "msft_copy", "msft_status_str",
           "msft_last_error")


def msft_status_str(status: int) -> str:
    return _lib.msft_status_str(int(status)).decode()


def msft_last_error() -> str:
    return _lib.msft_last_error().decode()


def _check(status: int, where: str):
    if status != MSFT_OK:
        raise MSFTError(status, where, msft_last_error())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_geometry(wavelength, theta_max_deg, det_n, grid, pitch, precision="fp32",
                  strength="msft", allow_alias=False, detector="flat") -> msft_geometry:
    """Fill an msft_geometry from Python values (grid = (nx, ny, nz), pitch = (dx, dy, dz));
    detector is "flat" or "uniform_q" (MSFT_DETECTOR_UNIFORM_Q)."""
    g = msft_geometry()
    g.struct_size = ctypes.sizeof(msft_geometry)
    g.wavelength = float(wavelength)
    g.theta_max_deg = float(theta_max_deg)
    g.det_n = int(det_n)
    g.nx, g.ny, g.nz = (int(v) for v in grid)
    g.dx, g.dy, g.dz = (float(v) for v in pitch)
    g.precision = PRECISIONS.get(precision, precision)
    g.strength = STRENGTHS.get(strength, strength)
    g.flags = (MSFT_ALLOW_ALIAS if allow_alias else 0) | DETECTORS[detector]
    return g


# What the binding knows of each live plan, to check the buffers it is handed
# before their pointers cross the boundary: handle -> (grid, npix, device, workspace).
_PLANS: dict = {}


def _register(handle: int, geometry: msft_geometry, device: int) -> int:
    npix, ws, _, _ = msft_plan_query(handle)
    _PLANS[handle] = ((geometry.nx, geometry.ny, geometry.nz), npix, int(device), ws)
    return handle


def _plan_info(plan: int):
    info = _PLANS.get(plan)
    if info is None:
        raise ValueError("unknown plan handle (create plans with msft_plan / msft_plan_qlist)")
    return info


def _check_tensor(t, name, numel, device, dtype=torch.float32, shape=None):
    """A float32, contiguous buffer of `numel` values on the plan's device."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must live on cuda:{device}, got {t.device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} values, got {t.numel()}")


def _check_workspace(ws, device):
    _check_tensor(ws, "workspace", ws.numel(), device, dtype=ws.dtype)
    return ws.numel() * ws.element_size()


def _check_io(plan, delta=None, beta=None, intensity=None, amplitude=None):
    grid, npix, dev, _ = _plan_info(plan)
    V = grid[0] * grid[1] * grid[2]
    for name, t in (("delta", delta), ("beta", beta)):
        if t is not None:
            _check_tensor(t, name, V, dev)
    if intensity is not None:
        _check_tensor(intensity, "intensity", npix, dev)
    if amplitude is not None:
        _check_tensor(amplitude, "amplitude", 2 * npix, dev)
    return dev


def msft_plan(geometry: msft_geometry, device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.msft_plan(ctypes.byref(geometry), int(device), ctypes.byref(h)), "msft_plan")
    return _register(h.value, geometry, device)


def msft_plan_qlist(geometry: msft_geometry, q, device: int = 0) -> int:
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    h = ctypes.c_void_p()
    _check(_lib.msft_plan_qlist(ctypes.byref(geometry), q.ctypes.data_as(ctypes.c_void_p),
                                q.shape[0], int(device), ctypes.byref(h)), "msft_plan_qlist")
    return _register(h.value, geometry, device)


def msft_plan_destroy(plan: int) -> None:
    _check(_lib.msft_plan_destroy(ctypes.c_void_p(plan)), "msft_plan_destroy")
    _PLANS.pop(plan, None)


def msft_plan_query(plan: int):
    """(npix, workspace_bytes, resident_bytes, per_request_bytes)."""
    n, w, r, q = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.msft_plan_query(ctypes.c_void_p(plan), ctypes.byref(n), ctypes.byref(w),
                                ctypes.byref(r), ctypes.byref(q)), "msft_plan_query")
    return n.value, w.value, r.value, q.value


def msft_plan_qmap(plan: int) -> np.ndarray:
    npix = msft_plan_query(plan)[0]
    out = np.empty((npix, 3), np.float64)
    _check(_lib.msft_plan_qmap(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.c_void_p)),
           "msft_plan_qmap")
    return out


def msft_plan_grid(plan: int, shape):
    x, y, z = (np.empty(int(n), np.float64) for n in shape)
    _check(_lib.msft_plan_grid(ctypes.c_void_p(plan), *(a.ctypes.data_as(ctypes.c_void_p)
                                                        for a in (x, y, z))), "msft_plan_grid")
    return x, y, z


def msft_simulate(plan, delta, beta, intensity, amplitude, workspace, stream=None) -> None:
    dev = _check_io(plan, delta, beta, intensity, amplitude)
    nbytes = _check_workspace(workspace, dev)
    _check(_lib.msft_simulate(ctypes.c_void_p(plan), _ptr(delta), _ptr(beta), _ptr(intensity),
                              _ptr(amplitude), _ptr(workspace), nbytes, _stream(stream)),
           "msft_simulate")


def msft_simulate_scan(plan, delta, beta, workspace, stream=None) -> None:
    dev = _check_io(plan, delta, beta)
    nbytes = _check_workspace(workspace, dev)
    _check(_lib.msft_simulate_scan(ctypes.c_void_p(plan), _ptr(delta), _ptr(beta), _ptr(workspace),
                                   nbytes, _stream(stream)), "msft_simulate_scan")


def msft_simulate_contract(plan, workspace, intensity, amplitude, stream=None) -> None:
    dev = _check_io(plan, intensity=intensity, amplitude=amplitude)
    nbytes = _check_workspace(workspace, dev)
    _check(_lib.msft_simulate_contract(ctypes.c_void_p(plan), _ptr(workspace), nbytes,
                                       _ptr(intensity), _ptr(amplitude), _stream(stream)),
           "msft_simulate_contract")


def msft_simulate_noalloc(plan, delta, beta, intensity, amplitude, stream=None) -> None:
    """msft_simulate with the library's fixed per-device scratch (no workspace, no
    allocation in the call); calls that overlap on one device race."""
    _check_io(plan, delta, beta, intensity, amplitude)
    _check(_lib.msft_simulate_noalloc(ctypes.c_void_p(plan), _ptr(delta), _ptr(beta),
                                      _ptr(intensity), _ptr(amplitude), _stream(stream)),
           "msft_simulate_noalloc")


def msft_pixel_block() -> int:
    return int(_lib.msft_pixel_block())


def _requests(reqs):
    """The C request array; every buffer is checked against its plan first."""
    arr = (msft_request * max(len(reqs), 1))()
    for k, r in enumerate(reqs):
        plan, delta, beta, inten, amp = r[:5]
        rng = r[5] if len(r) > 5 else (-1, -1)
        _check_io(plan, delta, beta, inten, amp)
        arr[k] = msft_request(plan, delta.data_ptr(), beta.data_ptr(), inten.data_ptr(),
                              amp.data_ptr() if amp is not None else None, int(rng[0]), int(rng[1]))
    return arr


def msft_batch_query(reqs) -> int:
    """reqs: sequence of (plan, delta, beta, intensity, amplitude[, (tile_begin, tile_end)])."""
    arr = _requests(reqs)
    n = ctypes.c_size_t()
    _check(_lib.msft_batch_query(arr, len(reqs), ctypes.byref(n)), "msft_batch_query")
    return n.value


def msft_simulate_batch(reqs, workspace, stream=None) -> None:
    arr = _requests(reqs)
    dev = _plan_info(reqs[0][0])[2] if len(reqs) else workspace.device.index
    nbytes = _check_workspace(workspace, dev)
    _check(_lib.msft_simulate_batch(arr, len(reqs), _ptr(workspace), nbytes, _stream(stream)),
           "msft_simulate_batch")


def msft_backward(plan, delta, beta, amplitude, grad_intensity, grad_delta, grad_beta, workspace,
                  stream=None) -> None:
    dev = _check_io(plan, delta, beta, grad_intensity, amplitude)
    _check_io(plan, grad_delta, grad_beta)
    nbytes = _check_workspace(workspace, dev)
    _check(_lib.msft_backward(ctypes.c_void_p(plan), _ptr(delta), _ptr(beta), _ptr(amplitude),
                              _ptr(grad_intensity), _ptr(grad_delta), _ptr(grad_beta),
                              _ptr(workspace), nbytes, _stream(stream)), "msft_backward")


def workspace_tensor(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes, 256-byte aligned (torch's allocator aligns to 512)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Plan:
    """Owning wrapper of an msft plan; simulate() allocates outputs with torch."""

    def __init__(self, wavelength, theta_max_deg, det_n, grid, pitch, precision="fp32",
                 strength="msft", device=0, allow_alias=False, q=None, detector="flat"):
        self.geometry = make_geometry(wavelength, theta_max_deg, det_n, grid, pitch, precision,
                                      strength, allow_alias, detector)
        self.grid = tuple(int(v) for v in grid)
        self.pitch = tuple(float(v) for v in pitch)
        self.device_index = int(device)
        if q is None:
            self.handle = msft_plan(self.geometry, self.device_index)
        else:
            self.handle = msft_plan_qlist(self.geometry, q, self.device_index)
        (self.npix, self.workspace_bytes, self.resident_bytes,
         self.per_request_bytes) = msft_plan_query(self.handle)
        self._ws = None

    @classmethod
    def for_workload(cls, wl, precision="fp32", device=0, **kw):
        mode = {0: "msft", 1: "born", 2: "density"}[wl.mode]
        return cls(wl.wavelength, wl.theta_max_deg, wl.det_n, wl.grid, wl.pitch, precision, mode,
                   device, **kw)

    @property
    def device(self):
        return torch.device("cuda", self.device_index) if self.device_index >= 0 else torch.device("cpu")

    def workspace(self):
        if self._ws is None:
            self._ws = workspace_tensor(self.workspace_bytes, self.device)
        return self._ws

    def qmap(self):
        return msft_plan_qmap(self.handle)

    def voxel_grid(self):
        return msft_plan_grid(self.handle, self.grid)

    def simulate(self, delta, beta, amplitude=False, out=None, stream=None):
        dev = self.device
        if tuple(delta.shape) != self.grid or tuple(beta.shape) != self.grid:
            raise ValueError(f"delta/beta must have shape {self.grid}")
        if delta.dtype != torch.float32 or beta.dtype != torch.float32:
            raise TypeError("delta and beta must be float32")
        if delta.device != dev or beta.device != dev:
            raise ValueError("delta and beta must live on the plan's device")
        delta, beta = delta.contiguous(), beta.contiguous()
        I = out if out is not None else torch.empty(self.npix, dtype=torch.float32, device=dev)
        A = torch.empty(self.npix, 2, dtype=torch.float32, device=dev) if amplitude else None
        msft_simulate(self.handle, delta, beta, I, A, self.workspace(), stream)
        return (I, torch.view_as_complex(A)) if amplitude else I

    def detect_ideal(self, intensity, photon_density, seed, expected=False, stream=None):
        """One recording of the Ideal detector: Poisson counts [N*N] (float32) of the
        intensity for an incident fluence photon_density (photons per unit area); with
        expected=True also the mean counts."""
        if intensity.dtype != torch.float32 or intensity.numel() != self.npix:
            raise ValueError(f"intensity must be float32 with {self.npix} values")
        if intensity.device != self.device:
            raise ValueError("intensity must live on the plan's device")
        intensity = intensity.contiguous()
        counts = torch.empty(self.npix, dtype=torch.float32, device=self.device)
        mu = torch.empty_like(counts) if expected else None
        msft_detect_ideal(self.handle, intensity, photon_density, seed, counts, mu, stream)
        return (counts, mu) if expected else counts

    def close(self):
        if getattr(self, "handle", None):
            msft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def make_shape_grid(grid, pitch, edge=0.0, delta0=0.01, beta0=0.02) -> msft_shape_grid:
    """Fill an msft_shape_grid (grid = (nx, ny, nz), pitch = (dx, dy, dz))."""
    g = msft_shape_grid()
    g.struct_size = ctypes.sizeof(msft_shape_grid)
    g.nx, g.ny, g.nz = (int(v) for v in grid)
    g.dx, g.dy, g.dz = (float(v) for v in pitch)
    g.edge, g.delta0, g.beta0 = float(edge), float(delta0), float(beta0)
    return g


def msft_render_sh(shape_grid, lmax, r0, coeffs, delta, beta, stream=None) -> None:
    _check(_lib.msft_render_sh(ctypes.byref(shape_grid), int(lmax), float(r0), _ptr(coeffs),
                               _ptr(delta), _ptr(beta), _stream(stream)), "msft_render_sh")


def msft_render_sh_query(lmax) -> int:
    n = ctypes.c_size_t()
    _check(_lib.msft_render_sh_query(int(lmax), ctypes.byref(n)), "msft_render_sh_query")
    return n.value


def msft_render_sh_backward(shape_grid, lmax, r0, coeffs, grad_delta, grad_beta, grad_coeffs,
                            workspace, stream=None) -> None:
    _check(_lib.msft_render_sh_backward(ctypes.byref(shape_grid), int(lmax), float(r0), _ptr(coeffs),
                                        _ptr(grad_delta), _ptr(grad_beta), _ptr(grad_coeffs),
                                        _ptr(workspace), workspace.numel() * workspace.element_size(),
                                        _stream(stream)), "msft_render_sh_backward")


def msft_render_ellipsoid(shape_grid, axes, rot, delta, beta, stream=None) -> None:
    ax = np.ascontiguousarray(axes, dtype=np.float64).reshape(3)
    R = np.ascontiguousarray(rot, dtype=np.float64).reshape(9)
    _check(_lib.msft_render_ellipsoid(ctypes.byref(shape_grid), ax.ctypes.data_as(ctypes.c_void_p),
                                      R.ctypes.data_as(ctypes.c_void_p), _ptr(delta), _ptr(beta),
                                      _stream(stream)), "msft_render_ellipsoid")


def msft_render_volume(shape_grid, src_delta, src_beta, src_pitch, delta, beta, stream=None) -> None:
    """Resample a (delta, beta) map on its own centred grid (src_pitch) onto shape_grid."""
    sx, sy, sz = (int(v) for v in src_delta.shape)
    sdx, sdy, sdz = (float(v) for v in src_pitch)
    _check(_lib.msft_render_volume(ctypes.byref(shape_grid), sx, sy, sz, sdx, sdy, sdz,
                                   _ptr(src_delta), _ptr(src_beta), _ptr(delta), _ptr(beta),
                                   _stream(stream)), "msft_render_volume")


def msft_peak_mfma(precision, iters, nblocks, sink, stream=None) -> float:
    """Launch the matrix-core peak probe; sink: float32 device tensor of nblocks * 256.
    Returns the real flops of the launch."""
    prec = {"fp32": MSFT_FP32, "bf16x3": MSFT_BF16X3}[precision]
    _check_tensor(sink, "sink", int(nblocks) * 256, sink.device.index if sink.is_cuda else 0)
    flops = ctypes.c_double(0.0)
    _check(_lib.msft_peak_mfma(prec, int(iters), int(nblocks), _ptr(sink), ctypes.byref(flops), _stream(stream)),
           "msft_peak_mfma")
    return flops.value


def msft_copy(src, dst, stream=None) -> None:
    """dst = src for two contiguous device tensors of the same byte size."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
            and dst.numel() * dst.element_size() == nbytes and src.device == dst.device):
        raise ValueError("msft_copy: contiguous device tensors of one size on one device")
    _check(_lib.msft_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "msft_copy")


def msft_detect_ideal(plan_handle, intensity, photon_density, seed, counts, expected=None,
                      stream=None) -> None:
    """One Poisson recording of a flat-detector intensity (see Plan.detect_ideal)."""
    _check(_lib.msft_detect_ideal(plan_handle, _ptr(intensity), float(photon_density),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(counts),
                                  _ptr(expected), _stream(stream)),
           "msft_detect_ideal")
