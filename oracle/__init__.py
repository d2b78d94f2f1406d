"""FP64 CPU oracle of the MSFT forward model and its gradient -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it and shares no code with it.
The arithmetic lives in ``msft_oracle.c`` (plain double-precision C written from
Sec. 2 of the paper, Eqs. (1)-(9)); this module only marshals numpy arrays.

Strength modes: 0 = MSFT (Eq. (9), incident field propagated by Eq. (8)),
1 = BORN (undisturbed incident field, Eq. (1) with (5)), 2 = DENSITY (the two
inputs are the real and imaginary parts of a scattering density, Eq. (1)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

MSFT, BORN, DENSITY = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over pixels)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_qmap.argtypes = [d, d, i32, p]
        lib.oracle_qmap_uniform.argtypes = [d, d, i32, p]
        lib.oracle_grid.argtypes = [i32, d, p]
        lib.oracle_strength.argtypes = [i32, i32, i32, i32, d, d, d, d, p, p, p]
        lib.oracle_amplitude.argtypes = [i32, p, i64, i32, i32, i32, d, d, d, p, p]
        lib.oracle_backward.argtypes = [i32, p, i64, p, p, i32, i32, i32, d, d, d, d,
                                        p, p, p, i64, p, p]
        lib.oracle_ylm.argtypes = [i32, i32, d, d]
        lib.oracle_ylm.restype = ctypes.c_double
        lib.oracle_render_sh.argtypes = [i32, i32, i32, d, d, d, i32, p, d, d, d, d, p, p]
        lib.oracle_render_sh_backward.argtypes = [i32, i32, i32, d, d, d, i32, p, d, d, d, d,
                                                  p, p, p]
        lib.oracle_render_ellipsoid.argtypes = [i32, i32, i32, d, d, d, p, p, d, d, d, p, p]
        lib.oracle_render_volume.argtypes = [i32, i32, i32, d, d, d, i32, i32, i32, d, d, d, p, p, p, p]
        u64 = ctypes.c_uint64
        lib.oracle_philox.argtypes = [p, p, p]
        lib.oracle_pixel_solid_angle.argtypes = [d, i32, i32, i32]
        lib.oracle_pixel_solid_angle.restype = ctypes.c_double
        lib.oracle_detect_ideal.argtypes = [d, d, i32, p, d, u64, p, p]
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        for f in (lib.oracle_render_sh, lib.oracle_render_sh_backward, lib.oracle_render_ellipsoid,
                  lib.oracle_render_volume, lib.oracle_philox, lib.oracle_detect_ideal,
                  lib.oracle_qmap, lib.oracle_qmap_uniform, lib.oracle_grid, lib.oracle_strength,
                  lib.oracle_amplitude, lib.oracle_backward):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def qmap(wavelength: float, theta_max_deg: float, n: int) -> np.ndarray:
    """Transfer momentum of every pixel of a flat n x n detector, shape (n*n, 3)."""
    out = np.empty((n * n, 3), np.float64)
    _load().oracle_qmap(float(wavelength), float(theta_max_deg), int(n), _ptr(out))
    return out


def qmap_uniform(wavelength: float, theta_max_deg: float, n: int) -> np.ndarray:
    """Transfer momentum of every pixel of the uniform transverse-q virtual detector,
    shape (n*n, 3); q_z is NaN where no outgoing wave exists."""
    out = np.empty((n * n, 3), np.float64)
    _load().oracle_qmap_uniform(float(wavelength), float(theta_max_deg), int(n), _ptr(out))
    return out


def grid(n: int, d: float) -> np.ndarray:
    """Voxel centres of n cells of pitch d, centred on the origin."""
    out = np.empty(n, np.float64)
    _load().oracle_grid(int(n), float(d), _ptr(out))
    return out


def strength(mode: int, delta, beta, pitch, wavelength: float) -> np.ndarray:
    """Effective scattering strength w (complex128, same [x][y][z] shape as delta)."""
    delta, beta = _f64(delta), _f64(beta)
    nx, ny, nz = delta.shape
    out = np.empty(delta.shape + (2,), np.float64)
    dx, dy, dz = (float(v) for v in pitch)
    _load().oracle_strength(int(mode), nx, ny, nz, dx, dy, dz, float(wavelength),
                            _ptr(delta), _ptr(beta), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def amplitude(q, w, pitch, method: int = 1) -> np.ndarray:
    """A_p = sum_v w_v exp(-i q_p . r_v) for every row of q (complex128 vector)."""
    q = _f64(q).reshape(-1, 3)
    w = np.asarray(w)
    nx, ny, nz = w.shape
    wr = _f64(np.stack([w.real, w.imag], axis=-1))
    out = np.empty((q.shape[0], 2), np.float64)
    dx, dy, dz = (float(v) for v in pitch)
    _load().oracle_amplitude(int(method), _ptr(q), q.shape[0], nx, ny, nz, dx, dy, dz,
                             _ptr(wr), _ptr(out))
    return out[:, 0] + 1j * out[:, 1]


def backward(mode: int, q, g, A, delta, beta, pitch, wavelength: float, cols=None):
    """dL/d delta and dL/d beta for a loss with dL/dI = g over the pixels q.

    ``A`` are the oracle's own amplitudes of those pixels.  ``cols`` (flat a*ny+b
    column indices) restricts the output to some columns; the result then has
    shape (len(cols), nz), otherwise the shape of delta.
    """
    q = _f64(q).reshape(-1, 3)
    g = _f64(g).reshape(-1)
    A = np.asarray(A).reshape(-1)
    Ar = _f64(np.stack([A.real, A.imag], axis=-1))
    delta, beta = _f64(delta), _f64(beta)
    nx, ny, nz = delta.shape
    dx, dy, dz = (float(v) for v in pitch)
    if cols is None:
        colp, ncols, oshape = None, nx * ny, delta.shape
    else:
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        colp, ncols, oshape = _ptr(cols), cols.size, (cols.size, nz)
    gd = np.empty(ncols * nz, np.float64)
    gb = np.empty(ncols * nz, np.float64)
    _load().oracle_backward(int(mode), _ptr(q), q.shape[0], _ptr(g), _ptr(Ar), nx, ny, nz,
                            dx, dy, dz, float(wavelength), _ptr(delta), _ptr(beta),
                            colp, ncols, _ptr(gd), _ptr(gb))
    return gd.reshape(oshape), gb.reshape(oshape)


def simulate(mode: int, wavelength: float, theta_max_deg: float, n: int, delta, beta,
             pitch, pixels=None, method: int = 1):
    """Intensity |A|^2 of the pixels ``pixels`` (flat j*n+i, default all) and A itself."""
    q = qmap(wavelength, theta_max_deg, n)
    if pixels is not None:
        q = q[np.asarray(pixels, dtype=np.int64)]
    w = strength(mode, delta, beta, pitch, wavelength)
    A = amplitude(q, w, pitch, method)
    return np.abs(A) ** 2, A


def ylm(l: int, m: int, cos_theta: float, phi: float) -> float:
    """Real orthonormal spherical harmonic (m > 0: cos(m phi), m < 0: sin(|m| phi))."""
    return float(_load().oracle_ylm(int(l), int(m), float(cos_theta), float(phi)))


def render_sh(grid, pitch, coeffs, r0: float, edge: float, delta0: float, beta0: float):
    """Star body r0 (1 + sum c_lm Y_lm) as (delta, beta) on the centred grid; coeffs is a
    vector of (lmax + 1)^2 values at l*l + l + m; edge = 0 gives hard voxels."""
    c = _f64(coeffs).reshape(-1)
    lmax = int(round(np.sqrt(c.size))) - 1
    assert (lmax + 1) ** 2 == c.size
    nx, ny, nz = (int(v) for v in grid)
    dx, dy, dz = (float(v) for v in pitch)
    d = np.empty((nx, ny, nz), np.float64)
    b = np.empty((nx, ny, nz), np.float64)
    _load().oracle_render_sh(nx, ny, nz, dx, dy, dz, lmax, _ptr(c), float(r0), float(edge),
                             float(delta0), float(beta0), _ptr(d), _ptr(b))
    return d, b


def render_sh_backward(grid, pitch, coeffs, r0, edge, delta0, beta0, grad_delta, grad_beta):
    """dL/dc for a loss with dL/d delta = grad_delta, dL/d beta = grad_beta (edge > 0)."""
    c = _f64(coeffs).reshape(-1)
    lmax = int(round(np.sqrt(c.size))) - 1
    nx, ny, nz = (int(v) for v in grid)
    dx, dy, dz = (float(v) for v in pitch)
    gd, gb = _f64(grad_delta), _f64(grad_beta)
    out = np.empty(c.size, np.float64)
    _load().oracle_render_sh_backward(nx, ny, nz, dx, dy, dz, lmax, _ptr(c), float(r0), float(edge),
                                      float(delta0), float(beta0), _ptr(gd), _ptr(gb), _ptr(out))
    return out


def render_ellipsoid(grid, pitch, axes, rot, edge: float, delta0: float, beta0: float):
    """Ellipsoid with semi-axes along the columns of rot (3 x 3) as (delta, beta)."""
    nx, ny, nz = (int(v) for v in grid)
    dx, dy, dz = (float(v) for v in pitch)
    ax = _f64(axes).reshape(3)
    R = _f64(rot).reshape(9)
    d = np.empty((nx, ny, nz), np.float64)
    b = np.empty((nx, ny, nz), np.float64)
    _load().oracle_render_ellipsoid(nx, ny, nz, dx, dy, dz, _ptr(ax), _ptr(R), float(edge),
                                    float(delta0), float(beta0), _ptr(d), _ptr(b))
    return d, b


def render_volume(grid, pitch, src_delta, src_beta, src_pitch):
    """A (delta, beta) volume map on its own centred grid resampled at the centres of
    `grid` by trilinear interpolation, zero beyond the source grid."""
    sd, sb = _f64(src_delta), _f64(src_beta)
    sx, sy, sz = sd.shape
    nx, ny, nz = (int(v) for v in grid)
    dx, dy, dz = (float(v) for v in pitch)
    sdx, sdy, sdz = (float(v) for v in src_pitch)
    d = np.empty((nx, ny, nz), np.float64)
    b = np.empty((nx, ny, nz), np.float64)
    _load().oracle_render_volume(nx, ny, nz, dx, dy, dz, sx, sy, sz, sdx, sdy, sdz, _ptr(sd),
                                 _ptr(sb), _ptr(d), _ptr(b))
    return d, b


def philox(counter, key) -> np.ndarray:
    """Philox4x64-10 of a 4-word counter under a 2-word key: four uint64 words."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, np.uint64)
    _load().oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def pixel_solid_angle(theta_max_deg: float, n: int, i: int, j: int) -> float:
    """Solid angle of pixel (i, j) of the flat N x N detector."""
    return float(_load().oracle_pixel_solid_angle(theta_max_deg, n, i, j))


def detect_ideal(wavelength: float, theta_max_deg: float, n: int, intensity, fluence: float,
                 seed: int):
    """(expected counts, Poisson counts), both [N*N] float64, of an intensity [N*N] on
    the flat detector for an incident fluence (photons per unit area)."""
    I = _f64(intensity).reshape(-1)
    assert I.size == n * n
    mu = np.empty(n * n, np.float64)
    counts = np.empty(n * n, np.float64)
    _load().oracle_detect_ideal(wavelength, theta_max_deg, n, _ptr(I), float(fluence),
                                int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(mu), _ptr(counts))
    return mu, counts
