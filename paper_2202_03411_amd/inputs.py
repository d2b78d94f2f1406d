"""Seeded synthetic inputs: shapes rendered to voxel grids of delta and beta.

This module holds no part of the scattering model; it only produces the voxel
maps of the complex refractive index n = 1 - delta + i beta (Eq. (7)) that both
the library and the FP64 oracle consume.  The shape families follow the ones the
paper's software offers (Sec. 5): a homogeneous sphere, ellipsoids with an
arbitrary orientation, and star-shaped bodies whose radius is a sum of spherical
harmonics (the triplet form of Sec. 5.2).  Where the paper leaves a convention
open, the choice made here is:

* spherical harmonics are the real orthonormal ones (cos(m phi) for m > 0,
  sin(|m| phi) for m < 0), theta polar from +z, phi the azimuth;
* a voxel is inside a hard shape iff its centre is inside the closed surface;
* soft voxelization uses occupancy sigmoid((r(theta, phi) - |r_v|) / eps);
* orientations are Haar-uniform rotations (unit quaternion from three uniforms).

Every generator takes an explicit seed; workload presets use
``SEED_BASE + index``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20220203

MODE_MSFT, MODE_BORN, MODE_DENSITY = 0, 1, 2


@dataclass
class Workload:
    """One simulation request: experiment + voxel map (float32 [x][y][z], z = beam)."""

    name: str
    wavelength: float
    theta_max_deg: float
    det_n: int
    pitch: tuple
    mode: int
    delta: np.ndarray
    beta: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def grid(self):
        return tuple(self.delta.shape)


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------

def centres(n: int, extent: float) -> np.ndarray:
    """Cell centres of n cells covering [-extent/2, extent/2]."""
    d = extent / n
    return (np.arange(n, dtype=np.float64) * 2.0 + 1.0 - n) * d / 2.0


def _mesh(n, extent):
    c = centres(n, extent)
    return np.meshgrid(c, c, c, indexing="ij")


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix (Shoemake's unit quaternion from 3 uniforms)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    qw = a * math.sin(2 * math.pi * u2)
    qx = a * math.cos(2 * math.pi * u2)
    qy = b * math.sin(2 * math.pi * u3)
    qz = b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


# --------------------------------------------------------------------------
# real spherical harmonics
# --------------------------------------------------------------------------

def sh_index(lmin: int, lmax: int):
    """(l, m) pairs for lmin <= l <= lmax, -l <= m <= l."""
    return [(l, m) for l in range(lmin, lmax + 1) for m in range(-l, l + 1)]


def real_sh(lmax: int, theta: np.ndarray, phi: np.ndarray) -> dict:
    """Real orthonormal spherical harmonics Y_lm(theta, phi) for l <= lmax.

    Uses the normalized associated Legendre recurrences (no Condon-Shortley
    phase), so the m > 0 functions carry cos(m phi) and m < 0 carry sin(|m| phi),
    each with norm 1 on the unit sphere.
    """
    x = np.cos(theta)
    s = np.sin(theta)
    qbar = {(0, 0): np.full_like(x, 1.0 / math.sqrt(4.0 * math.pi))}
    for m in range(1, lmax + 1):
        qbar[(m, m)] = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * qbar[(m - 1, m - 1)]
    for m in range(0, lmax):
        qbar[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * x * qbar[(m, m)]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            qbar[(l, m)] = a * (x * qbar[(l - 1, m)] - b * qbar[(l - 2, m)])
    out = {}
    for l in range(lmax + 1):
        out[(l, 0)] = qbar[(l, 0)]
        for m in range(1, l + 1):
            out[(l, m)] = math.sqrt(2.0) * qbar[(l, m)] * np.cos(m * phi)
            out[(l, -m)] = math.sqrt(2.0) * qbar[(l, m)] * np.sin(m * phi)
    return out


def sh_coefficients(rng: np.random.Generator, lmin: int, lmax: int, sigma: float):
    """Random real-SH coefficients c_lm ~ N(0, sigma^2) as [(l, m, c), ...]."""
    idx = sh_index(lmin, lmax)
    vals = rng.normal(0.0, sigma, size=len(idx))
    return [(l, m, float(v)) for (l, m), v in zip(idx, vals)]


def sh_radius(coeffs, r0: float, theta, phi):
    """r(theta, phi) = r0 (1 + sum c_lm Y_lm), the same harmonics as real_sh.

    Evaluated order by order with the same normalized recurrences, keeping only
    two degrees of the Legendre table at a time, so large grids fit in memory.
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    cmap = {}
    for l, m, c in coeffs:
        cmap[(l, m)] = cmap.get((l, m), 0.0) + c
    lmax = max((l for l, _ in cmap), default=0)
    x = np.cos(theta)
    s = np.sin(theta)
    acc = np.zeros_like(theta)
    qmm = np.full_like(theta, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(0, lmax + 1):
        if m > 0:
            qmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * qmm
        cos_m = np.cos(m * phi) if m > 0 else None
        sin_m = np.sin(m * phi) if m > 0 else None
        q_lm2, q_lm1 = None, qmm
        for l in range(m, lmax + 1):
            if l == m:
                q = qmm
            elif l == m + 1:
                q = math.sqrt(2.0 * m + 3.0) * x * qmm
            else:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                q = a * (x * q_lm1 - b * q_lm2)
            if l > m:
                q_lm2, q_lm1 = q_lm1, q
            if m == 0:
                c = cmap.get((l, 0), 0.0)
                if c:
                    acc += c * q
            else:
                cp, cn = cmap.get((l, m), 0.0), cmap.get((l, -m), 0.0)
                if cp:
                    acc += (cp * math.sqrt(2.0)) * q * cos_m
                if cn:
                    acc += (cn * math.sqrt(2.0)) * q * sin_m
    return r0 * (1.0 + acc)


def sh_radius_range(coeffs, r0: float, n_theta: int = 181, n_phi: int = 361):
    """(min, max) of r over a regular (theta, phi) grid."""
    th = np.linspace(0.0, math.pi, n_theta)
    ph = np.linspace(0.0, 2.0 * math.pi, n_phi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    r = sh_radius(coeffs, r0, T, P)
    return float(r.min()), float(r.max())


def _spherical(X, Y, Z):
    rr = np.sqrt(X * X + Y * Y + Z * Z)
    theta = np.arccos(np.clip(Z / np.where(rr > 0, rr, 1.0), -1.0, 1.0))
    phi = np.arctan2(Y, X)
    return rr, theta, phi


# --------------------------------------------------------------------------
# shape renderers
# --------------------------------------------------------------------------

def render_sphere(n: int, extent: float, radius: float, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Occupancy (1 inside the closed ball, else 0) as float32 [n][n][n]."""
    X, Y, Z = _mesh(n, extent)
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    return (r2 <= radius * radius).astype(np.float32)


def render_star(n: int, extent: float, coeffs, r0: float, soft_eps: float | None = None):
    """Occupancy of a star-shaped body r <= r0 (1 + sum c Y), hard or sigmoid-soft."""
    X, Y, Z = _mesh(n, extent)
    rr, th, ph = _spherical(X, Y, Z)
    rs = sh_radius(coeffs, r0, th, ph)
    if soft_eps is None:
        return (rr <= rs).astype(np.float32)
    return (1.0 / (1.0 + np.exp(-(rs - rr) / soft_eps))).astype(np.float32)


def render_ellipsoid(n: int, extent: float, axes, rot: np.ndarray) -> np.ndarray:
    """Occupancy of sum_i ((R^T r)_i / a_i)^2 <= 1."""
    X, Y, Z = _mesh(n, extent)
    P = np.stack([X, Y, Z], axis=-1) @ rot  # rows are r^T R = (R^T r)^T
    a = np.asarray(axes, dtype=np.float64)
    s = (P[..., 0] / a[0]) ** 2 + (P[..., 1] / a[1]) ** 2 + (P[..., 2] / a[2]) ** 2
    return (s <= 1.0).astype(np.float32)


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------

def sphere_workload(n: int = 32, det_n: int = 64, radius: float = 150.0,
                    wavelength: float = 45.0, theta_max_deg: float = 30.0) -> Workload:
    """Homogeneous sphere as a unit scattering density (first Born form factor check)."""
    extent = 2.0 * radius
    occ = render_sphere(n, extent, radius)
    d = extent / n
    return Workload("sphere_born", wavelength, theta_max_deg, det_n, (d, d, d), MODE_DENSITY,
                    occ, np.zeros_like(occ), {"radius": radius, "extent": extent})


def star_workload(n: int = 128, det_n: int = 512, lmax: int = 6, r0: float = 200.0,
                  sigma: float = 0.08, delta0: float = 0.01, beta0: float = 0.02,
                  wavelength: float = 45.0, theta_max_deg: float = 60.0,
                  seed: int = SEED_BASE + 1, voids: int = 0,
                  void_radius=(20.0, 60.0), name: str = "star") -> Workload:
    """Star-shaped harmonic body (1 <= l <= lmax, c_00 = 0), grid extent 2 r_max 1.02."""
    rng = np.random.default_rng(seed)
    coeffs = sh_coefficients(rng, 1, lmax, sigma)
    rmin, rmax = sh_radius_range(coeffs, r0)
    extent = 2.0 * rmax * 1.02
    d = extent / n
    occ = render_star(n, extent, coeffs, r0)
    void_list = []
    for _ in range(voids):
        rv = float(rng.uniform(*void_radius))
        lim = max(rmin - rv - 2.0 * d, 0.0)
        while True:
            c = rng.uniform(-lim, lim, size=3)
            if float(c @ c) <= lim * lim:
                break
        void_list.append((tuple(float(v) for v in c), rv))
        occ = occ * (1.0 - render_sphere(n, extent, rv, c))
    delta = (occ * delta0).astype(np.float32)
    beta = (occ * beta0).astype(np.float32)
    return Workload(name, wavelength, theta_max_deg, det_n, (d, d, d), MODE_MSFT, delta, beta,
                    {"coeffs": coeffs, "r0": r0, "extent": extent, "rmin": rmin, "rmax": rmax,
                     "voids": void_list, "seed": seed})


def pattern_workload() -> Workload:
    """128^3 star body (l <= 6, R0 = 200 nm), 512^2 detector to 60 deg, lambda = 45 nm."""
    return star_workload(n=128, det_n=512, lmax=6, r0=200.0, sigma=0.08, seed=SEED_BASE + 1,
                         name="star_l6_128c_512px")


def large_workload() -> Workload:
    """256^3 star body (l <= 10, R0 = 300 nm, 3 voids), 1024^2 detector to 80 deg, 13.5 nm."""
    return star_workload(n=256, det_n=1024, lmax=10, r0=300.0, sigma=0.08 * math.sqrt(48.0 / 120.0),
                         delta0=0.02, beta0=0.01, wavelength=13.5, theta_max_deg=80.0,
                         seed=SEED_BASE + 3, voids=3, name="star_l10_voids_256c_1024px")


def random_request(rng: np.random.Generator, grids=(64, 96, 128, 192), dets=(256, 512, 1024),
                   box: float = 700.0, wavelength: float = 45.0, theta_max_deg: float = 60.0,
                   delta0: float = 0.01, beta0: float = 0.02) -> Workload:
    """One serving request: a random ellipsoid or l <= 8 harmonic body in a fixed box."""
    n = int(rng.choice(grids))
    det = int(rng.choice(dets))
    d = box / n
    if rng.random() < 0.5:
        axes = rng.uniform(80.0, 250.0, size=3)
        rot = haar_rotation(rng)
        occ = render_ellipsoid(n, box, axes, rot)
        meta = {"kind": "ellipsoid", "axes": axes.tolist()}
    else:
        while True:
            r0 = float(rng.uniform(80.0, 170.0))
            coeffs = sh_coefficients(rng, 1, 8, 0.08)
            _, rmax = sh_radius_range(coeffs, r0, 91, 181)
            if rmax <= 340.0:
                break
        occ = render_star(n, box, coeffs, r0)
        meta = {"kind": "harmonic", "r0": r0}
    return Workload("request", wavelength, theta_max_deg, det, (d, d, d), MODE_MSFT,
                    (occ * delta0).astype(np.float32), (occ * beta0).astype(np.float32), meta)


def random_columns(shape, count: int, seed: int) -> np.ndarray:
    """Seeded distinct flat column indices a*ny + b of a grid."""
    rng = np.random.default_rng(seed)
    ncol = shape[0] * shape[1]
    return np.sort(rng.choice(ncol, size=min(count, ncol), replace=False)).astype(np.int64)


def random_pixels(det_n: int, count: int, seed: int) -> np.ndarray:
    """Seeded distinct flat pixel indices j*det_n + i."""
    rng = np.random.default_rng(seed)
    P = det_n * det_n
    return np.sort(rng.choice(P, size=min(count, P), replace=False)).astype(np.int64)
