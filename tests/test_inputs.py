"""The seeded input generators (no model arithmetic): harmonic shapes and
renderers checked against library routines and closed forms."""
import math

import numpy as np
import scipy.special as sp

from paper_2202_03411_amd import inputs


def test_real_harmonics_match_scipy_convention():
    rng = np.random.default_rng(0)
    th = rng.uniform(0, np.pi, 500)
    ph = rng.uniform(-np.pi, np.pi, 500)
    Y = inputs.real_sh(8, th, ph)
    for l in range(9):
        for m in range(-l, l + 1):
            y = sp.sph_harm_y(l, abs(m), th, ph)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * y.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * y.imag
            else:
                ref = y.real
            assert np.allclose(Y[(l, m)], ref, atol=1e-12)


def test_sh_radius_streaming_equals_table():
    rng = np.random.default_rng(1)
    th = rng.uniform(0, np.pi, 300)
    ph = rng.uniform(-np.pi, np.pi, 300)
    coeffs = inputs.sh_coefficients(rng, 0, 10, 0.1)
    Y = inputs.real_sh(10, th, ph)
    ref = 150.0 * (1 + sum(c * Y[(l, m)] for l, m, c in coeffs))
    assert np.allclose(inputs.sh_radius(coeffs, 150.0, th, ph), ref, rtol=0, atol=1e-10)


def test_sphere_voxel_count_and_symmetry():
    occ = inputs.render_sphere(32, 300.0, 150.0)
    # closed ball: the voxelized volume is within a few percent of 4/3 pi R^3
    vol = occ.sum() * (300.0 / 32) ** 3
    assert abs(vol / (4.0 / 3.0 * math.pi * 150.0 ** 3) - 1.0) < 0.03
    assert np.array_equal(occ, occ[::-1, :, :]) and np.array_equal(occ, occ.transpose(1, 2, 0))


def test_ellipsoid_identity_rotation_and_haar():
    occ = inputs.render_ellipsoid(48, 480.0, (200.0, 100.0, 50.0), np.eye(3))
    c = inputs.centres(48, 480.0)
    # extent along each axis equals the semi-axis within one pitch
    for ax, a in enumerate((200.0, 100.0, 50.0)):
        proj = occ.any(axis=tuple(k for k in range(3) if k != ax))
        assert abs(c[proj].max() - a) <= 10.0
    R = inputs.haar_rotation(np.random.default_rng(2))
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and abs(np.linalg.det(R) - 1.0) < 1e-12


def test_workloads_seeded_and_in_range():
    a = inputs.star_workload(n=32, det_n=16)
    b = inputs.star_workload(n=32, det_n=16)
    assert np.array_equal(a.delta, b.delta)
    assert set(np.unique(a.delta)) <= {0.0, np.float32(0.01)}
    rmin, rmax = a.meta["rmin"], a.meta["rmax"]
    assert 0 < rmin < 200.0 < rmax
    assert math.isclose(a.meta["extent"], 2 * rmax * 1.02)
