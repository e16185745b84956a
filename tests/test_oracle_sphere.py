"""Oracle pins for the plane-sphere intersection (Sec. 3): the cap volume of
the unit-volume sphere against quadrature of its cross-sections and a voxel
count, and the bisection inverse against the volume, its symmetries and its
end points."""
import numpy as np
import pytest


def test_cap_volume_by_quadrature(orc):
    """V(d0) = integral from -r to d0 of the disc area pi (r^2 - x^2), by
    Gauss-Legendre quadrature (exact for this quadratic integrand)."""
    r = orc.sphere_radius()
    assert abs(4.0 / 3.0 * np.pi * r ** 3 - 1.0) < 1e-15
    xg, wg = np.polynomial.legendre.leggauss(4)
    d = np.linspace(-r, r, 201)
    quad = np.array([np.sum(0.5 * (di + r) * wg * np.pi * (r * r - (0.5 * (di + r) * xg + 0.5 * (di - r)) ** 2))
                     for di in d])
    assert np.max(np.abs(orc.sphere_volume(d) - quad)) < 1e-14


def test_cap_volume_voxel_count(orc):
    """Fraction of grid points of the ball below the plane, converging as
    O(1/K) to the cap volume."""
    r = orc.sphere_radius()
    K = 160
    g = (np.arange(K) + 0.5) / K * 2 * r - r
    z, y, x = np.meshgrid(g, g, g, indexing="ij", sparse=True)
    inside = (x * x + y * y + z * z) <= r * r
    for d0 in (-0.4, -0.1, 0.0, 0.23, 0.5):
        frac = np.count_nonzero(inside & (z <= d0)) / np.count_nonzero(inside)
        assert abs(frac - orc.sphere_volume(np.array([d0]))[0]) < 8.0 / K


def test_end_points_and_centre(orc):
    r = orc.sphere_radius()
    v = orc.sphere_volume(np.array([-2 * r, -r, 0.0, r, 2 * r]))
    assert v[0] == 0.0 and v[1] == 0.0 and abs(v[2] - 0.5) < 1e-15 and v[3] == 1.0 and v[4] == 1.0
    d = orc.sphere_offset(np.array([-0.5, 0.0, 0.5, 1.0, 1.5]))
    assert d[0] == -r and d[1] == -r and abs(d[2]) < 1e-15 and d[3] == r and d[4] == r
    assert np.isnan(orc.sphere_offset(np.array([np.nan]))[0])


def test_inverse_round_trip_symmetry_monotone(orc):
    rng = np.random.default_rng(0)
    V = np.sort(rng.random(20001))
    d = orc.sphere_offset(V)
    assert np.max(np.abs(orc.sphere_volume(d) - V)) < 1e-15
    assert np.all(np.diff(d) >= 0)
    # d0'(V0) = 1 / A with A = pi (r^2 - d0^2) the cross-section: rounding of
    # the volume (and of 1 - V0) moves the root by about eps / A
    r = orc.sphere_radius()
    A = np.pi * (r * r - d * d)
    tol = 1e-15 + 4e-16 / np.maximum(A, 1e-12)
    assert np.all(np.abs(orc.sphere_offset(1.0 - V) + d) <= tol)
