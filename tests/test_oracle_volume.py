"""Pins for the oracle's forward volume V0(n, d0) (Sec. 2.2, five-case volume).

Independent checks: exact rational inclusion-exclusion over the 8 cube corners,
brute-force sub-cell counting, and the symmetries of the problem.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest


def exact_reduced_volume(a, u):
    """Volume of {z in [0,1]^3 : a.z <= u}, a_k > 0, exact rational arithmetic:
    inclusion-exclusion over the corners v of the cube,
    sum_v (-1)^|v| max(u - a.v, 0)^3 / (6 a1 a2 a3)."""
    tot = Fraction(0)
    for v in itertools.product((0, 1), repeat=3):
        s = u - sum(ak * vk for ak, vk in zip(a, v))
        if s > 0:
            tot += (-1) ** sum(v) * s ** 3
    return tot / (6 * a[0] * a[1] * a[2])


def test_volume_matches_exact_inclusion_exclusion(orc):
    rng = np.random.default_rng(1)
    worst = 0.0
    for trial in range(400):
        # dyadic rationals: exactly representable in float64
        if trial % 4 == 0:
            a = [Fraction(int(rng.integers(1, 64)), 1 << 16) for _ in range(2)] + \
                [Fraction(int(rng.integers(1 << 10, 1 << 12)), 1 << 12)]
        else:
            a = [Fraction(int(rng.integers(1, 1 << 20)), 1 << 20) for _ in range(3)]
        S = sum(a)
        u = Fraction(int(rng.integers(0, 1 << 24)), 1 << 24) * S
        exact = float(exact_reduced_volume(a, u))
        signs = rng.choice([-1.0, 1.0], size=3)
        perm = rng.permutation(3)
        n = [float(a[p]) * s for p, s in zip(perm, signs)]
        d0 = float(u - S / 2)
        got = orc.volume1(*n, d0)
        worst = max(worst, abs(got - exact))
    assert worst <= 2e-15


def test_volume_voxel_count(orc):
    """Fraction of K^3 sub-cell centres below the plane converges to V0."""
    rng = np.random.default_rng(2)
    K = 160
    o = (np.arange(K) + 0.5) / K - 0.5
    X, Y, Z = np.meshgrid(o, o, o, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    for _ in range(40):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        S = np.abs(n).sum()
        d0 = rng.uniform(-S / 2, S / 2)
        frac = np.mean(pts @ n <= d0)
        assert abs(frac - orc.volume1(*n, d0)) < 2.0 / K


def test_volume_symmetries_and_endpoints(orc):
    rng = np.random.default_rng(3)
    for _ in range(500):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        S = np.abs(n).sum()
        d0 = rng.uniform(-S / 2, S / 2)
        v = orc.volume1(*n, d0)
        # complement: the half-space n.x >= d0 is the region for (n, -d0) mirrored
        assert abs(orc.volume1(*n, -d0) - (1.0 - v)) <= 1e-15
        assert abs(orc.volume1(*(-n), -d0) - (1.0 - v)) <= 1e-15
        # mirroring one axis and permuting axes leave the volume unchanged
        m = n.copy()
        m[rng.integers(0, 3)] *= -1
        assert orc.volume1(*m, d0) == v
        assert orc.volume1(*n[rng.permutation(3)], d0) == v
        # scaling (n, d0) together describes the same plane
        assert abs(orc.volume1(*(2.5 * n), 2.5 * d0) - v) <= 1e-15
        assert abs(orc.volume1(*n, -S / 2)) <= 1e-15
        assert abs(orc.volume1(*n, S / 2) - 1.0) <= 1e-15


def test_volume_monotone(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        n = rng.standard_normal(3)
        S = np.abs(n).sum()
        d = np.linspace(-S / 2, S / 2, 2001)
        v = orc.volume(np.full_like(d, n[0]), np.full_like(d, n[1]), np.full_like(d, n[2]), d)
        assert np.all(np.diff(v) > 0)


def test_volume_special_normals(orc):
    # 1D: V0 = d0 + 1/2 (Sec. 2.3)
    for d0 in np.linspace(-0.5, 0.5, 11):
        assert abs(orc.volume1(0.0, -1.0, 0.0, d0) - (d0 + 0.5)) <= 1e-16
    # 2D face diagonal: V = d^2 for d = S/2 - |d0| (Sec. 2.3, d = sqrt(2 V n2 n3))
    h = 1.0 / np.sqrt(2.0)
    for d in np.linspace(0, h, 9):
        assert abs(orc.volume1(h, 0.0, h, d - h) - d * d / (2 * h * h)) <= 1e-15


def test_volume_nan_and_zero_normal(orc):
    assert np.isnan(orc.volume1(0.0, 0.0, 0.0, 0.0))
    assert np.isnan(orc.volume1(np.nan, 0.0, 1.0, 0.0))
    assert np.isnan(orc.volume1(0.0, 0.0, 1.0, np.nan))


def test_volume_at_case_boundaries_exact(orc):
    """At the case boundaries u in {a1, a2, a3, a1 + a2} (Sec. 2.2) the volume
    must still equal the exact inclusion-exclusion value.  The printed range of
    case (5), min(n1+n2, n3) <= d <= n3, is a single point d = n3 when
    n3 < n1 + n2 and selects the wrong formula there."""
    rng = np.random.default_rng(6)
    worst = 0.0
    for trial in range(300):
        a = sorted(Fraction(int(rng.integers(1, 1 << 20)), 1 << 20) for _ in range(3))
        S = sum(a)
        for u in (a[0], a[1], a[2], a[0] + a[1]):
            if u > S / 2:
                continue
            exact = float(exact_reduced_volume(a, u))
            got = orc.volume1(float(a[0]), float(a[1]), float(a[2]), float(u - S / 2))
            worst = max(worst, abs(got - exact))
    assert worst <= 2e-15


@pytest.mark.parametrize("a1", [1e-12, 1e-8, 1e-4])
def test_reduced_volume_small_n1_is_stable(orc, a1):
    """The divided form has no cancellation when n1 -> 0: compare with the exact
    rational value for a tiny first component."""
    a = [Fraction(a1), Fraction(0.6), Fraction(0.8)]
    for t in np.linspace(0.05, 0.95, 19):
        u = Fraction(float(t)) * sum(a) / 2
        exact = float(exact_reduced_volume(a, u))
        got = orc.reduced_volume(float(a[0]), 0.6, 0.8, float(u))
        assert abs(got - exact) <= 4e-16 * max(1.0, exact)
