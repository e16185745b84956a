"""Pins for the oracle's inverse d0(n, V0) (bisection on the forward volume).

Checked against the paper's closed forms evaluated at 50 digits
(tests/golden/plic_closed_forms.txt, written by make_plic_closed_forms.py from
Sec. 2.1 and 2.3), the 1D/2D/diagonal special cases, exact rational
bisection, the round trip V0(n, d0(n, V0)) = V0 (the paper's error E_i of
Sec. 2.6.2), the complement symmetry and the range endpoints.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

from tests.test_oracle_volume import exact_reduced_volume

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plic_closed_forms.txt")


def load_golden():
    rows = [ln.split() for ln in open(GOLDEN) if not ln.startswith("#")]
    arr = np.array([[float(x) for x in r[:5]] for r in rows])
    cases = np.array([int(r[5]) for r in rows])
    return arr, cases


def test_offset_matches_paper_closed_forms(orc):
    arr, cases = load_golden()
    assert set(cases.tolist()) == {1, 2, 3, 4, 5}
    d = orc.offset(arr[:, 0], arr[:, 1], arr[:, 2], arr[:, 3])
    assert np.max(np.abs(d - arr[:, 4])) <= 1e-15


def test_offset_special_normals(orc):
    for V0 in np.linspace(0, 1, 17):
        # 1D (Sec. 2.3): d = V, so d0 = V0 - 1/2
        assert abs(orc.offset1(0.0, 0.0, -1.0, V0) - (V0 - 0.5)) <= 1e-16
        # face diagonal: d = sqrt(2 V n2 n3) = sqrt(V)
        h = 1.0 / math.sqrt(2.0)
        V = min(V0, 1 - V0)
        ref = math.copysign(2 * h / 2 - math.sqrt(2 * V * h * h), V0 - 0.5) if V0 != 0.5 else 0.0
        assert abs(orc.offset1(h, -h, 0.0, V0) - ref) <= 2e-16
    # space diagonal, case (1): d = cbrt(6 V n1 n2 n3) while d < n1
    s = 1.0 / math.sqrt(3.0)
    for V0 in (1e-12, 1e-6, 0.01, 0.1, 1.0 / 6.0 - 1e-9):
        ref = -(1.5 * s - (6 * V0 * s ** 3) ** (1.0 / 3.0))
        assert abs(orc.offset1(s, s, -s, V0) - ref) <= 4e-16


def test_offset_case1_and_case5_closed_forms(orc):
    rng = np.random.default_rng(11)
    n_checked = [0, 0]
    for _ in range(4000):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        a1, a2, a3 = sorted(np.abs(n))
        V0 = rng.random()
        V = min(V0, 1 - V0)
        S = a1 + a2 + a3
        if 6 * V * a2 * a3 < a1 * a1:                       # case (1), a priori
            d = (6 * V * a1 * a2 * a3) ** (1.0 / 3.0)
            n_checked[0] += 1
        elif a1 + a2 <= 2 * V * a3:                          # case (5)
            d = V * a3 + 0.5 * (a1 + a2)
            n_checked[1] += 1
        else:
            continue
        ref = math.copysign(S / 2 - d, V0 - 0.5)
        assert abs(orc.offset1(*n, V0) - ref) <= 5e-16
    assert min(n_checked) > 100


def test_offset_endpoints_clamp_nan(orc):
    rng = np.random.default_rng(12)
    for _ in range(200):
        n = rng.standard_normal(3)
        S = np.abs(n).sum()
        assert orc.offset1(*n, 0.5) == 0.0
        # S summed in a different order here: allow a few ulps
        assert abs(orc.offset1(*n, 0.0) + S / 2) <= 4e-16
        assert abs(orc.offset1(*n, 1.0) - S / 2) <= 4e-16
        assert orc.offset1(*n, -0.25) == orc.offset1(*n, 0.0)
        assert orc.offset1(*n, 7.0) == orc.offset1(*n, 1.0)
    assert math.isnan(orc.offset1(0.0, 0.0, 0.0, 0.3))
    assert math.isnan(orc.offset1(0.3, math.nan, 0.1, 0.3))
    assert math.isnan(orc.offset1(0.3, 0.2, 0.1, math.nan))


def test_offset_round_trip_and_complement(orc):
    rng = np.random.default_rng(13)
    N = 20000
    n = rng.standard_normal((N, 3))
    n /= np.linalg.norm(n, axis=1)[:, None]
    V0 = rng.random(N)
    V0[:2000] *= 1e-9                      # tiny volumes (case 1, cube root sensitivity)
    V0[2000:3000] = 1 - V0[2000:3000] * 1e-9
    V0 = np.round(V0 * 2.0 ** 52) / 2.0 ** 52   # multiples of 2^-52: 1 - V0 is exact
    d = orc.offset(n[:, 0], n[:, 1], n[:, 2], V0)
    Vb = orc.volume(n[:, 0], n[:, 1], n[:, 2], d)
    assert np.max(np.abs(Vb - V0)) <= 1e-15
    dc = orc.offset(n[:, 0], n[:, 1], n[:, 2], 1.0 - V0)
    assert np.max(np.abs(dc + d)) <= 1e-15
    # monotone in V0 for a fixed normal
    v = np.linspace(0, 1, 4001)
    for k in range(20):
        dd = orc.offset(np.full_like(v, n[k, 0]), np.full_like(v, n[k, 1]), np.full_like(v, n[k, 2]), v)
        assert np.all(np.diff(dd) > 0)


def exact_bisection(a, V, steps=70):
    lo, hi = Fraction(0), sum(a) / 2
    for _ in range(steps):
        mid = (lo + hi) / 2
        if exact_reduced_volume(a, mid) < V:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def test_offset_matches_exact_rational_bisection(orc):
    rng = np.random.default_rng(14)
    for _ in range(40):
        a = sorted(Fraction(int(rng.integers(1, 1 << 20)), 1 << 20) for _ in range(3))
        V = Fraction(int(rng.integers(1, 1 << 23)), 1 << 24)      # V in (0, 1/2)
        u = exact_bisection(a, V)
        d0_exact = -(sum(a) / 2 - u)
        got = orc.offset1(float(a[0]), float(a[1]), float(a[2]), float(V))
        assert abs(got - float(d0_exact)) <= 1e-15


@pytest.mark.parametrize("V0", [0.0, 1.0])
def test_offset_kawano_edge_is_finite(orc, V0):
    """The SZ translation of the paper returns NaN for n = (1,0,0), V0 in {0,1}
    (Sec. 2.6.2); the definition gives -+1/2."""
    assert orc.offset1(1.0, 0.0, 0.0, V0) == (V0 - 0.5)
