"""Pins for the oracle's derivatives of d0(n, V0) (explicit polygon).

dd0/dV0 = |n| / A and dd0/dn = centroid of the plane-cube intersection polygon
(implicit differentiation of V0(n, d0) = volume of {x in cube : n.x <= d0}).
Checked against central finite differences of the (already pinned) inverse and
forward volume, the Euler identity n . dd0/dn = d0 of a degree-1 homogeneous
function, and the 1D closed form.
"""
import math

import numpy as np


def _random_problems(rng, N):
    n = rng.standard_normal((N, 3))
    n /= np.linalg.norm(n, axis=1)[:, None]
    V0 = rng.uniform(0.01, 0.99, N)
    return n, V0


def test_grad_V_matches_finite_difference(orc):
    rng = np.random.default_rng(21)
    n, V0 = _random_problems(rng, 3000)
    d0, dv, gx, gy, gz = orc.offset_grad(n[:, 0], n[:, 1], n[:, 2], V0)
    h = 1e-6
    dp = orc.offset(n[:, 0], n[:, 1], n[:, 2], V0 + h)
    dm = orc.offset(n[:, 0], n[:, 1], n[:, 2], V0 - h)
    fd = (dp - dm) / (2 * h)
    assert np.max(np.abs(dv - fd) / np.abs(fd)) < 2e-6


def test_grad_n_matches_finite_difference(orc):
    rng = np.random.default_rng(22)
    n, V0 = _random_problems(rng, 2000)
    d0, dv, gx, gy, gz = orc.offset_grad(n[:, 0], n[:, 1], n[:, 2], V0)
    g = np.stack([gx, gy, gz], 1)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        dp = orc.offset(*(n + e).T, V0)
        dm = orc.offset(*(n - e).T, V0)
        fd = (dp - dm) / (2 * h)
        assert np.max(np.abs(g[:, k] - fd)) < 2e-7


def test_grad_euler_identity_and_area(orc):
    rng = np.random.default_rng(23)
    n, V0 = _random_problems(rng, 2000)
    d0, dv, gx, gy, gz = orc.offset_grad(n[:, 0], n[:, 1], n[:, 2], V0)
    # the centroid lies on the plane: n . x_bar = d0
    assert np.max(np.abs(n[:, 0] * gx + n[:, 1] * gy + n[:, 2] * gz - d0)) <= 1e-13
    # area = |n| dV0/dd0 by finite differences of the forward volume
    h = 1e-6
    A_fd = (orc.volume(*n.T, d0 + h) - orc.volume(*n.T, d0 - h)) / (2 * h)
    assert np.max(np.abs(1.0 / dv - A_fd)) < 1e-7


def test_grad_1d_closed_form(orc):
    for V0 in (0.0, 0.2, 0.5, 0.9, 1.0):
        d0, dv, g, area, nv = orc.offset_grad1(1.0, 0.0, 0.0, V0)
        assert abs(area - 1.0) < 1e-15 and abs(dv - 1.0) < 1e-15
        assert np.allclose(g, [V0 - 0.5, 0.0, 0.0], atol=1e-15)


def test_grad_face_diagonal_closed_form(orc):
    """n = (1,1,0)/sqrt2, V <= 1/2, d = sqrt(V): below the plane lies the prism
    over the triangle z1 + z2 <= sqrt(2) d, so the polygon is a rectangle of
    height 1 and width sqrt(2) * sqrt(2) d = 2 d; its centroid is the midpoint of
    the cut."""
    h = 1.0 / math.sqrt(2.0)
    for V0 in (0.05, 0.2, 0.45):
        d = math.sqrt(V0)
        d0, dv, g, area, nv = orc.offset_grad1(h, h, 0.0, V0)
        assert abs(area - 2.0 * d) < 1e-14
        # corner at (-1/2,-1/2); the cut runs from (-1/2 + sqrt2 d, -1/2) to (-1/2, -1/2 + sqrt2 d)
        c = -0.5 + math.sqrt(2.0) * d / 2
        assert np.allclose(g, [c, c, 0.0], atol=1e-14)


def test_grad_degenerate_polygon(orc):
    n = np.array([0.3, 0.5, 0.8])
    n /= np.linalg.norm(n)
    d0, dv, g, area, nv = orc.offset_grad1(*n, 0.0)
    assert area == 0.0 and math.isinf(dv)
    assert np.allclose(g, [-0.5, -0.5, -0.5])
