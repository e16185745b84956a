"""Pins for the oracle's PLIC curvature (Sec. 4.2 and Appendix B).

Checked against: exact recovery of synthetic paraboloids by the least-squares
fit (B.3), the textbook mean curvature of a Monge patch from its fundamental
forms (B.2), planes (zero curvature), the sphere (1/R) and the cylinder (1/(2R))
of the paper's validation (Sec. 4.3), rotation invariance of the fit in the
tangent plane (independence of the auxiliary vector r), lattice symmetries, the
fluid/gas complement, and the Parker-Youngs normal error (B.1).
"""
import math

import numpy as np
import pytest

import workloads


def textbook_mean_curvature(fx, fy, fxx, fyy, fxy):
    """H = (e G - 2 f F + g E) / (2 (E G - F^2)) of the Monge patch z = f(x, y)
    with unit normal (-fx, -fy, 1)/W (first form E, F, G; second form e, f, g)."""
    E, F, G = 1 + fx * fx, fx * fy, 1 + fy * fy
    W = math.sqrt(1 + fx * fx + fy * fy)
    e, f, g = fxx / W, fxy / W, fyy / W
    return (e * G - 2 * f * F + g * E) / (2 * (E * G - F * F))


def test_paraboloid_kappa_matches_fundamental_forms(orc):
    rng = np.random.default_rng(31)
    for _ in range(200):
        A, B, C, H, I = rng.standard_normal(5)
        ref = textbook_mean_curvature(H, I, 2 * A, 2 * B, C)
        assert abs(orc.paraboloid_kappa([A, B, C, H, I]) - ref) <= 1e-14 * max(1, abs(ref))
    # H = I = 0: kappa = A + B; osculating paraboloid of a sphere: 1/R
    assert orc.paraboloid_kappa([0.3, -0.1, 5.0, 0.0, 0.0]) == pytest.approx(0.2, abs=1e-16)
    R = 7.0
    assert orc.paraboloid_kappa([1 / (2 * R), 1 / (2 * R), 0, 0, 0]) == pytest.approx(1 / R)


def test_fit_recovers_exact_paraboloid(orc):
    rng = np.random.default_rng(32)
    for npts in (5, 8, 12, 26):
        for _ in range(50):
            coef = rng.standard_normal(5)
            x = rng.uniform(-1.5, 1.5, npts)
            y = rng.uniform(-1.5, 1.5, npts)
            z = coef[0] * x * x + coef[1] * y * y + coef[2] * x * y + coef[3] * x + coef[4] * y
            got, bits, cond = orc.fit_paraboloid(x, y, z)
            assert bits == 31
            assert np.max(np.abs(got - coef)) <= 1e-11 * max(1.0, cond ** 0.5)


def test_fit_reduced_dimension_and_rank_rule(orc):
    # fewer than 5 points: leading k x k block (A, B, C for k = 3), the rest 0
    x = np.array([1.0, 0.0, 1.0])
    y = np.array([0.0, 1.0, 1.0])
    z = 0.5 * x * x - 0.25 * y * y + 0.1 * x * y
    coef, bits, _ = orc.fit_paraboloid(x, y, z)
    assert bits == 0b111
    assert np.allclose(coef, [0.5, -0.25, 0.1, 0, 0], atol=1e-14)
    # points on the x-axis only: y^2, xy and y columns vanish -> dropped
    x = np.array([-1.0, -0.5, 0.5, 1.0, 2.0, 1.5])
    y = np.zeros_like(x)
    z = 0.3 * x * x + 0.2 * x
    coef, bits, _ = orc.fit_paraboloid(x, y, z)
    assert bits == 0b01001
    assert np.allclose(coef, [0.3, 0, 0, 0.2, 0], atol=1e-13)


def plane_lattice(orc, n, d, N=12):
    """phi of the half-space n.x <= d (x in lattice units) cell by cell, from the
    (pinned) forward volume: the cell at c holds V0(n, d - n.c)."""
    n = np.asarray(n, dtype=np.float64)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    c = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float64)
    v = orc.volume(np.full(c.shape[0], n[0]), np.full(c.shape[0], n[1]),
                   np.full(c.shape[0], n[2]), d - c @ n)
    return v.reshape(N, N, N).astype(np.float32)


@pytest.mark.parametrize("n", [(0, 0, 1), (0, -1, 0), (1, 1, 0), (0, 1, -1), (1, 1, 1)])
def test_planes_have_zero_curvature(orc, n):
    n = np.asarray(n, float)
    n /= np.linalg.norm(n)
    phi = plane_lattice(orc, n, float(n @ np.full(3, 5.5)) + 0.123)
    k, fl = orc.curvature(phi, flags=True)
    assert (fl & 1).sum() > 10
    # the Parker-Youngs normal is exact by symmetry for these planes; what is
    # left comes from rounding phi to float32 (about 3e-8, so heights move by
    # ~1e-7); an axis-aligned plane has one phi per layer and gives exactly 0
    tol = 0.0 if np.count_nonzero(n) == 1 else 2e-6
    assert np.max(np.abs(k)) <= tol


def test_general_plane_curvature_is_small(orc):
    # Youngs' normal is not exact for a general plane, so kappa is small, not 0
    n = np.array([0.31, 0.52, 0.79])
    n /= np.linalg.norm(n)
    phi = plane_lattice(orc, n, float(n @ np.full(3, 5.5)) + 0.07)
    k, fl = orc.curvature(phi, flags=True)
    assert np.max(np.abs(k[(fl & 1) > 0])) < 0.05


@pytest.fixture(scope="module")
def sphere20():
    phi, c = workloads.sphere_lattice(N=56, R=20.0, seed=3)
    return phi, c


def test_sphere_mean_curvature(orc, sphere20):
    phi, c = sphere20
    k, fl = orc.curvature(phi, flags=True)
    sel = (fl & 1) > 0
    assert sel.sum() > 3000
    ratio = k[sel].mean() * 20.0
    assert 0.97 < ratio < 1.03          # kappa -> 1/R, positive for a drop
    E = np.abs(k[sel] - 1 / 20.0).sum() / (sel.sum() / 20.0)
    assert E < 0.3                      # L1 error E(kappa) of Sec. 4.3 (no relaxation)


def test_sphere_normal_is_radial_within_a_degree(orc, sphere20):
    phi, c = sphere20
    k, fl = orc.curvature(phi, flags=True)
    cells = np.flatnonzero((fl & 1) > 0)[::7]
    Z, Y, X = phi.shape
    angs = []
    for cc in cells:
        x, y, z = cc % X, (cc // X) % Y, cc // (X * Y)
        nb = phi[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].astype(np.float64).ravel()
        _, info, nrm, coef = orc.curv_cell(nb, full=True)
        rad = np.array([x, y, z]) - c
        rad /= np.linalg.norm(rad)
        angs.append(math.degrees(math.acos(min(1.0, float(nrm @ rad)))))
    assert np.mean(angs) < 2.0


def test_cylinder_mean_curvature(orc):
    R = 14.0
    phi, c = workloads.cylinder_lattice(N=44, R=R, seed=1)
    k, fl = orc.curvature(phi, flags=True)
    sel = (fl & 1) > 0
    # away from the z-boundary layers
    zz = np.arange(phi.shape[0])[:, None, None] * np.ones_like(phi)
    sel &= (zz > 2) & (zz < phi.shape[0] - 3)
    ratio = k[sel].mean() * 2 * R
    assert 0.95 < ratio < 1.05          # mean curvature 1/(2R), not 1/R


def test_complement_flips_sign(orc, sphere20):
    phi, _ = sphere20
    k = orc.curvature(phi)
    kc = orc.curvature((1.0 - phi).astype(np.float32))
    assert np.max(np.abs(k + kc)) <= 1e-12


def test_lattice_symmetry(orc, sphere20):
    """Permuting or mirroring the lattice axes permutes kappa.  Only cells with
    a full 5-parameter fit are compared: with fewer than 5 points the paper's
    reduced-dimension rule keeps the leading parameters of the local frame, and
    that frame depends on the fixed vector r, which the symmetry does not move."""
    phi, _ = sphere20
    k, fl = orc.curvature(phi, flags=True)
    full = fl == 1
    assert full.sum() > 3000
    kt = orc.curvature(np.ascontiguousarray(phi.transpose(2, 0, 1)))
    sel = full.transpose(2, 0, 1)
    assert np.max(np.abs(kt - k.transpose(2, 0, 1))[sel]) <= 1e-12
    kf = orc.curvature(np.ascontiguousarray(phi[:, ::-1, :]))
    assert np.max(np.abs(kf - k[:, ::-1, :])[full[:, ::-1, :]]) <= 1e-12


def test_independent_of_auxiliary_vector(orc, sphere20):
    """The 5-parameter quadratic is invariant under rotations of the tangent
    plane, so the choice of r changes kappa only at rounding level."""
    phi, _ = sphere20
    rng = np.random.default_rng(33)
    k, fl = orc.curvature(phi, flags=True)
    cells = np.flatnonzero(fl == 1)[::11]
    Z, Y, X = phi.shape
    for cc in cells:
        x, y, z = cc % X, (cc // X) % Y, cc // (X * Y)
        nb = phi[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].astype(np.float64).ravel()
        r = rng.standard_normal(3)
        r /= np.linalg.norm(r)
        k2, info, _ = orc.curv_cell_r(nb, r)
        if info[1] == 31:
            assert abs(k2 - k.ravel()[cc]) <= 1e-9 * max(1.0, info[2])


def test_fd_gradient_converges_and_respects_complement(orc, sphere20):
    phi, _ = sphere20
    k, fl = orc.curvature(phi, flags=True)
    cells = np.flatnonzero(fl == 1)[::97][:20]
    Z, Y, X = phi.shape
    for cc in cells:
        x, y, z = cc % X, (cc // X) % Y, cc // (X * Y)
        nb = phi[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].astype(np.float64).ravel()
        if np.any((nb > 0) & (nb < 1e-4)) or np.any((nb < 1) & (nb > 1 - 1e-4)):
            continue
        g1, bad1 = orc.curv_cell_fd_grad(nb, h=1e-6)
        g2, bad2 = orc.curv_cell_fd_grad(nb, h=2e-6)
        if bad1 or bad2:
            continue
        scale = max(1.0, np.abs(g1).max())
        assert np.max(np.abs(g1 - g2)) <= 1e-6 * scale
        # kappa(phi) = -kappa(1 - phi)  =>  the gradient is the same at 1 - phi
        mask = (nb > 0) & (nb < 1)
        gc, badc = orc.curv_cell_fd_grad(1.0 - nb, mask, h=1e-6)
        assert np.max(np.abs(gc - g1)) <= 1e-6 * scale


def test_lattice_gradient_is_directional_derivative_of_forward(orc):
    """The lattice gradient (per-cell differences scattered into grad_phi) is
    pinned by a directional derivative of the lattice forward: for a random
    direction v on the cells that keep the interface mask, grad . v equals
    d/de sum(gk * kappa(phi + e v)) at e = 0 (central differences with
    Richardson extrapolation, float32 lattice rounding aside).  A wrong
    scatter index or neighbour order fails it.  Richardson's extrapolation
    (h = 1e-5 against 2e-5) agrees with plain differences at h = 1e-6."""
    phi, _, _ = workloads.perturbed_sphere_lattice(N=24, R=7.0, seed=3, ss=4)
    rng = np.random.default_rng(9)
    iface = (phi > 0) & (phi < 1)
    gk = np.where(iface, rng.standard_normal(phi.shape), 0.0).astype(np.float32)
    _, bad = orc.curvature_grad_richardson(phi, gk, h=1e-5)
    gk[bad] = 0.0                                   # cells whose differences are inadmissible
    g, _ = orc.curvature_grad_richardson(phi, gk, h=1e-5)
    g6, _ = orc.curvature_grad(phi, gk, h=1e-6)
    scale = np.abs(g).max()
    assert scale > 0
    assert np.abs(g - g6).max() <= 1e-8 * scale
    # direction on the cells whose perturbation keeps them strictly inside (0,1) or at 0/1
    movable = iface & (phi > 0.05) & (phi < 0.95)
    worst = 0.0
    for trial in range(3):
        v = np.where(movable, rng.standard_normal(phi.shape), 0.0)
        eps = 1e-3

        def K(e):
            k = orc.curvature((phi + e * v).astype(np.float32))
            return float((k * gk).sum())

        dK = (8 * (K(eps) - K(-eps)) - (K(2 * eps) - K(-2 * eps))) / (12 * eps)
        gv = float((g * v).sum())
        worst = max(worst, abs(dK - gv) / max(abs(gv), 1e-12))
    print(f"directional derivative: worst relative error {worst:.2e}, {int(bad.sum())} inadmissible cells")
    assert worst <= 2e-3
