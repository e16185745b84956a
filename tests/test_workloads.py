"""The seeded input generators (no GPU): every test and the benchmark draw their
inputs from them, so their distributions, edge-case mix and lattice geometry
are pinned here against what they promise."""
import math

import numpy as np

import workloads


def test_plic_problems_seeded_and_shaped():
    a = workloads.plic_problems(1 << 14, seed=5)
    b = workloads.plic_problems(1 << 14, seed=5)
    c = workloads.plic_problems(1 << 14, seed=6)
    for x, y in zip(a, b):
        assert x.dtype == np.float32 and x.flags["C_CONTIGUOUS"] and x.shape == (1 << 14,)
        assert np.array_equal(x, y)
    assert not np.array_equal(a[3], c[3])
    f64 = workloads.plic_problems(1 << 10, seed=5, dtype=np.float64)
    assert all(x.dtype == np.float64 for x in f64)


def test_plic_problems_distribution_and_edge_cases():
    n = 1 << 16
    nx, ny, nz, V0 = workloads.plic_problems(n, seed=1)
    nrm = np.sqrt(nx.astype(np.float64) ** 2 + ny.astype(np.float64) ** 2 + nz.astype(np.float64) ** 2)
    assert np.abs(nrm - 1.0).max() <= 4 * 2.0 ** -24
    assert V0.min() >= 0.0 and V0.max() <= 1.0
    # multiples of 2^-24, so that 1 - V0 is exact
    assert np.all(np.floor(V0.astype(np.float64) * 2 ** 24) == V0.astype(np.float64) * 2 ** 24)
    assert np.all((1.0 - V0).astype(np.float64) == 1.0 - V0.astype(np.float64))
    n_edge = int(round(0.02 * n))
    n_v = n_edge // 2
    n_ax = (n_edge - n_v) // 2
    n_fd = n_edge - n_v - n_ax
    assert ((V0 == 0.0) | (V0 == 1.0)).sum() >= n_v
    comps = np.stack([nx, ny, nz], 1)
    axis = (np.abs(comps) == 1.0).sum(1) == 1
    assert axis.sum() >= n_ax
    h = np.float32(1.0 / math.sqrt(2.0))
    face = ((np.abs(comps) == h).sum(1) == 2) & ((comps == 0.0).sum(1) == 1)
    assert face.sum() >= n_fd
    # the random normals are uniform on the sphere: each component has mean 0
    # and variance 1/3
    rnd = ~(axis | face)
    for k in range(3):
        assert abs(comps[rnd, k].mean()) < 0.02
        assert abs(comps[rnd, k].astype(np.float64).var() - 1.0 / 3.0) < 0.01


def test_paper_mix_normals():
    n = 1024
    nx, ny, nz = workloads.paper_mix_normals(n, seed=2)
    assert (nx[0], ny[0], nz[0]) == (1.0, 0.0, 0.0)
    h = np.float32(1.0 / math.sqrt(2.0))
    assert (nx[1], ny[1], nz[1]) == (h, h, 0.0)
    n2d = n // 8 - 2
    assert np.all(nz[2:2 + n2d] == 0.0)
    nrm = np.sqrt(nx.astype(np.float64) ** 2 + ny.astype(np.float64) ** 2 + nz.astype(np.float64) ** 2)
    assert np.abs(nrm - 1.0).max() <= 4 * 2.0 ** -24
    assert np.count_nonzero(nz[2 + n2d:]) == n - 2 - n2d


def test_near_degenerate_normals():
    n = 4096
    nrm, boundary, complement, jitter = workloads.near_degenerate_normals(n, seed=3, max_angle=1e-4)
    assert np.abs(np.linalg.norm(nrm, axis=1) - 1.0).max() < 1e-14
    dirs = np.vstack([np.eye(3), -np.eye(3), workloads._FACE, workloads._SPACE])
    cosines = np.clip(nrm @ dirs.T, -1.0, 1.0).max(1)
    assert np.arccos(cosines).max() <= 1e-4 * (1 + 1e-6)
    assert set(np.unique(boundary)) <= {0, 1, 2, 3, 4}
    assert complement.dtype == bool and 0.4 < complement.mean() < 0.6
    assert np.abs(jitter).max() <= 1e-6


def test_upstream_grad_is_standard_normal():
    g = workloads.upstream_grad((64, 64, 32), seed=4)
    assert g.dtype == np.float32 and g.shape == (64, 64, 32)
    assert abs(g.mean()) < 0.01 and abs(g.astype(np.float64).std() - 1.0) < 0.01


def test_sphere_lattice_volume_and_band():
    N, R = 40, 11.0
    phi, c = workloads.sphere_lattice(N=N, R=R, seed=7)
    assert phi.dtype == np.float32 and phi.shape == (N, N, N)
    assert phi.min() >= 0.0 and phi.max() <= 1.0
    assert np.abs(c - (N - 1) / 2.0).max() <= 0.15
    # the fill levels integrate to the sphere's volume (8^3 sub-points)
    assert abs(phi.astype(np.float64).sum() / (4.0 / 3.0 * math.pi * R ** 3) - 1.0) < 2e-3
    # interface cells only within sqrt(3)/2 of the surface
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    dist = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    iface = (phi > 0) & (phi < 1)
    assert np.abs(dist[iface] - R).max() <= math.sqrt(3.0) / 2.0
    assert np.all(phi[dist < R - 1.0] == 1.0) and np.all(phi[dist > R + 1.0] == 0.0)
    same, _ = workloads.sphere_lattice(N=N, R=R, seed=7)
    assert np.array_equal(phi, same)


def test_cylinder_lattice_area():
    N, R = 32, 9.0
    phi, c = workloads.cylinder_lattice(N=N, R=R, seed=1)
    per_slice = phi.astype(np.float64).sum(axis=(1, 2))
    assert np.allclose(per_slice, per_slice[0])
    assert abs(per_slice[0] / (math.pi * R ** 2) - 1.0) < 3e-3


def test_perturbed_sphere_lattice_volume():
    """The fill levels integrate to the volume of r(theta, phi) =
    R (1 + amp s), i.e. the integral of r^3 / 3 over the sphere of directions,
    and the rescaled coefficients give max |s| = 1."""
    N, R, amp = 48, 15.0, 0.05
    phi, c, a = workloads.perturbed_sphere_lattice(N=N, R=R, seed=3, amp=amp, ss=4)
    th, ph = np.meshgrid(np.linspace(0, math.pi, 361), np.linspace(0, 2 * math.pi, 721), indexing="ij")
    s = (workloads._real_sph_harm_basis(6, th.ravel(), ph.ravel()) @ a).reshape(th.shape)
    assert abs(np.abs(s).max() - 1.0) < 1e-12
    # midpoint quadrature of r^3/3 sin(theta) over the directions
    tq = (np.arange(400) + 0.5) * math.pi / 400
    pq = (np.arange(800) + 0.5) * 2 * math.pi / 800
    T, Pq = np.meshgrid(tq, pq, indexing="ij")
    sq = (workloads._real_sph_harm_basis(6, T.ravel(), Pq.ravel()) @ a).reshape(T.shape)
    vol = ((R * (1 + amp * sq)) ** 3 / 3.0 * np.sin(T)).sum() * (math.pi / 400) * (2 * math.pi / 800)
    assert abs(phi.astype(np.float64).sum() / vol - 1.0) < 5e-3
    assert np.abs(c - (N - 1) / 2.0).max() <= 0.15


def test_spherical_harmonic_series_matches_basis():
    """The perturbed sphere's radius series (Legendre recurrences, one term at
    a time) equals the basis-matrix form built on scipy's lpmv."""
    import math

    from scipy.special import lpmv

    x = np.linspace(-1.0, 1.0, 2001)
    P = workloads._assoc_legendre(6, x)
    for l in range(7):
        for m in range(l + 1):
            assert np.allclose(P[(l, m)], lpmv(m, l, x), rtol=1e-12, atol=1e-12)
    rng = np.random.default_rng(0)
    th, ph = rng.uniform(0, math.pi, 5000), rng.uniform(0, 2 * math.pi, 5000)
    a = rng.standard_normal(48)
    ref = workloads._real_sph_harm_basis(6, th, ph) @ a
    assert np.abs(workloads._real_sph_harm_series(6, a, th, ph) - ref).max() <= 1e-12
