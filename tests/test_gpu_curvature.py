"""GPU parity of plic_curvature against the FP64 oracle, cell by cell.

Tolerance per interface cell, on cells with a fit of 5 points or more whose
pivot ratio (largest / smallest LDL^T pivot, the oracle's conditioning proxy)
is at most 1e6: |kappa - kappa_ref| <= 1e-5 + 1e-3 |kappa_ref| in every
precision.  FP32 PLIC points carry errors of ~3e-7 in the heights, far below
this; an FP32 fit ("fp32") adds about (pivot ratio) * 2^-23 relative to the
coefficients, and the pivot ratios of these lattices stay below 40 (the
distribution of err/tol is printed: at most 0.009).  The remaining cells
(about 1 in 500 on a sphere) are checked for finiteness only: their fit is
decided by pivots near the rank threshold.  Non-interface and boundary cells
are exactly 0.
"""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import PRECISIONS, SOLVERS, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


def gpu_kappa(P, phi, solver="analytic", precision="mixed"):
    t = dev(phi)
    k = torch.empty_like(t)
    P.plic_curvature_f32(t, k, solver, precision)
    return host(k)


def cell_reference(orc, phi, normal="py", neighbour_normals=False):
    """Oracle kappa on the interface cells and their conditioning info."""
    kref, flags = orc.curvature(phi, flags=True, normal=normal, neighbour_normals=neighbour_normals)
    cells = np.flatnonzero(flags & 1)
    _, info = orc.curvature_cells(phi, cells, normal=normal, neighbour_normals=neighbour_normals)
    return cells, kref.ravel()[cells], info


def check_against(ref, phi, k, precision, report=""):
    cells, kr, info = ref
    good = (info[:, 0] >= 5) & (info[:, 2] <= 1e6)
    kg = k.ravel()[cells].astype(np.float64)
    tol = 1e-5 + 1e-3 * np.abs(kr)
    err = np.abs(kg - kr) / tol
    if precision == "fp32" and good.any():
        q = np.quantile(err[good], [0.5, 0.99, 0.999])
        print(f"{report}: FP32 fit, err/tol p50 {q[0]:.3g} p99 {q[1]:.3g} p99.9 {q[2]:.3g} "
              f"max {err[good].max():.3g}; largest pivot ratio {info[good, 2].max():.3g}")
    print(f"{report}: {cells.size} interface cells, {int((~good).sum())} loose; "
          f"max err/tol {err[good].max() if good.any() else 0:.3f}")
    assert np.isfinite(kg).all()
    if good.any():
        assert err[good].max() <= 1.0
    off = np.ones(phi.size, bool)
    off[cells] = False
    assert np.all(k.ravel()[off] == 0.0)
    return kg, kr, good


def check_cells(orc, phi, k, precision, report=""):
    return check_against(cell_reference(orc, phi), phi, k, precision, report)


@pytest.fixture(scope="module")
def sphere():
    return workloads.sphere_lattice(N=48, R=14.0, seed=0)[0]


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("solver", SOLVERS)
def test_sphere_parity(P, orc, sphere, solver, precision):
    k = gpu_kappa(P, sphere, solver, precision)
    check_cells(orc, sphere, k, precision, f"{solver}/{precision}")


def test_full_size_sphere(P, orc):
    """256^3 lattice, R = 40 sphere with a sub-cell jitter of the centre: every
    interface cell against the oracle; aggregate 2 kappa R/2 against 2/R."""
    for seed in (0, 1):
        phi, c = workloads.sphere_lattice(N=256, R=40.0, seed=seed)
        k = gpu_kappa(P, phi)
        kg, kr, good = check_cells(orc, phi, k, "mixed", f"256^3 R=40 seed {seed}")
        mean_g, mean_r = kg.mean() * 40.0, kr.mean() * 40.0
        E = np.abs(2 * kg - 2 / 40.0).sum() / (kg.size * 2 / 40.0)
        print(f"mean kappa R: gpu {mean_g:.6f} oracle {mean_r:.6f}; E(kappa) vs 2/R {E:.4f}")
        assert abs(mean_g - mean_r) <= 1e-4 * abs(mean_r)
        assert 0.97 < mean_r < 1.03


def test_full_size_sphere_other_solvers(P, orc):
    """The other three solvers' points on the 256^3 R = 40 sphere: every
    interface cell against the same oracle (its offsets do not depend on the
    solver)."""
    phi, _ = workloads.sphere_lattice(N=256, R=40.0, seed=0)
    ref = cell_reference(orc, phi)
    for solver in ("sz", "newton", "nested"):
        check_against(ref, phi, gpu_kappa(P, phi, solver, "mixed"), "mixed", f"256^3 {solver}")


@pytest.mark.parametrize("dims", [(67, 45, 37), (64, 4, 4), (65, 5, 5), (130, 9, 17)])
def test_ragged_lattices(P, orc, dims):
    """Lattice sizes that are not multiples of the 64x4x4 tile."""
    X, Y, Z = dims
    rng = np.random.default_rng(X * Y * Z)
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    c = np.array([X, Y, Z]) / 2.0 + rng.uniform(-0.3, 0.3, 3)
    R = 0.4 * min(X, Y, Z) + 3.0
    dist = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    phi = np.clip(R - dist + 0.5, 0.0, 1.0).astype(np.float32)   # smooth ramp across one cell
    for precision in PRECISIONS:
        k = gpu_kappa(P, phi, "sz", precision)
        check_cells(orc, phi, k, precision, f"{dims}/{precision}")


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 3, 3), (2, 9, 9), (9, 2, 9), (3, 4, 5)])
def test_tiny_lattices(P, orc, dims):
    X, Y, Z = dims
    rng = np.random.default_rng(sum(dims))
    phi = rng.choice(np.array([0.0, 1.0, 0.3, 0.7, 0.5], np.float32), size=(Z, Y, X))
    k = gpu_kappa(P, phi)
    check_cells(orc, phi, k, "mixed", f"{dims}")


def test_random_fill_levels(P, orc):
    """Every cell an interface cell with random fill levels: exercises tiles
    full of work and the rank rule; oracle parity on the well-conditioned ones."""
    rng = np.random.default_rng(5)
    phi = rng.uniform(0.01, 0.99, size=(12, 10, 70)).astype(np.float32)
    for precision in PRECISIONS:
        k = gpu_kappa(P, phi, "analytic", precision)
        check_cells(orc, phi, k, precision, f"random/{precision}")


def test_planes_and_complement(P, orc):
    n = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    N = 20
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    cc = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float64)
    d = n @ np.full(3, 9.5) + 0.1
    phi = orc.volume(np.full(cc.shape[0], n[0]), np.full(cc.shape[0], n[1]),
                     np.full(cc.shape[0], n[2]), d - cc @ n).reshape(N, N, N).astype(np.float32)
    for precision in PRECISIONS:
        k = gpu_kappa(P, phi, "analytic", precision)
        assert np.abs(k).max() <= 2e-5
    sph, _ = workloads.sphere_lattice(N=40, R=11.0, seed=4)
    k1 = gpu_kappa(P, sph, "analytic", "fp64")
    k2 = gpu_kappa(P, (1.0 - sph).astype(np.float32), "analytic", "fp64")
    assert np.max(np.abs(k1 + k2)) <= 1e-6


def test_determinism(P, sphere):
    a = gpu_kappa(P, sphere)
    b = gpu_kappa(P, sphere)
    assert np.array_equal(a, b)


def test_autograd_forward_matches_raw(P, sphere):
    t = dev(sphere)
    k = P.curvature(t)
    assert np.array_equal(host(k), gpu_kappa(P, sphere))


def interior_interface_count(phi):
    """Interface cells as defined for the fit: 0 < phi < 1, not on the outer layer."""
    inner = phi[1:-1, 1:-1, 1:-1]
    return int(((inner > 0) & (inner < 1)).sum())


@pytest.mark.parametrize("precision", PRECISIONS)
def test_forward_status_and_count(P, precision):
    """The status query after a forward reports the lattice's interface
    count, on the 256^3 sphere, a lattice of one tile and one without
    interface cells; repeated calls on one workspace give the same bits."""
    cases = [workloads.sphere_lattice(N=256, R=40.0, seed=0)[0],
             np.ascontiguousarray(workloads.sphere_lattice(N=12, R=3.0, seed=2)[0][4:8, 4:8, :]),
             np.zeros((9, 10, 11), np.float32)]
    for phi in cases:
        Z, Y, X = phi.shape
        t = dev(phi)
        ws = torch.empty(P.plic_curvature_workspace_bytes(X, Y, Z), dtype=torch.uint8, device="cuda")
        outs = []
        for _ in range(3):
            k = torch.empty_like(t)
            P.plic_curvature_f32(t, k, "sz", precision, ws)
            rc, cells, _ = P.plic_curvature_status(ws, X, Y, Z)
            assert rc == 0, P.plic_status_string(rc)
            assert cells == interior_interface_count(phi)
            outs.append(host(k))
        assert all(np.array_equal(outs[0], o) for o in outs[1:])
        if cells == 0:
            assert np.all(outs[0] == 0.0)


def test_vanishing_gradient_cells(P, orc):
    """Interface cells whose 26 neighbours all hold the same fill level have a
    zero fill-level gradient, hence no normal: kappa = 0 there (the oracle's
    rule |g| < 1e-12), and they pass nothing back in any backward (every
    variant, the reusing one included) even with a unit upstream gradient."""
    N = 24
    phi = np.zeros((N, N, N), np.float32)
    phi[6:18, 6:18, 6:18] = 0.5
    inner = np.zeros_like(phi, dtype=bool)
    inner[7:17, 7:17, 7:17] = True
    for precision in PRECISIONS:
        k = gpu_kappa(P, phi, "analytic", precision)
        assert np.all(k[inner] == 0.0)
        check_cells(orc, phi, k, precision, f"flat block {precision}")
    t = dev(phi)
    gk = torch.from_numpy(inner.astype(np.float32)).cuda()
    for normal, nbr in (("py", False), ("cm", False), ("py", True)):
        g = torch.full_like(t, float("nan"))
        P.plic_curvature_backward_ex_f32(t, gk, g, "analytic", "mixed", normal, nbr)
        assert int(torch.count_nonzero(g).item()) == 0, (normal, nbr)
    ws = torch.empty(P.plic_curvature_workspace_bytes(N, N, N), dtype=torch.uint8, device="cuda")
    kap = torch.empty_like(t)
    P.plic_curvature_f32(t, kap, "analytic", "mixed", ws)
    g = torch.full_like(t, float("nan"))
    P.plic_curvature_backward_reuse_f32(t, gk, g, "analytic", "mixed", "py", False, ws)
    assert int(torch.count_nonzero(g).item()) == 0
