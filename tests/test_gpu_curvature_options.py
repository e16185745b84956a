"""GPU parity of the curvature options against the FP64 oracle: the
centre-of-mass normal (forward and backward) and the neighbour-normal
variant (forward; its backward has a file of its own), with the per-cell bar
of the curvature tests; both at the benchmark's 256^3 sphere too, the
backward on sampled, isolated cells."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import PRECISIONS, SOLVERS, dev, host
from tests.test_gpu_curvature import cell_reference, check_against
from tests.test_gpu_curvature_grad import BARS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.fixture(scope="module")
def sphere():
    return workloads.sphere_lattice(N=48, R=14.0, seed=0)[0]


def gpu_kappa(P, phi, solver, precision, normal, nbr):
    t = dev(phi)
    k = torch.empty_like(t)
    P.plic_curvature_ex_f32(t, k, solver, precision, normal, nbr)
    return host(k)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("solver", SOLVERS)
def test_cm_normal_parity(P, orc, sphere, solver, precision):
    ref = cell_reference(orc, sphere, normal="cm")
    check_against(ref, sphere, gpu_kappa(P, sphere, solver, precision, "cm", False), precision,
                  f"cm {solver}/{precision}")


@pytest.mark.parametrize("normal", ["py", "cm"])
@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("solver", SOLVERS)
def test_neighbour_normals_parity(P, orc, sphere, solver, precision, normal):
    ref = cell_reference(orc, sphere, normal=normal, neighbour_normals=True)
    check_against(ref, sphere, gpu_kappa(P, sphere, solver, precision, normal, True), precision,
                  f"nbr {normal} {solver}/{precision}")


@pytest.mark.parametrize("shape", [(37, 35, 67), (9, 70, 13)])
def test_neighbour_normals_ragged(P, orc, shape):
    """Lattices that are not a multiple of the 64x4x4 tile, the interface
    crossing tile boundaries and reaching the outer layers."""
    Z, Y, X = shape
    N = max(shape)
    full, _, _ = workloads.perturbed_sphere_lattice(N=N, R=0.42 * min(shape), seed=4, ss=4)
    z0, y0, x0 = (N - Z) // 2, (N - Y) // 2, (N - X) // 2
    phi = np.ascontiguousarray(full[z0:z0 + Z, y0:y0 + Y, x0:x0 + X])
    assert ((phi > 0) & (phi < 1)).sum() > 50
    for normal in ("py", "cm"):
        ref = cell_reference(orc, phi, normal=normal, neighbour_normals=True)
        check_against(ref, phi, gpu_kappa(P, phi, "analytic", "mixed", normal, True), "mixed",
                      f"ragged {shape} {normal}")


@pytest.mark.parametrize("normal", ["py", "cm"])
def test_neighbour_normals_planes(P, orc, normal):
    N = 12
    for nrm, off in (((0.0, 0.0, 1.0), 0.3), ((1 / np.sqrt(2), 1 / np.sqrt(2), 0.0), 0.17)):
        n = np.array(nrm)
        r = np.arange(N) - N / 2
        z, y, x = np.meshgrid(r, r, r, indexing="ij")
        d0 = off - (n[0] * x + n[1] * y + n[2] * z)
        phi = orc.volume(np.full(d0.size, n[0]), np.full(d0.size, n[1]), np.full(d0.size, n[2]),
                         d0.ravel()).reshape(d0.shape).astype(np.float32)
        for precision in PRECISIONS:
            k = gpu_kappa(P, phi, "analytic", precision, normal, True)
            assert np.abs(k).max() <= 2e-6, (nrm, precision)


@pytest.fixture(scope="module")
def cm_case(orc):
    phi, _, _ = workloads.perturbed_sphere_lattice(N=36, R=11.0, seed=2, ss=4)
    kref, flags = orc.curvature(phi, flags=True, normal="cm")
    cells = np.flatnonzero(flags & 1)
    _, info = orc.curvature_cells(phi, cells, normal="cm")
    ok = (info[:, 0] >= 5) & (info[:, 2] <= 1e4)
    _, bad = orc.curvature_grad_richardson(phi, np.ones_like(phi), normal="cm")
    sel = cells[ok & ~bad.ravel()[cells]]
    gk = np.zeros(phi.size, np.float32)
    gk[sel] = np.random.default_rng(3).standard_normal(sel.size).astype(np.float32)
    gk = gk.reshape(phi.shape)
    gref, _ = orc.curvature_grad_richardson(phi, gk, normal="cm")
    return phi, gk, gref


@pytest.mark.parametrize("precision", PRECISIONS)
def test_cm_backward_matches_oracle(P, cm_case, precision):
    phi, gk, gref = cm_case
    tp, tg = dev(phi, gk)
    out = torch.empty_like(tp)
    P.plic_curvature_backward_ex_f32(tp, tg, out, "analytic", precision, "cm")
    err = np.abs(host(out).astype(np.float64) - gref).max() / np.abs(gref).max()
    print(f"cm backward {precision}: {err:.3e}")
    assert err <= BARS[precision]


def test_autograd_options(P, cm_case):
    phi, gk, gref = cm_case
    t = dev(phi).requires_grad_(True)
    (P.curvature(t, "analytic", "mixed", normal="cm") * dev(gk)).sum().backward()
    assert np.abs(host(t.grad).astype(np.float64) - gref).max() / np.abs(gref).max() <= BARS["mixed"]
    # the neighbour-normal variant differentiates too (its parity: test_gpu_curvature_nbr_grad)
    t2 = dev(phi).requires_grad_(True)
    k = P.curvature(t2, "analytic", "mixed", neighbour_normals=True)
    k.sum().backward()
    assert torch.isfinite(t2.grad).all()


@pytest.fixture(scope="module")
def bench_sphere():
    return workloads.sphere_lattice(N=256, R=40.0, seed=0)[0]


@pytest.mark.parametrize("normal, nbr", [("cm", False), ("py", True)])
def test_full_size_variants(P, orc, bench_sphere, normal, nbr):
    """The variants the benchmark times, on its 256^3 R = 40 sphere: every
    interface cell against the oracle."""
    phi = bench_sphere
    ref = cell_reference(orc, phi, normal=normal, neighbour_normals=nbr)
    check_against(ref, phi, gpu_kappa(P, phi, "analytic", "mixed", normal, nbr), "mixed",
                  f"256^3 {normal} neighbour_normals={nbr}")


@pytest.mark.parametrize("normal, nbr", [("cm", False), ("py", True)])
def test_full_size_variants_backward_sampled(P, orc, bench_sphere, normal, nbr):
    """The variants' backward on the benchmark's 256^3 sphere with the
    recommended workspace: isolated upstream cells (their gradients reach
    one cell, or two with neighbour normals, and do not overlap), each
    neighbourhood against the oracle's finite differences."""
    phi = bench_sphere
    _, flags = orc.curvature(phi, flags=True, normal=normal, neighbour_normals=nbr)
    cells = np.flatnonzero(flags & 1)
    _, info = orc.curvature_cells(phi, cells, normal=normal, neighbour_normals=nbr)
    ok = cells[(info[:, 0] >= 5) & (info[:, 2] <= 1e4)]
    H = 2 if nbr else 1
    rng = np.random.default_rng(11)
    pick = rng.choice(ok, 300, replace=False)
    Z, Y, X = phi.shape
    coords = np.stack([pick % X, (pick // X) % Y, pick // (X * Y)], 1)
    keep = []
    for i, c in enumerate(coords):
        if all(np.abs(c - coords[j]).max() > 2 * H for j in keep):
            keep.append(i)
    pick = pick[keep][:40]
    gk = np.zeros(phi.size, np.float32)
    gk[pick] = 1.0
    tp, tg = dev(phi, gk.reshape(phi.shape))
    out = torch.empty_like(tp)
    P.plic_curvature_backward_ex_f32(tp, tg, out, "analytic", "mixed", normal, nbr)
    g = host(out).astype(np.float64)
    worst, checked = 0.0, 0
    for c in pick:
        x, y, z = c % X, (c // X) % Y, c // (X * Y)
        blk = (slice(z - H, z + H + 1), slice(y - H, y + H + 1), slice(x - H, x + H + 1))
        nb = phi[blk].astype(np.float64).ravel()
        fd = orc.curv_cell_nbr_fd_grad if nbr else orc.curv_cell_fd_grad
        r1, bad1 = fd(nb, normal=normal, h=1e-5)
        r2, bad2 = fd(nb, normal=normal, h=2e-5)
        if bad1 or bad2:
            continue
        ref = (4.0 * r1 - r2) / 3.0                      # Richardson: O(h^2) term cancelled
        checked += 1
        worst = max(worst, np.abs(g[blk].ravel() - ref).max() / np.abs(ref).max())
    print(f"256^3 {normal} neighbour_normals={nbr} sampled backward: {checked} cells, worst {worst:.3e}")
    assert checked >= 20
    assert worst <= BARS["mixed"]
