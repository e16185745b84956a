"""GPU backward of the neighbour-normal curvature variant (each interface
neighbour's point from its own normal): stored rows with the adjoints of the
neighbours' own fill-level gradients, a second pass that sums them per
interface cell, and the deterministic gather; against the oracle's FP64
finite-difference gradient over each cell's 5^3 neighbourhood and against
central differences of the GPU forward.  The gradient reaches no further than
one cell from an interface cell (a neighbour's own normal reads that
neighbour's 3^3, and the neighbour is an interface cell)."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import PRECISIONS, dev, host
from tests.test_gpu_curvature_grad import BARS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


def band_of(phi):
    band = np.zeros(phi.shape, bool)
    iface = (phi > 0) & (phi < 1)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                band |= np.roll(iface, (dz, dy, dx), (0, 1, 2))
    return band


def make_case(orc, normal):
    """Perturbed sphere; upstream gradient N(0,1) on interface cells whose
    fit is well conditioned and whose finite differences keep the masks and
    the fit's parameter set."""
    phi, _, _ = workloads.perturbed_sphere_lattice(N=36, R=11.0, seed=2, ss=4)
    _, flags = orc.curvature(phi, flags=True, normal=normal, neighbour_normals=True)
    cells = np.flatnonzero(flags & 1)
    _, info = orc.curvature_cells(phi, cells, normal=normal, neighbour_normals=True)
    ok = (info[:, 0] >= 5) & (info[:, 2] <= 1e4)
    _, bad = orc.curvature_grad_richardson(phi, np.ones_like(phi), normal=normal, neighbour_normals=True)
    gk = np.zeros(phi.size, np.float32)
    rng = np.random.default_rng(5)
    sel = cells[ok & ~bad.ravel()[cells]]
    gk[sel] = rng.standard_normal(sel.size).astype(np.float32)
    gk = gk.reshape(phi.shape)
    gref, _ = orc.curvature_grad_richardson(phi, gk, normal=normal, neighbour_normals=True)
    return phi, gk, gref, sel


@pytest.fixture(scope="module")
def case(orc):
    return make_case(orc, "py")


def gpu_grad(P, phi, gk, solver="analytic", precision="mixed", normal="py", workspace=None, check=True):
    tp, tg = dev(phi, gk)
    out = torch.empty_like(tp)
    P.plic_curvature_backward_ex_f32(tp, tg, out, solver, precision, normal, True, workspace, check=check)
    return host(out)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_matches_oracle(P, case, precision):
    phi, gk, gref, sel = case
    g = gpu_grad(P, phi, gk, "analytic", precision).astype(np.float64)
    scale = np.abs(gref).max()
    err = np.abs(g - gref).max() / scale
    print(f"{precision}: {sel.size} cells, max |g - g_ref| / max|g_ref| = {err:.3e}")
    assert err <= BARS[precision]
    assert np.all(g[~band_of(phi)] == 0.0)
    # the variant's gradient differs from the base method's
    tp, tg = dev(phi, gk)
    base = torch.empty_like(tp)
    P.plic_curvature_backward_f32(tp, tg, base, "analytic", precision)
    assert np.abs(host(base) - g).max() > 1e-3 * scale


def test_centre_of_mass_normal(P, orc):
    phi, gk, gref, _ = make_case(orc, "cm")
    g = gpu_grad(P, phi, gk, "analytic", "fp64", "cm").astype(np.float64)
    err = np.abs(g - gref).max() / np.abs(gref).max()
    print(f"cm/fp64: max |g - g_ref| / max|g_ref| = {err:.3e}")
    assert err <= BARS["fp64"]


@pytest.mark.parametrize("solver", ["sz", "newton", "nested"])
def test_other_solvers(P, case, solver):
    phi, gk, gref, _ = case
    g = gpu_grad(P, phi, gk, solver, "mixed").astype(np.float64)
    err = np.abs(g - gref).max() / np.abs(gref).max()
    print(f"{solver}/mixed: max |g - g_ref| / max|g_ref| = {err:.3e}")
    assert err <= BARS["mixed"]


def test_against_gpu_finite_differences(P, case):
    """d/dphi_j of sum(gk * kappa) by central differences (h = 1e-4) of the
    GPU forward of the variant in FP64, including cells two away from the
    upstream cells (reached only through the neighbours' own normals)."""
    phi, gk, _, sel = case
    g = gpu_grad(P, phi, gk, "analytic", "fp64").astype(np.float64)
    rng = np.random.default_rng(6)
    h = 1e-4
    cand = np.flatnonzero(((phi > 2 * h) & (phi < 1 - 2 * h)).ravel())
    js = rng.choice(cand, 40, replace=False)
    tp = dev(phi)
    tg = dev(gk).double()
    k = torch.empty_like(tp)
    worst = 0.0
    for j in js:
        vals = []
        for s in (+1, -1):
            t = tp.clone().view(-1)
            t[j] += s * h
            P.plic_curvature_ex_f32(t.view(phi.shape), k, "analytic", "fp64", "py", True)
            vals.append((k.double() * tg).sum().item())
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(fd - g.ravel()[j]) / max(1.0, abs(g.ravel()[j])))
    print(f"GPU FD check: worst relative error {worst:.3e}")
    assert worst <= 2e-3


def test_determinism_and_zero(P, case):
    phi, gk, _, _ = case
    a = gpu_grad(P, phi, gk)
    b = gpu_grad(P, phi, gk)
    assert np.array_equal(a, b)
    assert np.all(gpu_grad(P, phi, np.zeros_like(gk)) == 0.0)


def test_workspace_rows(P, case):
    """Without a recomputing fallback, a row that does not fit turns the
    affected band into NaN (never a silent wrong value); below one row the
    call is rejected.  With every row stored the result does not depend on
    the workspace size."""
    phi, gk, _, _ = case
    Z, Y, X = phi.shape
    ntiles = ((X + 63) // 64) * ((Y + 3) // 4) * ((Z + 3) // 4)
    fixed = 256 + 784 * ntiles
    full = P.plic_curvature_workspace_bytes_ex(X, Y, Z, True)
    assert full == fixed + ntiles * 64 * 432
    tp, tg = dev(phi, gk)
    out = torch.empty_like(tp)
    small = torch.empty(fixed + 431, dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception):
        P.plic_curvature_backward_ex_f32(tp, tg, out, "analytic", "mixed", "py", True, small)
    g_full = gpu_grad(P, phi, gk)
    n_iface = int(((phi > 0) & (phi < 1)).sum())
    g_big = gpu_grad(P, phi, gk, workspace=torch.empty(fixed + 432 * (n_iface + 50), dtype=torch.uint8,
                                                       device="cuda"))
    assert np.array_equal(g_full, g_big)
    few = torch.empty(fixed + 432 * 100, dtype=torch.uint8, device="cuda")
    g_few = gpu_grad(P, phi, gk, workspace=few, check=False)
    nan = np.isnan(g_few)
    assert nan.any() and not nan[~band_of(phi)].any()
    fin = ~nan
    assert np.array_equal(g_few[fin], g_full[fin])
    # the overflow is reported: the status query names it and the size that
    # holds every row; the checked call raises for a caller's workspace
    interior = np.zeros(phi.shape, bool)
    interior[1:-1, 1:-1, 1:-1] = True
    n_cells = int((((phi > 0) & (phi < 1)) & interior).sum())
    rc, cells, need = P.plic_curvature_status(few, X, Y, Z, True)
    assert (rc, cells, need) == (-3, n_cells, fixed + 432 * n_cells)
    with pytest.raises(RuntimeError, match="PLIC_EWORKSPACE"):
        gpu_grad(P, phi, gk, workspace=few)
    # a workspace with exactly one row per interface cell is complete
    exact = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert np.array_equal(gpu_grad(P, phi, gk, workspace=exact), g_full)
    assert P.plic_curvature_status(exact, X, Y, Z, True)[0] == 0


def test_dense_interface_through_autograd(P):
    """A lattice where every interior cell is an interface cell (noisy fill
    levels) needs far more rows than the default workspace's 64 per tile:
    the autograd path detects the overflow, repeats the call with a
    workspace that holds every row, and returns a finite gradient equal to a
    call given that size directly."""
    rng = np.random.default_rng(11)
    phi = rng.uniform(0.05, 0.95, size=(16, 16, 64)).astype(np.float32)
    gk = rng.standard_normal(phi.shape).astype(np.float32)
    Z, Y, X = phi.shape
    default = P.plic_curvature_workspace_bytes_ex(X, Y, Z, True)
    ntiles = 16
    assert default == 256 + 784 * ntiles + 64 * ntiles * 432 and 14 * 14 * 62 > 64 * ntiles
    tp = dev(phi).requires_grad_(True)
    k = P.curvature(tp, neighbour_normals=True)
    (k * dev(gk)).sum().backward()
    g = host(tp.grad)
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    need = 256 + 784 * ntiles + 432 * 14 * 14 * 62
    ref = gpu_grad(P, phi, gk, workspace=torch.empty(need, dtype=torch.uint8, device="cuda"))
    assert np.array_equal(g, ref)


def test_autograd(P, case):
    phi, gk, _, _ = case
    tp = dev(phi).requires_grad_(True)
    k = P.curvature(tp, neighbour_normals=True)
    (k * dev(gk)).sum().backward()
    assert np.array_equal(host(tp.grad), gpu_grad(P, phi, gk))
