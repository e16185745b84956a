"""Oracle pins for the curvature options: the centre-of-mass normal (App. B.1)
and the neighbour-normal variant (Sec. 4.2, Sec. 4.3).

* Both normal estimators are exact for a linear fill-level field: the
  weighted sum of e_i (g . e_i) is a multiple of g by the lattice symmetry.
* The paper's accuracy ranking of the normals (about 4 degrees for CM, 1 for
  PY) shows on a sphere.
* The neighbour-normal variant reduces to the base method when every normal
  is equal (linear fields), is exact on planes whose estimated normals are
  exact, recovers 1/R on a sphere, and is invariant under lattice rotations.
"""
import numpy as np
import pytest

import workloads


def linear_field(rng, size):
    """phi = 0.5 + g . x on a size^3 block centred at 0, inside (0, 1)."""
    g = rng.standard_normal(3)
    g *= 0.08 / np.abs(g).sum()
    r = np.arange(size) - size // 2
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    return 0.5 + g[0] * x + g[1] * y + g[2] * z, g


@pytest.mark.parametrize("normal", ["py", "cm"])
def test_normals_exact_on_linear_fields(orc, normal):
    rng = np.random.default_rng(0)
    for _ in range(50):
        phi, g = linear_field(rng, 3)
        _, _, n = orc.curv_cell_k(phi.ravel(), normal)
        assert np.allclose(n, -g / np.linalg.norm(g), atol=1e-12)


def test_cm_normal_less_accurate_than_py_on_sphere(orc):
    """Mean angle between the estimated and the radial normal on interface
    cells of a radius-20 sphere: PY below 2 degrees and CM above it."""
    phi, c = workloads.sphere_lattice(N=56, R=20.0, seed=1)
    Z, Y, X = phi.shape
    _, fl = orc.curvature(phi, flags=True)
    cells = np.flatnonzero(fl & 1)
    ang = {}
    for normal in ("py", "cm"):
        a = []
        for cell in cells[::7]:
            x, y, z = cell % X, (cell // X) % Y, cell // (X * Y)
            nb = phi[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].astype(np.float64).ravel()
            _, _, n = orc.curv_cell_k(nb, normal)
            radial = np.array([x, y, z], float) - np.asarray(c, float)
            radial /= np.linalg.norm(radial)
            a.append(np.degrees(np.arccos(np.clip(n @ radial, -1, 1))))
        ang[normal] = float(np.mean(a))
    print(f"mean normal error: PY {ang['py']:.2f} deg, CM {ang['cm']:.2f} deg")
    assert ang["py"] < 2.0 < ang["cm"]


@pytest.mark.parametrize("normal", ["py", "cm"])
def test_neighbour_normals_reduce_to_base_on_linear_fields(orc, normal):
    """Every neighbour normal equals the centre normal up to rounding, so the
    variant's points and curvature equal the base method's."""
    rng = np.random.default_rng(1)
    for _ in range(30):
        phi, _ = linear_field(rng, 5)
        k_nbr, info_n = orc.curv_cell_nbr(phi.ravel(), normal)
        inner = phi[1:4, 1:4, 1:4].ravel()
        k_base, info_b, _ = orc.curv_cell_k(inner, normal)
        assert info_n[0] == info_b[0]
        assert abs(k_nbr - k_base) <= 1e-9 * max(1.0, abs(k_base))


@pytest.mark.parametrize("normal", ["py", "cm"])
def test_neighbour_normals_zero_on_exact_planes(orc, normal):
    """Planes along an axis or a face diagonal, fill levels from the exact
    plane-cube volume: every estimated normal is exact by symmetry (neighbours
    on the outer layer keep the centre normal), so every PLIC point lies on the
    plane and kappa vanishes up to the FP32 rounding of phi."""
    N = 12
    for nrm, off in (((0.0, 0.0, 1.0), 0.3), ((1 / np.sqrt(2), 1 / np.sqrt(2), 0.0), 0.17)):
        n = np.array(nrm)
        r = np.arange(N) - N / 2
        z, y, x = np.meshgrid(r, r, r, indexing="ij")
        d0 = off - (n[0] * x + n[1] * y + n[2] * z)            # plane n.X = off, cell-local offsets
        phi = orc.volume(np.full(d0.size, n[0]), np.full(d0.size, n[1]), np.full(d0.size, n[2]),
                         d0.ravel()).reshape(d0.shape).astype(np.float32)
        k, fl = orc.curvature(phi, flags=True, normal=normal, neighbour_normals=True)
        sel = (fl & 1) == 1
        assert sel.sum() > 20
        assert np.abs(k[sel]).max() <= 1e-6


@pytest.mark.parametrize("normal", ["py", "cm"])
def test_neighbour_normals_sphere(orc, normal):
    phi, _ = workloads.sphere_lattice(N=48, R=14.0, seed=0)
    kb, fb = orc.curvature(phi, flags=True, normal=normal)
    kn, fn = orc.curvature(phi, flags=True, normal=normal, neighbour_normals=True)
    assert np.array_equal(fb & 1, fn & 1)                    # same interface cells
    sel = (fn & 1) == 1
    mean_n = float(np.mean(kn[sel])) * 14.0
    e_b = np.abs(kb[sel] - 1 / 14).sum() / (sel.sum() / 14)
    e_n = np.abs(kn[sel] - 1 / 14).sum() / (sel.sum() / 14)
    print(f"{normal}: mean kR {mean_n:.4f}, L1 error base {e_b:.4f} neighbour normals {e_n:.4f}")
    assert abs(mean_n - 1.0) < 0.02
    assert e_n < 1.1 * e_b


def test_neighbour_normals_lattice_rotation(orc):
    """A quarter turn of the 5^3 neighbourhood about z maps kappa to itself
    (cells with a full-rank fit)."""
    phi, _, _ = workloads.perturbed_sphere_lattice(N=40, R=12.0, seed=3, ss=4)
    Z, Y, X = phi.shape
    _, fl = orc.curvature(phi, flags=True)
    cells = np.flatnonzero(fl == 1)[::11]
    checked = 0
    for cell in cells:
        x, y, z = cell % X, (cell // X) % Y, cell // (X * Y)
        if min(x, y, z) < 2 or x > X - 3 or y > Y - 3 or z > Z - 3:
            continue
        nb = phi[z - 2:z + 3, y - 2:y + 3, x - 2:x + 3].astype(np.float64)
        k0, info0 = orc.curv_cell_nbr(nb.ravel(), "py")
        k1, info1 = orc.curv_cell_nbr(np.rot90(nb, 1, axes=(1, 2)).copy().ravel(), "py")
        if info0[0] < 5 or info0[2] > 1e4:
            continue
        assert abs(k0 - k1) <= 1e-9 * max(1.0, abs(k0))
        checked += 1
    assert checked > 20


def test_neighbour_normals_fd_gradient_converges_and_respects_complement(orc):
    """The variant's gradient reaches two cells out (each neighbour's own
    normal).  Central differences at h and 2h agree, and since kappa(1 - phi) =
    -kappa(phi) for this variant too (every normal and offset flips), the
    gradient at 1 - phi equals the gradient at phi."""
    phi, _, _ = workloads.perturbed_sphere_lattice(N=36, R=11.0, seed=2, ss=4)
    kn = orc.curvature(phi, neighbour_normals=True)
    kc = orc.curvature((1.0 - phi).astype(np.float32), neighbour_normals=True)
    _, fl = orc.curvature(phi, flags=True)
    assert np.max(np.abs(kn + kc)[(fl & 1) == 1]) <= 1e-12
    Z, Y, X = phi.shape
    cells = np.flatnonzero(fl == 1)[::53][:16]
    checked = 0
    for cc in cells:
        x, y, z = cc % X, (cc // X) % Y, cc // (X * Y)
        if min(x, y, z) < 2 or x > X - 3 or y > Y - 3 or z > Z - 3:
            continue
        nb = phi[z - 2:z + 3, y - 2:y + 3, x - 2:x + 3].astype(np.float64)
        inner = nb[1:4, 1:4, 1:4]
        if np.any((inner > 0) & (inner < 1e-4)) or np.any((inner < 1) & (inner > 1 - 1e-4)):
            continue
        g1, bad1 = orc.curv_cell_nbr_fd_grad(nb.ravel(), h=1e-6)
        g2, bad2 = orc.curv_cell_nbr_fd_grad(nb.ravel(), h=2e-6)
        if bad1 or bad2:
            continue
        scale = max(1.0, np.abs(g1).max())
        assert np.max(np.abs(g1 - g2)) <= 1e-6 * scale
        gc, badc = orc.curv_cell_nbr_fd_grad((1.0 - nb).ravel(), h=1e-6)
        assert not badc
        assert np.max(np.abs(gc - g1)) <= 1e-6 * scale
        # the outer layer of the 5^3 matters (own normals of the neighbours)
        outer = np.ones((5, 5, 5), bool)
        outer[1:4, 1:4, 1:4] = False
        assert np.abs(g1.reshape(5, 5, 5)[outer]).max() > 1e-5 * scale     # FD noise is ~1e-9
        checked += 1
    assert checked >= 5
