"""The backward that reuses the forward's interface scan
(plic_curvature_backward_reuse_f32) gives the same bits as the backward that
scans phi itself, in every precision, both normals and the neighbour-normal
variant, also with a workspace too small for every contribution row (the
recomputing fallback); when the workspace's last scan was for another phi or
lattice it scans phi itself.  The autograd path (which reuses) equals the
plain backward.  The full-size case (256^3 sphere) is held against the oracle
through the plain backward's own parity tests."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import PRECISIONS, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.fixture(scope="module")
def lattice():
    phi, _, _ = workloads.perturbed_sphere_lattice(N=40, R=12.0, seed=5, ss=4)
    gk = workloads.upstream_grad(phi.shape, seed=6)
    return phi, gk


def plain(P, tp, tg, solver, precision, normal="py", nbr=False, nbytes=None):
    Z, Y, X = tp.shape
    ws = torch.empty(nbytes or P.plic_curvature_workspace_bytes_ex(X, Y, Z, nbr), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(tp)
    P.plic_curvature_backward_ex_f32(tp, tg, out, solver, precision, normal, nbr, ws)
    return host(out)


def reused(P, tp, tg, solver, precision, normal="py", nbr=False, nbytes=None, fwd_phi=None):
    Z, Y, X = tp.shape
    ws = torch.empty(nbytes or P.plic_curvature_workspace_bytes_ex(X, Y, Z, nbr), dtype=torch.uint8, device="cuda")
    src = tp if fwd_phi is None else fwd_phi
    P.plic_curvature_ex_f32(src, torch.empty_like(src), solver, precision, normal, nbr, ws)
    out = torch.full_like(tp, float("nan"))                 # every cell must be written
    P.plic_curvature_backward_reuse_f32(tp, tg, out, solver, precision, normal, nbr, ws)
    return host(out)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("normal,nbr", [("py", False), ("cm", False), ("py", True)])
def test_reuse_same_bits(P, lattice, precision, normal, nbr):
    phi, gk = lattice
    tp, tg = dev(phi, gk)
    a = plain(P, tp, tg, "analytic", precision, normal, nbr)
    b = reused(P, tp, tg, "analytic", precision, normal, nbr)
    assert np.isfinite(a).all() and np.abs(a).max() > 0
    assert np.array_equal(a, b)


def test_reuse_with_fallback_rows(P, lattice):
    """Workspaces of the fixed part alone (every row recomputed) and of the
    fixed part plus 37 rows (most rows recomputed)."""
    phi, gk = lattice
    tp, tg = dev(phi, gk)
    Z, Y, X = phi.shape
    ntiles = ((X + 63) // 64) * ((Y + 3) // 4) * ((Z + 3) // 4)
    fixed = 256 + 784 * ntiles
    for nbytes in (fixed, fixed + 108 * 37):
        assert np.array_equal(plain(P, tp, tg, "sz", "mixed", nbytes=nbytes),
                              reused(P, tp, tg, "sz", "mixed", nbytes=nbytes)), nbytes


def test_reuse_other_phi_scans(P, lattice):
    """The workspace's last scan was for another phi (another address): the
    call scans phi itself and matches the plain backward."""
    phi, gk = lattice
    tp, tg = dev(phi, gk)
    other = dev(np.ascontiguousarray(phi[::-1]))
    assert np.array_equal(plain(P, tp, tg, "analytic", "mixed"),
                          reused(P, tp, tg, "analytic", "mixed", fwd_phi=other))


def test_reuse_other_lattice_scans(P):
    """Same phi address, other lattice dimensions: the call scans."""
    phi, _ = workloads.sphere_lattice(N=24, R=7.0, seed=3)
    gk = workloads.upstream_grad(phi.shape, seed=4)
    tp, tg = dev(phi, gk)
    flat = tp.view(24, 48, 12)                              # the same memory, read as another lattice
    nbytes = max(P.plic_curvature_workspace_bytes(24, 24, 24), P.plic_curvature_workspace_bytes(12, 48, 24))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P.plic_curvature_f32(flat, torch.empty_like(flat), "analytic", "mixed", ws)
    out = torch.empty_like(tp)
    P.plic_curvature_backward_reuse_f32(tp, tg, out, "analytic", "mixed", "py", False, ws)
    assert np.array_equal(host(out), plain(P, tp, tg, "analytic", "mixed"))


def test_autograd_reuses_and_matches(P, lattice):
    phi, gk = lattice
    tp, tg = dev(phi, gk)
    x = tp.clone().requires_grad_(True)
    k = P.curvature(x, "analytic", "mixed")
    k.backward(tg)
    assert np.array_equal(host(x.grad), plain(P, tp, tg, "analytic", "mixed"))


def test_reuse_repeated_and_after_a_scanning_backward(P, lattice):
    """Right after its forward the reusing backward also skips the counter
    reset (the forward's reset covered it); repeated, or after a scanning
    backward on the workspace, it resets them: every call gives the same bits."""
    phi, gk = lattice
    tp, tg = dev(phi, gk)
    ref = plain(P, tp, tg, "analytic", "mixed")
    Z, Y, X = phi.shape
    ws = torch.empty(P.plic_curvature_workspace_bytes(X, Y, Z), dtype=torch.uint8, device="cuda")
    P.plic_curvature_f32(tp, torch.empty_like(tp), "analytic", "mixed", ws)
    for k in range(3):
        out = torch.full_like(tp, float("nan"))
        P.plic_curvature_backward_reuse_f32(tp, tg, out, "analytic", "mixed", "py", False, ws)
        assert np.array_equal(host(out), ref), k
    out = torch.empty_like(tp)
    P.plic_curvature_backward_f32(tp, tg, out, "analytic", "mixed", ws)
    out = torch.full_like(tp, float("nan"))
    P.plic_curvature_backward_reuse_f32(tp, tg, out, "analytic", "mixed", "py", False, ws)
    assert np.array_equal(host(out), ref)
