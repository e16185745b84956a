"""Lattices of more than 256 x 256 tiles take the two-pass row prefix (the
gather list and per-workgroup totals, then a second pass that adds the totals
of the workgroups before each one).  A curvature result depends only on each
interface cell's neighbourhood, so two copies of a small perturbed sphere
embedded far apart in a 64 x 1028 x 1024 lattice of zeros (65,792 tiles) give,
inside each copy, the same bits as the small lattice alone, and zero
everywhere else: forward, the backward that scans, the backward that reuses
the forward's records, and the neighbour-normal backward.  The second copy's
contribution rows start after the first copy's, hundreds of workgroups later,
so its gradient is right only if the second pass carried the first copy's
count across them."""
import pytest
import torch

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu

BIG = (1024, 1028, 64)                        # (Z, Y, X)
# (z, y, x) corners of the two copies: one in the lattice's first workgroups
# of tiles, one in its last
CORNERS = ((8, 8, 12), (960, 980, 12))


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.fixture(scope="module")
def small():
    phi, _, _ = workloads.perturbed_sphere_lattice(N=40, R=12.0, seed=11, ss=4)
    gk = workloads.upstream_grad(phi.shape, seed=12)
    # the copies sit in a lattice of zeros: the small lattice's own border must be empty too
    assert not phi[:4].any() and not phi[-4:].any() and not phi[:, :4].any() and not phi[:, -4:].any()
    assert not phi[:, :, :4].any() and not phi[:, :, -4:].any()
    return phi, gk


def full_workspace(P, phi, nbr=False):
    Z, Y, X = phi.shape
    rows = int(((phi > 0) & (phi < 1)).sum())
    nbytes = P.plic_curvature_workspace_bytes_ex(X, Y, Z, nbr) + rows * (432 if nbr else 108)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def embed(small_arr, fill):
    big = fill
    for z, y, x in CORNERS:
        n = small_arr.shape
        big[z:z + n[0], y:y + n[1], x:x + n[2]] = small_arr
    return big


def check_embedded(big, small_arr, what):
    n = small_arr.shape
    rest = big.clone()
    for k, (z, y, x) in enumerate(CORNERS):
        blk = big[z:z + n[0], y:y + n[1], x:x + n[2]]
        assert torch.equal(blk, small_arr), (what, k, float((blk - small_arr).abs().max()))
        rest[z:z + n[0], y:y + n[1], x:x + n[2]] = 0.0
    assert int(torch.count_nonzero(rest).item()) == 0, what


def test_two_pass_lattice_takes_the_second_pass(P):
    Z, Y, X = BIG
    ntiles = ((X + 63) // 64) * ((Y + 3) // 4) * ((Z + 3) // 4)
    assert (ntiles + 255) // 256 > 256        # more workgroups of tiles than the one-pass limit


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_forward_and_backward_embedded(P, small, precision):
    phi, gk = small
    sp, sg = dev(phi), dev(gk)
    ks = torch.empty_like(sp)
    P.plic_curvature_f32(sp, ks, "analytic", precision)
    gs = torch.empty_like(sp)
    # every contribution row fits (the recomputing fallback would add dense tiles in chunks)
    P.plic_curvature_backward_f32(sp, sg, gs, "analytic", precision, full_workspace(P, phi))
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(ks).item()) > 500 and int(torch.count_nonzero(gs).item()) > 1000

    Z, Y, X = BIG
    bp = embed(sp, torch.zeros(BIG, device="cuda"))
    gen = torch.Generator(device="cuda").manual_seed(3)
    bg = embed(sg, torch.randn(BIG, device="cuda", generator=gen))
    ws = torch.empty(P.plic_curvature_workspace_bytes(X, Y, Z), dtype=torch.uint8, device="cuda")
    kb = torch.full(BIG, float("nan"), device="cuda")
    P.plic_curvature_f32(bp, kb, "analytic", precision, ws)
    # right after the forward: the backward that reuses its records
    gr = torch.full(BIG, float("nan"), device="cuda")
    P.plic_curvature_backward_reuse_f32(bp, bg, gr, "analytic", precision, "py", False, ws)
    gb = torch.full(BIG, float("nan"), device="cuda")
    P.plic_curvature_backward_f32(bp, bg, gb, "analytic", precision, ws)
    torch.cuda.synchronize()
    check_embedded(kb, ks, "kappa")
    check_embedded(gb, gs, "grad_phi")
    check_embedded(gr, gs, "grad_phi (reusing backward)")
    status = P.plic_curvature_status(ws, X, Y, Z)
    assert status[0] == 0 and status[1] == 2 * int(((phi > 0) & (phi < 1)).sum()), status


def test_neighbour_normal_backward_embedded(P, small):
    phi, gk = small
    sp, sg = dev(phi), dev(gk)
    gs = torch.empty_like(sp)
    P.plic_curvature_backward_ex_f32(sp, sg, gs, "analytic", "mixed", "py", True, full_workspace(P, phi, True))
    Z, Y, X = BIG
    bp = embed(sp, torch.zeros(BIG, device="cuda"))
    bg = embed(sg, torch.zeros(BIG, device="cuda"))
    ws = torch.empty(P.plic_curvature_workspace_bytes_ex(X, Y, Z, True), dtype=torch.uint8, device="cuda")
    gb = torch.full(BIG, float("nan"), device="cuda")
    P.plic_curvature_backward_ex_f32(bp, bg, gb, "analytic", "mixed", "py", True, ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gs).all()) and int(torch.count_nonzero(gs).item()) > 1000
    check_embedded(gb, gs, "grad_phi (neighbour normals)")
