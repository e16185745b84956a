"""Sizes beyond one dispatch and beyond 32-bit cell indices.

* PLIC entry points on 2^30 + 4099 problems: a dispatch holds at most 2^32 - 1
  work-items, so the library launches chunks of 2^30 problems and one ragged
  tail block.  The input is a seeded 2^20-problem set repeated on the device,
  and every problem is independent of its position, so each copy of the output
  must equal the first bit for bit (NaN where the first is NaN); the first is
  checked against the oracle.
* Curvature on a 1024 x 1024 x 2100 lattice (2.2e9 cells, above 2^31): a
  small sphere placed near the far end, beyond cell index 2^31, gives the same
  kappa and the same gradient bits as that sphere in its own small lattice
  (every cell depends only on its neighbourhood; with a contribution row for
  every interface cell the gather sums each cell's sources in a fixed order),
  and zero elsewhere.
"""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev, host, max_abs_err

pytestmark = pytest.mark.gpu

BASE = 1 << 20
BIG = (1 << 30) + 4099


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.fixture
def free_memory():
    yield
    torch.cuda.empty_cache()


def tiled(t):
    """t (BASE,) repeated to BIG elements on the device"""
    reps = BIG // BASE + 1
    return t.repeat(reps)[:BIG].contiguous()


def same_bits_as_base(big, base):
    """every BASE-long copy in `big` (and the tail) equals `base`, NaN-aware"""
    full = BIG // BASE
    body = big[: full * BASE].view(full, BASE)
    eq = (body == base[None, :]) | (torch.isnan(body) & torch.isnan(base)[None, :])
    tail = big[full * BASE:]
    teq = (tail == base[: tail.numel()]) | (torch.isnan(tail) & torch.isnan(base[: tail.numel()]))
    return bool(eq.all().item()) and bool(teq.all().item())


def test_offset_volume_backward_beyond_one_dispatch(P, orc, free_memory):
    nx, ny, nz, V0 = workloads.plic_problems(BASE, seed=7)
    g = workloads.upstream_grad(BASE, seed=8)
    base = dev(nx, ny, nz, V0, g)
    big = [tiled(t) for t in base]
    print(f"problems: {BIG} ({BIG * 4 / 2**30:.1f} GiB per array)", flush=True)
    for solver in ("analytic", "sz", "newton", "nested"):
        d_base = torch.empty_like(base[3])
        P.plic_offset_f32(*base[:4], d_base, solver, "fp32")
        d_big = torch.empty_like(big[3])
        P.plic_offset_f32(*big[:4], d_big, solver, "fp32")
        torch.cuda.synchronize()
        assert same_bits_as_base(d_big, d_base), solver
        if solver == "sz":
            assert max_abs_err(host(d_base), orc.offset(nx, ny, nz, V0)) <= 1e-5
            v_base = torch.empty_like(d_base)
            P.plic_volume_f32(*base[:3], d_base, v_base, "fp32")
            v_big = torch.empty_like(d_big)
            P.plic_volume_f32(*big[:3], d_big, v_big, "fp32")
            assert same_bits_as_base(v_big, v_base)
            del v_big
        del d_big
    outs_base = [torch.empty_like(base[3]) for _ in range(4)]
    P.plic_offset_backward_f32(*base, *outs_base, "sz", "fp32")
    outs_big = [torch.empty_like(big[3]) for _ in range(4)]
    P.plic_offset_backward_f32(*big, *outs_big, "sz", "fp32")
    torch.cuda.synchronize()
    for k in range(4):
        assert same_bits_as_base(outs_big[k], outs_base[k]), k
    # the plane-sphere inversion has the same chunked launch
    s_base = torch.empty_like(base[3])
    P.plic_sphere_offset_f32(base[3], s_base)
    s_big = torch.empty_like(big[3])
    P.plic_sphere_offset_f32(big[3], s_big)
    torch.cuda.synchronize()
    assert same_bits_as_base(s_big, s_base)


def test_curvature_beyond_32bit_cells(P, free_memory):
    X, Y, Z = 1024, 1024, 2100
    small, _ = workloads.sphere_lattice(N=48, R=14.0, seed=4)
    gk_small = workloads.upstream_grad(small.shape, seed=5)
    # block origin: tile-aligned (64 x 4 x 4), its first cell beyond index 2^31
    ox, oy, oz = 896, 960, 2048
    assert (oz * Y + oy) * X + ox > 2**31
    ts, tg = dev(small, gk_small)
    # a workspace with a row for every interface cell of the small lattice (its
    # recommended size holds 16 per tile, fewer than this sphere has), so that
    # both lattices take the direct gather
    ws = torch.empty(64 * P.plic_curvature_workspace_bytes(*small.shape[::-1]), dtype=torch.uint8, device="cuda")
    k_small = torch.empty_like(ts)
    P.plic_curvature_f32(ts, k_small, "analytic", "mixed", ws)
    g_small = torch.empty_like(ts)
    P.plic_curvature_backward_f32(ts, tg, g_small, "analytic", "mixed", ws)

    phi = torch.zeros((Z, Y, X), dtype=torch.float32, device="cuda")
    gk = torch.zeros_like(phi)
    n = small.shape[0]
    phi[oz:oz + n, oy:oy + n, ox:ox + n] = ts
    gk[oz:oz + n, oy:oy + n, ox:ox + n] = tg
    print(f"lattice {X}x{Y}x{Z} = {X * Y * Z} cells", flush=True)
    kappa = torch.full_like(phi, 7.0)
    P.plic_curvature_f32(phi, kappa, "analytic", "mixed")
    torch.cuda.synchronize()
    blk = kappa[oz:oz + n, oy:oy + n, ox:ox + n]
    assert torch.equal(blk, k_small)
    nz_all = int(torch.count_nonzero(kappa).item())
    assert nz_all == int(torch.count_nonzero(k_small).item())      # zero outside the block
    del kappa
    gphi = torch.full_like(phi, 7.0)
    P.plic_curvature_backward_f32(phi, gk, gphi, "analytic", "mixed")
    torch.cuda.synchronize()
    assert torch.equal(gphi[oz:oz + n, oy:oy + n, ox:ox + n], g_small)
    assert int(torch.count_nonzero(gphi).item()) == int(torch.count_nonzero(g_small).item())
