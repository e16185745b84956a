"""The entry points run asynchronously on the caller's stream and record into
a HIP graph: a side stream gives the same bits as the default stream, and a
captured sequence (batched inversion, forward volume, curvature forward and
backward, the backward that reuses the forward's scan, the neighbour-normal
backward, all with caller-owned outputs and
workspaces) replays correctly several times with eager work and new inputs
between the replays.  The curvature clears its counters with a kernel, not a
memset, and sizes its launches on the host, so nothing in it depends on
reading device memory from the host."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


def test_side_stream_same_bits(P):
    nx, ny, nz, V0 = workloads.plic_problems(1 << 20, seed=21)
    t = dev(nx, ny, nz, V0)
    ref = torch.empty_like(t[3])
    P.plic_offset_f32(*t, ref, "analytic", "fp32")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = torch.empty_like(t[3])
        P.plic_offset_f32(*t, out, "analytic", "fp32")
        kap_side = torch.empty((40, 40, 40), device="cuda")
        phi, _ = workloads.sphere_lattice(N=40, R=12.0, seed=2)
        tphi = torch.from_numpy(phi).to("cuda", non_blocking=False)
        P.plic_curvature_f32(tphi, kap_side, "analytic", "mixed")
    side.synchronize()
    assert torch.equal(out.nan_to_num(7.0), ref.nan_to_num(7.0))
    kap = torch.empty_like(kap_side)
    P.plic_curvature_f32(tphi, kap, "analytic", "mixed")
    torch.cuda.synchronize()
    assert torch.equal(kap, kap_side)


def test_graph_replays_match_eager(P):
    N = 1 << 20
    probs = [workloads.plic_problems(N, seed=30 + k) for k in range(3)]
    lattices = [workloads.sphere_lattice(N=48, R=r, seed=k)[0] for k, r in enumerate((12.0, 14.0, 15.5))]
    grads = [workloads.upstream_grad((48, 48, 48), seed=40 + k) for k in range(3)]
    # static inputs, outputs and workspace of the graph
    sn = [torch.empty(N, device="cuda") for _ in range(4)]
    d0 = torch.empty(N, device="cuda")
    vb = torch.empty(N, device="cuda")
    phi = torch.empty((48, 48, 48), device="cuda")
    gk = torch.empty_like(phi)
    kap = torch.empty_like(phi)
    gphi = torch.empty_like(phi)
    gnbr = torch.empty_like(phi)
    greu = torch.empty_like(phi)
    ws = torch.empty(P.plic_curvature_workspace_bytes(48, 48, 48), dtype=torch.uint8, device="cuda")
    ws_nbr = torch.empty(P.plic_curvature_workspace_bytes_ex(48, 48, 48, True), dtype=torch.uint8, device="cuda")

    def load(k):
        for dst, src in zip(sn, probs[k]):
            dst.copy_(torch.from_numpy(src))
        phi.copy_(torch.from_numpy(lattices[k]))
        gk.copy_(torch.from_numpy(grads[k]))

    def work():
        P.plic_offset_f32(*sn, d0, "nested", "fp32")
        P.plic_volume_f32(sn[0], sn[1], sn[2], d0, vb, "fp32")
        P.plic_curvature_f32(phi, kap, "analytic", "mixed", ws)
        # the backward that reuses the forward's scan (decided at capture: no scan in the graph)
        P.plic_curvature_backward_reuse_f32(phi, gk, greu, "analytic", "mixed", "py", False, ws)
        P.plic_curvature_backward_f32(phi, gk, gphi, "analytic", "mixed", ws)
        P.plic_curvature_backward_ex_f32(phi, gk, gnbr, "analytic", "mixed", "py", True, ws_nbr)

    load(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                      # warm-up before capture
        work()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    torch.cuda.synchronize()
    for rep in range(3):
        k = rep % 3
        load(k)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [x.clone() for x in (d0, vb, kap, gphi, gnbr, greu)]
        assert torch.equal(got[5], got[3]), rep                # reusing and scanning backward: same bits
        # eager work between the replays, on the same buffers
        work()
        torch.cuda.synchronize()
        for a, b, name in zip(got, (d0, vb, kap, gphi, gnbr, greu),
                              ("d0", "V0", "kappa", "grad_phi", "grad_phi_nbr", "grad_phi_reuse")):
            assert torch.equal(a.nan_to_num(7.0), b.nan_to_num(7.0)), (rep, name)
        assert int(torch.count_nonzero(kap).item()) > 500
        assert bool(torch.isfinite(gnbr).all()) and int(torch.count_nonzero(gnbr).item()) > 500
