"""The compute-isolated benchmark kernel (the paper's GPU test method,
Sec. 2.6.2): every offset it computes matches the FP64 oracle within the FP32
bar, its round-trip errors are at FP32 rounding level, bounded like the
batched round trip, and average to what the library's batched inversion and
forward volume give on the same problems.  (Inlined in one kernel the
compiler may contract the arithmetic differently, so single errors, each
about one ulp of V0, need not match bit for bit.)"""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import SOLVERS, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.mark.parametrize("solver", SOLVERS)
def test_isolated_offsets_match_oracle(P, orc, solver):
    """The offsets of the benchmark's sweep (paper mix of normals, L = 256
    fill levels j / 255 per normal, 0 and 1 included), element by element
    against the oracle at 1e-5; the error sums are those of the offsets."""
    n, L = 4096, 256
    nx, ny, nz = workloads.paper_mix_normals(n, seed=8)
    tx, ty, tz = dev(nx, ny, nz)
    err = torch.empty_like(tx)
    d0 = torch.empty(L * n, dtype=torch.float32, device="cuda")
    P.plic_bench_isolated_f32(tx, ty, tz, err, L, solver, False, d0)
    got = host(d0).astype(np.float64)
    V0 = (np.arange(L, dtype=np.float32) / np.float32(L - 1)).astype(np.float32)
    ref = orc.offset(np.tile(nx, L), np.tile(ny, L), np.tile(nz, L), np.repeat(V0, n))
    e = np.abs(got - ref).max()
    print(f"{solver}: {n * L} offsets, max |d0 - oracle| = {e:.2e}")
    assert e <= 1e-5
    # the timed instance (no offsets kept) gives the same error sums
    err2 = torch.empty_like(tx)
    P.plic_bench_isolated_f32(tx, ty, tz, err2, L, solver, False)
    assert torch.equal(err, err2)
    # each error sum is that of the kept offsets through the FP64 volume, up
    # to the FP32 rounding of the kernel's own volume (a few ulp of V0 each)
    Vr = orc.volume(np.tile(nx, L), np.tile(ny, L), np.tile(nz, L), got.astype(np.float32))
    Eref = np.abs(Vr - np.repeat(V0, n)).reshape(L, n).sum(0)
    assert np.abs(host(err) - Eref).max() <= L * 2e-7


@pytest.mark.parametrize("solver", SOLVERS)
def test_isolated_matches_batched_round_trip(P, solver):
    n, L = 2048, 64
    nx, ny, nz = workloads.paper_mix_normals(n, seed=5)
    V0 = (np.arange(L, dtype=np.float32) / np.float32(L - 1)).astype(np.float32)
    assert V0[0] == 0.0 and V0[-1] == 1.0
    tx, ty, tz = dev(nx, ny, nz)
    err = torch.empty_like(tx)
    P.plic_bench_isolated_f32(tx, ty, tz, err, L, solver, False)
    got = host(err)
    # the same n L problems through the batched kernels
    bx, by, bz = (np.repeat(a, L) for a in (nx, ny, nz))
    bv = np.tile(V0, n)
    cx, cy, cz, cv = dev(bx, by, bz, bv)
    d0 = torch.empty_like(cv)
    P.plic_offset_f32(cx, cy, cz, cv, d0, solver, "fp32")
    V = torch.empty_like(cv)
    P.plic_volume_f32(cx, cy, cz, d0, V, "fp32")
    E = np.abs(host(V) - bv).reshape(n, L)
    assert np.all(got <= L * 2e-6)                       # the batched round-trip bound per evaluation
    e_avg = float(got.astype(np.float64).sum() / (n * L))
    e_ref = float(E.astype(np.float64).sum() / (n * L))
    print(f"{solver}: E_avg {e_avg:.3e} (batched {e_ref:.3e})")
    assert e_avg < 2e-7
    assert abs(e_avg - e_ref) <= 0.25 * e_ref + 1e-9


def test_blank_run(P):
    """The blank run inverts nothing: d0 = V0 - 1/2 through the forward volume."""
    n, L = 1024, 32
    nx, ny, nz = workloads.paper_mix_normals(n, seed=6)
    tx, ty, tz = dev(nx, ny, nz)
    err = torch.empty_like(tx)
    P.plic_bench_isolated_f32(tx, ty, tz, err, L, "sz", True)
    V0 = (np.arange(L, dtype=np.float32) / np.float32(L - 1)).astype(np.float32)
    bx, by, bz = (np.repeat(a, L) for a in (nx, ny, nz))
    bd = np.tile(V0 - np.float32(0.5), n).astype(np.float32)
    cx, cy, cz, cd = dev(bx, by, bz, bd)
    V = torch.empty_like(cd)
    P.plic_volume_f32(cx, cy, cz, cd, V, "fp32")
    E = np.abs(host(V) - np.tile(V0, n)).reshape(n, L)
    ref = np.zeros(n, np.float32)
    for j in range(L):
        ref = (ref + E[:, j]).astype(np.float32)
    assert np.allclose(host(err), ref, rtol=1e-5, atol=1e-9)
    # the kept offsets of the blank run are V0 - 1/2 exactly
    d0 = torch.empty(L * n, dtype=torch.float32, device="cuda")
    P.plic_bench_isolated_f32(tx, ty, tz, err, L, "sz", True, d0)
    assert np.array_equal(host(d0), np.repeat(V0 - np.float32(0.5), n))
