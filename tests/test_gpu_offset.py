"""GPU parity of plic_offset (all four solvers, three precisions) and
plic_volume against the FP64 oracle.  Tolerances: |d0 - d0_ref| <= 1e-5 for
float32 storage, <= 1e-12 for float64; |V0 - V0_ref| <= 1e-6 / 1e-14."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import (PRECISIONS, SOLVERS, dev, gpu_offset, host, max_abs_err,
                            near_degenerate_problems)

pytestmark = pytest.mark.gpu

TOL32, TOL64 = 1e-5, 1e-12


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


@pytest.fixture(scope="module")
def small(orc):
    """2^20 problems, seed 0 (2 % forced edge cases)."""
    nx, ny, nz, V0 = workloads.plic_problems(1 << 20, seed=0)
    return nx, ny, nz, V0, orc.offset(nx, ny, nz, V0)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("solver", SOLVERS)
def test_offset_parity_f32(P, small, solver, precision):
    nx, ny, nz, V0, ref = small
    d0 = gpu_offset(P, nx, ny, nz, V0, solver, precision)
    assert not np.isnan(d0).any()
    err = max_abs_err(d0, ref)
    print(f"{solver}/{precision}: max |d0 - oracle| = {err:.3e}")
    assert err <= TOL32


@pytest.mark.parametrize("solver", SOLVERS)
def test_offset_parity_f64(P, orc, solver):
    nx, ny, nz, V0 = workloads.plic_problems(300007, seed=1, dtype=np.float64)
    ref = orc.offset(nx, ny, nz, V0)
    d0 = gpu_offset(P, nx, ny, nz, V0, solver)
    err = max_abs_err(d0, ref)
    print(f"{solver}/f64: max |d0 - oracle| = {err:.3e}")
    assert err <= TOL64


@pytest.mark.parametrize("solver", SOLVERS)
def test_ragged_and_unaligned(P, orc, solver):
    """Counts that are not a multiple of the vector width, and pointers that are
    4-byte but not 16-byte aligned (the scalar path)."""
    nx, ny, nz, V0 = workloads.plic_problems(100003, seed=2)
    ref = orc.offset(nx, ny, nz, V0)
    for start in (0, 1, 3):
        t = dev(nx, ny, nz, V0)
        sl = [x[start:] for x in t]
        out = torch.empty(V0.size + 1, dtype=torch.float32, device="cuda")[1:]
        P.plic_offset_f32(*sl, out[: V0.size - start], solver, "fp32")
        assert max_abs_err(host(out[: V0.size - start]), ref[start:]) <= TOL32
    for n in (1, 2, 3, 5, 255, 257, 1023, 1025):
        d = gpu_offset(P, nx[:n], ny[:n], nz[:n], V0[:n], solver)
        assert max_abs_err(d, ref[:n]) <= TOL32


def edge_problems():
    s2 = np.float32(1 / np.sqrt(2))
    s3 = np.float32(1 / np.sqrt(3))
    normals = [(1, 0, 0), (0, -1, 0), (0, 0, 1), (s2, s2, 0), (0, -s2, s2), (s2, 0, -s2),
               (s3, s3, s3), (-s3, s3, -s3), (1e-30, 0.6, 0.8), (1e-7, 1e-7, 1.0),
               (0.3, 0.3, 0.3), (2.0, 0.0, 0.0), (0.0, 3.0, 4.0)]
    vols = [0.0, 1.0, 0.5, 1e-7, 1 - 6e-8, 0.25, 0.75, -0.5, 1.5, 2 ** -24, 0.49999997]
    rows = [(a, b, c, v) for (a, b, c) in normals for v in vols]
    arr = np.array(rows, dtype=np.float32)
    return [np.ascontiguousarray(arr[:, i]) for i in range(4)]


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("solver", SOLVERS)
def test_edge_cases(P, orc, solver, precision):
    """Axis (1D), face-diagonal (2D) and space-diagonal normals, V0 in {0, 1/2, 1},
    tiny and near-1 fill levels, out-of-range V0 (clamped), non-unit normals;
    no solver may return NaN here (the SZ translation of the paper does for
    n = (1,0,0), V0 in {0,1})."""
    nx, ny, nz, V0 = edge_problems()
    ref = orc.offset(nx, ny, nz, V0)
    d0 = gpu_offset(P, nx, ny, nz, V0, solver, precision)
    assert not np.isnan(d0).any()
    assert max_abs_err(d0, ref) <= TOL32


@pytest.mark.parametrize("solver", SOLVERS)
def test_nan_and_zero_normal(P, solver):
    nx = np.array([np.nan, 0.0, 0.5, 0.0], dtype=np.float32)
    ny = np.array([0.5, 0.0, 0.5, 0.0], dtype=np.float32)
    nz = np.array([0.5, 0.0, np.nan, 0.0], dtype=np.float32)
    V0 = np.array([0.3, 0.3, 0.3, np.nan], dtype=np.float32)
    d0 = gpu_offset(P, nx, ny, nz, V0, solver)
    assert np.isnan(d0).all()


@pytest.mark.parametrize("solver", SOLVERS)
def test_near_degenerate(P, orc, solver):
    """Precision-study workload: normals within 1e-4 rad of axes and diagonals,
    fill levels within 1e-6 of 0, 1 and the case-boundary volumes."""
    nx, ny, nz, V0 = near_degenerate_problems(orc, 200003, seed=3)
    ref = orc.offset(nx, ny, nz, V0)
    for precision in PRECISIONS:
        err = max_abs_err(gpu_offset(P, nx, ny, nz, V0, solver, precision), ref)
        print(f"{solver}/{precision}: near-degenerate max err {err:.3e}")
        assert err <= TOL32
    n64 = [a.astype(np.float64) for a in (nx, ny, nz, V0)]
    assert max_abs_err(gpu_offset(P, *n64, solver), orc.offset(*n64)) <= TOL64


@pytest.mark.parametrize("solver", SOLVERS)
def test_round_trip_complement_determinism(P, small, solver):
    nx, ny, nz, V0, _ = small
    tx, ty, tz, tv = dev(nx, ny, nz, V0)
    d0 = torch.empty_like(tv)
    P.plic_offset_f32(tx, ty, tz, tv, d0, solver, "fp32")
    d1 = torch.empty_like(tv)
    P.plic_offset_f32(tx, ty, tz, tv, d1, solver, "fp32")
    assert torch.equal(d0, d1)                               # bitwise deterministic
    Vb = torch.empty_like(tv)
    P.plic_volume_f32(tx, ty, tz, d0, Vb, "fp64")            # E_i of Sec. 2.6.2
    E = (Vb.double() - tv.double()).abs()
    print(f"{solver}: round trip E_avg {E.mean().item():.3e} E_max {E.max().item():.3e}")
    assert E.max().item() <= 2e-6
    tc = 1.0 - tv                                            # exact for V0 = k 2^-24
    dc = torch.empty_like(tv)
    P.plic_offset_f32(tx, ty, tz, tc, dc, solver, "fp32")
    assert (dc + d0).abs().max().item() <= 2e-6


def test_volume_parity(P, orc, small):
    nx, ny, nz, V0, ref = small
    d = ref.astype(np.float32)
    vref = orc.volume(nx, ny, nz, d)
    tx, ty, tz, td = dev(nx, ny, nz, d)
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-14)):
        out = torch.empty_like(td)
        P.plic_volume_f32(tx, ty, tz, td, out, prec)
        err = max_abs_err(host(out), vref)
        print(f"volume/{prec}: {err:.3e}")
        assert err <= max(tol, 6e-8)   # f32 storage rounds the result
    n64 = [a.astype(np.float64) for a in (nx, ny, nz, d)]
    t64 = dev(*n64)
    out = torch.empty_like(t64[3])
    P.plic_volume_f64(*t64, out)
    assert max_abs_err(host(out), orc.volume(*n64)) <= 1e-14
    # outside [-S/2, S/2] -> 0 / 1; NaN propagates
    e = np.array([5.0, -5.0, np.nan], dtype=np.float32)
    o = np.array([0.6, 0.6, 0.6], dtype=np.float32)
    q = np.array([0.0, 0.0, 0.0], dtype=np.float32)
    t = dev(o, np.full(3, 0.8, np.float32), q, e)
    out = torch.empty_like(t[3])
    P.plic_volume_f32(*t, out)
    h = host(out)
    assert h[0] == 1.0 and h[1] == 0.0 and np.isnan(h[2])


def test_full_size_sampled(P, orc):
    """2^26 problems (the throughput workload), every solver; the oracle checks a
    sample of 2^17 problems plus every forced edge case; the round trip through
    the GPU volume is checked on all 2^26."""
    N = 1 << 26
    nx, ny, nz, V0 = workloads.plic_problems(N, seed=0)
    rng = np.random.default_rng(99)
    edge = np.flatnonzero((V0 == 0) | (V0 == 1) | (np.abs(nx) == 1) | (np.abs(ny) == 1) |
                          (np.abs(nz) == 1) | (nx == 0) | (ny == 0) | (nz == 0))
    idx = np.unique(np.concatenate([rng.choice(N, 1 << 17, replace=False), edge]))
    ref = orc.offset(nx[idx], ny[idx], nz[idx], V0[idx])
    tx, ty, tz, tv = dev(nx, ny, nz, V0)
    d0 = torch.empty_like(tv)
    Vb = torch.empty_like(tv)
    ti = torch.from_numpy(idx).cuda()
    for solver in SOLVERS:
        P.plic_offset_f32(tx, ty, tz, tv, d0, solver, "fp32")
        err = max_abs_err(host(d0[ti]), ref)
        P.plic_volume_f32(tx, ty, tz, d0, Vb, "fp64")
        E = (Vb.double() - tv.double()).abs()
        print(f"{solver}: sampled max err {err:.3e}; round trip E_avg {E.mean().item():.3e} "
              f"E_max {E.max().item():.3e}; NaN {torch.isnan(d0).sum().item()}")
        assert err <= TOL32
        assert not torch.isnan(d0).any()
        assert E.max().item() <= 2e-6
    del tx, ty, tz, tv, d0, Vb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("solver", SOLVERS + ["sz_kawano"])
@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_packing_does_not_change_bits(P, solver, precision):
    """The open problems of a workgroup are packed (and, for Newton, grouped by
    case) before the cubic stage.  Shifting the arrays by one or five elements
    misaligns them (the one-problem-per-lane path) and regroups every problem
    with other neighbours; each result must keep its bits."""
    nx, ny, nz, V0 = workloads.plic_problems((1 << 20) + 37, seed=17)
    t = dev(nx, ny, nz, V0)
    ref = torch.empty_like(t[3])
    P.plic_offset_f32(*t, ref, solver, precision)
    for shift in (1, 5):
        out = torch.empty_like(t[3][shift:])
        P.plic_offset_f32(*(x[shift:] for x in t), out, solver, precision)
        torch.cuda.synchronize()
        assert torch.equal(out.nan_to_num(7.0), ref[shift:].nan_to_num(7.0)), (solver, precision, shift)
