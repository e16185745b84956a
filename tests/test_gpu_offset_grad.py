"""GPU backward of plic_offset against the oracle's explicit-polygon gradient
(dd0/dV0 = |n|/A, dd0/dn = centroid) and against central finite differences of
the GPU forward; the torch.autograd.Function wiring; fwd+bwd at 2^24.

Bars with FP32 storage, every precision mode: dd0/dV0 relative 1e-5 (measured
at most 1.1e-6 with V0 in [0.01, 0.99]: the FP32 rounding of the root and of
1/A), the centroid absolute 2e-5 times the largest upstream gradient."""
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


def interior_problems(n, seed, dtype=np.float32):
    nx, ny, nz, V0 = workloads.plic_problems(n, seed=seed, edge_frac=0.0, dtype=dtype)
    rng = np.random.default_rng(seed + 100)
    V0 = rng.uniform(0.01, 0.99, n).astype(dtype)
    return nx, ny, nz, V0


def gpu_backward(P, nx, ny, nz, V0, gd, solver, precision="fp32"):
    t = dev(nx, ny, nz, V0, gd)
    outs = [torch.empty_like(t[0]) for _ in range(4)]
    if t[0].dtype == torch.float64:
        P.plic_offset_backward_f64(*t, *outs, solver)
    else:
        P.plic_offset_backward_f32(*t, *outs, solver, precision)
    return [host(o) for o in outs]


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("precision", ["fp32", "mixed", "fp64"])
def test_backward_matches_oracle_f32(P, orc, solver, precision):
    nx, ny, nz, V0 = interior_problems(200003, seed=5)
    gd = workloads.upstream_grad(V0.size, seed=6)
    _, dv, gx, gy, gz = orc.offset_grad(nx, ny, nz, V0)
    ox, oy, oz, ov = gpu_backward(P, nx, ny, nz, V0, gd, solver, precision)
    g64 = gd.astype(np.float64)
    rel_v = np.abs(ov - g64 * dv) / np.maximum(np.abs(g64 * dv), 1e-30)
    # dV error is relative (|n|/A can be large for small polygons)
    print(f"{solver}/{precision}: max relative error of dd0/dV0 {rel_v.max():.2e}")
    assert rel_v.max() <= 1e-5
    for o, r in ((ox, gx), (oy, gy), (oz, gz)):
        assert np.max(np.abs(o - g64 * r)) <= 2e-5 * max(1.0, np.abs(g64).max())


@pytest.mark.parametrize("solver", SOLVERS)
def test_backward_matches_oracle_f64(P, orc, solver):
    nx, ny, nz, V0 = interior_problems(100003, seed=7, dtype=np.float64)
    gd = workloads.upstream_grad(V0.size, seed=8, dtype=np.float64)
    _, dv, gx, gy, gz = orc.offset_grad(nx, ny, nz, V0)
    ox, oy, oz, ov = gpu_backward(P, nx, ny, nz, V0, gd, solver)
    assert np.max(np.abs(ov - gd * dv) / np.abs(gd * dv)) <= 1e-9
    for o, r in ((ox, gx), (oy, gy), (oz, gz)):
        assert np.max(np.abs(o - gd * r)) <= 1e-11


def test_backward_against_finite_differences(P):
    """Central differences of the GPU FP64 forward with h = 1e-3 (O(h^2) error)."""
    nx, ny, nz, V0 = interior_problems(4099, seed=9, dtype=np.float64)
    V0 = np.clip(V0, 0.02, 0.98)
    h = 1e-3
    ones = np.ones_like(V0)
    ox, oy, oz, ov = gpu_backward(P, nx, ny, nz, V0, ones, "analytic")

    def fwd(a, b, c, v):
        t = dev(a, b, c, v)
        d = torch.empty_like(t[0])
        P.plic_offset_f64(*t, d, "analytic")
        return host(d)

    fdv = (fwd(nx, ny, nz, V0 + h) - fwd(nx, ny, nz, V0 - h)) / (2 * h)
    fdx = (fwd(nx + h, ny, nz, V0) - fwd(nx - h, ny, nz, V0)) / (2 * h)
    fdz = (fwd(nx, ny, nz + h, V0) - fwd(nx, ny, nz - h, V0)) / (2 * h)
    # exclude problems whose +-h step crosses a case boundary of the polygon
    for a, b in ((ov, fdv), (ox, fdx), (oz, fdz)):
        err = np.abs(a - b) / np.maximum(1.0, np.abs(a))
        assert np.quantile(err, 0.99) <= 1e-3


def test_autograd_function(P, orc):
    nx, ny, nz, V0 = interior_problems(10007, seed=10)
    tn = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (nx, ny, nz, V0)]
    n = torch.stack(tn[:3], -1)
    d0 = P.offset(n, tn[3], solver="sz")
    w = torch.from_numpy(workloads.upstream_grad(V0.size, seed=11)).cuda()
    (d0 * w).sum().backward()
    _, dv, gx, gy, gz = orc.offset_grad(nx, ny, nz, V0)
    wn = host(w).astype(np.float64)
    assert np.max(np.abs(host(tn[0].grad) - wn * gx)) <= 2e-5 * np.abs(wn).max()
    assert np.max(np.abs(host(tn[3].grad) - wn * dv) / np.abs(wn * dv)) <= 1e-5
    # float64 tensors take the f64 entry points
    t64 = [torch.from_numpy(a.astype(np.float64)).cuda().requires_grad_(True) for a in (nx, ny, nz, V0)]
    P.offset(tuple(t64[:3]), t64[3]).sum().backward()
    assert np.max(np.abs(host(t64[3].grad) - dv) / dv) <= 1e-9


def test_degenerate_polygon_gradient(P):
    # V0 = 0 with a generic normal: the polygon is a corner, dd0/dV0 = +inf
    nx = np.array([0.3, 1.0], np.float32)
    ny = np.array([0.5, 0.0], np.float32)
    nz = np.array([0.8, 0.0], np.float32)
    V0 = np.array([0.0, 0.0], np.float32)
    ox, oy, oz, ov = gpu_backward(P, nx, ny, nz, V0, np.ones(2, np.float32), "analytic")
    assert np.isinf(ov[0]) and ov[0] > 0
    assert ov[1] == pytest.approx(1.0)                 # axis normal: the polygon is a face
    assert np.allclose([ox[1], oy[1], oz[1]], [-0.5, 0.0, 0.0])


def test_fwd_bwd_2p24_sampled(P, orc):
    """Differentiation workload: fwd + bwd on 2^24 problems, upstream N(0,1)."""
    N = 1 << 24
    nx, ny, nz, V0 = workloads.plic_problems(N, seed=4, edge_frac=0.0)
    gd = workloads.upstream_grad(N, seed=12)
    t = dev(nx, ny, nz, V0, gd)
    outs = [torch.empty_like(t[0]) for _ in range(4)]
    P.plic_offset_backward_f32(*t, *outs, "sz", "fp32")
    rng = np.random.default_rng(13)
    idx = rng.choice(N, 1 << 15, replace=False)
    idx = idx[(V0[idx] > 0.01) & (V0[idx] < 0.99)]
    _, dv, gx, gy, gz = orc.offset_grad(nx[idx], ny[idx], nz[idx], V0[idx])
    ti = torch.from_numpy(idx).cuda()
    g = gd[idx].astype(np.float64)
    rel = np.abs(host(outs[3][ti]) - g * dv) / np.abs(g * dv)
    print(f"2^24 sampled: max relative error of dd0/dV0 {rel.max():.2e}")
    assert rel.max() <= 1e-5
    assert np.max(np.abs(host(outs[0][ti]) - g * gx)) <= 2e-5 * np.abs(g).max()
