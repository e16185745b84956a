"""Precision study: every solver and precision mode on 2^24 near-degenerate
problems (normals within 1e-4 rad of the axes and diagonals, fill levels
within 1e-6 of 0, 1 and the case-boundary volumes), and the curvature modes
on the 256^3 sphere of radius 40, against the FP64 oracle.

Prints one table per workload (max / RMS error, time per call) and asserts the
parity bars: |d0 - d0_ref| <= 1e-5 for FP32 storage (every mode), <= 1e-12 for
FP64 storage, and the per-cell curvature bar of the curvature tests."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import PRECISIONS, SOLVERS, dev, host, near_degenerate_problems
from tests.test_gpu_curvature import cell_reference, check_against

pytestmark = pytest.mark.gpu

TOL32, TOL64 = 1e-5, 1e-12


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


def timed(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e3


def stats(err):
    err = np.asarray(err, dtype=np.float64)
    return float(err.max()), float(np.sqrt(np.mean(err * err)))


def test_offset_modes_near_degenerate(P, orc):
    n = 1 << 24
    nx, ny, nz, V0 = near_degenerate_problems(orc, n, seed=11)
    ref = orc.offset(nx, ny, nz, V0)
    n64 = [a.astype(np.float64) for a in (nx, ny, nz, V0)]
    t32 = dev(nx, ny, nz, V0)
    t64 = dev(*n64)
    rows = []
    for solver in SOLVERS:
        for mode in PRECISIONS + ["f64 storage"]:
            if mode == "f64 storage":
                out = torch.empty_like(t64[3])
                fn = lambda: P.plic_offset_f64(*t64, out, solver)
            else:
                out = torch.empty_like(t32[3])
                fn = lambda: P.plic_offset_f32(*t32, out, solver, mode)
            us = timed(fn)
            d0 = host(out).astype(np.float64)
            assert not np.isnan(d0).any()
            dmax, drms = stats(np.abs(d0 - ref))
            # round trip through the oracle's FP64 forward volume
            vmax, vrms = stats(np.abs(orc.volume(*n64[:3], d0) - n64[3]))
            rows.append((solver, mode, dmax, drms, vmax, vrms, us))
            assert dmax <= (TOL64 if mode == "f64 storage" else TOL32), (solver, mode, dmax)
    print(f"\nnear-degenerate set, 2^24 problems: error against the FP64 oracle")
    print(f"{'solver':9s} {'mode':12s} {'max|dd0|':>10s} {'rms|dd0|':>10s} {'max|dV|':>10s} {'rms|dV|':>10s} {'us/call':>9s}")
    for r in rows:
        print(f"{r[0]:9s} {r[1]:12s} {r[2]:10.2e} {r[3]:10.2e} {r[4]:10.2e} {r[5]:10.2e} {r[6]:9.1f}")


def test_curvature_modes_sphere(P, orc):
    phi, _ = workloads.sphere_lattice(N=256, R=40.0, seed=0)
    ref = cell_reference(orc, phi)
    tp = dev(phi)
    ws = torch.empty(P.plic_curvature_workspace_bytes(256, 256, 256), dtype=torch.uint8, device="cuda")
    rows = []
    for solver in ("analytic", "sz"):
        for mode in PRECISIONS:
            k = torch.empty_like(tp)
            us = timed(lambda: P.plic_curvature_f32(tp, k, solver, mode, ws))
            kg, kr, good = check_against(ref, phi, host(k), mode, f"256^3 {solver}/{mode}")
            kg, kr = kg[good], kr[good]
            emax, erms = stats(np.abs(kg - kr))
            rmax, rrms = stats(np.abs(kg - kr) * 40.0)          # relative to the sphere's 1/R
            rows.append((solver, mode, int(good.sum()), emax, erms, rmax, rrms, float(np.mean(kg)) * 40.0, us))
    print(f"\n256^3 sphere R = 40: kappa on well-conditioned interface cells against the FP64 oracle")
    print(f"{'solver':9s} {'mode':6s} {'cells':>6s} {'max|dk|':>10s} {'rms|dk|':>10s} {'max|dk|R':>10s} {'rms|dk|R':>10s} {'mean kR':>8s} {'us/call':>9s}")
    for r in rows:
        print(f"{r[0]:9s} {r[1]:6s} {r[2]:6d} {r[3]:10.2e} {r[4]:10.2e} {r[5]:10.2e} {r[6]:10.2e} {r[7]:8.4f} {r[8]:9.1f}")
