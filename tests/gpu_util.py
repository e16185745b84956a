"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import torch

SOLVERS = ["analytic", "sz", "newton", "nested"]
PRECISIONS = ["fp32", "mixed", "fp64"]


def dev(*arrays):
    out = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]
    return out if len(out) > 1 else out[0]


def host(t):
    return t.detach().cpu().numpy()


def gpu_offset(P, nx, ny, nz, V0, solver, precision="fp32"):
    tx, ty, tz, tv = dev(nx, ny, nz, V0)
    d0 = torch.empty_like(tv)
    if tv.dtype == torch.float64:
        P.plic_offset_f64(tx, ty, tz, tv, d0, solver)
    else:
        P.plic_offset_f32(tx, ty, tz, tv, d0, solver, precision)
    return host(d0)


def max_abs_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_nan = np.isnan(a) & np.isnan(b)
    d = np.abs(a - b)
    d[both_nan] = 0.0
    d[np.isnan(d)] = np.inf
    return float(d.max()) if d.size else 0.0


def near_degenerate_problems(orc, n, seed, dtype=np.float32):
    """The precision-study workload (workloads.near_degenerate_problems) with
    the boundary volumes from the oracle's forward volume."""
    import workloads

    return workloads.near_degenerate_problems(orc.volume, n, seed, dtype)
