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
    """The precision-study workload: normals within 1e-4 rad of an axis, face or
    space diagonal, fill levels within 1e-6 of 0, 1 or a case-boundary volume.
    Boundary volumes come from the oracle's forward volume at the boundary
    offsets the generator names."""
    import workloads

    nrm, which, comp, jit = workloads.near_degenerate_normals(n, seed)
    nrm = nrm.astype(dtype).astype(np.float64)
    a = np.sort(np.abs(nrm), axis=1)
    S = a.sum(1)
    dred = np.select([which == 0, which == 1, which == 2, which == 3],
                     [np.zeros(n), a[:, 0], a[:, 1], np.minimum(a[:, 0] + a[:, 1], a[:, 2])],
                     0.5 * S)
    V = orc.volume(nrm[:, 0], nrm[:, 1], nrm[:, 2], dred - 0.5 * S)
    V = np.where(comp, 1.0 - V, V) + jit
    V = np.clip(V, 0.0, 1.0).astype(dtype)
    nrm = nrm.astype(dtype)
    return (np.ascontiguousarray(nrm[:, 0]), np.ascontiguousarray(nrm[:, 1]),
            np.ascontiguousarray(nrm[:, 2]), V)
