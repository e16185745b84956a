"""PLIC inversion and PLIC curvature on AMD MI355X (gfx950).

Lehmann & Gekle, "Analytic Solution to the Piecewise Linear Interface
Construction Problem and its Application in Curvature Calculation for
Volume-of-Fluid Simulation Codes" (arXiv 2006.12838).

All computation runs in the hand-written HIP kernels of ``libplic.so``; this
package marshals torch tensors (device memory, the current stream) into its C
ABI and wraps the forward/backward pairs as ``torch.autograd.Function``s.

    d0 = offset(n, V0, solver="sz")          # n (..., 3), V0 (...) -> d0 (...)
    V0 = volume(n, d0)
    kappa = curvature(phi)                   # phi (Z, Y, X) float32
"""
from __future__ import annotations

import torch

from ._lib import (  # noqa: F401  (re-exported: the C ABI by name)
    EXPORTED,
    NORMALS,
    PAPER_SOLVERS,
    PRECISIONS,
    SOLVERS,
    VALU_OPS,
    plic_bench_isolated_f32,
    plic_bench_valu,
    plic_curvature_backward_ex_f32,
    plic_curvature_backward_f32,
    plic_curvature_backward_reuse_f32,
    plic_curvature_ex_f32,
    plic_curvature_f32,
    plic_curvature_noalloc_f32,
    plic_curvature_status,
    plic_curvature_workspace_bytes,
    plic_curvature_workspace_bytes_ex,
    plic_last_hip_error,
    plic_offset_backward_f32,
    plic_offset_backward_f64,
    plic_offset_f32,
    plic_offset_f64,
    plic_sphere_offset_f32,
    plic_sphere_offset_f64,
    plic_sphere_volume_f32,
    plic_sphere_volume_f64,
    plic_status_string,
    plic_version,
    plic_volume_f32,
    plic_volume_f64,
)

__all__ = ["offset", "volume", "curvature", "PlicOffset", "PlicCurvature", "SOLVERS", "PAPER_SOLVERS", "PRECISIONS",
           "NORMALS",
           "plic_version"]


def _split_normal(n):
    if isinstance(n, (tuple, list)):
        if len(n) != 3:
            raise ValueError("normal must be three tensors (nx, ny, nz)")
        return tuple(n)
    if n.shape[-1] != 3:
        raise ValueError("normal tensor must have a trailing dimension of 3")
    return n.unbind(-1)


class PlicOffset(torch.autograd.Function):
    """d0(n, V0) with the backward dd0/dV0 = |n|/A, dd0/dn = polygon centroid."""

    @staticmethod
    def forward(ctx, nx, ny, nz, V0, solver="sz", precision="fp32"):
        shape = V0.shape
        nx, ny, nz, V0 = (t.contiguous().reshape(-1) for t in torch.broadcast_tensors(nx, ny, nz, V0))
        d0 = torch.empty_like(V0)
        if V0.dtype == torch.float64:
            plic_offset_f64(nx, ny, nz, V0, d0, solver)
        else:
            plic_offset_f32(nx, ny, nz, V0, d0, solver, precision)
        ctx.save_for_backward(nx, ny, nz, V0)
        ctx.solver, ctx.precision, ctx.shape = solver, precision, shape
        return d0.reshape(shape)

    @staticmethod
    def backward(ctx, grad_d0):
        nx, ny, nz, V0 = ctx.saved_tensors
        g = grad_d0.contiguous().reshape(-1)
        gx, gy, gz, gv = (torch.empty_like(V0) for _ in range(4))
        if V0.dtype == torch.float64:
            plic_offset_backward_f64(nx, ny, nz, V0, g, gx, gy, gz, gv, ctx.solver)
        else:
            plic_offset_backward_f32(nx, ny, nz, V0, g, gx, gy, gz, gv, ctx.solver, ctx.precision)
        s = ctx.shape
        return gx.reshape(s), gy.reshape(s), gz.reshape(s), gv.reshape(s), None, None


def offset(n, V0, solver: str = "sz", precision: str = "fp32"):
    """Plane offset d0 of the PLIC problem for normals ``n`` and fill levels ``V0``.

    ``n`` is a (..., 3) tensor or a tuple (nx, ny, nz); float32 tensors use the
    chosen ``precision`` ("fp32", "mixed", "fp64"), float64 tensors compute in
    FP64.  ``solver``: "analytic", "sz", "newton", "nested", or "sz_kawano" (the
    unoptimized SZ comparison variant: NaN for an axis normal at V0 in {0, 1},
    not held to the 1e-5 bound)."""
    nx, ny, nz = _split_normal(n)
    return PlicOffset.apply(nx, ny, nz, V0, solver, precision)


def volume(n, d0, precision: str = "fp32"):
    """Forward volume V0(n, d0) (no gradient)."""
    nx, ny, nz = _split_normal(n)
    shape = d0.shape
    nx, ny, nz, d0 = (t.detach().contiguous().reshape(-1) for t in torch.broadcast_tensors(nx, ny, nz, d0))
    out = torch.empty_like(d0)
    if d0.dtype == torch.float64:
        plic_volume_f64(nx, ny, nz, d0, out)
    else:
        plic_volume_f32(nx, ny, nz, d0, out, precision)
    return out.reshape(shape)


class PlicCurvature(torch.autograd.Function):
    """kappa(phi) on a (Z, Y, X) lattice with the recomputing backward.  The
    forward's workspace is kept for the backward, which reuses its interface
    scan (autograd's saved-tensor check rejects a phi changed in place)."""

    @staticmethod
    def forward(ctx, phi, solver="analytic", precision="mixed", normal="py", neighbour_normals=False):
        phi = phi.contiguous()
        kappa = torch.empty_like(phi)
        Z, Y, X = phi.shape
        ws = torch.empty(max(plic_curvature_workspace_bytes_ex(X, Y, Z, neighbour_normals), 1), dtype=torch.uint8,
                         device=phi.device)
        plic_curvature_ex_f32(phi, kappa, solver, precision, normal, neighbour_normals, ws)
        ctx.save_for_backward(phi)
        ctx.opts = (solver, precision, normal, neighbour_normals)
        ctx.ws = ws
        return kappa

    @staticmethod
    def backward(ctx, grad_kappa):
        (phi,) = ctx.saved_tensors
        solver, precision, normal, neighbour_normals = ctx.opts
        grad_phi = torch.empty_like(phi)
        plic_curvature_backward_ex_f32(phi, grad_kappa.contiguous(), grad_phi, solver, precision, normal,
                                       neighbour_normals, ctx.ws, reuse=True, grow=True)
        ctx.ws = None
        return grad_phi, None, None, None, None


def curvature(phi, solver: str = "analytic", precision: str = "mixed", normal: str = "py",
              neighbour_normals: bool = False):
    """Mean curvature kappa of the VoF lattice ``phi`` (float32, shape (Z, Y, X)):
    0 off the interface, +1/R for a fluid sphere of radius R.  normal: "py"
    (Parker-Youngs) or "cm" (centre of mass); neighbour_normals: each interface
    neighbour's PLIC plane from its own normal."""
    return PlicCurvature.apply(phi, solver, precision, normal, neighbour_normals)
