"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Plain, slow reference for PLIC inversion and PLIC curvature, written from the
paper's definitions (see ``plic_oracle.c`` for the passage each routine
follows).  Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library never imports it,
and it imports nothing from the GPU library.

numpy arrays in, numpy float64 arrays out; inputs are converted to float64
exactly (float32 inputs are represented exactly in float64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    c_d, c_i64 = ctypes.c_double, ctypes.c_int64
    lib.orc_volume1.restype = c_d
    lib.orc_volume1.argtypes = [c_d] * 4
    lib.orc_offset1.restype = c_d
    lib.orc_offset1.argtypes = [c_d] * 4
    lib.orc_reduced_volume.restype = c_d
    lib.orc_reduced_volume.argtypes = [c_d] * 4
    lib.orc_offset_grad1.restype = ctypes.c_int
    lib.orc_offset_grad1.argtypes = [c_d] * 4 + [_D, _D, _D, _D]
    lib.orc_volume.argtypes = [_D] * 5 + [c_i64]
    lib.orc_offset.argtypes = [_D] * 5 + [c_i64]
    lib.orc_offset_grad.argtypes = [_D] * 9 + [c_i64]
    lib.orc_offset_kawano.argtypes = [_D] * 5 + [ctypes.POINTER(ctypes.c_int32), _D, c_i64]
    lib.orc_curv_cell.restype = c_d
    lib.orc_curv_cell.argtypes = [_D, _U8, _D]
    lib.orc_curv_cell_full.restype = c_d
    lib.orc_curv_cell_full.argtypes = [_D, _U8, _D, _D, _D]
    lib.orc_curv_cell_r.restype = c_d
    lib.orc_curv_cell_r.argtypes = [_D, _U8, _D, _D, _D, _D]
    lib.orc_fit_paraboloid.restype = ctypes.c_int
    lib.orc_fit_paraboloid.argtypes = [_D, _D, _D, ctypes.c_int, _D, _D]
    lib.orc_paraboloid_kappa.restype = c_d
    lib.orc_paraboloid_kappa.argtypes = [_D]
    lib.orc_curvature.argtypes = [_F, c_i64, c_i64, c_i64, _D, _U8]
    lib.orc_curvature_cells.argtypes = [_F, c_i64, c_i64, c_i64, _I64, c_i64, _D, _D]
    lib.orc_curv_cell_fd_grad.restype = ctypes.c_int
    lib.orc_curv_cell_fd_grad.argtypes = [_D, _U8, c_d, _D]
    lib.orc_curvature_grad.restype = c_i64
    lib.orc_curvature_grad.argtypes = [_F, c_i64, c_i64, c_i64, _F, c_d, _D, _U8]
    lib.orc_sphere_volume1.restype = c_d
    lib.orc_sphere_volume1.argtypes = [c_d]
    lib.orc_sphere_offset1.restype = c_d
    lib.orc_sphere_offset1.argtypes = [c_d]
    lib.orc_sphere_volume.argtypes = [_D, _D, c_i64]
    lib.orc_sphere_offset.argtypes = [_D, _D, c_i64]
    lib.orc_curv_cell_k.restype = c_d
    lib.orc_curv_cell_k.argtypes = [_D, _U8, ctypes.c_int, _D, _D]
    lib.orc_curv_cell_nbr.restype = c_d
    lib.orc_curv_cell_nbr.argtypes = [_D, _U8, ctypes.c_int, _D]
    lib.orc_curvature_ex.argtypes = [_F, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int, _D, _U8]
    lib.orc_curvature_cells_ex.argtypes = [_F, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int, _I64, c_i64,
                                           _D, _D]
    lib.orc_curv_cell_fd_grad_k.restype = ctypes.c_int
    lib.orc_curv_cell_fd_grad_k.argtypes = [_D, _U8, ctypes.c_int, c_d, _D]
    lib.orc_curvature_grad_ex.restype = c_i64
    lib.orc_curvature_grad_ex.argtypes = [_F, c_i64, c_i64, c_i64, ctypes.c_int, _F, c_d, _D, _U8]
    lib.orc_curv_cell_nbr_fd_grad.restype = ctypes.c_int
    lib.orc_curv_cell_nbr_fd_grad.argtypes = [_D, _U8, ctypes.c_int, c_d, _D]
    lib.orc_curvature_grad_nbr.restype = c_i64
    lib.orc_curvature_grad_nbr.argtypes = [_F, c_i64, c_i64, c_i64, ctypes.c_int, _F, c_d, _D, _U8]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=_D):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------- PLIC

def volume(nx, ny, nz, d0):
    """V0(n, d0), elementwise, float64."""
    lib = _load()
    nx, ny, nz, d0 = (_d(a).ravel() for a in np.broadcast_arrays(nx, ny, nz, d0))
    out = np.empty_like(nx)
    lib.orc_volume(_p(nx), _p(ny), _p(nz), _p(d0), _p(out), nx.size)
    return out


def offset(nx, ny, nz, V0):
    """d0(n, V0) by bisection on the forward volume, elementwise, float64."""
    lib = _load()
    nx, ny, nz, V0 = (_d(a).ravel() for a in np.broadcast_arrays(nx, ny, nz, V0))
    out = np.empty_like(nx)
    lib.orc_offset(_p(nx), _p(ny), _p(nz), _p(V0), _p(out), nx.size)
    return out


def offset_kawano(nx, ny, nz, V0):
    """(d0, case, acos argument) of the SZ solution as implemented by Kawano
    (Sec. 2.4), elementwise in float64: NaN for an axis normal at V0 in {0, 1}
    (Sec. 2.6); case 1..5; the argument of acos in the cubic cases, else NaN."""
    lib = _load()
    nx, ny, nz, V0 = (_d(a).ravel() for a in np.broadcast_arrays(nx, ny, nz, V0))
    out, arg = np.empty_like(nx), np.empty_like(nx)
    kase = np.empty(nx.size, dtype=np.int32)
    lib.orc_offset_kawano(_p(nx), _p(ny), _p(nz), _p(V0), _p(out), kase.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          _p(arg), nx.size)
    return out, kase, arg


def offset_grad(nx, ny, nz, V0):
    """(d0, dd0/dV0, dd0/dnx, dd0/dny, dd0/dnz) from the explicit polygon."""
    lib = _load()
    nx, ny, nz, V0 = (_d(a).ravel() for a in np.broadcast_arrays(nx, ny, nz, V0))
    outs = [np.empty_like(nx) for _ in range(5)]
    lib.orc_offset_grad(_p(nx), _p(ny), _p(nz), _p(V0), *(_p(o) for o in outs), nx.size)
    return tuple(outs)


def offset_grad1(nx, ny, nz, V0):
    """Single problem: (d0, dd0/dV0, (dd0/dn), area, n_vertices)."""
    lib = _load()
    d0, dv, area = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    g = (ctypes.c_double * 3)()
    nv = lib.orc_offset_grad1(float(nx), float(ny), float(nz), float(V0), ctypes.byref(d0),
                              ctypes.byref(dv), g, ctypes.byref(area))
    return d0.value, dv.value, np.array(list(g)), area.value, nv


def reduced_volume(a1, a2, a3, u):
    return _load().orc_reduced_volume(float(a1), float(a2), float(a3), float(u))


def volume1(nx, ny, nz, d0):
    return _load().orc_volume1(float(nx), float(ny), float(nz), float(d0))


def offset1(nx, ny, nz, V0):
    return _load().orc_offset1(float(nx), float(ny), float(nz), float(V0))


# ---------------------------------------------------------------- curvature

def curv_cell(phi27, mask27=None, full=False):
    """Curvature of one 3^3 neighbourhood, phi27[q], q = (dz+1)*9+(dy+1)*3+(dx+1).
    Returns kappa (and with ``full``: info[3], normal[3], coef[5])."""
    lib = _load()
    p = _d(phi27).ravel()
    if mask27 is None:
        mask27 = (p > 0) & (p < 1)
    m = np.ascontiguousarray(np.asarray(mask27, dtype=np.uint8).ravel())
    info = np.zeros(3)
    if not full:
        return lib.orc_curv_cell(_p(p), _p(m, _U8), _p(info))
    nrm = np.zeros(3)
    coef = np.zeros(5)
    k = lib.orc_curv_cell_full(_p(p), _p(m, _U8), _p(info), _p(nrm), _p(coef))
    return k, info, nrm, coef


def curv_cell_r(phi27, raux, mask27=None):
    """Curvature of one neighbourhood with a chosen auxiliary vector r."""
    lib = _load()
    p = _d(phi27).ravel()
    if mask27 is None:
        mask27 = (p > 0) & (p < 1)
    m = np.ascontiguousarray(np.asarray(mask27, dtype=np.uint8).ravel())
    r = _d(raux).ravel()
    info, nrm, coef = np.zeros(3), np.zeros(3), np.zeros(5)
    k = lib.orc_curv_cell_r(_p(p), _p(m, _U8), _p(r), _p(info), _p(nrm), _p(coef))
    return k, info, coef


def fit_paraboloid(px, py, pz):
    lib = _load()
    px, py, pz = _d(px), _d(py), _d(pz)
    coef = np.zeros(5)
    cond = ctypes.c_double()
    bits = lib.orc_fit_paraboloid(_p(px), _p(py), _p(pz), int(px.size), _p(coef),
                                  ctypes.cast(ctypes.pointer(cond), _D))
    return coef, bits, cond.value


def paraboloid_kappa(coef):
    c = _d(coef)
    return _load().orc_paraboloid_kappa(_p(c))


def sphere_volume(d0):
    """volume of the unit-volume sphere below the plane at distance d0 (Sec. 3)"""
    d = _d(d0)
    out = np.empty_like(d)
    _load().orc_sphere_volume(_p(d), _p(out), d.size)
    return out


def sphere_offset(V0):
    """inverse of sphere_volume by bisection (the plane-sphere PLIC problem)"""
    v = _d(V0)
    out = np.empty_like(v)
    _load().orc_sphere_offset(_p(v), _p(out), v.size)
    return out


def sphere_radius() -> float:
    return float(np.cbrt(3.0 / (4.0 * np.pi)))


NORMALS = {"py": 0, "cm": 1}


def _kind(normal):
    if normal not in NORMALS:
        raise ValueError(f"normal must be one of {sorted(NORMALS)}")
    return NORMALS[normal]


def curvature(phi, flags=False, normal="py", neighbour_normals=False):
    """kappa over a (Z, Y, X) float32 lattice, float64 out (and per-cell flags).
    normal: "py" (Parker-Youngs) or "cm" (centre of mass), App. B.1;
    neighbour_normals: each interface neighbour's plane uses its own normal."""
    lib = _load()
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
    Z, Y, X = phi.shape
    k = np.empty(phi.shape, dtype=np.float64)
    fl = np.empty(phi.shape, dtype=np.uint8)
    lib.orc_curvature_ex(_p(phi, _F), X, Y, Z, _kind(normal), int(bool(neighbour_normals)), _p(k), _p(fl, _U8))
    return (k, fl) if flags else k


def curvature_cells(phi, cells, normal="py", neighbour_normals=False):
    """kappa at selected linear cell indices, plus info[ncells, 3]."""
    lib = _load()
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
    Z, Y, X = phi.shape
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    k = np.empty(cells.size)
    info = np.empty((cells.size, 3))
    lib.orc_curvature_cells_ex(_p(phi, _F), X, Y, Z, _kind(normal), int(bool(neighbour_normals)),
                               _p(cells, _I64), cells.size, _p(k), _p(info))
    return k, info


def curv_cell_k(phi27, normal="py", mask27=None):
    """one cell with the chosen normal; returns (kappa, info[3], normal[3])"""
    lib = _load()
    p = _d(phi27).ravel()
    if mask27 is None:
        mask27 = (p > 0) & (p < 1)
    m = np.ascontiguousarray(np.asarray(mask27, dtype=np.uint8).ravel())
    info, n = np.zeros(3), np.zeros(3)
    k = lib.orc_curv_cell_k(_p(p), _p(m, _U8), _kind(normal), _p(info), _p(n))
    return k, info, n


def curv_cell_nbr(phi125, normal="py", inside27=None):
    """neighbour-normal variant on a 5^3 neighbourhood [dz+2][dy+2][dx+2];
    inside27[q] = 0 makes neighbour q keep the centre normal"""
    lib = _load()
    p = _d(phi125).ravel()
    assert p.size == 125
    ins = np.ones(27, np.uint8) if inside27 is None else np.ascontiguousarray(np.asarray(inside27, np.uint8).ravel())
    info = np.zeros(3)
    return lib.orc_curv_cell_nbr(_p(p), _p(ins, _U8), _kind(normal), _p(info)), info


def curv_cell_fd_grad(phi27, mask27=None, h=1e-6, normal="py"):
    lib = _load()
    p = _d(phi27).ravel()
    if mask27 is None:
        mask27 = (p > 0) & (p < 1)
    m = np.ascontiguousarray(np.asarray(mask27, dtype=np.uint8).ravel())
    g = np.zeros(27)
    bad = lib.orc_curv_cell_fd_grad_k(_p(p), _p(m, _U8), _kind(normal), float(h), _p(g))
    return g, bool(bad)


def curv_cell_nbr_fd_grad(phi125, normal="py", inside27=None, h=1e-6):
    """central-difference gradient of the neighbour-normal cell over its 5^3
    neighbourhood (index (dz+2)*25 + (dy+2)*5 + (dx+2)); bad when a mask or the
    fit's rank would change"""
    v = _d(phi125).ravel()
    ins = None if inside27 is None else np.ascontiguousarray(np.asarray(inside27, dtype=np.uint8))
    g = np.empty(125)
    bad = _load().orc_curv_cell_nbr_fd_grad(_p(v), None if ins is None else _p(ins, _U8), _kind(normal), float(h), _p(g))
    return g, bool(bad)


def curvature_grad(phi, grad_kappa, h=1e-6, normal="py", neighbour_normals=False):
    """grad_phi (float64) of sum(grad_kappa * kappa) by finite differences of the
    oracle's curvature with the interface mask fixed; also the bad-cell mask.
    With neighbour_normals, of the neighbour-normal variant (5^3 per cell)."""
    lib = _load()
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
    gk = np.ascontiguousarray(np.asarray(grad_kappa, dtype=np.float32))
    Z, Y, X = phi.shape
    out = np.empty(phi.shape, dtype=np.float64)
    bad = np.empty(phi.shape, dtype=np.uint8)
    fn = lib.orc_curvature_grad_nbr if neighbour_normals else lib.orc_curvature_grad_ex
    fn(_p(phi, _F), X, Y, Z, _kind(normal), _p(gk, _F), float(h), _p(out), _p(bad, _U8))
    return out, bad.astype(bool)


def _gomp():
    _load()                                   # the oracle links the OpenMP runtime
    return ctypes.CDLL("libgomp.so.1")


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_gomp().omp_get_max_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (for timing it on one core)."""
    _gomp().omp_set_num_threads(int(n))


def curvature_grad_richardson(phi, grad_kappa, h=1e-5, normal="py", neighbour_normals=False):
    """curvature_grad with Richardson extrapolation of the central differences:
    (4 g(h) - g(2h)) / 3 cancels their O(h^2) term.  Bad cells are those of
    either step (a perturbation by 2h that would cross 0 or 1, or change the
    fit's parameter set)."""
    g1, b1 = curvature_grad(phi, grad_kappa, h=h, normal=normal, neighbour_normals=neighbour_normals)
    g2, b2 = curvature_grad(phi, grad_kappa, h=2 * h, normal=normal, neighbour_normals=neighbour_normals)
    return (4.0 * g1 - g2) / 3.0, b1 | b2
