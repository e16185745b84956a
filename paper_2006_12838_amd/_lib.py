"""ctypes binding of libplic.so: one Python function per C entry point, same
names, argument marshalling only (torch tensors -> device pointers, the
current torch stream -> hipStream_t).  Every computation runs in the library's
HIP kernels; a missing library is an ImportError, never a fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads torch's HIP runtime first; libplic binds to the same one

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libplic.so")

PLIC_OK, PLIC_EINVAL, PLIC_EHIP, PLIC_EWORKSPACE = 0, -1, -2, -3
SOLVERS = {"analytic": 0, "sz": 1, "newton": 2, "nested": 3, "sz_kawano": 4}
# the paper's four solvers, held to the accuracy bound; "sz_kawano" is the
# unoptimized comparison variant (offset, offset backward, benchmark only)
PAPER_SOLVERS = ("analytic", "sz", "newton", "nested")
PRECISIONS = {"fp32": 0, "mixed": 1, "fp64": 2}
NORMALS = {"py": 0, "cm": 1}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_2006_12838_amd/_build.py)")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int


def _sig(name, args):
    f = getattr(_lib, name)
    f.restype = ctypes.c_int
    f.argtypes = args
    return f


_c = {
    "plic_offset_f32": _sig("plic_offset_f32", [_vp] * 5 + [_i64, _int, _int, _vp]),
    "plic_offset_f64": _sig("plic_offset_f64", [_vp] * 5 + [_i64, _int, _vp]),
    "plic_volume_f32": _sig("plic_volume_f32", [_vp] * 5 + [_i64, _int, _vp]),
    "plic_volume_f64": _sig("plic_volume_f64", [_vp] * 5 + [_i64, _vp]),
    "plic_offset_backward_f32": _sig("plic_offset_backward_f32", [_vp] * 9 + [_i64, _int, _int, _vp]),
    "plic_offset_backward_f64": _sig("plic_offset_backward_f64", [_vp] * 9 + [_i64, _int, _vp]),
    "plic_curvature_f32": _sig("plic_curvature_f32",
                               [_vp, _i64, _i64, _i64, _vp, _int, _int, _vp, ctypes.c_size_t, _vp]),
    "plic_curvature_noalloc_f32": _sig("plic_curvature_noalloc_f32", [_vp, _i64, _i64, _i64, _vp, _int, _int, _vp]),
    "plic_curvature_backward_f32": _sig("plic_curvature_backward_f32",
                                        [_vp, _i64, _i64, _i64, _vp, _vp, _int, _int, _vp,
                                         ctypes.c_size_t, _vp]),
    "plic_bench_isolated_f32": _sig("plic_bench_isolated_f32",
                                    [_vp, _vp, _vp, _i64, _int, _int, _int, _vp, _vp, _vp]),
    "plic_bench_valu": _sig("plic_bench_valu", [_int, _i64, _int, ctypes.c_float, _vp, _vp]),
    "plic_sphere_offset_f32": _sig("plic_sphere_offset_f32", [_vp, _vp, _i64, _vp]),
    "plic_sphere_offset_f64": _sig("plic_sphere_offset_f64", [_vp, _vp, _i64, _vp]),
    "plic_sphere_volume_f32": _sig("plic_sphere_volume_f32", [_vp, _vp, _i64, _vp]),
    "plic_sphere_volume_f64": _sig("plic_sphere_volume_f64", [_vp, _vp, _i64, _vp]),
    "plic_curvature_ex_f32": _sig("plic_curvature_ex_f32",
                                  [_vp, _i64, _i64, _i64, _vp, _int, _int, _int, _int, _vp, ctypes.c_size_t, _vp]),
    "plic_curvature_backward_ex_f32": _sig("plic_curvature_backward_ex_f32",
                                           [_vp, _i64, _i64, _i64, _vp, _vp, _int, _int, _int, _int, _vp,
                                            ctypes.c_size_t, _vp]),
    "plic_curvature_backward_reuse_f32": _sig("plic_curvature_backward_reuse_f32",
                                              [_vp, _i64, _i64, _i64, _vp, _vp, _int, _int, _int, _int, _vp,
                                               ctypes.c_size_t, _vp]),
}
_lib.plic_curvature_workspace_bytes.restype = ctypes.c_size_t
_lib.plic_curvature_workspace_bytes.argtypes = [_i64, _i64, _i64]
_lib.plic_curvature_workspace_bytes_ex.restype = ctypes.c_size_t
_lib.plic_curvature_workspace_bytes_ex.argtypes = [_i64, _i64, _i64, _int]
_lib.plic_curvature_status.restype = ctypes.c_int
_lib.plic_curvature_status.argtypes = [_vp, ctypes.c_size_t, _i64, _i64, _i64, _int,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t), _vp]
_lib.plic_status_string.restype = ctypes.c_char_p
_lib.plic_status_string.argtypes = [_int]
_lib.plic_version.restype = ctypes.c_char_p
_lib.plic_version.argtypes = []
_lib.plic_last_hip_error.restype = ctypes.c_int
_lib.plic_last_hip_error.argtypes = []

EXPORTED = tuple(_c) + ("plic_status_string", "plic_version", "plic_last_hip_error",
                        "plic_curvature_workspace_bytes", "plic_curvature_workspace_bytes_ex",
                        "plic_curvature_status")


def plic_curvature_workspace_bytes(X: int, Y: int, Z: int) -> int:
    return int(_lib.plic_curvature_workspace_bytes(int(X), int(Y), int(Z)))


def plic_curvature_workspace_bytes_ex(X: int, Y: int, Z: int, neighbour_normals: bool = False) -> int:
    return int(_lib.plic_curvature_workspace_bytes_ex(int(X), int(Y), int(Z), int(bool(neighbour_normals))))


def plic_curvature_status(workspace, X: int, Y: int, Z: int, neighbour_normals: bool = False, stream=None):
    """(status, interface_cells, bytes_for_all_rows) of the last curvature call
    on ``workspace`` (a uint8 device tensor); synchronises ``stream`` (default:
    the current stream of the workspace's device)."""
    cells, need = ctypes.c_int64(0), ctypes.c_size_t(0)
    st = ctypes.c_void_p(stream) if stream is not None else _stream(workspace)
    rc = _lib.plic_curvature_status(ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(X), int(Y),
                                    int(Z), int(bool(neighbour_normals)), ctypes.byref(cells), ctypes.byref(need),
                                    st)
    return int(rc), int(cells.value), int(need.value)


def plic_status_string(status: int) -> str:
    return _lib.plic_status_string(int(status)).decode()


def plic_version() -> str:
    return _lib.plic_version().decode()


def plic_last_hip_error() -> int:
    return int(_lib.plic_last_hip_error())


def raw(name):
    """The raw ctypes function (plain integers / pointers in, status out)."""
    return _c[name]


def _check(status: int, name: str):
    if status != PLIC_OK:
        extra = f" (hipError {plic_last_hip_error()})" if status == PLIC_EHIP else ""
        raise RuntimeError(f"{name}: {plic_status_string(status)}{extra}")


def _ptr(t: torch.Tensor, dtype, n: int, what: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must live on a GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what}: expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _enum(table, value, what):
    if isinstance(value, int):
        return value
    try:
        return table[value]
    except KeyError:
        raise ValueError(f"unknown {what} {value!r}; one of {sorted(table)}") from None


def _same_device(*ts):
    dev = ts[0].device
    for t in ts[1:]:
        if t.device != dev:
            raise ValueError("all tensors must be on the same device")


# ---------------------------------------------------------------- entry points

def plic_offset_f32(nx, ny, nz, V0, d0, solver="analytic", precision="fp32"):
    n = V0.numel()
    _same_device(nx, ny, nz, V0, d0)
    args = [_ptr(t, torch.float32, n, w) for t, w in ((nx, "nx"), (ny, "ny"), (nz, "nz"), (V0, "V0"), (d0, "d0"))]
    _check(_c["plic_offset_f32"](*args, n, _enum(SOLVERS, solver, "solver"),
                                 _enum(PRECISIONS, precision, "precision"), _stream(V0)), "plic_offset_f32")
    return d0


def plic_offset_f64(nx, ny, nz, V0, d0, solver="analytic"):
    n = V0.numel()
    _same_device(nx, ny, nz, V0, d0)
    args = [_ptr(t, torch.float64, n, w) for t, w in ((nx, "nx"), (ny, "ny"), (nz, "nz"), (V0, "V0"), (d0, "d0"))]
    _check(_c["plic_offset_f64"](*args, n, _enum(SOLVERS, solver, "solver"), _stream(V0)), "plic_offset_f64")
    return d0


def plic_volume_f32(nx, ny, nz, d0, V0, precision="fp32"):
    n = d0.numel()
    _same_device(nx, ny, nz, d0, V0)
    args = [_ptr(t, torch.float32, n, w) for t, w in ((nx, "nx"), (ny, "ny"), (nz, "nz"), (d0, "d0"), (V0, "V0"))]
    _check(_c["plic_volume_f32"](*args, n, _enum(PRECISIONS, precision, "precision"), _stream(d0)),
           "plic_volume_f32")
    return V0


def plic_volume_f64(nx, ny, nz, d0, V0):
    n = d0.numel()
    _same_device(nx, ny, nz, d0, V0)
    args = [_ptr(t, torch.float64, n, w) for t, w in ((nx, "nx"), (ny, "ny"), (nz, "nz"), (d0, "d0"), (V0, "V0"))]
    _check(_c["plic_volume_f64"](*args, n, _stream(d0)), "plic_volume_f64")
    return V0


def plic_offset_backward_f32(nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0,
                             solver="analytic", precision="fp32"):
    n = V0.numel()
    ts = (nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0)
    _same_device(*ts)
    names = ("nx", "ny", "nz", "V0", "grad_d0", "grad_nx", "grad_ny", "grad_nz", "grad_V0")
    args = [_ptr(t, torch.float32, n, w) for t, w in zip(ts, names)]
    _check(_c["plic_offset_backward_f32"](*args, n, _enum(SOLVERS, solver, "solver"),
                                          _enum(PRECISIONS, precision, "precision"), _stream(V0)),
           "plic_offset_backward_f32")


def plic_offset_backward_f64(nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0,
                             solver="analytic"):
    n = V0.numel()
    ts = (nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0)
    _same_device(*ts)
    names = ("nx", "ny", "nz", "V0", "grad_d0", "grad_nx", "grad_ny", "grad_nz", "grad_V0")
    args = [_ptr(t, torch.float64, n, w) for t, w in zip(ts, names)]
    _check(_c["plic_offset_backward_f64"](*args, n, _enum(SOLVERS, solver, "solver"), _stream(V0)),
           "plic_offset_backward_f64")


def _lattice_dims(phi):
    if phi.dim() != 3:
        raise ValueError("phi must be a 3-D tensor of shape (Z, Y, X)")
    Z, Y, X = phi.shape
    return X, Y, Z


def _workspace(phi, workspace, X, Y, Z, neighbour_normals=False):
    """The recommended workspace when none is given; a caller's workspace may
    be smaller (down to the fixed part, which the library checks: interface
    cells beyond its contribution store are recomputed; the neighbour-normal
    backward needs one row at least and gives NaN where a row is missing)."""
    if workspace is None:
        need = plic_curvature_workspace_bytes_ex(X, Y, Z, neighbour_normals)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=phi.device)
    if not (workspace.is_cuda and workspace.is_contiguous() and workspace.dtype == torch.uint8):
        raise ValueError("workspace must be a contiguous uint8 GPU tensor")
    return workspace


def plic_curvature_ex_f32(phi, kappa, solver="analytic", precision="mixed", normal="py",
                          neighbour_normals=False, workspace=None):
    """workspace: optional uint8 device tensor, at least the fixed part and
    best plic_curvature_workspace_bytes bytes (allocated through torch's
    caching allocator when omitted).  normal: "py" or "cm"; neighbour_normals:
    each interface neighbour's plane from its own normal."""
    X, Y, Z = _lattice_dims(phi)
    n = X * Y * Z
    _same_device(phi, kappa)
    ws = _workspace(phi, workspace, X, Y, Z)
    _check(_c["plic_curvature_ex_f32"](_ptr(phi, torch.float32, n, "phi"), X, Y, Z,
                                       _ptr(kappa, torch.float32, n, "kappa"),
                                       _enum(SOLVERS, solver, "solver"),
                                       _enum(PRECISIONS, precision, "precision"),
                                       _enum(NORMALS, normal, "normal"), int(bool(neighbour_normals)),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(phi)),
           "plic_curvature_ex_f32")
    return kappa


def plic_curvature_f32(phi, kappa, solver="analytic", precision="mixed", workspace=None):
    X, Y, Z = _lattice_dims(phi)
    n = X * Y * Z
    _same_device(phi, kappa)
    ws = _workspace(phi, workspace, X, Y, Z)
    _check(_c["plic_curvature_f32"](_ptr(phi, torch.float32, n, "phi"), X, Y, Z,
                                    _ptr(kappa, torch.float32, n, "kappa"),
                                    _enum(SOLVERS, solver, "solver"),
                                    _enum(PRECISIONS, precision, "precision"),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(phi)),
           "plic_curvature_f32")
    return kappa


def plic_curvature_noalloc_f32(phi, kappa, solver="analytic", precision="mixed"):
    """plic_curvature_f32 without a workspace: the library's static 16 MiB
    device array serves as one (lattices up to 21,399 tiles of 64x4x4 cells;
    calls that overlap in time on one GPU race)."""
    X, Y, Z = _lattice_dims(phi)
    n = X * Y * Z
    _same_device(phi, kappa)
    _check(_c["plic_curvature_noalloc_f32"](_ptr(phi, torch.float32, n, "phi"), X, Y, Z,
                                            _ptr(kappa, torch.float32, n, "kappa"),
                                            _enum(SOLVERS, solver, "solver"),
                                            _enum(PRECISIONS, precision, "precision"), _stream(phi)),
           "plic_curvature_noalloc_f32")
    return kappa


def plic_curvature_backward_ex_f32(phi, grad_kappa, grad_phi, solver="analytic", precision="mixed", normal="py",
                                   neighbour_normals=False, workspace=None, check=True, reuse=False, grow=False):
    """With neighbour_normals and check (the default), and outside graph
    capture, the call is followed by plic_curvature_status (one stream
    synchronisation): when the workspace held
    fewer rows than the lattice has interface cells, a workspace that holds
    them all is allocated and the call repeated if the workspace was the
    library's own choice (or grow is set), and a RuntimeError is raised for a
    caller's workspace (its grad_phi holds NaN where rows were missing).
    reuse: plic_curvature_backward_reuse_f32 on the caller's workspace, which
    holds the records of the last forward on this phi (phi unchanged since)."""
    X, Y, Z = _lattice_dims(phi)
    n = X * Y * Z
    _same_device(phi, grad_kappa, grad_phi)
    if reuse and workspace is None:
        raise ValueError("reuse needs the workspace of the forward call")
    own = workspace is None or grow
    ws = _workspace(phi, workspace, X, Y, Z, neighbour_normals)
    for attempt in range(2):
        name = "plic_curvature_backward_reuse_f32" if reuse and attempt == 0 else "plic_curvature_backward_ex_f32"
        _check(_c[name](_ptr(phi, torch.float32, n, "phi"), X, Y, Z,
                        _ptr(grad_kappa, torch.float32, n, "grad_kappa"),
                        _ptr(grad_phi, torch.float32, n, "grad_phi"),
                        _enum(SOLVERS, solver, "solver"),
                        _enum(PRECISIONS, precision, "precision"),
                        _enum(NORMALS, normal, "normal"), int(bool(neighbour_normals)),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(phi)),
               name)
        # the status query synchronises the stream, which a stream under graph
        # capture may not do: there the caller sizes the workspace (and may
        # query plic_curvature_status after a replay)
        if not (neighbour_normals and check) or torch.cuda.is_current_stream_capturing():
            break
        rc, cells, need = plic_curvature_status(ws, X, Y, Z, True, stream=_stream(phi).value)
        if rc == PLIC_OK:
            break
        if rc != PLIC_EWORKSPACE or not own or attempt == 1:
            raise RuntimeError(f"plic_curvature_backward_ex_f32: {plic_status_string(rc)} "
                               f"({cells} interface cells need {need} bytes, workspace has {ws.numel()})")
        ws = torch.empty(need, dtype=torch.uint8, device=phi.device)
    return grad_phi


def plic_curvature_backward_reuse_f32(phi, grad_kappa, grad_phi, solver="analytic", precision="mixed",
                                      normal="py", neighbour_normals=False, workspace=None, check=True):
    """The backward on the workspace of the last forward on phi (its scan is
    not repeated; see plic_curvature_backward_ex_f32 for check)."""
    return plic_curvature_backward_ex_f32(phi, grad_kappa, grad_phi, solver, precision, normal, neighbour_normals,
                                          workspace, check, reuse=True)


def plic_curvature_backward_f32(phi, grad_kappa, grad_phi, solver="analytic", precision="mixed",
                                workspace=None):
    X, Y, Z = _lattice_dims(phi)
    n = X * Y * Z
    _same_device(phi, grad_kappa, grad_phi)
    ws = _workspace(phi, workspace, X, Y, Z)
    _check(_c["plic_curvature_backward_f32"](_ptr(phi, torch.float32, n, "phi"), X, Y, Z,
                                             _ptr(grad_kappa, torch.float32, n, "grad_kappa"),
                                             _ptr(grad_phi, torch.float32, n, "grad_phi"),
                                             _enum(SOLVERS, solver, "solver"),
                                             _enum(PRECISIONS, precision, "precision"),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(phi)),
           "plic_curvature_backward_f32")
    return grad_phi


def _sphere(name, src, dst, dtype):
    n = src.numel()
    if dst.numel() != n:
        raise ValueError(f"{name}: input and output sizes differ")
    _same_device(src, dst)
    _check(_c[name](_ptr(src, dtype, n, "in"), _ptr(dst, dtype, n, "out"), n, _stream(src)), name)
    return dst


def plic_sphere_offset_f32(V0, d0):
    """plane-sphere PLIC (Sec. 3): V0 -> d0 for the unit-volume sphere"""
    return _sphere("plic_sphere_offset_f32", V0, d0, torch.float32)


def plic_sphere_offset_f64(V0, d0):
    return _sphere("plic_sphere_offset_f64", V0, d0, torch.float64)


def plic_sphere_volume_f32(d0, V0):
    """spherical-cap volume below the plane at distance d0 from the centre"""
    return _sphere("plic_sphere_volume_f32", d0, V0, torch.float32)


def plic_sphere_volume_f64(d0, V0):
    return _sphere("plic_sphere_volume_f64", d0, V0, torch.float64)


VALU_OPS = {name: i for i, name in enumerate(
    ("fma_f32", "fma_f64", "sqrt_f32", "rsq_f32", "rcp_f32", "sin_f32", "exp_f32", "log_f32", "rcp_f64",
     "sqrt_f64", "fma_sin_f32"))}


def plic_bench_valu(op, sink, iters, seed=0.7):
    """VALU issue-rate probe (include/plic_bench.h): sink.numel() threads, each
    issuing 32 * iters instructions of `op` (a name from VALU_OPS)."""
    n = sink.numel()
    _check(_c["plic_bench_valu"](_enum(VALU_OPS, op, "op"), n, int(iters), float(seed),
                                 _ptr(sink, torch.float32, n, "sink"), _stream(sink)), "plic_bench_valu")
    return sink


def plic_bench_isolated_f32(nx, ny, nz, err, L=256, solver="sz", blank=False, d0=None):
    """Compute-isolated timing kernel (include/plic_bench.h): err[i] = sum over
    V0 = j/(L-1), j < L, of |V(n_i, d0(n_i, V0)) - V0|; blank=True swaps the
    inversion for d0 = V0 - 1/2.  d0, if given (L * count floats), receives
    every offset, d0[j * count + i]."""
    n = err.numel()
    _same_device(nx, ny, nz, err)
    args = [_ptr(t, torch.float32, n, w) for t, w in zip((nx, ny, nz), ("nx", "ny", "nz"))]
    dp = None
    if d0 is not None:
        _same_device(err, d0)
        dp = _ptr(d0, torch.float32, n * int(L), "d0")
    _check(_c["plic_bench_isolated_f32"](*args, n, int(L), _enum(SOLVERS, solver, "solver"), int(bool(blank)),
                                         _ptr(err, torch.float32, n, "err"), dp, _stream(err)),
           "plic_bench_isolated_f32")
    return err
