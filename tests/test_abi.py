"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/plic.h, and rejects invalid arguments before touching the
HIP runtime (null / misaligned / overlapping pointers, negative sizes, unknown
enums); empty inputs succeed without any HIP call."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(plic_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2006_12838_amd._lib as L
    return L


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("plic_offset_f32", "plic_offset_f64", "plic_volume_f32", "plic_volume_f64",
                     "plic_offset_backward_f32", "plic_offset_backward_f64", "plic_curvature_f32",
                     "plic_curvature_backward_f32", "plic_status_string", "plic_version"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(so, name), name
    assert set(declared_functions()) == set(lib.EXPORTED)


def test_status_and_version(lib):
    assert "gfx950" in lib.plic_version()
    assert lib.plic_status_string(0).startswith("PLIC_OK")
    assert lib.plic_status_string(-1).startswith("PLIC_EINVAL")
    assert lib.plic_status_string(-2).startswith("PLIC_EHIP")
    assert lib.plic_status_string(-3).startswith("PLIC_EWORKSPACE")
    assert lib.plic_status_string(12345) == "unknown PLIC status"
    assert lib.plic_last_hip_error() == 0


A = 0x10000      # fake, 16-byte aligned device addresses: never dereferenced,
B = 0x20000      # every call below is rejected (or is empty) before any HIP call
C = 0x30000
D = 0x40000
E = 0x50000


def test_offset_validation(lib):
    f = lib.raw("plic_offset_f32")
    assert f(A, B, C, D, E, 0, 0, 0, None) == 0                       # empty: OK
    assert f(None, None, None, None, None, 0, 0, 0, None) == 0        # empty, null: OK
    assert f(A, B, C, D, E, -1, 0, 0, None) == -1                     # negative count
    assert f(None, B, C, D, E, 8, 0, 0, None) == -1                   # null input
    assert f(A, B, C, D, None, 8, 0, 0, None) == -1                   # null output
    assert f(A + 2, B, C, D, E, 8, 0, 0, None) == -1                  # misaligned
    assert f(A, B, C, D, E, 8, 5, 0, None) == -1                      # bad solver (4 is Kawano's SZ)
    assert f(A, B, C, D, E, 8, -1, 0, None) == -1
    assert f(A, B, C, D, E, 8, 0, 3, None) == -1                      # bad precision
    assert f(A, B, C, D, A + 4, 8, 0, 0, None) == -1                  # d0 overlaps nx
    g = lib.raw("plic_offset_f64")
    assert g(A, B, C, D, E, 0, 0, None) == 0
    assert g(A + 4, B, C, D, E, 8, 0, None) == -1                     # 8-byte alignment
    assert g(A, B, C, D, E, 8, 7, None) == -1


def test_volume_validation(lib):
    f = lib.raw("plic_volume_f32")
    assert f(A, B, C, D, E, 0, 0, None) == 0
    assert f(A, B, C, D, E, -5, 0, None) == -1
    assert f(A, B, C, D, E, 8, 9, None) == -1
    assert f(A, B, C, D, B, 8, 0, None) == -1                         # V0 overlaps ny
    g = lib.raw("plic_volume_f64")
    assert g(A, B, C, D, E, 0, None) == 0
    assert g(A, B, None, D, E, 8, None) == -1


def test_backward_validation(lib):
    f = lib.raw("plic_offset_backward_f32")
    F, G, H, I = 0x60000, 0x70000, 0x80000, 0x90000
    assert f(A, B, C, D, E, F, G, H, I, 0, 0, 0, None) == 0
    assert f(A, B, C, D, E, F, G, H, I, -1, 0, 0, None) == -1
    assert f(A, B, C, D, E, F, F, H, I, 8, 0, 0, None) == -1         # outputs alias
    assert f(A, B, C, D, E, A, G, H, I, 8, 0, 0, None) == -1         # output aliases input
    assert f(A, B, C, D, E, F, G, H, I, 8, 0, 5, None) == -1
    g = lib.raw("plic_offset_backward_f64")
    assert g(A, B, C, D, E, F, G, H, I, 0, 0, None) == 0
    assert g(A, B, C, D, None, F, G, H, I, 8, 0, None) == -1


def test_curvature_validation(lib):
    per_tile = 784 + 16 * 108                     # fixed part + 16 contribution rows
    assert lib.plic_curvature_workspace_bytes(256, 256, 256) == 256 + 16384 * per_tile
    assert lib.plic_curvature_workspace_bytes(65, 5, 5) == 256 + 8 * per_tile   # 2x2x2 tiles
    assert lib.plic_curvature_workspace_bytes(64 * 4096, 4 * 4096, 4) == 0        # 2^24 tiles: too many
    assert lib.plic_curvature_workspace_bytes(64 * 4096, 4 * 4095, 4) > 0
    assert lib.plic_curvature_workspace_bytes(0, 5, 5) == 0
    assert lib.plic_curvature_workspace_bytes(-1, 5, 5) == 0
    W = 0xA0000
    f = lib.raw("plic_curvature_f32")
    ws = lib.plic_curvature_workspace_bytes(4, 4, 4)
    assert f(A, 0, 5, 5, B, 0, 1, None, 0, None) == 0                 # empty lattice
    assert f(A, -1, 5, 5, B, 0, 1, W, ws, None) == -1
    assert f(None, 4, 4, 4, B, 0, 1, W, ws, None) == -1
    assert f(A, 4, 4, 4, A + 64, 0, 1, W, ws, None) == -1             # kappa overlaps phi
    assert f(A, 4, 4, 4, B, 9, 1, W, ws, None) == -1
    assert f(A, 4, 4, 4, B, 4, 1, W, ws, None) == -1                  # Kawano's SZ: not for the curvature
    assert f(A, 4, 4, 4, B, 0, 7, W, ws, None) == -1
    assert f(A, 4, 4, 4, B, 0, 1, None, ws, None) == -1               # no workspace
    assert f(A, 4, 4, 4, B, 0, 1, W, 256 + 783, None) == -3           # below the fixed part
    assert f(A, 4, 4, 4, None, 0, 1, W, 256 + 783, None) == -1        # an invalid argument comes first
    assert f(A, 4, 4, 4, B, 0, 1, W + 2, 256 + 784, None) == -1       # misaligned
    assert f(A, 4, 4, 4, B, 0, 1, W + 2, ws, None) == -1              # misaligned workspace
    assert f(A, 4, 4, 4, B, 0, 1, B, ws, None) == -1                  # workspace overlaps kappa
    assert f(A, 1 << 40, 1 << 40, 4, B, 0, 1, W, ws, None) == -1      # size overflow
    g = lib.raw("plic_curvature_backward_f32")
    assert g(A, 3, 3, 0, B, C, 0, 1, None, 0, None) == 0
    assert g(A, 3, 3, 3, B, A, 0, 1, W, ws, None) == -1               # grad_phi overlaps phi
    assert g(A, 3, 3, 3, B, B + 4, 0, 1, W, ws, None) == -1           # grad_phi overlaps grad_kappa
    assert g(A, 3, 3, 3, None, C, 0, 1, W, ws, None) == -1
    assert g(A, 3, 3, 3, B, C, 0, 1, C, ws, None) == -1               # workspace overlaps grad_phi
    assert g(A, 3, 3, 3, B, C, 0, 1, W, 256 + 783, None) == -3        # below the fixed part


def test_curvature_options_validation(lib):
    W = 0xA0000
    ws = lib.plic_curvature_workspace_bytes(4, 4, 4)
    f = lib.raw("plic_curvature_ex_f32")
    assert f(A, 0, 5, 5, B, 0, 1, 0, 0, None, 0, None) == 0             # empty lattice
    assert f(A, 4, 4, 4, B, 0, 1, 2, 0, W, ws, None) == -1              # bad normal
    assert f(A, 4, 4, 4, B, 0, 1, -1, 0, W, ws, None) == -1
    assert f(A, 4, 4, 4, B, 0, 1, 1, 2, W, ws, None) == -1              # bad neighbour flag
    assert f(A, 4, 4, 4, A + 64, 0, 1, 1, 1, W, ws, None) == -1         # kappa overlaps phi
    g = lib.raw("plic_curvature_backward_ex_f32")
    assert g(A, 3, 3, 0, B, C, 0, 1, 1, 1, None, 0, None) == 0           # empty lattice
    assert g(A, 3, 3, 3, B, C, 0, 1, 5, 0, W, ws, None) == -1           # bad normal
    assert g(A, 3, 3, 3, B, C, 0, 1, 0, 2, W, ws, None) == -1           # bad neighbour flag
    assert g(A, 3, 3, 3, B, A, 0, 1, 1, 1, W, ws, None) == -1           # grad_phi overlaps phi
    fixed = 256 + 784                                                   # one tile
    assert g(A, 3, 3, 3, B, C, 0, 1, 0, 1, W, fixed + 431, None) == -3  # neighbour normals: no row
    assert lib.plic_curvature_workspace_bytes_ex(4, 4, 4, 1) == fixed + 64 * 432
    assert lib.plic_curvature_workspace_bytes_ex(4, 4, 4, 0) == lib.plic_curvature_workspace_bytes(4, 4, 4)
    assert lib._lib.plic_curvature_workspace_bytes_ex(4, 4, 4, 2) == 0       # bad flag (C entry point)


def test_curvature_noalloc_validation(lib):
    """Refusals of the workspace-free forward happen on the host, before any
    HIP call: bad enums and lattices, overlapping arrays, and a lattice whose
    fixed part exceeds the static 16 MiB array (21,399 tiles of 64x4x4)."""
    f = lib.raw("plic_curvature_noalloc_f32")
    far = [k << 40 for k in (1, 2)]
    assert f(None, 0, 5, 5, None, 0, 1, None) == 0                       # empty lattice
    assert f(far[0], 8, 8, 8, far[1], 4, 1, None) == -1                  # Kawano's solver
    assert f(far[0], 8, 8, 8, far[1], 0, 3, None) == -1                  # bad precision
    assert f(far[0], -1, 8, 8, far[1], 0, 1, None) == -1                 # negative size
    assert f(far[0], 8, 8, 8, far[0] + 64, 0, 1, None) == -1             # kappa overlaps phi
    assert f(far[0], 8, 8, 8, far[1] + 2, 0, 1, None) == -1              # misaligned
    assert f(far[0], 64 * 21399 + 1, 4, 4, far[1], 0, 1, None) == -3    # beyond the static array


def test_curvature_status_validation(lib):
    """The status query rejects what it cannot read before any HIP call."""
    import ctypes
    f = lib._lib.plic_curvature_status
    W = 0xA0000
    cells, need = ctypes.c_int64(-7), ctypes.c_size_t(7)
    fixed = 256 + 784                                                   # one tile
    assert f(W, fixed, 0, 4, 4, 0, ctypes.byref(cells), ctypes.byref(need), None) == -1   # empty lattice
    assert f(W, fixed, 4, 4, 4, 2, None, None, None) == -1             # bad flag
    assert f(None, fixed, 4, 4, 4, 0, None, None, None) == -1          # no workspace
    assert f(W + 2, fixed, 4, 4, 4, 0, None, None, None) == -1         # misaligned
    assert f(W, fixed - 1, 4, 4, 4, 0, None, None, None) == -3         # below the fixed part
    assert f(W, fixed + 431, 4, 4, 4, 1, None, None, None) == -3       # neighbour normals: no row
    assert (cells.value, need.value) == (-7, 7)                         # nothing written on rejection


def test_sphere_validation(lib):
    for name in ("plic_sphere_offset_f32", "plic_sphere_volume_f32", "plic_sphere_offset_f64",
                 "plic_sphere_volume_f64"):
        f = lib.raw(name)
        assert f(A, B, 0, None) == 0                                     # empty
        assert f(None, None, 0, None) == 0
        assert f(A, B, -1, None) == -1
        assert f(None, B, 8, None) == -1
        assert f(A, A + 8, 8, None) == -1                                # partial overlap
    assert lib.raw("plic_sphere_offset_f32")(A + 2, B, 8, None) == -1    # misaligned
    assert lib.raw("plic_sphere_offset_f64")(A + 4, B, 8, None) == -1


def test_valu_probe_validation(lib):
    f = lib.raw("plic_bench_valu")
    assert f(0, 0, 8, 0.5, None, None) == 0                             # empty
    assert f(-1, 8, 8, 0.5, D, None) == -1                              # bad op
    assert f(11, 8, 8, 0.5, D, None) == -1
    assert f(0, -1, 8, 0.5, D, None) == -1
    assert f(0, 8, -1, 0.5, D, None) == -1
    assert f(0, 8, 8, 0.5, None, None) == -1                            # null sink
    assert f(0, 8, 8, 0.5, D + 2, None) == -1                           # misaligned
    assert f(0, (1 << 31) + 1, 8, 0.5, 1 << 40, None) == -1             # grid limit


def test_bench_validation(lib):
    f = lib.raw("plic_bench_isolated_f32")
    assert f(A, B, C, 0, 256, 0, 0, D, None, None) == 0               # empty
    assert f(A, B, C, -1, 256, 0, 0, D, None, None) == -1
    assert f(A, B, C, 8, 1, 0, 0, D, None, None) == -1                # L < 2
    assert f(A, B, C, 8, 256, 5, 0, D, None, None) == -1              # bad solver
    assert f(A, B, C, 8, 256, 0, 2, D, None, None) == -1              # bad blank flag
    assert f(A, B, C, 8, 256, 0, 0, A + 4, None, None) == -1          # err overlaps nx
    assert f(A + 2, B, C, 8, 256, 0, 0, D, None, None) == -1          # misaligned
    far = [k << 40 for k in (1, 2, 3, 4, 5)]                            # disjoint 1 TiB-spaced ranges
    assert f(*far[:3], (1 << 31) + 1, 256, 0, 0, far[3], None, None) == -1   # grid limit
    # the optional offsets output: L * count floats, aligned, overlapping nothing
    assert f(*far[:3], 8, 4, 0, 0, far[3], far[3] + 16, None) == -1    # d0 overlaps err
    assert f(*far[:3], 8, 4, 0, 0, far[3], far[0] + 4, None) == -1     # d0 overlaps nx
    assert f(*far[:3], 8, 4, 0, 0, far[3], far[4] + 2, None) == -1     # d0 misaligned
    assert f(*far[:3], 1 << 31, (1 << 31) - 1, 0, 0, far[3], far[4], None) == -1   # count * L * 4 overflows


def test_python_layer_rejects_cpu_tensors(lib):
    import torch
    x = torch.zeros(8)
    with pytest.raises(ValueError):
        lib.plic_offset_f32(x, x, x, x, x)
