"""GPU parity of the plane-sphere intersection (Sec. 3) against the FP64
oracle: the closed-form inverse and the cap volume, FP32 and FP64, with edge
values, NaN, in-place calls and unaligned, ragged sizes."""
import numpy as np
import pytest
import torch

from tests.gpu_util import dev, host, max_abs_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2006_12838_amd as P
    return P


def inputs(n, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    v = rng.random(n).astype(dtype)
    edges = np.array([0.0, 1.0, 0.5, -0.25, 1.5, 1e-7, 1 - 1e-7, 2.0 ** -24], dtype=dtype)
    v[:edges.size] = edges
    return v


def test_offset_and_volume_f32(P, orc):
    V0 = inputs((1 << 20) + 5, 0)
    ref = orc.sphere_offset(V0.astype(np.float64))
    tv = dev(V0)
    d = torch.empty_like(tv)
    P.plic_sphere_offset_f32(tv, d)
    err = max_abs_err(host(d), ref)
    print(f"sphere offset f32: max err {err:.3e}")
    assert err <= 1e-5
    dd = np.linspace(-0.7, 0.7, 100003).astype(np.float32)
    V = torch.empty_like(dev(dd))
    P.plic_sphere_volume_f32(dev(dd), V)
    assert max_abs_err(host(V), orc.sphere_volume(dd.astype(np.float64))) <= 1e-6


def test_offset_and_volume_f64(P, orc):
    V0 = inputs((1 << 18) + 3, 1, np.float64)
    tv = dev(V0)
    d = torch.empty_like(tv)
    P.plic_sphere_offset_f64(tv, d)
    assert max_abs_err(host(d), orc.sphere_offset(V0)) <= 1e-12
    dd = np.linspace(-0.7, 0.7, 100001)
    V = torch.empty_like(dev(dd))
    P.plic_sphere_volume_f64(dev(dd), V)
    assert max_abs_err(host(V), orc.sphere_volume(dd)) <= 1e-14


def test_nan_in_place_unaligned(P, orc):
    V0 = inputs(4099, 2)
    V0[7] = np.nan
    t = dev(V0)
    P.plic_sphere_offset_f32(t, t)                                   # in place
    d = host(t)
    assert np.isnan(d[7])
    ref = orc.sphere_offset(V0.astype(np.float64))
    assert max_abs_err(np.delete(d, 7), np.delete(ref, 7)) <= 1e-5
    big = dev(np.concatenate([[0.0], V0]).astype(np.float32))
    out = torch.empty(big.numel() + 1, device="cuda")
    P.plic_sphere_offset_f32(big[1:], out[1:big.numel()])           # 4-byte offsets: scalar path
    assert max_abs_err(host(out[1:big.numel()]), ref) <= 1e-5


def test_round_trip_and_symmetry(P):
    # multiples of 2^-24, so 1 - V0 is exact (near the poles d0'(V0) ~ 1e2
    # would amplify a rounded complement)
    V0 = np.random.default_rng(3).random(1 << 16, dtype=np.float32)
    tv = dev(V0)
    d = torch.empty_like(tv)
    P.plic_sphere_offset_f32(tv, d)
    V = torch.empty_like(tv)
    P.plic_sphere_volume_f32(d, V)
    assert (V - tv).abs().max().item() <= 2e-6
    dc = torch.empty_like(tv)
    P.plic_sphere_offset_f32(1.0 - tv, dc)
    assert (dc + d).abs().max().item() <= 2e-6
