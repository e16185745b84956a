"""Oracle pins for the Scardovelli-Zaleski solution as implemented by Kawano
(Sec. 2.4), the unoptimized SZ variant of the paper's comparison.

* It reaches the plane offset, so away from its failure case it equals the
  bisection root of the forward volume (an independent definition), in every
  one of its five cases.
* The paper reports NaN for this variant exactly in the edge case of an axis
  normal with V0 in {0, 1} (Sec. 2.6.1, Tables of Sec. 2.6): on the paper's
  CPU test set (4096 normals: one axis, one face diagonal, 510 in the x-y
  plane, the rest 3D, times 4096 equally spaced V0) the NaN appears there and
  nowhere else.
* Closed forms: an axis normal gives d0 = V0 - 1/2, a face diagonal
  sign(V0 - 1/2) (1/sqrt(2) - sqrt(min(V0, 1 - V0))).
* Complement: d0(1 - V0) = -d0(V0) exactly where 1 - V0 is exact.
"""
import numpy as np
import pytest

import workloads


def random_problems(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v[:, 0], v[:, 1], v[:, 2], rng.random(n)


def test_matches_bisection_in_every_case(orc):
    nx, ny, nz, V0 = random_problems(100_000, seed=0)
    d, kase, arg = orc.offset_kawano(nx, ny, nz, V0)
    ref = orc.offset(nx, ny, nz, V0)
    for c in range(1, 6):
        assert (kase == c).sum() > 5000, c
    err = np.abs(d - ref)
    print("max |d0 - d0_bisection| per case:", [float(err[kase == c].max()) for c in range(1, 6)])
    assert err.max() <= 1e-13
    cubic = (kase == 3) | (kase == 4)
    assert np.all(np.isfinite(arg[cubic])) and np.all(np.isnan(arg[~cubic]))


def test_near_degenerate_normals(orc):
    """Normals within 1e-4 rad of the axes and diagonals, fill levels at the
    case boundaries: the L1 form's cancellation for small m1 costs accuracy
    (about 4e-10 in FP64) but gives no NaN apart from the axis edge case."""
    from tests.gpu_util import near_degenerate_problems
    nx, ny, nz, V0 = near_degenerate_problems(orc, 1 << 14, seed=11)
    d, kase, _ = orc.offset_kawano(nx, ny, nz, V0)
    ref = orc.offset(nx, ny, nz, V0)
    assert not np.isnan(d).any()
    assert np.abs(d - ref).max() <= 1e-8


def test_nan_exactly_at_the_axis_edge_case(orc):
    nx, ny, nz = workloads.paper_mix_normals(4096, seed=5)
    assert (nx[0], ny[0], nz[0]) == (1.0, 0.0, 0.0)
    L = 4096
    V = (np.arange(L, dtype=np.float32) / np.float32(L - 1)).astype(np.float32)
    X, Y, Z = (np.repeat(a, L) for a in (nx, ny, nz))
    W = np.tile(V, nx.size)
    d, kase, _ = orc.offset_kawano(X, Y, Z, W)
    bad = np.flatnonzero(np.isnan(d))
    assert bad.tolist() == [0, L - 1]                  # the axis normal at V0 = 0 and V0 = 1
    assert kase[0] == 4 and kase[L - 1] == 4           # case (5) with alpha = 0 fell through to (4)
    sample = np.arange(L, d.size, 97)
    ref = orc.offset(X[sample], Y[sample], Z[sample], W[sample])
    assert np.abs(d[sample] - ref).max() <= 1e-13


@pytest.mark.parametrize("axis", range(3))
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_axis_normals(orc, axis, sign):
    n = np.zeros(3)
    n[axis] = sign
    V0 = np.r_[0.0, np.linspace(0.01, 0.99, 99), 1.0]
    d, kase, _ = orc.offset_kawano(n[0], n[1], n[2], V0)
    assert np.isnan(d[0]) and np.isnan(d[-1])
    assert np.allclose(d[1:-1], V0[1:-1] - 0.5, rtol=0, atol=1e-15)
    assert np.all(kase[1:-1] == 5)


def test_face_diagonals_and_planar_normals(orc):
    s = 1 / np.sqrt(2)
    V0 = np.r_[0.0, np.linspace(0.001, 0.999, 999), 1.0]
    V = np.minimum(V0, 1 - V0)
    d, _, _ = orc.offset_kawano(s, -s, 0.0, V0)
    want = np.sign(V0 - 0.5) * (s - np.sqrt(V))
    assert np.abs(d - want).max() <= 1e-15
    # every normal in a coordinate plane stays finite, also at V0 in {0, 1}
    rng = np.random.default_rng(3)
    t = rng.uniform(0, 2 * np.pi, 2000)
    nx, ny = np.cos(t), np.sin(t)
    Vr = np.r_[rng.random(2000 - 2), 0.0, 1.0]
    d, kase, _ = orc.offset_kawano(nx, ny, 0.0, Vr)
    assert np.isfinite(d).all()
    assert set(np.unique(kase)) <= {2, 5}


def test_complement(orc):
    rng = np.random.default_rng(4)
    nx, ny, nz, _ = random_problems(20000, seed=4)
    V0 = rng.integers(0, 1 << 24, 20000) / float(1 << 24)
    V0 = V0[V0 != 0.5]
    nx, ny, nz = nx[:V0.size], ny[:V0.size], nz[:V0.size]
    a, _, _ = orc.offset_kawano(nx, ny, nz, V0)
    b, _, _ = orc.offset_kawano(nx, ny, nz, 1.0 - V0)
    ok = np.isfinite(a)
    assert ok.sum() > 19000
    assert np.array_equal(a[ok], -b[ok])
