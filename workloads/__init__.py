"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and lays out geometry (normals, fill
levels of spheres sampled on a lattice).  It holds none of the PLIC method's
arithmetic: no plane-cube volume, no offset, no curvature.  Inputs that need
the method (for example volumes placed exactly on a case boundary) are built by
the caller from a normal and a reduced offset returned here.

Workloads follow the paper's synthetic set-up (Sec. "Performance and Accuracy
Comparison": random unit normals, uniformly spaced or random fill levels, axis
and face-diagonal edge normals, V0 in {0, 1}) and the sphere validation of
Sec. "Validating Curvature Calculation" (fill levels of a sphere of radius R on
a cubic lattice).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "plic_problems",
    "near_degenerate_normals",
    "sphere_lattice",
    "perturbed_sphere_lattice",
    "cylinder_lattice",
    "upstream_grad",
    "paper_mix_normals",
]


def _unit_normals(rng: np.random.Generator, n: int) -> np.ndarray:
    """Normalized Gaussian 3-vectors in float64: uniform on the unit sphere."""
    g = rng.standard_normal((n, 3))
    nrm = np.sqrt(np.einsum("ij,ij->i", g, g))
    # a zero Gaussian vector has probability 0; guard anyway
    nrm[nrm == 0.0] = 1.0
    return g / nrm[:, None]


def plic_problems(n: int, seed: int, edge_frac: float = 0.02, dtype=np.float32):
    """Independent plane-cube problems (nx, ny, nz, V0), structure of arrays.

    * normals: normalized standard-normal 3-vectors, rounded to ``dtype``;
    * V0: uniform in [0, 1) (``rng.random`` in float32 gives multiples of 2^-24,
      so ``1 - V0`` is exact);
    * ``edge_frac`` of the problems are forced edge cases, half of them with
      V0 exactly 0 or 1 and a random normal, a quarter with axis normals +-e_k,
      a quarter with face diagonals (+-e_i +- e_j)/sqrt(2), random signs.
    Returns four contiguous arrays of ``dtype``.
    """
    rng = np.random.default_rng(seed)
    nrm = _unit_normals(rng, n)
    if dtype == np.float64:
        V0 = rng.random(n)
    else:
        V0 = rng.random(n, dtype=np.float32).astype(np.float64)
    n_edge = int(round(edge_frac * n))
    if n_edge > 0:
        idx = rng.choice(n, size=n_edge, replace=False)
        n_v = n_edge // 2
        n_ax = (n_edge - n_v) // 2
        n_fd = n_edge - n_v - n_ax
        iv, iax, ifd = idx[:n_v], idx[n_v:n_v + n_ax], idx[n_v + n_ax:]
        V0[iv] = rng.integers(0, 2, size=n_v).astype(np.float64)
        # axis normals
        k = rng.integers(0, 3, size=n_ax)
        s = rng.choice(np.array([-1.0, 1.0]), size=n_ax)
        ax = np.zeros((n_ax, 3))
        ax[np.arange(n_ax), k] = s
        nrm[iax] = ax
        # face diagonals with the rounded 1/sqrt(2) of the storage type
        h = float(np.asarray(1.0 / math.sqrt(2.0), dtype=dtype))
        pair = rng.integers(0, 3, size=n_fd)  # which component is zero
        s1 = rng.choice(np.array([-1.0, 1.0]), size=n_fd)
        s2 = rng.choice(np.array([-1.0, 1.0]), size=n_fd)
        fd = np.zeros((n_fd, 3))
        a = (pair + 1) % 3
        b = (pair + 2) % 3
        fd[np.arange(n_fd), a] = s1 * h
        fd[np.arange(n_fd), b] = s2 * h
        nrm[ifd] = fd
    nrm = nrm.astype(dtype)
    return (np.ascontiguousarray(nrm[:, 0]), np.ascontiguousarray(nrm[:, 1]),
            np.ascontiguousarray(nrm[:, 2]), V0.astype(dtype))


def paper_mix_normals(n: int, seed: int, dtype=np.float32):
    """The paper's benchmark normal mix: one axis normal (1,0,0), one face
    diagonal (1,1,0)/sqrt(2), 1/8 of the rest random in the x-y plane, the
    remainder random in 3D."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3))
    out[0] = (1.0, 0.0, 0.0)
    if n > 1:
        out[1] = (1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0), 0.0)
    n2d = n // 8 - 2 if n >= 16 else 0
    if n2d > 0:
        phi = rng.random(n2d) * 2.0 * math.pi
        out[2:2 + n2d] = np.stack([np.cos(phi), np.sin(phi), np.zeros(n2d)], 1)
    rest = n - 2 - max(n2d, 0)
    if rest > 0:
        out[n - rest:] = _unit_normals(rng, rest)
    out = out.astype(dtype)
    return tuple(np.ascontiguousarray(out[:, i]) for i in range(3))


_AXES = np.eye(3)
_FACE = np.array([[s1 * (i == a) + s2 * (i == b) for i in range(3)]
                  for a, b in ((0, 1), (0, 2), (1, 2)) for s1 in (1, -1) for s2 in (1, -1)],
                 dtype=np.float64) / math.sqrt(2.0)
_SPACE = np.array([[sx, sy, sz] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)],
                  dtype=np.float64) / math.sqrt(3.0)


def near_degenerate_normals(n: int, seed: int, max_angle: float = 1e-4,
                            include_space_diagonals: bool = True):
    """Normals within ``max_angle`` radians of one of the 6 axis, 12 face-diagonal
    (and optionally 8 space-diagonal) directions, plus, per problem, which
    case boundary its fill level should sit on and a jitter for it.

    Returns ``(normals[n,3] float64, boundary[n] int, complement[n] bool,
    jitter[n] float64)``:
    ``boundary`` indexes the reduced offsets ``0 -> d = 0`` (V = 0),
    ``1 -> d = n1``, ``2 -> d = n2``, ``3 -> d = min(n1 + n2, n3)``,
    ``4 -> d = S/2`` (V = 1/2); ``complement`` says whether 1 - V is used.
    The caller turns (normal, reduced offset) into a volume with its own volume
    routine, adds ``jitter`` (uniform in [-1e-6, 1e-6]) and clamps to [0, 1].
    """
    rng = np.random.default_rng(seed)
    dirs = [np.vstack([_AXES, -_AXES]), _FACE]
    if include_space_diagonals:
        dirs.append(_SPACE)
    base = np.vstack(dirs)
    pick = rng.integers(0, base.shape[0], size=n)
    d = base[pick]
    # random unit axis perpendicular to d
    t = _unit_normals(rng, n)
    t -= np.einsum("ij,ij->i", t, d)[:, None] * d
    tn = np.sqrt(np.einsum("ij,ij->i", t, t))
    tn[tn == 0] = 1.0
    t /= tn[:, None]
    theta = rng.random(n) * max_angle
    nrm = np.cos(theta)[:, None] * d + np.sin(theta)[:, None] * t
    nrm /= np.sqrt(np.einsum("ij,ij->i", nrm, nrm))[:, None]
    boundary = rng.integers(0, 5, size=n)
    complement = rng.integers(0, 2, size=n).astype(bool)
    jitter = rng.uniform(-1e-6, 1e-6, size=n)
    return nrm, boundary, complement, jitter


def near_degenerate_problems(volume, n: int, seed: int, dtype=np.float32):
    """The precision-study workload: normals within 1e-4 rad of an axis, face or
    space diagonal, fill levels within 1e-6 of 0, 1 or a case-boundary volume.
    ``volume(nx, ny, nz, d0) -> V0`` is the caller's forward volume (float64),
    which turns the boundary offsets that near_degenerate_normals names into
    fill levels.  Returns (nx, ny, nz, V0) in ``dtype``."""
    nrm, which, comp, jit = near_degenerate_normals(n, seed)
    nrm = nrm.astype(dtype).astype(np.float64)
    a = np.sort(np.abs(nrm), axis=1)
    S = a.sum(1)
    dred = np.select([which == 0, which == 1, which == 2, which == 3],
                     [np.zeros(n), a[:, 0], a[:, 1], np.minimum(a[:, 0] + a[:, 1], a[:, 2])],
                     0.5 * S)
    V = np.asarray(volume(nrm[:, 0], nrm[:, 1], nrm[:, 2], dred - 0.5 * S), dtype=np.float64)
    V = np.where(comp, 1.0 - V, V) + jit
    V = np.clip(V, 0.0, 1.0).astype(dtype)
    nrm = nrm.astype(dtype)
    return (np.ascontiguousarray(nrm[:, 0]), np.ascontiguousarray(nrm[:, 1]),
            np.ascontiguousarray(nrm[:, 2]), V)


def upstream_grad(shape, seed: int, dtype=np.float32):
    """Upstream gradient ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape).astype(dtype)


# ----------------------------------------------------------------------------
# fill-level lattices (x fastest: array shape (Z, Y, X); cell (i, j, k) has its
# centre at integer coordinates (x=i, y=j, z=k))
# ----------------------------------------------------------------------------

def _subpoints(ss: int) -> np.ndarray:
    o = (np.arange(ss) + 0.5) / ss - 0.5
    gz, gy, gx = np.meshgrid(o, o, o, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1)  # (ss^3, 3) as (x,y,z)


def _fill_from_inside(shape, centre, band_lo, band_hi, inside_fn, ss, chunk=4096):
    """phi = fraction of ss^3 sub-points inside; cells whose centre distance from
    ``centre`` is below ``band_lo`` are full, above ``band_hi`` empty, the rest
    are supersampled with ``inside_fn(points[..., 3]) -> bool``."""
    Z, Y, X = shape
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    dist = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    phi = np.zeros(shape, dtype=np.float32)
    phi[dist < band_lo] = 1.0
    band = np.nonzero((dist >= band_lo) & (dist <= band_hi))
    cells = np.stack([x[band], y[band], z[band]], 1).astype(np.float64)
    sub = _subpoints(ss)
    vals = np.empty(cells.shape[0], dtype=np.float64)
    for s in range(0, cells.shape[0], chunk):
        c = cells[s:s + chunk]
        pts = c[:, None, :] + sub[None, :, :]
        vals[s:s + chunk] = inside_fn(pts).mean(axis=1)
    phi[band] = vals.astype(np.float32)
    return phi


def sphere_lattice(N: int = 256, R: float = 40.0, seed: int = 0, ss: int = 8,
                   jitter: float = 0.15):
    """Fill levels of a sphere of radius ``R`` centred at the lattice centre plus
    a uniform sub-cell jitter in [-jitter, jitter]^3 drawn from ``seed``.
    phi = fraction of the ss^3 sub-points with |x - c| <= R.  Returns
    ``(phi float32 (N,N,N), centre (3,))``."""
    rng = np.random.default_rng(seed)
    c = np.full(3, (N - 1) / 2.0) + rng.uniform(-jitter, jitter, size=3)

    def inside(p):
        return ((p - c) ** 2).sum(-1) <= R * R

    h = math.sqrt(3.0) / 2.0 + 1e-9
    return _fill_from_inside((N, N, N), c, R - h, R + h, inside, ss), c


def cylinder_lattice(N: int = 64, R: float = 16.0, seed: int = 0, ss: int = 8,
                     jitter: float = 0.15):
    """Infinite cylinder along z of radius R (mean curvature 1/(2R))."""
    rng = np.random.default_rng(seed)
    c = np.full(3, (N - 1) / 2.0) + rng.uniform(-jitter, jitter, size=3)
    Z = Y = X = N
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    dist = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2)
    phi = np.zeros((Z, Y, X), dtype=np.float32)
    h = math.sqrt(2.0) / 2.0 + 1e-9
    phi[dist < R - h] = 1.0
    band = np.nonzero((dist >= R - h) & (dist <= R + h))
    cells = np.stack([x[band], y[band]], 1).astype(np.float64)
    o = (np.arange(ss) + 0.5) / ss - 0.5
    gy, gx = np.meshgrid(o, o, indexing="ij")
    sub = np.stack([gx.ravel(), gy.ravel()], 1)
    pts = cells[:, None, :] + sub[None, :, :]
    vals = (((pts - c[:2]) ** 2).sum(-1) <= R * R).mean(axis=1)
    phi[band] = vals.astype(np.float32)
    return phi, c


def _real_sph_harm_basis(lmax: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonics Y_lm(theta, phi), l = 1..lmax,
    m = -l..l, stacked along the last axis (theta polar, phi azimuth)."""
    from scipy.special import lpmv

    ct = np.cos(theta)
    cols = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            P = lpmv(am, l, ct)
            if m == 0:
                cols.append(norm * P)
            elif m > 0:
                cols.append(math.sqrt(2.0) * norm * P * np.cos(am * phi))
            else:
                cols.append(math.sqrt(2.0) * norm * P * np.sin(am * phi))
    return np.stack(cols, -1)


def _assoc_legendre(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x) for 0 <= m <= l <= lmax, with the Condon-Shortley phase (the
    convention of scipy.special.lpmv), by the standard recurrences in m and l."""
    P = {}
    s = np.sqrt(np.maximum(1.0 - x * x, 0.0))
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = (2 * m + 1) * x * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def _real_sph_harm_series(lmax: int, a: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """sum_{l=1..lmax} sum_{m=-l..l} a_lm Y_lm(theta, phi) with the real
    orthonormal harmonics of _real_sph_harm_basis (same coefficient order),
    accumulated term by term from one table of Legendre functions and of
    cos / sin(m phi)."""
    P = _assoc_legendre(lmax, np.cos(theta))
    cos_m = [None] + [np.cos(m * phi) for m in range(1, lmax + 1)]
    sin_m = [None] + [np.sin(m * phi) for m in range(1, lmax + 1)]
    out = np.zeros_like(theta, dtype=np.float64)
    k = 0
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                out += (a[k] * norm) * P[(l, 0)]
            elif m > 0:
                out += (a[k] * math.sqrt(2.0) * norm) * P[(l, am)] * cos_m[am]
            else:
                out += (a[k] * math.sqrt(2.0) * norm) * P[(l, am)] * sin_m[am]
            k += 1
    return out


def perturbed_sphere_lattice(N: int = 192, R: float = 50.0, seed: int = 0, amp: float = 0.05,
                             lmax: int = 6, ss: int = 4, jitter: float = 0.15):
    """Perturbed sphere r(theta, phi) = R (1 + amp * s(theta, phi)) with
    s = sum_{l=1..lmax} sum_m a_lm Y_lm, a_lm ~ N(0, 1), rescaled so that
    max |s| = 1 on a dense angular grid.  phi by ss^3 supersampling.
    Returns ``(phi float32 (N,N,N), centre, coeffs)``."""
    rng = np.random.default_rng(seed)
    c = np.full(3, (N - 1) / 2.0) + rng.uniform(-jitter, jitter, size=3)
    ncoef = (lmax + 1) ** 2 - 1
    a = rng.standard_normal(ncoef)
    tg, pg = np.meshgrid(np.linspace(0, math.pi, 361), np.linspace(0, 2 * math.pi, 721),
                         indexing="ij")
    s_grid = _real_sph_harm_basis(lmax, tg.ravel(), pg.ravel()) @ a
    a = a / np.abs(s_grid).max()

    def radius(p):
        v = p - c
        r = np.sqrt((v ** 2).sum(-1))
        th = np.arccos(np.clip(v[..., 2] / np.maximum(r, 1e-300), -1.0, 1.0))
        ph = np.arctan2(v[..., 1], v[..., 0])
        shp = th.shape
        Y = _real_sph_harm_series(lmax, a, th.ravel(), ph.ravel())
        return r, (R * (1.0 + amp * Y)).reshape(shp)

    def inside(p):
        r, rr = radius(p)
        return r <= rr

    h = math.sqrt(3.0) / 2.0 + 1e-9
    return (_fill_from_inside((N, N, N), c, R * (1 - amp) - h, R * (1 + amp) + h, inside, ss,
                              chunk=2048), c, a)
