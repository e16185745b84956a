"""Writes plic_closed_forms.txt: the paper's closed-form PLIC offsets at 50 digits.

Each row is a problem (nx, ny, nz, V0), stored as float64 values, and the offset
d0 that the paper's analytic solution gives for exactly those inputs, evaluated
with mpmath at 50 significant digits.  Sources (Lehmann & Gekle, arXiv 2006.12838):

  * symmetry reduction, Sec. 2.1 (sorted |n|, V = 1/2 - |V0 - 1/2|,
    d0 = sign(V0 - 1/2) (S/2 - d));
  * the analytic solution of Sec. 2.3 ("Inverting the inverse PLIC formulation
    analytically"): d1 = cbrt(6 V n1 n2 n3), d2 = n1/2 + sqrt(2 V n2 n3 - n1^2/12),
    d3 = f(x3, y3, a3, b3, c3), d4 = f(x4, y4, a4, b4, c4), d5 = V n3 + (n1 + n2)/2,
    in the order 5, 2, 1, 3, 4 with the a-priori conditions for cases 5, 2 and 1
    (case 2 as n1^2 <= 6 V n2 n3 and 3 n2 (2 V n3 + n1 - n2) <= n1^2, the form
    that follows from n1 <= d2 <= n2 and that the paper's listing uses) and
    d3 <= n3 deciding between 3 and 4.  The trigonometric root f and the
    coefficients x3 ... c4 are as printed; they assume |n| = 1, so the stored
    normal is normalised at 50 digits and the result scaled by |n| (the plane
    n.x = d0 is the plane (n/|n|).x = d0/|n|).  The a-posteriori form of case 5
    is not used: where n3 < n1 + n2 its range shrinks to the single point d = n3,
    which d5 reaches at the wrong volume (for example V = 0 on the space diagonal);
  * the 1D and 2D special cases of the same section.

This script does not import the oracle or the GPU library.
Run:  python tests/golden/make_plic_closed_forms.py
"""
from __future__ import annotations

import os

import mpmath as mp
import numpy as np

mp.mp.dps = 50
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plic_closed_forms.txt")


def f_trig(x, y, a, b, c):
    r2 = x * x + y * y
    return c - 2 * (a + b * mp.cbrt(r2)) / mp.root(r2, 6) * mp.sin(mp.pi / 6 - mp.atan2(y, x) / 3)


def paper_offset(nx, ny, nz, V0):
    n = [mp.mpf(nx), mp.mpf(ny), mp.mpf(nz)]
    V0 = mp.mpf(V0)
    L = mp.sqrt(sum(c * c for c in n))
    a = sorted(abs(c) / L for c in n)
    n1, n2, n3 = a
    S = n1 + n2 + n3
    V = mp.mpf(1) / 2 - abs(V0 - mp.mpf(1) / 2)
    label = None
    d = None
    if n1 + n2 <= 2 * V * n3:                                            # case (5)
        d, label = V * n3 + (n1 + n2) / 2, 5
    elif n1 * n1 <= 6 * V * n2 * n3 and 3 * n2 * (2 * V * n3 + n1 - n2) <= n1 * n1:  # (2)
        d, label = n1 / 2 + mp.sqrt(2 * V * n2 * n3 - n1 * n1 / 12), 2
    elif 6 * V * n2 * n3 < n1 * n1:                                      # case (1)
        d, label = mp.cbrt(6 * V * n1 * n2 * n3), 1
    if d is None:
        x3 = 81 * n1 * n2 * (n1 + n2 - 2 * V * n3)
        y3 = mp.sqrt(max(23328 * (n1 * n2) ** 3 - x3 * x3, 0))
        d3 = f_trig(x3, y3, mp.cbrt(54) * n1 * n2, 1 / mp.cbrt(432), n1 + n2)
        if d3 <= n3:
            d, label = d3, 3
    if d is None:
        t4 = 9 * S * S - 18
        x4 = 324 * n1 * n2 * n3 * (1 - 2 * V)
        y4 = mp.sqrt(max(4 * t4 ** 3 - x4 * x4, 0))
        if x4 == 0 and y4 == 0:
            d4 = S / 2
        else:
            d4 = f_trig(x4, y4, t4 / mp.cbrt(864), 1 / mp.cbrt(3456), S / 2)
        d, label = d4, 4
    sgn = 0 if V0 == mp.mpf(1) / 2 else (1 if V0 > mp.mpf(1) / 2 else -1)
    d0 = sgn * (S / 2 - d) * L
    return d0, label


def problems():
    rng = np.random.default_rng(20061283)
    rows = []
    # 1D: normals along the axes (Sec. 2.3, d = V)
    for ax in range(3):
        for s in (1.0, -1.0):
            for V0 in (0.0, 0.125, 0.3, 0.5, 0.75, 1.0):
                n = [0.0, 0.0, 0.0]
                n[ax] = s
                rows.append((*n, V0, "1D"))
    # 2D: face diagonal and random in-plane normals (Sec. 2.3, cases (2)/(5))
    h = float(1.0 / np.sqrt(2.0))
    for V0 in (0.0, 0.01, 0.1, 0.25, 0.4, 0.5, 0.6, 0.9, 1.0):
        rows.append((h, h, 0.0, V0, "2D"))
    for _ in range(12):
        t = rng.random() * 2 * np.pi
        rows.append((0.0, float(np.cos(t)), float(np.sin(t)), float(rng.random()), "2D"))
    # space diagonal
    s3 = float(1.0 / np.sqrt(3.0))
    for V0 in (0.0, 0.01, 1.0 / 6.0, 0.3, 0.5, 0.8, 1.0):
        rows.append((s3, -s3, s3, V0, "diag"))
    # random 3D normals with fill levels spread over [0,1]
    for _ in range(160):
        g = rng.standard_normal(3)
        g /= np.linalg.norm(g)
        V0 = float(rng.random()) if rng.random() < 0.8 else float(rng.random() * 1e-3)
        rows.append((float(g[0]), float(g[1]), float(g[2]), V0, "3D"))
    return rows


def main():
    lines = ["# PLIC offsets d0 from the paper's closed forms at 50 digits (see the script",
             "# make_plic_closed_forms.py for the passages).  Columns: nx ny nz V0 d0 case kind",
             "# Inputs are float64 values written with repr(); d0 is rounded to 20 digits."]
    for nx, ny, nz, V0, kind in problems():
        d0, label = paper_offset(nx, ny, nz, V0)
        lines.append(f"{nx!r} {ny!r} {nz!r} {V0!r} {mp.nstr(d0, 20)} {label} {kind}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {len(lines) - 3} rows to {OUT}")


if __name__ == "__main__":
    main()
