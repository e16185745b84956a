/*
 * FP64 CPU oracle for PLIC inversion and PLIC curvature.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-correct reference the
 * GPU library is checked against.  Only the tests, the package smoke check and
 * the benchmark's CPU-baseline leg load it.  It shares no code with the GPU
 * library (no common headers, helpers or constants).
 *
 * Paper: M. Lehmann, S. Gekle, "Analytic Solution to the Piecewise Linear
 * Interface Construction Problem and its Application in Curvature Calculation
 * for Volume-of-Fluid Simulation Codes" (arXiv 2006.12838).
 *
 * What is computed, and from which passage:
 *  - forward volume: Sec. 2.2 ("Formulating the inverse PLIC problem"), the
 *    five-case volume in reduced symmetry space, with the symmetry reduction of
 *    Sec. 2.1 (sorted |n|, V = min(V0, 1 - V0), d = S/2 - |d0|);
 *  - inverse (the PLIC problem itself, Sec. 2, problem statement V0, n -> d0):
 *    the unique root of the monotone forward volume, found by bisection.  This
 *    is the definition the paper's closed forms reach faster;
 *  - gradient of d0: implicit differentiation of V0(n, d0) = volume below the
 *    plane; dV0/dd0 = A/|n| and dV0/dn = -(A/|n|) * centroid, with A and the
 *    centroid of the plane-cube intersection polygon built explicitly;
 *  - the SZ solution in the form of Kawano's implementation (Sec. 2.4), the
 *    unoptimized variant of the paper's comparison, with its own case order
 *    and its NaN in the axis edge case (Sec. 2.6);
 *  - plane-sphere intersection (Sec. 3): the spherical-cap volume of the
 *    unit-volume sphere and its inverse by bisection;
 *  - curvature: Sec. 4.2 (PLIC point neighbourhood, coordinate transform with
 *    the fixed vector r), App. B.1 (Parker-Youngs normal, or the centre-of-mass
 *    normal as an option), B.2 (paraboloid mean curvature at the origin), B.3
 *    (least-squares normal equations, reduced dimension when fewer than 5
 *    points); as an option, the variant of Sec. 4.2 and Sec. 4.3 in which each
 *    interface neighbour's PLIC plane uses that neighbour's own normal.
 *
 * Readings where the paper is silent or ambiguous (each also used by the GPU
 * library, written independently there):
 *  - V0 outside [0,1] is clamped; NaN inputs and n = 0 give NaN;
 *  - fit solve: symmetric LDL^T in the fixed order A,B,C,H,I; a pivot below
 *    1e-10 * (largest diagonal entry of the leading block) drops that
 *    parameter (kept 0); with k < 5 points the leading k x k block is solved;
 *  - kappa is reported with the sign flipped relative to the paper's formula so
 *    that a fluid drop (normal pointing out of the fluid) has kappa = +1/R;
 *  - |g| < 1e-12 gives kappa = 0; if |n x r| < 1e-6 the vector r is replaced
 *    by (r_y, r_z, r_x);
 *  - kappa = 0 on non-interface cells and on the outer one-cell layer;
 *  - neighbour-normal variant: neighbour q's point is the foot of its own
 *    plane, e_q + d0(phi_q, n_q) n_q - d0(phi_0, n) n, in the centre frame; a
 *    neighbour on the outer lattice layer (its 3^3 neighbourhood leaves the
 *    lattice) or with |g| < 1e-12 keeps the centre normal.
 */
#include "plic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* forward volume                                                             */
/* ------------------------------------------------------------------------- */

static void sort3_asc(double *a, double *b, double *c)
{
    double t;
    if (*a > *b) { t = *a; *a = *b; *b = t; }
    if (*b > *c) { t = *b; *b = *c; *c = t; }
    if (*a > *b) { t = *a; *a = *b; *b = t; }
}

/* Volume below the plane a1*z1 + a2*z2 + a3*z3 = u inside the unit cube [0,1]^3,
 * for 0 <= a1 <= a2 <= a3, a3 > 0 and 0 <= u <= (a1+a2+a3)/2.
 *
 * Five-case volume of Sec. 2.2 with the factor 1/(6 n1 n2 n3) divided through
 * analytically where it would otherwise cancel:
 *   case (1) u <  a1:                      u^3 / (6 a1 a2 a3)
 *   case (5) a1+a2 <= u <= a3:             (u - (a1+a2)/2) / a3
 * The printed case-(5) range min(a1+a2, a3) <= u <= a3 shrinks to the single
 * point u = a3 when a3 < a1 + a2, where the case-(5) formula is not the volume
 * (the general form below is); the range is therefore read as a1+a2 <= u <= a3.
 *   cases (2)-(4):  [u^3 - (u-a1)^3 - (u-a2)+^3 - (u-a3)+^3] / (6 a1 a2 a3)
 *                 = [3u(u-a1) + a1^2 - ((u-a2)+^3 + (u-a3)+^3)/a1] / (6 a2 a3)
 * (the case-(2) rewrite is the one the paper's inverse-PLIC listing uses).
 * Normals in a coordinate plane (a1 = 0) and along an axis (a2 = 0) follow the
 * 2D and 1D special cases of Sec. 2.3. */
double orc_reduced_volume(double a1, double a2, double a3, double u)
{
    if (u <= 0.0) return 0.0;
    if (a2 == 0.0) return u / a3;                              /* 1D */
    if (a1 == 0.0)                                             /* 2D */
        return u <= a2 ? u * u / (2.0 * a2 * a3) : (u - 0.5 * a2) / a3;
    if (u < a1) return u * u * u / (6.0 * a1 * a2 * a3);       /* case (1) */
    if (u >= a1 + a2 && u <= a3)                               /* case (5) */
        return (u - 0.5 * (a1 + a2)) / a3;
    {
        double p2 = u > a2 ? u - a2 : 0.0;
        double p3 = u > a3 ? u - a3 : 0.0;
        return (3.0 * u * (u - a1) + a1 * a1 - (p2 * p2 * p2 + p3 * p3 * p3) / a1)
               / (6.0 * a2 * a3);                              /* cases (2),(3),(4) */
    }
}

double orc_volume1(double nx, double ny, double nz, double d0)
{
    double a1 = fabs(nx), a2 = fabs(ny), a3 = fabs(nz), S, u;
    if (isnan(nx) || isnan(ny) || isnan(nz) || isnan(d0)) return NAN;
    sort3_asc(&a1, &a2, &a3);
    if (!(a3 > 0.0)) return NAN;                               /* n = 0 */
    S = a1 + a2 + a3;
    u = d0 + 0.5 * S;              /* origin moved to the cube corner (Sec. 2.1) */
    if (u <= 0.0) return 0.0;
    if (u >= S) return 1.0;
    if (u <= 0.5 * S) return orc_reduced_volume(a1, a2, a3, u);
    return 1.0 - orc_reduced_volume(a1, a2, a3, S - u);        /* V0 > 1/2 by symmetry */
}

/* ------------------------------------------------------------------------- */
/* inverse PLIC: bisection on the forward volume                              */
/* ------------------------------------------------------------------------- */

/* reduced root u in [0, S/2] with F(u) = V, V in [0, 1/2] */
static double reduced_root(double a1, double a2, double a3, double V)
{
    double lo = 0.0, hi = 0.5 * (a1 + a2 + a3), S = a1 + a2 + a3;
    int it;
    if (V <= 0.0) return 0.0;                  /* F is strictly increasing, F(0) = 0 */
    if (V >= 0.5) return hi;
    for (it = 0; it < 200; ++it) {
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;    /* adjacent doubles */
        if (orc_reduced_volume(a1, a2, a3, mid) < V) lo = mid; else hi = mid;
        if (hi - lo <= ldexp(S, -60)) break;
    }
    return lo + 0.5 * (hi - lo);
}

double orc_offset1(double nx, double ny, double nz, double V0)
{
    double a1 = fabs(nx), a2 = fabs(ny), a3 = fabs(nz), V, u, d;
    if (isnan(nx) || isnan(ny) || isnan(nz) || isnan(V0)) return NAN;
    sort3_asc(&a1, &a2, &a3);
    if (!(a3 > 0.0)) return NAN;
    if (V0 < 0.0) V0 = 0.0;
    if (V0 > 1.0) V0 = 1.0;
    V = V0 <= 0.5 ? V0 : 1.0 - V0;            /* reduced volume (Sec. 2.1), exact */
    u = reduced_root(a1, a2, a3, V);
    d = 0.5 * (a1 + a2 + a3) - u;              /* |d0| */
    if (V0 > 0.5) return d;
    if (V0 < 0.5) return -d;
    return 0.0;
}

/* ------------------------------------------------------------------------- */
/* gradient of d0 from the explicit intersection polygon                      */
/* ------------------------------------------------------------------------- */

static double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1]*b[2] - a[2]*b[1];
    c[1] = a[2]*b[0] - a[0]*b[2];
    c[2] = a[0]*b[1] - a[1]*b[0];
}

/* vertices of { x in [-1/2,1/2]^3 : n . x = d0 } on the 12 cube edges, deduplicated */
static int plane_cube_vertices(const double n[3], double d0, double v[16][3])
{
    int nv = 0, k, j, l, s1, s2, i;
    const double eps = 1e-12;
    for (k = 0; k < 3; ++k) {
        j = (k + 1) % 3; l = (k + 2) % 3;
        for (s1 = 0; s1 < 2; ++s1) for (s2 = 0; s2 < 2; ++s2) {
            double xj = s1 ? 0.5 : -0.5, xl = s2 ? 0.5 : -0.5;
            double cand[2][3];
            int nc = 0, c;
            if (n[k] != 0.0) {
                double t = (d0 - n[j] * xj - n[l] * xl) / n[k];
                if (t >= -0.5 - eps && t <= 0.5 + eps) {
                    if (t < -0.5) t = -0.5;
                    if (t > 0.5) t = 0.5;
                    cand[0][k] = t; cand[0][j] = xj; cand[0][l] = xl; nc = 1;
                }
            } else if (fabs(n[j] * xj + n[l] * xl - d0) <= eps) {
                /* the whole edge lies in the plane: both endpoints are vertices */
                cand[0][k] = -0.5; cand[0][j] = xj; cand[0][l] = xl;
                cand[1][k] = 0.5;  cand[1][j] = xj; cand[1][l] = xl; nc = 2;
            }
            for (c = 0; c < nc; ++c) {
                int dup = 0;
                for (i = 0; i < nv; ++i)
                    if (fabs(v[i][0] - cand[c][0]) < 1e-10 && fabs(v[i][1] - cand[c][1]) < 1e-10 &&
                        fabs(v[i][2] - cand[c][2]) < 1e-10) { dup = 1; break; }
                if (!dup && nv < 16) { v[nv][0] = cand[c][0]; v[nv][1] = cand[c][1]; v[nv][2] = cand[c][2]; ++nv; }
            }
        }
    }
    return nv;
}

int orc_offset_grad1(double nx, double ny, double nz, double V0,
                     double *d0_out, double *dd_dV0, double dd_dn[3], double *area_out)
{
    double n[3] = {nx, ny, nz}, v[16][3], m[3] = {0, 0, 0}, t1[3], t2[3], e[3] = {0, 0, 0};
    double ang[16], area = 0.0, cen[3] = {0, 0, 0}, nn, d0;
    int nv, i, j, order[16], kmin = 0;

    d0 = orc_offset1(nx, ny, nz, V0);
    if (d0_out) *d0_out = d0;
    nn = sqrt(dot3(n, n));
    if (isnan(d0) || !(nn > 0.0)) {
        *dd_dV0 = NAN; dd_dn[0] = dd_dn[1] = dd_dn[2] = NAN;
        if (area_out) *area_out = NAN;
        return 0;
    }
    nv = plane_cube_vertices(n, d0, v);
    for (i = 0; i < nv; ++i) { m[0] += v[i][0]; m[1] += v[i][1]; m[2] += v[i][2]; }
    if (nv > 0) { m[0] /= nv; m[1] /= nv; m[2] /= nv; }
    if (nv < 3) {
        /* degenerate polygon (a corner or an edge): zero area, centroid = limit */
        *dd_dV0 = INFINITY;
        dd_dn[0] = m[0]; dd_dn[1] = m[1]; dd_dn[2] = m[2];
        if (area_out) *area_out = 0.0;
        return nv;
    }
    /* in-plane orthonormal basis t1, t2 */
    if (fabs(n[1]) < fabs(n[kmin])) kmin = 1;
    if (fabs(n[2]) < fabs(n[kmin])) kmin = 2;
    e[kmin] = 1.0;
    cross3(e, n, t1);
    { double s = sqrt(dot3(t1, t1)); t1[0] /= s; t1[1] /= s; t1[2] /= s; }
    { double nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn}; cross3(nh, t1, t2); }
    for (i = 0; i < nv; ++i) {
        double w[3] = {v[i][0] - m[0], v[i][1] - m[1], v[i][2] - m[2]};
        ang[i] = atan2(dot3(w, t2), dot3(w, t1));
        order[i] = i;
    }
    for (i = 1; i < nv; ++i) {                 /* insertion sort by angle */
        int o = order[i];
        j = i - 1;
        while (j >= 0 && ang[order[j]] > ang[o]) { order[j + 1] = order[j]; --j; }
        order[j + 1] = o;
    }
    /* triangle fan from the first vertex: areas and centroids */
    for (i = 1; i + 1 < nv; ++i) {
        const double *p0 = v[order[0]], *p1 = v[order[i]], *p2 = v[order[i + 1]];
        double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]}, c[3], at;
        cross3(a, b, c);
        at = 0.5 * sqrt(dot3(c, c));
        area += at;
        for (j = 0; j < 3; ++j) cen[j] += at * (p0[j] + p1[j] + p2[j]) / 3.0;
    }
    if (area > 0.0) {
        for (j = 0; j < 3; ++j) cen[j] /= area;
        *dd_dV0 = nn / area;
    } else {
        for (j = 0; j < 3; ++j) cen[j] = m[j];
        *dd_dV0 = INFINITY;
    }
    dd_dn[0] = cen[0]; dd_dn[1] = cen[1]; dd_dn[2] = cen[2];
    if (area_out) *area_out = area;
    return nv;
}

void orc_volume(const double *nx, const double *ny, const double *nz, const double *d0,
                double *V0, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) V0[i] = orc_volume1(nx[i], ny[i], nz[i], d0[i]);
}

void orc_offset(const double *nx, const double *ny, const double *nz, const double *V0,
                double *d0, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) d0[i] = orc_offset1(nx[i], ny[i], nz[i], V0[i]);
}

/* ------------------------------------------------------------------------- */
/* Scardovelli-Zaleski solution as implemented by Kawano (Sec. 2.4)           */
/* ------------------------------------------------------------------------- */

/* The SZ solution in the form the paper reproduces from Kawano's Fortran code,
 * kept with that code's characteristic choices, in FP64:
 *  - the normal is L1-normalized, m_k = |n_k| / l with l = |nx| + |ny| + |nz|,
 *    and the plane offset is alpha in [0, 1] from the cube corner, so the
 *    cube-centred offset is l (1/2 - alpha) with the sign of V0 - 1/2;
 *  - the reduced volume is the printed w = 1/2 - |V0 - 1/2|;
 *  - m1 = min m_k, m3 = max m_k and the middle one is taken as 1 - m1 - m3
 *    (not below 0);
 *  - the thresholds are the volumes at alpha = m1 (V1, with a tiny 1e-25 added
 *    to its denominator), the case-(2) end V1 + (m2 - m1) / (2 m3), and V3, the
 *    volume at alpha = m3 when m3 < m1 + m2 (where case (4) exists), else at
 *    alpha = m1 + m2 (the start of case (5));
 *  - the cases are tested in the order (1), (2), then (5), (3), (4).  Case (5)
 *    records its alpha, and alpha == 0 means "not settled yet": a case-(5)
 *    root of exactly 0 (an axis normal at V0 in {0, 1}) falls through to the
 *    cubic of case (4), whose trigonometric root then takes the square root of
 *    a negative number.  This is the NaN the paper reports for this variant
 *    (Sec. 2.6.1 and 2.6.2, the edge case n = (1, 0, 0), V0 in {0, 1});
 *  - cases (3) and (4) solve the monic cubic alpha^3 + a2 alpha^2 + a1 alpha
 *    + a0 = 0 of the case's volume (inclusion-exclusion of the cut corners:
 *    (3) removes the corners at m1 and m2, (4) all three, where m1 + m2 + m3
 *    = 1 simplifies the coefficients), by the trigonometric (Viete) form of
 *    its third real root: with p = a1 - a2^2 / 3 and sp = sqrt(-p / 3),
 *    alpha = 2 sp cos(4 pi / 3 + acos(q0 / sp^3) / 3) - a2 / 3,
 *    q0 = (a1 a2 - 3 a0) / 6 - a2^3 / 27.
 * V0 is clamped to [0, 1] first (as for every solver here); NaN inputs and
 * n = 0 give NaN.  *kase receives the case taken (1..5, 0 for NaN inputs) and
 * *acos_arg the argument q0 / sp^3 of the cubic cases (NaN otherwise). */
double orc_offset_kawano1(double nx, double ny, double nz, double V0, int *kase, double *acos_arg)
{
    double l, m[3], m1, m2, m3, m12, w, V1, w6, V3, alpha = 0.0;
    int k = 0;
    *kase = 0;
    *acos_arg = NAN;
    if (isnan(nx) || isnan(ny) || isnan(nz) || isnan(V0)) return NAN;
    if (V0 < 0.0) V0 = 0.0;
    if (V0 > 1.0) V0 = 1.0;
    l = fabs(nx) + fabs(ny) + fabs(nz);
    if (!(l > 0.0)) return NAN;
    m[0] = fabs(nx) / l; m[1] = fabs(ny) / l; m[2] = fabs(nz) / l;
    w = 0.5 - fabs(V0 - 0.5);
    m1 = fmin(fmin(m[0], m[1]), m[2]);
    m3 = fmax(fmax(m[0], m[1]), m[2]);
    m2 = fmax(1.0 - (m1 + m3), 0.0);
    m12 = m1 + m2;
    V1 = m1 * m1 / (6.0 * m2 * m3 + 1e-25);
    w6 = 6.0 * m1 * m2 * m3 * w;
    if (w < V1) {
        k = 1;
        alpha = cbrt(w6);
    } else if (w < V1 + 0.5 * (m2 - m1) / m3) {
        k = 2;
        alpha = 0.5 * (m1 + sqrt(m1 * m1 + 8.0 * m2 * m3 * (w - V1)));
    } else {
        if (m3 < m12) {
            /* volume at alpha = m3: [m3^3 - (m3 - m1)^3 - (m3 - m2)^3] / (6 m1 m2 m3), expanded */
            V3 = (m3 * m3 * (3.0 * m12 - m3) + m1 * m1 * (m1 - 3.0 * m3) + m2 * m2 * (m2 - 3.0 * m3))
                 / (6.0 * m1 * m2 * m3);
        } else {
            V3 = 0.5 * m12 / m3;
            if (V3 <= w) { k = 5; alpha = m3 * w + 0.5 * m12; }
        }
        if (alpha == 0.0) {
            double a2, a1, a0, q0, sp, arg;
            if (w < V3) {
                k = 3;
                a2 = -3.0 * m12;
                a1 = 3.0 * (m1 * m1 + m2 * m2);
                a0 = w6 - m1 * m1 * m1 - m2 * m2 * m2;
            } else {
                k = 4;
                a2 = -1.5;
                a1 = 1.5 * (m1 * m1 + m2 * m2 + m3 * m3);
                a0 = 0.5 * (w6 - m1 * m1 * m1 - m2 * m2 * m2 - m3 * m3 * m3);
            }
            q0 = (a1 * a2 - 3.0 * a0) / 6.0 - a2 * a2 * a2 / 27.0;
            sp = sqrt(a2 * a2 / 9.0 - a1 / 3.0);
            arg = q0 / (sp * sp * sp);
            *acos_arg = arg;
            alpha = 2.0 * sp * cos(4.0 * 3.14159265358979323846 / 3.0 + acos(arg) / 3.0) - a2 / 3.0;
        }
    }
    *kase = k;
    return l * copysign(0.5 - alpha, V0 - 0.5);
}

void orc_offset_kawano(const double *nx, const double *ny, const double *nz, const double *V0,
                       double *d0, int32_t *kase, double *acos_arg, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) {
        int k;
        d0[i] = orc_offset_kawano1(nx[i], ny[i], nz[i], V0[i], &k, &acos_arg[i]);
        kase[i] = k;
    }
}

void orc_offset_grad(const double *nx, const double *ny, const double *nz, const double *V0,
                     double *d0, double *dd_dV0, double *dd_dnx, double *dd_dny,
                     double *dd_dnz, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) {
        double g[3];
        orc_offset_grad1(nx[i], ny[i], nz[i], V0[i], &d0[i], &dd_dV0[i], g, NULL);
        dd_dnx[i] = g[0]; dd_dny[i] = g[1]; dd_dnz[i] = g[2];
    }
}

/* ------------------------------------------------------------------------- */
/* plane-sphere intersection (Sec. 3)                                         */
/* ------------------------------------------------------------------------- */

/* radius of the unit-volume sphere */
static double sphere_radius(void) { return cbrt(3.0 / (4.0 * 3.14159265358979323846)); }

/* volume of the unit-volume sphere below the plane at signed distance d0 from
 * its centre: the spherical cap (pi/3) (r + d0)^2 (2r - d0), 0 / 1 outside [-r, r] */
double orc_sphere_volume1(double d0)
{
    double r = sphere_radius(), h;
    if (isnan(d0)) return NAN;
    if (d0 <= -r) return 0.0;
    if (d0 >= r) return 1.0;
    h = r + d0;
    return 3.14159265358979323846 / 3.0 * h * h * (2.0 * r - d0);
}

/* the inverse: d0 in [-r, r] with volume V0 (clamped to [0, 1]), by bisection
 * of the monotone cap volume down to adjacent doubles */
double orc_sphere_offset1(double V0)
{
    double r = sphere_radius(), lo = -r, hi = r;
    int it;
    if (isnan(V0)) return NAN;
    if (V0 <= 0.0) return -r;
    if (V0 >= 1.0) return r;
    for (it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_sphere_volume1(mid) < V0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

void orc_sphere_volume(const double *d0, double *V0, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) V0[i] = orc_sphere_volume1(d0[i]);
}

void orc_sphere_offset(const double *V0, double *d0, int64_t count)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < count; ++i) d0[i] = orc_sphere_offset1(V0[i]);
}

/* ------------------------------------------------------------------------- */
/* curvature                                                                  */
/* ------------------------------------------------------------------------- */

/* the fixed auxiliary vector r of Sec. 4.2 */
static const double R_AUX[3] = {0.56270900, 0.32704452, 0.75921047};

/* mean curvature of z = A x^2 + B y^2 + C x y + H x + I y at x = y = 0
 * (App. B.2): (A (I^2+1) + B (H^2+1) - C H I) / (H^2 + I^2 + 1)^(3/2) */
double orc_paraboloid_kappa(const double coef[5])
{
    double A = coef[0], B = coef[1], C = coef[2], H = coef[3], I = coef[4];
    double w = H * H + I * I + 1.0;
    return (A * (I * I + 1.0) + B * (H * H + 1.0) - C * H * I) / (w * sqrt(w));
}

/* least-squares fit of App. B.3: M = sum Q Q^T, b = sum z Q, Q = (x^2, y^2, xy, x, y),
 * solved by LDL^T (M is symmetric) over the leading min(5, npts) parameters */
int orc_fit_paraboloid(const double *px, const double *py, const double *pz, int npts,
                       double coef[5], double *cond)
{
    double M[5][5], b[5], L[5][5], D[5], y[5], x[5], maxdiag = 0.0, tol, dmax = 0.0, dmin = 0.0;
    int act[5], N, i, j, k, nact = 0;
    memset(M, 0, sizeof M); memset(b, 0, sizeof b); memset(L, 0, sizeof L);
    for (i = 0; i < npts; ++i) {
        double Q[5] = {px[i] * px[i], py[i] * py[i], px[i] * py[i], px[i], py[i]};
        for (j = 0; j < 5; ++j) {
            b[j] += pz[i] * Q[j];
            for (k = 0; k < 5; ++k) M[j][k] += Q[j] * Q[k];
        }
    }
    for (j = 0; j < 5; ++j) coef[j] = 0.0;
    if (cond) *cond = 0.0;
    N = npts < 5 ? npts : 5;
    if (N <= 0) return 0;
    for (j = 0; j < N; ++j) if (M[j][j] > maxdiag) maxdiag = M[j][j];
    tol = 1e-10 * maxdiag;
    for (j = 0; j < N; ++j) {
        double dj = M[j][j];
        for (k = 0; k < j; ++k) if (act[k]) dj -= L[j][k] * L[j][k] * D[k];
        act[j] = dj > tol && maxdiag > 0.0;
        if (!act[j]) continue;
        D[j] = dj;
        if (nact == 0 || dj > dmax) dmax = dj;
        if (nact == 0 || dj < dmin) dmin = dj;
        ++nact;
        for (i = j + 1; i < N; ++i) {
            double s = M[i][j];
            for (k = 0; k < j; ++k) if (act[k]) s -= L[i][k] * L[j][k] * D[k];
            L[i][j] = s / dj;
        }
    }
    for (j = 0; j < N; ++j) {                  /* L y = b */
        if (!act[j]) continue;
        y[j] = b[j];
        for (k = 0; k < j; ++k) if (act[k]) y[j] -= L[j][k] * y[k];
    }
    for (j = N - 1; j >= 0; --j) {             /* D L^T x = y */
        if (!act[j]) continue;
        x[j] = y[j] / D[j];
        for (i = j + 1; i < N; ++i) if (act[i]) x[j] -= L[i][j] * x[i];
    }
    for (j = 0; j < N; ++j) coef[j] = act[j] ? x[j] : 0.0;
    if (cond) *cond = nact > 0 ? dmax / dmin : 0.0;
    {
        int bits = 0;
        for (j = 0; j < N; ++j) if (act[j]) bits |= 1 << j;
        return bits;
    }
}

/* fill-level gradient of a 3^3 neighbourhood (App. B.1): Parker-Youngs
 * weights 4 / 2 / 1 for |e| = 1 / sqrt2 / sqrt3 (kind 0), or the centre-of-mass
 * method with equal weights (kind 1); returns |g|, n = -g / |g| */
static double normal_of(const double p27[27], int kind, double n[3])
{
    double g[3] = {0, 0, 0}, gn;
    int dx, dy, dz;
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), e2 = dx * dx + dy * dy + dz * dz;
        double w;
        if (e2 == 0) continue;
        w = kind == 1 ? 1.0 : (e2 == 1 ? 4.0 : (e2 == 2 ? 2.0 : 1.0));
        g[0] += w * dx * p27[q];
        g[1] += w * dy * p27[q];
        g[2] += w * dz * p27[q];
    }
    gn = sqrt(dot3(g, g));
    if (gn > 0.0) { n[0] = -g[0] / gn; n[1] = -g[1] / gn; n[2] = -g[2] / gn; }
    else { n[0] = n[1] = n[2] = 0.0; }
    return gn;
}

/* One interface cell (Sec. 4.2 and App. B).  nbrn == NULL: every neighbour's
 * PLIC plane uses the centre normal n, the point of neighbour i is
 * (e_i.b_x, e_i.b_y, e_i.n + d0(phi_i, n) - d0(phi_0, n)).  Otherwise nbrn[q]
 * is neighbour q's own normal n_q and its point is the foot of its own plane,
 * P_q = e_q + d0(phi_q, n_q) n_q - d0(phi_0, n) n, in the centre frame
 * (x, y, z) = (P_q.b_x, P_q.b_y, P_q.n); this reduces to the first form when
 * n_q = n. */
static double cell_core(const double phi[27], const unsigned char mask[27], const double raux[3],
                        int kind, const double (*nbrn)[3], double info[3], double normal[3],
                        double coef[5])
{
    double gn, n[3], u[3], r[3], un, by[3], bx[3], D0;
    double px[26], py[26], pz[26], cond = 0.0;
    int dx, dy, dz, npts = 0, bits;
    double c5[5];
    if (!coef) coef = c5;
    for (int j = 0; j < 5; ++j) coef[j] = 0.0;
    if (info) { info[0] = 0; info[1] = 0; info[2] = 0; }
    gn = normal_of(phi, kind, n);
    if (!(gn >= 1e-12)) { if (normal) normal[0] = normal[1] = normal[2] = 0; return 0.0; }
    if (normal) { normal[0] = n[0]; normal[1] = n[1]; normal[2] = n[2]; }
    /* local frame (Sec. 4.2): b_z = n, b_y = n x r / |n x r|, b_x = b_y x b_z */
    r[0] = raux[0]; r[1] = raux[1]; r[2] = raux[2];
    cross3(n, r, u);
    un = sqrt(dot3(u, u));
    if (un < 1e-6) {
        r[0] = raux[1]; r[1] = raux[2]; r[2] = raux[0];
        cross3(n, r, u);
        un = sqrt(dot3(u, u));
    }
    by[0] = u[0] / un; by[1] = u[1] / un; by[2] = u[2] / un;
    cross3(by, n, bx);
    /* PLIC points of the interface neighbours */
    D0 = orc_offset1(n[0], n[1], n[2], phi[13]);
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        double e[3] = {(double)dx, (double)dy, (double)dz}, P[3];
        if (q == 13 || !mask[q]) continue;
        if (nbrn) {
            const double *nq = nbrn[q];
            double Di = orc_offset1(nq[0], nq[1], nq[2], phi[q]);
            for (int k = 0; k < 3; ++k) P[k] = e[k] + Di * nq[k] - D0 * n[k];
        } else {
            double Di = orc_offset1(n[0], n[1], n[2], phi[q]);
            for (int k = 0; k < 3; ++k) P[k] = e[k] + (Di - D0) * n[k];
        }
        px[npts] = dot3(P, bx);
        py[npts] = dot3(P, by);
        pz[npts] = dot3(P, n);
        ++npts;
    }
    bits = orc_fit_paraboloid(px, py, pz, npts, coef, &cond);
    if (info) { info[0] = npts; info[1] = bits; info[2] = cond; }
    /* sign: positive for a fluid drop (the normal points out of the fluid) */
    return -orc_paraboloid_kappa(coef);
}

double orc_curv_cell_full(const double phi[27], const unsigned char mask[27], double info[3],
                          double normal[3], double coef[5])
{
    return cell_core(phi, mask, R_AUX, 0, NULL, info, normal, coef);
}

double orc_curv_cell_r(const double phi[27], const unsigned char mask[27], const double raux[3],
                       double info[3], double normal[3], double coef[5])
{
    return cell_core(phi, mask, raux, 0, NULL, info, normal, coef);
}

double orc_curv_cell(const double phi[27], const unsigned char mask[27], double info[3])
{
    return cell_core(phi, mask, R_AUX, 0, NULL, info, NULL, NULL);
}

double orc_curv_cell_k(const double phi[27], const unsigned char mask[27], int kind, double info[3],
                       double normal[3])
{
    return cell_core(phi, mask, R_AUX, kind, NULL, info, normal, NULL);
}

/* neighbour-normal variant on a 5^3 neighbourhood p125[(dz+2)*25 + (dy+2)*5 + (dx+2)];
 * a neighbour keeps the centre normal when its own 3^3 neighbourhood is not
 * inside the lattice (inside27[q] == 0; NULL: all inside) or its gradient
 * vanishes (|g| < 1e-12) */
/* the variant with the interface mask of the inner 3^3 given (mask27), as the
 * finite-difference gradient holds it fixed; NULL: from the values */
static double cell_nbr_core(const double p125[125], const unsigned char mask27[27],
                            const unsigned char inside27[27], int kind, double info[3])
{
    double p27[27], nbrn[27][3], nc[3];
    unsigned char mask[27];
    int dx, dy, dz;
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        double v = p125[(dz + 2) * 25 + (dy + 2) * 5 + (dx + 2)];
        p27[q] = v;
        mask[q] = mask27 ? mask27[q] : (unsigned char)(v > 0.0 && v < 1.0);
    }
    if (!(normal_of(p27, kind, nc) >= 1e-12)) {
        if (info) { info[0] = 0; info[1] = 0; info[2] = 0; }
        return 0.0;
    }
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), a, b, c;
        double s27[27];
        for (c = -1; c <= 1; ++c) for (b = -1; b <= 1; ++b) for (a = -1; a <= 1; ++a)
            s27[(c + 1) * 9 + (b + 1) * 3 + (a + 1)] = p125[(dz + c + 2) * 25 + (dy + b + 2) * 5 + (dx + a + 2)];
        if ((inside27 && !inside27[q]) || !(normal_of(s27, kind, nbrn[q]) >= 1e-12)) {
            nbrn[q][0] = nc[0]; nbrn[q][1] = nc[1]; nbrn[q][2] = nc[2];
        }
    }
    return cell_core(p27, mask, R_AUX, kind, (const double (*)[3])nbrn, info, NULL, NULL);
}

double orc_curv_cell_nbr(const double p125[125], const unsigned char inside27[27], int kind, double info[3])
{
    return cell_nbr_core(p125, NULL, inside27, kind, info);
}

static int is_interface(float p) { return p > 0.0f && p < 1.0f; }

static void gather27(const float *phi, int64_t X, int64_t Y, int64_t x, int64_t y, int64_t z,
                     double v[27], unsigned char m[27])
{
    int dx, dy, dz;
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        float p = phi[((z + dz) * Y + (y + dy)) * X + (x + dx)];
        v[q] = (double)p;
        m[q] = (unsigned char)is_interface(p);
    }
}

/* 5^3 neighbourhood (outside the lattice: 0, never used), and per neighbour
 * whether its own 3^3 neighbourhood lies inside the lattice */
static void gather125(const float *phi, int64_t X, int64_t Y, int64_t Z, int64_t x, int64_t y, int64_t z,
                      double v[125], unsigned char inside27[27])
{
    int dx, dy, dz;
    for (dz = -2; dz <= 2; ++dz) for (dy = -2; dy <= 2; ++dy) for (dx = -2; dx <= 2; ++dx) {
        int64_t gx = x + dx, gy = y + dy, gz = z + dz;
        int k = (dz + 2) * 25 + (dy + 2) * 5 + (dx + 2);
        v[k] = (gx >= 0 && gy >= 0 && gz >= 0 && gx < X && gy < Y && gz < Z) ?
               (double)phi[(gz * Y + gy) * X + gx] : 0.0;
    }
    for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
        int64_t gx = x + dx, gy = y + dy, gz = z + dz;
        inside27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] =
            (unsigned char)(gx >= 1 && gy >= 1 && gz >= 1 && gx <= X - 2 && gy <= Y - 2 && gz <= Z - 2);
    }
}

/* one interior interface cell with the options; info may be NULL */
static double lattice_cell(const float *phi, int64_t X, int64_t Y, int64_t Z, int64_t x, int64_t y,
                           int64_t z, int kind, int nbr, double info[3])
{
    if (nbr) {
        double v[125];
        unsigned char inside[27];
        gather125(phi, X, Y, Z, x, y, z, v, inside);
        return orc_curv_cell_nbr(v, inside, kind, info);
    } else {
        double v[27];
        unsigned char m[27];
        gather27(phi, X, Y, x, y, z, v, m);
        return cell_core(v, m, R_AUX, kind, NULL, info, NULL, NULL);
    }
}

void orc_curvature_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind, int nbr,
                      double *kappa, uint8_t *flags)
{
    int64_t c, total = X * Y * Z;
#pragma omp parallel for schedule(dynamic, 4096)
    for (c = 0; c < total; ++c) {
        int64_t x = c % X, y = (c / X) % Y, z = c / (X * Y);
        double info[3];
        kappa[c] = 0.0;
        if (flags) flags[c] = 0;
        if (x < 1 || y < 1 || z < 1 || x > X - 2 || y > Y - 2 || z > Z - 2) continue;
        if (!is_interface(phi[c])) continue;
        kappa[c] = lattice_cell(phi, X, Y, Z, x, y, z, kind, nbr, info);
        if (flags) {
            flags[c] = 1;
            if (info[2] > 1e8) flags[c] |= 2;
            if (info[0] < 5) flags[c] |= 4;
        }
    }
}

void orc_curvature(const float *phi, int64_t X, int64_t Y, int64_t Z, double *kappa,
                   uint8_t *flags)
{
    orc_curvature_ex(phi, X, Y, Z, 0, 0, kappa, flags);
}

void orc_curvature_cells_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind, int nbr,
                            const int64_t *cells, int64_t ncells, double *kappa, double *info3)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
    for (i = 0; i < ncells; ++i) {
        int64_t c = cells[i], x = c % X, y = (c / X) % Y, z = c / (X * Y);
        double info[3] = {0, 0, 0};
        kappa[i] = 0.0;
        if (x >= 1 && y >= 1 && z >= 1 && x <= X - 2 && y <= Y - 2 && z <= Z - 2 &&
            is_interface(phi[c]))
            kappa[i] = lattice_cell(phi, X, Y, Z, x, y, z, kind, nbr, info);
        if (info3) { info3[3 * i] = info[0]; info3[3 * i + 1] = info[1]; info3[3 * i + 2] = info[2]; }
    }
}

void orc_curvature_cells(const float *phi, int64_t X, int64_t Y, int64_t Z,
                         const int64_t *cells, int64_t ncells, double *kappa, double *info3)
{
    orc_curvature_cells_ex(phi, X, Y, Z, 0, 0, cells, ncells, kappa, info3);
}

int orc_curv_cell_fd_grad_k(const double phi[27], const unsigned char mask[27], int kind, double h,
                            double grad[27])
{
    double base[3], ip[3], im[3], p[27];
    int q, bad = 0;
    orc_curv_cell_k(phi, mask, kind, base, NULL);
    for (q = 0; q < 27; ++q) {
        double kp, km;
        memcpy(p, phi, sizeof p);
        if (mask[q] || q == 13) {
            if (!(phi[q] - h > 0.0 && phi[q] + h < 1.0)) bad = 1;
        }
        p[q] = phi[q] + h; kp = orc_curv_cell_k(p, mask, kind, ip, NULL);
        p[q] = phi[q] - h; km = orc_curv_cell_k(p, mask, kind, im, NULL);
        if (ip[0] != base[0] || im[0] != base[0] || ip[1] != base[1] || im[1] != base[1]) bad = 1;
        grad[q] = (kp - km) / (2.0 * h);
    }
    return bad;
}

int orc_curv_cell_fd_grad(const double phi[27], const unsigned char mask[27], double h,
                          double grad[27])
{
    return orc_curv_cell_fd_grad_k(phi, mask, 0, h, grad);
}

int64_t orc_curvature_grad_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind,
                              const float *grad_kappa, double h, double *grad_phi,
                              uint8_t *bad_cells)
{
    int64_t total = X * Y * Z, c, nif = 0, k, nbad = 0;
    int64_t *list;
    double *part;
    int *bad;
    for (c = 0; c < total; ++c) { grad_phi[c] = 0.0; if (bad_cells) bad_cells[c] = 0; }
    for (c = 0; c < total; ++c) {
        int64_t x = c % X, y = (c / X) % Y, z = c / (X * Y);
        if (x >= 1 && y >= 1 && z >= 1 && x <= X - 2 && y <= Y - 2 && z <= Z - 2 &&
            is_interface(phi[c])) ++nif;
    }
    list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nif > 0 ? nif : 1));
    part = (double *)malloc(sizeof(double) * 27 * (size_t)(nif > 0 ? nif : 1));
    bad = (int *)malloc(sizeof(int) * (size_t)(nif > 0 ? nif : 1));
    k = 0;
    for (c = 0; c < total; ++c) {
        int64_t x = c % X, y = (c / X) % Y, z = c / (X * Y);
        if (x >= 1 && y >= 1 && z >= 1 && x <= X - 2 && y <= Y - 2 && z <= Z - 2 &&
            is_interface(phi[c])) list[k++] = c;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < nif; ++k) {
        int64_t cc = list[k], x = cc % X, y = (cc / X) % Y, z = cc / (X * Y);
        double v[27];
        unsigned char m[27];
        gather27(phi, X, Y, x, y, z, v, m);
        bad[k] = orc_curv_cell_fd_grad_k(v, m, kind, h, part + 27 * k);
    }
    for (k = 0; k < nif; ++k) {                /* fixed-order scatter */
        int64_t cc = list[k], x = cc % X, y = (cc / X) % Y, z = cc / (X * Y);
        double gk = (double)grad_kappa[cc];
        int dx, dy, dz;
        for (dz = -1; dz <= 1; ++dz) for (dy = -1; dy <= 1; ++dy) for (dx = -1; dx <= 1; ++dx) {
            int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
            grad_phi[((z + dz) * Y + (y + dy)) * X + (x + dx)] += gk * part[27 * k + q];
        }
        if (bad[k]) { ++nbad; if (bad_cells) bad_cells[cc] = 1; }
    }
    free(list); free(part); free(bad);
    return nbad;
}

/* neighbour-normal variant: central differences over the whole 5^3
 * neighbourhood (the neighbours' own normals reach two cells out) with the
 * interface mask held fixed; bad when a perturbed interface entry of the inner
 * 3^3 (or the centre) would cross 0 or 1, or the active fit parameters change */
int orc_curv_cell_nbr_fd_grad(const double p125[125], const unsigned char inside27[27], int kind, double h,
                              double grad[125])
{
    double base[3], ip[3], im[3], p[125];
    unsigned char mask[27];
    int k, bad = 0;
    for (k = 0; k < 27; ++k) {
        double v = p125[(k / 9 + 1) * 25 + ((k / 3) % 3 + 1) * 5 + (k % 3 + 1)];
        mask[k] = (unsigned char)(v > 0.0 && v < 1.0);
    }
    cell_nbr_core(p125, mask, inside27, kind, base);
    for (k = 0; k < 125; ++k) {
        int dx = k % 5 - 2, dy = (k / 5) % 5 - 2, dz = k / 25 - 2;
        double kp, km;
        memcpy(p, p125, sizeof p);
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
            double v = p125[k];
            int centre = dx == 0 && dy == 0 && dz == 0;
            if ((centre || (v > 0.0 && v < 1.0)) && !(v - h > 0.0 && v + h < 1.0)) bad = 1;
        }
        p[k] = p125[k] + h; kp = cell_nbr_core(p, mask, inside27, kind, ip);
        p[k] = p125[k] - h; km = cell_nbr_core(p, mask, inside27, kind, im);
        if (ip[0] != base[0] || im[0] != base[0] || ip[1] != base[1] || im[1] != base[1]) bad = 1;
        grad[k] = (kp - km) / (2.0 * h);
    }
    return bad;
}

int64_t orc_curvature_grad_nbr(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind,
                               const float *grad_kappa, double h, double *grad_phi, uint8_t *bad_cells)
{
    int64_t total = X * Y * Z, c, nif = 0, k, nbad = 0;
    int64_t *list;
    double *part;
    int *bad;
    for (c = 0; c < total; ++c) { grad_phi[c] = 0.0; if (bad_cells) bad_cells[c] = 0; }
    for (c = 0; c < total; ++c) {
        int64_t x = c % X, y = (c / X) % Y, z = c / (X * Y);
        if (x >= 1 && y >= 1 && z >= 1 && x <= X - 2 && y <= Y - 2 && z <= Z - 2 &&
            is_interface(phi[c])) ++nif;
    }
    list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nif > 0 ? nif : 1));
    part = (double *)malloc(sizeof(double) * 125 * (size_t)(nif > 0 ? nif : 1));
    bad = (int *)malloc(sizeof(int) * (size_t)(nif > 0 ? nif : 1));
    k = 0;
    for (c = 0; c < total; ++c) {
        int64_t x = c % X, y = (c / X) % Y, z = c / (X * Y);
        if (x >= 1 && y >= 1 && z >= 1 && x <= X - 2 && y <= Y - 2 && z <= Z - 2 &&
            is_interface(phi[c])) list[k++] = c;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < nif; ++k) {
        int64_t cc = list[k], x = cc % X, y = (cc / X) % Y, z = cc / (X * Y);
        double v[125];
        unsigned char inside[27];
        gather125(phi, X, Y, Z, x, y, z, v, inside);
        bad[k] = orc_curv_cell_nbr_fd_grad(v, inside, kind, h, part + 125 * k);
    }
    for (k = 0; k < nif; ++k) {                /* fixed-order scatter, entries inside the lattice */
        int64_t cc = list[k], x = cc % X, y = (cc / X) % Y, z = cc / (X * Y);
        double gk = (double)grad_kappa[cc];
        int dx, dy, dz;
        for (dz = -2; dz <= 2; ++dz) for (dy = -2; dy <= 2; ++dy) for (dx = -2; dx <= 2; ++dx) {
            int64_t gx = x + dx, gy = y + dy, gz = z + dz;
            if (gx < 0 || gy < 0 || gz < 0 || gx >= X || gy >= Y || gz >= Z) continue;
            grad_phi[(gz * Y + gy) * X + gx] += gk * part[125 * k + (dz + 2) * 25 + (dy + 2) * 5 + (dx + 2)];
        }
        if (bad[k]) { ++nbad; if (bad_cells) bad_cells[cc] = 1; }
    }
    free(list); free(part); free(bad);
    return nbad;
}

int64_t orc_curvature_grad(const float *phi, int64_t X, int64_t Y, int64_t Z,
                           const float *grad_kappa, double h, double *grad_phi,
                           uint8_t *bad_cells)
{
    return orc_curvature_grad_ex(phi, X, Y, Z, 0, grad_kappa, h, grad_phi, bad_cells);
}
