/*
 * FP64 CPU oracle for PLIC inversion and PLIC curvature.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and plic_oracle.c are the plain, slow
 * reference that the GPU library is checked against.  Only the test-suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load or call it;
 * the GPU library neither includes nor links it, and it includes nothing from
 * the GPU library.
 *
 * Conventions (Lehmann & Gekle, "Analytic Solution to the Piecewise Linear
 * Interface Construction Problem ...", Sec. 2 "Plane-Cube Intersection"):
 *   unit cube [-1/2, 1/2]^3 centred at the origin; plane n . x = d0;
 *   V0 = volume of { x in cube : n . x <= d0 } in [0, 1];
 *   d0 in [-S/2, S/2], S = |nx| + |ny| + |nz|.
 * Every routine works for any non-zero n (the plane n . x = d0, so d0 is
 * homogeneous of degree 1 in n); n = 0 or a NaN input gives NaN.
 */
#ifndef PLIC_ORACLE_H
#define PLIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* forward volume V0(n, d0) (Sec. 2.2, eq. of the five-case volume) */
double orc_volume1(double nx, double ny, double nz, double d0);
/* inverse: d0(n, V0) by bisection on the forward volume; V0 clamped to [0,1] */
double orc_offset1(double nx, double ny, double nz, double V0);
/* reduced-space volume F(u) for sorted 0 <= a1 <= a2 <= a3, a3 > 0, u in [0, S/2] */
double orc_reduced_volume(double a1, double a2, double a3, double u);
/* derivatives of d0(n, V0): dd0/dV0 = |n| / A (A = area of the intersection
 * polygon) and dd0/dn = centroid of that polygon (cube-centred coordinates).
 * Built from the explicit polygon.  Returns the number of polygon vertices. */
int orc_offset_grad1(double nx, double ny, double nz, double V0,
                     double *d0, double *dd_dV0, double dd_dn[3], double *area);

/* batched versions (OpenMP over problems) */
void orc_volume(const double *nx, const double *ny, const double *nz, const double *d0,
                double *V0, int64_t count);
void orc_offset(const double *nx, const double *ny, const double *nz, const double *V0,
                double *d0, int64_t count);
void orc_offset_grad(const double *nx, const double *ny, const double *nz, const double *V0,
                     double *d0, double *dd_dV0, double *dd_dnx, double *dd_dny,
                     double *dd_dnz, int64_t count);

/* Scardovelli-Zaleski solution in the form of Kawano's implementation (Sec.
 * 2.4), with that code's case order, reduced volume and "alpha == 0 means
 * unsettled" rule (NaN for an axis normal at V0 in {0, 1}, Sec. 2.6).  kase:
 * 1..5 (0 for NaN inputs); acos_arg: the trigonometric root's argument in the
 * cubic cases (3), (4), NaN otherwise. */
double orc_offset_kawano1(double nx, double ny, double nz, double V0, int *kase, double *acos_arg);
void orc_offset_kawano(const double *nx, const double *ny, const double *nz, const double *V0,
                       double *d0, int32_t *kase, double *acos_arg, int64_t count);

/* ---- plane-sphere intersection (Sec. 3): sphere of unit volume, radius
 * r = (3 / (4 pi))^(1/3); d0 = signed distance of the plane from the centre,
 * V0 = volume on the side n.x <= d0 (any unit normal: the sphere is isotropic) */
double orc_sphere_volume1(double d0);
double orc_sphere_offset1(double V0);
void orc_sphere_volume(const double *d0, double *V0, int64_t count);
void orc_sphere_offset(const double *V0, double *d0, int64_t count);

/* ---- curvature (Sec. 4 and Appendix B) ----
 * Neighbourhood index q = (dz+1)*9 + (dy+1)*3 + (dx+1), centre q = 13.
 * mask[q] != 0 marks interface neighbours (0 < phi < 1) used as fit points.
 * info (may be NULL) receives: info[0] = number of fit points,
 * info[1] = bitmask of active fit parameters (A,B,C,H,I -> bits 0..4),
 * info[2] = ratio largest/smallest accepted LDL^T pivot (conditioning proxy). */
double orc_curv_cell(const double phi[27], const unsigned char mask[27], double info[3]);
/* same, also returning the normal, the fit coefficients (A,B,C,H,I) */
double orc_curv_cell_full(const double phi[27], const unsigned char mask[27], double info[3],
                          double normal[3], double coef[5]);
/* same with a caller-chosen auxiliary vector r instead of the paper's */
double orc_curv_cell_r(const double phi[27], const unsigned char mask[27], const double raux[3],
                       double info[3], double normal[3], double coef[5]);
/* least-squares paraboloid through points (x_i, y_i, z_i) with the rank rule;
 * returns the number of active parameters, coef[5] = (A,B,C,H,I) */
int orc_fit_paraboloid(const double *px, const double *py, const double *pz, int npts,
                       double coef[5], double *cond);
/* mean curvature of z = Ax^2+By^2+Cxy+Hx+Iy at the origin (paper's sign) */
double orc_paraboloid_kappa(const double coef[5]);
/* whole lattice, phi[(z*Y + y)*X + x] (x fastest); kappa = 0 off the interface
 * and on the outer one-cell layer.  flags (may be NULL) per cell: bit0 interface
 * computed, bit1 ill-conditioned fit (pivot ratio > 1e8), bit2 fewer than 5 points. */
void orc_curvature(const float *phi, int64_t X, int64_t Y, int64_t Z, double *kappa,
                   uint8_t *flags);
/* curvature of selected cells only (cell = linear index) */
void orc_curvature_cells(const float *phi, int64_t X, int64_t Y, int64_t Z,
                         const int64_t *cells, int64_t ncells, double *kappa, double *info3);
/* d kappa(cell) / d phi over the 27 neighbours by central finite differences
 * with step h, the interface mask held fixed.  bad != 0 when a perturbation
 * crosses 0 or 1, changes the active parameter set or the point count. */
int orc_curv_cell_fd_grad(const double phi[27], const unsigned char mask[27], double h,
                          double grad[27]);
/* lattice gradient: grad_phi = sum over interior interface cells c of
 * gk[c] * d kappa_c / d phi, by the finite differences above (serial,
 * fixed accumulation order).  Returns the number of cells flagged bad. */
int64_t orc_curvature_grad(const float *phi, int64_t X, int64_t Y, int64_t Z,
                           const float *grad_kappa, double h, double *grad_phi,
                           uint8_t *bad_cells);

/* ---- curvature options ----
 * kind: 0 = Parker-Youngs normal (weights 4/2/1), 1 = centre-of-mass normal
 * (equal weights), App. B.1.  nbr: 0 = every neighbour's PLIC plane uses the
 * centre normal (Sec. 4.2), 1 = each interface neighbour uses its own normal
 * (needs the 5^3 neighbourhood; neighbours on the outer lattice layer keep the
 * centre normal). */
double orc_curv_cell_k(const double phi[27], const unsigned char mask[27], int kind, double info[3],
                       double normal[3]);
/* neighbour-normal variant on p125[(dz+2)*25 + (dy+2)*5 + (dx+2)]; inside27[q]
 * (NULL: all 1) says whether neighbour q's 3^3 neighbourhood is in the lattice;
 * a neighbour outside, or with a vanishing gradient, keeps the centre normal */
double orc_curv_cell_nbr(const double p125[125], const unsigned char inside27[27], int kind, double info[3]);
void orc_curvature_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind, int nbr,
                      double *kappa, uint8_t *flags);
void orc_curvature_cells_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind, int nbr,
                            const int64_t *cells, int64_t ncells, double *kappa, double *info3);
int orc_curv_cell_fd_grad_k(const double phi[27], const unsigned char mask[27], int kind, double h,
                            double grad[27]);
int64_t orc_curvature_grad_ex(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind,
                              const float *grad_kappa, double h, double *grad_phi,
                              uint8_t *bad_cells);
/* the neighbour-normal variant's gradient: central differences over each
 * cell's 5^3 neighbourhood, scattered in cell order (same conventions) */
int orc_curv_cell_nbr_fd_grad(const double p125[125], const unsigned char inside27[27], int kind, double h,
                              double grad[125]);
int64_t orc_curvature_grad_nbr(const float *phi, int64_t X, int64_t Y, int64_t Z, int kind,
                               const float *grad_kappa, double h, double *grad_phi, uint8_t *bad_cells);

#ifdef __cplusplus
}
#endif
#endif
