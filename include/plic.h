/*
 * libplic — PLIC inversion and PLIC curvature on AMD Instinct MI355X (gfx950).
 *
 * Method: M. Lehmann, S. Gekle, "Analytic Solution to the Piecewise Linear
 * Interface Construction Problem and its Application in Curvature Calculation
 * for Volume-of-Fluid Simulation Codes", arXiv 2006.12838.
 *
 * Geometry (Sec. 2, problem statement): the unit cube [-1/2, 1/2]^3 centred at
 * the origin, cut by the plane n . x = d0.  V0 in [0, 1] is the volume of the
 * part with n . x <= d0; d0 lies in [-S/2, S/2] with S = |nx| + |ny| + |nz|.
 * The paper states the problem for a unit normal; every entry point here
 * accepts any non-zero n and describes the plane n . x = d0, so d0 is
 * homogeneous of degree 1 in n (for |n| = 1 this is the paper's d0).
 *
 * Common rules for every entry point
 *  - Array arguments are DEVICE pointers owned by the caller.  The library
 *    allocates nothing and keeps no state between calls, with two stated
 *    exceptions: the static device array of plic_curvature_noalloc_f32, and a
 *    small host-side note, per curvature workspace address, of the phi and
 *    lattice its last scan was for (plic_curvature_backward_reuse_f32).
 *  - Arrays are structure-of-arrays, one element per problem (or per lattice
 *    cell), naturally aligned (4 bytes for float, 8 for double).  Outputs may
 *    alias an input of the same element index only where stated.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *    default stream) and the call returns without waiting.  Kernel faults are
 *    reported by the HIP runtime at the next synchronisation, not here.
 *  - Arguments are validated before anything is enqueued; a call that returns
 *    an error has enqueued nothing.  count == 0 (or an empty lattice) is valid
 *    and does nothing.  No call aborts the process or throws.
 *  - Inputs: V0 is clamped to [0, 1]; a NaN in (n, V0) gives NaN; n = 0 gives NaN.
 *  - Results are deterministic: the same inputs on the same device give the
 *    same bits.
 */
#ifndef PLIC_H
#define PLIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PLIC_OK 0
#define PLIC_EINVAL (-1)  /* null / misaligned / overlapping pointer, negative size, bad enum */
#define PLIC_EHIP (-2)    /* the HIP runtime refused the launch (see plic_last_hip_error) */
#define PLIC_EWORKSPACE (-3) /* the workspace is smaller than the call needs (every other argument valid) */

/* PLIC solvers: the four inversion methods of Sec. 2.3-2.5, compared in Sec. 2.6 */
#define PLIC_ANALYTIC 0   /* the paper's analytic solution (Sec. 2.3, trigonometric root via atan) */
#define PLIC_SZ 1         /* optimized Scardovelli-Zaleski solution (Sec. 2.4, root via asin)      */
#define PLIC_NEWTON 2     /* Newton-Raphson on the cubic cases (Sec. 2.5), |step| <= 1e-6 (f32)    */
#define PLIC_NESTED 3     /* nested intervals (bisection) on the cubic cases (Sec. 2.5)            */
/* The SZ solution as implemented by Kawano (Sec. 2.4): the unoptimized variant
 * of the comparison, root via acos / cos, with that code's case order and
 * reduced volume.  It returns NaN for an axis normal at V0 in {0, 1}, as the
 * paper reports (Sec. 2.6), and is not held to the accuracy bound of the
 * offset entry points: its cubic coefficients cancel for a small m1, so in
 * FP32 it loses up to about 5e-5 on random unit normals and far more (and
 * gives NaN) near the axes and face diagonals; in FP64 it stays within
 * 1e-13 of the exact root on random normals.  Accepted by the offset, offset
 * backward and benchmark entry points; the curvature returns PLIC_EINVAL. */
#define PLIC_SZ_KAWANO 4

/* arithmetic precision of the computation (independent of the storage type) */
#define PLIC_FP32 0       /* all FP32                                                              */
#define PLIC_MIXED 1      /* FP32 bulk; FP64 for a cubic-case root within 2^-16 S of a case
                             boundary (one FP64 Newton step on the case's cubic) and for the
                             curvature's fit solve                                               */
#define PLIC_FP64 2       /* all FP64                                                              */

/* interface normal of the curvature step (App. B.1) */
#define PLIC_NORMAL_PY 0  /* Parker-Youngs: fill-level gradient with weights 4 / 2 / 1              */
#define PLIC_NORMAL_CM 1  /* centre of mass: equal weights                                         */

/*
 * plic_offset_f32 / plic_offset_f64 — the PLIC problem (Sec. 2): n, V0 -> d0.
 *   nx, ny, nz, V0 : inputs, `count` elements each.
 *   d0             : output, `count` elements; may alias V0 (read before write).
 *   solver         : PLIC_ANALYTIC, PLIC_SZ, PLIC_NEWTON, PLIC_NESTED or
 *                    PLIC_SZ_KAWANO.
 *   precision      : (f32 only) PLIC_FP32, PLIC_MIXED or PLIC_FP64; the f64 entry
 *                    point always computes in FP64.
 * Accuracy: |d0 - exact| <= 1e-5 (f32 storage) and <= 1e-12 (f64), absolute,
 * for unit normals, for the paper's four solvers (PLIC_SZ_KAWANO: see there).
 * Returns PLIC_OK, PLIC_EINVAL or PLIC_EHIP.
 */
int plic_offset_f32(const float *nx, const float *ny, const float *nz, const float *V0,
                    float *d0, int64_t count, int solver, int precision, void *stream);
int plic_offset_f64(const double *nx, const double *ny, const double *nz, const double *V0,
                    double *d0, int64_t count, int solver, void *stream);

/*
 * plic_volume_f32 / plic_volume_f64 — the inverse PLIC problem (Sec. 2.2,
 * five-case volume): n, d0 -> V0.  d0 outside [-S/2, S/2] gives 0 or 1.
 *   V0 : output, may alias d0.
 *   precision : (f32 only) PLIC_FP32 or PLIC_FP64 (PLIC_MIXED means FP32 here).
 */
int plic_volume_f32(const float *nx, const float *ny, const float *nz, const float *d0,
                    float *V0, int64_t count, int precision, void *stream);
int plic_volume_f64(const double *nx, const double *ny, const double *nz, const double *d0,
                    double *V0, int64_t count, void *stream);

/*
 * plic_offset_backward_f32 / _f64 — vector-Jacobian product of plic_offset.
 * Implicit differentiation of V0 = volume{x in cube : n.x <= d0}:
 *   dd0/dV0 = |n| / A  and  dd0/dn = c,
 * A the area and c the centroid (cube-centred) of the polygon where the plane
 * cuts the cube.  d0 is recomputed with `solver` (nothing is stored by the
 * forward call).  Outputs: grad_n* = grad_d0 * c_*, grad_V0 = grad_d0 * |n| / A.
 * Where A = 0 (V0 in {0, 1} with a corner or an edge as the polygon)
 * dd0/dV0 is +inf.  Outputs must not alias inputs.
 */
int plic_offset_backward_f32(const float *nx, const float *ny, const float *nz, const float *V0,
                             const float *grad_d0, float *grad_nx, float *grad_ny,
                             float *grad_nz, float *grad_V0, int64_t count, int solver,
                             int precision, void *stream);
int plic_offset_backward_f64(const double *nx, const double *ny, const double *nz,
                             const double *V0, const double *grad_d0, double *grad_nx,
                             double *grad_ny, double *grad_nz, double *grad_V0, int64_t count,
                             int solver, void *stream);

/*
 * plic_curvature_workspace_bytes — recommended size of the device workspace of
 * plic_curvature_f32 and plic_curvature_backward_f32 for an X*Y*Z lattice.
 * The workspace holds a fixed part of 256 + 784 * tiles bytes (64x4x4 tiles:
 * work-list counters, per-tile interface flags, bitmasks and work lists;
 * about 0.8 byte per cell) and, for the backward pass, a store of 108 bytes
 * (27 floats) per interface cell.  The recommended size budgets 16 interface
 * cells per tile (41 MB at 256^3); any size of at least the fixed part is
 * valid: rows go to the interface cells in tile order, and cells beyond the
 * store's capacity are recomputed by the backward pass (slower; the same bits
 * unless the 3x3x3-grown neighbourhood of a 64x4x4 tile holds more than 128
 * interface cells, where the summation order differs in the last bits).
 * Results are deterministic for a given size.  The forward pass uses only the fixed
 * part.  0 for an empty or invalid lattice (2^24 tiles or more, i.e. about
 * 1.7e10 cells, is invalid).
 * The workspace is caller-owned device memory; its contents need no
 * initialisation (each call clears what it uses with a kernel) and are
 * scratch after the call.
 */
size_t plic_curvature_workspace_bytes(int64_t X, int64_t Y, int64_t Z);

/*
 * plic_curvature_workspace_bytes_ex — as plic_curvature_workspace_bytes, and
 * with neighbour_normals = 1 the recommended size for the backward of the
 * neighbour-normal variant (plic_curvature_backward_ex_f32): its rows hold 105
 * floats (the 27 contributions and the adjoints of the 26 neighbours' own
 * fill-level gradients) plus 3 (the adjoint of the cell's own gradient),
 * 432 bytes per interface cell, 64 per tile budgeted (that variant has no
 * recomputing fallback; 453 MB at 256^3).  0 for an invalid lattice or flag.
 */
size_t plic_curvature_workspace_bytes_ex(int64_t X, int64_t Y, int64_t Z, int neighbour_normals);

/*
 * plic_curvature_f32 — PLIC curvature of a VoF fill-level lattice (Sec. 4.1-4.2,
 * Appendix B): for every interface cell (0 < phi < 1) away from the outer
 * one-cell layer: Parker-Youngs normal from the 3x3x3 fill levels, local frame
 * from the fixed vector r, PLIC points of the interface neighbours (centre
 * normal for all), least-squares paraboloid z = Ax^2+By^2+Cxy+Hx+Iy, mean
 * curvature at the origin.
 *   phi   : X*Y*Z floats, x fastest (index (z*Y + y)*X + x, torch shape (Z,Y,X)).
 *   kappa : X*Y*Z floats, written everywhere; 0 on non-interface cells and on
 *           the outer layer.  Must not overlap phi or the workspace.
 *   solver, precision : PLIC solver for the points (the paper's four;
 *           PLIC_SZ_KAWANO gives PLIC_EINVAL); PLIC_FP32 fits in FP32,
 *           PLIC_MIXED fits in FP64 (FP32 points), PLIC_FP64 is FP64 throughout.
 *   workspace, workspace_bytes : device scratch, 4-byte aligned, not
 *           overlapping phi or kappa, of at least the fixed part (see
 *           plic_curvature_workspace_bytes); a smaller one gives
 *           PLIC_EWORKSPACE.  Calls that overlap in time must use distinct
 *           workspaces.  The call leaves its interface-cell count in the
 *           workspace (plic_curvature_status).
 * Sign: kappa = +1/R for a fluid sphere of radius R (the normal points out of
 * the fluid); the paper's formula is negated for this.  Fits with fewer than 5
 * points use the leading parameters only (App. B.3); a pivot of the LDL^T
 * factorisation below 1e-10 (FP64 fit) / 1e-5 (FP32 fit) of the largest
 * diagonal entry drops its parameter.  X, Y, Z >= 1.  Deterministic.
 */
int plic_curvature_f32(const float *phi, int64_t X, int64_t Y, int64_t Z, float *kappa,
                       int solver, int precision, void *workspace, size_t workspace_bytes,
                       void *stream);

/*
 * plic_curvature_noalloc_f32 — plic_curvature_f32 (Parker-Youngs normal, the
 * centre normal for every point) for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It takes no workspace and allocates nothing: its
 * workspace is a static device array of 16 MiB inside the library, one per
 * GPU the library runs on, held until the process ends.  Lattices of up to
 * 21,399 tiles of 64x4x4 cells (256^3 has 16,384) fit; a larger lattice
 * returns PLIC_EWORKSPACE before anything is launched.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents (each call
 * clears what it uses): calls that overlap in time on one GPU (several
 * streams or host threads) race and must be serialised by the caller.
 * Arguments, status codes and results (bit for bit) are otherwise those of
 * plic_curvature_f32.
 */
int plic_curvature_noalloc_f32(const float *phi, int64_t X, int64_t Y, int64_t Z, float *kappa,
                               int solver, int precision, void *stream);

/*
 * plic_curvature_backward_f32 — vector-Jacobian product of plic_curvature:
 * grad_phi[j] = sum over interface cells c of grad_kappa[c] * d kappa_c / d phi_j.
 * The neighbourhood of each cell is recomputed (nothing is stored by the
 * forward call).  The interface mask, the case of each PLIC point and the set
 * of fit parameters are held fixed (they are piecewise constant in phi).
 * grad_phi is written everywhere (zero away from the interface band); it must
 * not overlap phi, grad_kappa or the workspace.  Workspace as for the forward
 * call.  Deterministic (fixed summation order).
 */
int plic_curvature_backward_f32(const float *phi, int64_t X, int64_t Y, int64_t Z,
                                const float *grad_kappa, float *grad_phi, int solver,
                                int precision, void *workspace, size_t workspace_bytes,
                                void *stream);

/*
 * plic_sphere_offset_f32 / _f64 — the PLIC problem for a spherical cell of
 * unit volume (Sec. 3): V0 -> d0, the signed distance of the plane from the
 * sphere's centre with volume V0 on the side n.x <= d0 (any normal: the
 * sphere is isotropic), d0 in [-r, r], r = (3 / (4 pi))^(1/3).  The paper's
 * closed form d0 = (6/pi)^(1/3) sin(pi/6 - atan2(2 sqrt(V0 - V0^2), 2 V0 - 1)/3).
 * V0 is clamped to [0, 1]; NaN stays NaN.
 * plic_sphere_volume_f32 / _f64 — the inverse: the spherical cap
 * (pi/3) (r + d0)^2 (2r - d0), 0 below -r and 1 above r.
 *   in, out : count elements each (V0 -> d0, or d0 -> V0); out may be the
 *             same array as in, otherwise they must not overlap.
 * Status codes and stream as for plic_offset_f32; the f32 entries compute in
 * FP32.
 */
int plic_sphere_offset_f32(const float *V0, float *d0, int64_t count, void *stream);
int plic_sphere_offset_f64(const double *V0, double *d0, int64_t count, void *stream);
int plic_sphere_volume_f32(const float *d0, float *V0, int64_t count, void *stream);
int plic_sphere_volume_f64(const double *d0, double *V0, int64_t count, void *stream);

/*
 * plic_curvature_ex_f32 — plic_curvature_f32 with the options of the paper's
 * curvature section:
 *   normal            : PLIC_NORMAL_PY (as plic_curvature_f32) or PLIC_NORMAL_CM
 *                       (App. B.1; about 4 degrees of normal error against 1).
 *   neighbour_normals : 0 = every neighbour's PLIC plane uses the centre
 *                       normal (Sec. 4.2, as plic_curvature_f32); 1 = each
 *                       interface neighbour's plane uses that neighbour's own
 *                       normal from its 3x3x3 fill levels (the variant of
 *                       Sec. 4.2 and Sec. 4.3), its point being the foot of
 *                       its plane, e + d0(phi_q, n_q) n_q - d0(phi_0, n) n, in
 *                       the centre frame.  A neighbour on the outer lattice
 *                       layer, or with a vanishing gradient, keeps the centre
 *                       normal.  Reads a 5x5x5 neighbourhood per cell.
 * Other arguments, workspace and results as plic_curvature_f32.
 */
int plic_curvature_ex_f32(const float *phi, int64_t X, int64_t Y, int64_t Z, float *kappa,
                          int solver, int precision, int normal, int neighbour_normals,
                          void *workspace, size_t workspace_bytes, void *stream);

/*
 * plic_curvature_backward_ex_f32 — plic_curvature_backward_f32 with the options
 * of plic_curvature_ex_f32.  normal: its weights enter the normal's adjoint.
 * neighbour_normals = 1: the backward of the neighbour-normal variant, whose
 * gradient reaches two cells from an interface cell (each neighbour's own
 * normal reads that neighbour's 3x3x3).  Each interface cell stores its 27
 * contributions and the adjoints of its neighbours' own fill-level gradients
 * in a row; a second pass sums, for every interface cell, the adjoints of its
 * own gradient that its neighbours stored; the gather adds both in a fixed
 * order (deterministic).  This variant has no recomputing fallback: the
 * workspace must hold at least one row (fixed part + 432 bytes, else
 * PLIC_EWORKSPACE), and where a row does not fit, the gradient on the
 * affected tile's cells next to the interface is NaN.  Such a call still
 * returns PLIC_OK (the interface count is only known on the device);
 * plic_curvature_status then returns PLIC_EWORKSPACE with the size that
 * holds every row.  plic_curvature_workspace_bytes_ex (X, Y, Z, 1) gives room
 * for 64 interface cells per tile.  The interface masks and the choice of
 * each neighbour's normal are held fixed.
 */
int plic_curvature_backward_ex_f32(const float *phi, int64_t X, int64_t Y, int64_t Z,
                                   const float *grad_kappa, float *grad_phi, int solver,
                                   int precision, int normal, int neighbour_normals,
                                   void *workspace, size_t workspace_bytes, void *stream);

/*
 * plic_curvature_backward_reuse_f32 — plic_curvature_backward_ex_f32 after a
 * forward (Sec. 4.2 and App. B; the derivative itself is not in the paper) on
 * the same workspace: the interface scan's records that the forward left there
 * (bitmasks, prefix counts, work items, tile counts; they depend on phi only)
 * are used again instead of scanning phi a second time, as a training step's
 * backward follows its forward.  The caller guarantees that phi's contents did
 * not change since the last curvature call on `workspace` (forward or
 * backward, any options) and that no other use of the workspace memory came
 * between.  The library checks what it can see: when the last call it
 * launched on this workspace address was not on the same phi address and
 * lattice, this call scans phi as plic_curvature_backward_ex_f32 does.
 * Arguments, status codes and results (bit for bit) as
 * plic_curvature_backward_ex_f32.
 */
int plic_curvature_backward_reuse_f32(const float *phi, int64_t X, int64_t Y, int64_t Z,
                                      const float *grad_kappa, float *grad_phi, int solver,
                                      int precision, int normal, int neighbour_normals,
                                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * plic_curvature_status — what the last curvature call (forward or backward,
 * any variant) found on `workspace`, read after it completed: this call
 * synchronises `stream` (the stream of that call) and copies 24 bytes of the
 * workspace header to the host.  Not for use under graph capture.
 *   X, Y, Z, neighbour_normals, workspace_bytes : as in that call.
 *   interface_cells    : if not NULL, receives its interface-cell count.
 *   bytes_for_all_rows : if not NULL, receives the workspace size that holds
 *                        a backward row for every one of those cells (fixed
 *                        part + 108 bytes per cell, 432 with neighbour normals).
 * Returns PLIC_EWORKSPACE when neighbour_normals = 1 and the workspace holds
 * fewer rows than there are interface cells (a backward of the
 * neighbour-normal variant on it has NaN where rows were missing; give it
 * bytes_for_all_rows and call it again), else PLIC_OK (the base backward
 * recomputes missing rows, so its result is complete for any size).
 * PLIC_EINVAL for an invalid lattice, flag or pointer, PLIC_EHIP when the
 * stream or the copy fails.  Row indices are 32-bit: the neighbour-normal
 * variant holds at most 10,226,107 rows, whatever the workspace.
 */
int plic_curvature_status(const void *workspace, size_t workspace_bytes, int64_t X, int64_t Y, int64_t Z,
                          int neighbour_normals, int64_t *interface_cells, size_t *bytes_for_all_rows,
                          void *stream);

/* human-readable status; never NULL */
const char *plic_status_string(int status);
/* library version string, e.g. "plic-mi355x 0.1.0 (gfx950)" */
const char *plic_version(void);
/* the hipError_t value behind the last PLIC_EHIP returned on this thread (0 if none) */
int plic_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PLIC_H */
