/*
 * plic_bench.h — compute-isolated timing of the PLIC inversion in the manner
 * of the paper's GPU benchmark (Lehmann & Gekle, arXiv 2006.12838, Sec. 2.6.2
 * and Table 3): every thread keeps one normal and sweeps L equally spaced
 * fill levels V0 = j / (L - 1), j = 0 .. L-1 (edge cases included) in series,
 * inverting each and measuring the round trip E = |V(n, d0(n, V0)) - V0|
 * with the forward volume (the paper's "inverse PLIC").  The blank run
 * replaces the inversion by d0 = V0 - 1/2; its time, subtracted from a
 * solver's, isolates the inversion (per evaluation: divide by count * L).
 *
 * Same status codes and library as plic.h.  Not part of the production path:
 * it exists to make per-evaluation times comparable with the paper's table.
 */
#ifndef PLIC_BENCH_H
#define PLIC_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * plic_bench_isolated_f32 — FP32, one thread per normal.
 *   nx, ny, nz : device arrays of count normals (any non-zero length), read.
 *   count      : number of normals (0 does nothing).
 *   L          : fill levels per normal, L >= 2.
 *   solver     : PLIC_ANALYTIC / PLIC_SZ / PLIC_NEWTON / PLIC_NESTED /
 *                PLIC_SZ_KAWANO (plic.h); Kawano's form gives err = NaN for an
 *                axis normal (its V0 = 0 and V0 = 1 evaluations).
 *   blank      : 0 = invert with the solver, 1 = blank run (d0 = V0 - 1/2).
 *   err        : device array of count floats, written: the sum over the L
 *                fill levels of E for that normal (E_avg = sum / (count L)).
 *   d0         : NULL, or a device array of count * L floats that receives
 *                every offset the sweep computes, d0[j * count + i] for
 *                normal i and fill level V0 = j / (L - 1) (for checking the
 *                kernel against a reference; a timed run passes NULL, which
 *                launches an instance that stores nothing per fill level).
 *   stream     : hipStream_t as void* (NULL: the null stream).
 * Returns PLIC_OK, PLIC_EINVAL (null / misaligned pointer, count < 0, L < 2,
 * bad solver or blank flag, err or d0 overlapping another array,
 * count > 2^31) or PLIC_EHIP (launch error).  Asynchronous on stream.
 */
int plic_bench_isolated_f32(const float* nx, const float* ny, const float* nz, int64_t count, int L, int solver,
                            int blank, float* err, float* d0, void* stream);

/*
 * plic_bench_valu — issue-rate probe for the vector ALU (the ceiling against
 * which the PLIC kernels' instruction issue is compared).  Each of `threads`
 * threads (workgroups of 256) runs 8 independent dependency chains of one
 * instruction, 4 deep per loop trip, for `iters` trips: exactly 32 * iters
 * instructions of the op per thread, with no other vector instruction in the
 * loop.  Time the launch (minus an iters = 0 launch) to get the op's rate:
 * threads * 32 * iters lane-operations per second.
 *   op      : one of PLIC_VALU_* below (non-packed FMA, or a transcendental).
 *   threads : >= 0 and <= 2^31; use many waves per SIMD (for example 2^22).
 *   iters   : >= 0.
 *   seed    : start value of the chains (kept finite by each op's form).
 *   sink    : device array of `threads` floats, written (keeps results live).
 * Returns PLIC_OK, PLIC_EINVAL (bad op, negative size, null or misaligned
 * sink) or PLIC_EHIP.  Asynchronous on stream.
 */
#define PLIC_VALU_FMA_F32 0   /* v_fma_f32                                   */
#define PLIC_VALU_FMA_F64 1   /* v_fma_f64                                   */
#define PLIC_VALU_SQRT_F32 2  /* v_sqrt_f32                                  */
#define PLIC_VALU_RSQ_F32 3   /* v_rsq_f32                                   */
#define PLIC_VALU_RCP_F32 4   /* v_rcp_f32                                   */
#define PLIC_VALU_SIN_F32 5   /* v_sin_f32                                   */
#define PLIC_VALU_EXP_F32 6   /* v_exp_f32 (of -x)                           */
#define PLIC_VALU_LOG_F32 7   /* v_log_f32 (of |x|)                          */
#define PLIC_VALU_RCP_F64 8   /* v_rcp_f64                                   */
#define PLIC_VALU_SQRT_F64 9  /* v_sqrt_f64                                  */
#define PLIC_VALU_FMA_SIN_F32 10 /* 16 v_fma_f32 and 16 v_sin_f32 per trip  */
int plic_bench_valu(int op, int64_t threads, int iters, float seed, float* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PLIC_BENCH_H */
