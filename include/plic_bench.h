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
 *   stream     : hipStream_t as void* (NULL: the null stream).
 * Returns PLIC_OK, PLIC_EINVAL (null / misaligned pointer, count < 0, L < 2,
 * bad solver or blank flag, err overlapping an input) or PLIC_EHIP (launch
 * error).  Asynchronous on stream.
 */
int plic_bench_isolated_f32(const float* nx, const float* ny, const float* nz, int64_t count, int L, int solver,
                            int blank, float* err, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PLIC_BENCH_H */
