// Compute-isolated PLIC timing after the paper's GPU benchmark (Sec. 2.6.2,
// Table 3): one normal per thread, L fill levels in series, round trip
// through the forward volume; the blank run swaps the inversion for
// d0 = V0 - 1/2.  One problem per thread, as in the paper's kernels.  An
// optional second output keeps every offset (for checking the kernel against
// a reference); the timed kernel is the instance that writes none.
#include <hip/hip_runtime.h>

#include "../../include/plic_bench.h"
#include "plic_host.hpp"
#include "plic_math.hpp"

namespace plic {
namespace {

constexpr int kBenchBlock = 256;

template <int SOLVER, bool BLANK, bool KEEP>
__global__ __launch_bounds__(kBenchBlock) void k_isolated(const float* __restrict__ nx, const float* __restrict__ ny,
                                                          const float* __restrict__ nz, int64_t count, int L,
                                                          float* __restrict__ err, float* __restrict__ d0_out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBenchBlock + threadIdx.x;
    if (i >= count) return;
    const float a = nx[i], b = ny[i], c = nz[i];
    const float last = static_cast<float>(L - 1);
    float e = 0.0f;
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
        const float V0 = static_cast<float>(j) / last;          // exact 0 and 1 at the ends
        const float d0 = BLANK ? V0 - 0.5f : offset<SOLVER, float, float>(a, b, c, V0);
        if (KEEP) d0_out[static_cast<int64_t>(j) * count + i] = d0;      // [L][count]: coalesced per j
        e += fabsf(volume<float>(a, b, c, d0) - V0);
    }
    err[i] = e;
}

template <int SOLVER>
void launch_isolated(bool blank, const float* nx, const float* ny, const float* nz, int64_t count, int L,
                     float* err, float* d0, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((count + kBenchBlock - 1) / kBenchBlock)), block(kBenchBlock);
    if (blank && d0)
        hipLaunchKernelGGL((k_isolated<SOLVER, true, true>), grid, block, 0, st, nx, ny, nz, count, L, err, d0);
    else if (blank)
        hipLaunchKernelGGL((k_isolated<SOLVER, true, false>), grid, block, 0, st, nx, ny, nz, count, L, err, d0);
    else if (d0)
        hipLaunchKernelGGL((k_isolated<SOLVER, false, true>), grid, block, 0, st, nx, ny, nz, count, L, err, d0);
    else
        hipLaunchKernelGGL((k_isolated<SOLVER, false, false>), grid, block, 0, st, nx, ny, nz, count, L, err, d0);
}

// ---- VALU issue-rate probe ----------------------------------------------------
// Each thread runs kChains independent dependency chains of one instruction,
// kUnroll deep per loop trip: kChains * kUnroll = 32 instructions of the op per
// trip, no other vector instruction inside the loop (the trip count lives in
// scalar registers).  With enough waves per SIMD the chains hide the
// instruction latency, so the launch time measures the op's issue rate.
constexpr int kChains = 8, kUnroll = 4;

template <int OP> struct ValuOp;
template <> struct ValuOp<PLIC_VALU_FMA_F32> {
    using T = float;
    static __device__ __forceinline__ float f(float x, float a, float b) { return __builtin_fmaf(x, a, b); }
};
template <> struct ValuOp<PLIC_VALU_FMA_F64> {
    using T = double;
    static __device__ __forceinline__ double f(double x, double a, double b) { return __builtin_fma(x, a, b); }
};
template <> struct ValuOp<PLIC_VALU_SQRT_F32> {
    using T = float;
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_sqrtf(x); }
};
template <> struct ValuOp<PLIC_VALU_RSQ_F32> {
    using T = float;
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_rsqf(x); }
};
template <> struct ValuOp<PLIC_VALU_RCP_F32> {
    using T = float;
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_rcpf(x); }
};
template <> struct ValuOp<PLIC_VALU_SIN_F32> {
    using T = float;
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_sinf(x); }
};
template <> struct ValuOp<PLIC_VALU_EXP_F32> {
    using T = float;    // exp2(-x): bounded, the negation is a source modifier
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_exp2f(-x); }
};
template <> struct ValuOp<PLIC_VALU_LOG_F32> {
    using T = float;    // log2(|x|): the absolute value is a source modifier
    static __device__ __forceinline__ float f(float x, float, float) { return __builtin_amdgcn_logf(__builtin_fabsf(x)); }
};
template <> struct ValuOp<PLIC_VALU_RCP_F64> {
    using T = double;
    static __device__ __forceinline__ double f(double x, double, double) { return __builtin_amdgcn_rcp(x); }
};
template <> struct ValuOp<PLIC_VALU_SQRT_F64> {
    using T = double;
    static __device__ __forceinline__ double f(double x, double, double) { return __builtin_amdgcn_sqrt(x); }
};

template <> struct ValuOp<PLIC_VALU_FMA_SIN_F32> {
    using T = float;    // chains 0-3 v_fma_f32, chains 4-7 v_sin_f32 (does the sine overlap the FMAs?)
    static __device__ __forceinline__ float f(float x, float a, float b) { return __builtin_fmaf(x, a, b); }
    static __device__ __forceinline__ float g(float x, float, float) { return __builtin_amdgcn_sinf(x); }
};

template <int OP>
__global__ __launch_bounds__(kBenchBlock) void k_valu(int64_t threads, int iters, float seed, float* __restrict__ sink) {
    using T = typename ValuOp<OP>::T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBenchBlock + threadIdx.x;
    if (i >= threads) return;
    const T a = T(seed) * T(0.5), b = T(seed) * T(0.25);
    T x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = T(seed) + T(c) * T(0.125) + T(threadIdx.x) * T(1e-6);
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (OP == PLIC_VALU_FMA_SIN_F32)
                    x[c] = c < kChains / 2 ? ValuOp<OP>::f(x[c], a, b) : ValuOp<OP>::g(x[c], a, b);
                else
                    x[c] = ValuOp<OP>::f(x[c], a, b);
            }
        }
    }
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc += x[c];
    sink[i] = float(acc);
}

template <int OP>
void launch_valu(int64_t threads, int iters, float seed, float* sink, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((threads + kBenchBlock - 1) / kBenchBlock)), block(kBenchBlock);
    hipLaunchKernelGGL((k_valu<OP>), grid, block, 0, st, threads, iters, seed, sink);
}

}  // namespace
}  // namespace plic

using namespace plic;

extern "C" int plic_bench_valu(int op, int64_t threads, int iters, float seed, float* sink, void* stream) {
    if (op < PLIC_VALU_FMA_F32 || op > PLIC_VALU_FMA_SIN_F32 || threads < 0 || iters < 0) return PLIC_EINVAL;
    if (!valid_array(sink, threads)) return PLIC_EINVAL;
    if (threads > (int64_t(1) << 31)) return PLIC_EINVAL;                 // grid: 32-bit work-item count
    if (threads == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (op) {
        case PLIC_VALU_FMA_F32: launch_valu<PLIC_VALU_FMA_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_FMA_F64: launch_valu<PLIC_VALU_FMA_F64>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_SQRT_F32: launch_valu<PLIC_VALU_SQRT_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_RSQ_F32: launch_valu<PLIC_VALU_RSQ_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_RCP_F32: launch_valu<PLIC_VALU_RCP_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_SIN_F32: launch_valu<PLIC_VALU_SIN_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_EXP_F32: launch_valu<PLIC_VALU_EXP_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_LOG_F32: launch_valu<PLIC_VALU_LOG_F32>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_RCP_F64: launch_valu<PLIC_VALU_RCP_F64>(threads, iters, seed, sink, st); break;
        case PLIC_VALU_SQRT_F64: launch_valu<PLIC_VALU_SQRT_F64>(threads, iters, seed, sink, st); break;
        default: launch_valu<PLIC_VALU_FMA_SIN_F32>(threads, iters, seed, sink, st); break;
    }
    return launch_status();
}

extern "C" int plic_bench_isolated_f32(const float* nx, const float* ny, const float* nz, int64_t count, int L,
                                       int solver, int blank, float* err, float* d0, void* stream) {
    if (count < 0 || L < 2 || !valid_solver(solver) || (blank != 0 && blank != 1)) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) || !valid_array(err, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(float);
    if (overlap(err, nb, nx, nb) || overlap(err, nb, ny, nb) || overlap(err, nb, nz, nb)) return PLIC_EINVAL;
    if (count > (int64_t(1) << 31)) return PLIC_EINVAL;                   // grid: 32-bit work-item count
    if (d0 != nullptr) {
        if (count > INT64_MAX / L / static_cast<int64_t>(sizeof(float))) return PLIC_EINVAL;
        const int64_t nd = count * L;
        const size_t db = static_cast<size_t>(nd) * sizeof(float);
        if (!valid_array(d0, nd) || overlap(d0, db, nx, nb) || overlap(d0, db, ny, nb) || overlap(d0, db, nz, nb) ||
            overlap(d0, db, err, nb))
            return PLIC_EINVAL;
    }
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (solver) {
        case kSZ: launch_isolated<kSZ>(blank, nx, ny, nz, count, L, err, d0, st); break;
        case kNewton: launch_isolated<kNewton>(blank, nx, ny, nz, count, L, err, d0, st); break;
        case kNested: launch_isolated<kNested>(blank, nx, ny, nz, count, L, err, d0, st); break;
        case kKawano: launch_isolated<kKawano>(blank, nx, ny, nz, count, L, err, d0, st); break;
        default: launch_isolated<kAnalytic>(blank, nx, ny, nz, count, L, err, d0, st); break;
    }
    return launch_status();
}
