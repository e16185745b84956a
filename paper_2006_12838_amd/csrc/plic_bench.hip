// Compute-isolated PLIC timing after the paper's GPU benchmark (Sec. 2.6.2,
// Table 3): one normal per thread, L fill levels in series, round trip
// through the forward volume; the blank run swaps the inversion for
// d0 = V0 - 1/2.  One problem per thread, as in the paper's kernels.
#include <hip/hip_runtime.h>

#include "../../include/plic_bench.h"
#include "plic_host.hpp"
#include "plic_math.hpp"

namespace plic {
namespace {

constexpr int kBenchBlock = 256;

template <int SOLVER, bool BLANK>
__global__ __launch_bounds__(kBenchBlock) void k_isolated(const float* __restrict__ nx, const float* __restrict__ ny,
                                                          const float* __restrict__ nz, int64_t count, int L,
                                                          float* __restrict__ err) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBenchBlock + threadIdx.x;
    if (i >= count) return;
    const float a = nx[i], b = ny[i], c = nz[i];
    const float last = static_cast<float>(L - 1);
    float e = 0.0f;
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
        const float V0 = static_cast<float>(j) / last;          // exact 0 and 1 at the ends
        const float d0 = BLANK ? V0 - 0.5f : offset<SOLVER, float, float>(a, b, c, V0);
        e += fabsf(volume<float>(a, b, c, d0) - V0);
    }
    err[i] = e;
}

template <int SOLVER>
void launch_isolated(bool blank, const float* nx, const float* ny, const float* nz, int64_t count, int L,
                     float* err, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((count + kBenchBlock - 1) / kBenchBlock)), block(kBenchBlock);
    if (blank)
        hipLaunchKernelGGL((k_isolated<SOLVER, true>), grid, block, 0, st, nx, ny, nz, count, L, err);
    else
        hipLaunchKernelGGL((k_isolated<SOLVER, false>), grid, block, 0, st, nx, ny, nz, count, L, err);
}

}  // namespace
}  // namespace plic

using namespace plic;

extern "C" int plic_bench_isolated_f32(const float* nx, const float* ny, const float* nz, int64_t count, int L,
                                       int solver, int blank, float* err, void* stream) {
    if (count < 0 || L < 2 || !valid_solver(solver) || (blank != 0 && blank != 1)) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) || !valid_array(err, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(float);
    if (overlap(err, nb, nx, nb) || overlap(err, nb, ny, nb) || overlap(err, nb, nz, nb)) return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    if (count > (int64_t(1) << 31)) return PLIC_EINVAL;                   // grid: 32-bit work-item count
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (solver) {
        case kSZ: launch_isolated<kSZ>(blank, nx, ny, nz, count, L, err, st); break;
        case kNewton: launch_isolated<kNewton>(blank, nx, ny, nz, count, L, err, st); break;
        case kNested: launch_isolated<kNested>(blank, nx, ny, nz, count, L, err, st); break;
        case kKawano: launch_isolated<kKawano>(blank, nx, ny, nz, count, L, err, st); break;
        default: launch_isolated<kAnalytic>(blank, nx, ny, nz, count, L, err, st); break;
    }
    return launch_status();
}
