// Host-side helpers shared by the C-ABI entry points: argument validation,
// launch error capture.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/plic.h"

namespace plic {

// hipError_t of the last PLIC_EHIP returned on this thread
void set_last_hip_error(int e);

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

template <class T>
inline bool valid_array(const T* p, int64_t count) {
    return count == 0 || (p != nullptr && aligned(p, sizeof(T)));
}

// [a, a + na) and [b, b + nb) (bytes) overlap
inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

inline bool valid_solver(int s) { return s >= PLIC_ANALYTIC && s <= PLIC_SZ_KAWANO; }
// the curvature takes the paper's four solvers, not Kawano's unoptimized SZ
inline bool valid_curvature_solver(int s) { return s >= PLIC_ANALYTIC && s <= PLIC_NESTED; }
inline bool valid_precision(int p) { return p >= PLIC_FP32 && p <= PLIC_FP64; }
inline bool valid_normal(int n) { return n == PLIC_NORMAL_PY || n == PLIC_NORMAL_CM; }

// check the launch that was just enqueued
inline int launch_status() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_hip_error(static_cast<int>(e));
        return PLIC_EHIP;
    }
    return PLIC_OK;
}

}  // namespace plic
