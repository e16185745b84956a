// Batched PLIC kernels on gfx950: inversion (four solvers), forward volume and
// the backward (vector-Jacobian) pass of the inversion.
//
// Layout: structure of arrays in HBM (nx, ny, nz, V0 / d0), one problem per
// element.  Each thread handles VEC consecutive problems with 16-byte loads
// and stores per array (4 floats or 2 doubles), so a wavefront moves 1 KiB per
// array per access; VEC = 1 covers unaligned pointers, and the last thread's
// partial vector is loaded element by element.  One pass over HBM, no reuse.
// The inversion kernels settle the closed-form cases in registers and pack the
// rest (the cubic cases, about 40 % of uniformly random problems) densely in
// LDS before the iterative / trigonometric stage, so that stage runs on full
// wavefronts.
#include <hip/hip_runtime.h>

#include "plic_host.hpp"
#include "plic_math.hpp"

namespace plic {
namespace {

constexpr int kBlock = 256;
// The backward streams 5 input and 4 output arrays; workgroups of 512 keep
// twice the consecutive bytes of each array in flight per workgroup, which
// the memory system serves faster for this many streams (measured: a plain
// 5-read / 4-write copy and this kernel both about 6 % faster than with 256).
constexpr int kBwdBlock = 512;

// Input streams are read once: the loads carry the non-temporal hint (the
// "nt" bit), which keeps them from allocating in the caches as reusable data.
// Measured on a plain 4-read / 1-write stream of 2^26 floats per array:
// 0.84 of the HBM peak against 0.71 without the hint.
template <class S, int VEC> struct NVec;
template <> struct NVec<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NVec<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };

template <class S, int VEC>
__device__ __forceinline__ void load(const S* __restrict__ p, int64_t i, S (&v)[VEC]) {
    if constexpr (VEC == 1) {
        v[0] = __builtin_nontemporal_load(p + i);
    } else {
        using V = typename NVec<S, VEC>::type;
        const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(p + i));
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = t[k];
    }
}

// Outputs are written once and not read back by the kernel: non-temporal
// stores, so they do not sit in the last-level cache as dirty lines that the
// next kernel in the stream has to write back.
template <class S, int VEC>
__device__ __forceinline__ void store(S* __restrict__ p, int64_t i, const S (&v)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(v[0], p + i);
    } else {
        using V = typename NVec<S, VEC>::type;
        V t;
#pragma unroll
        for (int k = 0; k < VEC; ++k) t[k] = v[k];
        __builtin_nontemporal_store(t, reinterpret_cast<V*>(p + i));
    }
}

// Loads VEC consecutive elements at i, or those below count (others 0).
// FULL: the launch covers whole blocks only, no bounds checks.
template <class S, int VEC, bool FULL>
__device__ __forceinline__ void load_part(const S* p, int64_t i, int64_t count, S (&v)[VEC]) {
    if (FULL || i + VEC <= count) {
        load<S, VEC>(p, i, v);
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = i + k < count ? p[i + k] : S(0);
    }
}

template <class S, int VEC, bool FULL>
__device__ __forceinline__ void store_part(S* p, int64_t i, int64_t count, const S (&v)[VEC]) {
    if (FULL || i + VEC <= count) {
        store<S, VEC>(p, i, v);
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            if (i + k < count) p[i + k] = v[k];
    }
}

// LDS of one workgroup: its open problems packed densely.  The cubic stage
// replaces each problem's n1 with its root (the thread that reads an entry
// writes it), which keeps the FP32 kernels within 20 KiB of LDS: 8
// workgroups, 8 waves per SIMD.
template <class T, int VEC> struct PackLds {
    Open<T> q[kBlock * VEC];
    int count[VEC][kBlock / 64];
};

// Reduced offsets d (solver units) of the VEC problems of every thread of the
// workgroup; every thread must call it.  The closed-form cases finish in
// registers; the open ones are packed into LDS in (k, wave, lane) order and
// solved one per lane, so the iterative or trigonometric stage runs on full
// wavefronts instead of on the fraction of lanes that need it.  The result of
// each problem does not depend on the packing (the same stages run on the
// same values), so it equals the one-thread-per-problem offset().
template <int SOLVER, class T, class U, int VEC>
__device__ __forceinline__ void solve_packed(const Reduced<T> (&r)[VEC], const bool (&valid)[VEC], T (&d)[VEC],
                                             PackLds<T, VEC>& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Open<T> o[VEC];
    bool open[VEC];
    unsigned long long bal[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        open[k] = valid[k] && !closed_stage<SOLVER>(r[k], d[k], o[k]);
        bal[k] = __ballot(open[k]);
        if (lane == 0) sm.count[k][wave] = __popcll(bal[k]);
    }
    __syncthreads();
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int slot[VEC];
    int total = 0;
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            const int c = sm.count[k][w];
            before += w < wave ? c : 0;
            all += c;
        }
        slot[k] = total + before + __popcll(bal[k] & below);
        total += all;
        if (open[k]) sm.q[slot[k]] = o[k];
    }
    __syncthreads();
#pragma unroll 1
    for (int e = tid; e < total; e += kBlock) sm.q[e].n1 = cubic_stage<SOLVER, T, U>(sm.q[e]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VEC; ++k)
        if (open[k]) d[k] = sm.q[slot[k]].n1;
}

// S: storage type, T: bulk arithmetic, U: cubic-case arithmetic.  d0 may be
// V0 (each element is read and written by the same thread).  FULL launches
// cover whole blocks (kBlock * VEC problems each) and skip the bounds checks;
// the remainder goes to one checked block.
template <int SOLVER, class S, class T, class U, int VEC, bool FULL>
__global__ __launch_bounds__(kBlock) void k_offset(const S* __restrict__ nx, const S* __restrict__ ny,
                                                   const S* __restrict__ nz, const S* V0, S* d0,
                                                   int64_t count) {
    __shared__ PackLds<T, VEC> sm;
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) * VEC;
    S a[VEC], b[VEC], c[VEC], v[VEC];
    load_part<S, VEC, FULL>(nx, i, count, a); load_part<S, VEC, FULL>(ny, i, count, b);
    load_part<S, VEC, FULL>(nz, i, count, c); load_part<S, VEC, FULL>(V0, i, count, v);
    Reduced<T> r[VEC];
    bool valid[VEC];
    T d[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        r[k] = reduce(T(a[k]), T(b[k]), T(c[k]), T(v[k]));
        valid[k] = FULL || i + k < count;
        d[k] = T(0);
    }
    solve_packed<SOLVER, T, U, VEC>(r, valid, d, sm);
    S out[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k)
        out[k] = S(finish<SOLVER>(r[k], d[k], T(a[k]), T(b[k]), T(c[k]), T(v[k])));
    store_part<S, VEC, FULL>(d0, i, count, out);
}

template <class S, class T, int VEC>
__global__ __launch_bounds__(kBlock) void k_volume(const S* __restrict__ nx, const S* __restrict__ ny,
                                                   const S* __restrict__ nz, const S* d0, S* V0,
                                                   int64_t count) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) * VEC;
    if (i + VEC <= count) {
        S a[VEC], b[VEC], c[VEC], v[VEC], r[VEC];
        load<S, VEC>(nx, i, a); load<S, VEC>(ny, i, b); load<S, VEC>(nz, i, c); load<S, VEC>(d0, i, v);
#pragma unroll
        for (int k = 0; k < VEC; ++k) r[k] = S(volume<T>(T(a[k]), T(b[k]), T(c[k]), T(v[k])));
        store<S, VEC>(V0, i, r);
    } else {
        for (int64_t j = i; j < count; ++j)
            V0[j] = S(volume<T>(T(nx[j]), T(ny[j]), T(nz[j]), T(d0[j])));
    }
}

// plane-sphere intersection (Sec. 3): one input and one output array;
// OP 0 inverts (V0 -> d0), OP 1 evaluates the cap volume (d0 -> V0)
template <int OP, class S, class T, int VEC>
__global__ __launch_bounds__(kBlock) void k_sphere(const S* in, S* out, int64_t count) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) * VEC;
    if (i + VEC <= count) {
        S a[VEC], r[VEC];
        load<S, VEC>(in, i, a);
#pragma unroll
        for (int k = 0; k < VEC; ++k) r[k] = S(OP == 0 ? sphere_offset<T>(T(a[k])) : sphere_volume<T>(T(a[k])));
        store<S, VEC>(out, i, r);
    } else {
        for (int64_t j = i; j < count; ++j)
            out[j] = S(OP == 0 ? sphere_offset<T>(T(in[j])) : sphere_volume<T>(T(in[j])));
    }
}

// vector-Jacobian product of one problem given its offset d0
template <class T>
__device__ __forceinline__ void backward1(T nx, T ny, T nz, T V0, T d0, T gd, T& gx, T& gy, T& gz, T& gv) {
    T g[3];
    const T dv = offset_grad_from_d0<T>(nx, ny, nz, V0, d0, g);
    gx = gd * g[0];
    gy = gd * g[1];
    gz = gd * g[2];
    gv = gd * dv;
    if (__builtin_isnan(d0)) gx = gy = gz = gv = d0;
}

// The backward solves one problem per thread (no packing): its gradient stage
// is as long as the solve, and the packing's LDS and barriers cost more
// occupancy than they save there.  grad_d0 is loaded with the other inputs.
template <int SOLVER, class S, class T, class U, int VEC, bool FULL>
__global__ __launch_bounds__(kBwdBlock) void k_offset_bwd(const S* __restrict__ nx, const S* __restrict__ ny,
                                                       const S* __restrict__ nz, const S* __restrict__ V0,
                                                       const S* __restrict__ gd, S* __restrict__ gnx,
                                                       S* __restrict__ gny, S* __restrict__ gnz,
                                                       S* __restrict__ gV0, int64_t count) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * kBwdBlock + threadIdx.x) * VEC;
    S a[VEC], b[VEC], c[VEC], v[VEC], g[VEC];
    load_part<S, VEC, FULL>(nx, i, count, a); load_part<S, VEC, FULL>(ny, i, count, b);
    load_part<S, VEC, FULL>(nz, i, count, c); load_part<S, VEC, FULL>(V0, i, count, v);
    load_part<S, VEC, FULL>(gd, i, count, g);
    S ox[VEC], oy[VEC], oz[VEC], ov[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        const T d0 = offset<SOLVER, T, U>(T(a[k]), T(b[k]), T(c[k]), T(v[k]));
        T x, y, z, w;
        backward1<T>(T(a[k]), T(b[k]), T(c[k]), T(v[k]), d0, T(g[k]), x, y, z, w);
        ox[k] = S(x); oy[k] = S(y); oz[k] = S(z); ov[k] = S(w);
    }
    store_part<S, VEC, FULL>(gnx, i, count, ox); store_part<S, VEC, FULL>(gny, i, count, oy);
    store_part<S, VEC, FULL>(gnz, i, count, oz); store_part<S, VEC, FULL>(gV0, i, count, ov);
}

inline unsigned grid_for(int64_t count, int vec, int block = kBlock) {
    const int64_t per = static_cast<int64_t>(block) * vec;
    return static_cast<unsigned>((count + per - 1) / per);
}

template <class S> constexpr int kVec = 16 / sizeof(S);

// A dispatch holds at most 2^32 - 1 work-items; batches are launched in
// chunks of 2^30 problems (a multiple of every block's problem count).
constexpr int64_t kChunkProblems = int64_t(1) << 30;

template <class S, class T, int VEC>
void launch_volume_v(const S* nx, const S* ny, const S* nz, const S* d0, S* V0, int64_t count, hipStream_t st) {
    for (int64_t base = 0; base < count; base += kChunkProblems) {
        const int64_t n = count - base < kChunkProblems ? count - base : kChunkProblems;
        hipLaunchKernelGGL((k_volume<S, T, VEC>), dim3(grid_for(n, VEC)), dim3(kBlock), 0, st, nx + base, ny + base,
                           nz + base, d0 + base, V0 + base, n);
    }
}

// ---- dispatch ------------------------------------------------------------------
// whole blocks unchecked, then the remainder in one checked block
template <int OP, class S>
void launch_sphere(const S* in, S* out, int64_t count, hipStream_t st) {
    const bool vec = aligned(in, 16) && aligned(out, 16);
    for (int64_t base = 0; base < count; base += kChunkProblems) {
        const int64_t n = count - base < kChunkProblems ? count - base : kChunkProblems;
        if (vec)
            hipLaunchKernelGGL((k_sphere<OP, S, S, kVec<S>>), dim3(grid_for(n, kVec<S>)), dim3(kBlock), 0, st,
                               in + base, out + base, n);
        else
            hipLaunchKernelGGL((k_sphere<OP, S, S, 1>), dim3(grid_for(n, 1)), dim3(kBlock), 0, st, in + base,
                               out + base, n);
    }
}

template <int SOLVER, class S, class T, class U, int VEC>
void launch_offset_v(const S* nx, const S* ny, const S* nz, const S* V0, S* d0, int64_t count, hipStream_t st) {
    const int64_t per = static_cast<int64_t>(kBlock) * VEC, full = count / per * per, rem = count - full;
    for (int64_t base = 0; base < full; base += kChunkProblems) {
        const int64_t n = full - base < kChunkProblems ? full - base : kChunkProblems;
        hipLaunchKernelGGL((k_offset<SOLVER, S, T, U, VEC, true>), dim3(grid_for(n, VEC)), dim3(kBlock), 0, st,
                           nx + base, ny + base, nz + base, V0 + base, d0 + base, n);
    }
    if (rem)
        hipLaunchKernelGGL((k_offset<SOLVER, S, T, U, VEC, false>), dim3(1), dim3(kBlock), 0, st,
                           nx + full, ny + full, nz + full, V0 + full, d0 + full, rem);
}

template <int SOLVER, class S, class T, class U>
void launch_offset_t(const S* nx, const S* ny, const S* nz, const S* V0, S* d0, int64_t count,
                     bool vec, hipStream_t st) {
    if (vec) launch_offset_v<SOLVER, S, T, U, kVec<S>>(nx, ny, nz, V0, d0, count, st);
    else launch_offset_v<SOLVER, S, T, U, 1>(nx, ny, nz, V0, d0, count, st);
}

template <class S, class T, class U>
void launch_offset_s(int solver, const S* nx, const S* ny, const S* nz, const S* V0, S* d0,
                     int64_t count, bool vec, hipStream_t st) {
    switch (solver) {
        case kSZ: launch_offset_t<kSZ, S, T, U>(nx, ny, nz, V0, d0, count, vec, st); break;
        case kNewton: launch_offset_t<kNewton, S, T, U>(nx, ny, nz, V0, d0, count, vec, st); break;
        case kNested: launch_offset_t<kNested, S, T, U>(nx, ny, nz, V0, d0, count, vec, st); break;
        case kKawano: launch_offset_t<kKawano, S, T, U>(nx, ny, nz, V0, d0, count, vec, st); break;
        default: launch_offset_t<kAnalytic, S, T, U>(nx, ny, nz, V0, d0, count, vec, st); break;
    }
}

template <int SOLVER, class S, class T, class U, int VEC>
void launch_bwd_v(const S* nx, const S* ny, const S* nz, const S* V0, const S* gd, S* gx, S* gy, S* gz, S* gv,
                  int64_t count, hipStream_t st) {
    const int64_t per = static_cast<int64_t>(kBwdBlock) * VEC, full = count / per * per, rem = count - full;
    for (int64_t base = 0; base < full; base += kChunkProblems) {
        const int64_t n = full - base < kChunkProblems ? full - base : kChunkProblems;
        hipLaunchKernelGGL((k_offset_bwd<SOLVER, S, T, U, VEC, true>), dim3(grid_for(n, VEC, kBwdBlock)), dim3(kBwdBlock), 0,
                           st, nx + base, ny + base, nz + base, V0 + base, gd + base, gx + base, gy + base, gz + base,
                           gv + base, n);
    }
    if (rem)
        hipLaunchKernelGGL((k_offset_bwd<SOLVER, S, T, U, VEC, false>), dim3(1), dim3(kBwdBlock), 0, st,
                           nx + full, ny + full, nz + full, V0 + full, gd + full, gx + full, gy + full, gz + full,
                           gv + full, rem);
}

template <int SOLVER, class S, class T, class U>
void launch_bwd_t(const S* nx, const S* ny, const S* nz, const S* V0, const S* gd, S* gx, S* gy,
                  S* gz, S* gv, int64_t count, bool vec, hipStream_t st) {
    if (vec) launch_bwd_v<SOLVER, S, T, U, kVec<S>>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, st);
    else launch_bwd_v<SOLVER, S, T, U, 1>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, st);
}

template <class S, class T, class U>
void launch_bwd_s(int solver, const S* nx, const S* ny, const S* nz, const S* V0, const S* gd, S* gx,
                  S* gy, S* gz, S* gv, int64_t count, bool vec, hipStream_t st) {
    switch (solver) {
        case kSZ: launch_bwd_t<kSZ, S, T, U>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, vec, st); break;
        case kNewton: launch_bwd_t<kNewton, S, T, U>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, vec, st); break;
        case kNested: launch_bwd_t<kNested, S, T, U>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, vec, st); break;
        case kKawano: launch_bwd_t<kKawano, S, T, U>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, vec, st); break;
        default: launch_bwd_t<kAnalytic, S, T, U>(nx, ny, nz, V0, gd, gx, gy, gz, gv, count, vec, st); break;
    }
}

template <class S>
bool all_aligned16(std::initializer_list<const void*> ps) {
    for (const void* p : ps)
        if (!aligned(p, 16)) return false;
    return true;
}

// plane-sphere entry points: in and out may be the same array (each element
// is read and written by the same thread); otherwise they must not overlap
template <int OP, class S>
int sphere_entry(const S* in, S* out, int64_t count, void* stream) {
    if (count < 0 || !valid_array(in, count) || !valid_array(out, count)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(S);
    if (static_cast<const void*>(in) != static_cast<const void*>(out) && overlap(in, nb, out, nb)) return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    launch_sphere<OP, S>(in, out, count, static_cast<hipStream_t>(stream));
    return launch_status();
}

}  // namespace
}  // namespace plic

using namespace plic;

extern "C" {

int plic_offset_f32(const float* nx, const float* ny, const float* nz, const float* V0, float* d0,
                    int64_t count, int solver, int precision, void* stream) {
    if (count < 0 || !valid_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) ||
        !valid_array(V0, count) || !valid_array(d0, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(float);
    if ((overlap(d0, nb, nx, nb) || overlap(d0, nb, ny, nb) || overlap(d0, nb, nz, nb) ||
         overlap(d0, nb, V0, nb)) && d0 != V0)
        return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = all_aligned16<float>({nx, ny, nz, V0, d0});
    if (precision == PLIC_FP32) launch_offset_s<float, float, float>(solver, nx, ny, nz, V0, d0, count, vec, st);
    else if (precision == PLIC_MIXED) launch_offset_s<float, float, double>(solver, nx, ny, nz, V0, d0, count, vec, st);
    else launch_offset_s<float, double, double>(solver, nx, ny, nz, V0, d0, count, vec, st);
    return launch_status();
}

int plic_offset_f64(const double* nx, const double* ny, const double* nz, const double* V0, double* d0,
                    int64_t count, int solver, void* stream) {
    if (count < 0 || !valid_solver(solver)) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) ||
        !valid_array(V0, count) || !valid_array(d0, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(double);
    if ((overlap(d0, nb, nx, nb) || overlap(d0, nb, ny, nb) || overlap(d0, nb, nz, nb) ||
         overlap(d0, nb, V0, nb)) && d0 != V0)
        return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = all_aligned16<double>({nx, ny, nz, V0, d0});
    launch_offset_s<double, double, double>(solver, nx, ny, nz, V0, d0, count, vec, st);
    return launch_status();
}

int plic_volume_f32(const float* nx, const float* ny, const float* nz, const float* d0, float* V0,
                    int64_t count, int precision, void* stream) {
    if (count < 0 || !valid_precision(precision)) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) ||
        !valid_array(d0, count) || !valid_array(V0, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(float);
    if ((overlap(V0, nb, nx, nb) || overlap(V0, nb, ny, nb) || overlap(V0, nb, nz, nb) ||
         overlap(V0, nb, d0, nb)) && V0 != d0)
        return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = all_aligned16<float>({nx, ny, nz, d0, V0});
    if (precision == PLIC_FP64) {
        if (vec) launch_volume_v<float, double, 4>(nx, ny, nz, d0, V0, count, st);
        else launch_volume_v<float, double, 1>(nx, ny, nz, d0, V0, count, st);
    } else {
        if (vec) launch_volume_v<float, float, 4>(nx, ny, nz, d0, V0, count, st);
        else launch_volume_v<float, float, 1>(nx, ny, nz, d0, V0, count, st);
    }
    return launch_status();
}

int plic_volume_f64(const double* nx, const double* ny, const double* nz, const double* d0, double* V0,
                    int64_t count, void* stream) {
    if (count < 0) return PLIC_EINVAL;
    if (!valid_array(nx, count) || !valid_array(ny, count) || !valid_array(nz, count) ||
        !valid_array(d0, count) || !valid_array(V0, count))
        return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(double);
    if ((overlap(V0, nb, nx, nb) || overlap(V0, nb, ny, nb) || overlap(V0, nb, nz, nb) ||
         overlap(V0, nb, d0, nb)) && V0 != d0)
        return PLIC_EINVAL;
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (all_aligned16<double>({nx, ny, nz, d0, V0})) launch_volume_v<double, double, 2>(nx, ny, nz, d0, V0, count, st);
    else launch_volume_v<double, double, 1>(nx, ny, nz, d0, V0, count, st);
    return launch_status();
}

int plic_offset_backward_f32(const float* nx, const float* ny, const float* nz, const float* V0,
                             const float* grad_d0, float* grad_nx, float* grad_ny, float* grad_nz,
                             float* grad_V0, int64_t count, int solver, int precision, void* stream) {
    if (count < 0 || !valid_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    const float* ins[5] = {nx, ny, nz, V0, grad_d0};
    float* outs[4] = {grad_nx, grad_ny, grad_nz, grad_V0};
    for (const float* p : ins) if (!valid_array(p, count)) return PLIC_EINVAL;
    for (float* p : outs) if (!valid_array(p, count)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(float);
    for (int a = 0; a < 4; ++a) {
        for (const float* p : ins) if (overlap(outs[a], nb, p, nb)) return PLIC_EINVAL;
        for (int b = a + 1; b < 4; ++b) if (overlap(outs[a], nb, outs[b], nb)) return PLIC_EINVAL;
    }
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = all_aligned16<float>({nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0});
    if (precision == PLIC_FP32)
        launch_bwd_s<float, float, float>(solver, nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0, count, vec, st);
    else if (precision == PLIC_MIXED)
        launch_bwd_s<float, float, double>(solver, nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0, count, vec, st);
    else
        launch_bwd_s<float, double, double>(solver, nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0, count, vec, st);
    return launch_status();
}

int plic_offset_backward_f64(const double* nx, const double* ny, const double* nz, const double* V0,
                             const double* grad_d0, double* grad_nx, double* grad_ny, double* grad_nz,
                             double* grad_V0, int64_t count, int solver, void* stream) {
    if (count < 0 || !valid_solver(solver)) return PLIC_EINVAL;
    const double* ins[5] = {nx, ny, nz, V0, grad_d0};
    double* outs[4] = {grad_nx, grad_ny, grad_nz, grad_V0};
    for (const double* p : ins) if (!valid_array(p, count)) return PLIC_EINVAL;
    for (double* p : outs) if (!valid_array(p, count)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(count) * sizeof(double);
    for (int a = 0; a < 4; ++a) {
        for (const double* p : ins) if (overlap(outs[a], nb, p, nb)) return PLIC_EINVAL;
        for (int b = a + 1; b < 4; ++b) if (overlap(outs[a], nb, outs[b], nb)) return PLIC_EINVAL;
    }
    if (count == 0) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = all_aligned16<double>({nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0});
    launch_bwd_s<double, double, double>(solver, nx, ny, nz, V0, grad_d0, grad_nx, grad_ny, grad_nz, grad_V0, count, vec, st);
    return launch_status();
}


int plic_sphere_offset_f32(const float* V0, float* d0, int64_t count, void* stream) {
    return sphere_entry<0, float>(V0, d0, count, stream);
}
int plic_sphere_offset_f64(const double* V0, double* d0, int64_t count, void* stream) {
    return sphere_entry<0, double>(V0, d0, count, stream);
}
int plic_sphere_volume_f32(const float* d0, float* V0, int64_t count, void* stream) {
    return sphere_entry<1, float>(d0, V0, count, stream);
}
int plic_sphere_volume_f64(const double* d0, double* V0, int64_t count, void* stream) {
    return sphere_entry<1, double>(d0, V0, count, stream);
}

}  // extern "C"
