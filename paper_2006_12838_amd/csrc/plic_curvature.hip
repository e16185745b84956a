// PLIC curvature of a VoF fill-level lattice on gfx950 (Sec. 5.1-5.2 and
// Appendix B of Lehmann & Gekle, arXiv 2006.12838), forward and backward.
//
// Layout: phi, kappa, grad_kappa, grad_phi are X*Y*Z floats, x fastest.
// Both kernels are fused tile kernels: a workgroup owns a 64x4x4 tile, stages
// the tile plus a halo of fill levels in LDS, writes the zeros of every
// non-interface cell, and computes the interface cells of the tile from LDS.
// The interface is one cell thick (about 0.2 % of a 256^3 sphere lattice), so
// the kernels stream at HBM speed over the bulk and spend their arithmetic in
// the few tiles the interface crosses.  Workgroups are mapped to tiles so that
// each XCD (own L2) works on one contiguous slab and the halo re-reads of
// neighbouring tiles hit in its L2.
#include <hip/hip_runtime.h>

#include "plic_host.hpp"
#include "plic_math.hpp"

namespace plic {
namespace {

constexpr int TX = 64, TY = 4, TZ = 4;       // tile
constexpr int kTile = TX * TY * TZ;           // 1024 cells
constexpr int kThreads = 256;                 // 4 wave64, 4 cells per thread
constexpr int kCellsPerThread = kTile / kThreads;

// fixed auxiliary vector r of Sec. 5.2 (non-collinear with the normal)
constexpr double kR0 = 0.56270900, kR1 = 0.32704452, kR2 = 0.75921047;

// Workgroup -> tile: XCD k (workgroups dispatched round-robin, b % 8) takes a
// contiguous run of tiles; a ragged tail keeps the identity mapping.
__device__ __forceinline__ int tile_of_block(int b, int nb) {
    const int q = nb >> 3;
    return b < (q << 3) ? (b & 7) * q + (b >> 3) : b;
}

// neighbour q = (dz+1)*9 + (dy+1)*3 + (dx+1); centre q = 13
__host__ __device__ constexpr int q_dx(int q) { return q % 3 - 1; }
__host__ __device__ constexpr int q_dy(int q) { return (q / 3) % 3 - 1; }
__host__ __device__ constexpr int q_dz(int q) { return q / 9 - 1; }

__device__ __forceinline__ bool is_iface(float p) { return p > 0.0f && p < 1.0f; }

// ---------------------------------------------------------------------------
// LDL^T factorisation and solve of the symmetric 5x5 normal equations
// (App. B.3).  The lower triangle of m holds M on entry and L on exit, the
// diagonal holds D.  Only the leading N = min(5, #points) parameters are
// fitted (reduced dimension, the rest stay 0); a pivot below pivot_rel times
// the largest diagonal entry of the leading block drops its parameter.
// ---------------------------------------------------------------------------
template <class F>
__device__ __forceinline__ void ldlt_factor(F (&m)[5][5], int N, bool (&act)[5]) {
    F maxd = F(0);
#pragma unroll
    for (int j = 0; j < 5; ++j)
        if (j < N) maxd = M<F>::fmax(maxd, m[j][j]);
    const F tol = M<F>::pivot_rel * maxd;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        F dj = m[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= m[j][k] * m[j][k] * m[k][k];
        act[j] = (j < N) && (dj > tol) && (maxd > F(0));
        const F inv = act[j] ? F(1) / dj : F(0);
        m[j][j] = act[j] ? dj : F(0);
#pragma unroll
        for (int i = j + 1; i < 5; ++i) {
            F sij = m[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) sij -= m[i][k] * m[j][k] * m[k][k];
            m[i][j] = sij * inv;
        }
    }
}

template <class F>
__device__ __forceinline__ void ldlt_solve(const F (&m)[5][5], const bool (&act)[5], const F (&rhs)[5],
                                           F (&x)[5]) {
    F y[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        F t = rhs[j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= m[j][k] * y[k];
        y[j] = act[j] ? t : F(0);
    }
#pragma unroll
    for (int j = 4; j >= 0; --j) {
        F t = act[j] ? y[j] / m[j][j] : F(0);
#pragma unroll
        for (int i = j + 1; i < 5; ++i) t -= m[i][j] * x[i];
        x[j] = act[j] ? t : F(0);
    }
}

// ---------------------------------------------------------------------------
// Per-cell state of the forward computation, shared by both kernels.
// s: LDS fill levels, c: centre index, sy/sz: LDS strides.
// ---------------------------------------------------------------------------
template <class T, class F>
struct CellState {
    T n[3], bx[3], by[3], r[3];
    T ign, iun, D0;
    unsigned mask;          // interface neighbours (bit q)
    int npts;
    F m[5][5];              // factorised normal equations
    F a[5];                 // A, B, C, H, I
    bool act[5];
    bool valid;             // |g| large enough
};

template <int SOLVER, class T, class U, class F>
__device__ __forceinline__ void cell_forward(const float* __restrict__ s, int c, int sy, int sz,
                                             CellState<T, F>& st) {
    using mt = M<T>;
    // Parker-Youngs gradient (App. B.1): weights 4 / 2 / 1 for |e|^2 = 1 / 2 / 3
    T gx = T(0), gy = T(0), gz = T(0);
    unsigned mask = 0;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        if (q == 13) continue;
        constexpr int dummy = 0;
        (void)dummy;
        const int dx = q_dx(q), dy = q_dy(q), dz = q_dz(q);
        const float p = s[c + dz * sz + dy * sy + dx];
        const int e2 = dx * dx + dy * dy + dz * dz;
        const T w = T(e2 == 1 ? 4 : (e2 == 2 ? 2 : 1)) * T(p);
        gx += T(dx) * w;
        gy += T(dy) * w;
        gz += T(dz) * w;
        mask |= is_iface(p) ? (1u << q) : 0u;
    }
    st.mask = mask;
    for (int j = 0; j < 5; ++j) st.a[j] = F(0);
    const T gn2 = gx * gx + gy * gy + gz * gz;
    st.valid = gn2 >= T(1e-24);
    if (!st.valid) { st.npts = 0; return; }
    const T gn = mt::sqrt(gn2);
    st.ign = mt::rcp(gn);
    st.n[0] = -gx * st.ign; st.n[1] = -gy * st.ign; st.n[2] = -gz * st.ign;
    // local frame (Sec. 5.2): b_z = n, b_y = n x r / |n x r|, b_x = b_y x b_z
    st.r[0] = T(kR0); st.r[1] = T(kR1); st.r[2] = T(kR2);
    T u0 = st.n[1] * st.r[2] - st.n[2] * st.r[1];
    T u1 = st.n[2] * st.r[0] - st.n[0] * st.r[2];
    T u2 = st.n[0] * st.r[1] - st.n[1] * st.r[0];
    T un2 = u0 * u0 + u1 * u1 + u2 * u2;
    if (un2 < T(1e-12)) {            // n parallel to r: use (r_y, r_z, r_x)
        st.r[0] = T(kR1); st.r[1] = T(kR2); st.r[2] = T(kR0);
        u0 = st.n[1] * st.r[2] - st.n[2] * st.r[1];
        u1 = st.n[2] * st.r[0] - st.n[0] * st.r[2];
        u2 = st.n[0] * st.r[1] - st.n[1] * st.r[0];
        un2 = u0 * u0 + u1 * u1 + u2 * u2;
    }
    st.iun = mt::rcp(mt::sqrt(un2));
    st.by[0] = u0 * st.iun; st.by[1] = u1 * st.iun; st.by[2] = u2 * st.iun;
    st.bx[0] = st.by[1] * st.n[2] - st.by[2] * st.n[1];
    st.bx[1] = st.by[2] * st.n[0] - st.by[0] * st.n[2];
    st.bx[2] = st.by[0] * st.n[1] - st.by[1] * st.n[0];
    // PLIC points (eq. of the coordinate transformation, Sec. 5.2), centre normal for all
    st.D0 = offset<SOLVER, T, U>(st.n[0], st.n[1], st.n[2], T(s[c]));
    F (&m)[5][5] = st.m;
    F b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        b[i] = F(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) m[i][j] = F(0);
    }
    int npts = 0;
    unsigned mm = mask;
    while (mm) {
        const int q = __builtin_ctz(mm);
        mm &= mm - 1u;
        const int dx = q_dx(q), dy = q_dy(q), dz = q_dz(q);
        const T D = offset<SOLVER, T, U>(st.n[0], st.n[1], st.n[2], T(s[c + dz * sz + dy * sy + dx]));
        const T ex = T(dx), ey = T(dy), ez = T(dz);
        const F x = F(ex * st.bx[0] + ey * st.bx[1] + ez * st.bx[2]);
        const F y = F(ex * st.by[0] + ey * st.by[1] + ez * st.by[2]);
        const F z = F(ex * st.n[0] + ey * st.n[1] + ez * st.n[2] + (D - st.D0));
        const F Q[5] = {x * x, y * y, x * y, x, y};
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            b[i] += z * Q[i];
#pragma unroll
            for (int j = 0; j <= i; ++j) m[i][j] += Q[i] * Q[j];
        }
        ++npts;
    }
    st.npts = npts;
    ldlt_factor<F>(m, npts < 5 ? npts : 5, st.act);
    ldlt_solve<F>(m, st.act, b, st.a);
}

// mean curvature of the paraboloid at the origin (App. B.2), negated so that a
// fluid drop (normal pointing out of the fluid) is positive
template <class F>
__device__ __forceinline__ F kappa_of(const F (&a)[5]) {
    const F A = a[0], B = a[1], C = a[2], H = a[3], I = a[4];
    const F w = H * H + I * I + F(1);
    return -(A * (I * I + F(1)) + B * (H * H + F(1)) - C * H * I) / (w * M<F>::sqrt(w));
}

// ---------------------------------------------------------------------------
// Adjoint of one cell: out[q] = gk * d kappa / d phi_q for the 27 fill levels
// of the neighbourhood (interface mask, active fit parameters and PLIC cases
// held fixed).  Recomputes the forward state, then reverses: kappa -> fit
// coefficients -> lambda = M^-1 abar -> points -> (PLIC offsets: dd/dV = 1/A,
// dd/dn = polygon centroid) and (local frame) -> normal -> Parker-Youngs sums.
// out must hold 27 floats owned by this thread.
// ---------------------------------------------------------------------------
template <int SOLVER, class T, class U, class F>
__device__ __forceinline__ void cell_adjoint(const float* __restrict__ s, int c, int sy, int sz, float gk,
                                             float* out) {
#pragma unroll
    for (int q = 0; q < 27; ++q) out[q] = 0.0f;
    CellState<T, F> st;
    cell_forward<SOLVER, T, U, F>(s, c, sy, sz, st);
    if (!st.valid || gk == 0.0f) return;
    using mt = M<T>;
    // d kappa / d(A, B, C, H, I) with kappa = -(A(I^2+1) + B(H^2+1) - CHI) / W^(3/2)
    const F A = st.a[0], B = st.a[1], C = st.a[2], H = st.a[3], I = st.a[4];
    const F W = H * H + I * I + F(1);
    const F iW32 = F(1) / (W * M<F>::sqrt(W));
    const F num = A * (I * I + F(1)) + B * (H * H + F(1)) - C * H * I;
    const F g = -F(gk);
    F abar[5];
    abar[0] = g * (I * I + F(1)) * iW32;
    abar[1] = g * (H * H + F(1)) * iW32;
    abar[2] = g * (-H * I) * iW32;
    abar[3] = g * ((F(2) * B * H - C * I) * iW32 - F(3) * num * H * iW32 / W);
    abar[4] = g * ((F(2) * A * I - C * H) * iW32 - F(3) * num * I * iW32 / W);
#pragma unroll
    for (int j = 0; j < 5; ++j) abar[j] = st.act[j] ? abar[j] : F(0);
    F lam[5];
    ldlt_solve<F>(st.m, st.act, abar, lam);
    // reverse over the points: zbar = lam.Q, Qbar = lam (z - a.Q) - a (lam.Q)
    T bxb[3] = {T(0), T(0), T(0)}, byb[3] = {T(0), T(0), T(0)}, nb[3] = {T(0), T(0), T(0)};
    T sumz = T(0);
    unsigned mm = st.mask;
    while (mm) {
        const int q = __builtin_ctz(mm);
        mm &= mm - 1u;
        const int dx = q_dx(q), dy = q_dy(q), dz = q_dz(q);
        const T phq = T(s[c + dz * sz + dy * sy + dx]);
        const T D = offset<SOLVER, T, U>(st.n[0], st.n[1], st.n[2], phq);
        T cq[3];
        const T dv = offset_grad_from_d0<T>(st.n[0], st.n[1], st.n[2], phq, D, cq);
        const T ex = T(dx), ey = T(dy), ez = T(dz);
        const F x = F(ex * st.bx[0] + ey * st.bx[1] + ez * st.bx[2]);
        const F y = F(ex * st.by[0] + ey * st.by[1] + ez * st.by[2]);
        const F z = F(ex * st.n[0] + ey * st.n[1] + ez * st.n[2] + (D - st.D0));
        const F Q[5] = {x * x, y * y, x * y, x, y};
        F zb = F(0), aQ = F(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) { zb += lam[i] * Q[i]; aQ += st.a[i] * Q[i]; }
        F Qb[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) Qb[i] = lam[i] * (z - aQ) - st.a[i] * zb;
        const T xb = T(F(2) * x * Qb[0] + y * Qb[2] + Qb[3]);
        const T yb = T(F(2) * y * Qb[1] + x * Qb[2] + Qb[4]);
        const T zt = T(zb);
        bxb[0] += xb * ex; bxb[1] += xb * ey; bxb[2] += xb * ez;
        byb[0] += yb * ex; byb[1] += yb * ey; byb[2] += yb * ez;
        nb[0] += zt * (ex + cq[0]); nb[1] += zt * (ey + cq[1]); nb[2] += zt * (ez + cq[2]);
        out[q] += float(zt * dv);
        sumz += zt;
    }
    {   // centre offset D0 enters every z with a minus sign
        const T ph0 = T(s[c]);
        T c0[3];
        const T dv0 = offset_grad_from_d0<T>(st.n[0], st.n[1], st.n[2], ph0, st.D0, c0);
        out[13] += float(-sumz * dv0);
        nb[0] -= sumz * c0[0]; nb[1] -= sumz * c0[1]; nb[2] -= sumz * c0[2];
    }
    // b_x = b_y x n
    byb[0] += st.n[1] * bxb[2] - st.n[2] * bxb[1];
    byb[1] += st.n[2] * bxb[0] - st.n[0] * bxb[2];
    byb[2] += st.n[0] * bxb[1] - st.n[1] * bxb[0];
    nb[0] += bxb[1] * st.by[2] - bxb[2] * st.by[1];
    nb[1] += bxb[2] * st.by[0] - bxb[0] * st.by[2];
    nb[2] += bxb[0] * st.by[1] - bxb[1] * st.by[0];
    // b_y = u / |u|, u = n x r
    const T bdot = st.by[0] * byb[0] + st.by[1] * byb[1] + st.by[2] * byb[2];
    const T ub0 = (byb[0] - st.by[0] * bdot) * st.iun;
    const T ub1 = (byb[1] - st.by[1] * bdot) * st.iun;
    const T ub2 = (byb[2] - st.by[2] * bdot) * st.iun;
    nb[0] += st.r[1] * ub2 - st.r[2] * ub1;
    nb[1] += st.r[2] * ub0 - st.r[0] * ub2;
    nb[2] += st.r[0] * ub1 - st.r[1] * ub0;
    // n = -g / |g|
    const T ndot = st.n[0] * nb[0] + st.n[1] * nb[1] + st.n[2] * nb[2];
    const T gb0 = -(nb[0] - st.n[0] * ndot) * st.ign;
    const T gb1 = -(nb[1] - st.n[1] * ndot) * st.ign;
    const T gb2 = -(nb[2] - st.n[2] * ndot) * st.ign;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        if (q == 13) continue;
        const int dx = q_dx(q), dy = q_dy(q), dz = q_dz(q);
        const int e2 = dx * dx + dy * dy + dz * dz;
        const T w = T(e2 == 1 ? 4 : (e2 == 2 ? 2 : 1));
        out[q] += float(w * (T(dx) * gb0 + T(dy) * gb1 + T(dz) * gb2));
    }
    (void)mt::fabs(T(0));
}

// ---------------------------------------------------------------------------
// forward kernel: halo 1
// ---------------------------------------------------------------------------
constexpr int F_RX = TX + 2, F_RY = TY + 2, F_RZ = TZ + 2, F_REGION = F_RX * F_RY * F_RZ;

template <int SOLVER, class T, class U, class F>
__global__ __launch_bounds__(kThreads) void k_curv_fwd(const float* __restrict__ phi, float* __restrict__ kappa,
                                                        int X, int Y, int Z, int ntx, int nty) {
    __shared__ float s[F_REGION];
    __shared__ unsigned short list[kTile];
    __shared__ int nlist;
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    const int tid = threadIdx.x;
    if (tid == 0) nlist = 0;
    for (int i = tid; i < F_REGION; i += kThreads) {
        const int lx = i % F_RX, ly = (i / F_RX) % F_RY, lz = i / (F_RX * F_RY);
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly, gz = z0 - 1 + lz;
        float v = 0.0f;
        if (gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z)
            v = phi[(static_cast<int64_t>(gz) * Y + gy) * X + gx];
        s[i] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCellsPerThread; ++k) {
        const int cl = tid + k * kThreads;
        const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
        const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
        if (gx < X && gy < Y && gz < Z) {
            const float p = s[((cz + 1) * F_RY + (cy + 1)) * F_RX + (cx + 1)];
            const bool interior = gx >= 1 && gy >= 1 && gz >= 1 && gx <= X - 2 && gy <= Y - 2 && gz <= Z - 2;
            if (interior && is_iface(p)) list[atomicAdd(&nlist, 1)] = static_cast<unsigned short>(cl);
            else kappa[(static_cast<int64_t>(gz) * Y + gy) * X + gx] = 0.0f;
        }
    }
    __syncthreads();
    const int n = nlist;
    for (int i = tid; i < n; i += kThreads) {
        const int cl = list[i];
        const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
        CellState<T, F> st;
        cell_forward<SOLVER, T, U, F>(s, ((cz + 1) * F_RY + (cy + 1)) * F_RX + (cx + 1), F_RX, F_RX * F_RY, st);
        const float kv = st.valid ? float(kappa_of<F>(st.a)) : 0.0f;
        kappa[(static_cast<int64_t>(z0 + cz) * Y + (y0 + cy)) * X + (x0 + cx)] = kv;
    }
}

// ---------------------------------------------------------------------------
// backward kernel: halo 2.  Candidates are the interface cells of the tile
// grown by one cell (every cell whose neighbourhood touches the tile); they are
// listed in region order (ordered wave compaction), processed in chunks of
// kChunk, and each target cell of the tile gathers the contributions of its 27
// neighbours chunk by chunk in a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int B_RX = TX + 4, B_RY = TY + 4, B_RZ = TZ + 4, B_REGION = B_RX * B_RY * B_RZ;
constexpr int C_RX = TX + 2, C_RY = TY + 2, C_RZ = TZ + 2, C_REGION = C_RX * C_RY * C_RZ;
constexpr int kChunk = 128;
constexpr unsigned short kNoSlot = 0xFFFFu;

template <int SOLVER, class T, class U, class F>
__global__ __launch_bounds__(kThreads) void k_curv_bwd(const float* __restrict__ phi,
                                                        const float* __restrict__ gkap,
                                                        float* __restrict__ gphi, int X, int Y, int Z,
                                                        int ntx, int nty) {
    __shared__ float s[B_REGION];
    __shared__ unsigned short cand[C_REGION];
    __shared__ unsigned short slot[C_REGION];
    __shared__ float contrib[kChunk][27];
    __shared__ int wcount[kThreads / 64];
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < B_REGION; i += kThreads) {
        const int lx = i % B_RX, ly = (i / B_RX) % B_RY, lz = i / (B_RX * B_RY);
        const int gx = x0 - 2 + lx, gy = y0 - 2 + ly, gz = z0 - 2 + lz;
        float v = 0.0f;
        if (gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z)
            v = phi[(static_cast<int64_t>(gz) * Y + gy) * X + gx];
        s[i] = v;
    }
    for (int i = tid; i < C_REGION; i += kThreads) slot[i] = kNoSlot;
    __syncthreads();
    // ordered compaction of the candidate cells (region order)
    int ncand = 0;
    for (int base = 0; base < C_REGION; base += kThreads) {
        const int i = base + tid;
        bool is = false;
        if (i < C_REGION) {
            const int lx = i % C_RX, ly = (i / C_RX) % C_RY, lz = i / (C_RX * C_RY);
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly, gz = z0 - 1 + lz;
            const bool interior = gx >= 1 && gy >= 1 && gz >= 1 && gx <= X - 2 && gy <= Y - 2 && gz <= Z - 2;
            is = interior && is_iface(s[((lz + 1) * B_RY + (ly + 1)) * B_RX + (lx + 1)]);
        }
        const unsigned long long bal = __ballot(is);
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            before += w < wave ? wcount[w] : 0;
            total += wcount[w];
        }
        if (is) {
            const unsigned long long below = lane ? (bal & ((~0ull) >> (64 - lane))) : 0ull;
            cand[ncand + before + __popcll(below)] = static_cast<unsigned short>(i);
        }
        ncand += total;
        __syncthreads();
    }
    float acc[kCellsPerThread];
#pragma unroll
    for (int k = 0; k < kCellsPerThread; ++k) acc[k] = 0.0f;
    for (int c0 = 0; c0 < ncand; c0 += kChunk) {
        const int nc = min(kChunk, ncand - c0);
        for (int i = tid; i < nc; i += kThreads) slot[cand[c0 + i]] = static_cast<unsigned short>(i);
        for (int i = tid; i < nc; i += kThreads) {
            const int ci = cand[c0 + i];
            const int lx = ci % C_RX, ly = (ci / C_RX) % C_RY, lz = ci / (C_RX * C_RY);
            const float gk = gkap[(static_cast<int64_t>(z0 - 1 + lz) * Y + (y0 - 1 + ly)) * X + (x0 - 1 + lx)];
            cell_adjoint<SOLVER, T, U, F>(s, ((lz + 1) * B_RY + (ly + 1)) * B_RX + (lx + 1), B_RX,
                                          B_RX * B_RY, gk, contrib[i]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCellsPerThread; ++k) {
            const int cl = tid + k * kThreads;
            const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
            // the target sits at candidate-region coordinates (cx+1, cy+1, cz+1);
            // the neighbour owning offset q is at target - e_q
            float a = acc[k];
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                const int ci = ((cz + 1 - q_dz(q)) * C_RY + (cy + 1 - q_dy(q))) * C_RX + (cx + 1 - q_dx(q));
                const unsigned short sl = slot[ci];
                if (sl != kNoSlot) a += contrib[sl][q];
            }
            acc[k] = a;
        }
        __syncthreads();
        for (int i = tid; i < nc; i += kThreads) slot[cand[c0 + i]] = kNoSlot;
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kCellsPerThread; ++k) {
        const int cl = tid + k * kThreads;
        const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
        const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
        if (gx < X && gy < Y && gz < Z) gphi[(static_cast<int64_t>(gz) * Y + gy) * X + gx] = acc[k];
    }
}

// ---- dispatch -----------------------------------------------------------------
template <int SOLVER>
void launch_fwd(int precision, const float* phi, float* kappa, int X, int Y, int Z, int ntx, int nty,
                unsigned nblk, hipStream_t st) {
    if (precision == PLIC_FP32)
        hipLaunchKernelGGL((k_curv_fwd<SOLVER, float, float, float>), dim3(nblk), dim3(kThreads), 0, st, phi, kappa, X, Y, Z, ntx, nty);
    else if (precision == PLIC_MIXED)
        hipLaunchKernelGGL((k_curv_fwd<SOLVER, float, double, double>), dim3(nblk), dim3(kThreads), 0, st, phi, kappa, X, Y, Z, ntx, nty);
    else
        hipLaunchKernelGGL((k_curv_fwd<SOLVER, double, double, double>), dim3(nblk), dim3(kThreads), 0, st, phi, kappa, X, Y, Z, ntx, nty);
}

template <int SOLVER>
void launch_bwd(int precision, const float* phi, const float* gk, float* gp, int X, int Y, int Z, int ntx,
                int nty, unsigned nblk, hipStream_t st) {
    if (precision == PLIC_FP32)
        hipLaunchKernelGGL((k_curv_bwd<SOLVER, float, float, float>), dim3(nblk), dim3(kThreads), 0, st, phi, gk, gp, X, Y, Z, ntx, nty);
    else if (precision == PLIC_MIXED)
        hipLaunchKernelGGL((k_curv_bwd<SOLVER, float, double, double>), dim3(nblk), dim3(kThreads), 0, st, phi, gk, gp, X, Y, Z, ntx, nty);
    else
        hipLaunchKernelGGL((k_curv_bwd<SOLVER, double, double, double>), dim3(nblk), dim3(kThreads), 0, st, phi, gk, gp, X, Y, Z, ntx, nty);
}

// validates the lattice; returns PLIC_OK with *empty set when nothing to do
int check_lattice(int64_t X, int64_t Y, int64_t Z, bool* empty, int* ntx, int* nty, unsigned* nblk) {
    if (X < 0 || Y < 0 || Z < 0) return PLIC_EINVAL;
    *empty = X == 0 || Y == 0 || Z == 0;
    if (*empty) return PLIC_OK;
    const int64_t lim = 0x7fffffff;
    if (X > lim || Y > lim || Z > lim) return PLIC_EINVAL;
    if (X > (int64_t(1) << 62) / Y / Z) return PLIC_EINVAL;
    const int64_t tx = (X + TX - 1) / TX, ty = (Y + TY - 1) / TY, tz = (Z + TZ - 1) / TZ;
    if (tx > lim / ty || tx * ty > lim / tz) return PLIC_EINVAL;   // grid limit
    *ntx = static_cast<int>(tx);
    *nty = static_cast<int>(ty);
    *nblk = static_cast<unsigned>(tx * ty * tz);
    return PLIC_OK;
}

}  // namespace
}  // namespace plic

using namespace plic;

extern "C" {

int plic_curvature_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, float* kappa, int solver,
                       int precision, void* stream) {
    if (!valid_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    bool empty;
    int ntx = 0, nty = 0;
    unsigned nblk = 0;
    if (check_lattice(X, Y, Z, &empty, &ntx, &nty, &nblk) != PLIC_OK) return PLIC_EINVAL;
    const int64_t n = empty ? 0 : X * Y * Z;
    if (!valid_array(phi, n) || !valid_array(kappa, n)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(n) * sizeof(float);
    if (overlap(phi, nb, kappa, nb)) return PLIC_EINVAL;
    if (empty) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int x = static_cast<int>(X), y = static_cast<int>(Y), z = static_cast<int>(Z);
    switch (solver) {
        case kSZ: launch_fwd<kSZ>(precision, phi, kappa, x, y, z, ntx, nty, nblk, st); break;
        case kNewton: launch_fwd<kNewton>(precision, phi, kappa, x, y, z, ntx, nty, nblk, st); break;
        case kNested: launch_fwd<kNested>(precision, phi, kappa, x, y, z, ntx, nty, nblk, st); break;
        default: launch_fwd<kAnalytic>(precision, phi, kappa, x, y, z, ntx, nty, nblk, st); break;
    }
    return launch_status();
}

int plic_curvature_backward_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, const float* grad_kappa,
                                float* grad_phi, int solver, int precision, void* stream) {
    if (!valid_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    bool empty;
    int ntx = 0, nty = 0;
    unsigned nblk = 0;
    if (check_lattice(X, Y, Z, &empty, &ntx, &nty, &nblk) != PLIC_OK) return PLIC_EINVAL;
    const int64_t n = empty ? 0 : X * Y * Z;
    if (!valid_array(phi, n) || !valid_array(grad_kappa, n) || !valid_array(grad_phi, n)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(n) * sizeof(float);
    if (overlap(grad_phi, nb, phi, nb) || overlap(grad_phi, nb, grad_kappa, nb)) return PLIC_EINVAL;
    if (empty) return PLIC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int x = static_cast<int>(X), y = static_cast<int>(Y), z = static_cast<int>(Z);
    switch (solver) {
        case kSZ: launch_bwd<kSZ>(precision, phi, grad_kappa, grad_phi, x, y, z, ntx, nty, nblk, st); break;
        case kNewton: launch_bwd<kNewton>(precision, phi, grad_kappa, grad_phi, x, y, z, ntx, nty, nblk, st); break;
        case kNested: launch_bwd<kNested>(precision, phi, grad_kappa, grad_phi, x, y, z, ntx, nty, nblk, st); break;
        default: launch_bwd<kAnalytic>(precision, phi, grad_kappa, grad_phi, x, y, z, ntx, nty, nblk, st); break;
    }
    return launch_status();
}

}  // extern "C"
