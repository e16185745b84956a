// PLIC curvature of a VoF fill-level lattice on gfx950 (Sec. 4.1-4.2 and
// Appendix B of Lehmann & Gekle, arXiv 2006.12838), forward and backward.
//
// Layout: phi, kappa, grad_kappa, grad_phi are X*Y*Z floats, x fastest.  The
// lattice is cut into 64x4x4 tiles.  A call runs:
//  1. a one-thread kernel that zeroes the work-list counters in the workspace
//     (a kernel, not a memset, so the call can be captured in a graph);
//  2. a streaming scan over the whole lattice (float4 loads and stores) that
//     writes the zero result everywhere, records each tile's interface bitmask
//     (0 < phi < 1, away from the outer layer) with its prefix counts, and
//     lists one work item per 8 interface cells of each tile; the backward
//     also records each tile's interface count;
//  3. a persistent kernel over the work list in which each interface cell is
//     computed by a group of 16 lanes: the group finds its cell from the
//     bitmask, stages its neighbourhood in LDS, and lane j takes slots j and
//     j + 16 of the 3x3x3 neighbourhood (their PLIC offsets and rows of the
//     normal equations; slot 26 is the centre).  Sums over the neighbours go
//     through a small LDS tile and are added in a fixed order, so results are
//     bitwise reproducible.
// The backward first assigns contribution rows by a prefix over the tiles'
// interface counts in tile order and lists the tiles next to the interface;
// the work items store each interface cell's 27 contributions in its row; a
// direct gather sums, for every cell next to the interface, its sources' rows
// in a fixed order; a fallback gather handles the tiles with a source whose
// row did not fit the workspace, recomputing those rows.
// The interface is one cell thick (about 0.2 % of a 256^3 sphere lattice), so
// the scan carries the HBM traffic and the list kernels the arithmetic.
//
// Floating-point contraction is limited to single expressions in this file,
// so the per-cell arithmetic gives the same bits in every kernel that inlines
// it (a contribution stored by the work items and one recomputed by the
// fallback gather are identical).
#pragma clang fp contract(on)

#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "plic_host.hpp"
#include "plic_math.hpp"

namespace plic {
namespace {

constexpr int TX = 64, TY = 4, TZ = 4;       // tile
constexpr int kTile = TX * TY * TZ;           // 1024 cells
constexpr int kThreads = 256;                 // 4 wave64
constexpr int kCellsPerThread = kTile / kThreads;
constexpr int kGroup = 32;                    // lanes per interface cell
constexpr int kGroups = kThreads / kGroup;    // 8 cells in flight per workgroup
constexpr int kPersistentBlocks = 2048;
constexpr int kFallbackBlocks = 256;            // one per CU of an MI355X

// fixed auxiliary vector r of Sec. 4.2 (non-collinear with the normal)
constexpr double kR0 = 0.56270900, kR1 = 0.32704452, kR2 = 0.75921047;

// neighbour q = (dz+1)*9 + (dy+1)*3 + (dx+1); centre q = 13
enum Normal : int { kNormalPY = PLIC_NORMAL_PY, kNormalCM = PLIC_NORMAL_CM };

__host__ __device__ constexpr int q_dx(int q) { return q % 3 - 1; }
__host__ __device__ constexpr int q_dy(int q) { return (q / 3) % 3 - 1; }
__host__ __device__ constexpr int q_dz(int q) { return q / 9 - 1; }

__device__ __forceinline__ bool is_iface(float p) { return p > 0.0f && p < 1.0f; }

// ---------------------------------------------------------------------------
// LDL^T factorisation and solve of the symmetric 5x5 normal equations
// (App. B.3).  The lower triangle of m holds M on entry and L on exit; dinv
// holds the reciprocals of D (0 for a dropped parameter), so that the solves
// (the fit and, in the backward, its adjoint) multiply instead of divide.
// Only the leading N = min(5, #points) parameters are fitted (reduced
// dimension, the rest stay 0); a pivot below pivot_rel times the largest
// diagonal entry of the leading block drops its parameter.
// ---------------------------------------------------------------------------
template <class F>
__device__ __forceinline__ void ldlt_factor(F (&m)[5][5], int N, bool (&act)[5], F (&dinv)[5]) {
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
        dinv[j] = inv;
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
__device__ __forceinline__ void ldlt_solve(const F (&m)[5][5], const bool (&act)[5], const F (&dinv)[5],
                                           const F (&rhs)[5], F (&x)[5]) {
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
        F t = y[j] * dinv[j];
#pragma unroll
        for (int i = j + 1; i < 5; ++i) t -= m[i][j] * x[i];
        x[j] = act[j] ? t : F(0);
    }
}

// mean curvature of the paraboloid at the origin (App. B.2), negated so that a
// fluid drop (normal pointing out of the fluid) is positive
template <class F>
__device__ __forceinline__ F kappa_of(const F (&a)[5]) {
    const F A = a[0], B = a[1], C = a[2], H = a[3], I = a[4];
    const F w = H * H + I * I + F(1);
    return -(A * (I * I + F(1)) + B * (H * H + F(1)) - C * H * I) / (w * M<F>::sqrt(w));
}

// lower-triangle index of the 5x5 normal matrix
__host__ __device__ constexpr int tri(int i, int k) { return i * (i + 1) / 2 + k; }

// weight of neighbour offset e in the fill-level gradient (App. B.1):
// Parker-Youngs 4 / 2 / 1 for |e|^2 = 1 / 2 / 3, centre of mass 1
template <int NRM>
__host__ __device__ constexpr int nrm_weight(int e2) {
    return NRM == kNormalCM ? 1 : (e2 == 1 ? 4 : (e2 == 2 ? 2 : 1));
}

// fill-level gradient of the 3^3 neighbourhood centred at LDS index c
template <int NRM, class T>
__device__ __forceinline__ void gradient27(const float* __restrict__ s, int c, int sy, int sz, T& gx, T& gy, T& gz) {
    gx = T(0); gy = T(0); gz = T(0);
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        if (q == 13) continue;
        const int e2 = q_dx(q) * q_dx(q) + q_dy(q) * q_dy(q) + q_dz(q) * q_dz(q);
        const T w = T(nrm_weight<NRM>(e2)) * T(s[c + q_dz(q) * sz + q_dy(q) * sy + q_dx(q)]);
        gx += T(q_dx(q)) * w;
        gy += T(q_dy(q)) * w;
        gz += T(q_dz(q)) * w;
    }
}

// ---------------------------------------------------------------------------
// One interface cell on a group of 16 lanes, four cells per wavefront.  The
// normal, the frame, the fit and kappa are computed once per group (every
// lane forms the same values), so per cell they cost half of what they would
// on 32 lanes; lane j owns the points of slots j and j + 16 (slot s < 26:
// neighbour q(s), the 26 offsets other than the centre; slot 26: the centre),
// so each lane inverts at most two PLIC problems.  The fit's sums run over
// the group's lanes in a fixed order (each lane's two points first), so every
// call gives the same bits.
// ---------------------------------------------------------------------------
constexpr int kQuad = 16;                       // lanes per interface cell
constexpr int kQuads = kThreads / kQuad;        // cells in flight per workgroup

template <class F, int COLS>
struct alignas(16) QuadLds {
    F stage[kQuad][COLS];
    F res[24];                                  // 20 sums, the centre offset at 20
};

// sum over the group's 16 lanes of each of the NV entries of row, through a
// [16][COLS] staging tile (lane k sums column k of each pass in lane order)
template <class F, int NV, int COLS>
__device__ __forceinline__ void quad_colsum(QuadLds<F, COLS>& L, int j, const F (&row)[NV], F (&sum)[NV]) {
#pragma unroll
    for (int c0 = 0; c0 < NV; c0 += COLS) {
#pragma unroll
        for (int k = 0; k < COLS; ++k)
            if (c0 + k < NV) L.stage[j][k] = row[c0 + k];
        __syncwarp();
        if (j < COLS && c0 + j < NV) {
            F acc = F(0);
#pragma unroll
            for (int l = 0; l < kQuad; ++l) acc += L.stage[l][j];
            L.res[c0 + j] = acc;
        }
        __syncwarp();
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) sum[k] = L.res[k];
    __syncwarp();
}

// this lane's point of slot q (x, y in the frame, z along n), zero when q is
// not an interface neighbour
template <class T, class F>
__device__ __forceinline__ void quad_point(int q, bool iface, T D, T D0, T bx0, T bx1, T bx2, T by0, T by1, T by2,
                                           T n0, T n1, T n2, F& x, F& y, F& z) {
    x = F(0); y = F(0); z = F(0);
    if (iface) {
        const T ex = T(q_dx(q)), ey = T(q_dy(q)), ez = T(q_dz(q));
        x = F(ex * bx0 + ey * bx1 + ez * bx2);
        y = F(ex * by0 + ey * by1 + ez * by2);
        z = F(ex * n0 + ey * n1 + ez * n2 + (D - D0));
    }
}

// neighbour-normal variant: the normal of slot q's plane, the neighbour's own
// -h / |h| (h its 3^3 fill-level gradient) when it is an interface cell whose
// 3^3 lies in the lattice and h does not vanish, else the centre normal that m
// holds on entry (the rule of the oracle's variant)
template <int NRM, class T>
__device__ __forceinline__ void own_normal(const float* __restrict__ s, int c, int sy, int sz, int q, bool iface,
                                           int gx0, int gy0, int gz0, int X, int Y, int Z, T (&m)[3], bool& own,
                                           T& ih_out) {
    const int dx = q_dx(q), dy = q_dy(q), dz = q_dz(q);
    const int ax = gx0 + dx, ay = gy0 + dy, az = gz0 + dz;
    const bool inside = ax >= 1 && ay >= 1 && az >= 1 && ax <= X - 2 && ay <= Y - 2 && az <= Z - 2;
    if (iface && inside) {
        T hx, hy, hz;
        gradient27<NRM, T>(s, c + dz * sz + dy * sy + dx, sy, sz, hx, hy, hz);
        const T h2 = hx * hx + hy * hy + hz * hz;
        if (h2 >= T(1e-24)) {
            const T ih = M<T>::rcp(M<T>::sqrt(h2));
            m[0] = -hx * ih; m[1] = -hy * ih; m[2] = -hz * ih;
            own = true;
            ih_out = ih;
        }
    }
}

// neighbour-normal variant: slot q's point, the foot of its own plane
// e + D m - D0 n, in the frame (zero when q is not an interface neighbour)
template <class T, class F>
__device__ __forceinline__ void quad_point_own(int q, bool iface, T D, T D0, const T (&m)[3], T bx0, T bx1, T bx2,
                                               T by0, T by1, T by2, T n0, T n1, T n2, F& x, F& y, F& z) {
    x = F(0); y = F(0); z = F(0);
    if (iface) {
        const T P0 = T(q_dx(q)) + D * m[0] - D0 * n0, P1 = T(q_dy(q)) + D * m[1] - D0 * n1,
                P2 = T(q_dz(q)) + D * m[2] - D0 * n2;
        x = F(P0 * bx0 + P1 * bx1 + P2 * bx2);
        y = F(P0 * by0 + P1 * by1 + P2 * by2);
        z = F(P0 * n0 + P1 * n1 + P2 * n2);
    }
}

// s: LDS fill levels, c: centre index, sy/sz: LDS strides, j: lane in the
// group (0..15), lane: lane in the wavefront.  Every lane of the group must
// call it; returns kappa (same bits on every lane).  With ADJ, also writes
// out[q] = gk * d kappa / d phi_q (q = 0..26) from the lane that owns q, with
// the interface mask, the PLIC cases and the active fit parameters held
// fixed.  With NBR (neighbour normals: each interface neighbour's point from
// its own normal m = -h / |h|; gx0.. and X.. locate the cell in the lattice),
// out[q] holds the derivative with every m held fixed, and the owner of slot t
// also writes out[27 + 3t .. 29 + 3t] = gk * d kappa / d h of its neighbour
// (zero where the neighbour keeps the centre normal); spreading that over the
// neighbour's 3^3 is left to the gathers.
template <int SOLVER, class T, class U, class F, bool ADJ, int NRM, int COLS, bool NBR = false>
__device__ __forceinline__ float quad_cell(const float* __restrict__ s, int c, int sy, int sz, int j, int lane,
                                           float gk, float* __restrict__ out, QuadLds<F, COLS>& L, int gx0 = 0,
                                           int gy0 = 0, int gz0 = 0, int X = 0, int Y = 0, int Z = 0) {
    using mt = M<T>;
    T gx, gy, gz;
    gradient27<NRM, T>(s, c, sy, sz, gx, gy, gz);
    const int qa = j < 13 ? j : j + 1;          // slot j: a neighbour
    const int sb = j + kQuad;                   // slot j + 16: a neighbour below 26, the centre at 26
    const bool nbb = sb < 26, centre = sb == 26;
    const int qb = nbb ? sb + 1 : 13;
    const float pa = s[c + q_dz(qa) * sz + q_dy(qa) * sy + q_dx(qa)];
    const float pb = (nbb || centre) ? s[c + q_dz(qb) * sz + q_dy(qb) * sy + q_dx(qb)] : 0.0f;
    const bool ia = is_iface(pa), ib = nbb && is_iface(pb);
    const int g0 = lane & 48;                   // this group's lanes in the wave
    const int npts = __popcll((__ballot(ia) >> g0) & 0xFFFFull) + __popcll((__ballot(ib) >> g0) & 0xFFFFull);
    const T gn2 = gx * gx + gy * gy + gz * gz;
    if (!(gn2 >= T(1e-24))) {                   // no usable normal: kappa = 0 (uniform per group)
        if constexpr (ADJ) {
            out[qa] = 0.0f;
            if (nbb || centre) out[qb] = 0.0f;
            if constexpr (NBR) {
                out[27 + 3 * j] = out[28 + 3 * j] = out[29 + 3 * j] = 0.0f;
                if (nbb) out[27 + 3 * sb] = out[28 + 3 * sb] = out[29 + 3 * sb] = 0.0f;
            }
        }
        return 0.0f;
    }
    const T ign = mt::rcp(mt::sqrt(gn2));
    const T n0 = -gx * ign, n1 = -gy * ign, n2 = -gz * ign;
    // local frame (Sec. 4.2): b_z = n, b_y = n x r / |n x r|, b_x = b_y x b_z
    T r0 = T(kR0), r1 = T(kR1), r2 = T(kR2);
    T u0 = n1 * r2 - n2 * r1, u1 = n2 * r0 - n0 * r2, u2 = n0 * r1 - n1 * r0;
    T un2 = u0 * u0 + u1 * u1 + u2 * u2;
    if (un2 < T(1e-12)) {
        r0 = T(kR1); r1 = T(kR2); r2 = T(kR0);
        u0 = n1 * r2 - n2 * r1; u1 = n2 * r0 - n0 * r2; u2 = n0 * r1 - n1 * r0;
        un2 = u0 * u0 + u1 * u1 + u2 * u2;
    }
    const T iun = mt::rcp(mt::sqrt(un2));
    const T by0 = u0 * iun, by1 = u1 * iun, by2 = u2 * iun;
    const T bx0 = by1 * n2 - by2 * n1, bx1 = by2 * n0 - by0 * n2, bx2 = by0 * n1 - by1 * n0;
    // PLIC offsets of the two slots with the centre normal (neighbour normals:
    // each interface neighbour with its own)
    T Da = T(0), Db = T(0), D0;
    F xa, ya, za, xb, yb, zb;
    T ma[3] = {n0, n1, n2}, mb[3] = {n0, n1, n2};     // neighbour normals: each slot's plane normal
    bool owna = false, ownb = false;                  // the slot's point uses its own normal
    T iha = T(0), ihb = T(0);                         // 1 / |h| of that normal's gradient
    if constexpr (NBR) {
        own_normal<NRM, T>(s, c, sy, sz, qa, ia, gx0, gy0, gz0, X, Y, Z, ma, owna, iha);
        own_normal<NRM, T>(s, c, sy, sz, qb, ib, gx0, gy0, gz0, X, Y, Z, mb, ownb, ihb);
        if (ia) Da = offset<SOLVER, T, U>(ma[0], ma[1], ma[2], T(pa));
        if (ib || centre) Db = offset<SOLVER, T, U>(mb[0], mb[1], mb[2], T(pb));
        if (centre) L.res[20] = F(Db);
        __syncwarp();
        D0 = T(L.res[20]);
        quad_point_own<T, F>(qa, ia, Da, D0, ma, bx0, bx1, bx2, by0, by1, by2, n0, n1, n2, xa, ya, za);
        quad_point_own<T, F>(qb, ib, Db, D0, mb, bx0, bx1, bx2, by0, by1, by2, n0, n1, n2, xb, yb, zb);
    } else {
        if (ia) Da = offset<SOLVER, T, U>(n0, n1, n2, T(pa));
        if (ib || centre) Db = offset<SOLVER, T, U>(n0, n1, n2, T(pb));
        if (centre) L.res[20] = F(Db);
        __syncwarp();
        D0 = T(L.res[20]);
        quad_point<T, F>(qa, ia, Da, D0, bx0, bx1, bx2, by0, by1, by2, n0, n1, n2, xa, ya, za);
        quad_point<T, F>(qb, ib, Db, D0, bx0, bx1, bx2, by0, by1, by2, n0, n1, n2, xb, yb, zb);
    }
    const F Qa[5] = {xa * xa, ya * ya, xa * ya, xa, ya}, Qb[5] = {xb * xb, yb * yb, xb * yb, xb, yb};
    F row[20], sum[20];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int k = 0; k <= i; ++k) row[tri(i, k)] = Qa[i] * Qa[k] + Qb[i] * Qb[k];
        row[15 + i] = za * Qa[i] + zb * Qb[i];
    }
    quad_colsum<F, 20, COLS>(L, j, row, sum);
    F m[5][5], b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        b[i] = sum[15 + i];
#pragma unroll
        for (int k = 0; k <= i; ++k) m[i][k] = sum[tri(i, k)];
    }
    bool act[5];
    F a[5], dinv[5];
    ldlt_factor<F>(m, npts < 5 ? npts : 5, act, dinv);
    // in mixed precision the adjoint's solve reads the factor back from LDS
    // (the staging tile is free until the adjoint's own sums): the same values,
    // and the registers that held them are free in between, so that adjoint
    // fits 4 waves per SIMD (in FP32 and FP64 the occupancy does not change and
    // the factor stays in registers)
    constexpr bool FAC = ADJ && sizeof(T) == 4 && sizeof(F) == 8;
    F* const fac = &L.stage[0][0];
    if constexpr (FAC) {
        if (j == 0) {
#pragma unroll
            for (int i = 0; i < 5; ++i) {
#pragma unroll
                for (int k = 0; k < i; ++k) fac[tri(i, k)] = m[i][k];
                fac[15 + i] = dinv[i];
            }
        }
    }
    ldlt_solve<F>(m, act, dinv, b, a);
    const float kappa = float(kappa_of<F>(a));
    if constexpr (ADJ) {
        // d kappa / d(A,B,C,H,I), kappa = -(A(I^2+1) + B(H^2+1) - CHI) / W^(3/2)
        const F A = a[0], B = a[1], C = a[2], H = a[3], I = a[4];
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
        for (int i = 0; i < 5; ++i) abar[i] = act[i] ? abar[i] : F(0);
        F lam[5];
        if constexpr (FAC) {
            __syncwarp();
            F lm[5][5], ld[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) {
#pragma unroll
                for (int k = 0; k < i; ++k) lm[i][k] = fac[tri(i, k)];
                lm[i][i] = F(0);                            // not read: the solve uses 1 / D
                ld[i] = fac[15 + i];
            }
            ldlt_solve<F>(lm, act, ld, abar, lam);           // M symmetric: lambda = M^-1 abar
        } else {
            ldlt_solve<F>(m, act, dinv, abar, lam);
        }
        // each slot's point: zbar = lam.Q, Qbar = lam (z - a.Q) - a (lam.Q); the
        // frame's adjoint rows of the two slots add up per lane
        T phia = T(0), phibb = T(0);
        T hba[3] = {T(0), T(0), T(0)}, hbb[3] = {T(0), T(0), T(0)};   // neighbour normals: adjoints of h
        F arow[10];
#pragma unroll
        for (int i = 0; i < 10; ++i) arow[i] = F(0);
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const bool on = sl == 0 ? ia : ib;
            if (!on) continue;
            const int q = sl == 0 ? qa : qb;
            const F x = sl == 0 ? xa : xb, y = sl == 0 ? ya : yb, z = sl == 0 ? za : zb;
            const T D = sl == 0 ? Da : Db;
            const float p = sl == 0 ? pa : pb;
            const F Q[5] = {x * x, y * y, x * y, x, y};
            F zq = F(0), aQ = F(0);
#pragma unroll
            for (int i = 0; i < 5; ++i) { zq += lam[i] * Q[i]; aQ += a[i] * Q[i]; }
            F Qbar[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) Qbar[i] = lam[i] * (z - aQ) - a[i] * zq;
            const T xbar = T(F(2) * x * Qbar[0] + y * Qbar[2] + Qbar[3]);
            const T ybar = T(F(2) * y * Qbar[1] + x * Qbar[2] + Qbar[4]);
            const T zt = T(zq);
            const T ex = T(q_dx(q)), ey = T(q_dy(q)), ez = T(q_dz(q));
            if constexpr (NBR) {
                // x = P.b_x, y = P.b_y, z = P.n with P = e + D m - D0 n, D = d0(phi_q, m)
                const T(&mm)[3] = sl == 0 ? ma : mb;
                const bool own = sl == 0 ? owna : ownb;
                const T P0 = ex + D * mm[0] - D0 * n0, P1 = ey + D * mm[1] - D0 * n1, P2 = ez + D * mm[2] - D0 * n2;
                const T Pb0 = xbar * bx0 + ybar * by0 + zt * n0;
                const T Pb1 = xbar * bx1 + ybar * by1 + zt * n1;
                const T Pb2 = xbar * bx2 + ybar * by2 + zt * n2;
                T cq[3];
                const T dv = offset_grad_from_d0<T>(mm[0], mm[1], mm[2], T(p), D, cq);   // 1/A, centroid for m
                const T Dbar = Pb0 * mm[0] + Pb1 * mm[1] + Pb2 * mm[2];
                const T mb0 = D * Pb0 + Dbar * cq[0], mb1 = D * Pb1 + Dbar * cq[1], mb2 = D * Pb2 + Dbar * cq[2];
                (sl == 0 ? phia : phibb) = Dbar * dv;
                arow[0] += F(xbar * P0); arow[1] += F(xbar * P1); arow[2] += F(xbar * P2);
                arow[3] += F(ybar * P0); arow[4] += F(ybar * P1); arow[5] += F(ybar * P2);
                // n enters through z = P.n, through -D0 n in P, and as m where the slot keeps it
                arow[6] += F(zt * P0 - D0 * Pb0 + (own ? T(0) : mb0));
                arow[7] += F(zt * P1 - D0 * Pb1 + (own ? T(0) : mb1));
                arow[8] += F(zt * P2 - D0 * Pb2 + (own ? T(0) : mb2));
                arow[9] += F(zt);
                if (own) {                                   // m = -h / |h|: the adjoint of h
                    const T ih = sl == 0 ? iha : ihb;
                    const T md = mm[0] * mb0 + mm[1] * mb1 + mm[2] * mb2;
                    T(&hb)[3] = sl == 0 ? hba : hbb;
                    hb[0] = -(mb0 - mm[0] * md) * ih;
                    hb[1] = -(mb1 - mm[1] * md) * ih;
                    hb[2] = -(mb2 - mm[2] * md) * ih;
                }
            } else {
                T cq[3];
                const T dv = offset_grad_from_d0<T>(n0, n1, n2, T(p), D, cq);   // 1/A, centroid
                (sl == 0 ? phia : phibb) = zt * dv;
                arow[0] += F(xbar * ex); arow[1] += F(xbar * ey); arow[2] += F(xbar * ez);
                arow[3] += F(ybar * ex); arow[4] += F(ybar * ey); arow[5] += F(ybar * ez);
                arow[6] += F(zt * (ex + cq[0])); arow[7] += F(zt * (ey + cq[1])); arow[8] += F(zt * (ez + cq[2]));
                arow[9] += F(zt);
            }
        }
        T dvc = T(0);
        if (centre) {
            T cc[3];
            dvc = offset_grad_from_d0<T>(n0, n1, n2, T(pb), Db, cc);
            L.res[21] = F(cc[0]); L.res[22] = F(cc[1]); L.res[23] = F(cc[2]);
        }
        F asum[10];
        quad_colsum<F, 10, COLS>(L, j, arow, asum);   // its barriers also publish res[21..23]
        const T c00 = T(L.res[21]), c01 = T(L.res[22]), c02 = T(L.res[23]);
        const T sbx0 = T(asum[0]), sbx1 = T(asum[1]), sbx2 = T(asum[2]);
        const T sz_ = T(asum[9]);
        // the centre offset D0 enters every z with a minus sign
        T nb0 = T(asum[6]) - sz_ * c00, nb1 = T(asum[7]) - sz_ * c01, nb2 = T(asum[8]) - sz_ * c02;
        // b_x = b_y x n
        const T yb0 = T(asum[3]) + (n1 * sbx2 - n2 * sbx1);
        const T yb1 = T(asum[4]) + (n2 * sbx0 - n0 * sbx2);
        const T yb2 = T(asum[5]) + (n0 * sbx1 - n1 * sbx0);
        nb0 += sbx1 * by2 - sbx2 * by1;
        nb1 += sbx2 * by0 - sbx0 * by2;
        nb2 += sbx0 * by1 - sbx1 * by0;
        // b_y = u / |u|, u = n x r
        const T bd = by0 * yb0 + by1 * yb1 + by2 * yb2;
        const T ub0 = (yb0 - by0 * bd) * iun, ub1 = (yb1 - by1 * bd) * iun, ub2 = (yb2 - by2 * bd) * iun;
        nb0 += r1 * ub2 - r2 * ub1;
        nb1 += r2 * ub0 - r0 * ub2;
        nb2 += r0 * ub1 - r1 * ub0;
        // n = -g / |g|
        const T nd = n0 * nb0 + n1 * nb1 + n2 * nb2;
        const T gb0 = -(nb0 - n0 * nd) * ign, gb1 = -(nb1 - n1 * nd) * ign, gb2 = -(nb2 - n2 * nd) * ign;
        {
            const T ex = T(q_dx(qa)), ey = T(q_dy(qa)), ez = T(q_dz(qa));
            const int e2 = q_dx(qa) * q_dx(qa) + q_dy(qa) * q_dy(qa) + q_dz(qa) * q_dz(qa);
            out[qa] = float(phia + T(nrm_weight<NRM>(e2)) * (ex * gb0 + ey * gb1 + ez * gb2));
        }
        if (nbb) {
            const T ex = T(q_dx(qb)), ey = T(q_dy(qb)), ez = T(q_dz(qb));
            const int e2 = q_dx(qb) * q_dx(qb) + q_dy(qb) * q_dy(qb) + q_dz(qb) * q_dz(qb);
            out[qb] = float(phibb + T(nrm_weight<NRM>(e2)) * (ex * gb0 + ey * gb1 + ez * gb2));
        }
        if (centre) out[13] = float(-sz_ * dvc);
        if constexpr (NBR) {
            // the adjoints of the slots' own fill-level gradients, gathered later at
            // those neighbours and spread over their 3^3 by the gradient's weights
            out[27 + 3 * j] = float(hba[0]); out[28 + 3 * j] = float(hba[1]); out[29 + 3 * j] = float(hba[2]);
            if (nbb) {
                out[27 + 3 * sb] = float(hbb[0]); out[28 + 3 * sb] = float(hbb[1]); out[29 + 3 * sb] = float(hbb[2]);
            }
        }
        __syncwarp();                              // res is reused by the next cell
    }
    return kappa;
}

// ---------------------------------------------------------------------------
// Fill levels of a box [x0-H, x0+TX+H) x ... into LDS, every load issued
// before the first store (out-of-lattice cells read as 0).
// ---------------------------------------------------------------------------
template <int RX, int RY, int RZ>
__device__ __forceinline__ void load_region(float* __restrict__ s, const float* __restrict__ phi, int gx0,
                                            int gy0, int gz0, int X, int Y, int Z) {
    constexpr int R = RX * RY * RZ, IT = (R + kThreads - 1) / kThreads;
    float v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * kThreads;
        const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
        const int gx = gx0 + lx, gy = gy0 + ly, gz = gz0 + lz;
        v[it] = 0.0f;
        if (i < R && gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z)
            v[it] = phi[(static_cast<int64_t>(gz) * Y + gy) * X + gx];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * kThreads;
        if (i < R) s[i] = v[it];
    }
}

// Ordered compaction: appends every i in [0, n) with pred(i) to out, in
// increasing i; returns the count (same on every thread).  Block-wide.
template <class Pred>
__device__ __forceinline__ int ordered_compact(int n, Pred pred, unsigned short* out, int* wcount) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int cnt = 0;
    for (int base = 0; base < n; base += kThreads) {
        const int i = base + tid;
        const bool is = i < n && pred(i);
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
            out[cnt + before + __popcll(below)] = static_cast<unsigned short>(i);
        }
        cnt += total;
        __syncthreads();
    }
    return cnt;
}

// ---------------------------------------------------------------------------
// Workspace (caller device memory, 4-byte aligned):
//   [0, 256)  header: [0] work items, [1] gather tiles, [2] overflow tiles,
//             [4..5] the call's interface-cell count (read by the status query)
//   flags     ntiles      interface cells in the tile (backward)
//   cbase     ntiles      first contribution row of the tile's interface cells
//                         (prefix of flags in tile order)
//   mask      32 ntiles   interface bit of each of the tile's 1024 cells
//   prefix    32 ntiles   set bits of mask before word w
//   items     128 ntiles  work items (tile << 7 | part), 8 interface cells each
//   tiles     ntiles      backward gather tiles
//   over      ntiles      row-prefix block totals, then the gather tiles with a
//                         source cell without a stored row
//   contrib   the rest:   27 floats per row (backward contributions)
// The fixed part (everything but contrib) is 784 bytes per tile.  The
// backward stores the 27 contributions of an interface cell in row
// cbase[tile] + rank when that row fits; cells beyond the capacity are
// recomputed by the fallback gather, so every workspace size >= the fixed part
// is correct and a larger one is faster.
// ---------------------------------------------------------------------------
constexpr int kPartCells = kGroups;           // interface cells per work item
constexpr int kMaxParts = kTile / kPartCells; // 128
constexpr int kWords = kTile / 32;            // mask words per tile
constexpr size_t kFixedPerTile = sizeof(unsigned) * (1 + 1 + kWords + kWords + kMaxParts + 1 + 1);
constexpr size_t kRowBytes = 27 * sizeof(float);
constexpr size_t kDefaultRowsPerTile = 16;    // contribution rows budgeted per tile by default
// rows are 32-bit indices: first rows saturate at kRowCap, so that a first
// row plus a rank (< kTile) never wraps and a saturated tile recomputes; the
// capacity is at most kRowLimit rows, so an entry's index row * 27 + q stays
// below 2^30 (a 32-bit byte offset from the store's base)
constexpr unsigned kRowCap = 0xF0000000u;
constexpr unsigned kRowLimit = (1u << 30) / 27u;
// The neighbour-normal variant's backward: a row holds the 27 contributions
// and, per neighbour, the adjoint of that neighbour's own fill-level gradient
// (26 x 3), followed in the workspace by one 3-vector per row, the sum of
// those adjoints at the row's cell
constexpr int kRowFloatsNbr = 27 + 26 * 3;
constexpr size_t kRowBytesNbr = (kRowFloatsNbr + 3) * sizeof(float);
constexpr unsigned kRowLimitNbr = (1u << 30) / kRowFloatsNbr;
// budgeted per tile by default: without a fallback a missing row is NaN, so
// the default leaves room for interfaces that cross a tile several times
constexpr size_t kDefaultRowsPerTileNbr = 64;

// header words: [0] work items, [1] gather tiles, [2] overflow tiles,
// [3] workgroup tickets of the one-pass row prefix
constexpr int kCounters = 4;
constexpr int kTicket = 3;

struct Workspace {
    unsigned* counter;  // header words (kCounters)
    unsigned* flags;
    unsigned* cbase;
    unsigned* mask;
    unsigned* prefix;
    unsigned* items;
    unsigned* tiles;
    unsigned* over;
    float* contrib;
    float* hbar;        // neighbour-normal backward: 3 floats per row
    unsigned rows;      // contribution capacity
};

// clears the header words and the first nstatus words of the overflow list
// (the one-pass row prefix publishes its workgroup totals there)
// (from header word first on: a backward that reuses a forward's records
// keeps its work item count, word 0)
__global__ void k_curv_zero(unsigned* counter, int first, unsigned* status, int nstatus) {
    const int t = threadIdx.x;
    if (t >= first && t < kCounters) counter[t] = 0u;
    for (int i = t; i < nstatus; i += blockDim.x) status[i] = 0u;
}

// ---------------------------------------------------------------------------
// 1. streaming scan: zero output everywhere; the tile's interface bitmask and
// the set bits before each of its words; one work item (tile << 7 | part) per
// kPartCells interface cells of the tile; the tile's interface count (its
// flag), from which the backward assigns contribution rows.  (A backward that
// reuses a forward's records runs no scan: its gather writes the zeros.)  Thread t handles 4 consecutive cells along x, which are the cells
// 4t .. 4t+3 of the tile in cell order (x fastest, then y, z).
// ---------------------------------------------------------------------------
template <bool VEC, bool FWD>
__global__ __launch_bounds__(kThreads) void k_curv_scan(const float* __restrict__ phi, float* __restrict__ out,
                                                        Workspace ws, int X, int Y, int Z, int ntx, int nty) {
    __shared__ int wsum[kThreads / 64];
    __shared__ unsigned smask[kWords];
    const int tile = blockIdx.x;
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    const int t = threadIdx.x;
    const int x = x0 + (t % 16) * 4, y = y0 + (t / 16) % TY, z = z0 + t / (16 * TY);
    if (t < kWords) smask[t] = 0u;
    unsigned nib = 0u;
    if (y < Y && z < Z) {
        const bool yz_in = y >= 1 && y <= Y - 2 && z >= 1 && z <= Z - 2;
        const int64_t row = (static_cast<int64_t>(z) * Y + y) * X;
        if (VEC && x + 4 <= X) {
            // a plain load: with the non-temporal hint this scan measured slower
            // (34 against 26 us at 256^3)
            const float4 v = *reinterpret_cast<const float4*>(phi + row + x);
            *reinterpret_cast<float4*>(out + row + x) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                nib |= (yz_in && x + k >= 1 && x + k <= X - 2 && is_iface(vv[k])) ? (1u << k) : 0u;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (x + k < X) {
                    const float v = phi[row + x + k];
                    out[row + x + k] = 0.0f;
                    nib |= (yz_in && x + k >= 1 && x + k <= X - 2 && is_iface(v)) ? (1u << k) : 0u;
                }
            }
        }
    }
    // block count of interface cells (wave butterflies, then 4 waves)
    int cnt = __popc(nib);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
    if ((t & 63) == 0) wsum[t >> 6] = cnt;
    __syncthreads();                                      // smask cleared
    if (nib) atomicOr(&smask[t / 8], nib << ((t % 8) * 4));
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) total += wsum[w];
    const unsigned parts = (total + kPartCells - 1) / kPartCells;
    if (t < 64) {                                         // the first wave writes the tile's records
        // mask words and the set bits before each (exclusive scan over lanes 0..31)
        const unsigned mw = t < kWords ? smask[t] : 0u, c = __popc(mw);
        unsigned incl = c;
#pragma unroll
        for (int d = 1; d < kWords; d <<= 1) {
            const unsigned o = __shfl_up(incl, d, 64);
            if (t >= d) incl += o;
        }
        if (t < kWords) {
            ws.mask[tile * kWords + t] = mw;
            ws.prefix[tile * kWords + t] = incl - c;
        }
        // the tile's interface count: the backward assigns rows from these,
        // and plic_curvature_status sums them (no shared counter here: every
        // atomic on one word serialises at the memory side)
        if (t == 0) ws.flags[tile] = static_cast<unsigned>(total);
        // only a tile with interface cells waits for an atomic's result (the
        // wait also covers the block's stores); parts is uniform per block
        if (parts) {
            unsigned base = 0u;
            if (t == 0) base = atomicAdd(ws.counter, parts);
            base = __shfl(base, 0, 64);
            for (unsigned p = static_cast<unsigned>(t); p < parts; p += 64u)
                ws.items[base + p] = (static_cast<unsigned>(tile) << 7) | p;
        }
    }
}

// Contribution rows in tile order: cbase[tile] = number of interface cells in
// the tiles before it (exclusive prefix of flags), saturated at kRowCap, so
// the cells that get a row for a given workspace size do not depend on the
// order in which the scan's blocks ran.  Two passes over workgroups of 256
// tiles: the first, with the gather list, writes each workgroup's local
// prefix and its total; the second adds the totals of the workgroups before
// it.  The totals live in the overflow list until the gather uses it.

// Gather list and the first prefix pass, one tile per thread.  The list holds
// every tile whose 3x3x3 tile neighbourhood has an interface cell (its cells
// can receive a contribution); its order does not affect any result.
// With ONEPASS (lattices of at most kOnePassBlocks workgroups of tiles) the
// workgroups also finish the prefix themselves: each takes a ticket, which
// orders it after every workgroup that took one before (those have started
// and never wait before they publish), publishes its total in the overflow
// list (cleared at the start of the call) with a ready bit, and adds up the
// totals of the workgroups before it, one per lane of its first wave, waiting
// for each to be published.  Otherwise the totals go to the overflow list for
// the second pass.
constexpr int kOnePassBlocks = 256;
constexpr unsigned kPublished = 0x80000000u;                   // totals are at most 256 * 1024

template <bool ONEPASS>
__global__ __launch_bounds__(kThreads) void k_curv_dilate(Workspace ws, int ntx, int nty, int ntz, int ntiles) {
    __shared__ unsigned wsum[kThreads / 64];
    __shared__ unsigned wact[kThreads / 64];
    __shared__ unsigned long long boff;
    __shared__ unsigned gbase;
    __shared__ int ticket;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int b = static_cast<int>(blockIdx.x);
    if constexpr (ONEPASS) {
        if (t == 0) ticket = static_cast<int>(atomicAdd(ws.counter + kTicket, 1u));
        __syncthreads();
        b = ticket;
    }
    const int tile = b * kThreads + t;
    bool act = false;
    unsigned c = 0u;
    if (tile < ntiles) {
        c = ws.flags[tile];
        const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int ax = tx + q_dx(q), ay = ty + q_dy(q), az = tz + q_dz(q);
            if (ax >= 0 && ax < ntx && ay >= 0 && ay < nty && az >= 0 && az < ntz)
                act |= ws.flags[(az * nty + ay) * ntx + ax] != 0u;
        }
    }
    unsigned incl = c;                                        // inclusive scan over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    const unsigned long long bal = __ballot(act);
    if (lane == 0) wact[wave] = static_cast<unsigned>(__popcll(bal));
    __syncthreads();
    unsigned woff = 0u, total = 0u, aoff = 0u, atotal = 0u;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        woff += w < wave ? wsum[w] : 0u;
        total += wsum[w];
        aoff += w < wave ? wact[w] : 0u;
        atotal += wact[w];
    }
    // the gather list: one atomic per workgroup (the atomics on one word are
    // served one at a time), taken after the total is published
    if constexpr (ONEPASS) {
        if (t == 0) {
            __hip_atomic_store(ws.over + b, total | kPublished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gbase = atotal ? atomicAdd(ws.counter + 1, atotal) : 0u;
        }
        if (wave == 0) {
            unsigned long long acc = 0ull;
            for (int p = lane; p < b; p += 64) {
                unsigned v;
                do {
                    v = __hip_atomic_load(ws.over + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while (!(v & kPublished));
                acc += v & ~kPublished;
            }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
            if (lane == 0) boff = acc;
        }
        __syncthreads();
        if (tile < ntiles) {
            const unsigned long long r = boff + woff + incl - c;
            ws.cbase[tile] = static_cast<unsigned>(r < kRowCap ? r : kRowCap);
        }
    } else {
        if (tile < ntiles) ws.cbase[tile] = woff + incl - c;
        if (t == 0) {
            ws.over[blockIdx.x] = total;                      // at most 256 * 1024 = 2^18
            gbase = atotal ? atomicAdd(ws.counter + 1, atotal) : 0u;
        }
        __syncthreads();
    }
    if (act) {
        const unsigned long long below = lane ? (bal & ((~0ull) >> (64 - lane))) : 0ull;
        ws.tiles[gbase + aoff + __popcll(below)] = static_cast<unsigned>(tile);
    }
}

// second prefix pass: workgroup b's offset is the sum of the totals of
// workgroups 0..b-1 (64-bit), added to its local prefixes with saturation
__global__ __launch_bounds__(kThreads) void k_curv_prefix(Workspace ws, int ntiles) {
    __shared__ unsigned long long part[kThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned long long acc = 0ull;
    for (int i = t; i < static_cast<int>(blockIdx.x); i += kThreads) acc += ws.over[i];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    unsigned long long off = 0ull;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) off += part[w];
    const int tile = blockIdx.x * kThreads + t;
    if (tile < ntiles) {
        const unsigned long long r = off + ws.cbase[tile];
        ws.cbase[tile] = static_cast<unsigned>(r < kRowCap ? r : kRowCap);
    }
}

// ---------------------------------------------------------------------------
// 2. work items: up to kPartCells interface cells of a tile, each cell on a
// group of 16 lanes (k_curv_quads; the neighbour-normal variant stages each
// cell's 5x5x5 neighbourhood, for each neighbour's own 3x3x3).  The group
// finds its cell, the i-th interface cell of the tile in cell order, from the
// tile's bitmask and prefix counts (two ballots), stages the cell's fill
// levels in LDS, and runs the cell.  Groups never wait for each other: no
// block barrier.  Forward: kappa.  Backward: the cell's contributions
// gk * d kappa / d phi_q into its contribution row (when it fits).
// ---------------------------------------------------------------------------

// Lattice position of the interface cell of rank i (in cell order) of a
// tile, found by the 32 lanes of a group together: lane j reads mask word j
// and the count of set bits before it.  False, for the whole group, when the
// tile has no more than i interface cells.
__device__ __forceinline__ bool tile_cell(const Workspace& ws, int tile, int i, int j, int half, int ntx, int nty,
                                          int& gx, int& gy, int& gz) {
    const unsigned mw = ws.mask[tile * kWords + j], pw = ws.prefix[tile * kWords + j];
    const int n = static_cast<int>(__shfl(pw + __popc(mw), kWords - 1, kGroup));
    if (i >= n) return false;
    const unsigned ui = static_cast<unsigned>(i);
    const unsigned in_word = static_cast<unsigned>(__ballot(pw <= ui && ui < pw + __popc(mw)) >> half);
    const int w = __ffs(static_cast<int>(in_word)) - 1;
    const unsigned word = __shfl(mw, w, kGroup);
    const unsigned k = ui - __shfl(pw, w, kGroup);
    const bool hit = ((word >> j) & 1u) && static_cast<unsigned>(__popc(word & ((1u << j) - 1u))) == k;
    const int b = __ffs(static_cast<int>(static_cast<unsigned>(__ballot(hit) >> half))) - 1;
    const int cl = w * 32 + b;
    gx = (tile % ntx) * TX + cl % TX;
    gy = ((tile / ntx) % nty) * TY + (cl / TX) % TY;
    gz = (tile / (ntx * nty)) * TZ + cl / (TX * TY);
    return true;
}

// threadIdx.x through an opaque move: what a loop derives from it is then
// recomputed in every iteration (a few ALU instructions) instead of being
// kept in registers across the loop, where it would spill
__device__ __forceinline__ int thread_index_per_iteration() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(static_cast<int>(threadIdx.x)));
    return t;
}

// The curvature without neighbour normals on groups of 16 lanes: a workgroup
// takes two work items at a time (its first two waves the first, the last two
// the second), each 32-lane half of a wave finds its two cells from the tile's
// bitmask, and each group of 16 stages its cell's 3x3x3 fill levels and runs
// quad_cell; the forward writes kappa, the backward (ADJ) the cell's
// contribution row when it fits the workspace.
// waves per SIMD, the most that compile without spilling: the forward 8
// (FP64: 4); the adjoint, which keeps two points' state per lane, 4 in FP32
// and mixed precision (3 with neighbour normals), in FP64 3 for the iterative
// solvers and 2 for the trigonometric ones and with neighbour normals
template <int SOLVER, class T, class U, bool ADJ, bool NBR>
constexpr int quad_waves() {
    if (!ADJ) return sizeof(T) == 4 ? 8 : 4;
    if (sizeof(U) == 4) return 4;                            // FP32
    if (sizeof(T) == 4) return NBR ? 3 : 4;                  // mixed
    return (!NBR && (SOLVER == kNewton || SOLVER == kNested)) ? 3 : 2;   // FP64
}

template <int SOLVER, class T, class U, class F, bool ADJ, int NRM, bool NBR>
__global__ __launch_bounds__(kThreads, (quad_waves<SOLVER, T, U, ADJ, NBR>())) void k_curv_quads(const float* __restrict__ phi,
                                                                                   const float* __restrict__ gkap,
                                                                                   float* __restrict__ kappa,
                                                                                   Workspace ws, int X, int Y, int Z,
                                                                                   int ntx, int nty) {
    constexpr int COLS = 10;                                 // 2 passes; 25 KiB of LDS with an FP64 fit
    // the cell's 3x3x3 fill levels (5x5x5 with neighbour normals)
    constexpr int H = NBR ? 2 : 1, W = 2 * H + 1, NB = W * W * W, C = (H * W + H) * W + H;
    __shared__ float nbh[kQuads][NB];
    __shared__ QuadLds<F, COLS> qlds[kQuads];
    const unsigned nitems = *static_cast<volatile unsigned*>(ws.counter);
    const unsigned npairs = (nitems + 1u) / 2u;
    for (unsigned pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
        const int tid = thread_index_per_iteration(), grp = tid / kQuad, j = tid % kQuad;
        const int lane = tid & 63, l32 = tid & 31, half = tid & 32;
        const unsigned item = 2u * pr + (tid >= kThreads / 2 ? 1u : 0u);
        if (item >= nitems) continue;                        // uniform per pair of waves
        const unsigned e = ws.items[item];
        const int tile = static_cast<int>(e >> 7), part = static_cast<int>(e & 127u);
        // the two ranks of this half-wave's groups among the tile's interface cells
        const unsigned mw = ws.mask[tile * kWords + l32], pw = ws.prefix[tile * kWords + l32];
        const unsigned n = __shfl(pw + __popc(mw), kWords - 1, 32);
        const unsigned i0 = static_cast<unsigned>(part * kPartCells + (grp % 8) / 2 * 2);
        int cl[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const unsigned ui = i0 + r < n ? i0 + r : n - 1u;    // n >= 1: the tile has an item
            const unsigned in_word = static_cast<unsigned>(__ballot(pw <= ui && ui < pw + __popc(mw)) >> half);
            const int w = __ffs(static_cast<int>(in_word)) - 1;
            const unsigned word = __shfl(mw, w, 32);
            const unsigned k = ui - __shfl(pw, w, 32);
            const bool hit = ((word >> l32) & 1u) && static_cast<unsigned>(__popc(word & ((1u << l32) - 1u))) == k;
            const int b = __ffs(static_cast<int>(static_cast<unsigned>(__ballot(hit) >> half))) - 1;
            cl[r] = w * 32 + b;
        }
        const unsigned ic = i0 + (grp & 1);
        if (ic >= n) continue;                               // uniform per group
        unsigned row = 0u;
        if constexpr (ADJ) {
            row = ws.cbase[tile] + ic;
            if (row >= ws.rows) continue;                    // uniform per group; the gather recomputes
        }
        const int c = (grp & 1) ? cl[1] : cl[0];
        const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
        const int gx = x0 + c % TX, gy = y0 + (c / TX) % TY, gz = z0 + c / (TX * TY);
        for (int t = j; t < NB; t += kQuad) {
            const int ax = gx + t % W - H, ay = gy + (t / W) % W - H, az = gz + t / (W * W) - H;
            nbh[grp][t] = (ax >= 0 && ax < X && ay >= 0 && ay < Y && az >= 0 && az < Z)
                              ? phi[(static_cast<int64_t>(az) * Y + ay) * X + ax] : 0.0f;
        }
        __syncwarp();
        const int64_t gi = (static_cast<int64_t>(gz) * Y + gy) * X + gx;
        if constexpr (ADJ) {
            constexpr int ROWF = NBR ? kRowFloatsNbr : 27;
            quad_cell<SOLVER, T, U, F, true, NRM, COLS, NBR>(nbh[grp], C, W, W * W, j, lane, gkap[gi],
                                                             ws.contrib + static_cast<size_t>(row) * ROWF, qlds[grp],
                                                             gx, gy, gz, X, Y, Z);
        } else {
            const float kv = quad_cell<SOLVER, T, U, F, false, NRM, COLS, NBR>(nbh[grp], C, W, W * W, j, lane, 0.0f,
                                                                               nullptr, qlds[grp], gx, gy, gz, X, Y,
                                                                               Z);
            if (j == 0) kappa[gi] = kv;
        }
        __syncwarp();                                        // nbh and qlds reused by the next pair
    }
}

// ---------------------------------------------------------------------------
// 3. backward gathers: every cell next to the interface adds the
// contributions of its interface neighbours in a fixed order (deterministic,
// no atomics).  The direct gather reads them from the stored rows; a tile with
// a source whose row did not fit goes to the overflow list, where the fallback
// gather copies the stored rows and recomputes the missing ones.
// ---------------------------------------------------------------------------
constexpr int B_RX = TX + 4, B_RY = TY + 4, B_RZ = TZ + 4;
constexpr int C_RX = TX + 2, C_RY = TY + 2, C_RZ = TZ + 2, C_REGION = C_RX * C_RY * C_RZ;
constexpr int kChunk = 128;
constexpr int kCopyBatch = 8;                 // contribution loads in flight per thread
constexpr unsigned short kNoSlot = 0xFFFFu;

// contribution row of an interior interface cell: cbase of its tile plus its
// rank among the tile's interface cells in cell order
__device__ __forceinline__ unsigned contrib_row(const Workspace& ws, int gx, int gy, int gz, int ntx, int nty) {
    const int ctile = ((gz / TZ) * nty + gy / TY) * ntx + gx / TX;
    const int l = ((gz % TZ) * TY + gy % TY) * TX + gx % TX;
    const unsigned w = ws.mask[ctile * kWords + l / 32];
    return ws.cbase[ctile] + ws.prefix[ctile * kWords + l / 32] + __popc(w & ((1u << (l % 32)) - 1u));
}

// Fallback gather over the overflow list: the tiles with a source cell whose
// row did not fit in the workspace.  Candidates (interface cells of the tile
// grown by one) are processed in chunks of kChunk in region order: stored rows
// are copied, missing ones recomputed (halo 2 in LDS); each target then adds
// its 27 neighbours' entries in q order.  With at most kChunk candidates this
// is the direct gather's order, so the result is the same bits.
template <int SOLVER, class T, class U, class F, int NRM>
__global__ __launch_bounds__(kThreads) void k_curv_gather_fallback(const float* __restrict__ phi,
                                                                    const float* __restrict__ gkap,
                                                                    float* __restrict__ gphi, Workspace ws, int X,
                                                                    int Y, int Z, int ntx, int nty) {
    constexpr int RX = B_RX, RY = B_RY, RZ = B_RZ, H = 2;
    __shared__ float s[RX * RY * RZ];
    __shared__ unsigned short cand[C_REGION];
    __shared__ unsigned short slot[C_REGION];
    __shared__ float contrib[kChunk][27];
    __shared__ unsigned crow[kChunk];
    __shared__ int wcount[kThreads / 64];
    __shared__ QuadLds<F, 10> qlds[kQuads];
    const int tid = threadIdx.x, grp = tid / kQuad, j = tid % kQuad;
    for (int i = tid; i < C_REGION; i += kThreads) slot[i] = kNoSlot;
    const unsigned ntl = *static_cast<volatile unsigned*>(ws.counter + 2);
    for (unsigned it = blockIdx.x; it < ntl; it += gridDim.x) {
        const int tile = static_cast<int>(ws.over[it]);
        const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
        load_region<RX, RY, RZ>(s, phi, x0 - H, y0 - H, z0 - H, X, Y, Z);
        __syncthreads();
        const int ncand = ordered_compact(C_REGION, [&](int ci) {
            const int lx = ci % C_RX, ly = (ci / C_RX) % C_RY, lz = ci / (C_RX * C_RY);
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly, gz = z0 - 1 + lz;
            return gx >= 1 && gy >= 1 && gz >= 1 && gx <= X - 2 && gy <= Y - 2 && gz <= Z - 2 &&
                   is_iface(s[((lz + H - 1) * RY + (ly + H - 1)) * RX + (lx + H - 1)]);
        }, cand, wcount);
        float acc[kCellsPerThread];
#pragma unroll
        for (int k = 0; k < kCellsPerThread; ++k) acc[k] = 0.0f;
        for (int c0 = 0; c0 < ncand; c0 += kChunk) {
            const int nc = min(kChunk, ncand - c0);
            // one thread per candidate: slot and contribution row
            for (int i = tid; i < nc; i += kThreads) {
                const int ci = cand[c0 + i];
                const int lx = ci % C_RX, ly = (ci / C_RX) % C_RY, lz = ci / (C_RX * C_RY);
                slot[ci] = static_cast<unsigned short>(i);
                crow[i] = contrib_row(ws, x0 - 1 + lx, y0 - 1 + ly, z0 - 1 + lz, ntx, nty);
            }
            __syncthreads();
            // stored rows: all threads, independent loads issued in batches
            const int nv = nc * 27;
            for (int b0 = 0; b0 < nv; b0 += kThreads * kCopyBatch) {
                float v[kCopyBatch];
                unsigned at[kCopyBatch];
#pragma unroll
                for (int u = 0; u < kCopyBatch; ++u) {
                    const int idx = b0 + u * kThreads + tid;
                    const int i = min(idx, nv - 1) / 27;
                    const unsigned r = idx < nv ? crow[i] : ws.rows;
                    at[u] = r < ws.rows ? static_cast<unsigned>(idx) : 0xFFFFFFFFu;
                    v[u] = r < ws.rows ? ws.contrib[static_cast<size_t>(r) * 27 + (idx - i * 27)] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kCopyBatch; ++u)
                    if (at[u] != 0xFFFFFFFFu) contrib[at[u] / 27][at[u] % 27] = v[u];
            }
            {
                // rows that did not fit: recomputed, one group of lanes per cell
                for (int i = grp; i < nc; i += kQuads) {
                    if (crow[i] < ws.rows) continue;                     // uniform per group
                    const int ci = cand[c0 + i];
                    const int lx = ci % C_RX, ly = (ci / C_RX) % C_RY, lz = ci / (C_RX * C_RY);
                    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly, gz = z0 - 1 + lz;
                    const float gk = gkap[(static_cast<int64_t>(gz) * Y + gy) * X + gx];
                    quad_cell<SOLVER, T, U, F, true, NRM, 10>(s, ((lz + 1) * RY + (ly + 1)) * RX + (lx + 1), RX,
                                                              RX * RY, j, tid & 63, gk, contrib[i], qlds[grp]);
                }
            }
            __syncthreads();
#pragma unroll 1
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
        __syncthreads();                                             // LDS reused by the next tile
    }
}

// Neighbour-normal backward, between the work items and the gather: over the
// work items, one 32-lane group per interface cell n, lane j < 26 taking the
// neighbour q of the adjoint's lane order.  The source c = n - e_q, when an
// interface cell, stored in slot j of its row the adjoint for its neighbour at
// +e_q, which is n: the adjoint of n's own fill-level gradient is the sum of
// these 26 slots (zero where c is no interface cell), formed by a fixed
// butterfly and written to the 3-vector beside n's row.  A source without a
// stored row makes it NaN.
__global__ __launch_bounds__(kThreads) void k_curv_hgather(Workspace ws, int X, int Y, int Z, int ntx, int nty) {
    const int tid = threadIdx.x, grp = tid / kGroup, j = tid % kGroup;
    const int half = tid & 32;
    const int q = j < 13 ? j : j + 1;
    const unsigned nitems = *static_cast<volatile unsigned*>(ws.counter);
    for (unsigned item = blockIdx.x; item < nitems; item += gridDim.x) {
        const unsigned e = ws.items[item];
        const int tile = static_cast<int>(e >> 7), part = static_cast<int>(e & 127u);
        const int i = part * kPartCells + grp;
        const unsigned row = ws.cbase[tile] + static_cast<unsigned>(i);
        if (row >= ws.rows) continue;                        // uniform per group; the gather sees the miss
        int gx, gy, gz;
        if (!tile_cell(ws, tile, i, j, half, ntx, nty, gx, gy, gz)) continue;
        const int cx = gx - q_dx(q), cy = gy - q_dy(q), cz = gz - q_dz(q);
        bool src = j < 26 && cx >= 0 && cx < X && cy >= 0 && cy < Y && cz >= 0 && cz < Z;
        unsigned r = 0u;
        if (src) {
            const int ctile = ((cz / TZ) * nty + cy / TY) * ntx + cx / TX;
            const int l = ((cz % TZ) * TY + cy % TY) * TX + cx % TX;
            const unsigned w = ws.mask[ctile * kWords + l / 32], bit = 1u << (l % 32);
            src = (w & bit) != 0u;
            r = ws.cbase[ctile] + ws.prefix[ctile * kWords + l / 32] + __popc(w & (bit - 1u));
        }
        const bool stored = src && r < ws.rows;
        const bool miss = ((__ballot(src && !stored) >> half) & 0xffffffffull) != 0ull;
        float h0 = 0.0f, h1 = 0.0f, h2 = 0.0f;
        if (stored) {
            const float* p = ws.contrib + static_cast<size_t>(r) * kRowFloatsNbr + 27 + 3 * j;
            h0 = p[0];
            h1 = p[1];
            h2 = p[2];
        }
#pragma unroll
        for (int o = kGroup / 2; o > 0; o >>= 1) {
            h0 += __shfl_xor(h0, o, kGroup);
            h1 += __shfl_xor(h1, o, kGroup);
            h2 += __shfl_xor(h2, o, kGroup);
        }
        if (j < 3) {
            const float h = j == 0 ? h0 : (j == 1 ? h1 : h2);
            ws.hbar[3u * row + static_cast<unsigned>(j)] = miss ? __builtin_nanf("") : h;
        }
    }
}

// Direct backward gather for the tiles whose sources all have a stored row.
// The interface bitmasks, prefix counts and first rows of the 3x3x3 tiles
// around the tile are staged in LDS.  Each of the tile's cells tests its 27
// sources (target - e_q) there; the cells with a source (the band along the
// interface; the rest keep the scan's zero) are listed in cell order, and each
// adds entry q of its sources' rows for q = 0..26 in order, all loads issued
// before the first add.  A tile with a source beyond the store goes to the
// overflow list; the fallback gather rewrites every cell of it.
struct SourceMap {
    unsigned smask[27][kWords];
    unsigned spref[27][kWords];
    unsigned sbase[27];
};

// row of source q of the cell (cx, cy, cz) of the centre tile; sets src when
// that source is an interface cell
__device__ __forceinline__ unsigned source_row(const SourceMap& m, int cx, int cy, int cz, int q, bool& src) {
    const int sx = cx - q_dx(q), sy = cy - q_dy(q), sz = cz - q_dz(q);
    const int rx = sx < 0 ? -1 : (sx >= TX ? 1 : 0);
    const int ry = sy < 0 ? -1 : (sy >= TY ? 1 : 0);
    const int rz = sz < 0 ? -1 : (sz >= TZ ? 1 : 0);
    const int tq = (rz + 1) * 9 + (ry + 1) * 3 + (rx + 1);
    const int l = ((sz - rz * TZ) * TY + (sy - ry * TY)) * TX + (sx - rx * TX);
    const unsigned word = m.smask[tq][l >> 5];
    const unsigned bit = 1u << (l & 31);
    src = (word & bit) != 0u;
    return m.sbase[tq] + m.spref[tq][l >> 5] + __popc(word & (bit - 1u));
}

// NBR: the neighbour-normal variant's rows, plus each source's own-gradient
// adjoint spread by the gradient weights of NRM; a tile with a source beyond
// the store gets NaN on its band (that variant has no fallback)
// thread t's cells 4t .. 4t+3 of a tile (row t / 16 in cell order) set to
// zero where bit k of keep is clear; vec: 16-byte stores are aligned
__device__ __forceinline__ void zero_cells(float* __restrict__ gphi, int tile, unsigned keep, bool vec, int X,
                                           int Y, int Z, int ntx, int nty) {
    const int t = threadIdx.x;
    const int gx = (tile % ntx) * TX + (t % (TX / 4)) * 4, gy = ((tile / ntx) % nty) * TY + (t / (TX / 4)) % TY,
              gz = (tile / (ntx * nty)) * TZ + t / (TX / 4 * TY);
    if (gx >= X || gy >= Y || gz >= Z) return;
    float* o = gphi + (static_cast<int64_t>(gz) * Y + gy) * X + gx;
    if (vec && keep == 0u) {
        *reinterpret_cast<float4*>(o) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (gx + k < X && !((keep >> k) & 1u)) o[k] = 0.0f;
    }
}

constexpr int kZeroBatch = kThreads / 32;     // tiles checked at a time by the zero fill

// Zero fill of a backward that ran no scan, tiles b0 .. b0 + kZeroBatch - 1:
// those with no interface cell in their 3x3x3 tile neighbourhood (the ones the
// gather list leaves out) get a zero gradient.  The 32 threads of group u
// check the 27 neighbours of tile b0 + u (the gather list's own test), then the
// workgroup zeroes the inactive ones.  zact: kZeroBatch words of LDS.
__device__ __forceinline__ void zero_away_batch_at(float* __restrict__ gphi, const Workspace& ws, int b0, bool vec,
                                                   int X, int Y, int Z, int ntx, int nty, int ntz, unsigned* zact) {
    const int ntiles = ntx * nty * ntz;
    const int tid = threadIdx.x, u = tid / 32, q = tid % 32;
    const int tile = b0 + u;
    bool act = false;
    if (tile < ntiles && q < 27) {
        const int ax = tile % ntx + q_dx(q), ay = (tile / ntx) % nty + q_dy(q), az = tile / (ntx * nty) + q_dz(q);
        if (ax >= 0 && ax < ntx && ay >= 0 && ay < nty && az >= 0 && az < ntz)
            act = ws.flags[(az * nty + ay) * ntx + ax] != 0u;
    }
    const unsigned long long bal = __ballot(act);
    if (q == 0) zact[u] = static_cast<unsigned>((tid & 32) ? (bal >> 32) : (bal & 0xFFFFFFFFull)) != 0u;
    __syncthreads();
#pragma unroll 1
    for (int uu = 0; uu < kZeroBatch; ++uu) {
        const int tl = b0 + uu;
        if (tl < ntiles && !zact[uu]) zero_cells(gphi, tl, 0u, vec, X, Y, Z, ntx, nty);   // uniform test
    }
}

// ZFILL: the call ran no scan (it reuses a forward's records), so nothing
// zeroed grad_phi: the gather writes the zeros on its tiles' cells off the
// band, and workgroups added past the first ngather zero the tiles it does not
// gather, one batch of kZeroBatch tiles each
template <bool NBR, int NRM, bool ZFILL>
__global__ __launch_bounds__(kThreads, (NBR ? 5 : 8)) void k_curv_gather_direct(float* __restrict__ gphi, Workspace ws, int X,
                                                                  int Y, int Z, int ntx, int nty, int ntz,
                                                                  bool vec, unsigned ngather) {
    constexpr unsigned ROWF = NBR ? kRowFloatsNbr : 27;
    __shared__ SourceMap m;
    __shared__ unsigned short band[kTile];
    __shared__ unsigned long long brow[TY * TZ];
    __shared__ int bpref[TY * TZ];
    __shared__ int bcount;
    __shared__ unsigned zact[kZeroBatch];
    if constexpr (ZFILL) {
        // workgroups past the first ngather: one zero-fill batch each (they
        // start as the gathering ones with fewer tiles finish)
        if (blockIdx.x >= ngather) {
            zero_away_batch_at(gphi, ws, static_cast<int>(blockIdx.x - ngather) * kZeroBatch, vec, X, Y, Z, ntx, nty,
                               ntz, zact);
            return;
        }
    }
    const unsigned ntl = *static_cast<volatile unsigned*>(ws.counter + 1);
    for (unsigned it = blockIdx.x; it < ntl; it += ngather) {
        const int tid = thread_index_per_iteration();
        const int tile = static_cast<int>(ws.tiles[it]);
        if (ws.rows == 0u) {                                         // nothing stored: all recomputed
            if (tid == 0) ws.over[atomicAdd(ws.counter + 2, 1u)] = static_cast<unsigned>(tile);
            continue;
        }
        const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        {
            // the 3x3x3 tiles' bitmasks, prefix counts and first rows (zeros
            // outside): word tid % 32 of tiles tid / 32 + 8u, and first row
            // tid for tid < 27; every load before the first store
            constexpr int kPer = kThreads / kWords, kStageIt = (27 + kPer - 1) / kPer;
            const int w = tid % kWords;
            unsigned smv[kStageIt], spv[kStageIt], sb = 0u;
#pragma unroll
            for (int u = 0; u < kStageIt; ++u) {
                const int t = tid / kWords + kPer * u;
                const int ax = tx + q_dx(t), ay = ty + q_dy(t), az = tz + q_dz(t);
                const bool in = t < 27 && ax >= 0 && ax < ntx && ay >= 0 && ay < nty && az >= 0 && az < ntz;
                const int nt = (az * nty + ay) * ntx + ax;
                smv[u] = in ? ws.mask[nt * kWords + w] : 0u;
                spv[u] = in ? ws.prefix[nt * kWords + w] : 0u;
            }
            if (tid < 27) {
                const int ax = tx + q_dx(tid), ay = ty + q_dy(tid), az = tz + q_dz(tid);
                if (ax >= 0 && ax < ntx && ay >= 0 && ay < nty && az >= 0 && az < ntz)
                    sb = ws.cbase[(az * nty + ay) * ntx + ax];
            }
#pragma unroll
            for (int u = 0; u < kStageIt; ++u) {
                const int t = tid / kWords + kPer * u;
                if (t < 27) {
                    m.smask[t][w] = smv[u];
                    m.spref[t][w] = spv[u];
                }
            }
            if (tid < 27) m.sbase[tid] = sb;
        }
        __syncthreads();
        // the band: cells with an interface source within one cell.  Row
        // (y, z) of a tile is one 64-bit word of its mask (bit = x); a target
        // row's band is the OR over the 9 neighbouring rows of the source row
        // dilated by one cell in x (bits carried in from the x-neighbour tiles)
        if (tid < TY * TZ) {
            const int cy = tid % TY, cz = tid / TY;
            unsigned long long d = 0ull;
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const int sy = cy + dy, sz = cz + dz;
                    const int ry = sy < 0 ? -1 : (sy >= TY ? 1 : 0), rz = sz < 0 ? -1 : (sz >= TZ ? 1 : 0);
                    const int w = ((sz - rz * TZ) * TY + (sy - ry * TY)) * 2;
                    const int tc = (rz + 1) * 9 + (ry + 1) * 3;                 // + (rx + 1)
                    const unsigned long long lft = m.smask[tc][w] | (static_cast<unsigned long long>(m.smask[tc][w + 1]) << 32);
                    const unsigned long long mid = m.smask[tc + 1][w] | (static_cast<unsigned long long>(m.smask[tc + 1][w + 1]) << 32);
                    const unsigned long long rgt = m.smask[tc + 2][w] | (static_cast<unsigned long long>(m.smask[tc + 2][w + 1]) << 32);
                    d |= mid | (mid << 1) | (mid >> 1) | (lft >> 63) | ((rgt & 1ull) << 63);
                }
            }
            // cells past the lattice edge are not targets
            const int gy = y0 + cy, gz = z0 + cz, nx = X - x0;
            if (gy >= Y || gz >= Z) d = 0ull;
            else if (nx < TX) d &= (1ull << nx) - 1ull;
            brow[tid] = d;
            // exclusive prefix of the rows' band counts (the 16 rows are lanes
            // 0..15 of the first wave)
            const int c = __popcll(d);
            int inc = c;
#pragma unroll
            for (int o = 1; o < TY * TZ; o <<= 1) {
                const int v = __shfl_up(inc, o, TY * TZ);
                if (tid >= o) inc += v;
            }
            bpref[tid] = inc - c;
            if (tid == TY * TZ - 1) bcount = inc;
        }
        __syncthreads();
        // band cells listed in cell order (rows in order, x ascending): each
        // band cell's place is its row's prefix plus the band bits before it
#pragma unroll
        for (int k = 0; k < kCellsPerThread; ++k) {
            const int cl = k * kThreads + tid, r = cl / TX, x = cl % TX;
            const unsigned long long d = brow[r];
            if ((d >> x) & 1ull)
                band[bpref[r] + __popcll(d & ((1ull << x) - 1ull))] = static_cast<unsigned short>(cl);
        }
        const int nband = bcount;
        __syncthreads();
        if constexpr (NBR) {
            // band cells: rows of their sources, all loads of a group of 9
            // issued before its adds; sums kept until the tile is known to be
            // complete (a missing row makes the tile's band NaN)
            float acc[kCellsPerThread];
            int miss = 0;
#pragma unroll
            for (int k = 0; k < kCellsPerThread; ++k) {
                const int e = k * kThreads + tid;
                float a = 0.0f;
                if (e < nband) {
                    const int cl = band[e];
                    const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
#pragma unroll 1
                    for (int q0 = 0; q0 < 27; q0 += 9) {
                        float v[9], hv[9][3];
                        unsigned has = 0u;
#pragma unroll
                        for (int qq = 0; qq < 9; ++qq) {
                            bool src;
                            const unsigned r = source_row(m, cx, cy, cz, q0 + qq, src);
                            const bool stored = src && r < ws.rows;
                            miss |= src && !stored;
                            has |= stored ? (1u << qq) : 0u;
                            const unsigned rr = stored ? r : 0u;  // rows >= 1: row 0 read and masked out
                            v[qq] = ws.contrib[rr * ROWF + static_cast<unsigned>(q0 + qq)];
                            hv[qq][0] = ws.hbar[3u * rr];
                            hv[qq][1] = ws.hbar[3u * rr + 1u];
                            hv[qq][2] = ws.hbar[3u * rr + 2u];
                        }
#pragma unroll
                        for (int qq = 0; qq < 9; ++qq) {
                            // the source's own gradient h = sum_q w_q e_q phi_(source + e_q)
                            const int q = q0 + qq;
                            const int e2 = q_dx(q) * q_dx(q) + q_dy(q) * q_dy(q) + q_dz(q) * q_dz(q);
                            const float wq = static_cast<float>(q == 13 ? 0 : nrm_weight<NRM>(e2));
                            const float t = v[qq] + wq * (static_cast<float>(q_dx(q)) * hv[qq][0] +
                                                          static_cast<float>(q_dy(q)) * hv[qq][1] +
                                                          static_cast<float>(q_dz(q)) * hv[qq][2]);
                            a += (has >> qq) & 1u ? t : 0.0f;
                        }
                    }
                }
                acc[k] = a;
            }
            if (__syncthreads_or(miss)) {                            // uniform per workgroup
#pragma unroll
                for (int k = 0; k < kCellsPerThread; ++k) acc[k] = __builtin_nanf("");
            }
#pragma unroll
            for (int k = 0; k < kCellsPerThread; ++k) {
                const int e = k * kThreads + tid;
                if (e < nband) {
                    const int cl = band[e];
                    const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
                    gphi[(static_cast<int64_t>(z0 + cz) * Y + (y0 + cy)) * X + (x0 + cx)] = acc[k];
                }
            }
        } else {
            // band cells: each sums entry q of its sources' rows in q order, the
            // loads of a group of 9 issued before its adds, and stores the sum
            // at once.  A tile with a source beyond the store goes to the
            // overflow list; the fallback gather, a later launch, rewrites all
            // of its cells.
            int miss = 0;
#pragma unroll 1
            for (int e = tid; e < nband; e += kThreads) {
                const int cl = band[e];
                const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
                float a = 0.0f;                                      // +0 + 0 stays +0: same bits as skipping
#pragma unroll 1
                for (int q0 = 0; q0 < 27; q0 += 9) {
                    float v[9];
                    unsigned has = 0u;
#pragma unroll
                    for (int qq = 0; qq < 9; ++qq) {
                        bool src;
                        const unsigned r = source_row(m, cx, cy, cz, q0 + qq, src);
                        const bool stored = src && r < ws.rows;
                        miss |= src && !stored;
                        has |= stored ? (1u << qq) : 0u;
                        // a non-source reads entry q of row 0 (rows >= 1 here) and is masked out
                        v[qq] = ws.contrib[(stored ? r : 0u) * 27u + static_cast<unsigned>(q0 + qq)];
                    }
#pragma unroll
                    for (int qq = 0; qq < 9; ++qq) a += (has >> qq) & 1u ? v[qq] : 0.0f;
                }
                gphi[(static_cast<int64_t>(z0 + cz) * Y + (y0 + cy)) * X + (x0 + cx)] = a;
            }
            if (__syncthreads_or(miss) && tid == 0) ws.over[atomicAdd(ws.counter + 2, 1u)] = static_cast<unsigned>(tile);
        }
        // the tile's cells outside the band have a zero gradient; thread t
        // takes cells 4t .. 4t+3, row t / 16.  After the sums' loads: loads and
        // stores share one in-order counter, so stores issued before them
        // would be waited for with them.
        if constexpr (ZFILL)
            zero_cells(gphi, tile, static_cast<unsigned>(brow[tid / (TX / 4)] >> ((tid % (TX / 4)) * 4)) & 0xFu, vec,
                       X, Y, Z, ntx, nty);
        __syncthreads();                                             // LDS reused by the next tile
    }
}

// ---- launch helpers -----------------------------------------------------------
struct Grid {
    int ntx, nty, ntz;
    int ntiles;
};

// validates the lattice; *empty when there is nothing to do
int check_lattice(int64_t X, int64_t Y, int64_t Z, bool* empty, Grid* g) {
    if (X < 0 || Y < 0 || Z < 0) return PLIC_EINVAL;
    *empty = X == 0 || Y == 0 || Z == 0;
    if (*empty) return PLIC_OK;
    const int64_t lim = 0x7fffffff;
    if (X > lim || Y > lim || Z > lim) return PLIC_EINVAL;
    if (X > (int64_t(1) << 62) / Y / Z) return PLIC_EINVAL;
    const int64_t tx = (X + TX - 1) / TX, ty = (Y + TY - 1) / TY, tz = (Z + TZ - 1) / TZ;
    if (tx > lim / ty || tx * ty > lim / tz) return PLIC_EINVAL;   // grid limit
    // the scan launches 256 work-items per tile (a dispatch holds < 2^32), and
    // work items hold a 25-bit tile index
    if (tx * ty * tz >= (int64_t(1) << 24)) return PLIC_EINVAL;
    g->ntx = static_cast<int>(tx);
    g->nty = static_cast<int>(ty);
    g->ntz = static_cast<int>(tz);
    g->ntiles = static_cast<int>(tx * ty * tz);
    return PLIC_OK;
}

size_t fixed_bytes(const Grid& g) { return 256 + static_cast<size_t>(g.ntiles) * kFixedPerTile; }

// nbr: the neighbour-normal backward's rows (and their gradient adjoints)
Workspace carve(void* base, size_t bytes, const Grid& g, bool nbr = false) {
    char* p = static_cast<char*>(base);
    const size_t nt = static_cast<size_t>(g.ntiles);
    Workspace w;
    w.counter = reinterpret_cast<unsigned*>(p);
    w.flags = reinterpret_cast<unsigned*>(p + 256);
    w.cbase = w.flags + nt;
    w.mask = w.cbase + nt;
    w.prefix = w.mask + nt * kWords;
    w.items = w.prefix + nt * kWords;
    w.tiles = w.items + nt * kMaxParts;
    w.over = w.tiles + nt;
    w.contrib = reinterpret_cast<float*>(w.over + nt);
    const size_t rows = (bytes - fixed_bytes(g)) / (nbr ? kRowBytesNbr : kRowBytes);
    const unsigned limit = nbr ? kRowLimitNbr : kRowLimit;
    w.rows = static_cast<unsigned>(rows < limit ? rows : limit);
    w.hbar = nbr ? w.contrib + static_cast<size_t>(w.rows) * kRowFloatsNbr : nullptr;
    return w;
}

template <bool FWD>
void launch_scan(const float* phi, float* out, Workspace ws, int X, int Y, int Z, const Grid& g,
                 hipStream_t st) {
    const int nb = (g.ntiles + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_curv_zero, dim3(1), dim3(kThreads), 0, st, ws.counter, 0, ws.over,
                       nb <= kOnePassBlocks ? nb : 0);
    const bool vec = X % 4 == 0 && aligned(phi, 16) && aligned(out, 16);
    if (vec)
        hipLaunchKernelGGL((k_curv_scan<true, FWD>), dim3(g.ntiles), dim3(kThreads), 0, st, phi, out, ws, X, Y, Z, g.ntx, g.nty);
    else
        hipLaunchKernelGGL((k_curv_scan<false, FWD>), dim3(g.ntiles), dim3(kThreads), 0, st, phi, out, ws, X, Y, Z, g.ntx, g.nty);
}

unsigned persistent_grid(int64_t items_max) {
    return static_cast<unsigned>(items_max < kPersistentBlocks ? items_max : kPersistentBlocks);
}

// gather list and contribution rows (one pass up to kOnePassBlocks workgroups
// of tiles, else two prefix passes)
void launch_rows(Workspace ws, const Grid& g, hipStream_t st) {
    const int nb = (g.ntiles + kThreads - 1) / kThreads;
    if (nb <= kOnePassBlocks) {
        hipLaunchKernelGGL(k_curv_dilate<true>, dim3(nb), dim3(kThreads), 0, st, ws, g.ntx, g.nty, g.ntz, g.ntiles);
    } else {
        hipLaunchKernelGGL(k_curv_dilate<false>, dim3(nb), dim3(kThreads), 0, st, ws, g.ntx, g.nty, g.ntz, g.ntiles);
        hipLaunchKernelGGL(k_curv_prefix, dim3(nb), dim3(kThreads), 0, st, ws, g.ntiles);
    }
}

template <int SOLVER, class T, class U, class F, bool ADJ, int NRM, bool NBR = false>
void launch_quads(const float* phi, const float* gk, float* kappa, Workspace ws, int X, int Y, int Z, const Grid& g,
                  hipStream_t st) {
    const dim3 grid(persistent_grid(static_cast<int64_t>(g.ntiles) * kMaxParts)), block(kThreads);
    hipLaunchKernelGGL((k_curv_quads<SOLVER, T, U, F, ADJ, NRM, NBR>), grid, block, 0, st, phi, gk, kappa, ws, X, Y, Z,
                       g.ntx, g.nty);
}

// forward: precision picks the types, then the normal and the variant
template <int SOLVER, class T, class U, class F>
void launch_fwd_t(int normal, bool nbr, const float* phi, float* kappa, Workspace ws, int X, int Y, int Z,
                  const Grid& g, hipStream_t st) {
    if (normal == kNormalCM) {
        if (nbr) launch_quads<SOLVER, T, U, F, false, kNormalCM, true>(phi, nullptr, kappa, ws, X, Y, Z, g, st);
        else launch_quads<SOLVER, T, U, F, false, kNormalCM>(phi, nullptr, kappa, ws, X, Y, Z, g, st);
    } else {
        if (nbr) launch_quads<SOLVER, T, U, F, false, kNormalPY, true>(phi, nullptr, kappa, ws, X, Y, Z, g, st);
        else launch_quads<SOLVER, T, U, F, false, kNormalPY>(phi, nullptr, kappa, ws, X, Y, Z, g, st);
    }
}

template <int SOLVER>
void launch_fwd(int precision, int normal, bool nbr, const float* phi, float* kappa, Workspace ws, int X, int Y,
                int Z, const Grid& g, hipStream_t st) {
    if (precision == PLIC_FP32) launch_fwd_t<SOLVER, float, float, float>(normal, nbr, phi, kappa, ws, X, Y, Z, g, st);
    else if (precision == PLIC_MIXED) launch_fwd_t<SOLVER, float, double, double>(normal, nbr, phi, kappa, ws, X, Y, Z, g, st);
    else launch_fwd_t<SOLVER, double, double, double>(normal, nbr, phi, kappa, ws, X, Y, Z, g, st);
}

// backward: adjoint work items (rows that fit), gather list, lean gather of
// the stored rows (independent of solver and precision), then the fallback
// gather that recomputes the rows that did not fit
template <bool NBR, int NRM>
void launch_gather(float* gp, Workspace ws, int X, int Y, int Z, const Grid& g, bool zfill, hipStream_t st) {
    const bool vec = X % 4 == 0 && aligned(gp, 16);
    const unsigned ngather = persistent_grid(g.ntiles);
    if (zfill) {
        const unsigned nbatch = static_cast<unsigned>((g.ntiles + kZeroBatch - 1) / kZeroBatch);
        hipLaunchKernelGGL((k_curv_gather_direct<NBR, NRM, true>), dim3(ngather + nbatch), dim3(kThreads), 0, st, gp,
                           ws, X, Y, Z, g.ntx, g.nty, g.ntz, vec, ngather);
    } else {
        hipLaunchKernelGGL((k_curv_gather_direct<NBR, NRM, false>), dim3(ngather), dim3(kThreads), 0, st, gp, ws, X,
                           Y, Z, g.ntx, g.nty, g.ntz, vec, ngather);
    }
}

template <int SOLVER, class T, class U, class F, int NRM>
void launch_bwd_t(const float* phi, const float* gk, float* gp, Workspace ws, int X, int Y, int Z,
                  const Grid& g, bool zfill, hipStream_t st) {
    launch_rows(ws, g, st);
    if (ws.rows > 0) launch_quads<SOLVER, T, U, F, true, NRM>(phi, gk, nullptr, ws, X, Y, Z, g, st);
    launch_gather<false, 0>(gp, ws, X, Y, Z, g, zfill, st);
    // usually empty.  Its registers and LDS allow one workgroup per CU, so a
    // grid of one per CU (256) runs in a single round, cheap when nothing
    // overflowed and as concurrent as any larger grid when something did
    hipLaunchKernelGGL((k_curv_gather_fallback<SOLVER, T, U, F, NRM>),
                       dim3(g.ntiles < kFallbackBlocks ? g.ntiles : kFallbackBlocks), dim3(kThreads), 0, st, phi,
                       gk, gp, ws, X, Y, Z, g.ntx, g.nty);
}

// neighbour-normal backward: the rows (contributions and the neighbours'
// gradient adjoints), the gradient adjoint per interface cell, then the
// gather; there is no fallback (the entry point requires one row at least)
template <int SOLVER, class T, class U, class F, int NRM>
void launch_bwd_nbr_t(const float* phi, const float* gk, float* gp, Workspace ws, int X, int Y, int Z,
                      const Grid& g, bool zfill, hipStream_t st) {
    launch_rows(ws, g, st);
    launch_quads<SOLVER, T, U, F, true, NRM, true>(phi, gk, nullptr, ws, X, Y, Z, g, st);
    hipLaunchKernelGGL(k_curv_hgather, dim3(persistent_grid(static_cast<int64_t>(g.ntiles) * kMaxParts)),
                       dim3(kThreads), 0, st, ws, X, Y, Z, g.ntx, g.nty);
    launch_gather<true, NRM>(gp, ws, X, Y, Z, g, zfill, st);
}

template <int SOLVER, class T, class U, class F>
void launch_bwd_n(int normal, bool nbr, const float* phi, const float* gk, float* gp, Workspace ws, int X, int Y,
                  int Z, const Grid& g, bool zfill, hipStream_t st) {
    if (nbr) {
        if (normal == kNormalCM) launch_bwd_nbr_t<SOLVER, T, U, F, kNormalCM>(phi, gk, gp, ws, X, Y, Z, g, zfill, st);
        else launch_bwd_nbr_t<SOLVER, T, U, F, kNormalPY>(phi, gk, gp, ws, X, Y, Z, g, zfill, st);
    } else {
        if (normal == kNormalCM) launch_bwd_t<SOLVER, T, U, F, kNormalCM>(phi, gk, gp, ws, X, Y, Z, g, zfill, st);
        else launch_bwd_t<SOLVER, T, U, F, kNormalPY>(phi, gk, gp, ws, X, Y, Z, g, zfill, st);
    }
}

template <int SOLVER>
void launch_bwd(int precision, int normal, bool nbr, const float* phi, const float* gk, float* gp, Workspace ws,
                int X, int Y, int Z, const Grid& g, bool zfill, hipStream_t st) {
    if (precision == PLIC_FP32)
        launch_bwd_n<SOLVER, float, float, float>(normal, nbr, phi, gk, gp, ws, X, Y, Z, g, zfill, st);
    else if (precision == PLIC_MIXED)
        launch_bwd_n<SOLVER, float, double, double>(normal, nbr, phi, gk, gp, ws, X, Y, Z, g, zfill, st);
    else
        launch_bwd_n<SOLVER, double, double, double>(normal, nbr, phi, gk, gp, ws, X, Y, Z, g, zfill, st);
}

// shared argument checks of the two entry points (the workspace's size is
// checked last, by each entry point: PLIC_EWORKSPACE only when every other
// argument is valid)
int check_common(const float* phi, int64_t X, int64_t Y, int64_t Z, int solver, int precision,
                 const void* ws, size_t ws_bytes, bool* empty, Grid* g, int64_t* n) {
    if (!valid_curvature_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    if (check_lattice(X, Y, Z, empty, g) != PLIC_OK) return PLIC_EINVAL;
    *n = *empty ? 0 : X * Y * Z;
    if (!valid_array(phi, *n)) return PLIC_EINVAL;
    if (!*empty) {
        if (ws == nullptr || !aligned(ws, 4)) return PLIC_EINVAL;
        if (overlap(ws, ws_bytes, phi, static_cast<size_t>(*n) * sizeof(float))) return PLIC_EINVAL;
    }
    return PLIC_OK;
}

// ---- which phi a workspace's scan records belong to -----------------------------
// The scan's records (interface masks, prefix counts, work items, tile counts)
// depend on phi and the lattice only.  The host notes, per workspace address,
// the phi and lattice of the last call that scanned into it, so that
// plic_curvature_backward_reuse_f32 skips the scan only when they match.  The
// table is bounded (cleared when full: a miss only costs a scan).
// clean: the last call was a forward, whose counter reset also cleared the
// backward's counters and row-prefix totals (nothing in the forward writes
// them afterwards), so a backward right after it needs no reset of its own
struct ScanRecord {
    const float* phi;
    int64_t X, Y, Z;
    bool clean;
};
constexpr size_t kMaxRecords = 4096;
std::mutex g_record_mutex;
std::unordered_map<const void*, ScanRecord> g_records;

void note_scan(const void* ws, const float* phi, int64_t X, int64_t Y, int64_t Z, bool ok, bool clean) {
    std::lock_guard<std::mutex> lock(g_record_mutex);
    if (!ok) {
        g_records.erase(ws);
        return;
    }
    if (g_records.size() >= kMaxRecords && g_records.find(ws) == g_records.end()) g_records.clear();
    g_records[ws] = ScanRecord{phi, X, Y, Z, clean};
}

// 0: no records of this phi; 1: records; 2: records and clean counters.  The
// note turns unclean (a backward is about to use the counters).
int take_scan(const void* ws, const float* phi, int64_t X, int64_t Y, int64_t Z) {
    std::lock_guard<std::mutex> lock(g_record_mutex);
    const auto it = g_records.find(ws);
    if (it == g_records.end() || it->second.phi != phi || it->second.X != X || it->second.Y != Y ||
        it->second.Z != Z)
        return 0;
    const bool clean = it->second.clean;
    it->second.clean = false;
    return clean ? 2 : 1;
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// the forward launches, after validation
int curvature_forward(const float* phi, int64_t X, int64_t Y, int64_t Z, float* kappa, int solver, int precision,
                      int normal, bool nbr, void* workspace, size_t workspace_bytes, const Grid& g, hipStream_t st) {
    const Workspace ws = carve(workspace, workspace_bytes, g);
    const int x = static_cast<int>(X), y = static_cast<int>(Y), z = static_cast<int>(Z);
    launch_scan<true>(phi, kappa, ws, x, y, z, g, st);
    switch (solver) {
        case kSZ: launch_fwd<kSZ>(precision, normal, nbr, phi, kappa, ws, x, y, z, g, st); break;
        case kNewton: launch_fwd<kNewton>(precision, normal, nbr, phi, kappa, ws, x, y, z, g, st); break;
        case kNested: launch_fwd<kNested>(precision, normal, nbr, phi, kappa, ws, x, y, z, g, st); break;
        default: launch_fwd<kAnalytic>(precision, normal, nbr, phi, kappa, ws, x, y, z, g, st); break;
    }
    const int rc = launch_status();
    note_scan(workspace, phi, X, Y, Z, rc == PLIC_OK, true);
    return rc;
}

// the backward, after the shared checks; reuse: skip the scan when the
// workspace holds this phi's records
int curvature_backward(const float* phi, int64_t X, int64_t Y, int64_t Z, const float* grad_kappa, float* grad_phi,
                       int solver, int precision, int normal, int neighbour_normals, void* workspace,
                       size_t workspace_bytes, void* stream, bool reuse) {
    bool empty;
    Grid g{};
    int64_t n = 0;
    if (check_common(phi, X, Y, Z, solver, precision, workspace, workspace_bytes, &empty, &g, &n) != PLIC_OK)
        return PLIC_EINVAL;
    if (!valid_normal(normal) || (neighbour_normals != 0 && neighbour_normals != 1)) return PLIC_EINVAL;
    if (!valid_array(grad_kappa, n) || !valid_array(grad_phi, n)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(n) * sizeof(float);
    if (overlap(grad_phi, nb, phi, nb) || overlap(grad_phi, nb, grad_kappa, nb)) return PLIC_EINVAL;
    if (!empty && (overlap(workspace, workspace_bytes, grad_phi, nb) ||
                   overlap(workspace, workspace_bytes, grad_kappa, nb)))
        return PLIC_EINVAL;
    if (empty) return PLIC_OK;
    // the neighbour-normal backward has no fallback: it needs one row at least
    if (workspace_bytes < fixed_bytes(g) + (neighbour_normals ? kRowBytesNbr : 0)) return PLIC_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool nbr = neighbour_normals != 0;
    const Workspace ws = carve(workspace, workspace_bytes, g, nbr);
    const int x = static_cast<int>(X), y = static_cast<int>(Y), z = static_cast<int>(Z);
    const int rec = reuse ? take_scan(workspace, phi, X, Y, Z) : 0;
    const bool scan = rec == 0;
    if (scan) {
        launch_scan<false>(phi, grad_phi, ws, x, y, z, g, st);
    } else if (rec == 1 || capturing(st)) {
        // (a captured graph may replay this backward without its forward)
        const int nb = (g.ntiles + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_curv_zero, dim3(1), dim3(kThreads), 0, st, ws.counter, 1, ws.over,
                           nb <= kOnePassBlocks ? nb : 0);
    }
    switch (solver) {
        case kSZ: launch_bwd<kSZ>(precision, normal, nbr, phi, grad_kappa, grad_phi, ws, x, y, z, g, !scan, st); break;
        case kNewton:
            launch_bwd<kNewton>(precision, normal, nbr, phi, grad_kappa, grad_phi, ws, x, y, z, g, !scan, st);
            break;
        case kNested:
            launch_bwd<kNested>(precision, normal, nbr, phi, grad_kappa, grad_phi, ws, x, y, z, g, !scan, st);
            break;
        default:
            launch_bwd<kAnalytic>(precision, normal, nbr, phi, grad_kappa, grad_phi, ws, x, y, z, g, !scan, st);
            break;
    }
    const int rc = launch_status();
    if (scan || rc != PLIC_OK) note_scan(workspace, phi, X, Y, Z, rc == PLIC_OK, false);
    return rc;
}

// ---- the forward without a caller workspace ------------------------------------
// A file-scope device array serves as the workspace of plic_curvature_noalloc_f32
// (every GPU the library runs on holds its own copy, for the life of the
// process).  Host code reaches it only through the address that
// hipGetSymbolAddress returns on each device; the array's name in host code
// is not a device address.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address, looked up once per device
int scratch_for_current_device(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_last_hip_error(static_cast<int>(e));
        return PLIC_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return PLIC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_last_hip_error(static_cast<int>(e != hipSuccess ? e : hipErrorInvalidSymbol));
            return PLIC_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PLIC_OK;
}

}  // namespace
}  // namespace plic

using namespace plic;

extern "C" {

size_t plic_curvature_workspace_bytes(int64_t X, int64_t Y, int64_t Z) {
    bool empty;
    Grid g;
    if (check_lattice(X, Y, Z, &empty, &g) != PLIC_OK || empty) return 0;
    return fixed_bytes(g) + static_cast<size_t>(g.ntiles) * kDefaultRowsPerTile * kRowBytes;
}

size_t plic_curvature_workspace_bytes_ex(int64_t X, int64_t Y, int64_t Z, int neighbour_normals) {
    bool empty;
    Grid g;
    if (neighbour_normals != 0 && neighbour_normals != 1) return 0;
    if (check_lattice(X, Y, Z, &empty, &g) != PLIC_OK || empty) return 0;
    if (!neighbour_normals) return fixed_bytes(g) + static_cast<size_t>(g.ntiles) * kDefaultRowsPerTile * kRowBytes;
    return fixed_bytes(g) + static_cast<size_t>(g.ntiles) * kDefaultRowsPerTileNbr * kRowBytesNbr;
}

int plic_curvature_ex_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, float* kappa, int solver,
                          int precision, int normal, int neighbour_normals, void* workspace, size_t workspace_bytes,
                          void* stream) {
    bool empty;
    Grid g{};
    int64_t n = 0;
    if (check_common(phi, X, Y, Z, solver, precision, workspace, workspace_bytes, &empty, &g, &n) != PLIC_OK)
        return PLIC_EINVAL;
    if (!valid_normal(normal) || (neighbour_normals != 0 && neighbour_normals != 1)) return PLIC_EINVAL;
    if (!valid_array(kappa, n)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(n) * sizeof(float);
    if (overlap(phi, nb, kappa, nb)) return PLIC_EINVAL;
    if (!empty && overlap(workspace, workspace_bytes, kappa, nb)) return PLIC_EINVAL;
    if (empty) return PLIC_OK;
    if (workspace_bytes < fixed_bytes(g)) return PLIC_EWORKSPACE;
    return curvature_forward(phi, X, Y, Z, kappa, solver, precision, normal, neighbour_normals != 0, workspace,
                             workspace_bytes, g, static_cast<hipStream_t>(stream));
}

int plic_curvature_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, float* kappa, int solver,
                       int precision, void* workspace, size_t workspace_bytes, void* stream) {
    return plic_curvature_ex_f32(phi, X, Y, Z, kappa, solver, precision, PLIC_NORMAL_PY, 0, workspace,
                                 workspace_bytes, stream);
}

int plic_curvature_noalloc_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, float* kappa, int solver,
                               int precision, void* stream) {
    bool empty;
    Grid g{};
    if (!valid_curvature_solver(solver) || !valid_precision(precision)) return PLIC_EINVAL;
    if (check_lattice(X, Y, Z, &empty, &g) != PLIC_OK) return PLIC_EINVAL;
    const int64_t n = empty ? 0 : X * Y * Z;
    if (!valid_array(phi, n) || !valid_array(kappa, n)) return PLIC_EINVAL;
    const size_t nb = static_cast<size_t>(n) * sizeof(float);
    if (overlap(phi, nb, kappa, nb)) return PLIC_EINVAL;
    if (empty) return PLIC_OK;
    if (fixed_bytes(g) > kScratchBytes) return PLIC_EWORKSPACE;          // beyond the static scratch
    void* ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc != PLIC_OK) return rc;
    return curvature_forward(phi, X, Y, Z, kappa, solver, precision, PLIC_NORMAL_PY, false, ws, kScratchBytes, g,
                             static_cast<hipStream_t>(stream));
}


int plic_curvature_backward_ex_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, const float* grad_kappa,
                                   float* grad_phi, int solver, int precision, int normal, int neighbour_normals,
                                   void* workspace, size_t workspace_bytes, void* stream) {
    return curvature_backward(phi, X, Y, Z, grad_kappa, grad_phi, solver, precision, normal, neighbour_normals,
                              workspace, workspace_bytes, stream, false);
}

int plic_curvature_backward_reuse_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, const float* grad_kappa,
                                      float* grad_phi, int solver, int precision, int normal, int neighbour_normals,
                                      void* workspace, size_t workspace_bytes, void* stream) {
    return curvature_backward(phi, X, Y, Z, grad_kappa, grad_phi, solver, precision, normal, neighbour_normals,
                              workspace, workspace_bytes, stream, true);
}

int plic_curvature_backward_f32(const float* phi, int64_t X, int64_t Y, int64_t Z, const float* grad_kappa,
                                float* grad_phi, int solver, int precision, void* workspace,
                                size_t workspace_bytes, void* stream) {
    return plic_curvature_backward_ex_f32(phi, X, Y, Z, grad_kappa, grad_phi, solver, precision, PLIC_NORMAL_PY, 0,
                                          workspace, workspace_bytes, stream);
}

int plic_curvature_status(const void* workspace, size_t workspace_bytes, int64_t X, int64_t Y, int64_t Z,
                          int neighbour_normals, int64_t* interface_cells, size_t* bytes_for_all_rows, void* stream) {
    bool empty;
    Grid g{};
    if (check_lattice(X, Y, Z, &empty, &g) != PLIC_OK || empty) return PLIC_EINVAL;
    if (neighbour_normals != 0 && neighbour_normals != 1) return PLIC_EINVAL;
    if (workspace == nullptr || !aligned(workspace, 4)) return PLIC_EINVAL;
    const bool nbr = neighbour_normals != 0;
    if (workspace_bytes < fixed_bytes(g) + (nbr ? kRowBytesNbr : 0)) return PLIC_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Workspace ws = carve(const_cast<void*>(workspace), workspace_bytes, g, nbr);
    // the call's interface count is the sum of the tiles' counts the scan wrote
    std::vector<unsigned> flags(static_cast<size_t>(g.ntiles));
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(flags.data(), ws.flags, flags.size() * sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_last_hip_error(static_cast<int>(e));
        return PLIC_EHIP;
    }
    uint64_t cells = 0;
    for (const unsigned f : flags) cells += f;
    const size_t row_bytes = nbr ? kRowBytesNbr : kRowBytes;
    if (interface_cells) *interface_cells = static_cast<int64_t>(cells);
    if (bytes_for_all_rows) *bytes_for_all_rows = fixed_bytes(g) + static_cast<size_t>(cells) * row_bytes;
    return nbr && cells > ws.rows ? PLIC_EWORKSPACE : PLIC_OK;
}

}  // extern "C"
