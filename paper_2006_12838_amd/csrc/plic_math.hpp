// Device-side PLIC mathematics for gfx950: symmetry reduction, the four
// inversion solvers, the forward volume and the derivatives of the offset.
//
// Paper: Lehmann & Gekle, arXiv 2006.12838.  Notation follows Sec. 2:
// reduced space has sorted 0 <= n1 <= n2 <= n3, the reduced volume
// V = min(V0, 1 - V0) in [0, 1/2] and the reduced offset d = S/2 - |d0| in
// [0, S/2] (origin at the cube corner), S = n1 + n2 + n3.
//
// Everything is templated on the arithmetic type T (float or double).  The
// cubic-case root recovery takes a second type U so that FP32 kernels can run
// that part in FP64 (mixed precision).
#pragma once

#include <hip/hip_runtime.h>
#include <cfloat>
#include <cstdint>

namespace plic {

// ---------------------------------------------------------------------------
// arithmetic primitives.  FP32 uses the native gfx950 instructions (v_sqrt,
// v_rsq, v_rcp: <= 1 ulp); FP64 uses the correctly rounded library routines.
// ---------------------------------------------------------------------------
template <class T> struct M;

template <> struct M<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float cbrt(float x) { return ::cbrtf(x); }
    static __device__ __forceinline__ float sin(float x) { return ::sinf(x); }
    // sin on |x| <= pi/6 by its Maclaurin series through x^9 (first omitted
    // term x^11/11! < 2e-11 there, far below FP32 rounding)
    static __device__ __forceinline__ float sin_small(float x) {
        const float x2 = x * x;
        float p = 1.0f / 362880.0f;
        p = p * x2 - 1.0f / 5040.0f;
        p = p * x2 + 1.0f / 120.0f;
        p = p * x2 - 1.0f / 6.0f;
        return x + x * x2 * p;
    }
    static __device__ __forceinline__ float asin(float x) { return ::asinf(x); }
    static __device__ __forceinline__ float acos(float x) { return ::acosf(x); }
    static __device__ __forceinline__ float cos(float x) { return ::cosf(x); }
    static __device__ __forceinline__ float atan(float x) { return ::atanf(x); }
    // atan(y / x) for y >= 0, x > 0
    static __device__ __forceinline__ float atan2_pos(float y, float x) { return ::atanf(y * __builtin_amdgcn_rcpf(x)); }
    static __device__ __forceinline__ float fmin(float a, float b) { return ::fminf(a, b); }
    static __device__ __forceinline__ float fmax(float a, float b) { return ::fmaxf(a, b); }
    static __device__ __forceinline__ float fabs(float a) { return ::fabsf(a); }
    static __device__ __forceinline__ float med3(float a, float b, float c) {
        return __builtin_amdgcn_fmed3f(a, b, c);
    }
    static constexpr float tiny = FLT_MIN;
    static constexpr float nan_v = __builtin_nanf("");
    // Newton step tolerance (|delta d|) and bisection halvings per bracket
    static constexpr float newton_tol = 1e-6f;
    static constexpr int bisect_steps = 24;
    // relative pivot threshold of the fit (rounding noise of a zero pivot ~1e-7)
    static constexpr float pivot_rel = 1e-5f;
};

template <> struct M<double> {
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double cbrt(double x) { return ::cbrt(x); }
    static __device__ __forceinline__ double sin(double x) { return ::sin(x); }
    // sin on |x| <= pi/6 by its Maclaurin series through x^17 (first omitted
    // term x^19/19! < 4e-23 there)
    static __device__ __forceinline__ double sin_small(double x) {
        const double x2 = x * x;
        double p = 1.0 / 355687428096000.0;         // 1/17!
        p = p * x2 - 1.0 / 1307674368000.0;         // 1/15!
        p = p * x2 + 1.0 / 6227020800.0;            // 1/13!
        p = p * x2 - 1.0 / 39916800.0;              // 1/11!
        p = p * x2 + 1.0 / 362880.0;                // 1/9!
        p = p * x2 - 1.0 / 5040.0;                  // 1/7!
        p = p * x2 + 1.0 / 120.0;                   // 1/5!
        p = p * x2 - 1.0 / 6.0;                     // 1/3!
        return x + x * x2 * p;
    }
    static __device__ __forceinline__ double asin(double x) { return ::asin(x); }
    static __device__ __forceinline__ double acos(double x) { return ::acos(x); }
    static __device__ __forceinline__ double cos(double x) { return ::cos(x); }
    static __device__ __forceinline__ double atan(double x) { return ::atan(x); }
    // atan(y / x) for y >= 0, x > 0 (within 3 ulp).  With a <= b the smaller
    // and larger of y and x, u = a / b in [0, 1] is reduced about tan(k pi/8),
    // k = 0, 1, 2, by atan(u) = k pi/8 + atan(v), v = (a - t b) / (b + t a),
    // |v| <= tan(pi/16); atan(v) by its Maclaurin series through v^21 (first
    // omitted term below 2^-53 |v|); y > x reflects through pi/2.
    static __device__ __forceinline__ double atan2_pos(double y, double x) {
        const bool sw = y > x;
        const double a = sw ? x : y, b = sw ? y : x;
        const bool k1 = a >= 0.19891236737965800691 * b;                // tan(pi/16)
        const bool k2 = a >= 0.66817863791929891999 * b;                // tan(3 pi/16)
        const double t = k2 ? 1.0 : (k1 ? 0.41421356237309504880 : 0.0);  // tan(k pi/8)
        const double c = k2 ? 0.78539816339744830962 : (k1 ? 0.39269908169872415481 : 0.0);
        const double v = (a - t * b) / (b + t * a);
        const double v2 = v * v;
        double p = 1.0 / 21.0;
        p = p * v2 - 1.0 / 19.0;
        p = p * v2 + 1.0 / 17.0;
        p = p * v2 - 1.0 / 15.0;
        p = p * v2 + 1.0 / 13.0;
        p = p * v2 - 1.0 / 11.0;
        p = p * v2 + 1.0 / 9.0;
        p = p * v2 - 1.0 / 7.0;
        p = p * v2 + 1.0 / 5.0;
        p = p * v2 - 1.0 / 3.0;
        const double r = c + (v + v * v2 * p);
        return sw ? 1.57079632679489661923 - r : r;
    }
    static __device__ __forceinline__ double fmin(double a, double b) { return ::fmin(a, b); }
    static __device__ __forceinline__ double fmax(double a, double b) { return ::fmax(a, b); }
    static __device__ __forceinline__ double fabs(double a) { return ::fabs(a); }
    static __device__ __forceinline__ double med3(double a, double b, double c) {
        return ::fmax(::fmin(a, b), ::fmin(::fmax(a, b), c));
    }
    static constexpr double tiny = DBL_MIN;
    static constexpr double nan_v = __builtin_nan("");
    static constexpr double newton_tol = 1e-13;
    static constexpr int bisect_steps = 52;
    static constexpr double pivot_rel = 1e-10;
};

enum Solver : int { kAnalytic = 0, kSZ = 1, kNewton = 2, kNested = 3, kKawano = 4 };

// ---------------------------------------------------------------------------
// Symmetry reduction (Sec. 2.1).  The reduced volume is taken as
// V0 <= 1/2 ? V0 : 1 - V0, which is exact in floating point (Sterbenz), where
// the printed 1/2 - |V0 - 1/2| rounds for V0 < 1/2 and the cube root of case
// (1) amplifies that rounding near V0 = 0.
// ---------------------------------------------------------------------------
template <class T> struct Reduced {
    T n1, n2, n3;  // sorted |n|
    T V;           // reduced volume in [0, 1/2]
    T V0;          // clamped input volume
};

template <class T>
__device__ __forceinline__ Reduced<T> reduce(T nx, T ny, T nz, T V0) {
    using m = M<T>;
    Reduced<T> r;
    const T ax = m::fabs(nx), ay = m::fabs(ny), az = m::fabs(nz);
    r.n1 = m::fmin(m::fmin(ax, ay), az);
    r.n3 = m::fmax(m::fmax(ax, ay), az);
    r.n2 = m::med3(ax, ay, az);
    const T v = m::fmin(m::fmax(V0, T(0)), T(1));
    r.V0 = v;
    r.V = v <= T(0.5) ? v : T(1) - v;
    return r;
}

// d0 = sign(V0 - 1/2) (S/2 - d)  (Sec. 2.1); NaN inputs and n = 0 give NaN.
template <class T>
__device__ __forceinline__ T unreduce(const Reduced<T>& r, T d, T nx, T ny, T nz, T V0raw) {
    T h = T(0.5) * (r.n1 + r.n2 + r.n3) - d;
    T d0 = r.V0 > T(0.5) ? h : (r.V0 < T(0.5) ? -h : T(0));
    if (__builtin_isnan(nx + ny + nz + V0raw) || !(r.n3 > T(0))) d0 = M<T>::nan_v;
    return d0;
}

// ---------------------------------------------------------------------------
// Closed-form cases, shared by every solver except Kawano's form.  Derived from
// the piecewise volume of the reduced problem (Sec. 2.2), written with
// k = 6 V n2 n3 (an area, like n1^2):
//   slab,  n1 + n2 <= d <= n3:  V n3 = d - (n1 + n2)/2
//          -> case (5) when 2 V n3 >= n1 + n2;
//   corner tetrahedron, d <= n1:  d^3 = k n1
//          -> case (1) when k < n1^2 (that is, d < n1);
//   cut wedge, n1 <= d <= n2:  (d - n1/2)^2 = (4k - n1^2) / 12
//          -> case (2) when d <= n2, that is k - n1^2 <= 3 n2 (n2 - n1)
//             (the a-priori condition of Sec. 2.3 with its factor 2 restored).
// Returns the case (5, 1 or 2) with d set, or 0 for the cubic cases.  A
// coordinate-plane normal (n1 = 0) lands in (2), an axis normal in (5).  The
// formulas are homogeneous of degree 1 in n, so they hold in any units (the
// SZ solver passes the L1-normalized normal).
// ---------------------------------------------------------------------------
template <class T, bool WITH_CASE1 = true>
__device__ __forceinline__ int closed_case(T n1, T n2, T n3, T V, T& d) {
    using m = M<T>;
    const T half_base = T(0.5) * (n1 + n2);           // d - V n3 inside the slab
    const T lift = V * n3;
    if (lift >= half_base) { d = lift + half_base; return 5; }
    const T k = T(6) * n2 * lift, a = n1 * n1;
    if (k < a) {
        if constexpr (WITH_CASE1) d = m::cbrt(k * n1);
        return 1;
    }
    if (k - a <= T(3) * n2 * (n2 - n1)) {
        d = T(0.5) * n1 + m::sqrt(m::fmax(T(4) * k - a, T(0)) * T(1.0 / 12.0));
        return 2;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Each solver runs in two stages.  The closed stage settles the closed-form
// cases and otherwise hands over an Open problem; the cubic stage solves that
// (cases (3) and (4), and case (1) for Newton-Raphson).  offset() chains the
// two per thread; the batched kernels pack the open problems of a workgroup
// densely before the cubic stage, so the costly part runs on full wavefronts.
// ---------------------------------------------------------------------------
template <class T> struct Open {
    T n1, n2, n3;  // sorted normal in the solver's units (L1 for SZ)
    T V;           // reduced volume; negative marks Newton's case (1)
};

// ---------------------------------------------------------------------------
// Volume at d = n3 in the divided form (times n3 / V): case (3) holds for
// n3 V < v3n3 when n3 < n1 + n2, always otherwise.  Scale-invariant, no
// cancellation for small n1 (the (n3 - n2)^3 / n1 term is at most n1^2).
// ---------------------------------------------------------------------------
template <class U>
__device__ __forceinline__ bool cubic_case3(U u1, U u2, U u3, U uV) {
    using m = M<U>;
    if (!(u3 < u1 + u2)) return true;
    const U w = u3 - u2;
    const U v3 = m::div(U(3) * u3 * (u3 - u1) + u1 * u1 - m::div(w * w * w, u1), U(6) * u2);
    return u3 * uV < v3;
}

// ---------------------------------------------------------------------------
// Analytic solution (Sec. 2.3): the trigonometric root
//   f(x, y, a, b, c) = c - 2 (a + b (x^2+y^2)^(1/3)) / (x^2+y^2)^(1/6)
//                      * sin(pi/6 - atan2(y, x)/3)
// with the printed coefficients of cases (3) and (4).  Two exact
// simplifications:
//  * x3^2 + y3^2 = 23328 (n1 n2)^3 and x4^2 + y4^2 = 4 t4^3, so the cube roots
//    cancel: the prefactor is 2 sqrt(2 n1 n2) in case (3) and sqrt(t4)/3 in
//    case (4);
//  * t4 = 9 (S^2 - 2) assumes |n| = 1 and cancels near the face diagonal; the
//    equal (for |n| = 1), degree-2 homogeneous
//    t4 = 9 (2 n1 (n2 + n3) - n1^2 - (n3 - n2)^2) is used instead.
// The paper evaluates case (3) and keeps it when d3 <= n3, else evaluates
// case (4).  Here the case is decided first by the volume at d = n3 (the same
// case; at the boundary both roots equal n3), so that each lane evaluates a
// single root: one atan and one sin, with the case's (x, y, prefactor, c).
// atan(y/x) replaces atan2 with x clamped to the smallest normal number, as
// the paper does for x4; x3 > 0 holds once (5) is excluded.
// ---------------------------------------------------------------------------
template <class T, class U>
__device__ __forceinline__ T cubic_analytic(const Open<T>& o) {
    using m = M<U>;
    const U u1 = o.n1, u2 = o.n2, u3 = o.n3, uV = o.V;
    const U p = u1 * u2, s = u1 + u2;
    const U pi6 = U(0.52359877559829887308), third = U(1) / U(3);
    U x, r2, pref, c;
    if (cubic_case3(u1, u2, u3, uV)) {                           // case (3)
        x = U(81) * p * (s - U(2) * u3 * uV);
        r2 = U(23328) * p * p * p;
        pref = U(2) * m::sqrt(U(2) * p);
        c = s;
    } else {                                                     // case (4)
        const U t4 = m::fmax(U(9) * (U(2) * u1 * (u2 + u3) - u1 * u1 - (u3 - u2) * (u3 - u2)), U(0));
        x = U(324) * p * u3 * (U(1) - U(2) * uV);
        r2 = U(4) * t4 * t4 * t4;
        pref = m::sqrt(t4) * third;
        c = U(0.5) * (s + u3);
    }
    x = m::fmax(x, m::tiny);
    const U y = m::sqrt(m::fmax(r2 - x * x, U(0)));
    // the sine's argument lies in (0, pi/6]: atan(y/x) is in [0, pi/2)
    return T(c - pref * m::sin_small(pi6 - third * m::atan2_pos(y, x)));
}

// ---------------------------------------------------------------------------
// Optimized Scardovelli-Zaleski solution (Sec. 2.4), on the L1-normalized
// normal (n1 + n2 + n3 = 1, so d in [0, 1/2]).  Cases (5), (2), (1) first,
// by the shared closed forms (closed_case) on the L1-normalized normal;
// the boundary between (3) and (4) is decided a priori through the volume v3
// at d = n3; one root d = c - 2 t sin(asin(arg)/3) serves both.  The printed
// coefficients t = sqrt(c^2 - b) and arg = (c^3 - a/2 - 3bc/2)/t^3 are 0/0 for
// small n1; the equal cancellation-free forms are used:
//   case (3): c = n1 + n2, t = sqrt(2 n1 n2), arg = 1.5 n1 n2 (n1 + n2 - 2 n3 V) / t^3
//   case (4): c = 1/2,     t = sqrt(2 n1 (n2+n3) - n1^2 - (n3-n2)^2) / 2,
//             arg = 0.75 n1 n2 n3 (1 - 2V) / t^3
// and arg is clamped to [-1, 1] before asin.  v3 is evaluated in the divided
// form 3 n3 (n3 - n1) + n1^2 - (n3 - n2)^3 / n1 (over 6 n2), which has no
// cancellation either.  d is in L1 units.
// ---------------------------------------------------------------------------
template <class T, class U>
__device__ __forceinline__ T cubic_sz(const Open<T>& o) {
    using m = M<U>;
    const U u1 = o.n1, u2 = o.n2, u3 = o.n3, uV = o.V, s = u1 + u2;
    const bool case3 = cubic_case3(u1, u2, u3, uV);
    U c, t, num;
    if (case3) {
        c = s;
        t = m::sqrt(U(2) * u1 * u2);
        num = U(1.5) * u1 * u2 * (s - U(2) * u3 * uV);
    } else {
        c = U(0.5);
        t = U(0.5) * m::sqrt(m::fmax(U(2) * u1 * (u2 + u3) - u1 * u1 - (u3 - u2) * (u3 - u2), U(0)));
        num = U(0.75) * u1 * u2 * u3 * (U(1) - U(2) * uV);
    }
    U arg = m::div(num, t * t * t);
    arg = m::fmin(m::fmax(arg, U(-1)), U(1));
    // asin(arg) / 3 lies in [-pi/6, pi/6]
    return T(c - U(2) * t * m::sin_small(m::asin(arg) * (U(1) / U(3))));
}

// ---------------------------------------------------------------------------
// The cubic cases for the iterative solvers, shifted to t = d - n2 and
// multiplied by n1 (the volume of Sec. 2.2 without a division by n1):
//   n1 * 6 n2 n3 (V(n2 + t) - V(n2))
//     = H3(t) = ((3 n1 - t) t + b) t,     b = n1 (6 n2 - 3 n1),  t <= delta
//     = H4(t) = H3(t) - (t - delta)^3,    delta = n3 - n2,       t >= delta
// and the root solves H(t) = c with c = n1 (6 n2 n3 V - 3 n2 (n2 - n1) - n1^2).
// Case (4) holds when delta < n1 and H3(delta) < c; its bracket is
// [delta, (n1 + delta) / 2] (up to d = S/2), that of case (3) is
// [0, min(n1, delta)].  Both are cubics a3 t^3 + a2 t^2 + a1 t in Horner form:
// case (3): (-1, 3 n1, b); case (4): (-2, 3 (n1 + delta), b - 3 delta^2) with
// c - delta^3 on the right.  Newton's case (1) (d < n1) is t = d, the cubic
// t^3 = 6 n1 n2 n3 V on [0, n1].
// ---------------------------------------------------------------------------
template <class U> struct Cubic {
    U base;            // d = base + t
    U a3, a2, a1, c;   // a3 t^3 + a2 t^2 + a1 t = c
    U lo, hi;          // bracket of t
};

template <class T, class U>
__device__ __forceinline__ Cubic<U> cubic_setup(const Open<T>& o) {
    using m = M<U>;
    const U n1 = o.n1, n2 = o.n2, n3 = o.n3;
    Cubic<U> q;
    if (o.V < T(0)) {                                            // Newton's case (1)
        q.base = U(0); q.a3 = U(1); q.a2 = U(0); q.a1 = U(0);
        q.c = U(6) * n1 * n2 * n3 * U(-o.V);
        q.lo = U(0); q.hi = n1;
        return q;
    }
    const U target = U(6) * n2 * n3 * U(o.V);
    const U c = n1 * (target - (U(3) * n2 * (n2 - n1) + n1 * n1));
    const U b = n1 * (U(6) * n2 - U(3) * n1);
    const U de = n3 - n2;
    const U h3 = ((U(3) * n1 - de) * de + b) * de;
    const bool case4 = de < n1 && h3 < c;
    q.base = n2;
    if (case4) {
        q.a3 = U(-2); q.a2 = U(3) * (n1 + de); q.a1 = b - U(3) * de * de; q.c = c - de * de * de;
        q.lo = de; q.hi = U(0.5) * (n1 + de);
    } else {
        q.a3 = U(-1); q.a2 = U(3) * n1; q.a1 = b; q.c = c;
        q.lo = U(0); q.hi = m::fmin(n1, de);
    }
    return q;
}

// ---------------------------------------------------------------------------
// Newton-Raphson (Sec. 2.5).  Cases (5) and (2) in closed form; case (1) and
// the cubic cases by Newton on the shifted cubic above, starting at the middle
// of the case's bracket (n1/2 for case (1), as printed).  The printed fixed
// step counts (7/4/4) do not converge for small V, so each iterate is
// safeguarded (kept inside the shrinking bracket, bisecting when a step leaves
// it); iteration stops after a Newton step of |step| <= 1e-6 (FP32) / 1e-13
// (FP64) or once the bracket is that narrow, at most 40 steps.  V = 0 returns
// d = 0 directly.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool closed_newton(T n1, T n2, T n3, T V, T& d, Open<T>& o) {
    const int c = closed_case<T, false>(n1, n2, n3, V, d);
    if (c >= 2) return true;                                            // (5) or (2)
    if (V == T(0)) { d = T(0); return true; }
    // the case follows the classifier's own decision, so that rounding
    // cannot place the root in a skipped case-(2) interval
    o = Open<T>{n1, n2, n3, c == 1 ? -V : V};
    return false;
}

template <class T, class U>
__device__ __forceinline__ T cubic_newton(const Open<T>& o) {
    using m = M<U>;
    const Cubic<U> q = cubic_setup<T, U>(o);
    U lo = q.lo, hi = q.hi;
    U x = U(0.5) * (lo + hi);
    const U tol = U(M<T>::newton_tol);
    const U a3x3 = U(3) * q.a3, a2x2 = U(2) * q.a2;
#pragma unroll 1
    for (int it = 0; it < 40; ++it) {
        const U f = ((q.a3 * x + q.a2) * x + q.a1) * x - q.c;
        const U fp = (a3x3 * x + a2x2) * x + q.a1;
        if (f < U(0)) lo = x; else hi = x;
        U xn = x - m::div(f, fp);
        // inclusive: at convergence the step vanishes and xn lands on the end
        // of the bracket that x just became
        const bool newton = xn >= lo && xn <= hi;
        if (!newton) xn = U(0.5) * (lo + hi);   // safeguard: bisect
        const U step = m::fabs(xn - x);
        x = xn;
        // a small Newton step bounds the error (quadratic convergence); a
        // bisection step does not, so only the bracket width ends it then
        if ((newton && step <= tol) || hi - lo <= tol) break;
    }
    return T(q.base + x);
}

// ---------------------------------------------------------------------------
// Nested intervals (Sec. 2.5).  Cases (5), (2) closed form, case (1) by cube
// root, as printed.  Cases (3) and (4) by bisection of the shifted cubic on
// the case's own bracket ([n2, min(n3, n1 + n2)] or [n3, S/2] in d; the case
// is decided by one evaluation at d = n3, where the printed version bisects
// the first bracket and then the second).  A fixed count of halvings (24 in
// FP32, 52 in FP64) replaces the printed exponent-based count, so all lanes of
// a wavefront run the same trip count; the midpoint of the last interval is
// returned.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool closed_nested(T n1, T n2, T n3, T V, T& d, Open<T>& o) {
    if (closed_case(n1, n2, n3, V, d)) return true;
    o = Open<T>{n1, n2, n3, V};
    return false;
}

template <class T, class U>
__device__ __forceinline__ T cubic_nested(const Open<T>& o) {
    const Cubic<U> q = cubic_setup<T, U>(o);
    U lo = q.lo;
    const U w0 = U(0.5) * (q.hi - q.lo);
    // the i-th half width is w0 2^-i exactly, a constant multiple of w0 once
    // the loop is unrolled, so each midpoint is one fused multiply-add
    U s = U(1);
#pragma unroll
    for (int i = 0; i < M<T>::bisect_steps; ++i) {
        const U mid = w0 * s + lo;
        const U h = ((q.a3 * mid + q.a2) * mid + q.a1) * mid;
        lo = h < q.c ? mid : lo;
        s *= U(0.5);
    }
    return T(q.base + (w0 * s + lo));
}

// ---------------------------------------------------------------------------
// The SZ solution as implemented by Kawano (Sec. 2.4): the unoptimized variant
// of the paper's comparison, kept with its own choices.  The normal is
// L1-normalized (m, sorted m1 <= m2 <= m3 with the middle one taken as
// 1 - m1 - m3), the offset alpha is measured from the cube corner, and the
// reduced volume is the printed w = 1/2 - |V0 - 1/2|.  The cases are tested
// (1), (2), then (5), (3), (4); alpha = 0 is read as "not settled", so an axis
// normal at V0 in {0, 1}, whose case-(5) root is 0, goes on to the cubic of
// case (4) and returns NaN (Sec. 2.6).  V1 (the volume at alpha = m1) carries
// a tiny 1e-25 in its denominator.  The cubic cases take the third real root
// of the monic cubic alpha^3 + a2 alpha^2 + a1 alpha + a0 in trigonometric
// form, through acos and cos.  The open problem carries (m1, m2, m3, w).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool closed_kawano(const Reduced<T>& r, T& alpha, Open<T>& o) {
    using m = M<T>;
    const T il = m::rcp(r.n1 + r.n2 + r.n3);
    const T m1 = r.n1 * il, m3 = r.n3 * il, m2 = m::fmax(T(1) - (m1 + m3), T(0));
    const T w = T(0.5) - m::fabs(r.V0 - T(0.5));
    const T v1 = m::div(m1 * m1, T(6) * m2 * m3 + T(1e-25));
    o = Open<T>{m1, m2, m3, w};
    if (w < v1) {                                                         // case (1)
        alpha = m::cbrt(T(6) * m1 * m2 * m3 * w);
        return true;
    }
    if (w < v1 + m::div(T(0.5) * (m2 - m1), m3)) {                        // case (2)
        alpha = T(0.5) * (m1 + m::sqrt(m1 * m1 + T(8) * m2 * m3 * (w - v1)));
        return true;
    }
    const T m12 = m1 + m2;
    if (!(m3 < m12)) {                                                    // no case (4)
        alpha = m3 * w + T(0.5) * m12;
        if (T(0.5) * m::div(m12, m3) <= w && alpha != T(0)) return true;  // case (5), unless alpha = 0
    }
    return false;
}

template <class T, class U>
__device__ __forceinline__ T cubic_kawano(const Open<T>& o) {
    using m = M<U>;
    const U m1 = o.n1, m2 = o.n2, m3 = o.n3, w = o.V, m12 = m1 + m2;
    const U s1 = m1 * m1, s2 = m2 * m2, w6 = U(6) * m1 * m2 * m3 * w;
    // volume at alpha = m3 (case (4) exists), else at alpha = m1 + m2
    const U v3 = m3 < m12 ? m::div(m3 * m3 * (U(3) * m12 - m3) + s1 * (m1 - U(3) * m3) + s2 * (m2 - U(3) * m3),
                                   U(6) * m1 * m2 * m3)
                          : U(0.5) * m::div(m12, m3);
    U a2, a1, a0;
    if (w < v3) {                                                         // case (3)
        a2 = U(-3) * m12;
        a1 = U(3) * (s1 + s2);
        a0 = w6 - s1 * m1 - s2 * m2;
    } else {                                                              // case (4)
        a2 = U(-1.5);
        a1 = U(1.5) * (s1 + s2 + m3 * m3);
        a0 = U(0.5) * (w6 - s1 * m1 - s2 * m2 - m3 * m3 * m3);
    }
    const U q0 = (a1 * a2 - U(3) * a0) * U(1.0 / 6.0) - a2 * a2 * a2 * U(1.0 / 27.0);
    const U sp = m::sqrt(a2 * a2 * U(1.0 / 9.0) - a1 * U(1.0 / 3.0));  // NaN below 0: the axis edge case
    const U ang = U(4.18879020478639098461) + m::acos(m::div(q0, sp * sp * sp)) * U(1.0 / 3.0);  // 4 pi / 3 + ...
    return T(U(2) * sp * m::cos(ang) - a2 * U(1.0 / 3.0));
}

// ---- the two stages per solver --------------------------------------------------
// Units of the solver: SZ works on the L1-normalized normal, the others on |n|.
template <int SOLVER, class T>
__device__ __forceinline__ T solver_scale(const Reduced<T>& r) {
    if constexpr (SOLVER == kSZ) return r.n1 + r.n2 + r.n3;
    else return T(1);
}

// closed stage on the reduced problem: true with d (solver units) set, or
// false with the open problem in o
template <int SOLVER, class T>
__device__ __forceinline__ bool closed_stage(const Reduced<T>& r, T& d, Open<T>& o) {
    if constexpr (SOLVER == kKawano) {
        return closed_kawano(r, d, o);
    } else if constexpr (SOLVER == kSZ) {
        const T l = r.n1 + r.n2 + r.n3, il = M<T>::rcp(l);
        const T n1 = r.n1 * il, n2 = r.n2 * il, n3 = r.n3 * il;
        if (closed_case(n1, n2, n3, r.V, d)) return true;
        o = Open<T>{n1, n2, n3, r.V};
        return false;
    } else if constexpr (SOLVER == kNewton) {
        return closed_newton(r.n1, r.n2, r.n3, r.V, d, o);
    } else if constexpr (SOLVER == kNested) {
        return closed_nested(r.n1, r.n2, r.n3, r.V, d, o);
    } else {
        if (closed_case(r.n1, r.n2, r.n3, r.V, d)) return true;
        o = Open<T>{r.n1, r.n2, r.n3, r.V};
        return false;
    }
}

template <int SOLVER, class T, class U>
__device__ __forceinline__ T cubic_root(const Open<T>& o) {
    if constexpr (SOLVER == kKawano) return cubic_kawano<T, U>(o);
    else if constexpr (SOLVER == kSZ) return cubic_sz<T, U>(o);
    else if constexpr (SOLVER == kNewton) return cubic_newton<T, U>(o);
    else if constexpr (SOLVER == kNested) return cubic_nested<T, U>(o);
    else return cubic_analytic<T, U>(o);
}

// ---------------------------------------------------------------------------
// The FP64 island of the mixed precision mode (FP32 bulk, U = double).  The
// cubic stage runs in FP32; a root that lands within kIslandWidth * S of a
// case boundary (d = n1, n2, n3 or n1 + n2 in the solver's units), where the
// FP32 a-priori tests may have picked the neighbouring case, is re-solved on
// the cubic of the case that FP64 selects: one Newton step in FP64 from the
// FP32 root, kept inside that case's bracket.  The FP32 root is within
// rounding of the answer (both cases' roots meet at the boundary), so one
// step leaves an error of order (FP32 error)^2; the step's quotient needs no
// FP64 division (the FP32 reciprocal of the slope errs by 1 ulp, times a step
// of FP32 size).  Elsewhere the FP32 root stands.  Kawano's form keeps its
// whole cubic stage in FP64 (its variables do not map onto the shifted cubic).
// ---------------------------------------------------------------------------
constexpr float kIslandWidth = 1.0f / 65536.0f;

template <class T>
__device__ __forceinline__ bool near_case_boundary(const Open<T>& o, T d) {
    using m = M<T>;
    const T w = (o.n1 + o.n2 + o.n3) * T(kIslandWidth);
    const T gap = m::fmin(m::fmin(m::fabs(d - o.n1), m::fabs(d - o.n2)),
                          m::fmin(m::fabs(d - o.n3), m::fabs(d - (o.n1 + o.n2))));
    return gap <= w;
}

template <class T>
__device__ __forceinline__ T island_refine(const Open<T>& o, T d) {
    using m = M<double>;
    const Cubic<double> q = cubic_setup<T, double>(o);
    const double x = m::fmin(m::fmax(double(d) - q.base, q.lo), q.hi);
    const double f = ((q.a3 * x + q.a2) * x + q.a1) * x - q.c;
    const double fp = (3.0 * q.a3 * x + 2.0 * q.a2) * x + q.a1;
    // a vanishing slope (case (1) at t = 0, or below FP32's normal range)
    // leaves the iterate where it is
    const float fpf = float(fp);
    const double step = fpf >= FLT_MIN ? f * double(__builtin_amdgcn_rcpf(fpf)) : 0.0;
    return T(q.base + m::fmin(m::fmax(x - step, q.lo), q.hi));
}

template <int SOLVER, class T, class U>
__device__ __forceinline__ T cubic_stage(const Open<T>& o) {
    constexpr bool island = sizeof(T) < sizeof(U) && SOLVER != kKawano;
    if constexpr (island) {
        const T d = cubic_root<SOLVER, T, T>(o);
        return near_case_boundary(o, d) ? island_refine(o, d) : d;
    } else {
        return cubic_root<SOLVER, T, U>(o);
    }
}

// d0 from the solver's reduced root: sign(V0 - 1/2) (S/2 - d), or for Kawano's
// form l (1/2 - alpha) with the sign of V0 - 1/2
template <int SOLVER, class T>
__device__ __forceinline__ T finish(const Reduced<T>& r, T d, T nx, T ny, T nz, T V0raw) {
    if constexpr (SOLVER == kKawano) {
        T d0 = (r.n1 + r.n2 + r.n3) * __builtin_copysign(T(0.5) - d, r.V0 - T(0.5));
        if (__builtin_isnan(nx + ny + nz + V0raw) || !(r.n3 > T(0))) d0 = M<T>::nan_v;
        return d0;
    } else {
        return unreduce(r, d * solver_scale<SOLVER>(r), nx, ny, nz, V0raw);
    }
}

// full problem: (n, V0) -> d0 with the chosen solver, one thread per problem
template <int SOLVER, class T, class U>
__device__ __forceinline__ T offset(T nx, T ny, T nz, T V0) {
    const Reduced<T> r = reduce(nx, ny, nz, V0);
    T d;
    Open<T> o;
    if (!closed_stage<SOLVER>(r, d, o)) d = cubic_stage<SOLVER, T, U>(o);
    return finish<SOLVER>(r, d, nx, ny, nz, V0);
}

// ---------------------------------------------------------------------------
// Forward volume (Sec. 2.2, the inverse PLIC problem), case (5) tested first
// as in the paper's inverse listing; cases (2)-(4) in the divided form (no
// cancellation, no division by n1 in case (2)).  d0 outside [-S/2, S/2] gives
// 0 or 1.  Case (5) is n1 + n2 <= d <= n3: the printed min(n1 + n2, n3) <= d
// admits the single point d = n3 when n3 < n1 + n2, where the case-(5)
// formula is wrong and the general form holds.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T volume(T nx, T ny, T nz, T d0) {
    using m = M<T>;
    const T ax = m::fabs(nx), ay = m::fabs(ny), az = m::fabs(nz);
    const T n1 = m::fmin(m::fmin(ax, ay), az), n3 = m::fmax(m::fmax(ax, ay), az);
    const T n2 = m::med3(ax, ay, az);
    const T n12 = n1 + n2;
    const T d = m::fmax(T(0.5) * (n12 + n3) - m::fabs(d0), T(0));
    T V;
    if (n12 <= d && d <= n3) {
        V = m::div(d - T(0.5) * n12, n3);                                // case (5)
    } else if (d < n1) {
        V = m::div(d * d * d, T(6) * n1 * n2 * n3);                       // case (1)
    } else {
        T g = T(3) * d * (d - n1) + n1 * n1;                              // case (2)
        if (d > n2) {                                                     // cases (3), (4)
            const T p2 = d - n2, p3 = m::fmax(d - n3, T(0));
            g -= m::div(p2 * p2 * p2 + p3 * p3 * p3, n1);
        }
        V = m::div(g, T(6) * n2 * n3);
    }
    T V0 = __builtin_copysign(T(0.5) - V, d0) + T(0.5);
    if (__builtin_isnan(nx + ny + nz + d0) || !(n3 > T(0))) V0 = m::nan_v;
    return V0;
}

// ---------------------------------------------------------------------------
// Derivatives of d0(n, V0).  With F(a, u) the reduced volume of the corner
// region {z in [0,1]^3 : a.z <= u} (a = sorted |n|, u = reduced d):
//   dV/du = A/|n|  and  dV/da_j = -(A/|n|) * zbar_j,
// A the area and zbar the centroid (corner coordinates) of the polygon, so
//   dd0/dV0 = 1 / F_u  and  zbar_j = -F_aj / F_u.
// F_u and F_aj come from differentiating the five-case volume of Sec. 2.2
// (divided forms, no cancellation):
//   case (5):  F_u = 1/a3,               zbar = (1/2, 1/2, F)
//   case (1):  F_u = u^2 / (2 a1 a2 a3),  zbar_j = u / (3 a_j)
//   (2)-(4):   G = 3u(u-a1) + a1^2 - (P2^3+P3^3)/a1,  Gu = 6u - 3a1 - 3(P2^2+P3^2)/a1,
//              F_u = Gu / (6 a2 a3),
//              zbar1 = (3u - 2a1 - (P2^3+P3^3)/a1^2) / Gu,
//              zbar2 = (G/a2 - 3 P2^2/a1) / Gu,  zbar3 = (G/a3 - 3 P3^2/a1) / Gu,
//              with P_j = max(u - a_j, 0) (case (2): P2 = P3 = 0, valid for a1 = 0).
// The centroid in cube-centred coordinates is mapped back through the sort and
// the sign of each component, and mirrored when V0 > 1/2.
// Returns dd0/dV0 (+inf for a degenerate polygon) and writes dd0/dn.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T offset_grad_from_d0(T nx, T ny, T nz, T V0, T d0, T g[3]) {
    using m = M<T>;
    const T ax = m::fabs(nx), ay = m::fabs(ny), az = m::fabs(nz);
    // sort with the permutation: rank of each component (stable on ties)
    const int rx = (ax > ay) + (ax > az);
    const int ry = (ay >= ax) + (ay > az);
    const int rz = (az >= ax) + (az >= ay);
    const T n1 = m::fmin(m::fmin(ax, ay), az), n3 = m::fmax(m::fmax(ax, ay), az);
    const T n2 = m::med3(ax, ay, az);
    const T u = m::fmax(T(0.5) * (n1 + n2 + n3) - m::fabs(d0), T(0));
    // one reciprocal per component, shared by the cases
    const T r1 = m::rcp(n1), r2 = m::rcp(n2), r3 = m::rcp(n3);
    T z1, z2, z3, Fu;
    if (n1 + n2 <= u && u <= n3) {                                        // case (5)
        Fu = r3;
        z1 = T(0.5); z2 = T(0.5);
        z3 = (u - T(0.5) * (n1 + n2)) * r3;
    } else if (u < n1) {                                                  // case (1)
        const T t = u * T(1.0 / 3.0);
        Fu = T(0.5) * u * u * r1 * r2 * r3;
        z1 = t * r1; z2 = t * r2; z3 = t * r3;
    } else {                                                              // cases (2)-(4)
        const T P2 = m::fmax(u - n2, T(0)), P3 = m::fmax(u - n3, T(0));
        // 1/a1 only where a corner is cut off (P2 > 0, hence a1 > 0); case (2)
        // has no such term, also for a1 = 0
        const T k1 = P2 > T(0) ? r1 : T(0);
        const T c3 = (P2 * P2 * P2 + P3 * P3 * P3) * k1;
        const T G = T(3) * u * (u - n1) + n1 * n1 - c3;
        const T Gu = T(6) * u - T(3) * n1 - T(3) * (P2 * P2 + P3 * P3) * k1;
        Fu = Gu * T(1.0 / 6.0) * r2 * r3;
        if (Gu > T(0)) {
            const T iG = m::rcp(Gu);
            z1 = (T(3) * u - T(2) * n1 - c3 * k1) * iG;
            z2 = (G * r2 - T(3) * P2 * P2 * k1) * iG;
            z3 = (G * r3 - T(3) * P3 * P3 * k1) * iG;
        } else {                                      // u = 0 with a1 = 0: an edge
            z1 = T(0.5); z2 = T(0); z3 = T(0);
        }
    }
    // selects, not an indexed array (which would live in scratch memory)
    auto pick = [&](int k) { return k == 0 ? z1 : (k == 1 ? z2 : z3); };
    // x_k = sign(n_k) (z_rank(k) - 1/2), mirrored through the centre for V0 > 1/2
    const T mir = V0 > T(0.5) ? T(-1) : T(1);
    g[0] = mir * __builtin_copysign(T(1), nx) * (pick(rx) - T(0.5));
    g[1] = mir * __builtin_copysign(T(1), ny) * (pick(ry) - T(0.5));
    g[2] = mir * __builtin_copysign(T(1), nz) * (pick(rz) - T(0.5));
    return Fu > T(0) ? m::rcp(Fu) : T(__builtin_inf());
}

// ---------------------------------------------------------------------------
// Plane-sphere intersection (Sec. 3): a sphere of unit volume, radius
// r = (3 / (4 pi))^(1/3); d0 is the signed distance of the plane from the
// centre and V0 the volume on the side n.x <= d0 (the normal does not matter).
// Forward: the spherical cap (pi/3) (r + d0)^2 (2r - d0), 0 / 1 beyond +-r.
// Inverse, as printed: d0 = (6/pi)^(1/3) sin(pi/6 - atan2(2 sqrt(V0 - V0^2),
// 2 V0 - 1) / 3); with x = 2 V0 - 1 < 0 the angle is pi - atan(y / |x|), so the
// sine's argument stays in [-pi/6, pi/6].  V0 is clamped to [0, 1]; NaN stays NaN.
// ---------------------------------------------------------------------------
template <class T> struct SphereConst;
template <> struct SphereConst<float> {
    static constexpr float r = 0.62035049089940001667f, two_r = 1.2407009817988000333f, pi3 = 1.0471975511965977462f;
};
template <> struct SphereConst<double> {
    static constexpr double r = 0.62035049089940001667, two_r = 1.2407009817988000333, pi3 = 1.0471975511965977462;
};

template <class T>
__device__ __forceinline__ T sphere_offset(T V0) {
    using m = M<T>;
    const T v = m::fmin(m::fmax(V0, T(0)), T(1));
    const T y = T(2) * m::sqrt(v * (T(1) - v));
    const T x = T(2) * v - T(1);
    const T theta = x >= T(0) ? m::atan2_pos(y, x) : T(3.14159265358979323846) - m::atan2_pos(y, -x);
    T d0 = SphereConst<T>::two_r * m::sin_small(T(0.52359877559829887308) - theta * (T(1) / T(3)));
    if (__builtin_isnan(V0)) d0 = V0;
    return d0;
}

template <class T>
__device__ __forceinline__ T sphere_volume(T d0) {
    const T r = SphereConst<T>::r;
    const T h = r + d0;
    T V = SphereConst<T>::pi3 * h * h * (T(2) * r - d0);
    V = d0 <= -r ? T(0) : (d0 >= r ? T(1) : V);
    if (__builtin_isnan(d0)) V = d0;
    return V;
}

}  // namespace plic
