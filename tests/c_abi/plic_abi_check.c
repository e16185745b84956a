/*
 * The C ABI used from plain C, without Python: device buffers from
 * hipMalloc, a stream of the caller's own, and the entry points of plic.h.
 *
 * Inputs are a deterministic sweep (normals on a grid of polar and azimuthal
 * angles, fill levels j / (L - 1)).  The program checks what holds without a
 * reference: the round trip V(n, d0(n, V0)) = V0 to 2e-6 for every solver,
 * the complement d0(n, 1 - V0) = -d0(n, V0), the curvature of a plane of
 * fill levels (zero) and of a lattice without interface (zero), and the
 * status codes of rejected calls.  Exit status 0 means every check passed.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "plic.h"

#define CHECK_HIP(x)                                                             \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));       \
            return 2;                                                            \
        }                                                                        \
    } while (0)

#define CHECK(cond, ...)                                                         \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, __VA_ARGS__);                                        \
            fprintf(stderr, "\n");                                               \
            return 1;                                                            \
        }                                                                        \
    } while (0)

enum { NA = 37, NB = 53, L = 65, N = NA * NB * L };

int main(void) {
    float *h[4], *hd, *hv;
    int i;
    for (i = 0; i < 4; ++i) h[i] = (float *)malloc(sizeof(float) * N);
    hd = (float *)malloc(sizeof(float) * N);
    hv = (float *)malloc(sizeof(float) * N);
    for (int a = 0; a < NA; ++a)
        for (int b = 0; b < NB; ++b)
            for (int j = 0; j < L; ++j) {
                const double th = 3.14159265358979323846 * (a + 0.5) / NA;
                const double ph = 2.0 * 3.14159265358979323846 * b / NB;
                const int k = (a * NB + b) * L + j;
                h[0][k] = (float)(sin(th) * cos(ph));
                h[1][k] = (float)(sin(th) * sin(ph));
                h[2][k] = (float)cos(th);
                h[3][k] = (float)j / (float)(L - 1);   /* 0 and 1 included, 1 - V0 exact */
            }
    printf("libplic %s\n", plic_version());

    hipStream_t st;
    CHECK_HIP(hipStreamCreate(&st));
    float *d[4], *dd, *dv, *dc;
    for (i = 0; i < 4; ++i) {
        CHECK_HIP(hipMalloc((void **)&d[i], sizeof(float) * N));
        CHECK_HIP(hipMemcpyAsync(d[i], h[i], sizeof(float) * N, hipMemcpyHostToDevice, st));
    }
    CHECK_HIP(hipMalloc((void **)&dd, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dv, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dc, sizeof(float) * N));

    const int solvers[4] = {PLIC_ANALYTIC, PLIC_SZ, PLIC_NEWTON, PLIC_NESTED};
    for (int s = 0; s < 4; ++s) {
        int rc = plic_offset_f32(d[0], d[1], d[2], d[3], dd, N, solvers[s], PLIC_FP32, st);
        CHECK(rc == PLIC_OK, "plic_offset_f32: %s", plic_status_string(rc));
        rc = plic_volume_f32(d[0], d[1], d[2], dd, dv, N, PLIC_FP32, st);
        CHECK(rc == PLIC_OK, "plic_volume_f32: %s", plic_status_string(rc));
        CHECK_HIP(hipMemcpyAsync(hd, dd, sizeof(float) * N, hipMemcpyDeviceToHost, st));
        CHECK_HIP(hipMemcpyAsync(hv, dv, sizeof(float) * N, hipMemcpyDeviceToHost, st));
        CHECK_HIP(hipStreamSynchronize(st));
        double worst = 0.0, worst_c = 0.0;
        for (i = 0; i < N; ++i) {
            const double e = fabs((double)hv[i] - (double)h[3][i]);
            if (!(e <= worst)) worst = e;
        }
        /* complement: V0 = j/(L-1) and 1 - V0 = (L-1-j)/(L-1) sit in the same sweep */
        for (int k0 = 0; k0 < NA * NB; ++k0)
            for (int j = 0; j < L; ++j) {
                const double e = fabs((double)hd[k0 * L + j] + (double)hd[k0 * L + (L - 1 - j)]);
                if (!(e <= worst_c)) worst_c = e;
            }
        printf("solver %d: max |V(d0) - V0| = %.2e, max |d0(1-V0) + d0(V0)| = %.2e\n", solvers[s], worst, worst_c);
        CHECK(worst <= 2e-6, "round trip too large for solver %d", solvers[s]);
        CHECK(worst_c <= 2e-6, "complement too large for solver %d", solvers[s]);
    }

    /* curvature: a plane of fill levels along z (kappa = 0) and a lattice
     * without interface (kappa = 0), through a workspace of the recommended size */
    {
        const int X = 64, Y = 16, Z = 16, n = X * Y * Z;
        float *hp = (float *)malloc(sizeof(float) * n), *hk = (float *)malloc(sizeof(float) * n);
        for (int z = 0; z < Z; ++z)
            for (int y = 0; y < Y; ++y)
                for (int x = 0; x < X; ++x) hp[(z * Y + y) * X + x] = z < 7 ? 1.0f : (z == 7 ? 0.3f : 0.0f);
        const size_t wsb = plic_curvature_workspace_bytes(X, Y, Z);
        float *dp, *dk;
        void *ws;
        CHECK_HIP(hipMalloc((void **)&dp, sizeof(float) * n));
        CHECK_HIP(hipMalloc((void **)&dk, sizeof(float) * n));
        CHECK_HIP(hipMalloc(&ws, wsb));
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1)
                for (i = 0; i < n; ++i) hp[i] = hp[i] > 0.5f ? 1.0f : 0.0f;   /* no interface */
            CHECK_HIP(hipMemcpyAsync(dp, hp, sizeof(float) * n, hipMemcpyHostToDevice, st));
            int rc = plic_curvature_f32(dp, X, Y, Z, dk, PLIC_ANALYTIC, PLIC_MIXED, ws, wsb, st);
            CHECK(rc == PLIC_OK, "plic_curvature_f32: %s", plic_status_string(rc));
            CHECK_HIP(hipMemcpyAsync(hk, dk, sizeof(float) * n, hipMemcpyDeviceToHost, st));
            CHECK_HIP(hipStreamSynchronize(st));
            double kmax = 0.0;
            for (i = 0; i < n; ++i)
                if (!(fabs(hk[i]) <= kmax)) kmax = fabs(hk[i]);
            printf("curvature %s: max |kappa| = %.2e\n", pass ? "without interface" : "of a plane", kmax);
            CHECK(kmax <= 1e-6, "curvature of a plane / empty lattice not zero");
            /* the call's interface-cell count: the plane z = 7 away from the
             * outer layer, 62 x 14 cells */
            int64_t cells = -1;
            size_t need = 0;
            rc = plic_curvature_status(ws, wsb, X, Y, Z, 0, &cells, &need, st);
            CHECK(rc == PLIC_OK, "plic_curvature_status: %s", plic_status_string(rc));
            CHECK(cells == (pass ? 0 : 62 * 14), "interface cells %lld", (long long)cells);
            /* the recommended size holds 16 rows in each of the 16 tiles */
            CHECK(need + 256 * 108 == wsb + (size_t)cells * 108, "bytes for all rows %zu", need);
        }
        /* rejected calls enqueue nothing and say why */
        int rc = plic_curvature_f32(dp, X, Y, Z, dk, PLIC_ANALYTIC, PLIC_MIXED, ws, 16, st);
        CHECK(rc == PLIC_EWORKSPACE, "workspace below the fixed part accepted");
        rc = plic_offset_f32(d[0], d[1], d[2], d[3], dd, -1, PLIC_SZ, PLIC_FP32, st);
        CHECK(rc == PLIC_EINVAL, "negative count accepted");
        rc = plic_offset_f32(d[0], d[1], d[2], d[3], dd, N, 17, PLIC_FP32, st);
        CHECK(rc == PLIC_EINVAL, "bad solver accepted");
        printf("rejected calls: %s\n", plic_status_string(rc));
        CHECK_HIP(hipFree(ws));
        CHECK_HIP(hipFree(dk));
        CHECK_HIP(hipFree(dp));
        free(hp);
        free(hk);
    }
    for (i = 0; i < 4; ++i) CHECK_HIP(hipFree(d[i]));
    CHECK_HIP(hipFree(dd));
    CHECK_HIP(hipFree(dv));
    CHECK_HIP(hipFree(dc));
    CHECK_HIP(hipStreamDestroy(st));
    printf("C ABI OK\n");
    return 0;
}
