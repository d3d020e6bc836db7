/*
 * Drives every entry point of the FP64 oracle on small ragged volumes, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (the CPU test
 * suite compiles and runs it). Exits 0 when every result is finite and the
 * calls report success; the sanitizers abort on any invalid access, leak or
 * undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "disc_oracle.h"

static unsigned long long rng = 0x9E3779B97F4A7C15ull;

static double uniform(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double* v, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    const int nx = 13, ny = 11, nz = 9;
    const long n = (long)nx * ny * nz;
    double* ct = malloc(n * sizeof(double));
    double* cb = malloc(n * sizeof(double));
    double* s = malloc(n * sizeof(double));
    double* r = calloc(3 * n, sizeof(double));
    double* m = malloc(n * sizeof(double));
    double* mu_m = malloc(n * sizeof(double));
    double* var_m = malloc(n * sizeof(double));
    double* mu_s = malloc(n * sizeof(double));
    double* var_s = malloc(n * sizeof(double));
    double* a = malloc(n * sizeof(double));
    double* b = malloc(n * sizeof(double));
    double* f = malloc(n * sizeof(double));
    double* u = malloc(3 * n * sizeof(double));
    double* g = malloc(3 * n * sizeof(double));
    double* A = malloc(n * sizeof(double));
    double* B = malloc(n * sizeof(double));
    unsigned char* xi = malloc(n);
    unsigned char* valid = malloc(n);
    unsigned char* pass_of = malloc(n);
    for (long i = 0; i < n; ++i) {
        ct[i] = -1000.0 + 2000.0 * uniform();
        cb[i] = 0.9 * ct[i] + 50.0 + 20.0 * uniform();
    }
    for (long i = 0; i < 3 * n; ++i) r[i] = 1.5 * (uniform() - 0.5);

    orc_set_threads(2);
    CHECK(orc_threads() >= 1);
    CHECK(isfinite(orc_mean(ct, n)));
    CHECK(isfinite(orc_global_shift(ct, cb, n, s)) && finite_all(s, n));

    const int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
    double* half = malloc((size_t)cx * cy * cz * sizeof(double));
    double* rc = malloc(3 * (size_t)cx * cy * cz * sizeof(double));
    orc_downsample2(ct, nx, ny, nz, half);
    CHECK(finite_all(half, (long)cx * cy * cz));
    for (long i = 0; i < 3L * cx * cy * cz; ++i) rc[i] = uniform() - 0.5;
    orc_upsample_field(rc, cx, cy, cz, u, nx, ny, nz);
    CHECK(finite_all(u, 3 * n));

    orc_warp(ct, r, nx, ny, nz, m);
    orc_patch_moments(m, nx, ny, nz, 5, 3, 7, mu_m, var_m);
    orc_patch_moments(s, nx, ny, nz, 5, 3, 7, mu_s, var_s);
    orc_correct(mu_m, var_m, mu_s, var_s, s, n, 1e-2, a, b, f);
    CHECK(finite_all(f, n));
    orc_force(m, f, nx, ny, nz, 1e-3, u);
    CHECK(finite_all(u, 3 * n));
    orc_force_double(m, f, nx, ny, nz, 1e-3, u);
    CHECK(finite_all(u, 3 * n));
    double w[2 * 64 + 1];
    CHECK(orc_gauss_taps(1.5, w) == 5 && orc_gauss_taps(0.0, w) == -1);
    orc_gauss(m, nx, ny, nz, 1.5, a);
    CHECK(finite_all(a, n));

    const int t[3] = {3, 5, 1};
    CHECK(orc_mask_fill(m, s, mu_m, var_m, mu_s, var_s, nx, ny, nz, 1e-2, 30.0, 0.5, 1.5, 30.0, t, 4, A, B,
                        xi) >= 0);
    CHECK(finite_all(A, n) && finite_all(B, n));
    for (long i = 0; i < n; ++i) valid[i] = (unsigned char)(uniform() < 0.3);
    orc_correct(mu_m, var_m, mu_s, var_s, s, n, 1e-2, a, b, f);
    CHECK(orc_fill(a, b, valid, s, nx, ny, nz, 30.0, t, 3, A, B) >= 0);
    CHECK(orc_fill_ex(a, b, valid, s, nx, ny, nz, 30.0, t, 3, A, B, pass_of) >= 0);
    CHECK(isfinite(orc_a_median(ct, s, nx, ny, nz, 3, 3, 3, 1e-2)));

    orc_params p;
    memset(&p, 0, sizeof p);
    p.patch[0] = 3; p.patch[1] = 5; p.patch[2] = 3;
    p.sigma = 1.0;
    p.levels = 2;
    p.iters[0] = 3; p.iters[1] = 4;
    p.global_shift = 1;
    p.var_floor = 1e-2;
    p.diff_floor = 1e-3;
    p.stop_lag = 2;
    p.stop_eps = 1e-3;
    p.a_lo = 0.5; p.a_hi = 1.5;
    p.fill_t[0] = 3; p.fill_t[1] = 3; p.fill_t[2] = 1;
    p.fill_passes = 3;
    orc_iterate(ct, s, mu_s, var_s, r, nx, ny, nz, &p, m, f, u);
    CHECK(finite_all(r, 3 * n));
    double* rout = malloc(3 * n * sizeof(double));
    CHECK(orc_register(ct, cb, nx, ny, nz, &p, rout, f) == 0 && finite_all(rout, 3 * n));
    int done[8];
    double hist[2 * 8];
    p.mask_mode = 1;
    p.force_mode = 1;
    CHECK(orc_register_ex(ct, cb, nx, ny, nz, &p, rout, f, done, hist, 8) == 0 && finite_all(rout, 3 * n));
    p.levels = 0;
    CHECK(orc_register(ct, cb, nx, ny, nz, &p, rout, f) == -1);

    /* point evaluators on FP32 state */
    float* ct32 = malloc(n * sizeof(float));
    float* s32 = malloc(n * sizeof(float));
    float* r32 = malloc(3 * n * sizeof(float));
    for (long i = 0; i < n; ++i) {
        ct32[i] = (float)ct[i];
        s32[i] = (float)s[i];
    }
    for (long i = 0; i < 3 * n; ++i) r32[i] = (float)r[i];
    const long pts[4] = {0, n / 3, n / 2, n - 1};
    double out[4 * 3];
    orc_warp_pts(ct32, r32, nx, ny, nz, pts, 4, out);
    orc_correct_pts(ct32, s32, nx, ny, nz, 3, 5, 3, 1e-2, pts, 4, out);
    orc_force_pts(ct32, s32, r32, nx, ny, nz, 1e-3, pts, 4, out);
    orc_gauss_pts(r32, nx, ny, nz, 1.5, pts, 4, out);
    CHECK(finite_all(out, 12));

    CHECK(isfinite(orc_ssd_loss(ct, s, r, nx, ny, nz, 3, 5, 3, 1e-2)));
    orc_ssd_grad(ct, s, r, nx, ny, nz, 3, 5, 3, 1e-2, g);
    CHECK(finite_all(g, 3 * n));
    orc_ssd_grad_pts(ct32, s32, r32, nx, ny, nz, 3, 5, 3, 1e-2, pts, 4, out);
    CHECK(finite_all(out, 12));

    free(ct32); free(s32); free(r32); free(rout); free(half); free(rc);
    free(ct); free(cb); free(s); free(r); free(m); free(mu_m); free(var_m); free(mu_s); free(var_s);
    free(a); free(b); free(f); free(u); free(g); free(A); free(B); free(xi); free(valid); free(pass_of);
    printf("oracle exercise: ok\n");
    return 0;
}
