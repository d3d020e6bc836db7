/*
 * disc_oracle.c -- plain FP64 CPU oracle of DISC (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY: the checker the HIP library is compared against.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does. No code, header or table
 * here is shared with the HIP library.
 *
 * Every step is written the slow, direct way, in FP64, in the order of
 * Algorithm A1 of Zhen et al. (arXiv 1204.6295):
 *   global shift (Sec. 2.3) -> pyramid (Sec. 2.3) -> per level:
 *     warp (Sec. 2.1 model) -> patch moments (Eq. 3) -> a, b (Eq. 5, 6)
 *     -> I'_s = a I_s + b (Sec. 2.2) -> force (Eq. 1, static-gradient term)
 *     -> r := r + dr (A1 step 5) -> Gaussian on r (A1 step 6)
 *   -> up-sample r to the next level (A1).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - field convention m(x) = CT(x + r(x)) (Sec. 2.1), so the A1 update
 *    "add dr" is r := r - u with u the Eq. 1 static-gradient force;
 *  - all stencils (warp corners, patches, gradient, Gaussian, pyramid)
 *    clamp indices to the volume (edge replicate);
 *  - central-difference gradient in intensity per voxel;
 *  - Gaussian taps exp(-k^2 / 2 sigma^2), |k| <= ceil(3 sigma), normalised;
 *  - Eq. 5 divides by STD(S); where var(S) <= tau the static patch is flat,
 *    its spread carries no information and only the first moment of Eq. 4
 *    is matched: a := 1, b := E(M) - E(S). This keeps identical images an
 *    exact fixed point;
 *  - u := 0 where |m - f| < eps_d or the denominator is 0;
 *  - the corrected image is always a * (original shifted CBCT) + b (Sec. 2.2);
 *  - pyramid: 2x2x2 block mean; field up-sampling: 2 * trilinear at
 *    (x + 1/2)/2 - 1/2.
 */
#include "disc_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

int orc_threads(void)
{
    return omp_get_max_threads();
}

/* Number of OpenMP threads of later calls (n >= 1); for timing the oracle
 * at one thread and at all host threads. */
void orc_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
}

static int clampi(int v, int n)
{
    if (v < 0) return 0;
    if (v > n - 1) return n - 1;
    return v;
}

static long lin(int x, int y, int z, int nx, int ny)
{
    return ((long)z * ny + y) * nx + x;
}

double orc_mean(const double* v, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += v[i];
    return s / (double)n;
}

double orc_global_shift(const double* ct, const double* cbct0, long n, double* s)
{
    double dhu = orc_mean(ct, n) - orc_mean(cbct0, n);
    for (long i = 0; i < n; ++i) s[i] = cbct0[i] + dhu;
    return dhu;
}

void orc_downsample2(const double* in, int nx, int ny, int nz, double* out)
{
    int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < cz; ++z)
        for (int y = 0; y < cy; ++y)
            for (int x = 0; x < cx; ++x) {
                double s = 0.0;
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx)
                            s += in[lin(clampi(2 * x + dx, nx), clampi(2 * y + dy, ny),
                                        clampi(2 * z + dz, nz), nx, ny)];
                out[lin(x, y, z, cx, cy)] = s / 8.0;
            }
}

/* Trilinear interpolation at the continuous position (px, py, pz): the eight
 * surrounding voxels weighted by the products of the 1-D linear weights;
 * corner indices are clamped (edge replicate). */
static double trilinear(const double* v, int nx, int ny, int nz,
                        double px, double py, double pz)
{
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    double tx = px - fx, ty = py - fy, tz = pz - fz;
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? tx : 1.0 - tx) * (dy ? ty : 1.0 - ty) * (dz ? tz : 1.0 - tz);
                s += w * v[lin(clampi(ix + dx, nx), clampi(iy + dy, ny), clampi(iz + dz, nz), nx, ny)];
            }
    return s;
}

/* Same as trilinear() but reading an FP32 volume. */
static double trilinear_f(const float* v, int nx, int ny, int nz,
                          double px, double py, double pz)
{
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    double tx = px - fx, ty = py - fy, tz = pz - fz;
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? tx : 1.0 - tx) * (dy ? ty : 1.0 - ty) * (dz ? tz : 1.0 - tz);
                s += w * (double)v[lin(clampi(ix + dx, nx), clampi(iy + dy, ny), clampi(iz + dz, nz), nx, ny)];
            }
    return s;
}

void orc_upsample_field(const double* rc, int cnx, int cny, int cnz,
                        double* rf, int fnx, int fny, int fnz)
{
    long nc = (long)cnx * cny * cnz, nf = (long)fnx * fny * fnz;
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < fnz; ++z)
            for (int y = 0; y < fny; ++y)
                for (int x = 0; x < fnx; ++x) {
                    double px = (x + 0.5) / 2.0 - 0.5;
                    double py = (y + 0.5) / 2.0 - 0.5;
                    double pz = (z + 0.5) / 2.0 - 0.5;
                    rf[c * nf + lin(x, y, z, fnx, fny)] =
                        2.0 * trilinear(rc + c * nc, cnx, cny, cnz, px, py, pz);
                }
    }
}

void orc_warp(const double* ct, const double* r, int nx, int ny, int nz, double* m)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                m[i] = trilinear(ct, nx, ny, nz, x + r[i], y + r[n + i], z + r[2 * n + i]);
            }
}

/* Mean and centred variance of the clamped patch centred at (x, y, z). */
static void patch_at(const double* img, int nx, int ny, int nz,
                     int px, int py, int pz, int x, int y, int z,
                     double* mu, double* var)
{
    int rx = px / 2, ry = py / 2, rz = pz / 2;
    double n = (double)px * py * pz;
    double s = 0.0;
    for (int k = -rz; k <= rz; ++k)
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i)
                s += img[lin(clampi(x + i, nx), clampi(y + j, ny), clampi(z + k, nz), nx, ny)];
    double e = s / n;
    double q = 0.0;
    for (int k = -rz; k <= rz; ++k)
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i) {
                double d = img[lin(clampi(x + i, nx), clampi(y + j, ny), clampi(z + k, nz), nx, ny)] - e;
                q += d * d;
            }
    *mu = e;
    *var = q / n;
}

static void patch_at_f(const float* img, int nx, int ny, int nz,
                       int px, int py, int pz, int x, int y, int z,
                       double* mu, double* var)
{
    int rx = px / 2, ry = py / 2, rz = pz / 2;
    double n = (double)px * py * pz;
    double s = 0.0;
    for (int k = -rz; k <= rz; ++k)
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i)
                s += (double)img[lin(clampi(x + i, nx), clampi(y + j, ny), clampi(z + k, nz), nx, ny)];
    double e = s / n;
    double q = 0.0;
    for (int k = -rz; k <= rz; ++k)
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i) {
                double d = (double)img[lin(clampi(x + i, nx), clampi(y + j, ny), clampi(z + k, nz), nx, ny)] - e;
                q += d * d;
            }
    *mu = e;
    *var = q / n;
}

void orc_patch_moments(const double* img, int nx, int ny, int nz,
                       int px, int py, int pz, double* mu, double* var)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                patch_at(img, nx, ny, nz, px, py, pz, x, y, z, &mu[i], &var[i]);
            }
}

/* Eq. 5 and Eq. 6 for one voxel; a flat static patch (var_s <= tau) matches
 * the mean only (a = 1). */
static void match_moments(double mu_m, double var_m, double mu_s, double var_s,
                          double tau, double* a, double* b)
{
    double av = (var_s > tau) ? sqrt(var_m / var_s) : 1.0;
    *a = av;
    *b = mu_m - av * mu_s;
}

void orc_correct(const double* mu_m, const double* var_m,
                 const double* mu_s, const double* var_s,
                 const double* s, long n, double tau,
                 double* a, double* b, double* f)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double av, bv;
        match_moments(mu_m[i], var_m[i], mu_s[i], var_s[i], tau, &av, &bv);
        if (a) a[i] = av;
        if (b) b[i] = bv;
        f[i] = av * s[i] + bv;
    }
}

/* Eq. 1 static-gradient term at one voxel: d = m - f, g = central-difference
 * gradient of f. Writes the three components of u. */
static void force_from(double d, double gx, double gy, double gz, double eps_d, double u[3])
{
    double den = gx * gx + gy * gy + gz * gz + d * d;
    if (den > 0.0 && fabs(d) >= eps_d) {
        u[0] = d * gx / den;
        u[1] = d * gy / den;
        u[2] = d * gz / den;
    } else {
        u[0] = u[1] = u[2] = 0.0;
    }
}

void orc_force(const double* m, const double* f, int nx, int ny, int nz,
               double eps_d, double* u)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                double gx = (f[lin(clampi(x + 1, nx), y, z, nx, ny)] - f[lin(clampi(x - 1, nx), y, z, nx, ny)]) / 2.0;
                double gy = (f[lin(x, clampi(y + 1, ny), z, nx, ny)] - f[lin(x, clampi(y - 1, ny), z, nx, ny)]) / 2.0;
                double gz = (f[lin(x, y, clampi(z + 1, nz), nx, ny)] - f[lin(x, y, clampi(z - 1, nz), nx, ny)]) / 2.0;
                double uu[3];
                force_from(m[i] - f[i], gx, gy, gz, eps_d, uu);
                u[i] = uu[0];
                u[n + i] = uu[1];
                u[2 * n + i] = uu[2];
            }
}

/* Eq. 1 first term plus its second (moving-gradient) term. */
void orc_force_double(const double* m, const double* f, int nx, int ny, int nz,
                      double eps_d, double* u)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                double d = m[i] - f[i];
                double g[2][3];
                const double* img[2] = {f, m};
                for (int t = 0; t < 2; ++t) {
                    const double* v = img[t];
                    g[t][0] = (v[lin(clampi(x + 1, nx), y, z, nx, ny)] - v[lin(clampi(x - 1, nx), y, z, nx, ny)]) / 2.0;
                    g[t][1] = (v[lin(x, clampi(y + 1, ny), z, nx, ny)] - v[lin(x, clampi(y - 1, ny), z, nx, ny)]) / 2.0;
                    g[t][2] = (v[lin(x, y, clampi(z + 1, nz), nx, ny)] - v[lin(x, y, clampi(z - 1, nz), nx, ny)]) / 2.0;
                }
                double uu[3] = {0.0, 0.0, 0.0};
                if (fabs(d) >= eps_d) {
                    for (int t = 0; t < 2; ++t) {
                        double den = g[t][0] * g[t][0] + g[t][1] * g[t][1] + g[t][2] * g[t][2] + d * d;
                        if (den > 0.0)
                            for (int c = 0; c < 3; ++c) uu[c] += d * g[t][c] / den;
                    }
                }
                u[i] = uu[0];
                u[n + i] = uu[1];
                u[2 * n + i] = uu[2];
            }
}

/* ---- Eq. 7-10: mask and fill ------------------------------------------------ */

int orc_fill(const double* a0, const double* b0, const unsigned char* valid0, const double* s,
             int nx, int ny, int nz, double h, const int t[3], int passes, double* A, double* B)
{
    return orc_fill_ex(a0, b0, valid0, s, nx, ny, nz, h, t, passes, A, B, NULL);
}

int orc_fill_ex(const double* a0, const double* b0, const unsigned char* valid0, const double* s,
                int nx, int ny, int nz, double h, const int t[3], int passes, double* A, double* B,
                unsigned char* pass_of)
{
    long n = (long)nx * ny * nz;
    int tx = t[0] / 2, ty = t[1] / 2, tz = t[2] / 2;
    unsigned char* valid = (unsigned char*)malloc(n);
    unsigned char* nvalid = (unsigned char*)malloc(n);
    double* nA = (double*)malloc(sizeof(double) * n);
    double* nB = (double*)malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) {
        valid[i] = valid0[i] ? 1 : 0;
        /* Eq. 7 paragraph: masked voxels start from a = b = 0 */
        A[i] = valid[i] ? a0[i] : 0.0;
        B[i] = valid[i] ? b0[i] : 0.0;
        if (pass_of) pass_of[i] = valid[i] ? 0 : 255;
    }
    int used = 0;
    for (int pass = 0; pass < passes; ++pass) {
        long left = 0;
        for (long i = 0; i < n; ++i) left += !valid[i];
        if (left == 0) break;
        long filled = 0;
#pragma omp parallel for schedule(static) reduction(+ : filled)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long i = lin(x, y, z, nx, ny);
                    nA[i] = A[i];
                    nB[i] = B[i];
                    nvalid[i] = valid[i];
                    if (valid[i]) continue;
                    /* Eq. 9 is a ratio of sums of the Eq. 10 weights, all of which
                     * are positive: dividing every weight by the largest one
                     * (smallest dS^2) leaves it unchanged and keeps it away from
                     * underflow, so any voxel with a valid neighbour is filled */
                    double d2min = INFINITY;
                    for (int k = -tz; k <= tz; ++k)
                        for (int jj = -ty; jj <= ty; ++jj)
                            for (int ii = -tx; ii <= tx; ++ii) {
                                int xx = x + ii, yy = y + jj, zz = z + k;
                                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
                                long q = lin(xx, yy, zz, nx, ny);
                                if (!valid[q]) continue;
                                double ds = s[q] - s[i];
                                if (ds * ds < d2min) d2min = ds * ds;
                            }
                    double sw = 0.0, sa = 0.0, sb = 0.0;
                    for (int k = -tz; k <= tz; ++k)
                        for (int jj = -ty; jj <= ty; ++jj)
                            for (int ii = -tx; ii <= tx; ++ii) {
                                int xx = x + ii, yy = y + jj, zz = z + k;
                                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
                                long q = lin(xx, yy, zz, nx, ny);
                                if (!valid[q]) continue;
                                double ds = s[q] - s[i];
                                double w = exp(-(ds * ds - d2min) / (h * h));
                                sw += w;
                                sa += w * A[q];
                                sb += w * B[q];
                            }
                    if (sw > 0.0) {
                        nA[i] = sa / sw;
                        nB[i] = sb / sw;
                        nvalid[i] = 1;
                        if (pass_of) pass_of[i] = (unsigned char)(pass + 1);
                        filled += 1;
                    }
                }
        memcpy(A, nA, sizeof(double) * n);
        memcpy(B, nB, sizeof(double) * n);
        memcpy(valid, nvalid, n);
        if (filled == 0) break;
        used = pass + 1;
    }
    /* leftover rule: a voxel never filled keeps its Eq. 5-6 values */
    for (long i = 0; i < n; ++i)
        if (!valid[i]) {
            A[i] = a0[i];
            B[i] = b0[i];
        }
    free(valid);
    free(nvalid);
    free(nA);
    free(nB);
    return used;
}

int orc_mask_fill(const double* m, const double* s, const double* mu_m, const double* var_m,
                  const double* mu_s, const double* var_s, int nx, int ny, int nz, double tau,
                  double hu0, double a_min, double a_max, double h, const int t[3], int passes,
                  double* A, double* B, unsigned char* xi)
{
    long n = (long)nx * ny * nz;
    double* a0 = (double*)malloc(sizeof(double) * n);
    double* b0 = (double*)malloc(sizeof(double) * n);
    unsigned char* valid = (unsigned char*)malloc(n);
    for (long i = 0; i < n; ++i) {
        match_moments(mu_m[i], var_m[i], mu_s[i], var_s[i], tau, &a0[i], &b0[i]);
        /* Eq. 7 */
        int masked = fabs(m[i] - s[i]) > hu0 || a0[i] < a_min || a0[i] > a_max;
        valid[i] = !masked;
        if (xi) xi[i] = (unsigned char)masked;
    }
    int used = orc_fill(a0, b0, valid, s, nx, ny, nz, h, t, passes, A, B);
    free(a0);
    free(b0);
    free(valid);
    return used;
}

static int cmp_double(const void* x, const void* y)
{
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

double orc_a_median(const double* ct, const double* s, int nx, int ny, int nz, int px, int py, int pz,
                    double tau)
{
    long n = (long)nx * ny * nz;
    double* buf = (double*)malloc(sizeof(double) * 4 * n);
    double *mu_m = buf, *var_m = buf + n, *mu_s = buf + 2 * n, *var_s = buf + 3 * n;
    orc_patch_moments(ct, nx, ny, nz, px, py, pz, mu_m, var_m);
    orc_patch_moments(s, nx, ny, nz, px, py, pz, mu_s, var_s);
    long cnt = 0;
    for (long i = 0; i < n; ++i)
        if (var_s[i] > tau && var_m[i] > tau) mu_m[cnt++] = sqrt(var_m[i] / var_s[i]); /* mu_m reused as the list */
    double med = 1.0;
    if (cnt > 0) {
        qsort(mu_m, (size_t)cnt, sizeof(double), cmp_double);
        med = (cnt % 2) ? mu_m[cnt / 2] : 0.5 * (mu_m[cnt / 2 - 1] + mu_m[cnt / 2]);
    }
    free(buf);
    return med;
}

int orc_gauss_taps(double sigma, double* w)
{
    if (!(sigma > 0.0)) return -1;
    int R = (int)ceil(3.0 * sigma);
    if (R > 64) return -1;
    double s = 0.0;
    for (int k = -R; k <= R; ++k) {
        w[k + R] = exp(-(double)k * k / (2.0 * sigma * sigma));
        s += w[k + R];
    }
    for (int k = 0; k <= 2 * R; ++k) w[k] /= s;
    return R;
}

void orc_gauss(const double* in, int nx, int ny, int nz, double sigma, double* out)
{
    double w[129];
    int R = orc_gauss_taps(sigma, w);
    long n = (long)nx * ny * nz;
    double* t1 = (double*)malloc(sizeof(double) * n);
    double* t2 = (double*)malloc(sizeof(double) * n);
    /* x pass */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int k = -R; k <= R; ++k) s += w[k + R] * in[lin(clampi(x + k, nx), y, z, nx, ny)];
                t1[lin(x, y, z, nx, ny)] = s;
            }
    /* y pass */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int k = -R; k <= R; ++k) s += w[k + R] * t1[lin(x, clampi(y + k, ny), z, nx, ny)];
                t2[lin(x, y, z, nx, ny)] = s;
            }
    /* z pass */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int k = -R; k <= R; ++k) s += w[k + R] * t2[lin(x, y, clampi(z + k, nz), nx, ny)];
                out[lin(x, y, z, nx, ny)] = s;
            }
    free(t1);
    free(t2);
}

void orc_iterate(const double* ct, const double* s, const double* mu_s,
                 const double* var_s, double* r, int nx, int ny, int nz,
                 const orc_params* p, double* m_out, double* f_out, double* rt_out)
{
    long n = (long)nx * ny * nz;
    double* m = (double*)malloc(sizeof(double) * n);
    double* mu_m = (double*)malloc(sizeof(double) * n);
    double* var_m = (double*)malloc(sizeof(double) * n);
    double* f = (double*)malloc(sizeof(double) * n);
    double* u = (double*)malloc(sizeof(double) * 3 * n);

    /* deformed moving image I_m^(k) */
    orc_warp(ct, r, nx, ny, nz, m);
    /* A1 step 1: patch moments (Eq. 3) and a, b (Eq. 5, 6); step 3: I'_s */
    orc_patch_moments(m, nx, ny, nz, p->patch[0], p->patch[1], p->patch[2], mu_m, var_m);
    if (p->mask_mode == 1) {
        /* Eq. 7-10 (hu0, a range and h already resolved to absolute values) */
        double* A = (double*)malloc(sizeof(double) * n);
        double* B = (double*)malloc(sizeof(double) * n);
        orc_mask_fill(m, s, mu_m, var_m, mu_s, var_s, nx, ny, nz, p->var_floor, p->hu0, p->a_lo, p->a_hi,
                      p->fill_h, p->fill_t, p->fill_passes, A, B, NULL);
        for (long i = 0; i < n; ++i) f[i] = A[i] * s[i] + B[i];
        free(A);
        free(B);
    } else {
        orc_correct(mu_m, var_m, mu_s, var_s, s, n, p->var_floor, NULL, NULL, f);
    }
    /* A1 step 4: Eq. 1 force on I'_s; step 5: add dr = -u to r */
    if (p->force_mode == 1)
        orc_force_double(m, f, nx, ny, nz, p->diff_floor, u);
    else
        orc_force(m, f, nx, ny, nz, p->diff_floor, u);
    for (long i = 0; i < 3 * n; ++i) r[i] -= u[i];
    if (rt_out) memcpy(rt_out, r, sizeof(double) * 3 * n);
    /* A1 step 6: Gaussian on each component of r */
    for (int c = 0; c < 3; ++c) {
        orc_gauss(r + c * n, nx, ny, nz, p->sigma, u + c * n);
        memcpy(r + c * n, u + c * n, sizeof(double) * n);
    }
    if (m_out) memcpy(m_out, m, sizeof(double) * n);
    if (f_out) memcpy(f_out, f, sizeof(double) * n);
    free(m);
    free(mu_m);
    free(var_m);
    free(f);
    free(u);
}

int orc_register(const double* ct, const double* cbct0, int nx, int ny, int nz,
                 const orc_params* p, double* r_out, double* f_out)
{
    int done[8];
    return orc_register_ex(ct, cbct0, nx, ny, nz, p, r_out, f_out, done, NULL, 0);
}

/* Sum over voxels of the Euclidean norm of a field [3][n]. */
static double field_norm_sum(const double* v, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += sqrt(v[i] * v[i] + v[n + i] * v[n + i] + v[2 * n + i] * v[2 * n + i]);
    return s;
}

int orc_register_ex(const double* ct, const double* cbct0, int nx, int ny, int nz,
                    const orc_params* p, double* r_out, double* f_out, int* iters_done,
                    double* l_hist, int hist_stride)
{
    if (!ct || !cbct0 || !p || !r_out || nx < 1 || ny < 1 || nz < 1) return -1;
    if (p->levels < 1 || p->levels > 8 || !(p->sigma > 0.0)) return -1;
    for (int d = 0; d < 3; ++d)
        if (p->patch[d] < 1 || p->patch[d] % 2 == 0) return -1;

    int L = p->levels;
    int dims[8][3];
    double* cts[8];
    double* ss[8];
    long ns[8];
    dims[L - 1][0] = nx;
    dims[L - 1][1] = ny;
    dims[L - 1][2] = nz;
    for (int l = L - 2; l >= 0; --l)
        for (int d = 0; d < 3; ++d) dims[l][d] = (dims[l + 1][d] + 1) / 2;
    for (int l = 0; l < L; ++l) ns[l] = (long)dims[l][0] * dims[l][1] * dims[l][2];

    /* A1: globally adjust the CBCT intensity (Sec. 2.3) */
    long n = ns[L - 1];
    cts[L - 1] = (double*)malloc(sizeof(double) * n);
    ss[L - 1] = (double*)malloc(sizeof(double) * n);
    memcpy(cts[L - 1], ct, sizeof(double) * n);
    double dhu = orc_mean(ct, n) - orc_mean(cbct0, n);
    if (p->global_shift)
        orc_global_shift(ct, cbct0, n, ss[L - 1]);
    else
        memcpy(ss[L - 1], cbct0, sizeof(double) * n);

    /* Sec. 2.3 parameter rules for the Eq. 7-10 mask, resolved once on the
     * initial finest-level images: HU_0 = 2 Delta HU, [a_lo, a_hi] a_m with
     * a_m the median of A, and h (Eq. 10, not given) = HU_0 (1 HU if HU_0 is 0) */
    orc_params q = *p;
    if (p->mask_mode == 1) {
        double am = orc_a_median(ct, ss[L - 1], nx, ny, nz, p->patch[0], p->patch[1], p->patch[2],
                                 p->var_floor);
        q.hu0 = p->hu0 > 0.0 ? p->hu0 : 2.0 * fabs(dhu);
        q.a_lo = p->a_lo * am;
        q.a_hi = p->a_hi * am;
        q.fill_h = p->fill_h > 0.0 ? p->fill_h : (q.hu0 > 0.0 ? q.hu0 : 1.0);
    }
    p = &q;

    /* A1: down-sample to the coarsest resolution */
    for (int l = L - 2; l >= 0; --l) {
        cts[l] = (double*)malloc(sizeof(double) * ns[l]);
        ss[l] = (double*)malloc(sizeof(double) * ns[l]);
        orc_downsample2(cts[l + 1], dims[l + 1][0], dims[l + 1][1], dims[l + 1][2], cts[l]);
        orc_downsample2(ss[l + 1], dims[l + 1][0], dims[l + 1][1], dims[l + 1][2], ss[l]);
    }

    /* A1: initialise r to zero */
    double* r = (double*)calloc(3 * ns[0], sizeof(double));
    double* f = NULL;

    for (int l = 0; l < L; ++l) {
        int lx = dims[l][0], ly = dims[l][1], lz = dims[l][2];
        if (l > 0) {
            double* rf = (double*)malloc(sizeof(double) * 3 * ns[l]);
            orc_upsample_field(r, dims[l - 1][0], dims[l - 1][1], dims[l - 1][2], rf, lx, ly, lz);
            free(r);
            r = rf;
        }
        /* the static image is the original (shifted) CBCT at every iteration
         * (Sec. 2.2), so its patch moments are fixed for the level */
        double* mu_s = (double*)malloc(sizeof(double) * ns[l]);
        double* var_s = (double*)malloc(sizeof(double) * ns[l]);
        orc_patch_moments(ss[l], lx, ly, lz, p->patch[0], p->patch[1], p->patch[2], mu_s, var_s);
        free(f);
        f = (double*)malloc(sizeof(double) * ns[l]);
        for (long i = 0; i < ns[l]; ++i) f[i] = ss[l][i];
        int k_done = 0;
        if (p->stop_eps > 0.0) {
            /* Sec. 2.3 stopping rule on l^(k) = sum |dr^(k+1)| / sum |r^(k)| */
            long nl = ns[l];
            double* r_prev = (double*)malloc(sizeof(double) * 3 * nl);
            double* dr = (double*)malloc(sizeof(double) * 3 * nl);
            double* hist = (double*)malloc(sizeof(double) * (p->iters[l] > 0 ? p->iters[l] : 1));
            for (int k = 0; k < p->iters[l]; ++k) {
                memcpy(r_prev, r, sizeof(double) * 3 * nl);
                orc_iterate(cts[l], ss[l], mu_s, var_s, r, lx, ly, lz, p, NULL, f, NULL);
                for (long i = 0; i < 3 * nl; ++i) dr[i] = r[i] - r_prev[i];
                double num = field_norm_sum(dr, nl), den = field_norm_sum(r_prev, nl);
                hist[k] = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
                if (l_hist) l_hist[(long)l * hist_stride + k] = hist[k];
                k_done = k + 1;
                if (k >= p->stop_lag && hist[k - p->stop_lag] - hist[k] <= p->stop_eps) break;
            }
            free(r_prev);
            free(dr);
            free(hist);
        } else {
            for (int k = 0; k < p->iters[l]; ++k)
                orc_iterate(cts[l], ss[l], mu_s, var_s, r, lx, ly, lz, p, NULL, f, NULL);
            k_done = p->iters[l];
        }
        if (iters_done) iters_done[l] = k_done;
        free(mu_s);
        free(var_s);
    }
    memcpy(r_out, r, sizeof(double) * 3 * n);
    if (f_out) memcpy(f_out, f, sizeof(double) * n);
    free(r);
    free(f);
    for (int l = 0; l < L; ++l) {
        free(cts[l]);
        free(ss[l]);
    }
    return 0;
}

/* ---- point evaluators ---------------------------------------------------- */

static void unlin(long i, int nx, int ny, int* x, int* y, int* z)
{
    *x = (int)(i % nx);
    *y = (int)((i / nx) % ny);
    *z = (int)(i / ((long)nx * ny));
}

void orc_warp_pts(const float* ct, const float* r, int nx, int ny, int nz,
                  const long* pts, long npts, double* out)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < npts; ++q) {
        int x, y, z;
        long i = pts[q];
        unlin(i, nx, ny, &x, &y, &z);
        out[q] = trilinear_f(ct, nx, ny, nz, x + (double)r[i], y + (double)r[n + i],
                             z + (double)r[2 * n + i]);
    }
}

void orc_correct_pts(const float* m, const float* s, int nx, int ny, int nz,
                     int px, int py, int pz, double tau,
                     const long* pts, long npts, double* out)
{
#pragma omp parallel for schedule(dynamic)
    for (long q = 0; q < npts; ++q) {
        int x, y, z;
        long i = pts[q];
        unlin(i, nx, ny, &x, &y, &z);
        double mu_m, var_m, mu_s, var_s, a, b;
        patch_at_f(m, nx, ny, nz, px, py, pz, x, y, z, &mu_m, &var_m);
        patch_at_f(s, nx, ny, nz, px, py, pz, x, y, z, &mu_s, &var_s);
        match_moments(mu_m, var_m, mu_s, var_s, tau, &a, &b);
        out[q] = a * (double)s[i] + b;
    }
}

void orc_force_pts(const float* m, const float* f, const float* r,
                   int nx, int ny, int nz, double eps_d,
                   const long* pts, long npts, double* out)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < npts; ++q) {
        int x, y, z;
        long i = pts[q];
        unlin(i, nx, ny, &x, &y, &z);
        double gx = ((double)f[lin(clampi(x + 1, nx), y, z, nx, ny)] - (double)f[lin(clampi(x - 1, nx), y, z, nx, ny)]) / 2.0;
        double gy = ((double)f[lin(x, clampi(y + 1, ny), z, nx, ny)] - (double)f[lin(x, clampi(y - 1, ny), z, nx, ny)]) / 2.0;
        double gz = ((double)f[lin(x, y, clampi(z + 1, nz), nx, ny)] - (double)f[lin(x, y, clampi(z - 1, nz), nx, ny)]) / 2.0;
        double u[3];
        force_from((double)m[i] - (double)f[i], gx, gy, gz, eps_d, u);
        for (int c = 0; c < 3; ++c) out[3 * q + c] = (double)r[c * n + i] - u[c];
    }
}

void orc_gauss_pts(const float* rt, int nx, int ny, int nz, double sigma,
                   const long* pts, long npts, double* out)
{
    double w[129];
    int R = orc_gauss_taps(sigma, w);
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(dynamic)
    for (long q = 0; q < npts; ++q) {
        int x, y, z;
        long i = pts[q];
        unlin(i, nx, ny, &x, &y, &z);
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = -R; k <= R; ++k)
                for (int j = -R; j <= R; ++j)
                    for (int ii = -R; ii <= R; ++ii)
                        s += w[k + R] * w[j + R] * w[ii + R] *
                             (double)rt[c * n + lin(clampi(x + ii, nx), clampi(y + j, ny), clampi(z + k, nz), nx, ny)];
            out[3 * q + c] = s;
        }
    }
}

/* ---- differentiable DISC: SSD between m and I'_s --------------------------
 *
 * Loss L(r) = sum_x (m(x) - I'_s(x))^2 with m = warp(CT, r) (Sec. 2.1 model)
 * and I'_s = a S + b from the patch moments of m and S (Eq. 3-6). The
 * gradient is the chain rule written out:
 *   dL/dm_j = 2 D_j - 2 sum_x D_x dI'_s(x)/dm_j,   D = m - I'_s,
 *   dI'_s(x)/dm_j = sum over patch offsets k with clamp(x + k) = j of
 *                   1/n + Y_x (m_j - E_x(M)) / (n STD_x(M)),
 * where Y = (S - E(S)) / STD(S); a flat static patch (a := 1) contributes
 * 1/n only, and so does a patch with STD(M) = 0 (a is not differentiable
 * there; its one-sided choice is 0). dL/dr = dL/dm * d trilinear / d position.
 */

/* Derivative of the trilinear interpolant of trilinear() with respect to the
 * sample position, same floor and clamp conventions. */
static void trilinear_grad(const double* v, int nx, int ny, int nz,
                           double px, double py, double pz, double g[3])
{
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    double tx = px - fx, ty = py - fy, tz = pz - fz;
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    g[0] = g[1] = g[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double c = v[lin(clampi(ix + dx, nx), clampi(iy + dy, ny), clampi(iz + dz, nz), nx, ny)];
                double wx = dx ? tx : 1.0 - tx, wy = dy ? ty : 1.0 - ty, wz = dz ? tz : 1.0 - tz;
                double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                g[0] += sx * wy * wz * c;
                g[1] += wx * sy * wz * c;
                g[2] += wx * wy * sz * c;
            }
}

static void trilinear_grad_f(const float* v, int nx, int ny, int nz,
                             double px, double py, double pz, double g[3])
{
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    double tx = px - fx, ty = py - fy, tz = pz - fz;
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    g[0] = g[1] = g[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double c = (double)v[lin(clampi(ix + dx, nx), clampi(iy + dy, ny), clampi(iz + dz, nz), nx, ny)];
                double wx = dx ? tx : 1.0 - tx, wy = dy ? ty : 1.0 - ty, wz = dz ? tz : 1.0 - tz;
                double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                g[0] += sx * wy * wz * c;
                g[1] += wx * sy * wz * c;
                g[2] += wx * wy * sz * c;
            }
}

/* m, its patch moments, the static moments and I'_s for the SSD functions. */
static void ssd_forward(const double* ct, const double* s, const double* r, int nx, int ny, int nz,
                        int px, int py, int pz, double tau, double* m, double* mu_m, double* var_m,
                        double* mu_s, double* var_s, double* f)
{
    long n = (long)nx * ny * nz;
    orc_warp(ct, r, nx, ny, nz, m);
    orc_patch_moments(m, nx, ny, nz, px, py, pz, mu_m, var_m);
    orc_patch_moments(s, nx, ny, nz, px, py, pz, mu_s, var_s);
    orc_correct(mu_m, var_m, mu_s, var_s, s, n, tau, NULL, NULL, f);
}

double orc_ssd_loss(const double* ct, const double* s, const double* r, int nx, int ny, int nz,
                    int px, int py, int pz, double tau)
{
    long n = (long)nx * ny * nz;
    double* buf = (double*)malloc(sizeof(double) * 6 * n);
    double *m = buf, *mu_m = buf + n, *var_m = buf + 2 * n, *mu_s = buf + 3 * n, *var_s = buf + 4 * n,
           *f = buf + 5 * n;
    ssd_forward(ct, s, r, nx, ny, nz, px, py, pz, tau, m, mu_m, var_m, mu_s, var_s, f);
    double L = 0.0;
    for (long i = 0; i < n; ++i) L += (m[i] - f[i]) * (m[i] - f[i]);
    free(buf);
    return L;
}

void orc_ssd_grad(const double* ct, const double* s, const double* r, int nx, int ny, int nz,
                  int px, int py, int pz, double tau, double* grad)
{
    long n = (long)nx * ny * nz;
    double np = (double)px * py * pz;
    int rx = px / 2, ry = py / 2, rz = pz / 2;
    double* buf = (double*)malloc(sizeof(double) * 7 * n);
    double *m = buf, *mu_m = buf + n, *var_m = buf + 2 * n, *mu_s = buf + 3 * n, *var_s = buf + 4 * n,
           *f = buf + 5 * n, *G = buf + 6 * n;
    ssd_forward(ct, s, r, nx, ny, nz, px, py, pz, tau, m, mu_m, var_m, mu_s, var_s, f);
    for (long i = 0; i < n; ++i) G[i] = 2.0 * (m[i] - f[i]);
    /* scatter every patch occurrence of every voxel j, literally */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                double D = m[i] - f[i];
                int flat = !(var_s[i] > tau);
                double sig = sqrt(var_m[i]);
                double coef = (!flat && sig > 0.0) ? (s[i] - mu_s[i]) / sqrt(var_s[i]) / (np * sig) : 0.0;
                for (int k = -rz; k <= rz; ++k)
                    for (int jj = -ry; jj <= ry; ++jj)
                        for (int ii = -rx; ii <= rx; ++ii) {
                            long j = lin(clampi(x + ii, nx), clampi(y + jj, ny), clampi(z + k, nz), nx, ny);
                            G[j] -= 2.0 * D * (1.0 / np + coef * (m[j] - mu_m[i]));
                        }
            }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = lin(x, y, z, nx, ny);
                double g[3];
                trilinear_grad(ct, nx, ny, nz, x + r[i], y + r[n + i], z + r[2 * n + i], g);
                for (int c = 0; c < 3; ++c) grad[c * n + i] = G[i] * g[c];
            }
    free(buf);
}

/* #{k in [-R, R] : clamp(x + k) = j} along one axis of length len. */
static int clamp_count(int x, int j, int R, int len)
{
    int c = 0;
    for (int k = -R; k <= R; ++k)
        if (clampi(x + k, len) == j) ++c;
    return c;
}

void orc_ssd_grad_pts(const float* ct, const float* s, const float* r, int nx, int ny, int nz,
                      int px, int py, int pz, double tau, const long* pts, long npts, double* out)
{
    long n = (long)nx * ny * nz;
    double np = (double)px * py * pz;
    int rx = px / 2, ry = py / 2, rz = pz / 2;
#pragma omp parallel for schedule(dynamic)
    for (long q = 0; q < npts; ++q) {
        int jx, jy, jz;
        long jl = pts[q];
        unlin(jl, nx, ny, &jx, &jy, &jz);
        /* m on the box of radius 2R around j (every value a patch of a patch
         * around j can touch), from the FP32 CT and field */
        int bx0 = jx - 2 * rx < 0 ? 0 : jx - 2 * rx, bx1 = jx + 2 * rx > nx - 1 ? nx - 1 : jx + 2 * rx;
        int by0 = jy - 2 * ry < 0 ? 0 : jy - 2 * ry, by1 = jy + 2 * ry > ny - 1 ? ny - 1 : jy + 2 * ry;
        int bz0 = jz - 2 * rz < 0 ? 0 : jz - 2 * rz, bz1 = jz + 2 * rz > nz - 1 ? nz - 1 : jz + 2 * rz;
        int wx = bx1 - bx0 + 1, wy = by1 - by0 + 1, wz = bz1 - bz0 + 1;
        double* mb = (double*)malloc(sizeof(double) * wx * wy * wz);
        for (int z = bz0; z <= bz1; ++z)
            for (int y = by0; y <= by1; ++y)
                for (int x = bx0; x <= bx1; ++x) {
                    long i = lin(x, y, z, nx, ny);
                    mb[((long)(z - bz0) * wy + (y - by0)) * wx + (x - bx0)] =
                        trilinear_f(ct, nx, ny, nz, x + (double)r[i], y + (double)r[n + i], z + (double)r[2 * n + i]);
                }
#define MB(X, Y, Z) mb[((long)((Z) - bz0) * wy + ((Y) - by0)) * wx + ((X) - bx0)]
        double mj = MB(jx, jy, jz);
        double G = 0.0;
        for (int z = jz - rz; z <= jz + rz; ++z)
            for (int y = jy - ry; y <= jy + ry; ++y)
                for (int x = jx - rx; x <= jx + rx; ++x) {
                    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) continue;
                    int mult = clamp_count(x, jx, rx, nx) * clamp_count(y, jy, ry, ny) * clamp_count(z, jz, rz, nz);
                    if (mult == 0 && !(x == jx && y == jy && z == jz)) continue;
                    /* moments of m (two-pass) and of s at x */
                    double sm = 0.0;
                    for (int k = -rz; k <= rz; ++k)
                        for (int jj = -ry; jj <= ry; ++jj)
                            for (int ii = -rx; ii <= rx; ++ii)
                                sm += MB(clampi(x + ii, nx), clampi(y + jj, ny), clampi(z + k, nz));
                    double mu = sm / np, qm = 0.0;
                    for (int k = -rz; k <= rz; ++k)
                        for (int jj = -ry; jj <= ry; ++jj)
                            for (int ii = -rx; ii <= rx; ++ii) {
                                double d = MB(clampi(x + ii, nx), clampi(y + jj, ny), clampi(z + k, nz)) - mu;
                                qm += d * d;
                            }
                    double var = qm / np, mu_s, var_s, a, b;
                    patch_at_f(s, nx, ny, nz, px, py, pz, x, y, z, &mu_s, &var_s);
                    match_moments(mu, var, mu_s, var_s, tau, &a, &b);
                    long i = lin(x, y, z, nx, ny);
                    double D = MB(x, y, z) - (a * (double)s[i] + b);
                    if (x == jx && y == jy && z == jz) G += 2.0 * D;
                    int flat = !(var_s > tau);
                    double sig = sqrt(var);
                    double coef = (!flat && sig > 0.0) ? ((double)s[i] - mu_s) / sqrt(var_s) / (np * sig) : 0.0;
                    G -= 2.0 * D * mult * (1.0 / np + coef * (mj - mu));
                }
#undef MB
        free(mb);
        double g[3];
        trilinear_grad_f(ct, nx, ny, nz, jx + (double)r[jl], jy + (double)r[n + jl], jz + (double)r[2 * n + jl], g);
        for (int c = 0; c < 3; ++c) out[3 * q + c] = G * g[c];
    }
}
