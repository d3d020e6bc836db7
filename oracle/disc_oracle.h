/*
 * disc_oracle.h -- plain FP64 CPU oracle of DISC (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY: the checker the HIP library is compared against.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it. It shares no code, header, table or helper with the HIP
 * library, and the HIP library never calls it.
 *
 * Method: Zhen, Gu, Yan, Zhou, Jia, Jiang, "CT to Cone-beam CT Deformable
 * Registration With Simultaneous Intensity Correction" (arXiv 1204.6295),
 * Sec. 2.1 (Eq. 1), Sec. 2.2 (Eq. 2-6 and Appendix A.1-A.7), Sec. 2.3
 * (global shift, multi-scale strategy) and Algorithm A1.
 *
 * Layout: scalar volumes are [nz][ny][nx] with x fastest; vector fields are
 * [3][nz][ny][nx], components (x, y, z), in voxel units. Arrays passed as
 * double are full FP64 volumes; the *_pts functions read FP32 state (the
 * precision a GPU stores) and promote every value to FP64 on load.
 *
 * Parity status: every function here is pinned by the CPU test-suite
 * (library routines, closed forms, invariants, brute force, and central
 * finite differences for the SSD gradient, closed forms of the double
 * force and of the stopping rule, a hand-worked Eq. 8-10 average and the
 * pass-by-pass reach of the Eq. 7-10 fill).
 */
#ifndef DISC_ORACLE_H
#define DISC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    patch[3];     /* odd patch extents (px, py, pz), Eq. 3 patch of n = px*py*pz voxels */
    double sigma;        /* Gaussian regularisation sigma, voxels */
    int    levels;       /* pyramid levels, 2x per level (Sec. 2.3) */
    int    iters[8];     /* iterations per level, coarsest first */
    int    global_shift; /* 1: shift CBCT by the mean difference (Sec. 2.3) */
    double var_floor;    /* tau: a static-patch variance <= tau counts as flat (a := 1) */
    double diff_floor;   /* eps_d: |m - f'| < eps_d gives a zero force */
    int    force_mode;   /* 0: Eq. 1 static-gradient term; 1: both terms of Eq. 1 */
    double stop_eps;     /* > 0: Sec. 2.3 stopping rule with this epsilon; iters[] caps */
    int    stop_lag;     /* the rule compares l^(k - lag) with l^(k) (10 in Sec. 2.3) */
    int    mask_mode;    /* 1: Eq. 7-10 mask and weighted fill of a, b (Sec. 2.2-2.3) */
    double hu0;          /* HU_0 of Eq. 7; <= 0: 2 |Delta HU| (Sec. 2.3) */
    double a_lo, a_hi;   /* a range as multiples of the median a_m (0.5, 1.5; Sec. 2.3) */
    double fill_h;       /* h of Eq. 10; <= 0: the HU_0 in use */
    int    fill_t[3];    /* region T of Eq. 8-9 (7, 7, 3) */
    int    fill_passes;  /* at most this many fill passes per iteration */
} orc_params;

/* Number of OpenMP threads the whole-volume functions use. */
int orc_threads(void);
void orc_set_threads(int n);

/* Sec. 2.3: plain mean over all voxels. */
double orc_mean(const double* v, long n);

/* Sec. 2.3 global intensity adjustment: Delta HU = mean(CT) - mean(CBCT);
 * s = cbct0 + Delta HU. Returns Delta HU. (The hot path is invariant to this
 * shift: b absorbs any constant added to the static image.) */
double orc_global_shift(const double* ct, const double* cbct0, long n, double* s);

/* Multi-scale strategy (Sec. 2.3): 2x2x2 block mean, indices clamped,
 * output dims ceil(n/2). */
void orc_downsample2(const double* in, int nx, int ny, int nz, double* out);

/* Algorithm A1, last step: r_f(x) = 2 * trilinear(r_c, (x + 1/2)/2 - 1/2). */
void orc_upsample_field(const double* rc, int cnx, int cny, int cnz,
                        double* rf, int fnx, int fny, int fnz);

/* Sec. 2.1 model I_m(x + v(x)) = I_s(x): m(x) = CT(x + r(x)), trilinear,
 * edge replicated. */
void orc_warp(const double* ct, const double* r, int nx, int ny, int nz, double* m);

/* Eq. 3 (p = 1 and the centred second moment used in Eq. 5): patch mean and
 * population variance over the clamped px*py*pz patch at every voxel. */
void orc_patch_moments(const double* img, int nx, int ny, int nz,
                       int px, int py, int pz, double* mu, double* var);

/* Eq. 5, 6 and Sec. 2.2 I'_s = a I_s + b. Where var_s <= tau (flat static
 * patch) only the mean is matched: a = 1. */
void orc_correct(const double* mu_m, const double* var_m,
                 const double* mu_s, const double* var_s,
                 const double* s, long n, double tau,
                 double* a, double* b, double* f);

/* Eq. 1, static-gradient term, on the corrected static image f = I'_s:
 * u = (m - f) grad f / (|grad f|^2 + (m - f)^2); central differences,
 * indices clamped. u is a field [3][N]. */
void orc_force(const double* m, const double* f, int nx, int ny, int nz,
               double eps_d, double* u);

/* Both terms of Eq. 1 (double force): u = d grad f / (|grad f|^2 + d^2)
 * + d grad m / (|grad m|^2 + d^2), d = m - f; each term 0 where its
 * denominator is 0, both 0 where |d| < eps_d. */
void orc_force_double(const double* m, const double* f, int nx, int ny, int nz,
                      double eps_d, double* u);

/* Truncated, normalised Gaussian taps w[0..2R], R = ceil(3 sigma).
 * Returns R (<= 64) or -1 when sigma is not positive. */
int orc_gauss_taps(double sigma, double* w);

/* Algorithm A1 step 6: separable Gaussian of one scalar volume (x, y, z
 * passes), indices clamped. */
void orc_gauss(const double* in, int nx, int ny, int nz, double sigma, double* out);

/* Sec. 2.2 Eq. 7-10 on one level: with (a, b) of Eq. 5-6 per voxel (flat
 * static patch: a = 1), the mask xi = 1 where |m - s| > hu0 or a outside
 * [a_min, a_max]; masked voxels get a, b := 0 and are then filled, pass by
 * pass, with the Eq. 8-9 average over the voxels of the T region (inside
 * the volume) that are unmasked or were filled by an earlier pass, weights
 * exp(-(s_i - s_x)^2 / h^2) (Eq. 10), each divided by the largest of them
 * (which leaves the Eq. 9 ratio unchanged and keeps it finite). A voxel with
 * no such neighbour waits for the next pass. Passes stop when every voxel is
 * filled or after `passes`; a voxel still unfilled then keeps its Eq. 5-6
 * values. Writes A, B (N each), xi (N, may be NULL) and returns the number
 * of passes that filled at least one voxel. */
int orc_mask_fill(const double* m, const double* s, const double* mu_m, const double* var_m,
                  const double* mu_s, const double* var_s, int nx, int ny, int nz, double tau,
                  double hu0, double a_min, double a_max, double h, const int t[3], int passes,
                  double* A, double* B, unsigned char* xi);

/* The fill alone (Eq. 8-10) from given (a, b) and initial validity
 * valid0[x] (1 = unmasked): same passes and leftover rule as above. */
int orc_fill(const double* a0, const double* b0, const unsigned char* valid0, const double* s,
             int nx, int ny, int nz, double h, const int t[3], int passes, double* A, double* B);

/* orc_fill that also records, per voxel, the pass that filled it: 0 for a
 * voxel valid from the start, p (1-based) for one filled by pass p, 255 for
 * one never filled (pass_of may be NULL). */
int orc_fill_ex(const double* a0, const double* b0, const unsigned char* valid0, const double* s,
                int nx, int ny, int nz, double h, const int t[3], int passes, double* A, double* B,
                unsigned char* pass_of);

/* a_m of Sec. 2.3: the median of a = STD(M)/STD(S) (Eq. 5) over the voxels
 * where neither patch is flat (var > tau: a flat CT patch gives a = 0, which
 * carries no contrast ratio), computed once on the initial images (m = CT,
 * finest level); an even count averages the two middle values; 1 if no
 * voxel qualifies. */
double orc_a_median(const double* ct, const double* s, int nx, int ny, int nz, int px, int py, int pz,
                    double tau);

/* One DISC iteration at one level (Algorithm A1 steps 1, 3-6):
 * m = warp(ct, r); moments of m; f = a s + b; u = force; r = G * (r - u).
 * mu_s / var_s are the patch moments of s. r is updated in place.
 * m_out, f_out and rt_out (r - u before smoothing) may be NULL. */
void orc_iterate(const double* ct, const double* s, const double* mu_s,
                 const double* var_s, double* r, int nx, int ny, int nz,
                 const orc_params* p, double* m_out, double* f_out, double* rt_out);

/* Whole Algorithm A1 with fixed iteration counts. r_out: finest field [3][N];
 * f_out: I'_s of the last iteration at the finest level (N). Returns 0, or -1
 * on invalid arguments. */
int orc_register(const double* ct, const double* cbct0, int nx, int ny, int nz,
                 const orc_params* p, double* r_out, double* f_out);

/* orc_register with the Sec. 2.3 stopping rule when p->stop_eps > 0: per
 * level, after iteration k (0-based) l^(k) = sum_x |r^(k+1) - r^(k)| /
 * sum_x |r^(k)| (Euclidean norm per voxel; 0 when both sums are 0, +inf
 * when only the denominator is), and the level ends once k >= lag and
 * l^(k - lag) - l^(k) <= eps, or after iters[level] iterations.
 * iters_done[level] receives the count run; l_hist (may be NULL) receives
 * l^(k) at l_hist[level * hist_stride + k]. */
int orc_register_ex(const double* ct, const double* cbct0, int nx, int ny, int nz,
                    const orc_params* p, double* r_out, double* f_out, int* iters_done,
                    double* l_hist, int hist_stride);

/* ---- point evaluators on FP32 state (sampled parity at full size) ------ */

/* m at the listed voxels (linear indices) from FP32 ct and r. */
void orc_warp_pts(const float* ct, const float* r, int nx, int ny, int nz,
                  const long* pts, long npts, double* out);

/* I'_s at the listed voxels from FP32 m and FP32 static image s. */
void orc_correct_pts(const float* m, const float* s, int nx, int ny, int nz,
                     int px, int py, int pz, double tau,
                     const long* pts, long npts, double* out);

/* r - u at the listed voxels from FP32 m, f, r; out is [npts][3]. */
void orc_force_pts(const float* m, const float* f, const float* r,
                   int nx, int ny, int nz, double eps_d,
                   const long* pts, long npts, double* out);

/* Gaussian of the FP32 field rt at the listed voxels; out is [npts][3]. */
void orc_gauss_pts(const float* rt, int nx, int ny, int nz, double sigma,
                   const long* pts, long npts, double* out);

/* ---- differentiable DISC: SSD between m = warp(ct, r) and I'_s ---------- */

/* L = sum_x (m(x) - I'_s(x))^2, I'_s from the patch moments of m and of the
 * static image s (Eq. 3-6, flat static patch: a = 1). */
double orc_ssd_loss(const double* ct, const double* s, const double* r, int nx, int ny, int nz,
                    int px, int py, int pz, double tau);

/* dL/dr [3][N], analytic (chain rule through Eq. 3-6 and the trilinear warp),
 * by a literal scatter over every clamped patch occurrence. */
void orc_ssd_grad(const double* ct, const double* s, const double* r, int nx, int ny, int nz,
                  int px, int py, int pz, double tau, double* grad);

/* dL/dr at the listed voxels from FP32 ct, s and r; out is [npts][3]. */
void orc_ssd_grad_pts(const float* ct, const float* s, const float* r, int nx, int ny, int nz,
                      int px, int py, int pz, double tau, const long* pts, long npts, double* out);

#ifdef __cplusplus
}
#endif
#endif
