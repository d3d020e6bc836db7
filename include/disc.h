/*
 * disc.h -- C ABI of libdisc, the MI355X (gfx950) implementation of the DISC
 * iteration: demons registration of a planning CT onto a cone-beam CT with a
 * simultaneous local intensity correction of the CBCT.
 *
 * Method: Zhen, Gu, Yan, Zhou, Jia, Jiang, "CT to Cone-beam CT Deformable
 * Registration With Simultaneous Intensity Correction" (arXiv 1204.6295).
 *   - registration model I_m(x + v(x)) = I_s(x), CT moving, CBCT static:
 *     Sec. 2.1 and the first paragraph of Sec. 2.2;
 *   - local linear correction I'_s = a I_s + b by matching the first two
 *     patch moments: Sec. 2.2, Eq. 2-6, Appendix A.1-A.7;
 *   - demons force: Sec. 2.1, Eq. 1 (static-gradient term, on I'_s);
 *   - global shift, multi-scale pyramid and the per-level loop:
 *     Sec. 2.3 and Algorithm A1 (fixed iteration counts per level).
 *
 * Conventions shared by every entry point
 *   Layout.   A volume is float32 [nz][ny][nx], x contiguous, no padding.
 *             A field is float32 [3][nz][ny][nx], components (x, y, z), in
 *             voxel units of its level. m(x) = CT(x + r(x)).
 *   Memory.   Every pointer argument named *_dev is device memory owned by
 *             the caller. The library never allocates device memory: the
 *             context works inside a caller-provided workspace.
 *   Streams.  `stream` is a hipStream_t (NULL = default stream). All device
 *             work is enqueued on it without host synchronisation; results
 *             are valid once the caller has synchronised that stream.
 *   Errors.   Every call returns a disc_status. Argument errors are found on
 *             the host before any device work is enqueued. HIP launch errors
 *             map to DISC_EHIP. disc_last_error() describes the last failure
 *             (per context, or per thread for the context-free calls).
 *   Threads.  A context is not thread-safe; use one context per stream.
 *   Sizes.    nx, ny, nz >= 1; nx * ny * nz < 2^30. Patch extents are odd,
 *             1 <= px, py <= 31 and 1 <= pz <= 15. Gaussian sigma in
 *             (0, 8/3] voxels (at most 17 taps).
 */
#ifndef DISC_H
#define DISC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DISC_MAX_LEVELS 8
#define DISC_MAX_BATCH 16

typedef struct disc_ctx disc_ctx;

typedef enum {
    DISC_OK = 0,
    DISC_EINVAL = -1,   /* invalid argument (null pointer, bad size, bad parameter) */
    DISC_ENOMEM = -2,   /* workspace smaller than disc_workspace_bytes() */
    DISC_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
    DISC_ESTATE = -4,   /* call out of order (e.g. iterate before set_volumes) */
    DISC_ENOTSUP = -5,  /* valid request outside what the library supports */
    DISC_ENONFINITE = -6 /* an input volume holds NaN or Inf (check_finite = 1) */
} disc_status;

typedef struct {
    int   patch[3];      /* odd patch extents (px, py, pz): the n-voxel patches M, S of Eq. 3 */
    float sigma;         /* Gaussian regularisation of r (Algorithm A1 step 6), voxels */
    int   levels;        /* pyramid levels, 2x per level (Sec. 2.3), 1..DISC_MAX_LEVELS */
    int   iters[DISC_MAX_LEVELS]; /* iterations per level, coarsest first */
    int   global_shift;  /* 1: add mean(CT) - mean(CBCT) to the CBCT first (Sec. 2.3) */
    float var_floor;     /* tau (HU^2): a static patch with variance <= tau is flat and
                            only its mean is matched (a = 1) */
    float diff_floor;    /* eps_d (HU): |m - I'_s| < eps_d gives a zero force */
    int   force_mode;    /* 0: Eq. 1 static-gradient term on I'_s; 1: both terms of Eq. 1
                            (double force: adds d grad m / (|grad m|^2 + d^2)) */
    float stop_eps;      /* 0: fixed iteration counts. > 0: Sec. 2.3 stopping rule with
                            epsilon stop_eps; iters[] then caps each level */
    int   stop_lag;      /* the rule compares l^(k - stop_lag) with l^(k) (10 in Sec. 2.3) */
    int   mask_mode;     /* 0: Eq. 5-6 everywhere. 1: Eq. 7 mask and Eq. 8-10 fill of a, b */
    float hu0;           /* HU_0 of Eq. 7 (HU); <= 0: 2 |mean(CT) - mean(CBCT)| (Sec. 2.3) */
    float a_lo, a_hi;    /* a range [a_lo a_m, a_hi a_m], a_m the median of Eq. 5 on the
                            initial images over voxels where neither patch is flat (0.5, 1.5) */
    float fill_h;        /* h of Eq. 10 (HU); <= 0: the HU_0 in use (1 HU if that is 0) */
    int   fill_t[3];     /* region T of Eq. 8-9, odd extents (7, 7, 3), counted inside the volume */
    int   fill_passes;   /* fill passes per iteration, 1..64 (10); a voxel still unfilled keeps
                            its Eq. 5-6 a, b */
    int   check_finite;  /* 1: disc_set_volumes counts NaN / Inf voxels of ct and cbct first and
                            returns DISC_ENONFINITE if there are any (synchronises the stream);
                            0 (default): inputs are trusted */
} disc_params;

/* Defaults: patch 11^3, sigma 2, 3 levels x 100 iterations, global shift on,
 * tau = 1e-2 HU^2, eps_d = 1e-3 HU, static-gradient force, fixed counts
 * (stop_eps = 0, stop_lag = 10), no mask (mask_mode 0; its settings default
 * to the Sec. 2.3 rules: hu0 0 = 2 Delta HU, a range 0.5..1.5 a_m, h = HU_0,
 * T = 7x7x3, 10 passes), no finite check of the inputs. */
int disc_params_default(disc_params* p);

/* Validates *p and creates a host-side context. Does not touch the GPU.
 * *out receives the context (NULL on error). */
int disc_create(const disc_params* p, disc_ctx** out);

/* Releases the context (host memory only). NULL is accepted. */
void disc_destroy(disc_ctx* c);

/* Message of the last failing call on c (or on this thread when c is NULL).
 * The string stays valid until the next call that fails. */
const char* disc_last_error(const disc_ctx* c);

/* Bytes of device workspace disc_set_volumes needs for these parameters and
 * finest-level dims; 0 if the arguments are invalid. */
size_t disc_workspace_bytes(const disc_params* p, int nx, int ny, int nz);

/* Algorithm A1 set-up (Sec. 2.3): global intensity shift of the CBCT, 2x2x2
 * block-mean pyramid of CT and CBCT, patch moments of the static image per
 * level (fixed for the whole run, Sec. 2.2 corrects the original I_s), and
 * r := 0 at the coarsest level. ct_dev is borrowed (read every iteration at
 * the finest level) until the next set_volumes or destroy; cbct_dev is only
 * read by this call. workspace_dev (256-byte aligned) is borrowed likewise.
 * Volumes are in voxel units: the method needs no voxel spacing (the field,
 * the patch and sigma are all in voxels). With check_finite = 1 a NaN or Inf
 * in ct or cbct returns DISC_ENONFINITE before any other device work (the
 * context is then not ready). */
int disc_set_volumes(disc_ctx* c, const float* ct_dev, const float* cbct_dev,
                     int nx, int ny, int nz, void* workspace_dev,
                     size_t workspace_bytes, void* stream);

/* Enqueues n DISC iterations (Algorithm A1 steps 1, 3-6): warp, patch
 * moments, correction, force, update, Gaussian. When the current level has
 * done its iters[] count and a finer level exists, the field is first
 * up-sampled (Algorithm A1, last step) and the next level starts. After the
 * finest level's count, further iterations stay at the finest level.
 * With stop_eps > 0 each iteration also evaluates the Sec. 2.3 rule on the
 * device, without host synchronisation: after iteration k of a level,
 * l^(k) = sum_x |r^(k+1)(x) - r^(k)(x)| / sum_x |r^(k)(x)| (Euclidean norm per
 * voxel; 0 if both sums are 0, +inf if only the denominator is), and once
 * k >= stop_lag and l^(k - stop_lag) - l^(k) <= stop_eps the level is done:
 * its remaining scheduled iterations become no-ops. disc_state keeps
 * counting scheduled iterations; disc_get_stats reports the ones run. */
int disc_iterate(disc_ctx* c, int n, void* stream);

/* Enqueues every iteration left in the schedule. */
int disc_run(disc_ctx* c, void* stream);

/* Current state: level index (0 = coarsest), iterations done at that level,
 * and the level's dims (nx, ny, nz). Any output pointer may be NULL. */
int disc_state(const disc_ctx* c, int* level, int* iter_in_level, int dims[3]);

/* Copies the current field r ([3][nz][ny][nx] at the current level's dims)
 * to out_dev; dims_out (host, may be NULL) receives (nx, ny, nz). */
int disc_get_field(disc_ctx* c, float* out_dev, int dims_out[3], void* stream);

/* Replaces the current field with r_dev (current level's dims). For resume
 * from a saved field and for tests that start from a given field. */
int disc_set_field(disc_ctx* c, const float* r_dev, void* stream);

/* Copies I'_s = a I_s + b of the most recent iteration at the current level
 * (Sec. 2.2; the corrected CBCT, Sec. 4) to out_dev [nz][ny][nx].
 * DISC_ESTATE before the first iteration of the current level. */
int disc_get_corrected(disc_ctx* c, float* out_dev, void* stream);

/* Sec. 2.3 stopping rule state of `level` (stop_eps > 0 only, else
 * DISC_ENOTSUP): *iters_done (may be NULL) = iterations the level ran so far;
 * l_hist (host, max_k doubles, may be NULL when max_k = 0) receives l^(0),
 * l^(1), ... (entries past iters_done are 0). Synchronises `stream`. */
int disc_get_stats(disc_ctx* c, int level, int* iters_done, double* l_hist, int max_k, void* stream);

/* Mask mode: the Sec. 2.3 values resolved at set-up, out = {HU_0, a_min,
 * a_max, h, a_m} (host array). DISC_ENOTSUP when mask_mode is 0.
 * Synchronises `stream`. */
int disc_get_mask_params(disc_ctx* c, float out[5], void* stream);

/* Mask mode: the Eq. 7 mask and the Eq. 8-10 fill of the most recent
 * iteration at the current level, one byte per voxel ([nz][ny][nx]) to
 * out_dev: 0 = not masked (Eq. 5-6 a, b), p in 1..fill_passes = masked and
 * filled by fill pass p, 255 = masked and never filled (keeps its Eq. 5-6
 * a, b). DISC_ENOTSUP when mask_mode is 0; DISC_ESTATE before the first
 * iteration of the current level. */
int disc_get_mask(disc_ctx* c, unsigned char* out_dev, void* stream);

/* ---- single steps, running the same kernels as disc_iterate ------------ */
/* All buffers are caller-owned device memory of the stated sizes; inputs
 * and outputs must not overlap. N = nx * ny * nz. */

/* Sec. 2.1 model: m(x) = trilinear(ct, x + r(x)), corner indices clamped.
 * ct, m: N floats; r: 3N floats. */
int disc_step_warp(const float* ct_dev, const float* r_dev, int nx, int ny, int nz,
                   float* m_dev, void* stream);

/* Patch moments of the static image s (Eq. 3) folded into its standardised
 * form ys = (s - E(S)) / STD(S), or s - E(S) on flat patches (var <= tau,
 * flagged in the lowest mantissa bit). Library-internal encoding consumed
 * by disc_step_correct. s, ys: N floats. */
int disc_step_static_stats(const float* s_dev, int nx, int ny, int nz, const int patch[3],
                           float var_floor, float* ys_dev, void* stream);

/* Eq. 3-6 and I'_s = a I_s + b: patch mean/variance of m, a = STD(M)/STD(S),
 * b = E(M) - a E(S), written as f = E(M) + STD(M) ys (flat static patch:
 * f = E(M) + ys). m, ys, f: N floats. */
int disc_step_correct(const float* m_dev, const float* ys_dev, int nx, int ny, int nz,
                      const int patch[3], float* f_dev, void* stream);

/* Eq. 1 force on f = I'_s, the A1 step-5 update and the step-6 Gaussian:
 * rt = r - u with u = (m - f) grad f / (|grad f|^2 + (m - f)^2) (force_mode
 * 0) or that plus (m - f) grad m / (|grad m|^2 + (m - f)^2) (force_mode 1),
 * zero where |m - f| < diff_floor (central differences, clamped), then
 * r_out = G_sigma * rt per component. q is 3N floats of scratch (the
 * xy-filtered field); rt (may be NULL) receives r - u. m, f: N floats;
 * r, r_out: 3N floats. ct and m_out (both NULL, or both N floats): the
 * Sec. 2.1 warp of the next iteration, m_out = trilinear(ct, x + r_out(x)),
 * made inside the z pass as disc_iterate does. */
int disc_step_force_smooth(const float* m_dev, const float* f_dev, const float* r_dev,
                           int nx, int ny, int nz, float sigma, float diff_floor, int force_mode,
                           float* q_dev, float* r_out_dev, float* rt_dev, const float* ct_dev,
                           float* m_out_dev, void* stream);

/* Algorithm A1 step 6 alone: separable Gaussian of each field component,
 * taps exp(-k^2 / 2 sigma^2) for |k| <= ceil(3 sigma), normalised, indices
 * clamped. rt, q (scratch), r: 3N floats. */
int disc_step_smooth(const float* rt_dev, int nx, int ny, int nz, float sigma,
                     float* q_dev, float* r_dev, void* stream);

/* Sec. 2.3 global shift: s = cbct + (mean(ct) - mean(cbct)), means in FP64.
 * dhu_dev (device, may be NULL) receives Delta HU as a double. scratch_dev
 * must hold disc_step_shift_scratch_bytes() bytes. */
size_t disc_step_shift_scratch_bytes(void);
int disc_step_shift(const float* ct_dev, const float* cbct_dev, long n, float* s_dev,
                    double* dhu_dev, void* scratch_dev, size_t scratch_bytes, void* stream);

/* Sec. 2.3 multi-scale strategy: 2x2x2 block mean, indices clamped; out has
 * dims (ceil(nx/2), ceil(ny/2), ceil(nz/2)). */
int disc_step_downsample(const float* in_dev, int nx, int ny, int nz, float* out_dev,
                         void* stream);

/* Algorithm A1, last step: r_f(x) = 2 trilinear(r_c, (x + 1/2)/2 - 1/2),
 * edge clamped, per component. rc: 3 * cnx*cny*cnz; rf: 3 * fnx*fny*fnz. */
int disc_step_upsample_field(const float* rc_dev, int cnx, int cny, int cnz,
                             float* rf_dev, int fnx, int fny, int fnz, void* stream);

/* ---- differentiable DISC ------------------------------------------------ */
/* Loss L(r) = sum_x (m(x) - I'_s(x))^2 between the warped CT m = CT(x + r)
 * (Sec. 2.1 model) and the static image corrected by patch moment matching
 * against m (Eq. 3-6; flat static patches match the mean only, a = 1).
 * ys is the standardised static image from disc_step_static_stats with the
 * same patch. Gradient (disc_ssd_grad), by the chain rule through Eq. 3-6
 * and the trilinear warp, recomputing the patch moments of m:
 *   dL/dm_j = 2 D_j - 2 sum_{x : j in P(x)} D_x (1/n + Y_x (m_j - E_x(M)) / (n STD_x(M)))
 * with D = m - I'_s, Y = (S - E(S)) / STD(S), P(x) the clamped patch (an
 * edge voxel counts once per patch offset that clamps onto it), and
 * dL/dr = dL/dm * d trilinear / d position (one-sided in the cell the warp
 * samples; 0 along an axis where both corners clamp to the same voxel).
 * Where STD(M) = 0 the derivative of a is taken as 0.
 *
 * ct, ys: N floats; r, grad: 3N floats (field layout); loss_dev: one double,
 * written by the call (disc_ssd_grad: may be NULL). scale_dev (may be NULL =
 * 1): one float multiplying the gradient (the upstream dL'/dL of autograd).
 * scratch_dev: caller-owned device memory, 256-byte aligned, of at least
 * disc_ssd_scratch_bytes() bytes (about 40 N bytes); contents are not
 * preserved. Results are deterministic (fixed-order FP64 reductions). */
size_t disc_ssd_scratch_bytes(int nx, int ny, int nz);
int disc_ssd_loss(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny, int nz,
                  const int patch[3], double* loss_dev, void* scratch_dev, size_t scratch_bytes,
                  void* stream);
int disc_ssd_grad(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny, int nz,
                  const int patch[3], const float* scale_dev, float* grad_dev, double* loss_dev,
                  void* scratch_dev, size_t scratch_bytes, void* stream);

/* Allocation-free variant of disc_ssd_loss, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same loss from the same kernels,
 * with the scratch (m, N floats, and the loss partials) in a fixed 32 MiB
 * device array that every GPU the library runs on holds until the process
 * ends. No device memory is allocated or freed by this call. Volumes whose
 * scratch exceeds 32 MiB (about 8.3 million voxels) return DISC_ENOMEM.
 * The array is shared by every call on one GPU: calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller. Runs on the current device; the stream must belong to it. */
int disc_ssd_loss_noalloc(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny,
                          int nz, const int patch[3], double* loss_dev, void* stream);

/* ---- batches of volumes ------------------------------------------------- */
/* Many independent CT/CBCT pairs of uneven sizes advanced together, one
 * resolution level, same parameters (Sec. 2.2-2.3 per pair, exactly as
 * disc_iterate with levels = 1). Each iteration of the whole batch is three
 * launches (moments + correction; force + xy smoothing; z smoothing, which
 * also warps the CT for the next iteration; the standalone warp runs once
 * after set_volumes), each covering the workgroups of every volume; with
 * use_graph = 1 the n
 * iterations are captured once into a HIP graph (on an internal stream) and
 * replayed on `stream` by later calls with the same n.
 *
 * disc_batch_create: p->levels must be 1, p->stop_eps 0 and p->mask_mode 0 (else
 * DISC_ENOTSUP; force_mode 0 or 1 both run); n in
 * 1..DISC_MAX_BATCH; dims is [n][3] (nx, ny, nz). Host only.
 * disc_batch_workspace_bytes: device workspace for all volumes (about 40
 * bytes per voxel). disc_batch_set_volumes: ct_dev[v], cbct_dev[v] are
 * device volumes of dims[v] (host arrays of n device pointers); ct is
 * borrowed until the next set_volumes or destroy; per pair: global shift,
 * static patch moments, r := 0. disc_batch_set_tiles: launch knobs (moments
 * tile edge 16 or 32 and workgroup targets per volume of the three sweep
 * kernels; results may differ in the last bits between knob settings).
 * disc_batch_iterate: n more iterations of every pair. disc_batch_run: up
 * to iters[0] in total. disc_batch_get_field / get_corrected: pair v's field
 * [3][nz][ny][nx] or I'_s of the latest iteration. Errors as elsewhere;
 * disc_batch_last_error describes the last failure on b. */
typedef struct disc_batch disc_batch;
int disc_batch_create(const disc_params* p, int n, const int* dims, disc_batch** out);
void disc_batch_destroy(disc_batch* b);
const char* disc_batch_last_error(const disc_batch* b);
size_t disc_batch_workspace_bytes(const disc_batch* b);
int disc_batch_set_tiles(disc_batch* b, int mom_ts, int mom_target, int plane_target, int z_target);
int disc_batch_set_volumes(disc_batch* b, const float* const* ct_dev, const float* const* cbct_dev,
                           void* workspace_dev, size_t workspace_bytes, void* stream);
int disc_batch_iterate(disc_batch* b, int n, int use_graph, void* stream);
int disc_batch_run(disc_batch* b, int use_graph, void* stream);
int disc_batch_get_field(disc_batch* b, int v, float* out_dev, void* stream);
int disc_batch_get_corrected(disc_batch* b, int v, float* out_dev, void* stream);

/* ---- measurement helpers ------------------------------------------------ */

/* Plain device copy of `bytes` bytes (16-byte aligned pointers), used to
 * calibrate hardware byte counters against a kernel of known traffic. */
int disc_copy_kernel(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/* Per-kernel timing with HIP events on the launch stream. While enabled,
 * every kernel disc_iterate launches is bracketed by an event pair; the
 * library keeps at most max_records pairs. disc_timing_read synchronises
 * the recorded events and returns, for kernel id k (0 warp, 1 correct,
 * 2 force + xy smoothing, 3 z smoothing, 4 upsample, 5 Eq. 8-10 fill passes
 * and I'_s = a S + b in mask mode) at pyramid level
 * `level` (-1 = all levels), the number of launches, their total
 * milliseconds and the total voxels they processed. Re-enabling (any
 * max_records, 0 = off) clears the records. */
int disc_timing_enable(disc_ctx* c, int max_records);
int disc_timing_read(disc_ctx* c, int kernel_id, int level, int* launches, double* total_ms,
                     double* total_voxels);

#ifdef __cplusplus
}
#endif
#endif
