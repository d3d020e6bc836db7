// Internal launch interface of the DISC kernels (gfx950). Every launcher
// enqueues on `stream` and returns the launch status; argument checking is
// done by the C ABI layer before these are called.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.h"

namespace disc {

// Raises `kernel`'s dynamic-LDS limit to `bytes` on the current device when
// that is above the 64 KB default, once per kernel and device (thread-safe).
// The following launch reports any failure.
void lds_limit(const void* kernel, size_t bytes);

// Builds taps exp(-k^2 / 2 sigma^2), |k| <= ceil(3 sigma), normalised in FP64.
// Returns false when sigma is outside (0, kMaxGaussR / 3].
bool make_gauss_taps(float sigma, GaussTaps* t);

// Kernels of an iteration take the level's stop flag (may be null): when it
// is set (the level met its Sec. 2.3 stopping rule) they return at once.

// m = CT(x + r(x)), trilinear, corner indices clamped.
hipError_t launch_warp(const float* ct, const float* r, float* m, Dims d, hipStream_t s,
                       const int* stop = nullptr);

// Static-image statistics: ys = (s - mu)/sd, or s - mu with the low mantissa
// bit set where var <= tau.
hipError_t launch_static_stats(const float* s, float* ys, Dims d, const int patch[3], float tau,
                               hipStream_t st, float* sd = nullptr);

// Corrected static image f = mu_M + c ys, c = sd_M (or 1 on flat static patches).
hipError_t launch_correct(const float* m, const float* ys, float* f, Dims d, const int patch[3],
                          hipStream_t st, const int* stop = nullptr);

// Per z plane: r~ = r - u (u the Eq. 1 force on f: static-gradient term,
// force_mode 0, or both terms, force_mode 1) on the tile plus the Gaussian
// halo, then the x and y Gaussian passes: q = G_xy * r~. rt (optional)
// receives r~.
hipError_t launch_force_xy(const float* m, const float* f, const float* r, float* q, float* rt,
                           Dims d, float eps_d, int force_mode, const GaussTaps& t, const int* stop,
                           hipStream_t st);

// q = G_xy * rt (x and y passes only).
hipError_t launch_smooth_xy(const float* rt, float* q, Dims d, const GaussTaps& t, hipStream_t st);

// out = G_z * q (z pass). ct and m (both or neither): also m = CT(x + out(x))
// at every output voxel, the next iteration's warp. norms (may be null): out holds r^(k) on entry and
// each workgroup writes (sum |r^(k+1) - r^(k)|, sum |r^(k)|) in FP64 to
// norms[2 b], norms[2 b + 1], b < smooth_z_blocks(d).
hipError_t launch_smooth_z(const float* q, float* out, Dims d, const GaussTaps& t, const int* stop,
                           double* norms, hipStream_t st, const float* ct = nullptr, float* m = nullptr);
int smooth_z_blocks(Dims d);
// Sec. 2.3 stopping rule after iteration k (see k_stop_rule).
hipError_t launch_stop_rule(const double* norms, int nparts, double* hist, int* flags, int k, int lag,
                            double eps, hipStream_t st);

// SSD loss and gradient (differentiable DISC).
// Moments sweep in SSD mode: dres = m - I'_s, bg = (beta, gamma) adjoint
// weights (bg may be null: loss only), one FP64 sum of dres^2 per workgroup
// into partial[0 .. ssd_partial_count(d)).
int ssd_partial_count(Dims d);
hipError_t launch_ssd_moments(const float* m, const float* ys, float* dres, double2* bg, double* partial,
                              Dims d, const int patch[3], hipStream_t st);
// Transpose of the clamped window sum of radius R along one axis (0 x, 1 y, 2 z).
hipError_t launch_box_adjoint(const double2* in, double2* out, Dims d, int axis, int R, hipStream_t st);
// grad = scale * (2 dres - 2 (m B(beta) + B(gamma))) * d trilinear / d position,
// with B = B_z B_y B_x: the z adjoint (radius R) of t = B_y B_x (beta, gamma)
// is fused with the gradient.
hipError_t launch_ssd_grad_z(const float* ct, const float* r, const float* m, const float* dres,
                             const double2* t, const float* scale, float* grad, Dims d, int R, hipStream_t st);
// loss = sum of n partial sums, fixed order.
hipError_t launch_ssd_finish(const double* partial, int n, double* loss, hipStream_t st);

// Eq. 7-10 (mask mode). Moments sweep writing ab = (a, b) of Eq. 5-6 and
// stamp = 255 where Eq. 7 masks the voxel (consts = {HU_0, a_min, a_max, h}
// on the device); sd is STD(S) from launch_static_stats.
hipError_t launch_mask_moments(const float* m, const float* ys, const float* s, const float* sd, float2* ab,
                               unsigned char* stamp, const float* consts, Dims d, const int patch[3],
                               hipStream_t st, const int* stop);
// Work lists of the Eq. 8-10 fill passes: queued[fill_tiles(d)] and
// wcount[passes + 2] zeroed per iteration, wl[(passes + 1) * fill_tiles(d)].
struct FillLists {
    int* queued;
    int* wl;
    int* wcount;
};
int fill_tiles(Dims d);
// Queue the tiles that pass 1 must visit (after the moments sweep has
// stamped the valid voxels).
hipError_t launch_fill_seed(const unsigned char* stamp, const FillLists& fl, Dims d, const int t[3],
                            const int* stop, hipStream_t st);
// Fill pass `pass` (1-based, of `passes`) of Eq. 8-10 over the T region t[3].
// filled[pass] counts the voxels it filled where the region is too large for
// the work-list kernel (filled zeroed per iteration).
hipError_t launch_fill_pass(float2* ab, unsigned char* stamp, const float* s, const float* consts, int* filled,
                            const FillLists& fl, int pass, int passes, Dims d, const int t[3], const int* stop,
                            hipStream_t st);
// f = a S + b.
hipError_t launch_apply_ab(const float2* ab, const float* s, float* f, Dims d, const int* stop, hipStream_t st);
// Set-up: a = STD(CT)/STD(S) per voxel (-1 where a patch is flat), then the
// exact median a_m and consts = {HU_0, a_lo a_m, a_hi a_m, h, a_m}.
hipError_t launch_amed_values(const float* ct, const float* ys, const float* sd, float* a_out, Dims d,
                              const int patch[3], float tau, hipStream_t st);
size_t median_scratch_bytes();
hipError_t launch_mask_consts(const float* a_vals, long n, const double* dhu, float hu0, float lo_frac,
                              float hi_frac, float h, void* scratch, float* consts, hipStream_t st);

// Moments + correction, z first (isotropic patches up to 15^3, batches up to
// 13^3; about `target` workgroups of 512 threads, 768 at 15^3).
bool correct_zf_applies(Dims d, const int patch[3]);
int correct_zf_resident(const int patch[3]);  // workgroups of the sweep per CU
hipError_t launch_correct_zf(const float* m, const float* ys, float* f, Dims d, const int patch[3], hipStream_t st,
                             const int* stop, int target);

struct BatchVol;
bool correct_zf_batch_applies(const int patch[3]);
hipError_t launch_correct_zf_batch(const BatchVol* vols, int n, const int patch[3], int target, hipStream_t st);

// Global shift: FP64 partial sums, then s = cbct + (mean ct - mean cbct).
size_t shift_scratch_bytes();
hipError_t launch_shift(const float* ct, const float* cbct, long n, float* s, double* dhu,
                        void* scratch, hipStream_t st);

hipError_t launch_downsample(const float* in, float* out, Dims d, hipStream_t st);
hipError_t launch_upsample_field(const float* rc, Dims dc, float* rf, Dims df, hipStream_t st);
hipError_t launch_fill(float* p, long n, float v, hipStream_t st);
// *count += number of NaN / Inf values in a[0..n) and b[0..n).
hipError_t launch_count_nonfinite(const float* a, const float* b, long n, int* count, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);

// Launch knobs of a batched iteration (chosen by the autotuner).
struct BatchTiles {
    int mom_ts;        // moments tile edge: 16 or 32
    int mom_target;    // moments: about this many workgroups per volume
    int plane_target;  // force + xy smoothing: workgroups per volume
    int z_target;      // z smoothing: workgroups per volume
};

// One volume of a batched iteration: its buffers and dims.
struct BatchVol {
    const float* ct;
    const float* ys;
    float* r;    // field, updated in place (r -> r~ -> smoothed)
    float* m;
    float* f;
    float* q;    // xy-filtered r~
    Dims d;
};

// One DISC iteration of every volume of a batch: the warp (only after set-up;
// afterwards the z pass of the previous iteration has produced m), the
// correction, force + xy smoothing, and the z pass.
hipError_t launch_warp_batch(const BatchVol* vols, int n, hipStream_t st);
hipError_t launch_correct_batch(const BatchVol* vols, int n, const int patch[3], const BatchTiles& tiles,
                                hipStream_t st);
hipError_t launch_force_xy_batch(const BatchVol* vols, int n, float eps_d, int force_mode, const GaussTaps& t,
                                 int target, hipStream_t st);
// warp: also m = CT(x + r(x)) with the new field, the next iteration's warp.
hipError_t launch_smooth_z_batch(const BatchVol* vols, int n, const GaussTaps& t, int target, bool warp,
                                 hipStream_t st);

}  // namespace disc
