// Internal launch interface of the DISC kernels (gfx950). Every launcher
// enqueues on `stream` and returns the launch status; argument checking is
// done by the C ABI layer before these are called.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace disc {

// Largest supported patch radii and Gaussian radius.
constexpr int kMaxPatchRxy = 15;   // px, py <= 31
constexpr int kMaxPatchZ = 15;     // pz <= 15 (z window held in registers)
constexpr int kMaxGaussR = 8;      // ceil(3 sigma) <= 8

struct Dims {
    int nx, ny, nz;
    long n() const { return (long)nx * ny * nz; }
};

// Normalised Gaussian taps, passed by value (lands in scalar registers).
struct GaussTaps {
    int R;
    float w[2 * kMaxGaussR + 1];
};

// Builds taps exp(-k^2 / 2 sigma^2), |k| <= ceil(3 sigma), normalised in FP64.
// Returns false when sigma is outside (0, kMaxGaussR / 3].
bool make_gauss_taps(float sigma, GaussTaps* t);

// m = CT(x + r(x)), trilinear, corner indices clamped.
hipError_t launch_warp(const float* ct, const float* r, float* m, Dims d, hipStream_t s);

// Static-image statistics: ys = (s - mu)/sd, or s - mu with the low mantissa
// bit set where var <= tau.
hipError_t launch_static_stats(const float* s, float* ys, Dims d, const int patch[3], float tau,
                               hipStream_t st);

// Corrected static image f = mu_M + c ys, c = sd_M (or 1 on flat static patches).
hipError_t launch_correct(const float* m, const float* ys, float* f, Dims d, const int patch[3],
                          hipStream_t st);

// Per z plane: r~ = r - u (u the Eq. 1 static-gradient force on f) on the tile
// plus the Gaussian halo, then the x and y Gaussian passes: q = G_xy * r~.
// rt (optional) receives r~.
hipError_t launch_force_xy(const float* m, const float* f, const float* r, float* q, float* rt,
                           Dims d, float eps_d, const GaussTaps& t, hipStream_t st);

// q = G_xy * rt (x and y passes only).
hipError_t launch_smooth_xy(const float* rt, float* q, Dims d, const GaussTaps& t, hipStream_t st);

// out = G_z * q (z pass).
hipError_t launch_smooth_z(const float* q, float* out, Dims d, const GaussTaps& t, hipStream_t st);

// Global shift: FP64 partial sums, then s = cbct + (mean ct - mean cbct).
size_t shift_scratch_bytes();
hipError_t launch_shift(const float* ct, const float* cbct, long n, float* s, double* dhu,
                        void* scratch, hipStream_t st);

hipError_t launch_downsample(const float* in, float* out, Dims d, hipStream_t st);
hipError_t launch_upsample_field(const float* rc, Dims dc, float* rf, Dims df, hipStream_t st);
hipError_t launch_fill(float* p, long n, float v, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);

// XCD-aware block order: consecutive logical tiles land on the same XCD
// (workgroups are dispatched round-robin over the 8 XCDs of the chip).
__device__ inline int xcd_logical_block(int bid, int nblocks)
{
    const int q = nblocks >> 3, rem = nblocks & 7;
    const int xcd = bid & 7, local = bid >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + local;
}

__device__ inline int clampi(int v, int n)
{
    return v < 0 ? 0 : (v > n - 1 ? n - 1 : v);
}

}  // namespace disc
