// Types and device functions shared by the DISC kernels (gfx950): sizes,
// Gaussian taps, index helpers, the trilinear warp and the batch argument
// block. Launch declarations live in kernels.h.
#pragma once

#include <hip/hip_runtime.h>

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

// Keeps float->int conversions in range for any input (NaN/Inf included);
// the clamped voxel index then always lies inside the volume.
__device__ inline int floor_to_int(float v)
{
    float f = floorf(v);
    f = fminf(fmaxf(f, -1048576.0f), 1048576.0f);
    return (int)f;
}

// Sec. 2.1 model I_m(x + v(x)) = I_s(x): the deformed moving image at x is the
// CT sampled at x + r(x), trilinear, corner indices clamped. The weights come
// from the fractional part of r alone and the integer voxel is added
// separately, so FP32 keeps the full sub-voxel resolution at any volume size.
// Shared by the warp kernel and the z-smoothing kernel (which warps with the
// field it has just produced), so both give bitwise the same m.
__device__ inline float warp_at(const float* __restrict__ ct, int x, int y, int z, float rx,
                                float ry, float rz, int nx, int ny, int nz)
{
    const float tx = rx - floorf(rx), ty = ry - floorf(ry), tz = rz - floorf(rz);
    const int ix = x + floor_to_int(rx), iy = y + floor_to_int(ry), iz = z + floor_to_int(rz);
    const int x0 = clampi(ix, nx), x1 = clampi(ix + 1, nx);
    const int y0 = clampi(iy, ny), y1 = clampi(iy + 1, ny);
    const int z0 = clampi(iz, nz), z1 = clampi(iz + 1, nz);
    // element offsets fit in 32 bits (the ABI bounds N below 2^31)
    const float* p00 = ct + (z0 * ny + y0) * nx;
    const float* p01 = ct + (z0 * ny + y1) * nx;
    const float* p10 = ct + (z1 * ny + y0) * nx;
    const float* p11 = ct + (z1 * ny + y1) * nx;
    const float c00 = fmaf(tx, p00[x1] - p00[x0], p00[x0]);
    const float c01 = fmaf(tx, p01[x1] - p01[x0], p01[x0]);
    const float c10 = fmaf(tx, p10[x1] - p10[x0], p10[x0]);
    const float c11 = fmaf(tx, p11[x1] - p11[x0], p11[x0]);
    const float c0 = fmaf(ty, c01 - c00, c00);
    const float c1 = fmaf(ty, c11 - c10, c10);
    return fmaf(tz, c1 - c0, c0);
}

// ---- batches of volumes in one launch --------------------------------------
// A batched launch covers the workgroups of up to kMaxBatch volumes:
// volume v owns workgroups [start[v], start[v + 1]) and its own argument
// block, all passed by value in the kernel arguments.
constexpr int kMaxBatch = 16;

template <class A>
struct Batch {
    int n;
    int start[kMaxBatch + 1];
    A v[kMaxBatch];
};

// Volume of workgroup bid (n <= kMaxBatch, wave-uniform).
__device__ inline int batch_volume(const int* start, int n, int bid)
{
    int v = 0;
    for (int i = 1; i < n; ++i) v += bid >= start[i] ? 1 : 0;
    return v;
}

}  // namespace disc
