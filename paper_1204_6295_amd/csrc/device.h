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

// ---- raw buffer access -----------------------------------------------------
// A buffer resource covers one array of at most 4 GiB (the ABI bounds
// volumes below 2^30 voxels). Every access splits its byte offset into a
// per-lane part (voffset) and a wave-uniform part (soffset, a scalar
// register), so walks over planes and the fixed corner pattern of the
// trilinear warp need no per-lane address arithmetic.
using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ inline Rsrc make_rsrc(const void* p, long bytes)
{
    // word 3: 32-bit data format for raw (untyped) dword access
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(unsigned)bytes, 0x00020000);
}

__device__ inline float ld(Rsrc r, int voff, int soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ inline void st(Rsrc r, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// The CT as the warp reads it: its buffer and, for the cell whose lowest
// corner is (xa, ya, za), the byte offsets of the eight corners (bit 0: +x,
// bit 1: +y, bit 2: +z; 0 along an axis of extent 1). Built once per thread,
// held in scalar registers.
struct WarpSrc {
    Rsrc ct;
    int nx, ny, nz;
    int xm, ym, zm;  // largest lowest-corner index per axis: max(n - 2, 0)
    int so[8];
};

__device__ inline WarpSrc warp_src(const float* ct, int nx, int ny, int nz)
{
    WarpSrc w;
    w.ct = make_rsrc(ct, (long)nx * ny * nz * 4);
    w.nx = nx;
    w.ny = ny;
    w.nz = nz;
    w.xm = nx > 1 ? nx - 2 : 0;
    w.ym = ny > 1 ? ny - 2 : 0;
    w.zm = nz > 1 ? nz - 2 : 0;
    const int sx = nx > 1 ? 4 : 0, sy = ny > 1 ? nx * 4 : 0, sz = nz > 1 ? nx * ny * 4 : 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) w.so[c] = (c & 1 ? sx : 0) + (c & 2 ? sy : 0) + (c & 4 ? sz : 0);
    return w;
}

// Sec. 2.1 model I_m(x + v(x)) = I_s(x): the deformed moving image at x is the
// CT sampled at x + r(x), trilinear, corner indices clamped (edge replicate).
// Along each axis the cell's lowest corner is clamped to [0, n - 2] and the
// weight t to [0, 1], which is the clamped interpolant: a sample beyond an
// edge gets t = 0 or 1 and so the edge value itself, and each lerp
// (1 - t) a + t b is exact at t = 0 and t = 1. The weights come from the
// fractional part of r alone and the integer voxel is added separately, so
// FP32 keeps the full sub-voxel resolution at any volume size. Shared by the
// warp kernel and the z-smoothing kernel (which warps with the field it has
// just produced), so both give bitwise the same m.
__device__ inline float warp_at(const WarpSrc& w, int x, int y, int z, float rx, float ry, float rz)
{
    const float fx = floorf(rx), fy = floorf(ry), fz = floorf(rz);
    const int ix = x + floor_to_int(rx), iy = y + floor_to_int(ry), iz = z + floor_to_int(rz);
    const int xa = min(max(ix, 0), w.xm), ya = min(max(iy, 0), w.ym), za = min(max(iz, 0), w.zm);
    const float tx = fminf(fmaxf((float)(ix - xa) + (rx - fx), 0.0f), 1.0f);
    const float ty = fminf(fmaxf((float)(iy - ya) + (ry - fy), 0.0f), 1.0f);
    const float tz = fminf(fmaxf((float)(iz - za) + (rz - fz), 0.0f), 1.0f);
    const int v = ((za * w.ny + ya) * w.nx + xa) * 4;
    float c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = ld(w.ct, v, w.so[k]);
    const float ux = 1.0f - tx, uy = 1.0f - ty, uz = 1.0f - tz;
    const float c00 = fmaf(tx, c[1], ux * c[0]);
    const float c01 = fmaf(tx, c[3], ux * c[2]);
    const float c10 = fmaf(tx, c[5], ux * c[4]);
    const float c11 = fmaf(tx, c[7], ux * c[6]);
    const float c0 = fmaf(ty, c01, uy * c00);
    const float c1 = fmaf(ty, c11, uy * c10);
    return fmaf(tz, c1, uz * c0);
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
