// Per-voxel DISC kernels for gfx950: the trilinear warp of the CT and the
// set-up / level-switch kernels (global shift reduction, 2x2x2 pyramid,
// field up-sampling).
//
// All of these are HBM-streaming kernels: one thread per voxel, x mapped to
// the 64 lanes of a wave so every plain load and store is a contiguous
// 256-byte wave access; warp-corner gathers hit the same or adjacent cache
// lines.
#include <cmath>
#include <mutex>
#include <set>
#include <utility>

#include "kernels.h"

namespace disc {

namespace {

constexpr int BX = 64;  // one wave along x
constexpr int BY = 4;   // four waves along y

inline dim3 grid_for(Dims d)
{
    return dim3((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
}

// Two rows per thread (y and y + BY) so that each thread has six field loads
// and sixteen corner gathers in flight. (bx, by, z) is the workgroup's tile.
__device__ inline void warp_body(const float* __restrict__ ct, const float* __restrict__ r,
                                 float* __restrict__ m, int nx, int ny, int nz, int bx, int by, int z)
{
    const int x = bx * BX + threadIdx.x;
    const int ya = by * (2 * BY) + threadIdx.y, yb = ya + BY;
    if (x >= nx || ya >= ny) return;
    const long N = (long)nx * ny * nz;
    const long ia = ((long)z * ny + ya) * nx + x;
    const long ib = ia + (long)BY * nx;
    const bool has_b = yb < ny;
    const float rxa = r[ia], rya = r[N + ia], rza = r[2 * N + ia];
    float rxb = 0.0f, ryb = 0.0f, rzb = 0.0f;
    if (has_b) {
        rxb = r[ib];
        ryb = r[N + ib];
        rzb = r[2 * N + ib];
    }
    const WarpSrc w = warp_src(ct, nx, ny, nz);
    const float ma = warp_at(w, x, ya, z, rxa, rya, rza);
    if (has_b) m[ib] = warp_at(w, x, yb, z, rxb, ryb, rzb);
    m[ia] = ma;
}

__global__ __launch_bounds__(BX * BY) void k_warp(const float* __restrict__ ct,
                                                 const float* __restrict__ r,
                                                 float* __restrict__ m, int nx, int ny, int nz,
                                                 const int* __restrict__ stop)
{
    if (stop && *stop) return;  // the level has met its stopping rule
    warp_body(ct, r, m, nx, ny, nz, blockIdx.x, blockIdx.y, blockIdx.z);
}

struct WarpArgs {
    const float* ct;
    const float* r;
    float* m;
    int nx, ny, nz;
    int gx, gy;  // workgroups along x and y (rows in pairs)
};

// Batched: the workgroups of volume v tile (x, y pairs, z) in that order.
__global__ __launch_bounds__(BX * BY) void k_warp_batch(Batch<WarpArgs> b)
{
    const int v = batch_volume(b.start, b.n, blockIdx.x);
    const WarpArgs& a = b.v[v];
    const int lb = blockIdx.x - b.start[v];
    const int bx = lb % a.gx, rest = lb / a.gx;
    warp_body(a.ct, a.r, a.m, a.nx, a.ny, a.nz, bx, rest % a.gy, rest / a.gy);
}

// Sec. 2.3 multi-scale strategy: 2x2x2 block mean, clamped at odd edges.
__global__ __launch_bounds__(BX * BY) void k_downsample(const float* __restrict__ in,
                                                       float* __restrict__ out, int nx, int ny,
                                                       int nz, int cx, int cy)
{
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= cx || y >= cy) return;
    float s = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const float* row =
                in + ((long)clampi(2 * z + dz, nz) * ny + clampi(2 * y + dy, ny)) * nx;
            s += row[clampi(2 * x, nx)] + row[clampi(2 * x + 1, nx)];
        }
    out[((long)z * cy + y) * cx + x] = s * 0.125f;
}

// Algorithm A1, last step: coarse field sampled at the cell-centred position
// (x + 1/2)/2 - 1/2 = x/2 - 1/4 and doubled (one coarse voxel = two fine).
__global__ __launch_bounds__(BX * BY) void k_upsample(const float* __restrict__ rc,
                                                     float* __restrict__ rf, int cnx, int cny,
                                                     int cnz, int fnx, int fny, int fnz)
{
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= fnx || y >= fny) return;
    const float px = 0.5f * x - 0.25f, py = 0.5f * y - 0.25f, pz = 0.5f * z - 0.25f;
    const float fx = floorf(px), fy = floorf(py), fz = floorf(pz);
    const float tx = px - fx, ty = py - fy, tz = pz - fz;
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const int x0 = clampi(ix, cnx), x1 = clampi(ix + 1, cnx);
    const int y0 = clampi(iy, cny), y1 = clampi(iy + 1, cny);
    const int z0 = clampi(iz, cnz), z1 = clampi(iz + 1, cnz);
    const long nc = (long)cnx * cny * cnz, nf = (long)fnx * fny * fnz;
    const long o = ((long)z * fny + y) * fnx + x;
    for (int c = 0; c < 3; ++c) {
        const float* v = rc + c * nc;
        const float* p00 = v + ((long)z0 * cny + y0) * cnx;
        const float* p01 = v + ((long)z0 * cny + y1) * cnx;
        const float* p10 = v + ((long)z1 * cny + y0) * cnx;
        const float* p11 = v + ((long)z1 * cny + y1) * cnx;
        const float c00 = fmaf(tx, p00[x1] - p00[x0], p00[x0]);
        const float c01 = fmaf(tx, p01[x1] - p01[x0], p01[x0]);
        const float c10 = fmaf(tx, p10[x1] - p10[x0], p10[x0]);
        const float c11 = fmaf(tx, p11[x1] - p11[x0], p11[x0]);
        const float c0 = fmaf(ty, c01 - c00, c00);
        const float c1 = fmaf(ty, c11 - c10, c10);
        rf[c * nf + o] = 2.0f * fmaf(tz, c1 - c0, c0);
    }
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, long n, float v)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = v;
}

// Number of NaN / Inf values (exponent bits all set) in a and b: one
// atomic add per wave of its ballot count.
__global__ __launch_bounds__(256) void k_count_nonfinite(const unsigned* __restrict__ a,
                                                         const unsigned* __restrict__ b, long n,
                                                         int* __restrict__ count)
{
    int bad = 0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        bad += ((a[i] & 0x7f800000u) == 0x7f800000u) + ((b[i] & 0x7f800000u) == 0x7f800000u);
    // wave sum of the per-lane counts
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src,
                                              float4* __restrict__ dst, long n16)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n16; i += (long)gridDim.x * 256)
        dst[i] = src[i];
}

// Global shift, pass 1: FP64 partial sums of CT and CBCT per block, in a
// fixed order (grid-stride, then a fixed LDS tree), so the result is
// reproducible run to run.
constexpr int kShiftBlocks = 1024;

__global__ __launch_bounds__(256) void k_shift_partial(const float* __restrict__ ct,
                                                       const float* __restrict__ cb, long n,
                                                       double2* __restrict__ part)
{
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)kShiftBlocks * 256) {
        a += (double)ct[i];
        b += (double)cb[i];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sa[0], sb[0]);
}

// Pass 2 (one block): Delta HU = (sum CT - sum CBCT) / n.
__global__ __launch_bounds__(256) void k_shift_finish(const double2* __restrict__ part, long n,
                                                      double* __restrict__ dhu)
{
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < kShiftBlocks; k += 256) {
        a += part[k].x;
        b += part[k].y;
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) dhu[0] = (sa[0] - sb[0]) / (double)n;
}

// Pass 3: s = cbct + Delta HU, rounded once to FP32.
__global__ __launch_bounds__(256) void k_shift_apply(const float* __restrict__ cb, long n,
                                                     const double* __restrict__ dhu,
                                                     float* __restrict__ s)
{
    const double d = dhu[0];
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        s[i] = (float)((double)cb[i] + d);
}

inline unsigned blocks_for(long n, long per_block)
{
    long b = (n + per_block - 1) / per_block;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

bool make_gauss_taps(float sigma, GaussTaps* t)
{
    if (!(sigma > 0.0f)) return false;
    const double s = (double)sigma;
    const int R = (int)std::ceil(3.0 * s);
    if (R > kMaxGaussR) return false;
    double w[2 * kMaxGaussR + 1];
    double sum = 0.0;
    for (int k = -R; k <= R; ++k) {
        w[k + R] = std::exp(-(double)k * k / (2.0 * s * s));
        sum += w[k + R];
    }
    t->R = R;
    for (int k = 0; k < 2 * kMaxGaussR + 1; ++k) t->w[k] = k <= 2 * R ? (float)(w[k] / sum) : 0.0f;
    return true;
}

hipError_t launch_warp(const float* ct, const float* r, float* m, Dims d, hipStream_t s, const int* stop)
{
    const dim3 g((d.nx + BX - 1) / BX, (d.ny + 2 * BY - 1) / (2 * BY), d.nz);
    hipLaunchKernelGGL(k_warp, g, dim3(BX, BY), 0, s, ct, r, m, d.nx, d.ny, d.nz, stop);
    return hipGetLastError();
}

hipError_t launch_warp_batch(const BatchVol* vols, int n, hipStream_t s)
{
    Batch<WarpArgs> b{};
    b.n = n;
    b.start[0] = 0;
    for (int v = 0; v < n; ++v) {
        WarpArgs& a = b.v[v];
        a.ct = vols[v].ct;
        a.r = vols[v].r;
        a.m = vols[v].m;
        a.nx = vols[v].d.nx;
        a.ny = vols[v].d.ny;
        a.nz = vols[v].d.nz;
        a.gx = (a.nx + BX - 1) / BX;
        a.gy = (a.ny + 2 * BY - 1) / (2 * BY);
        b.start[v + 1] = b.start[v] + a.gx * a.gy * a.nz;
    }
    hipLaunchKernelGGL(k_warp_batch, dim3(b.start[n]), dim3(BX, BY), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_downsample(const float* in, float* out, Dims d, hipStream_t s)
{
    Dims c{(d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2};
    hipLaunchKernelGGL(k_downsample, grid_for(c), dim3(BX, BY), 0, s, in, out, d.nx, d.ny, d.nz,
                       c.nx, c.ny);
    return hipGetLastError();
}

hipError_t launch_upsample_field(const float* rc, Dims dc, float* rf, Dims df, hipStream_t s)
{
    hipLaunchKernelGGL(k_upsample, grid_for(df), dim3(BX, BY), 0, s, rc, rf, dc.nx, dc.ny, dc.nz,
                       df.nx, df.ny, df.nz);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, long n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256 * 8)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* a, const float* b, long n, int* count, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks_for(n, 256 * 8)), dim3(256), 0, s,
                       reinterpret_cast<const unsigned*>(a), reinterpret_cast<const unsigned*>(b), n, count);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    const long n16 = (long)(bytes / 16);
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n16, 256 * 4)), dim3(256), 0, s,
                       (const float4*)src, (float4*)dst, n16);
    return hipGetLastError();
}

size_t shift_scratch_bytes()
{
    return (size_t)kShiftBlocks * sizeof(double2) + 2 * sizeof(double);
}

hipError_t launch_shift(const float* ct, const float* cbct, long n, float* s, double* dhu,
                        void* scratch, hipStream_t st)
{
    double2* part = (double2*)scratch;
    double* d = dhu ? dhu : (double*)(part + kShiftBlocks);
    hipLaunchKernelGGL(k_shift_partial, dim3(kShiftBlocks), dim3(256), 0, st, ct, cbct, n, part);
    hipLaunchKernelGGL(k_shift_finish, dim3(1), dim3(256), 0, st, part, n, d);
    hipLaunchKernelGGL(k_shift_apply, dim3(blocks_for(n, 256 * 8)), dim3(256), 0, st, cbct, n, d, s);
    return hipGetLastError();
}

void lds_limit(const void* kernel, size_t bytes)
{
    if (bytes <= 65536) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    static std::mutex mu;
    static std::set<std::pair<const void*, int>> done;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({kernel, dev})) return;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        done.insert({kernel, dev});
}

}  // namespace disc
