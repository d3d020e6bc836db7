// Eq. 7-10 of DISC for gfx950: the fill of the masked a, b and the Sec. 2.3
// parameter rules.
//
// Per iteration (mask mode), after the moments sweep has written the Eq. 5-6
// pair (a, b) of every voxel and a stamp (0 = valid, 255 = masked by Eq. 7):
//   fill pass p = 1..P   every masked voxel takes the Eq. 8-9 average over
//                        the in-volume voxels of its T region whose stamp is
//                        below p (valid, or filled by an earlier pass), with
//                        the Eq. 10 weights; it is then stamped p. Reading
//                        only stamps below p keeps each pass a function of
//                        the previous one (no ping-pong copies), and a voxel
//                        never filled keeps its Eq. 5-6 pair.
//   apply                I'_s = a S + b.
// A pass after one that filled nothing returns at once (device counter of
// the previous pass), so no host synchronisation is needed; within a pass
// only the tiles next to the previous pass's fills are visited.
//
// Set-up (once per registration): a_m is the exact median of the Eq. 5
// ratios on the initial images, by a two-pass radix select over the float
// bit patterns (non-negative floats order like their bits): 16-bit digit
// histograms with atomics, then a one-workgroup scan per digit.
#include <cmath>

#include "kernels.h"

namespace disc {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

inline dim3 grid_for(Dims d)
{
    return dim3((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
}

// One fill pass (Eq. 8-10). consts: {hu0, a_lo, a_hi, h}. filled[p] counts
// the voxels pass p filled; filled[p - 1] == 0 (nothing changed) skips the pass.
__global__ __launch_bounds__(BX* BY) void k_fill_pass(float2* __restrict__ ab, unsigned char* __restrict__ stamp,
                                                      const float* __restrict__ s, const float* __restrict__ consts,
                                                      int* __restrict__ filled, int pass, int nx, int ny, int nz,
                                                      int tx, int ty, int tz, const int* __restrict__ stop)
{
    if (stop && *stop) return;  // the level has met its stopping rule
    if (pass > 1 && filled[pass - 1] == 0) return;  // the previous pass filled nothing
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    bool got = false;
    if (x < nx && y < ny) {
        const long i = ((long)z * ny + y) * nx + x;
        if (stamp[i] == 255) {
            const float h = consts[3];
            const float inv_h2 = 1.0f / (h * h);
            const float sx = s[i];
            double sw = 0.0, sa = 0.0, sb = 0.0;
            const int z0 = max(0, z - tz), z1 = min(nz - 1, z + tz);
            const int y0 = max(0, y - ty), y1 = min(ny - 1, y + ty);
            const int x0 = max(0, x - tx), x1 = min(nx - 1, x + tx);
            for (int zz = z0; zz <= z1; ++zz)
                for (int yy = y0; yy <= y1; ++yy) {
                    const long row = ((long)zz * ny + yy) * nx;
                    for (int xx = x0; xx <= x1; ++xx) {
                        if (stamp[row + xx] >= pass) continue;
                        const float ds = s[row + xx] - sx;
                        const double w = (double)expf(-(ds * ds) * inv_h2);
                        const float2 v = ab[row + xx];
                        sw += w;
                        sa = fma(w, (double)v.x, sa);
                        sb = fma(w, (double)v.y, sb);
                    }
                }
            if (sw > 0.0) {
                ab[i] = make_float2((float)(sa / sw), (float)(sb / sw));
                stamp[i] = (unsigned char)pass;
                got = true;
            }
        }
    }
    // count the voxels filled (one atomic per wave that has any)
    const unsigned long long bal = __ballot(got);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&filled[pass], (int)__popcll(bal));
}

// The same pass with the T region staged in LDS: a 32 x 8 tile of one plane
// loads its region (tile plus the T halo, 2 tz + 1 planes) once as packed
// {S, a, b, valid}, so the 147-voxel gathers of its masked voxels hit LDS.
// A tile with no masked voxel returns after one flag test. Neighbours are
// visited in the same order with the same arithmetic as k_fill_pass, so the
// results are bitwise the same.
constexpr int FTX = 32, FTY = 8;

__global__ __launch_bounds__(FTX* FTY) void k_fill_tile(float2* __restrict__ ab, unsigned char* __restrict__ stamp,
                                                      const float* __restrict__ s, const float* __restrict__ consts,
                                                      int* __restrict__ filled, unsigned char* __restrict__ dirty,
                                                      int pass, int nx, int ny, int nz, int tx, int ty, int tz,
                                                      const int* __restrict__ stop)
{
    extern __shared__ __align__(16) float4 reg[];
    if (stop && *stop) return;  // the level has met its stopping rule
    // A masked voxel can only succeed if a voxel within its reach was filled
    // by the previous pass (its T region is unchanged otherwise, and it
    // failed with that region before): pass p visits only tiles next to a
    // tile that pass p - 1 filled into, and stops once a pass fills nothing.
    const int ntx = gridDim.x, nty = gridDim.y;
    const long ntiles = (long)ntx * nty * nz;
    const int z = blockIdx.z;
    if (pass > 1) {
        if (filled[pass - 1] == 0) return;
        const unsigned char* prev = dirty + (long)(pass - 1) * ntiles;
        const int rx = (tx + FTX - 1) / FTX, ry = (ty + FTY - 1) / FTY;
        bool any = false;
        for (int dz = max(0, z - tz); dz <= min(nz - 1, z + tz) && !any; ++dz)
            for (int dy = max(0, (int)blockIdx.y - ry); dy <= min(nty - 1, (int)blockIdx.y + ry) && !any; ++dy)
                for (int dx = max(0, (int)blockIdx.x - rx); dx <= min(ntx - 1, (int)blockIdx.x + rx); ++dx)
                    if (prev[((long)dz * nty + dy) * ntx + dx]) {
                        any = true;
                        break;
                    }
        if (!any) return;
    }
    const int lx = threadIdx.x % FTX, ly = threadIdx.x / FTX;
    const int x = blockIdx.x * FTX + lx, y = blockIdx.y * FTY + ly;
    const bool inside = x < nx && y < ny;
    const long i = ((long)z * ny + y) * nx + x;
    const bool mine = inside && stamp[i] == 255;
    if (!__syncthreads_or(mine)) return;  // nothing to fill in this tile
    // stage the region: x0 - tx .. x0 + FTX - 1 + tx, same in y, z - tz .. z + tz
    const int RW = FTX + 2 * tx, RH = FTY + 2 * ty, RD = 2 * tz + 1;
    const int rx0 = blockIdx.x * FTX - tx, ry0 = blockIdx.y * FTY - ty, rz0 = z - tz;
    for (int k = threadIdx.x; k < RW * RH * RD; k += FTX * FTY) {
        const int cx = k % RW, rest = k / RW;
        const int cy = rest % RH, cz = rest / RH;
        const int gx = rx0 + cx, gy = ry0 + cy, gz = rz0 + cz;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // outside the volume: not valid
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
            const long q = ((long)gz * ny + gy) * nx + gx;
            if (stamp[q] < pass) {
                const float2 w = ab[q];
                v = make_float4(s[q], w.x, w.y, 1.0f);
            }
        }
        reg[k] = v;
    }
    __syncthreads();
    bool got = false;
    if (mine) {
        const float h = consts[3];
        const float inv_h2 = 1.0f / (h * h);
        const float sx = s[i];
        double sw = 0.0, sa = 0.0, sb = 0.0;
        for (int dz = 0; dz < RD; ++dz)
            for (int dy = 0; dy <= 2 * ty; ++dy) {
                const float4* row = reg + (dz * RH + ly + dy) * RW + lx;
                for (int dx = 0; dx <= 2 * tx; ++dx) {
                    const float4 v = row[dx];
                    if (v.w == 0.0f) continue;
                    const float ds = v.x - sx;
                    const double w = (double)expf(-(ds * ds) * inv_h2);
                    sw += w;
                    sa = fma(w, (double)v.y, sa);
                    sb = fma(w, (double)v.z, sb);
                }
            }
        if (sw > 0.0) {
            ab[i] = make_float2((float)(sa / sw), (float)(sb / sw));
            stamp[i] = (unsigned char)pass;
            got = true;
        }
    }
    // count the voxels filled (one atomic per wave that has any) and mark
    // the tile for the next pass
    const unsigned long long bal = __ballot(got);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&filled[pass], (int)__popcll(bal));
    if (__syncthreads_or(got) && threadIdx.x == 0)
        dirty[(long)pass * ntiles + ((long)z * nty + blockIdx.y) * ntx + blockIdx.x] = 1;
}

// I'_s = a S + b.
__global__ __launch_bounds__(BX* BY) void k_apply_ab(const float2* __restrict__ ab, const float* __restrict__ s,
                                                     float* __restrict__ f, int nx, int ny, int nz,
                                                     const int* __restrict__ stop)
{
    if (stop && *stop) return;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const long i = ((long)blockIdx.z * ny + y) * nx + x;
    const float2 v = ab[i];
    f[i] = fmaf(v.x, s[i], v.y);
}

constexpr unsigned kBins = 65536;

// Histogram of the high (digit 1) or low (digit 0, restricted to values
// whose high half equals sel[...]) 16 bits of the included values (v >= 0).
__global__ __launch_bounds__(256) void k_median_hist(const float* __restrict__ v, long n, int digit,
                                                     const unsigned* __restrict__ sel,
                                                     unsigned* __restrict__ hist0, unsigned* __restrict__ hist1)
{
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float a = v[i];
        if (!(a >= 0.0f)) continue;
        const unsigned b = __float_as_uint(a);
        if (digit == 1) {
            atomicAdd(&hist0[b >> 16], 1u);
        } else {
            // sel: {hi bin of rank k0, hi bin of rank k1, ...}
            if ((b >> 16) == sel[0]) atomicAdd(&hist0[b & 0xffffu], 1u);
            if ((b >> 16) == sel[1]) atomicAdd(&hist1[b & 0xffffu], 1u);
        }
    }
}

// One workgroup: finds, for the ranks k0 = (cnt - 1) / 2 and k1 = cnt / 2,
// the bin holding each rank and the rank left inside that bin.
// digit 1: sel[0..1] = high bins, sel[2..3] = ranks inside them, sel[4] = cnt.
// digit 0: sel[5..6] = low bins of the two ranks (hist0 for k0, hist1 for k1).
__device__ void scan_find(const unsigned* __restrict__ hist, unsigned rank, unsigned* bin_out,
                          unsigned* rank_out)
{
    __shared__ unsigned part[1024];
    const int t = threadIdx.x;
    unsigned s = 0;
    for (int j = 0; j < 64; ++j) s += hist[t * 64 + j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        unsigned acc = 0;
        int chunk = 0;
        while (chunk < 1023 && acc + part[chunk] <= rank) acc += part[chunk++];
        int b = chunk * 64;
        while (b < chunk * 64 + 63 && acc + hist[b] <= rank) acc += hist[b++];
        *bin_out = (unsigned)b;
        *rank_out = rank - acc;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_median_select(const unsigned* __restrict__ hist0,
                                                        const unsigned* __restrict__ hist1, int digit,
                                                        unsigned* __restrict__ sel)
{
    __shared__ unsigned cnt_s;
    const int t = threadIdx.x;
    if (digit == 1) {
        // count of included values
        __shared__ unsigned part[1024];
        unsigned s = 0;
        for (int j = 0; j < 64; ++j) s += hist0[t * 64 + j];
        part[t] = s;
        __syncthreads();
        if (t == 0) {
            unsigned c = 0;
            for (int j = 0; j < 1024; ++j) c += part[j];
            cnt_s = c;
            sel[4] = c;
        }
        __syncthreads();
        const unsigned cnt = cnt_s;
        if (cnt == 0) return;
        unsigned b, r;
        scan_find(hist0, (cnt - 1) / 2, &b, &r);
        if (t == 0) {
            sel[0] = b;
            sel[2] = r;
        }
        scan_find(hist0, cnt / 2, &b, &r);
        if (t == 0) {
            sel[1] = b;
            sel[3] = r;
        }
    } else {
        if (sel[4] == 0) return;
        unsigned b, r;
        const unsigned r0 = sel[2], r1 = sel[3];
        scan_find(hist0, r0, &b, &r);
        if (t == 0) sel[5] = b;
        scan_find(hist1, r1, &b, &r);
        if (t == 0) sel[6] = b;
    }
}

// consts = {hu0, a_lo, a_hi, h} from a_m (the two middle values), Delta HU
// and the user's settings (hu0 <= 0: 2 |Delta HU|; h <= 0: HU_0, or 1 HU if
// HU_0 is 0).
__global__ void k_mask_consts(const unsigned* __restrict__ sel, const double* __restrict__ dhu, float hu0_user,
                              float lo_frac, float hi_frac, float h_user, float* __restrict__ consts)
{
    if (threadIdx.x != 0) return;
    double am = 1.0;
    if (sel[4] > 0) {
        const float v0 = __uint_as_float((sel[0] << 16) | sel[5]);
        const float v1 = __uint_as_float((sel[1] << 16) | sel[6]);
        am = 0.5 * ((double)v0 + (double)v1);
    }
    const double hu0 = hu0_user > 0.0f ? (double)hu0_user : 2.0 * fabs(dhu[0]);
    consts[0] = (float)hu0;
    consts[1] = (float)(lo_frac * am);
    consts[2] = (float)(hi_frac * am);
    consts[3] = h_user > 0.0f ? h_user : (hu0 > 0.0 ? (float)hu0 : 1.0f);
    consts[4] = (float)am;
}

}  // namespace

size_t fill_dirty_bytes(Dims d, int passes)
{
    const size_t ntiles = (size_t)((d.nx + FTX - 1) / FTX) * ((d.ny + FTY - 1) / FTY) * d.nz;
    return (size_t)(passes + 1) * ntiles;
}

hipError_t launch_fill_pass(float2* ab, unsigned char* stamp, const float* s, const float* consts, int* filled,
                            unsigned char* dirty, int pass, Dims d, const int t[3], const int* stop, hipStream_t st)
{
    const int tx = t[0] / 2, ty = t[1] / 2, tz = t[2] / 2;
    const size_t lds = (size_t)(FTX + 2 * tx) * (FTY + 2 * ty) * (2 * tz + 1) * sizeof(float4);
    if (lds <= 64 * 1024) {
        const dim3 g((d.nx + FTX - 1) / FTX, (d.ny + FTY - 1) / FTY, d.nz);
        hipLaunchKernelGGL(k_fill_tile, g, dim3(FTX * FTY), lds, st, ab, stamp, s, consts, filled, dirty, pass, d.nx,
                           d.ny, d.nz, tx, ty, tz, stop);
    } else {
        // large T regions: gathers straight from cache
        hipLaunchKernelGGL(k_fill_pass, grid_for(d), dim3(BX, BY), 0, st, ab, stamp, s, consts, filled, pass, d.nx,
                           d.ny, d.nz, tx, ty, tz, stop);
    }
    return hipGetLastError();
}

hipError_t launch_apply_ab(const float2* ab, const float* s, float* f, Dims d, const int* stop, hipStream_t st)
{
    hipLaunchKernelGGL(k_apply_ab, grid_for(d), dim3(BX, BY), 0, st, ab, s, f, d.nx, d.ny, d.nz, stop);
    return hipGetLastError();
}

size_t median_scratch_bytes()
{
    return 2 * kBins * sizeof(unsigned) + 16 * sizeof(unsigned);
}

hipError_t launch_mask_consts(const float* a_vals, long n, const double* dhu, float hu0, float lo_frac,
                              float hi_frac, float h, void* scratch, float* consts, hipStream_t st)
{
    unsigned* h0 = static_cast<unsigned*>(scratch);
    unsigned* h1 = h0 + kBins;
    unsigned* sel = h1 + kBins;
    const unsigned grid = 1024;
    hipError_t e = launch_fill(reinterpret_cast<float*>(h0), 2 * kBins + 16, 0.0f, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_median_hist, dim3(grid), dim3(256), 0, st, a_vals, n, 1, sel, h0, h1);
    hipLaunchKernelGGL(k_median_select, dim3(1), dim3(1024), 0, st, h0, h1, 1, sel);
    e = launch_fill(reinterpret_cast<float*>(h0), 2 * kBins, 0.0f, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_median_hist, dim3(grid), dim3(256), 0, st, a_vals, n, 0, sel, h0, h1);
    hipLaunchKernelGGL(k_median_select, dim3(1), dim3(1024), 0, st, h0, h1, 0, sel);
    hipLaunchKernelGGL(k_mask_consts, dim3(1), dim3(64), 0, st, sel, dhu, hu0, lo_frac, hi_frac, h, consts);
    return hipGetLastError();
}

}  // namespace disc
