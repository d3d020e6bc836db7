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
// A pass visits only the tiles queued for it by the previous pass (or by the
// seed), and in them evaluates only the masked voxels within reach of a
// voxel the previous pass filled; device-side queues need no host
// synchronisation.
//
// Set-up (once per registration): a_m is the exact median of the Eq. 5
// ratios on the initial images, by a two-pass radix select over the float
// bit patterns (non-negative floats order like their bits): 16-bit digit
// histograms with atomics, then a one-workgroup scan per digit.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace disc {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr float kLog2e = 1.44269504088896341f;

// Eq. 10 weight exp(-dS^2 / h^2) divided by exp(-dmin^2 / h^2):
// 2^(-kw (|dS| - dmin)(|dS| + dmin)), kw = log2(e) / h^2, on the hardware
// base-2 exponential (1 ulp). dmin = 0 gives the plain weight; dmin = the
// smallest |dS| over the valid voxels of the T region makes the largest
// weight exactly 1, so the sum cannot underflow. The Eq. 9 ratio is the same
// for any dmin.
__device__ inline float fill_weight(float ad, float dmin, float kw)
{
    return __builtin_amdgcn_exp2f(-kw * ((ad - dmin) * (ad + dmin)));
}

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
            const float kw = kLog2e / (h * h);  // Eq. 10 weight as a power of 2
            const float sx = s[i];
            const int z0 = max(0, z - tz), z1 = min(nz - 1, z + tz);
            const int y0 = max(0, y - ty), y1 = min(ny - 1, y + ty);
            const int x0 = max(0, x - tx), x1 = min(nx - 1, x + tx);
            float dmin = INFINITY;  // smallest |dS| over the valid voxels
            for (int zz = z0; zz <= z1; ++zz)
                for (int yy = y0; yy <= y1; ++yy) {
                    const long row = ((long)zz * ny + yy) * nx;
                    for (int xx = x0; xx <= x1; ++xx)
                        if (stamp[row + xx] < pass) dmin = fminf(dmin, fabsf(s[row + xx] - sx));
                }
            double sw = 0.0, sa = 0.0, sb = 0.0;
            for (int zz = z0; zz <= z1; ++zz)
                for (int yy = y0; yy <= y1; ++yy) {
                    const long row = ((long)zz * ny + yy) * nx;
                    for (int xx = x0; xx <= x1; ++xx) {
                        if (stamp[row + xx] >= pass) continue;
                        const float ad = fabsf(s[row + xx] - sx);
                        const double w = (double)fill_weight(ad, dmin, kw);
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

// The same pass driven by work lists, with the T region staged in LDS; one
// 32 x 8 tile of one plane at a time per workgroup. Few masked voxels can
// change in a pass: one whose T region holds no voxel filled by the previous
// pass (for pass 1: no valid voxel) has the valid set it already failed
// with, so it fails again. Hence
//   seed     every tile with a valid voxel queues, for pass 1, the tiles
//            within reach of its valid voxels
//   pass p   visits only the tiles queued for p: stages the region's stamps
//            (tile plus the T halo, 2 tz + 1 planes; one region row per
//            wave, four rows per round trip), ORs "filled by pass p - 1"
//            (pass 1: valid) along z and then over the x-y window, lists the
//            masked voxels that see such a voxel, and only if there are any
//            stages {S, a, b, valid} and evaluates them, one per thread;
//            tiles that fill something queue, for p + 1, the tiles within
//            reach of what they filled
// Listed voxels see the same neighbours with the same weights as in
// k_fill_pass; the FP64 sums are grouped by region rows (see below).
// Queues: queued[tile] = last pass the tile was queued for (an atomicMax
// admits each tile once per pass), wl[p * ntiles ...] the tiles of pass p,
// wcount[p] their number; queued and wcount start at zero every iteration.
constexpr int FTX = 32, FTY = 8, FW = FTX * FTY / 64;  // FW waves per tile

struct FillQ {
    int* queued;
    int* wl;
    int* wcount;
    int ntx, nty, nz;
    int tx, ty, tz;
};

// Queue for pass `to` every tile that holds a voxel within the T reach of a
// voxel of tile (bx, by, z) with src set. Block-wide; bb: 4 ints of LDS.
__device__ void queue_reach(const FillQ& q, bool src, int to, int bx, int by, int z, int* bb)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        bb[0] = FTX;
        bb[1] = -1;
        bb[2] = FTY;
        bb[3] = -1;
    }
    const unsigned long long m = __ballot(src);
    __syncthreads();
    if (lane == 0 && m) {
        // a wave holds rows 2 wave and 2 wave + 1 of the tile, 32 voxels each
        const unsigned cols = (unsigned)m | (unsigned)(m >> 32);
        atomicMin(&bb[0], __ffs(cols) - 1);
        atomicMax(&bb[1], 31 - __clz(cols));
        atomicMin(&bb[2], 2 * wave + ((unsigned)m ? 0 : 1));
        atomicMax(&bb[3], 2 * wave + ((m >> 32) ? 1 : 0));
    }
    __syncthreads();
    if (bb[1] < 0) return;  // uniform: nothing to spread
    const int X0 = max(0, (bx * FTX + bb[0] - q.tx) / FTX), X1 = min(q.ntx - 1, (bx * FTX + bb[1] + q.tx) / FTX);
    const int Y0 = max(0, (by * FTY + bb[2] - q.ty) / FTY), Y1 = min(q.nty - 1, (by * FTY + bb[3] + q.ty) / FTY);
    const int Z0 = max(0, z - q.tz), Z1 = min(q.nz - 1, z + q.tz);
    const int cx = X1 - X0 + 1, cy = Y1 - Y0 + 1;
    const int t = threadIdx.x;  // at most 3 x 3 x 15 tiles (tx, ty < 8; tz < 8)
    if (t < cx * cy * (Z1 - Z0 + 1)) {
        const int ix = X0 + t % cx, iy = Y0 + (t / cx) % cy, iz = Z0 + t / (cx * cy);
        const int tile = (iz * q.nty + iy) * q.ntx + ix;
        if (atomicMax(&q.queued[tile], to) < to) {
            const long ntiles = (long)q.ntx * q.nty * q.nz;
            const int slot = atomicAdd(&q.wcount[to], 1);
            q.wl[(long)to * ntiles + slot] = tile;
        }
    }
}

__global__ __launch_bounds__(FTX* FTY) void k_fill_seed(const unsigned char* __restrict__ stamp, FillQ q, int nx,
                                                      int ny, const int* __restrict__ stop)
{
    __shared__ int bb[4];
    if (stop && *stop) return;  // the level has met its stopping rule
    const int x = blockIdx.x * FTX + (int)threadIdx.x % FTX, y = blockIdx.y * FTY + (int)threadIdx.x / FTX;
    const bool src = x < nx && y < ny && stamp[((long)blockIdx.z * ny + y) * nx + x] == 0;
    if (!__syncthreads_or(src)) return;
    queue_reach(q, src, 1, blockIdx.x, blockIdx.y, blockIdx.z, bb);
}

// CTX, CTY, CTZ: the T half-widths as compile-time constants (0: taken from q)
template <int CTX, int CTY, int CTZ>
__global__ __launch_bounds__(FTX* FTY) void k_fill_list(float2* __restrict__ ab, unsigned char* __restrict__ stamp,
                                                      const float* __restrict__ s, const float* __restrict__ consts,
                                                      FillQ q, int pass, int passes, int nx, int ny,
                                                      const int* __restrict__ stop)
{
    extern __shared__ __align__(16) float4 reg[];
    __shared__ int count;
    __shared__ int bb[4];
    __shared__ double3 part[FTX * FTY];  // partial sums of the row groups
    __shared__ float dmins[FTX * FTY];   // smallest |dS| of the row groups
    __shared__ unsigned char zxa[(FTY + 2 * 7) * FTX];  // the x-window OR of zany (ty <= 7)
    if (stop && *stop) return;  // the level has met its stopping rule
    const int tx = CTX > 0 ? CTX : q.tx, ty = CTX > 0 ? CTY : q.ty, tz = CTX > 0 ? CTZ : q.tz, nz = q.nz;
    // region rows a wave loads per round trip: all of them for fixed T
    constexpr int NB = CTX > 0 ? ((FTY + 2 * CTY) * (2 * CTZ + 1) + FW - 1) / FW : 4;
    const long ntiles = (long)q.ntx * q.nty * nz;
    const int ntodo = q.wcount[pass];
    // LDS: {S, a, b, valid} per region voxel, the region's stamps (255
    // outside the volume), the z-OR of "filled by pass p - 1" per region
    // column, and the list of voxels to evaluate
    const int RW = FTX + 2 * tx, RH = FTY + 2 * ty, RD = 2 * tz + 1;
    const int plane = RW * RH, nreg = plane * RD, rows = RH * RD;
    unsigned char* rst = reinterpret_cast<unsigned char*>(reg + nreg);
    unsigned char* zany = rst + nreg;
    int* list = reinterpret_cast<int*>(rst + ((nreg + plane + 3) & ~3));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx = threadIdx.x % FTX, ly = threadIdx.x / FTX;
    const unsigned char fresh = (unsigned char)(pass - 1);  // pass 1: the valid voxels (stamp 0)
    const float h = consts[3];
    const float kw = kLog2e / (h * h);  // Eq. 10 weight as a power of 2
    for (int e = blockIdx.x; e < ntodo; e += gridDim.x) {
        const int tile = q.wl[(long)pass * ntiles + e];
        const int bx = tile % q.ntx, by = (tile / q.ntx) % q.nty, z = tile / (q.ntx * q.nty);
        const int x0 = bx * FTX, y0 = by * FTY;
        const int rx0 = x0 - tx, ry0 = y0 - ty, rz0 = z - tz;
        const int gx = rx0 + lane;
        const bool xin = lane < RW && gx >= 0 && gx < nx;  // RW <= 46 lanes
        __syncthreads();  // the previous tile is done with LDS
        for (int r0 = wave; r0 < rows; r0 += NB * FW) {
            unsigned char v[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int r = r0 + j * FW;  // wave-uniform
                const int gy = ry0 + r % RH, gz = rz0 + r / RH;
                v[j] = 255;
                if (r < rows && xin && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                    v[j] = stamp[((long)gz * ny + gy) * nx + gx];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (r0 + j * FW < rows && lane < RW) rst[(r0 + j * FW) * RW + lane] = v[j];
        }
        if (threadIdx.x == 0) count = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < plane; k += FTX * FTY) {
            unsigned char o = 0;
            for (int dz = 0; dz < RD; ++dz) o |= rst[dz * plane + k] == fresh;
            zany[k] = o;
        }
        __syncthreads();
        // then along x over the window, for the tile's columns (ty < 8)
        for (int k = threadIdx.x; k < RH * FTX; k += FTX * FTY) {
            const int yy = k / FTX, xx = k - yy * FTX;
            const unsigned char* row = zany + yy * RW + xx;
            unsigned char o = 0;
            for (int dx = 0; dx <= 2 * tx; ++dx) o |= row[dx];
            zxa[k] = o;
        }
        __syncthreads();
        const bool inside = x0 + lx < nx && y0 + ly < ny;
        const bool mine = inside && rst[(tz * RH + ly + ty) * RW + lx + tx] == 255;
        bool need = false;
        if (mine)
            for (int dy = 0; dy <= 2 * ty; ++dy) need |= zxa[(ly + dy) * FTX + lx] != 0;
        const unsigned long long nb = __ballot(need);
        int base = 0;
        if (lane == 0 && nb) base = atomicAdd(&count, (int)__popcll(nb));
        base = __shfl(base, 0);
        if (need) list[base + __popcll(nb & ((1ull << lane) - 1))] = threadIdx.x;
        __syncthreads();
        const int n = count;
        if (n == 0) continue;  // uniform: no voxel of this tile can change
        for (int r0 = wave; r0 < rows; r0 += NB * FW) {
            float sv[NB];
            float2 w[NB];
            bool ok[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int r = r0 + j * FW;
                const int gy = ry0 + r % RH, gz = rz0 + r / RH;
                // valid stamps only occur inside the volume
                ok[j] = r < rows && lane < RW && rst[r * RW + lane] < pass;
                sv[j] = 0.0f;
                w[j] = make_float2(0.0f, 0.0f);
                if (ok[j]) {
                    const long g = ((long)gz * ny + gy) * nx + gx;
                    sv[j] = s[g];
                    w[j] = ab[g];
                }
            }
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (r0 + j * FW < rows && lane < RW)
                    reg[(r0 + j * FW) * RW + lane] = make_float4(sv[j], w[j].x, w[j].y, ok[j] ? 1.0f : 0.0f);
        }
        __syncthreads();
        // Each listed voxel's T region is split into S groups of region rows
        // (S <= 7, as many as the workgroup has threads for); a thread sums
        // one group in FP64, and the voxel's own thread adds the S partial
        // sums in group order.
        const int RT = RD * (2 * ty + 1);  // region rows of one voxel
        const int S = min(7, (FTX * FTY) / n);
        const bool item = (int)threadIdx.x < n * S;
        const int v = item ? (int)threadIdx.x % n : 0, g = (int)threadIdx.x / n;
        const int t = list[v];
        const int vx = t % FTX, vy = t / FTX;
        const float sx = item ? s[((long)z * ny + (y0 + vy)) * nx + (x0 + vx)] : 0.0f;
        // Weights relative to 2^0 first (the plain Eq. 10 weights); only if
        // a listed voxel's weight sum comes out below 2^-60 (its nearest
        // valid intensity is over ~6.5 h away, so weights may have
        // underflowed) is the tile summed again relative to the largest
        // weight of each voxel. Both give the Eq. 9 ratio.
        double fw = 0.0, fa = 0.0, fb = 0.0;  // the own voxel's sums (thread < n)
        for (int norm = 0; norm < 2; ++norm) {
            if (norm) {
                // smallest |dS| over the valid voxels of this thread's rows
                if (item) {
                    float dm = INFINITY;
#pragma unroll 1
                    for (int r = g * RT / S; r < (g + 1) * RT / S; ++r) {
                        const int dz = r / (2 * ty + 1), dy = r - dz * (2 * ty + 1);
                        const float4* row = reg + (dz * RH + vy + dy) * RW + vx;
#pragma unroll
                        for (int dx = 0; dx <= 2 * tx; ++dx) {
                            const float4 v4 = row[dx];
                            const float ad = fabsf(v4.x - sx);
                            dm = v4.w != 0.0f ? fminf(dm, ad) : dm;
                        }
                    }
                    dmins[threadIdx.x] = dm;
                }
                __syncthreads();
            }
            // the weighted sums of the thread's rows in FP64
            if (item) {
                float dmin = 0.0f;
                if (norm) {
                    dmin = dmins[v];
                    for (int k = 1; k < S; ++k) dmin = fminf(dmin, dmins[k * n + v]);
                }
                double sw = 0.0, sa = 0.0, sb = 0.0;
#pragma unroll 1
                for (int r = g * RT / S; r < (g + 1) * RT / S; ++r) {
                    const int dz = r / (2 * ty + 1), dy = r - dz * (2 * ty + 1);
                    const float4* row = reg + (dz * RH + vy + dy) * RW + vx;
                    // branch-free: a voxel that is not valid adds an exact zero
#pragma unroll
                    for (int dx = 0; dx <= 2 * tx; ++dx) {
                        const float4 v4 = row[dx];
                        const float e = fill_weight(fabsf(v4.x - sx), dmin, kw);
                        const double w = (double)(v4.w != 0.0f ? e : 0.0f);
                        sw += w;
                        sa = fma(w, (double)v4.y, sa);
                        sb = fma(w, (double)v4.z, sb);
                    }
                }
                part[threadIdx.x] = make_double3(sw, sa, sb);
            }
            __syncthreads();
            bool redo = false;
            if ((int)threadIdx.x < n) {
                fw = fa = fb = 0.0;
                for (int k = 0; k < S; ++k) {
                    const double3 pg = part[k * n + threadIdx.x];
                    fw += pg.x;
                    fa += pg.y;
                    fb += pg.z;
                }
                redo = fw < 0x1p-60;
            }
            if (norm || !__syncthreads_or(redo)) break;  // uniform
        }
        bool got = false;
        int gl = 0;  // tile-local index of the voxel this thread filled
        if ((int)threadIdx.x < n && fw > 0.0) {
            const int t = list[threadIdx.x];
            const long i = ((long)z * ny + (y0 + t / FTX)) * nx + (x0 + t % FTX);
            ab[i] = make_float2((float)(fa / fw), (float)(fb / fw));
            stamp[i] = (unsigned char)pass;
            got = true;
            gl = t;
        }
        if (pass == passes || !__syncthreads_or(got)) continue;  // uniform
        // hand the filled voxels back to their own threads for the reach
        list[threadIdx.x] = 0;
        __syncthreads();
        if (got) list[gl] = 1;
        __syncthreads();
        queue_reach(q, list[threadIdx.x] != 0, pass + 1, bx, by, z, bb);
    }
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

int fill_tiles(Dims d)
{
    return ((d.nx + FTX - 1) / FTX) * ((d.ny + FTY - 1) / FTY) * d.nz;
}

namespace {

// Static LDS of k_fill_list (count, bb, part, dmins, zxa): the dynamic
// region must fit beside it in the default 64 KiB per workgroup.
constexpr size_t kFillStaticLds = sizeof(int) + 4 * sizeof(int) + FTX * FTY * sizeof(double3) +
                                  FTX * FTY * sizeof(float) + (FTY + 2 * 7) * FTX;

// the work-list kernels take a region row per wave (RW <= 64) and one
// neighbouring tile per thread when queueing
bool fill_lists_fit(const int t[3], size_t* lds)
{
    const int tx = t[0] / 2, ty = t[1] / 2, tz = t[2] / 2;
    const size_t plane = (size_t)(FTX + 2 * tx) * (FTY + 2 * ty), nreg = plane * (2 * tz + 1);
    *lds = nreg * sizeof(float4) + ((nreg + plane + 3) & ~(size_t)3) + FTX * FTY * sizeof(int);
    const int reach = 3 * 3 * (2 * tz + 1);
    return *lds + kFillStaticLds <= 64 * 1024 && FTX + 2 * tx <= 64 && tx < FTX && ty < FTY &&
           reach <= FTX * FTY;
}

FillQ make_q(const FillLists& fl, Dims d, const int t[3])
{
    return FillQ{fl.queued, fl.wl, fl.wcount, (d.nx + FTX - 1) / FTX, (d.ny + FTY - 1) / FTY, d.nz,
                 t[0] / 2, t[1] / 2, t[2] / 2};
}

}  // namespace

hipError_t launch_fill_seed(const unsigned char* stamp, const FillLists& fl, Dims d, const int t[3],
                            const int* stop, hipStream_t st)
{
    size_t lds;
    if (!fill_lists_fit(t, &lds)) return hipSuccess;  // the cache-gather pass needs no lists
    const dim3 g((d.nx + FTX - 1) / FTX, (d.ny + FTY - 1) / FTY, d.nz);
    hipLaunchKernelGGL(k_fill_seed, g, dim3(FTX * FTY), 0, st, stamp, make_q(fl, d, t), d.nx, d.ny, stop);
    return hipGetLastError();
}

hipError_t launch_fill_pass(float2* ab, unsigned char* stamp, const float* s, const float* consts, int* filled,
                            const FillLists& fl, int pass, int passes, Dims d, const int t[3], const int* stop,
                            hipStream_t st)
{
    size_t lds;
    if (fill_lists_fit(t, &lds)) {
        // up to 8192 workgroups walk the queued tiles: about one tile each at
        // 256x256x96, so the hardware dispatcher balances uneven tiles
        const unsigned grid = (unsigned)std::min(fill_tiles(d), 8192);
        if (t[0] == 7 && t[1] == 7 && t[2] == 3)  // the 7 x 7 x 3 region of Sec. 2.3
            hipLaunchKernelGGL((k_fill_list<3, 3, 1>), dim3(grid), dim3(FTX * FTY), lds, st, ab, stamp, s, consts,
                               make_q(fl, d, t), pass, passes, d.nx, d.ny, stop);
        else
            hipLaunchKernelGGL((k_fill_list<0, 0, 0>), dim3(grid), dim3(FTX * FTY), lds, st, ab, stamp, s, consts,
                               make_q(fl, d, t), pass, passes, d.nx, d.ny, stop);
    } else {
        // large T regions: every masked voxel gathers straight from cache
        const int tx = t[0] / 2, ty = t[1] / 2, tz = t[2] / 2;
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
