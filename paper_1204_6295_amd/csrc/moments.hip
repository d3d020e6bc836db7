// Patch moments (Eq. 3) and the moment-matching correction (Eq. 5-6,
// I'_s = a I_s + b) as one z-sweep kernel for gfx950.
//
// A workgroup owns a TS x TS column tile (TS = 32 for large volumes, 16 for
// small ones) and walks a chunk of z through four stages:
//   load   the tile plus the in-plane patch halo into LDS (the next plane's
//          global loads are in flight meanwhile);
//   x pass sliding window sums of m and m^2 along x, 4 outputs per item,
//          one lane per row, stored column-major with an odd pitch so the
//          writes here and the reads of the y pass are bank-conflict free;
//   y pass sliding window sums of those along y, 4 outputs per item;
//   z      each thread keeps a running sum over the last pz plane sums of
//          its column and a register ring of them (pz is a template
//          parameter) to subtract the plane leaving the window.
// The stages are software-pipelined over planes with double-buffered LDS:
// step q stashes plane q while waves 0-7 run the x pass of plane q-1, waves
// 8-11 the y pass of plane q-2 and every thread the z window of plane q-3,
// so one barrier per plane separates them and no stage waits for another.
// The in-plane radius is a template parameter for isotropic-in-xy patches
// (fully unrolled window loops) and a runtime value otherwise.
// All window sums are FP64: E(M^2) - E(M)^2 of 1500-HU data cancels far
// below FP32 resolution, and FP64 adds run at the FP32 rate on this chip.
// Static and moving images go through the same code, so identical inputs
// give bitwise identical moments.
#include <cmath>

#include "kernels.h"

namespace disc {

namespace {

constexpr int PRUN = 4;  // outputs per x / y item in the 16 x 16 plane-group kernel

// Epilogue of the sweep: what is made from the patch moments at each voxel.
// kMask: the Eq. 5-6 pair (a, b) and the Eq. 7 stamp per voxel; kAmed: the
// set-up ratio a = STD(CT)/STD(S) for the median a_m (-1 where a patch is flat).
enum MomMode { kCorrect = 0, kStatic = 1, kSsd = 2, kMask = 3, kAmed = 4 };

struct MomArgs {
    const float* img;    // image whose patch moments are taken (m, or s at set-up)
    const float* ys_in;  // standardised static image (correction and SSD passes)
    float* out;          // ys (set-up), f = I'_s (correction) or D = m - I'_s (SSD)
    double2* bg;         // SSD: adjoint weights (beta, gamma) per voxel, may be null
    double* partial;     // SSD: one sum of D^2 per workgroup
    const int* stop;     // level's stop flag (stopping rule), may be null
    float* sd_out;       // static pass: STD(S) per voxel (0 on flat patches), may be null
    const float* s_img;  // mask pass: the static image S
    const float* sd_s;   // mask / a_m passes: STD(S) per voxel
    float2* ab;          // mask pass: (a, b) of Eq. 5-6
    unsigned char* stamp;  // mask pass: 255 where Eq. 7 masks the voxel, else 0
    const float* consts;   // mask pass: {HU_0, a_min, a_max, h} on the device
    int nx, ny, nz;
    int rx, ry;
    int zchunk;
    int tiles_x, tiles_y, nblocks;
    float tau;
    double inv_n;
};

// Window sum over [0, 2r] of src and its squares, then RN - 1 slides; the
// RN results go to dst[0], dst[stride], ...
template <int RC, int RN>
__device__ inline void window_x(const float* src, int r, double2* dst, int stride)
{
    const int n = RC >= 0 ? 2 * RC : 2 * r;
    double u1 = 0.0, u2 = 0.0;
    if (RC >= 0) {
#pragma unroll
        for (int j = 0; j <= 2 * (RC >= 0 ? RC : 0); ++j) {
            const double v = (double)src[j];
            u1 += v;
            u2 = fma(v, v, u2);
        }
    } else {
#pragma unroll 4
        for (int j = 0; j <= n; ++j) {
            const double v = (double)src[j];
            u1 += v;
            u2 = fma(v, v, u2);
        }
    }
    dst[0] = make_double2(u1, u2);
#pragma unroll
    for (int k = 1; k < RN; ++k) {
        const double vi = (double)src[k + n], vo = (double)src[k - 1];
        u1 += vi - vo;
        u2 += fma(vi, vi, -vo * vo);
        dst[k * stride] = make_double2(u1, u2);
    }
}

// Dynamic LDS of one workgroup: double-buffered m region, x sums and y sums.
template <int RXY, int TS>
struct MomLds {
    static constexpr int RMAX = RXY >= 0 ? RXY : kMaxPatchRxy;
    static constexpr int MAXH = TS + 2 * RMAX;
    static constexpr int MAXPW = (TS + 2 * RMAX) | 1;  // odd pitch: the x pass reads rows conflict free
    static constexpr int PXH = MAXH | 1;  // odd pitch: column-major x sums are conflict free
    static constexpr size_t M_BYTES = ((size_t)MAXH * MAXPW * sizeof(float) + 15) & ~(size_t)15;
    static constexpr size_t X_BYTES = (size_t)TS * PXH * sizeof(double2);
    static constexpr size_t Y_BYTES = (size_t)TS * TS * sizeof(double2);
    static constexpr size_t BYTES = 2 * (M_BYTES + X_BYTES + Y_BYTES);
};

// One workgroup's sweep; bid is its workgroup index within the volume.
template <int PZ, int RXY, int MODE, int TS>
__device__ __forceinline__ void moments_body(const MomArgs& a, const int bid)
{
    constexpr bool STATIC = MODE == kStatic;
    if (a.stop && *a.stop) return;  // the level has met its stopping rule
    using L = MomLds<RXY, TS>;
    constexpr int NT = TS * TS;
    constexpr int MAXH = L::MAXH, MAXPW = L::MAXPW, PXH = L::PXH;
    constexpr int RZ = PZ / 2;
    constexpr int NQ = (MAXH * MAXPW + NT - 1) / NT;  // region values loaded per thread
    constexpr int RUN = TS == 32 ? 8 : 4;             // outputs per x / y item
    constexpr int XT = 64 * (TS / RUN);               // x workers: one lane per row, one wave per run
    constexpr int YT = TS * (TS / RUN);               // y workers
    constexpr int YB = (XT + YT <= NT) ? XT : 0;      // y workers follow the x workers if they fit
    static_assert(MAXH <= 64, "one lane per loaded row in the x pass");
    static_assert(XT <= NT && YT <= NT && YB % 64 == 0, "wave-uniform roles");
    extern __shared__ __align__(16) unsigned char smem[];
    float* s_m0 = reinterpret_cast<float*>(smem);
    double2* s_x0 = reinterpret_cast<double2*>(smem + 2 * L::M_BYTES);
    double2* s_y0 = reinterpret_cast<double2*>(smem + 2 * L::M_BYTES + 2 * L::X_BYTES);

    const int rx = RXY >= 0 ? RXY : a.rx;
    const int ry = RXY >= 0 ? RXY : a.ry;
    const int W = TS + 2 * rx, H = TS + 2 * ry;
    const int lb = xcd_logical_block(bid, a.nblocks);
    const int bx = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * TS, y0 = by * TS, z0 = bz * a.zchunk;
    const int z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    const int lx = t % TS, ly = t / TS;
    const int ox = x0 + lx, oy = y0 + ly;
    const bool own = ox < a.nx && oy < a.ny;
    const long plane = (long)a.nx * a.ny;

    double ring1[PZ], ring2[PZ];
#pragma unroll
    for (int k = 0; k < PZ; ++k) ring1[k] = ring2[k] = 0.0;
    double z1s = 0.0, z2s = 0.0;

    // region element -> (row, col), fixed over the sweep. Out-of-region slots
    // load a valid address and are never stored, so the loads stay
    // branch-free and remain in flight across barriers.
    int goff[NQ], soff[NQ];
    bool gval[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = t + q * NT;
        const int row = i / W, col = i - row * W;
        gval[q] = row < H;
        goff[q] = gval[q] ? clampi(y0 - ry + row, a.ny) * a.nx + clampi(x0 - rx + col, a.nx) : 0;
        soff[q] = gval[q] ? row * MAXPW + col : 0;
    }
    const int nplanes = (z1 - z0) + 2 * RZ;
    // buffer access: fixed per-lane byte offsets, the plane a scalar byte
    // offset (resources are rebuilt where used from the kernel arguments)
    const long vb = plane * 4 * (long)a.nz;
    const int pb = (int)plane * 4;
    auto fetch = [&](float(&dst)[NQ], int p) {
        const Rsrc ib = make_rsrc(a.img, vb);
        const int so = clampi(z0 - RZ + min(p, nplanes - 1), a.nz) * pb;
#pragma unroll
        for (int q = 0; q < NQ; ++q) dst[q] = ld(ib, goff[q] * 4, so);
    };
    // the epilogue's per-voxel input (ys, or the static image itself) for the
    // output made when plane p enters the window
    const int col_off = min(oy, a.ny - 1) * a.nx + min(ox, a.nx - 1);
    auto epi_load = [&](int p) {
        return ld(make_rsrc(STATIC ? a.img : a.ys_in, vb), col_off * 4, clampi(z0 + p - 2 * RZ, a.nz) * pb);
    };
    double loss = 0.0;  // SSD: sum of D^2 over this thread's voxels

    // Software pipeline, one barrier per step q:
    //   stash plane q | x pass of plane q-1 | y pass of plane q-2 | z window of plane q-3
    // with double buffers, so the four stages of one step touch disjoint LDS.
    // Global loads run PF steps ahead: step q requests the region of plane
    // q + PF and the per-voxel epilogue inputs of step q + PF, into register
    // slot q % PF, right after consuming what that slot held. With one
    // 1024-thread workgroup per CU no other workgroup covers memory latency,
    // so the loads must be in flight for several steps. Steps are unrolled
    // by PF, which fixes every slot index (and the LDS parity) at compile time.
    // (two steps where the z window or the mode's extra inputs leave no
    // registers for more: the hot correction sweep with pz < 13 gets four)
    constexpr int PF = (MODE == kCorrect && PZ < 13) ? 4 : 2;
    float pre[PF][NQ];
    float epi_q[PF], mid_q[PF], s_q[PF], sd_q[PF];
    // epilogue inputs of step q (the output made when plane q - 3 enters the window)
    auto epi_fetch = [&](int q, int slot) {
        epi_q[slot] = epi_load(q - 3);
        // SSD and mask: m at the output voxel itself; mask and a_m: S and STD(S) there
        const long vox_off = (long)clampi(z0 + q - 3 - 2 * RZ, a.nz) * plane + col_off;
        mid_q[slot] = (MODE == kSsd || MODE == kMask) ? a.img[vox_off] : 0.0f;
        s_q[slot] = MODE == kMask ? a.s_img[vox_off] : 0.0f;
        sd_q[slot] = (MODE == kMask || MODE == kAmed) ? a.sd_s[vox_off] : 0.0f;
    };
    auto step = [&](int q, const int par, const int slot) {
        const float epi_cur = epi_q[slot], mid_cur = mid_q[slot], s_cur = s_q[slot], sd_cur = sd_q[slot];
        epi_fetch(q + PF, slot);
        if (q < nplanes) {
            float* s_m = s_m0 + par * (MAXH * MAXPW);
#pragma unroll
            for (int k = 0; k < NQ; ++k)
                if (gval[k]) s_m[soff[k]] = pre[slot][k];
        }
        // unconditional (the plane index is clamped): always a valid address
        fetch(pre[slot], q + PF);
        if (q >= 1 && q - 1 < nplanes && t < XT) {
            // x pass: window [c, c + 2 rx] of the loaded row is the patch row of column c
            const int row = t & 63, run = t >> 6;
            if (row < H)
                window_x<RXY, RUN>(s_m0 + (par ^ 1) * (MAXH * MAXPW) + row * MAXPW + run * RUN, rx,
                              s_x0 + (par ^ 1) * (TS * PXH) + run * RUN * PXH + row, PXH);
        }
        if (q >= 2 && q - 2 < nplanes && t >= YB && t < YB + YT) {
            const int i = t - YB;
            const int col = i % TS, run = i / TS;
            const double2* xs = s_x0 + par * (TS * PXH) + col * PXH + run * RUN;
            double2* ys = s_y0 + par * (TS * TS) + run * RUN * TS + col;
            double u1 = 0.0, u2 = 0.0;
            if (RXY >= 0) {
#pragma unroll
                for (int j = 0; j <= 2 * (RXY >= 0 ? RXY : 0); ++j) {
                    const double2 v = xs[j];
                    u1 += v.x;
                    u2 += v.y;
                }
            } else {
#pragma unroll 4
                for (int j = 0; j <= 2 * ry; ++j) {
                    const double2 v = xs[j];
                    u1 += v.x;
                    u2 += v.y;
                }
            }
            ys[0] = make_double2(u1, u2);
#pragma unroll
            for (int rr = 1; rr < RUN; ++rr) {
                const double2 vi = xs[rr + 2 * ry], vo = xs[rr - 1];
                u1 += vi.x - vo.x;
                u2 += vi.y - vo.y;
                ys[rr * TS] = make_double2(u1, u2);
            }
        }
        if (q >= 3) {
            // z: the ring is a shift register with fixed slots; slot PZ - 1
            // holds the plane leaving the window
            const int p = q - 3;
            const double2 ps = s_y0[(par ^ 1) * (TS * TS) + ly * TS + lx];
            z1s += ps.x - ring1[PZ - 1];
            z2s += ps.y - ring2[PZ - 1];
#pragma unroll
            for (int j = PZ - 1; j > 0; --j) {
                ring1[j] = ring1[j - 1];
                ring2[j] = ring2[j - 1];
            }
            ring1[0] = ps.x;
            ring2[0] = ps.y;
            if (p >= PZ - 1 && own) {
                const int oz = z0 + p - 2 * RZ;
                const double mu = z1s * a.inv_n;
                double var = z2s * a.inv_n - mu * mu;
                var = var > 0.0 ? var : 0.0;
                const long idx = (long)oz * plane + col_off;
                if (MODE == kMask) {
                    // Eq. 5-6 (a flat static patch matches the mean only,
                    // a = 1), E(S) recovered from ys = (S - E(S)) / STD(S),
                    // and the Eq. 7 mask
                    const float yv = epi_cur;
                    const bool flat = __float_as_uint(yv) & 1u;
                    const double sds = flat ? 1.0 : (double)sd_cur;
                    const double av = flat ? 1.0 : sqrt(var) / sds;
                    const double bv = mu - av * ((double)s_cur - (double)yv * sds);
                    const bool xi = fabsf(mid_cur - s_cur) > a.consts[0] || av < (double)a.consts[1] ||
                                    av > (double)a.consts[2];
                    a.ab[idx] = make_float2((float)av, (float)bv);
                    a.stamp[idx] = xi ? 255 : 0;
                } else if (MODE == kAmed) {
                    // a = STD(CT) / STD(S) where neither patch is flat
                    const bool flat = __float_as_uint(epi_cur) & 1u;
                    a.out[idx] = (!flat && var > (double)a.tau) ? (float)(sqrt(var) / (double)sd_cur) : -1.0f;
                } else if (MODE == kSsd) {
                    // loss term and its adjoint weights: with D = m - I'_s,
                    // dL/dm_j = 2 D_j - 2 sum over patches P(x) containing j of
                    // D_x (1/n + Y_x (m_j - E_x(M)) / (n STD_x(M)))
                    //        = 2 D_j - 2 (m_j B(beta)_j + B(gamma)_j),
                    // beta = D Y / (n STD(M)), gamma = D / n - beta E(M), with B
                    // the adjoint of the clamped patch sum. Flat static patches
                    // (a = 1) and STD(M) = 0 give beta = 0.
                    const float yv = epi_cur;
                    const bool flat = __float_as_uint(yv) & 1u;
                    const float f = (float)fma(flat ? 1.0 : (double)sqrtf((float)var), (double)yv, mu);
                    const double D = (double)mid_cur - (double)f;
                    loss = fma(D, D, loss);
                    if (a.bg) {
                        const double sig = sqrt(var);
                        const double beta = (!flat && sig > 0.0) ? D * (double)yv * a.inv_n / sig : 0.0;
                        a.out[idx] = (float)D;
                        a.bg[idx] = make_double2(beta, fma(D, a.inv_n, -beta * mu));
                    }
                } else if (STATIC) {
                    // Eq. 5 denominator: STD(S). A flat static patch keeps only
                    // the mean match and is flagged in the low mantissa bit.
                    const double sv = (double)epi_cur;
                    const bool flat = !(var > (double)a.tau);
                    const double yv = flat ? (sv - mu) : (sv - mu) / sqrt(var);
                    unsigned bits = __float_as_uint((float)yv);
                    bits = flat ? (bits | 1u) : (bits & ~1u);
                    a.out[idx] = __uint_as_float(bits);
                    if (a.sd_out) a.sd_out[idx] = flat ? 0.0f : (float)sqrt(var);
                } else {
                    // I'_s = a S + b = E(M) + STD(M) (S - E(S)) / STD(S), combined
                    // in FP64 and rounded once: identical images then give
                    // |I'_s - m| well below eps_d.
                    const float yv = epi_cur;
                    const double c = (__float_as_uint(yv) & 1u) ? 1.0 : (double)sqrtf((float)var);
                    st(make_rsrc(a.out, vb), col_off * 4, oz * pb, (float)fma(c, (double)yv, mu));
                }
            }
        }
        __syncthreads();
    };

#pragma unroll
    for (int k = 0; k < PF; ++k) {
        fetch(pre[k], k);
        epi_fetch(k, k);
    }
    const int nsteps = nplanes + 3;
    static_assert(PF % 2 == 0, "the LDS parity follows the step index");
    for (int q = 0; q < nsteps; q += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k)
            if (q + k < nsteps) step(q + k, k & 1, k);
    }
    if (MODE == kSsd) {
        // fixed-order tree over the workgroup, one partial per workgroup
        double* red = reinterpret_cast<double*>(smem);
        red[t] = loss;
        __syncthreads();
#pragma unroll
        for (int h = NT / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) a.partial[bid] = red[0];
    }
}

template <int PZ, int RXY, int MODE, int TS>
__global__ __launch_bounds__(TS* TS) void k_moments(MomArgs a)
{
    moments_body<PZ, RXY, MODE, TS>(a, blockIdx.x);
}

template <int PZ, int RXY, int MODE, int TS>
__global__ __launch_bounds__(TS* TS) void k_moments_batch(Batch<MomArgs> b)
{
    const int v = batch_volume(b.start, b.n, blockIdx.x);
    moments_body<PZ, RXY, MODE, TS>(b.v[v], blockIdx.x - b.start[v]);
}

// ---- small volumes: several planes per step ------------------------------
// Coarse pyramid levels have few tiles, so the plane-serial sweep above is
// bound by the latency of its per-plane steps. Here a 1024-thread workgroup
// owns a 16 x 16 column tile and takes PP = 4 planes per step, one plane per
// 256-thread group: the group stages its plane, runs the x and y window sums,
// and stores the plane's y sums in an LDS ring of the last PZ + PP - 1
// planes; every thread then forms one output (its column, one of the PP
// window ends of the step) as the direct FP64 sum of PZ ring entries.
constexpr int PPS = 4;       // planes per step
constexpr int PTS = 16;      // tile edge
constexpr int PG = PTS * PTS;  // threads per plane group

template <int PZ, int RXY>
struct PpLds {
    static constexpr int H = PTS + 2 * RXY;
    static constexpr int PW = H | 1;  // odd pitch: the x pass reads rows conflict free
    static constexpr int PXH = H | 1;
    static constexpr int RING = PZ + PPS - 1;
    static constexpr size_t M_BYTES = ((size_t)PPS * H * PW * sizeof(float) + 15) & ~(size_t)15;
    static constexpr size_t X_BYTES = (size_t)PPS * PTS * PXH * sizeof(double2);
    static constexpr size_t Y_BYTES = (size_t)RING * PG * sizeof(double2);
    static constexpr size_t BYTES = M_BYTES + X_BYTES + Y_BYTES;
};

template <int MODE>
__device__ inline void mom_epilogue(const MomArgs& a, long idx, double mu, double var, float epi_v)
{
    if (MODE == kStatic) {
        const double sv = (double)epi_v;
        const bool flat = !(var > (double)a.tau);
        const double yv = flat ? (sv - mu) : (sv - mu) / sqrt(var);
        unsigned bits = __float_as_uint((float)yv);
        bits = flat ? (bits | 1u) : (bits & ~1u);
        a.out[idx] = __uint_as_float(bits);
        if (a.sd_out) a.sd_out[idx] = flat ? 0.0f : (float)sqrt(var);
    } else {
        const double c = (__float_as_uint(epi_v) & 1u) ? 1.0 : (double)sqrtf((float)var);
        a.out[idx] = (float)fma(c, (double)epi_v, mu);
    }
}

template <int PZ, int RXY, int MODE>
__global__ __launch_bounds__(PPS* PG) void k_moments_pp(MomArgs a)
{
    static_assert(RXY >= 0 && (MODE == kCorrect || MODE == kStatic), "isotropic correction / static only");
    using L = PpLds<PZ, RXY>;
    constexpr int H = L::H, PW = L::PW, PXH = L::PXH, RING = L::RING;
    constexpr int RZ = PZ / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    float* s_m = reinterpret_cast<float*>(smem);
    double2* s_x = reinterpret_cast<double2*>(smem + L::M_BYTES);
    double2* s_y = reinterpret_cast<double2*>(smem + L::M_BYTES + L::X_BYTES);
    if (a.stop && *a.stop) return;

    const int lb = xcd_logical_block(blockIdx.x, a.nblocks);
    const int bx = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * PTS, y0 = by * PTS, z0 = bz * a.zchunk;
    const int z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x, grp = t / PG, tl = t % PG;
    const int lx = tl % PTS, ly = tl / PTS;
    const int ox = x0 + lx, oy = y0 + ly;
    const bool own = ox < a.nx && oy < a.ny;
    const long plane = (long)a.nx * a.ny;
    const long col_off = (long)min(oy, a.ny - 1) * a.nx + min(ox, a.nx - 1);
    const float* epi = MODE == kStatic ? a.img : a.ys_in;
    const int nplanes = (z1 - z0) + 2 * RZ;
    float* sm = s_m + grp * (H * PW);
    double2* sx = s_x + grp * (PTS * PXH);

    // the group's region points, fixed over the sweep; out-of-region slots
    // load a valid address and are never stored (branch-free prefetch)
    constexpr int NQ = (H * H + PG - 1) / PG;
    int goff[NQ], soff[NQ];
    bool gval[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = tl + q * PG;
        const int row = i / H, col = i - row * H;
        gval[q] = row < H;
        goff[q] = gval[q] ? clampi(y0 - RXY + row, a.ny) * a.nx + clampi(x0 - RXY + col, a.nx) : 0;
        soff[q] = gval[q] ? row * PW + col : 0;
    }
    float pre[NQ];
    auto fetch = [&](int pl) {
        const float* src = a.img + (long)clampi(z0 - RZ + min(pl, nplanes - 1), a.nz) * plane;
#pragma unroll
        for (int q = 0; q < NQ; ++q) pre[q] = src[goff[q]];
    };
    fetch(grp);

    for (int p0 = 0; p0 < nplanes; p0 += PPS) {
        const int p = p0 + grp;  // this group's plane
        const bool live = p < nplanes;
        // the epilogue input of this step's output, requested before the passes
        const long idx = (long)clampi(z0 + p - 2 * RZ, a.nz) * plane + col_off;
        const float epi_v = epi[idx];
        // stash the prefetched plane, then request the group's next one
        if (live) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (gval[q]) sm[soff[q]] = pre[q];
        }
        fetch(p + PPS);
        __syncthreads();
        // x pass: one item per (row, run of 4 columns)
        if (live) {
            for (int i = tl; i < H * (PTS / PRUN); i += PG) {
                const int row = i % H, run = i / H;
                window_x<RXY, PRUN>(sm + row * PW + run * PRUN, RXY, sx + run * PRUN * PXH + row, PXH);
            }
        }
        __syncthreads();
        // y pass: one item per (column, run of 4 rows), into the ring slot of plane p
        if (live && tl < PTS * (PTS / PRUN)) {
            const int col = tl % PTS, run = tl / PTS;
            const double2* xs = sx + col * PXH + run * PRUN;
            double2* ys = s_y + (p % RING) * PG + run * PRUN * PTS + col;
            double u1 = 0.0, u2 = 0.0;
#pragma unroll
            for (int j = 0; j <= 2 * RXY; ++j) {
                const double2 v = xs[j];
                u1 += v.x;
                u2 += v.y;
            }
            ys[0] = make_double2(u1, u2);
#pragma unroll
            for (int rr = 1; rr < PRUN; ++rr) {
                const double2 vi = xs[rr + 2 * RXY], vo = xs[rr - 1];
                u1 += vi.x - vo.x;
                u2 += vi.y - vo.y;
                ys[rr * PTS] = make_double2(u1, u2);
            }
        }
        __syncthreads();
        // z: the window ending at plane e = p (planes e - PZ + 1 .. e)
        if (live && p >= PZ - 1 && own) {
            double z1s = 0.0, z2s = 0.0;
#pragma unroll
            for (int k = 0; k < PZ; ++k) {
                const double2 v = s_y[((p - k) % RING) * PG + tl];
                z1s += v.x;
                z2s += v.y;
            }
            const double mu = z1s * a.inv_n;
            double var = z2s * a.inv_n - mu * mu;
            var = var > 0.0 ? var : 0.0;
            mom_epilogue<MODE>(a, idx, mu, var, epi_v);
        }
        __syncthreads();
    }
}

template <int PZ, int MODE>
void launch_pp_kernel(const MomArgs& a, hipStream_t st)
{
    constexpr size_t lds = PpLds<PZ, PZ / 2>::BYTES;
    static_assert(lds <= 160 * 1024, "fits the LDS of one CU");
    lds_limit((const void*)k_moments_pp<PZ, PZ / 2, MODE>, lds);
    hipLaunchKernelGGL((k_moments_pp<PZ, PZ / 2, MODE>), dim3(a.nblocks), dim3(PPS * PG), lds, st, a);
}

template <int MODE>
hipError_t launch_pp(int pz, hipStream_t st, const MomArgs& a)
{
    switch (pz) {
#define DISC_PZ(P) \
    case P: launch_pp_kernel<P, MODE>(a, st); break;
        DISC_PZ(1) DISC_PZ(3) DISC_PZ(5) DISC_PZ(7) DISC_PZ(9) DISC_PZ(11) DISC_PZ(13) DISC_PZ(15)
#undef DISC_PZ
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PZ, int RXY, int MODE, int TS>
void launch_kernel(const MomArgs& a, hipStream_t st)
{
    constexpr size_t lds = MomLds<RXY, TS>::BYTES;
    static_assert(lds >= TS * TS * sizeof(double), "room for the loss reduction");
    lds_limit((const void*)k_moments<PZ, RXY, MODE, TS>, lds);
    hipLaunchKernelGGL((k_moments<PZ, RXY, MODE, TS>), dim3(a.nblocks), dim3(TS * TS), lds, st, a);
}

template <int PZ, int MODE, int TS>
void launch_one(const MomArgs& a, hipStream_t st)
{
    // the once-per-registration a_m pass uses the generic in-plane radius only
    if (MODE != kAmed && a.rx == PZ / 2 && a.ry == PZ / 2)
        launch_kernel<PZ, PZ / 2, MODE, TS>(a, st);
    else
        launch_kernel<PZ, -1, MODE, TS>(a, st);
}

template <int MODE, int TS>
hipError_t launch_pz(int pz, hipStream_t st, const MomArgs& a)
{
    switch (pz) {
#define DISC_PZ(P) \
    case P: launch_one<P, MODE, TS>(a, st); break;
        DISC_PZ(1) DISC_PZ(3) DISC_PZ(5) DISC_PZ(7) DISC_PZ(9) DISC_PZ(11) DISC_PZ(13) DISC_PZ(15)
#undef DISC_PZ
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Workgroup grid of the sweep for these dims (shared by the launcher and the
// SSD partial-sum sizing).
struct MomGrid {
    int TS, tiles_x, tiles_y, zchunk, nblocks;
};

MomGrid mom_grid_for(Dims d, int TS, int target, int min_chunk)
{
    MomGrid g;
    g.TS = TS;
    g.tiles_x = (d.nx + TS - 1) / TS;
    g.tiles_y = (d.ny + TS - 1) / TS;
    const int tiles = g.tiles_x * g.tiles_y;
    int chunks = (target + tiles - 1) / tiles;
    const int max_chunks = (d.nz + min_chunk - 1) / min_chunk;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    g.zchunk = (d.nz + chunks - 1) / chunks;
    chunks = (d.nz + g.zchunk - 1) / g.zchunk;
    g.nblocks = tiles * chunks;
    return g;
}

MomGrid mom_grid(Dims d)
{
    // Large volumes: 32 x 32 tiles, about one 1024-thread workgroup per CU and
    // z chunks of >= 16 planes. Small volumes: 16 x 16 tiles and short chunks,
    // trading halo planes for parallelism.
    const int t32 = ((d.nx + 31) / 32) * ((d.ny + 31) / 32);
    const bool big = (long)t32 * d.nz >= 256L * 16;
    return big ? mom_grid_for(d, 32, 256, 16) : mom_grid_for(d, 16, 1024, 2);
}

// Mode-specific pointers of the sweep (static, mask and a_m passes).
struct MomArgsExtra {
    float* sd_out;
    const float* s_img;
    const float* sd_s;
    float2* ab;
    unsigned char* stamp;
    const float* consts;
};

template <int MODE>
hipError_t launch_moments(const float* img, const float* ys_in, float* out, double2* bg,
                          double* partial, Dims d, const int patch[3], float tau, hipStream_t st,
                          const int* stop = nullptr, const MomArgsExtra* x = nullptr)
{
    MomArgs a{};
    a.stop = stop;
    a.img = img;
    a.ys_in = ys_in;
    a.out = out;
    a.bg = bg;
    a.partial = partial;
    if (x) {
        a.sd_out = x->sd_out;
        a.s_img = x->s_img;
        a.sd_s = x->sd_s;
        a.ab = x->ab;
        a.stamp = x->stamp;
        a.consts = x->consts;
    }
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.rx = patch[0] / 2;
    a.ry = patch[1] / 2;
    a.tau = tau;
    a.inv_n = 1.0 / ((double)patch[0] * patch[1] * patch[2]);
    const MomGrid g = mom_grid(d);
    const bool iso = patch[0] == patch[2] && patch[1] == patch[2];
    if (g.TS == 16 && iso && (MODE == kCorrect || MODE == kStatic)) {
        // small volume: several planes per step, about one workgroup per CU
        const MomGrid gp = mom_grid_for(d, PTS, 256, 1);
        a.tiles_x = gp.tiles_x;
        a.tiles_y = gp.tiles_y;
        a.zchunk = gp.zchunk;
        a.nblocks = gp.nblocks;
        return launch_pp<MODE == kStatic ? kStatic : kCorrect>(patch[2], st, a);
    }
    a.tiles_x = g.tiles_x;
    a.tiles_y = g.tiles_y;
    a.zchunk = g.zchunk;
    a.nblocks = g.nblocks;
    return g.TS == 32 ? launch_pz<MODE, 32>(patch[2], st, a) : launch_pz<MODE, 16>(patch[2], st, a);
}

// Batched correction pass (every volume shares the patch and the tile edge).
template <int PZ, int RXY, int TS>
void launch_batch_kernel(const Batch<MomArgs>& b, hipStream_t st)
{
    constexpr size_t lds = MomLds<RXY, TS>::BYTES;
    lds_limit((const void*)k_moments_batch<PZ, RXY, kCorrect, TS>, lds);
    hipLaunchKernelGGL((k_moments_batch<PZ, RXY, kCorrect, TS>), dim3(b.start[b.n]), dim3(TS * TS), lds,
                       st, b);
}

template <int TS>
hipError_t launch_batch_pz(const Batch<MomArgs>& b, const int patch[3], hipStream_t st)
{
    const bool iso = patch[0] == patch[2] && patch[1] == patch[2];
    switch (patch[2]) {
#define DISC_PZ(P)                                          \
    case P:                                                 \
        if (iso)                                            \
            launch_batch_kernel<P, P / 2, TS>(b, st);       \
        else                                                \
            launch_batch_kernel<P, -1, TS>(b, st);          \
        break;
        DISC_PZ(1) DISC_PZ(3) DISC_PZ(5) DISC_PZ(7) DISC_PZ(9) DISC_PZ(11) DISC_PZ(13) DISC_PZ(15)
#undef DISC_PZ
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_static_stats(const float* s, float* ys, Dims d, const int patch[3], float tau,
                               hipStream_t st, float* sd)
{
    if (!sd) return launch_moments<kStatic>(s, nullptr, ys, nullptr, nullptr, d, patch, tau, st);
    MomArgsExtra x{};
    x.sd_out = sd;
    return launch_moments<kStatic>(s, nullptr, ys, nullptr, nullptr, d, patch, tau, st, nullptr, &x);
}

hipError_t launch_mask_moments(const float* m, const float* ys, const float* s, const float* sd, float2* ab,
                               unsigned char* stamp, const float* consts, Dims d, const int patch[3],
                               hipStream_t st, const int* stop)
{
    MomArgsExtra x{};
    x.s_img = s;
    x.sd_s = sd;
    x.ab = ab;
    x.stamp = stamp;
    x.consts = consts;
    return launch_moments<kMask>(m, ys, nullptr, nullptr, nullptr, d, patch, 0.0f, st, stop, &x);
}

hipError_t launch_amed_values(const float* ct, const float* ys, const float* sd, float* a_out, Dims d,
                              const int patch[3], float tau, hipStream_t st)
{
    MomArgsExtra x{};
    x.sd_s = sd;
    return launch_moments<kAmed>(ct, ys, a_out, nullptr, nullptr, d, patch, tau, st, nullptr, &x);
}

hipError_t launch_correct(const float* m, const float* ys, float* f, Dims d, const int patch[3],
                          hipStream_t st, const int* stop)
{
    // isotropic patches: the z-first sweep (correct_zf.hip), one round of
    // resident 512-thread workgroups on large volumes (three per CU at 11^3:
    // 32.8 against 35.3 us at 256 x 256 x 96 with two), 256 on small ones
    // (128 x 128 x 48: 11 against 13 us)
    if (correct_zf_applies(d, patch)) {
        const long t32 = (long)((d.nx + 31) / 32) * ((d.ny + 31) / 32);
        return launch_correct_zf(m, ys, f, d, patch, st, stop,
                                 t32 * d.nz >= 4096 ? 256 * correct_zf_resident(patch) : 256);
    }
    return launch_moments<kCorrect>(m, ys, f, nullptr, nullptr, d, patch, 0.0f, st, stop);
}

int ssd_partial_count(Dims d)
{
    return mom_grid(d).nblocks;
}

hipError_t launch_ssd_moments(const float* m, const float* ys, float* dres, double2* bg, double* partial,
                              Dims d, const int patch[3], hipStream_t st)
{
    return launch_moments<kSsd>(m, ys, dres, bg, partial, d, patch, 0.0f, st);
}

hipError_t launch_correct_batch(const BatchVol* vols, int n, const int patch[3], const BatchTiles& tiles,
                                hipStream_t st)
{
    if (n < 1 || n > kMaxBatch || (tiles.mom_ts != 16 && tiles.mom_ts != 32)) return hipErrorInvalidValue;
    // 32 x 32 tiles and an isotropic patch: the z-first sweep, two 512-thread
    // workgroups for every 1024-thread one of mom_target
    if (tiles.mom_ts == 32 && correct_zf_batch_applies(patch))
        return launch_correct_zf_batch(vols, n, patch, 2 * tiles.mom_target, st);
    Batch<MomArgs> b{};
    b.n = n;
    b.start[0] = 0;
    for (int v = 0; v < n; ++v) {
        MomArgs& a = b.v[v];
        a.img = vols[v].m;
        a.ys_in = vols[v].ys;
        a.out = vols[v].f;
        a.bg = nullptr;
        a.partial = nullptr;
        a.stop = nullptr;
        a.nx = vols[v].d.nx;
        a.ny = vols[v].d.ny;
        a.nz = vols[v].d.nz;
        a.rx = patch[0] / 2;
        a.ry = patch[1] / 2;
        a.tau = 0.0f;
        a.inv_n = 1.0 / ((double)patch[0] * patch[1] * patch[2]);
        const MomGrid g = mom_grid_for(vols[v].d, tiles.mom_ts, tiles.mom_target, tiles.mom_ts == 32 ? 16 : 2);
        a.tiles_x = g.tiles_x;
        a.tiles_y = g.tiles_y;
        a.zchunk = g.zchunk;
        a.nblocks = g.nblocks;
        b.start[v + 1] = b.start[v] + g.nblocks;
    }
    return tiles.mom_ts == 32 ? launch_batch_pz<32>(b, patch, st) : launch_batch_pz<16>(b, patch, st);
}

}  // namespace disc
