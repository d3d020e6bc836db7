// Eq. 1 force, the Algorithm A1 step-5 update and the step-6 Gaussian
// regularisation of the displacement field, as two kernels for gfx950:
//
//   k_plane_pipe  one workgroup per 32 x 32 tile and chunk of z planes. It
//               forms r~ = r - u on the tile plus the R-voxel Gaussian halo
//               (R = ceil(3 sigma)), u being the Eq. 1 demons force on the
//               corrected image f (three f planes are staged in LDS for the
//               gradient), then runs the x and y passes out of LDS with
//               register-blocked runs of 8 (x) and 4 (y) outputs and writes
//               the xy-filtered field q; the four stages are
//               software-pipelined over planes.
//   k_smooth_z  one thread per (x, y) column over a chunk of z: a register
//               ring of the last 2R + 1 planes of q gives the z pass, and the
//               CT is warped with the new field for the next iteration. Halo
//               planes of a chunk are only re-read, never re-filtered.
//
// Splitting at the xy / z boundary keeps every filter pass free of
// redundant halo arithmetic in z (the 13-tap passes are VALU-bound on this
// chip) while the force is fused where its inputs are already resident.
// Taps are applied in ascending offset order in every pass.
#include "kernels.h"

namespace disc {

namespace {

constexpr int SRUN = 4;  // outputs per y-pass item
// outputs per x-pass item (a multiple of 4): 3 x 44 rows x 4 items fit one
// pass of the 1024 threads at R = 6, where runs of 4 need 1056 items
// (force + xy 53.4 against 54.2 us at 256 x 256 x 96)
constexpr int XRUN = 8;

struct PlaneArgs {
    const float* m;    // deformed moving image (force mode)
    const float* f;    // corrected static image (force mode)
    const float* r;    // field r (force mode) or r~ (plain smoothing)
    float* q;          // xy-filtered r~
    float* rt;         // optional copy of r~ (force mode), may be null
    const int* stop;   // level's stop flag (stopping rule), may be null
    int nx, ny, nz;
    int zchunk;
    int tiles_x, tiles_y, nblocks;
    float eps_d;
    GaussTaps taps;
};

// ---- force + xy smoothing, software-pipelined over planes ------------------
// FM: 0 smoothing only, 1 Eq. 1 static-gradient force, 2 both Eq. 1 terms.
// A workgroup owns a 32 x 32 column tile and a z chunk. Four stages per
// plane: stash the f (and m) region in LDS; form r~ = r - u on the tile
// plus halo; the x pass; the y pass into q. Step s runs the stash of the f
// region of plane s+1 (the m region of plane s), the force of plane s-1,
// the x pass of plane s-2 and the y pass of plane s-3, so one barrier per
// plane separates them and no stage waits for another. The f regions sit in
// four LDS slots, so the force reads the z neighbours of f (planes s-2 and
// s) from LDS as it reads the in-plane ones: f is fetched from memory once
// per plane (at 512 x 512 x 160, where the working set is far beyond the
// Infinity Cache, re-reading them per point cost 16 % of the kernel). The
// other LDS buffers are double-buffered. Global loads run ahead: the f
// region of plane s+2 and the per-point data of plane s+1 are requested in
// step s (the per-point data is consumed in step s+2, hence two register
// sets and steps taken in pairs).
constexpr int QTX = 32, QTY = 32;

template <int R, int FM>
struct PipeLds {
    static constexpr int W = QTX + 2 * R, PW = (W + 3) & ~3, H = QTY + 2 * R;
    static constexpr int FW = W + 2, FH = H + 2;
    static constexpr size_t F_BYTES = (size_t)FH * FW * sizeof(float);
    static constexpr size_t IN_BYTES = (size_t)3 * H * PW * sizeof(float);
    static constexpr size_t X_BYTES = (size_t)3 * H * QTX * sizeof(float);
    // f: four plane slots (z - 1, z, z + 1 of the plane whose force is formed, and
    // the one being stashed); m (double force): two
    static constexpr int F_SLOTS = FM > 0 ? 4 : 0, M_SLOTS = FM == 2 ? 2 : 0;
    static constexpr size_t BYTES = (F_SLOTS + M_SLOTS) * F_BYTES + 2 * (IN_BYTES + X_BYTES);
};

template <int R, int FM>
__device__ __forceinline__ void plane_pipe_body(const PlaneArgs& a, const int bid)
{
    constexpr bool FORCE = FM > 0, DBL = FM == 2;
    constexpr int NT = QTX * QTY;
    constexpr int K = 2 * R + 1;
    using L = PipeLds<R, FM>;
    constexpr int W = L::W, PW = L::PW, H = L::H, FW = L::FW, FH = L::FH;
    constexpr int XITEMS = 3 * H * (QTX / XRUN);
    constexpr int YITEMS = 3 * QTX * (QTY / SRUN);
    constexpr int NF = FORCE ? (FH * FW + NT - 1) / NT : 1;
    constexpr int NP = (H * W + NT - 1) / NT;
    static_assert(YITEMS <= NT, "one y item per thread");
    if (a.stop && *a.stop) return;  // the level has met its stopping rule

    extern __shared__ __align__(16) unsigned char smem[];
    float* s_f0 = reinterpret_cast<float*>(smem);                                         // [4][FH*FW]
    float* s_mm0 = s_f0 + L::F_SLOTS * FH * FW;                                           // [2][FH*FW] (DBL)
    float* s_in0 = reinterpret_cast<float*>(smem + (L::F_SLOTS + L::M_SLOTS) * L::F_BYTES);  // [2][3][H][PW]
    float* s_x0 = s_in0 + 2 * 3 * H * PW;                                                 // [2][3][H][QTX]

    const int lb = xcd_logical_block(bid, a.nblocks);
    const int bx = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * QTX, y0 = by * QTY;
    const int z0 = bz * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    // element offsets fit in 32 bits (the ABI bounds N below 2^30)
    const int plane = a.nx * a.ny;
    const long N = (long)plane * a.nz;

    // per-thread geometry, fixed over the sweep. Region point q of this
    // thread sits at clamped voxel (gx, gy); its f neighbours are the clamped
    // voxels, looked up inside the staged f region.
    int foff[NF], pofs[NP], pslot[NP], fc_[NP], fxp_[NP], fxm_[NP], fyp_[NP], fym_[NP];
    bool fval[NF], pval[NP], pint[NP];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const int i = t + q * NT;
        fval[q] = FORCE && i < FH * FW;
        if (fval[q]) {
            const int row = i / FW, col = i - row * FW;
            foff[q] = clampi(y0 - R - 1 + row, a.ny) * a.nx + clampi(x0 - R - 1 + col, a.nx);
        } else {
            foff[q] = 0;  // loaded but never stored: keeps the load branch-free
        }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int i = t + q * NT;
        const int row = i / W, col = i - row * W;
        if (i < H * W) {
            const int gx = clampi(x0 - R + col, a.nx), gy = clampi(y0 - R + row, a.ny);
            pofs[q] = gy * a.nx + gx;
            pslot[q] = row * PW + col;
            const int bxf = x0 - R - 1, byf = y0 - R - 1;
            fc_[q] = (gy - byf) * FW + (gx - bxf);
            fxp_[q] = (gy - byf) * FW + (clampi(gx + 1, a.nx) - bxf);
            fxm_[q] = (gy - byf) * FW + (clampi(gx - 1, a.nx) - bxf);
            fyp_[q] = (clampi(gy + 1, a.ny) - byf) * FW + (gx - bxf);
            fym_[q] = (clampi(gy - 1, a.ny) - byf) * FW + (gx - bxf);
            pint[q] = row >= R && row < R + QTY && col >= R && col < R + QTX && x0 - R + col < a.nx &&
                      y0 - R + row < a.ny;
            pval[q] = true;
        } else {
            pofs[q] = pslot[q] = fc_[q] = fxp_[q] = fxm_[q] = fyp_[q] = fym_[q] = 0;
            pint[q] = false;
            pval[q] = false;
        }
    }

    const int nplanes = z1 - z0;
    // buffer access: fixed per-lane byte offsets (region slots), the plane a
    // scalar byte offset. Resources are rebuilt where used from the kernel
    // arguments (scalar work the compiler hoists; none is captured by a lambda)
    const long cb = N * 4;
    const int pb = plane * 4;
    // registers: the f region of the plane after next and the m region of the
    // next plane; per-point data in two sets. The f region is staged for
    // planes z0 - 1 .. z1 (clamped to the volume), so the force takes its z
    // neighbours, like its in-plane ones, from LDS.
    float pf[NF], pmf[DBL ? NF : 1];
    struct Pt {
        float r0[NP], r1[NP], r2[NP], m[NP], mu[DBL ? NP : 1], md[DBL ? NP : 1];
    };
    Pt setA, setB;
    auto fetch_f = [&](int p) {  // f region of plane z0 + p (clamped: always valid)
        if (FORCE) {
            const int so = clampi(z0 + p, a.nz) * pb;
            const Rsrc fb = make_rsrc(a.f, cb);
#pragma unroll
            for (int q = 0; q < NF; ++q) pf[q] = ld(fb, foff[q] * 4, so);
        }
    };
    auto fetch_m = [&](int p) {  // m region of plane z0 + p (double force; clamped)
        if (DBL) {
            const int so = (z0 + min(p, nplanes - 1)) * pb;
            const Rsrc mb = make_rsrc(a.m, cb);
#pragma unroll
            for (int q = 0; q < NF; ++q) pmf[q] = ld(mb, foff[q] * 4, so);
        }
    };
    // LDS slot of the f region of relative plane p (-1 .. nplanes)
    auto f_slot = [&](int p) { return s_f0 + ((p + 1) & 3) * (FH * FW); };
    auto stash_f = [&](int p) {
        float* sf = f_slot(p);
#pragma unroll
        for (int q = 0; q < NF; ++q)
            if (fval[q]) sf[t + q * NT] = pf[q];
    };
    auto fetch_points = [&](Pt& d, int p) {
        const int z = z0 + min(p, nplanes - 1);
        const int so = z * pb;
        const int su = clampi(z + 1, a.nz) * pb, sd = clampi(z - 1, a.nz) * pb;
        const Rsrc rb0 = make_rsrc(a.r, cb), rb1 = make_rsrc(a.r + N, cb), rb2 = make_rsrc(a.r + 2 * N, cb);
        const Rsrc mb = make_rsrc(a.m, cb);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int vo = pofs[q] * 4;
            d.r0[q] = ld(rb0, vo, so);
            d.r1[q] = ld(rb1, vo, so);
            d.r2[q] = ld(rb2, vo, so);
            if (FORCE) d.m[q] = ld(mb, vo, so);
            if (DBL) {
                d.mu[q] = ld(mb, vo, su);
                d.md[q] = ld(mb, vo, sd);
            }
        }
    };

    // one pipeline step; `par` is s & 1, `cur` holds the point data of plane
    // s - 1 (consumed here) and receives that of plane s + 1
    auto step = [&](int s, const int par, Pt& cur) {
        const int ps = s, pc = s - 1, px = s - 2, py = s - 3;
        // stash the f region of plane s + 1 (and the m region of plane s),
        // request those of planes s + 2 (and s + 1)
        if (FORCE && ps + 1 <= nplanes) stash_f(ps + 1);
        if (DBL && ps < nplanes) {
            float* smm = s_mm0 + par * (FH * FW);
#pragma unroll
            for (int q = 0; q < NF; ++q)
                if (fval[q]) smm[t + q * NT] = pmf[q];
        }
        fetch_f(ps + 2);
        fetch_m(ps + 1);
        // force of plane s - 1 on the tile plus halo: r~ = r - u (f of planes
        // s - 2, s - 1, s were stashed in earlier steps)
        if (pc >= 0 && pc < nplanes) {
            const float* sf = f_slot(pc);
            const float* sfu = f_slot(pc + 1);
            const float* sfd = f_slot(pc - 1);
            const float* smm = s_mm0 + (par ^ 1) * (FH * FW);
            float* sin = s_in0 + (par ^ 1) * (3 * H * PW);
            const int zoff = (z0 + pc) * plane;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                if (!pval[q]) continue;
                float w0 = cur.r0[q], w1 = cur.r1[q], w2 = cur.r2[q];
                if (FORCE) {
                    const float fcv = sf[fc_[q]];
                    const float gxv = (sf[fxp_[q]] - sf[fxm_[q]]) * 0.5f;
                    const float gyv = (sf[fyp_[q]] - sf[fym_[q]]) * 0.5f;
                    const float gzv = (sfu[fc_[q]] - sfd[fc_[q]]) * 0.5f;
                    const float d = cur.m[q] - fcv;
                    const float den = gxv * gxv + gyv * gyv + gzv * gzv + d * d;
                    if (den > 0.0f && fabsf(d) >= a.eps_d) {
                        // den >= d^2 >= eps_d^2 is a normal number: the hardware
                        // reciprocal (1 ulp) replaces the IEEE division sequence
                        const float sc = d * __builtin_amdgcn_rcpf(den);
                        w0 -= sc * gxv;
                        w1 -= sc * gyv;
                        w2 -= sc * gzv;
                    }
                    if (DBL) {
                        // second term of Eq. 1: the same with the gradient of m
                        const float hx = (smm[fxp_[q]] - smm[fxm_[q]]) * 0.5f;
                        const float hy = (smm[fyp_[q]] - smm[fym_[q]]) * 0.5f;
                        const float hz = (cur.mu[q] - cur.md[q]) * 0.5f;
                        const float den2 = hx * hx + hy * hy + hz * hz + d * d;
                        if (den2 > 0.0f && fabsf(d) >= a.eps_d) {
                            const float sc2 = d * __builtin_amdgcn_rcpf(den2);
                            w0 -= sc2 * hx;
                            w1 -= sc2 * hy;
                            w2 -= sc2 * hz;
                        }
                    }
                    if (a.rt && pint[q]) {
                        a.rt[zoff + pofs[q]] = w0;
                        a.rt[N + zoff + pofs[q]] = w1;
                        a.rt[2 * N + zoff + pofs[q]] = w2;
                    }
                }
                sin[pslot[q]] = w0;
                sin[H * PW + pslot[q]] = w1;
                sin[2 * H * PW + pslot[q]] = w2;
            }
        }
        fetch_points(cur, ps + 1);
        // x pass of plane s - 2: XRUN consecutive outputs of one row per item
        if (px >= 0 && px < nplanes) {
            const float* sin = s_in0 + par * (3 * H * PW);
            float* sx = s_x0 + par * (3 * H * QTX);
            for (int i = t; i < XITEMS; i += NT) {
                const int run = i % (QTX / XRUN), cr = i / (QTX / XRUN);
                const int c = cr / H, row = cr - c * H;
                const float* src = sin + (c * H + row) * PW + run * XRUN;
                float v[(XRUN + 2 * R + 3) & ~3];
#pragma unroll
                for (int j = 0; j < (XRUN + 2 * R + 3) / 4; ++j) {
                    const float4 w4 = *reinterpret_cast<const float4*>(src + 4 * j);
                    v[4 * j] = w4.x;
                    v[4 * j + 1] = w4.y;
                    v[4 * j + 2] = w4.z;
                    v[4 * j + 3] = w4.w;
                }
                float o[XRUN];
#pragma unroll
                for (int rr = 0; rr < XRUN; ++rr) {
                    float sacc = 0.0f;
#pragma unroll
                    for (int j = 0; j < K; ++j) sacc = fmaf(a.taps.w[j], v[rr + j], sacc);
                    o[rr] = sacc;
                }
#pragma unroll
                for (int g = 0; g < XRUN / 4; ++g)
                    *reinterpret_cast<float4*>(sx + (c * H + row) * QTX + run * XRUN + 4 * g) =
                        make_float4(o[4 * g], o[4 * g + 1], o[4 * g + 2], o[4 * g + 3]);
            }
        }
        // y pass of plane s - 3: 4 consecutive outputs of one column per item, to q
        if (py >= 0 && py < nplanes && t < YITEMS) {
            const float* sx = s_x0 + (par ^ 1) * (3 * H * QTX);
            const int col = t % QTX, cr = t / QTX;
            const int run = cr % (QTY / SRUN), c = cr / (QTY / SRUN);
            float v[SRUN + 2 * R];
#pragma unroll
            for (int j = 0; j < SRUN + 2 * R; ++j) v[j] = sx[(c * H + run * SRUN + j) * QTX + col];
            const int ox = x0 + col;
            // c is uniform per wave (QTX * QTY / SRUN = 256 items per component)
            const Rsrc qc = make_rsrc(a.q + __builtin_amdgcn_readfirstlane(c) * N, cb);
            const int so = (z0 + py) * pb;
#pragma unroll
            for (int rr = 0; rr < SRUN; ++rr) {
                float sacc = 0.0f;
#pragma unroll
                for (int j = 0; j < K; ++j) sacc = fmaf(a.taps.w[j], v[rr + j], sacc);
                const int oy = y0 + run * SRUN + rr;
                if (ox < a.nx && oy < a.ny) st(qc, (oy * a.nx + ox) * 4, so, sacc);
            }
        }
        __syncthreads();
    };

    // the f regions of planes z0 - 1 and z0 go to LDS up front (visible to
    // every wave after step 0's barrier, before the first force in step 1)
    if (FORCE) {
        fetch_f(-1);
        stash_f(-1);
        fetch_f(0);
        stash_f(0);
    }
    fetch_f(1);
    fetch_m(0);
    fetch_points(setB, 0);  // plane 0's point data, consumed in step 1 (odd)
    const int nsteps = nplanes + 3;
    for (int s = 0; s < nsteps; s += 2) {
        // even steps consume plane s - 1 (odd) from setA and refill it with plane s + 1
        step(s, 0, setA);
        if (s + 1 < nsteps) step(s + 1, 1, setB);
    }
}

template <int R, int FM>
__global__ __launch_bounds__(QTX* QTY) void k_plane_pipe(PlaneArgs a)
{
    plane_pipe_body<R, FM>(a, blockIdx.x);
}

template <int R, int FM>
__global__ __launch_bounds__(QTX* QTY) void k_plane_pipe_batch(Batch<PlaneArgs> b)
{
    const int v = batch_volume(b.start, b.n, blockIdx.x);
    plane_pipe_body<R, FM>(b.v[v], blockIdx.x - b.start[v]);
}

template <int R, int FM>
void launch_pipe_one(const PlaneArgs& a, hipStream_t st)
{
    constexpr size_t lds = PipeLds<R, FM>::BYTES;
    static_assert(lds <= 160 * 1024, "fits the LDS of one CU");
    lds_limit((const void*)k_plane_pipe<R, FM>, lds);
    hipLaunchKernelGGL((k_plane_pipe<R, FM>), dim3(a.nblocks), dim3(QTX * QTY), lds, st, a);
}

template <int R, int FM>
void launch_pipe_batch_one(const Batch<PlaneArgs>& b, hipStream_t st)
{
    constexpr size_t lds = PipeLds<R, FM>::BYTES;
    lds_limit((const void*)k_plane_pipe_batch<R, FM>, lds);
    hipLaunchKernelGGL((k_plane_pipe_batch<R, FM>), dim3(b.start[b.n]), dim3(QTX * QTY), lds, st, b);
}

struct ZArgs {
    const float* q;
    float* out;
    const int* stop;  // level's stop flag (stopping rule), may be null
    double* norms;    // NORM: per workgroup (sum |r_new - r_old|, sum |r_old|)
    const float* ct;  // WARP: the CT warped with the new field ...
    float* m;         // ... into m, the next iteration's deformed moving image
    int nx, ny, nz;
    int zchunk;
    int colblocks;  // workgroups across the columns of one z chunk
    long ncols;
    GaussTaps taps;
};

constexpr int ZNT = 256;
constexpr int ZPF = 4;  // planes of z-pass loads in flight per thread

// One workgroup: ZNT columns of one z chunk; bid = chunk * colblocks + column
// block. NORM: out holds r^(k) on entry; the workgroup also sums, in FP64,
// the Euclidean norms of r^(k+1) - r^(k) and of r^(k) over its voxels (the
// two sums of l^(k), Sec. 2.3).
template <int R, bool NORM, bool WARP>
__device__ __forceinline__ void smooth_z_body(const ZArgs& a, const int bid)
{
    constexpr int K = 2 * R + 1;
    if (a.stop && *a.stop) return;  // the level has met its stopping rule
    // block -> (column block, chunk): workgroups are dealt round-robin over
    // the 8 XCDs; XCD k takes the contiguous column blocks [kG, kG + G), one
    // chunk after the other, so the halo planes neighbouring chunks share and
    // the CT rows the warp gathers around neighbouring rows of the volume are
    // both re-read from that XCD's L2 (blocks past the end are idle)
    const int G = (a.colblocks + 7) / 8;
    const int nch = (a.nz + a.zchunk - 1) / a.zchunk;
    const int xcd = bid & 7, local = bid >> 3;
    const int cblk = xcd * G + local % G, chunk = local / G;
    if (cblk >= a.colblocks || chunk >= nch) {
        if (NORM && threadIdx.x == 0) {
            a.norms[2 * bid] = 0.0;
            a.norms[2 * bid + 1] = 0.0;
        }
        return;
    }
    const int col0 = cblk * ZNT + (int)threadIdx.x;
    if (!NORM && col0 >= (int)a.ncols) return;
    const bool act = col0 < (int)a.ncols;
    const int col = act ? col0 : (int)a.ncols - 1;  // idle lanes (NORM) read a valid column
    const int xcol = col % a.nx, ycol = col / a.nx;
    const int z0 = chunk * a.zchunk;
    const int z1 = min(a.nz, z0 + a.zchunk);
    // buffer access: the lane's column is the per-lane byte offset, the plane
    // a scalar offset; each field component has its own resource
    const int pb = a.nx * a.ny * 4;
    const long N = (long)a.nx * a.ny * a.nz;
    const long cb = N * 4;
    const Rsrc q0 = make_rsrc(a.q, cb), q1 = make_rsrc(a.q + N, cb), q2 = make_rsrc(a.q + 2 * N, cb);
    const Rsrc o0 = make_rsrc(a.out, cb), o1 = make_rsrc(a.out + N, cb), o2 = make_rsrc(a.out + 2 * N, cb);
    const int vo = col * 4;
    float ring[3][K];
    // the next ZPF planes, loads in flight (a short shift register)
    float nx_[ZPF][3];
    double s_dr = 0.0, s_r = 0.0;
    auto load = [&](int p, float* dst) {
        const int so = clampi(z0 - R + p, a.nz) * pb;
        dst[0] = ld(q0, vo, so);
        dst[1] = ld(q1, vo, so);
        dst[2] = ld(q2, vo, so);
    };
    const int nplanes = (z1 - z0) + 2 * R;
#pragma unroll
    for (int j = 0; j < ZPF; ++j) load(j, nx_[j]);  // clamped plane index: always a valid address
    for (int p0 = 0; p0 < nplanes; p0 += K) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int p = p0 + k;
            if (NORM ? p >= nplanes : false) continue;  // uniform guard keeps the loop unrollable
            if (!NORM && p >= nplanes) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ring[c][k] = nx_[0][c];
#pragma unroll
                for (int j = 0; j + 1 < ZPF; ++j) nx_[j][c] = nx_[j + 1][c];
            }
            load(p + ZPF, nx_[ZPF - 1]);  // past the chunk end this re-reads a clamped plane
            if (p >= K - 1) {
                const int oz = z0 + p - 2 * R;
                const int so = oz * pb;
                float nv[3], ov[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float sacc = 0.0f;
#pragma unroll
                    for (int j = 0; j < K; ++j) sacc = fmaf(a.taps.w[j], ring[c][(k + 1 + j) % K], sacc);
                    nv[c] = sacc;
                }
                if (NORM) {
                    ov[0] = ld(o0, vo, so);
                    ov[1] = ld(o1, vo, so);
                    ov[2] = ld(o2, vo, so);
                }
                if (act) {
                    st(o0, vo, so, nv[0]);
                    st(o1, vo, so, nv[1]);
                    st(o2, vo, so, nv[2]);
                    if (WARP) {
                        const WarpSrc w = warp_src(a.ct, a.nx, a.ny, a.nz);
                        st(make_rsrc(a.m, cb), vo, so, warp_at(w, xcol, ycol, oz, nv[0], nv[1], nv[2]));
                    }
                }
                if (NORM && act) {
                    const float dx = nv[0] - ov[0], dy = nv[1] - ov[1], dz = nv[2] - ov[2];
                    s_dr += (double)sqrtf(dx * dx + dy * dy + dz * dz);
                    s_r += (double)sqrtf(ov[0] * ov[0] + ov[1] * ov[1] + ov[2] * ov[2]);
                }
            }
        }
    }
    if (NORM) {
        // fixed-order tree over the workgroup
        __shared__ double red[2][ZNT];
        const int t = threadIdx.x;
        red[0][t] = s_dr;
        red[1][t] = s_r;
        __syncthreads();
        for (int h = ZNT / 2; h > 0; h >>= 1) {
            if (t < h) {
                red[0][t] += red[0][t + h];
                red[1][t] += red[1][t + h];
            }
            __syncthreads();
        }
        if (t == 0) {
            a.norms[2 * bid] = red[0][0];
            a.norms[2 * bid + 1] = red[1][0];
        }
    }
}

template <int R, bool NORM, bool WARP>
__global__ __launch_bounds__(ZNT) void k_smooth_z(ZArgs a)
{
    smooth_z_body<R, NORM, WARP>(a, blockIdx.x);
}

template <int R, bool WARP>
__global__ __launch_bounds__(ZNT) void k_smooth_z_batch(Batch<ZArgs> b)
{
    const int v = batch_volume(b.start, b.n, blockIdx.x);
    smooth_z_body<R, false, WARP>(b.v[v], blockIdx.x - b.start[v]);
}

// One output voxel per thread (small volumes, where the chunk planner gives
// one-plane chunks): the 2R + 1 planes of its column are requested at once,
// instead of streaming them through the ring with two planes in flight.
template <int R, bool WARP>
__global__ __launch_bounds__(ZNT) void k_smooth_z_direct(ZArgs a)
{
    constexpr int K = 2 * R + 1;
    if (a.stop && *a.stop) return;  // the level has met its stopping rule
    // the block order of smooth_z_body with one-plane chunks
    const int G = (a.colblocks + 7) / 8;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int cblk = xcd * G + local % G, z = local / G;
    if (cblk >= a.colblocks || z >= a.nz) return;
    const int col = cblk * ZNT + (int)threadIdx.x;
    if (col >= (int)a.ncols) return;
    const int pb = a.nx * a.ny * 4;
    const long N = (long)a.nx * a.ny * a.nz;
    const long cb = N * 4;
    const Rsrc q0 = make_rsrc(a.q, cb), q1 = make_rsrc(a.q + N, cb), q2 = make_rsrc(a.q + 2 * N, cb);
    const int vo = col * 4;
    float v[3][K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int so = clampi(z - R + j, a.nz) * pb;
        v[0][j] = ld(q0, vo, so);
        v[1][j] = ld(q1, vo, so);
        v[2][j] = ld(q2, vo, so);
    }
    float nv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float sacc = 0.0f;
#pragma unroll
        for (int j = 0; j < K; ++j) sacc = fmaf(a.taps.w[j], v[c][j], sacc);
        nv[c] = sacc;
    }
    const int so = z * pb;
    st(make_rsrc(a.out, cb), vo, so, nv[0]);
    st(make_rsrc(a.out + N, cb), vo, so, nv[1]);
    st(make_rsrc(a.out + 2 * N, cb), vo, so, nv[2]);
    if (WARP) {
        const WarpSrc w = warp_src(a.ct, a.nx, a.ny, a.nz);
        st(make_rsrc(a.m, cb), vo, so, warp_at(w, col % a.nx, col / a.nx, z, nv[0], nv[1], nv[2]));
    }
}

// Sec. 2.3 stopping rule after iteration k of a level: l^(k) = sum |dr| /
// sum |r| from the workgroup partial sums (fixed order), recorded in hist[k];
// flags[0] := 1 once k >= lag and hist[k - lag] - l^(k) <= eps; flags[1]
// counts the iterations run.
__global__ __launch_bounds__(256) void k_stop_rule(const double* __restrict__ norms, int nparts,
                                                  double* __restrict__ hist, int* __restrict__ flags,
                                                  int k, int lag, double eps)
{
    if (flags[0]) return;
    __shared__ double red[2][256];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (int i = t; i < nparts; i += 256) {
        a0 += norms[2 * i];
        a1 += norms[2 * i + 1];
    }
    red[0][t] = a0;
    red[1][t] = a1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double num = red[0][0], den = red[1][0];
        const double l = den > 0.0 ? num / den : (num > 0.0 ? __builtin_huge_val() : 0.0);
        hist[k] = l;
        flags[1] = k + 1;
        if (k >= lag && hist[k - lag] - l <= eps) flags[0] = 1;
    }
}

// Tile of the xy kernel: 32 x 32 columns, 1024 threads.
constexpr int PTX = QTX;
constexpr int PTY = QTY;

template <int FM>
hipError_t launch_plane(const PlaneArgs& a, int R, hipStream_t st)
{
    switch (R) {
#define DISC_R(RR) \
    case RR: launch_pipe_one<RR, FM>(a, st); break;
        DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// z chunks: about `target` workgroups in the launch (measured best at 4096
// for the 256x256x96 registration: 6-plane chunks re-read 2R halo planes
// per 6 outputs, and still leave enough waves in flight for the fused
// warp's gathers); re-read halo planes come from cache.
ZArgs z_args(const float* q, float* out, Dims d, const GaussTaps& t, int target = 4096)
{
    ZArgs a;
    a.q = q;
    a.out = out;
    a.stop = nullptr;
    a.norms = nullptr;
    a.ct = nullptr;
    a.m = nullptr;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.ncols = (long)d.nx * d.ny;
    a.taps = t;
    const long colblocks = (a.ncols + ZNT - 1) / ZNT;
    int chunks = (int)((target + colblocks - 1) / colblocks);
    if (chunks > d.nz) chunks = d.nz;
    if (chunks < 1) chunks = 1;
    a.zchunk = (d.nz + chunks - 1) / chunks;
    // chunks of fewer than four planes re-read 2R halo planes per output or
    // two; use four whenever that still leaves about 512 workgroups
    // (measured: 128 x 128 x 48 at sigma 2, 17 -> 14 us)
    if (a.zchunk < 4 && colblocks * ((d.nz + 3) / 4) >= 512) a.zchunk = 4;
    a.colblocks = (int)colblocks;
    return a;
}

int z_blocks(const ZArgs& a)
{
    // (column blocks padded to a multiple of 8, see smooth_z_body)
    return 8 * ((a.colblocks + 7) / 8) * ((a.nz + a.zchunk - 1) / a.zchunk);
}

hipError_t launch_z(const float* q, float* out, Dims d, const GaussTaps& t, const int* stop, double* norms,
                    const float* ct, float* m, hipStream_t st)
{
    ZArgs a = z_args(q, out, d, t);
    a.stop = stop;
    a.norms = norms;
    a.ct = ct;
    a.m = m;
    const bool w = ct && m;
    const dim3 g((unsigned)z_blocks(a));
    if (!norms && a.zchunk == 1) {
        // one-plane chunks: every thread requests its whole column window at once
        switch (t.R) {
#define DISC_R(RR)                                                                          \
    case RR:                                                                                \
        if (w)                                                                              \
            hipLaunchKernelGGL((k_smooth_z_direct<RR, true>), g, dim3(ZNT), 0, st, a);      \
        else                                                                                \
            hipLaunchKernelGGL((k_smooth_z_direct<RR, false>), g, dim3(ZNT), 0, st, a);     \
        break;
            DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (t.R) {
#define DISC_R(RR)                                                                          \
    case RR:                                                                                \
        if (norms && w)                                                                     \
            hipLaunchKernelGGL((k_smooth_z<RR, true, true>), g, dim3(ZNT), 0, st, a);       \
        else if (norms)                                                                     \
            hipLaunchKernelGGL((k_smooth_z<RR, true, false>), g, dim3(ZNT), 0, st, a);      \
        else if (w)                                                                         \
            hipLaunchKernelGGL((k_smooth_z<RR, false, true>), g, dim3(ZNT), 0, st, a);      \
        else                                                                                \
            hipLaunchKernelGGL((k_smooth_z<RR, false, false>), g, dim3(ZNT), 0, st, a);     \
        break;
        DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// about `target` workgroups (measured best at 256: one 1024-thread workgroup
// per CU, longer z chunks)
PlaneArgs plane_args(Dims d, const GaussTaps& t, int tx = PTX, int ty = PTY, int target = 256)
{
    PlaneArgs a{};
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.tiles_x = (d.nx + tx - 1) / tx;
    a.tiles_y = (d.ny + ty - 1) / ty;
    // z chunks: about `target` workgroups in the launch
    const int tiles = a.tiles_x * a.tiles_y;
    int chunks = (target + tiles - 1) / tiles;
    if (chunks > d.nz) chunks = d.nz;
    if (chunks < 1) chunks = 1;
    a.zchunk = (d.nz + chunks - 1) / chunks;
    chunks = (d.nz + a.zchunk - 1) / a.zchunk;
    a.nblocks = tiles * chunks;
    a.taps = t;
    return a;
}

}  // namespace

hipError_t launch_force_xy(const float* m, const float* f, const float* r, float* q, float* rt,
                           Dims d, float eps_d, int force_mode, const GaussTaps& t, const int* stop,
                           hipStream_t st)
{
    PlaneArgs a = plane_args(d, t);
    a.m = m;
    a.f = f;
    a.r = r;
    a.q = q;
    a.rt = rt;
    a.stop = stop;
    a.eps_d = eps_d;
    return force_mode == 1 ? launch_plane<2>(a, t.R, st) : launch_plane<1>(a, t.R, st);
}

hipError_t launch_smooth_xy(const float* rt, float* q, Dims d, const GaussTaps& t, hipStream_t st)
{
    PlaneArgs a = plane_args(d, t);
    a.r = rt;
    a.q = q;
    a.stop = nullptr;
    return launch_plane<0>(a, t.R, st);
}

hipError_t launch_smooth_z(const float* q, float* out, Dims d, const GaussTaps& t, const int* stop,
                           double* norms, hipStream_t st, const float* ct, float* m)
{
    return launch_z(q, out, d, t, stop, norms, ct, m, st);
}

int smooth_z_blocks(Dims d)
{
    GaussTaps t{};
    return z_blocks(z_args(nullptr, nullptr, d, t));
}

hipError_t launch_stop_rule(const double* norms, int nparts, double* hist, int* flags, int k, int lag,
                            double eps, hipStream_t st)
{
    hipLaunchKernelGGL(k_stop_rule, dim3(1), dim3(256), 0, st, norms, nparts, hist, flags, k, lag, eps);
    return hipGetLastError();
}

hipError_t launch_force_xy_batch(const BatchVol* vols, int n, float eps_d, int force_mode, const GaussTaps& t,
                                 int target, hipStream_t st)
{
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    Batch<PlaneArgs> b{};
    b.n = n;
    b.start[0] = 0;
    for (int v = 0; v < n; ++v) {
        PlaneArgs& a = b.v[v];
        a = plane_args(vols[v].d, t, PTX, PTY, target);
        a.m = vols[v].m;
        a.f = vols[v].f;
        a.r = vols[v].r;
        a.q = vols[v].q;
        a.rt = nullptr;
        a.stop = nullptr;
        a.eps_d = eps_d;
        b.start[v + 1] = b.start[v] + a.nblocks;
    }
    switch (t.R) {
#define DISC_R(RR)                           \
    case RR:                                 \
        if (force_mode == 1)                 \
            launch_pipe_batch_one<RR, 2>(b, st); \
        else                                 \
            launch_pipe_batch_one<RR, 1>(b, st); \
        break;
        DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smooth_z_batch(const BatchVol* vols, int n, const GaussTaps& t, int target, bool warp,
                                 hipStream_t st)
{
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    Batch<ZArgs> b{};
    b.n = n;
    b.start[0] = 0;
    for (int v = 0; v < n; ++v) {
        b.v[v] = z_args(vols[v].q, vols[v].r, vols[v].d, t, target);
        if (warp) {
            b.v[v].ct = vols[v].ct;
            b.v[v].m = vols[v].m;
        }
        b.start[v + 1] = b.start[v] + z_blocks(b.v[v]);
    }
    const dim3 g((unsigned)b.start[n]);
    switch (t.R) {
#define DISC_R(RR)                                                                            \
    case RR:                                                                                  \
        if (warp)                                                                             \
            hipLaunchKernelGGL((k_smooth_z_batch<RR, true>), g, dim3(ZNT), 0, st, b);        \
        else                                                                                  \
            hipLaunchKernelGGL((k_smooth_z_batch<RR, false>), g, dim3(ZNT), 0, st, b);       \
        break;
        DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace disc
