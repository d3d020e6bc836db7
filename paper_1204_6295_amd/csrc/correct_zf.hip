// Patch moments (Eq. 3) and the moment-matching correction (Eq. 5-6) for
// isotropic patches on large volumes, z first.
//
// A workgroup of 512 threads (768 at 15^3) owns a 32 x 32 column tile and a
// chunk of output planes. Every column of the tile plus its in-plane patch
// halo keeps the FP64 sums of m and m^2 over its z window in registers,
// advanced by one plane per step (add the plane entering the window,
// subtract the one leaving it; both loads are requested one step ahead).
// Per output plane:
//   store   the column sums in LDS;                         barrier
//   x pass  sliding sums along x of those, 4 outputs per item, one lane per
//           region row (row-fastest lanes: conflict-free 16-byte accesses);
//                                                            barrier
//   y pass  sliding sums along y, 2 outputs per item (512 items), then
//           the epilogue I'_s = E(M) + STD(M) Y at those voxels.
// The x and y passes run only on output planes (the z halo costs one add
// per column and plane). The kernel is held to 80 VGPRs (six waves per
// SIMD), so with its 51 KB of LDS at 11^3 three workgroups share a CU and
// one workgroup's barrier waits overlap the others' work.
// Used for isotropic patches up to 15^3 at every volume size (batches: up to
// 13^3).
#include <cmath>

#include "kernels.h"

namespace disc {

namespace {

constexpr int ZTS = 32;   // output tile edge
// threads per workgroup: 512 up to 13^3; 768 at 15^3, whose 46 x 46 region
// columns then take three per thread
template <int PZ>
constexpr int zf_threads() { return PZ <= 13 ? 512 : 768; }
constexpr int XRUN = 4;   // outputs per x item
constexpr int YRUN = 2;   // outputs per y item (every thread takes one)
constexpr int ZPF = 1;    // steps of m loads in flight (two would not fit in 80 VGPRs)

struct ZfArgs {
    const float* m;    // deformed moving image
    const float* ys;   // standardised static image (flat patches flagged in bit 0)
    float* f;          // I'_s
    const int* stop;   // level's stop flag (stopping rule), may be null
    int nx, ny, nz;
    int tiles_x, tiles_y, zchunk, nblocks;
    double inv_n;
};

template <int R>
struct ZfLds {
    static constexpr int W = ZTS + 2 * R;  // region edge
    static constexpr int ZP = W | 1;       // odd pitch (double2) of the z-sum rows
    static constexpr int XP = W | 1;       // odd pitch of the column-major x sums
    static constexpr size_t BYTES = ((size_t)W * ZP + (size_t)ZTS * XP) * sizeof(double2);
};

template <int PZ, int R>
__device__ __forceinline__ void zf_body(const ZfArgs& a, const int bid)
{
    constexpr int ZFT = zf_threads<PZ>();
    constexpr int RZ = PZ / 2;
    using L = ZfLds<R>;
    constexpr int W = L::W, ZP = L::ZP, XP = L::XP;
    constexpr int NC = (W * W + ZFT - 1) / ZFT;  // region columns per thread
    constexpr int XI = W * (ZTS / XRUN);          // x items
    constexpr int YI = ZTS * (ZTS / YRUN);        // y items
    static_assert(XI <= ZFT && YI <= ZFT, "one x and one y item per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    double2* zs = reinterpret_cast<double2*>(smem);
    double2* xs = zs + W * ZP;
    if (a.stop && *a.stop) return;  // the level has met its stopping rule

    const int lb = xcd_logical_block(bid, a.nblocks);
    const int bx = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * ZTS, y0 = by * ZTS;
    const int z0 = bz * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    const int pb = a.nx * a.ny * 4;
    const long vb = (long)pb * a.nz;
    const Rsrc mb = make_rsrc(a.m, vb);

    // this thread's region columns: clamped source offset and LDS slot
    int goff[NC], slot[NC];
    bool cval[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int i = t + q * ZFT;
        const int row = i / W, col = i - row * W;
        cval[q] = i < W * W;
        goff[q] = cval[q] ? (clampi(y0 - R + row, a.ny) * a.nx + clampi(x0 - R + col, a.nx)) * 4 : 0;
        slot[q] = cval[q] ? row * ZP + col : 0;
    }
    // z window of output plane z: m(clamp(z + k)), |k| <= RZ
    double s1[NC], s2[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) s1[q] = s2[q] = 0.0;
#pragma unroll
    for (int k = -RZ; k <= RZ; ++k) {
        const int so = clampi(z0 + k, a.nz) * pb;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double v = (double)ld(mb, goff[q], so);
            s1[q] += v;
            s2[q] = fma(v, v, s2[q]);
        }
    }
    // loads of step j (output plane z0 + j, j >= 1): the plane entering the
    // window and the one leaving it, in slot j % ZPF
    float nw[ZPF][NC], od[ZPF][NC];
    auto request = [&](int j, int sl) {
        const int sn = clampi(z0 + j + RZ, a.nz) * pb, so = clampi(z0 + j - 1 - RZ, a.nz) * pb;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            nw[sl][q] = ld(mb, goff[q], sn);
            od[sl][q] = ld(mb, goff[q], so);
        }
    };
#pragma unroll
    for (int k = 1; k <= ZPF; ++k) request(k, k % ZPF);

    // y items: column c, rows run * YRUN .. + YRUN - 1
    const bool yact = t < YI;
    const int yc = t % ZTS, yrun = t / ZTS;
    const int ox = x0 + yc;
    const Rsrc yb = make_rsrc(a.ys, vb), fb = make_rsrc(a.f, vb);
    int yoff[YRUN];
#pragma unroll
    for (int o = 0; o < YRUN; ++o) yoff[o] = (min(y0 + yrun * YRUN + o, a.ny - 1) * a.nx + min(ox, a.nx - 1)) * 4;
    // x items: region row (fastest across lanes), run of output columns
    const bool xact = t < XI;
    const int xrow = t % W, xrun = t / W;

    const int nout = z1 - z0;
    for (int j0 = 0; j0 < nout; j0 += ZPF) {
#pragma unroll
        for (int jj = 0; jj < ZPF; ++jj) {
            const int j = j0 + jj;
            if (j >= nout) break;
            const int z = z0 + j;
            // the epilogue's Y values of this plane, consumed after both barriers
            float yv[YRUN];
#pragma unroll
            for (int o = 0; o < YRUN; ++o) yv[o] = yact ? ld(yb, yoff[o], z * pb) : 0.0f;
            if (j > 0) {
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    const double vn = (double)nw[jj][q], vo = (double)od[jj][q];
                    s1[q] += vn - vo;
                    s2[q] += fma(vn, vn, -vo * vo);
                }
                request(j + ZPF, jj);
            }
#pragma unroll
            for (int q = 0; q < NC; ++q)
                if (cval[q]) zs[slot[q]] = make_double2(s1[q], s2[q]);
            __syncthreads();
            if (xact) {
                const double2* src = zs + xrow * ZP + xrun * XRUN;
                double u1 = 0.0, u2 = 0.0;
#pragma unroll
                for (int k = 0; k <= 2 * R; ++k) {
                    const double2 v = src[k];
                    u1 += v.x;
                    u2 += v.y;
                }
                double2* dst = xs + (xrun * XRUN) * XP + xrow;
                dst[0] = make_double2(u1, u2);
#pragma unroll
                for (int o = 1; o < XRUN; ++o) {
                    const double2 vi = src[o + 2 * R], vo = src[o - 1];
                    u1 += vi.x - vo.x;
                    u2 += vi.y - vo.y;
                    dst[o * XP] = make_double2(u1, u2);
                }
            }
            __syncthreads();
            if (yact) {
                const double2* src = xs + yc * XP + yrun * YRUN;
                double u1 = 0.0, u2 = 0.0;
#pragma unroll
                for (int k = 0; k <= 2 * R; ++k) {
                    const double2 v = src[k];
                    u1 += v.x;
                    u2 += v.y;
                }
#pragma unroll
                for (int o = 0; o < YRUN; ++o) {
                    if (o > 0) {
                        const double2 vi = src[o + 2 * R], vo = src[o - 1];
                        u1 += vi.x - vo.x;
                        u2 += vi.y - vo.y;
                    }
                    const int oy = y0 + yrun * YRUN + o;
                    if (ox < a.nx && oy < a.ny) {
                        // I'_s = a S + b = E(M) + STD(M) (S - E(S)) / STD(S), combined
                        // in FP64 and rounded once (a flat static patch: E(M) + S - E(S))
                        const double mu = u1 * a.inv_n;
                        double var = u2 * a.inv_n - mu * mu;
                        var = var > 0.0 ? var : 0.0;
                        const double c = (__float_as_uint(yv[o]) & 1u) ? 1.0 : (double)sqrtf((float)var);
                        st(fb, yoff[o], z * pb, (float)fma(c, (double)yv[o], mu));
                    }
                }
            }
        }
    }
}

template <int PZ, int R>
__global__ __launch_bounds__(zf_threads<PZ>(), 6) void k_correct_zf(ZfArgs a)
{
    zf_body<PZ, R>(a, blockIdx.x);
}

template <int PZ, int R>
__global__ __launch_bounds__(zf_threads<PZ>(), 6) void k_correct_zf_batch(Batch<ZfArgs> b)
{
    const int v = batch_volume(b.start, b.n, blockIdx.x);
    zf_body<PZ, R>(b.v[v], blockIdx.x - b.start[v]);
}

// Tiles and z chunks for about `target` workgroups.
void zf_grid(ZfArgs& a, Dims d, int target)
{
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.tiles_x = (d.nx + ZTS - 1) / ZTS;
    a.tiles_y = (d.ny + ZTS - 1) / ZTS;
    const int tiles = a.tiles_x * a.tiles_y;
    int chunks = (target + tiles - 1) / tiles;
    if (chunks > d.nz) chunks = d.nz;
    if (chunks < 1) chunks = 1;
    a.zchunk = (d.nz + chunks - 1) / chunks;
    chunks = (d.nz + a.zchunk - 1) / a.zchunk;
    a.nblocks = tiles * chunks;
}

template <int PZ>
void launch_zf_batch_one(const Batch<ZfArgs>& b, hipStream_t st)
{
    constexpr int R = PZ / 2;
    constexpr size_t lds = ZfLds<R>::BYTES;
    lds_limit((const void*)k_correct_zf_batch<PZ, R>, lds);
    hipLaunchKernelGGL((k_correct_zf_batch<PZ, R>), dim3(b.start[b.n]), dim3(zf_threads<PZ>()), lds, st, b);
}

template <int PZ>
void launch_zf_one(const ZfArgs& a, hipStream_t st)
{
    constexpr int R = PZ / 2;
    constexpr size_t lds = ZfLds<R>::BYTES;
    lds_limit((const void*)k_correct_zf<PZ, R>, lds);
    hipLaunchKernelGGL((k_correct_zf<PZ, R>), dim3(a.nblocks), dim3(zf_threads<PZ>()), lds, st, a);
}

}  // namespace

int correct_zf_resident(const int patch[3])
{
    // workgroups per CU: 160 KB of LDS and six 80-VGPR waves per SIMD (three
    // 8-wave workgroups)
    size_t lds = 0;
    switch (patch[2]) {
        case 1: lds = ZfLds<0>::BYTES; break;
        case 3: lds = ZfLds<1>::BYTES; break;
        case 5: lds = ZfLds<2>::BYTES; break;
        case 7: lds = ZfLds<3>::BYTES; break;
        case 9: lds = ZfLds<4>::BYTES; break;
        case 11: lds = ZfLds<5>::BYTES; break;
        case 13: lds = ZfLds<6>::BYTES; break;
        default: lds = ZfLds<7>::BYTES; break;
    }
    const int by_lds = (int)((160 * 1024) / lds);
    return by_lds < 3 ? by_lds : 3;
}

bool correct_zf_applies(Dims d, const int patch[3])
{
    // (at 15^3: 768 threads, two workgroups per CU by LDS; 224.6 against
    // 232 us for the x -> y -> z sweep at 512^2 x 160, 241 us with 512 threads)
    (void)d;
    return patch[0] == patch[1] && patch[1] == patch[2] && patch[2] <= 15;
}

hipError_t launch_correct_zf(const float* m, const float* ys, float* f, Dims d, const int patch[3], hipStream_t st,
                             const int* stop, int target)
{
    ZfArgs a{};
    a.m = m;
    a.ys = ys;
    a.f = f;
    a.stop = stop;
    a.inv_n = 1.0 / ((double)patch[0] * patch[1] * patch[2]);
    zf_grid(a, d, target);
    switch (patch[2]) {
        case 1: launch_zf_one<1>(a, st); break;
        case 3: launch_zf_one<3>(a, st); break;
        case 5: launch_zf_one<5>(a, st); break;
        case 7: launch_zf_one<7>(a, st); break;
        case 9: launch_zf_one<9>(a, st); break;
        case 11: launch_zf_one<11>(a, st); break;
        case 13: launch_zf_one<13>(a, st); break;
        case 15: launch_zf_one<15>(a, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace disc

namespace disc {

bool correct_zf_batch_applies(const int patch[3])
{
    return patch[0] == patch[1] && patch[1] == patch[2] && patch[2] <= 13;
}

hipError_t launch_correct_zf_batch(const BatchVol* vols, int n, const int patch[3], int target, hipStream_t st)
{
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    Batch<ZfArgs> b{};
    b.n = n;
    b.start[0] = 0;
    for (int v = 0; v < n; ++v) {
        ZfArgs& a = b.v[v];
        a.m = vols[v].m;
        a.ys = vols[v].ys;
        a.f = vols[v].f;
        a.stop = nullptr;
        a.inv_n = 1.0 / ((double)patch[0] * patch[1] * patch[2]);
        zf_grid(a, vols[v].d, target);
        b.start[v + 1] = b.start[v] + a.nblocks;
    }
    switch (patch[2]) {
        case 1: launch_zf_batch_one<1>(b, st); break;
        case 3: launch_zf_batch_one<3>(b, st); break;
        case 5: launch_zf_batch_one<5>(b, st); break;
        case 7: launch_zf_batch_one<7>(b, st); break;
        case 9: launch_zf_batch_one<9>(b, st); break;
        case 11: launch_zf_batch_one<11>(b, st); break;
        case 13: launch_zf_batch_one<13>(b, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace disc
