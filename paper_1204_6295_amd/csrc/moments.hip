// Patch moments (Eq. 3) and the moment-matching correction (Eq. 5-6,
// I'_s = a I_s + b) as one z-sweep kernel for gfx950.
//
// A 512-thread workgroup owns a 64 x 8 column tile and walks a chunk of z.
// For each plane it stages the tile plus the in-plane patch halo in LDS,
// forms x-window sums, then y-window sums per owned column; the z-window is
// a ring of the last pz plane sums held in registers (pz is a template
// parameter), so each plane is read from HBM once per tile. Sums of m and
// m^2 are FP64: E(M^2) - E(M)^2 of 1500-HU data cancels far below FP32
// resolution, and FP64 runs at the FP32 rate on this chip. Every window sum
// is formed in plane/row/column order, so results do not depend on the tile
// or chunk decomposition.
#include <cmath>

#include "kernels.h"

namespace disc {

namespace {

constexpr int TX = 64;
constexpr int TY = 8;
constexpr int NT = TX * TY;

struct MomArgs {
    const float* img;    // image whose patch moments are taken (m, or s at set-up)
    const float* ys_in;  // standardised static image (correction pass)
    float* out;          // ys (set-up) or f = I'_s (correction)
    int nx, ny, nz;
    int rx, ry;
    int zchunk;
    int tiles_x, tiles_y, nblocks;
    float tau;
    double inv_n;
};

inline size_t lds_bytes(int rx, int ry)
{
    const size_t W = TX + 2 * rx, H = TY + 2 * ry;
    return ((H * W * sizeof(float) + 15) & ~(size_t)15) + H * TX * sizeof(double2);
}

template <int PZ, bool STATIC>
__global__ __launch_bounds__(NT) void k_moments(MomArgs a)
{
    constexpr int RZ = PZ / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = TX + 2 * a.rx, H = TY + 2 * a.ry;
    float* sm = reinterpret_cast<float*>(smem);
    double2* sx = reinterpret_cast<double2*>(smem + (((size_t)H * W * sizeof(float) + 15) & ~(size_t)15));

    const int lb = xcd_logical_block(blockIdx.x, a.nblocks);
    const int bx = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.zchunk;
    const int z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x, lx = t % TX, ly = t / TX;
    const int ox = x0 + lx, oy = y0 + ly;
    const bool own = ox < a.nx && oy < a.ny;
    const long plane = (long)a.nx * a.ny;

    double s1r[PZ], s2r[PZ];
#pragma unroll
    for (int k = 0; k < PZ; ++k) s1r[k] = s2r[k] = 0.0;

    const int nplanes = (z1 - z0) + 2 * RZ;
    for (int p0 = 0; p0 < nplanes; p0 += PZ) {
#pragma unroll
        for (int k = 0; k < PZ; ++k) {
            const int p = p0 + k;
            if (p >= nplanes) break;
            const float* src = a.img + (long)clampi(z0 - RZ + p, a.nz) * plane;
            __syncthreads();
            for (int i = t; i < H * W; i += NT) {
                const int row = i / W, col = i - row * W;
                const int gx = clampi(x0 - a.rx + col, a.nx), gy = clampi(y0 - a.ry + row, a.ny);
                sm[i] = src[(long)gy * a.nx + gx];
            }
            __syncthreads();
            for (int i = t; i < H * TX; i += NT) {
                const int row = i / TX, col = i - row * TX;
                const float* q = sm + row * W + col;
                double u1 = 0.0, u2 = 0.0;
                for (int j = 0; j <= 2 * a.rx; ++j) {
                    const double v = (double)q[j];
                    u1 += v;
                    u2 = fma(v, v, u2);
                }
                sx[i] = make_double2(u1, u2);
            }
            __syncthreads();
            double p1 = 0.0, p2 = 0.0;
            for (int j = 0; j <= 2 * a.ry; ++j) {
                const double2 q = sx[(ly + j) * TX + lx];
                p1 += q.x;
                p2 += q.y;
            }
            s1r[k] = p1;
            s2r[k] = p2;
            if (p >= PZ - 1) {
                // planes p-PZ+1 .. p are in slots (k+1) % PZ .. k, oldest first
                double z1s = 0.0, z2s = 0.0;
#pragma unroll
                for (int j = 0; j < PZ; ++j) {
                    z1s += s1r[(k + 1 + j) % PZ];
                    z2s += s2r[(k + 1 + j) % PZ];
                }
                const int oz = z0 + p - 2 * RZ;
                if (own) {
                    const double mu = z1s * a.inv_n;
                    double var = z2s * a.inv_n - mu * mu;
                    var = var > 0.0 ? var : 0.0;
                    const long idx = (long)oz * plane + (long)oy * a.nx + ox;
                    if (STATIC) {
                        // Eq. 5 denominator: STD(S). A flat static patch keeps
                        // only the mean match and is flagged in the low bit.
                        const double sv = (double)a.img[idx];
                        const bool flat = !(var > (double)a.tau);
                        const double yv = flat ? (sv - mu) : (sv - mu) / sqrt(var);
                        unsigned b = __float_as_uint((float)yv);
                        b = flat ? (b | 1u) : (b & ~1u);
                        a.out[idx] = __uint_as_float(b);
                    } else {
                        // I'_s = a S + b = E(M) + STD(M) (S - E(S)) / STD(S), formed in
                        // FP64 and rounded once: identical images then give
                        // |I'_s - m| well below eps_d.
                        const float yv = a.ys_in[idx];
                        const double c = (__float_as_uint(yv) & 1u) ? 1.0 : sqrt(var);
                        a.out[idx] = (float)fma(c, (double)yv, mu);
                    }
                }
            }
        }
    }
}

template <bool STATIC>
hipError_t launch_pz(int pz, dim3 g, size_t lds, hipStream_t st, const MomArgs& a)
{
    switch (pz) {
#define DISC_PZ(P) \
    case P: hipLaunchKernelGGL((k_moments<P, STATIC>), g, dim3(NT), lds, st, a); break;
        DISC_PZ(1) DISC_PZ(3) DISC_PZ(5) DISC_PZ(7) DISC_PZ(9) DISC_PZ(11) DISC_PZ(13) DISC_PZ(15)
#undef DISC_PZ
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool STATIC>
hipError_t launch_moments(const float* img, const float* ys_in, float* out, Dims d,
                          const int patch[3], float tau, hipStream_t st)
{
    MomArgs a;
    a.img = img;
    a.ys_in = ys_in;
    a.out = out;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.rx = patch[0] / 2;
    a.ry = patch[1] / 2;
    a.tiles_x = (d.nx + TX - 1) / TX;
    a.tiles_y = (d.ny + TY - 1) / TY;
    // split z so that the launch has at least ~4 workgroups per CU
    const int tiles = a.tiles_x * a.tiles_y;
    int chunks = (1024 + tiles - 1) / tiles;
    if (chunks > d.nz) chunks = d.nz;
    if (chunks < 1) chunks = 1;
    a.zchunk = (d.nz + chunks - 1) / chunks;
    chunks = (d.nz + a.zchunk - 1) / a.zchunk;
    a.nblocks = tiles * chunks;
    a.tau = tau;
    a.inv_n = 1.0 / ((double)patch[0] * patch[1] * patch[2]);
    return launch_pz<STATIC>(patch[2], dim3(a.nblocks), lds_bytes(a.rx, a.ry), st, a);
}

}  // namespace

hipError_t launch_static_stats(const float* s, float* ys, Dims d, const int patch[3], float tau,
                               hipStream_t st)
{
    return launch_moments<true>(s, nullptr, ys, d, patch, tau, st);
}

hipError_t launch_correct(const float* m, const float* ys, float* f, Dims d, const int patch[3],
                          hipStream_t st)
{
    return launch_moments<false>(m, ys, f, d, patch, 0.0f, st);
}

}  // namespace disc
