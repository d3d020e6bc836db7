// Gaussian regularisation of the displacement field (Algorithm A1 step 6) as a
// z-sweep kernel for gfx950.
//
// A 512-thread workgroup owns a 64 x 8 column tile of all three components
// and walks a chunk of z. Each plane (tile plus an R-voxel halo, R =
// ceil(3 sigma)) is staged in LDS once; the x pass and the y pass run out of
// LDS; the z pass is a register ring of the last 2R+1 xy-filtered planes, so
// every input plane is read from HBM once per tile and each output is
// written once. Taps are applied in ascending offset order in every pass.
#include "kernels.h"

namespace disc {

namespace {

constexpr int TX = 64;
constexpr int TY = 8;
constexpr int NT = TX * TY;

struct SmoothArgs {
    const float* in;
    float* out;
    int nx, ny, nz;
    int zchunk;
    int tiles_x, tiles_y, nblocks;
    GaussTaps taps;
};

template <int R>
__global__ __launch_bounds__(NT) void k_smooth(SmoothArgs a)
{
    constexpr int K = 2 * R + 1;
    constexpr int W = TX + 2 * R;
    constexpr int H = TY + 2 * R;
    __shared__ float sin_[3][H][W];
    __shared__ float sxp[3][H][TX];

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
    const long N = plane * a.nz;

    float ring[3][K];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) ring[c][k] = 0.0f;

    const int nplanes = (z1 - z0) + 2 * R;
    for (int p0 = 0; p0 < nplanes; p0 += K) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int p = p0 + k;
            if (p >= nplanes) break;
            const long zoff = (long)clampi(z0 - R + p, a.nz) * plane;
            __syncthreads();
            for (int i = t; i < 3 * H * W; i += NT) {
                const int c = i / (H * W);
                const int rem = i - c * (H * W);
                const int row = rem / W, col = rem - row * W;
                const int gx = clampi(x0 - R + col, a.nx), gy = clampi(y0 - R + row, a.ny);
                sin_[c][row][col] = a.in[c * N + zoff + (long)gy * a.nx + gx];
            }
            __syncthreads();
            for (int i = t; i < 3 * H * TX; i += NT) {
                const int c = i / (H * TX);
                const int rem = i - c * (H * TX);
                const int row = rem / TX, col = rem - row * TX;
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j < K; ++j) s = fmaf(a.taps.w[j], sin_[c][row][col + j], s);
                sxp[c][row][col] = s;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j < K; ++j) s = fmaf(a.taps.w[j], sxp[c][ly + j][lx], s);
                ring[c][k] = s;
            }
            if (p >= K - 1) {
                const int oz = z0 + p - 2 * R;
                if (own) {
                    const long idx = (long)oz * plane + (long)oy * a.nx + ox;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float s = 0.0f;
#pragma unroll
                        for (int j = 0; j < K; ++j) s = fmaf(a.taps.w[j], ring[c][(k + 1 + j) % K], s);
                        a.out[c * N + idx] = s;
                    }
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_smooth(const float* rt, float* r, Dims d, const GaussTaps& t, hipStream_t st)
{
    SmoothArgs a;
    a.in = rt;
    a.out = r;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.tiles_x = (d.nx + TX - 1) / TX;
    a.tiles_y = (d.ny + TY - 1) / TY;
    const int tiles = a.tiles_x * a.tiles_y;
    int chunks = (1024 + tiles - 1) / tiles;
    if (chunks > d.nz) chunks = d.nz;
    if (chunks < 1) chunks = 1;
    a.zchunk = (d.nz + chunks - 1) / chunks;
    chunks = (d.nz + a.zchunk - 1) / a.zchunk;
    a.nblocks = tiles * chunks;
    a.taps = t;
    const dim3 g(a.nblocks);
    switch (t.R) {
#define DISC_R(RR) \
    case RR: hipLaunchKernelGGL(k_smooth<RR>, g, dim3(NT), 0, st, a); break;
        DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7) DISC_R(8)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace disc
