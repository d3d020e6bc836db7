// Differentiable DISC for gfx950: the SSD loss L = sum (m - I'_s)^2 between
// the warped CT and the moment-matched static image (Sec. 2.1 model, Eq. 3-6)
// and its gradient with respect to the displacement field.
//
// Backward data flow (patch moments are recomputed, never stored):
//   warp                      m = CT(x + r)
//   moments sweep (SSD mode)  D = m - I'_s, adjoint weights (beta, gamma)
//   2 x box adjoint           x, then y: transpose of the clamped patch sum,
//                             one axis per launch
//   z adjoint + gradient      B(beta), B(gamma) along each column, then
//                             dL/dm = 2 D - 2 (m B(beta) + B(gamma)) times
//                             the derivative of the trilinear interpolant
// The adjoint sums stay in FP64: m B(beta) and B(gamma) cancel to the scale
// of the patch deviation, which in near-flat patches is far below the
// magnitude of either term.
#include <algorithm>

#include "kernels.h"

namespace disc {

namespace {

constexpr int BX = 64;  // one wave along x
constexpr int BY = 4;

inline dim3 grid_for(Dims d)
{
    return dim3((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
}

// Transpose of the clamped 1-D window sum out(x) = sum_{|k| <= R} in(clamp(x + k))
// along one axis: out(j) = sum_x count(x, j) in(x), count(x, j) = #{k : clamp(x + k) = j}.
// Interior j: every x within R counts once. The end voxels also collect the
// offsets that the clamp folds onto them: count(x, 0) = R - x + 1 for x <= R,
// and the mirror image at the far end (2R + 1 on an axis of one voxel).
__device__ inline int fold_count(int j, int xx, int len, int R)
{
    if (len == 1) return 2 * R + 1;
    if (j == 0) return R - xx + 1;
    if (j == len - 1) return R - (len - 1 - xx) + 1;
    return 1;
}

constexpr int kMaxAdjR = 15;  // patch extents up to 31

// Along x: the workgroup stages its four rows plus the R-voxel halo in LDS,
// then each thread sums its output's window there.
__global__ __launch_bounds__(BX* BY) void k_box_adjoint_x(const double2* __restrict__ in,
                                                         double2* __restrict__ out, int nx, int ny, int R)
{
    __shared__ double2 tile[BY][BX + 2 * kMaxAdjR];
    const int x0 = blockIdx.x * BX;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    const int yc = min(y, ny - 1);
    const double2* row = in + ((long)z * ny + yc) * nx;
    for (int i = threadIdx.x; i < BX + 2 * R; i += BX) {
        const int xx = x0 - R + i;
        tile[threadIdx.y][i] = (xx >= 0 && xx < nx) ? row[xx] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int x = x0 + threadIdx.x;
    if (x >= nx || y >= ny) return;
    const int lo = max(0, x - R), hi = min(nx - 1, x + R);
    const bool edge = x == 0 || x == nx - 1;
    double s1 = 0.0, s2 = 0.0;
    for (int xx = lo; xx <= hi; ++xx) {
        const double2 v = tile[threadIdx.y][xx - x0 + R];
        if (edge) {
            const double c = (double)fold_count(x, xx, nx, R);
            s1 = fma(c, v.x, s1);
            s2 = fma(c, v.y, s2);
        } else {
            s1 += v.x;
            s2 += v.y;
        }
    }
    out[((long)z * ny + y) * nx + x] = make_double2(s1, s2);
}

// Along y: a thread takes a run of YC outputs of its (x, z) column. It
// requests every row its windows touch at once (rows outside the volume
// read as zero, which truncates the window exactly as the clamp-free
// interior count requires), then slides the window sum down the run; the
// two end rows of the volume take the folded counts.
constexpr int YC = 16;

template <int R>
__global__ __launch_bounds__(BX* BY) void k_box_adjoint_y(const double2* __restrict__ in,
                                                         double2* __restrict__ out, int nx, int ny)
{
    constexpr int NV = YC + 2 * R;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int ya = (blockIdx.y * BY + threadIdx.y) * YC;
    const int z = blockIdx.z;
    if (x >= nx || ya >= ny) return;
    const double2* col = in + (long)z * ny * nx + x;
    double2* oc = out + (long)z * ny * nx + x;
    double2 v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int yy = ya - R + k;
        v[k] = (yy >= 0 && yy < ny) ? col[(long)yy * nx] : make_double2(0.0, 0.0);
    }
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        s1 += v[k].x;
        s2 += v[k].y;
    }
#pragma unroll
    for (int j = 0; j < YC; ++j) {
        const int y = ya + j;
        if (y >= ny) break;
        if (j > 0) {
            s1 += v[j + 2 * R].x - v[j - 1].x;
            s2 += v[j + 2 * R].y - v[j - 1].y;
        }
        double2 o = make_double2(s1, s2);
        if (y == 0 || y == ny - 1) {
            o = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k) {
                const int yy = y - R + k;
                if (yy < 0 || yy > ny - 1) continue;
                const double c = (double)fold_count(y, yy, ny, R);
                o.x = fma(c, v[j + k].x, o.x);
                o.y = fma(c, v[j + k].y, o.y);
            }
        }
        oc[(long)y * nx] = o;
    }
}

// dL/dr at voxel (x, y, z) = dL/dm * d m / d position, with
// dL/dm = 2 D - 2 (m B(beta) + B(gamma)) and the derivative of the trilinear
// interpolant of the warp in the cell the warp samples (the same clamped
// cell as warp_at: lowest corner clamped to [0, n - 2], weight to [0, 1]).
// Along an axis where the sample lies outside [0, n - 1] both corners of the
// clamped interpolant are the same voxel, so that component is 0. b =
// (B(beta), B(gamma)) at the voxel; vo / so: per-lane and scalar byte offsets
// of the voxel.
__device__ __forceinline__ void grad_at(const WarpSrc& w, Rsrc rb0, Rsrc rb1, Rsrc rb2, Rsrc mb, Rsrc db, Rsrc gb0,
                                        Rsrc gb1, Rsrc gb2, double sc, int x, int y, int z, int vo, int so,
                                        double2 b)
{
    const float rx = ld(rb0, vo, so), ry = ld(rb1, vo, so), rz = ld(rb2, vo, so);
    const float fx = floorf(rx), fy = floorf(ry), fz = floorf(rz);
    const int ix = x + floor_to_int(rx), iy = y + floor_to_int(ry), iz = z + floor_to_int(rz);
    const int xa = min(max(ix, 0), w.xm), ya = min(max(iy, 0), w.ym), za = min(max(iz, 0), w.zm);
    const float tx = fminf(fmaxf((float)(ix - xa) + (rx - fx), 0.0f), 1.0f);
    const float ty = fminf(fmaxf((float)(iy - ya) + (ry - fy), 0.0f), 1.0f);
    const float tz = fminf(fmaxf((float)(iz - za) + (rz - fz), 0.0f), 1.0f);
    const bool inx = ix >= 0 && ix <= w.nx - 2, iny = iy >= 0 && iy <= w.ny - 2, inz = iz >= 0 && iz <= w.nz - 2;
    const int v = ((za * w.ny + ya) * w.nx + xa) * 4;
    float c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = ld(w.ct, v, w.so[k]);
    // corner k: bit 0 +x, bit 1 +y, bit 2 +z
    const float ux = 1.0f - tx, uy = 1.0f - ty, uz = 1.0f - tz;
    const float gx = inx ? uz * (uy * (c[1] - c[0]) + ty * (c[3] - c[2])) + tz * (uy * (c[5] - c[4]) + ty * (c[7] - c[6]))
                         : 0.0f;
    const float gy = iny ? uz * (ux * (c[2] - c[0]) + tx * (c[3] - c[1])) + tz * (ux * (c[6] - c[4]) + tx * (c[7] - c[5]))
                         : 0.0f;
    const float gz = inz ? uy * (ux * (c[4] - c[0]) + tx * (c[5] - c[1])) + ty * (ux * (c[6] - c[2]) + tx * (c[7] - c[3]))
                         : 0.0f;
    const double G = 2.0 * ((double)ld(db, vo, so) - fma((double)ld(mb, vo, so), b.x, b.y));
    const double sg = sc * G;
    st(gb0, vo, so, (float)(sg * (double)gx));
    st(gb1, vo, so, (float)(sg * (double)gy));
    st(gb2, vo, so, (float)(sg * (double)gz));
}

// The z adjoint fused with the gradient: a thread takes a run of ZC planes of
// its column, requests every plane of the x-y adjoint t their windows touch
// at once (planes outside the volume read as zero), slides the z window sum
// down the run (the end planes take the clamp's folded counts), and forms the
// gradient at each voxel; B(beta), B(gamma) never go through memory.
constexpr int ZC = 16;

template <int R>
__global__ __launch_bounds__(BX* BY) void k_ssd_grad_z(const float* __restrict__ ct,
                                                      const float* __restrict__ r,
                                                      const float* __restrict__ m,
                                                      const float* __restrict__ dres,
                                                      const double2* __restrict__ t,
                                                      const float* __restrict__ scale,
                                                      float* __restrict__ grad, int nx, int ny, int nz)
{
    constexpr int NV = ZC + 2 * R;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int za = blockIdx.z * ZC;
    if (x >= nx || y >= ny) return;
    const long plane = (long)nx * ny;
    const long N = plane * nz, cb = N * 4;
    const double2* col = t + (long)y * nx + x;
    double2 v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int zz = za - R + k;
        v[k] = (zz >= 0 && zz < nz) ? col[zz * plane] : make_double2(0.0, 0.0);
    }
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        s1 += v[k].x;
        s2 += v[k].y;
    }
    const WarpSrc w = warp_src(ct, nx, ny, nz);
    const Rsrc rb0 = make_rsrc(r, cb), rb1 = make_rsrc(r + N, cb), rb2 = make_rsrc(r + 2 * N, cb);
    const Rsrc gb0 = make_rsrc(grad, cb), gb1 = make_rsrc(grad + N, cb), gb2 = make_rsrc(grad + 2 * N, cb);
    const Rsrc mb = make_rsrc(m, cb), db = make_rsrc(dres, cb);
    const double sc = scale ? (double)scale[0] : 1.0;
    const int vo = (y * nx + x) * 4, pb = (int)plane * 4;
#pragma unroll
    for (int j = 0; j < ZC; ++j) {
        const int z = za + j;
        if (z >= nz) break;
        if (j > 0) {
            s1 += v[j + 2 * R].x - v[j - 1].x;
            s2 += v[j + 2 * R].y - v[j - 1].y;
        }
        double2 bz = make_double2(s1, s2);
        if (z == 0 || z == nz - 1) {
            bz = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k) {
                const int zz = z - R + k;
                if (zz < 0 || zz > nz - 1) continue;
                const double c = (double)fold_count(z, zz, nz, R);
                bz.x = fma(c, v[j + k].x, bz.x);
                bz.y = fma(c, v[j + k].y, bz.y);
            }
        }
        grad_at(w, rb0, rb1, rb2, mb, db, gb0, gb1, gb2, sc, x, y, z, vo, z * pb, bz);
    }
}

// Loss = sum of the per-workgroup partial sums, in a fixed order.
__global__ __launch_bounds__(256) void k_ssd_finish(const double* __restrict__ partial, int n,
                                                   double* __restrict__ loss)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int i = t; i < n; i += 256) s += partial[i];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) loss[0] = red[0];
}

}  // namespace

hipError_t launch_box_adjoint(const double2* in, double2* out, Dims d, int axis, int R, hipStream_t st)
{
    if (R < 0 || R > kMaxAdjR) return hipErrorInvalidValue;
    const dim3 b(BX, BY);
    if (axis == 0) {
        hipLaunchKernelGGL(k_box_adjoint_x, grid_for(d), b, 0, st, in, out, d.nx, d.ny, R);
    } else if (axis == 1) {
        const int runs = (d.ny + YC - 1) / YC;
        const dim3 g((d.nx + BX - 1) / BX, (runs + BY - 1) / BY, d.nz);
        switch (R) {
#define DISC_R(RR) \
    case RR: hipLaunchKernelGGL(k_box_adjoint_y<RR>, g, b, 0, st, in, out, d.nx, d.ny); break;
            DISC_R(0) DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7)
            DISC_R(8) DISC_R(9) DISC_R(10) DISC_R(11) DISC_R(12) DISC_R(13) DISC_R(14) DISC_R(15)
#undef DISC_R
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;  // the z adjoint runs inside k_ssd_grad_z
    }
    return hipGetLastError();
}

hipError_t launch_ssd_grad_z(const float* ct, const float* r, const float* m, const float* dres,
                             const double2* t, const float* scale, float* grad, Dims d, int R, hipStream_t st)
{
    const dim3 g((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + ZC - 1) / ZC);
    switch (R) {
#define DISC_R(RR)                                                                                          \
    case RR:                                                                                                \
        hipLaunchKernelGGL(k_ssd_grad_z<RR>, g, dim3(BX, BY), 0, st, ct, r, m, dres, t, scale, grad, d.nx, d.ny, \
                           d.nz);                                                                           \
        break;
        DISC_R(0) DISC_R(1) DISC_R(2) DISC_R(3) DISC_R(4) DISC_R(5) DISC_R(6) DISC_R(7)
#undef DISC_R
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ssd_finish(const double* partial, int n, double* loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_ssd_finish, dim3(1), dim3(256), 0, st, partial, n, loss);
    return hipGetLastError();
}

}  // namespace disc
