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
// interpolant of the warp (same floor and clamp conventions: the cell is the
// one the warp samples). b = (B(beta), B(gamma)) at the voxel.
__device__ __forceinline__ void grad_at(const float* __restrict__ ct, const float* __restrict__ r,
                                        const float* __restrict__ m, const float* __restrict__ dres,
                                        const float* __restrict__ scale, float* __restrict__ grad, int x,
                                        int y, int z, int nx, int ny, int nz, double2 b)
{
    const long N = (long)nx * ny * nz;
    const long i = ((long)z * ny + y) * nx + x;
    const float rx = r[i], ry = r[N + i], rz = r[2 * N + i];
    const float tx = rx - floorf(rx), ty = ry - floorf(ry), tz = rz - floorf(rz);
    const int ix = x + floor_to_int(rx), iy = y + floor_to_int(ry), iz = z + floor_to_int(rz);
    const int x0 = clampi(ix, nx), x1 = clampi(ix + 1, nx);
    const int y0 = clampi(iy, ny), y1 = clampi(iy + 1, ny);
    const int z0 = clampi(iz, nz), z1 = clampi(iz + 1, nz);
    const float* p00 = ct + ((long)z0 * ny + y0) * nx;
    const float* p01 = ct + ((long)z0 * ny + y1) * nx;
    const float* p10 = ct + ((long)z1 * ny + y0) * nx;
    const float* p11 = ct + ((long)z1 * ny + y1) * nx;
    // corner values c[z][y][x]
    const float c000 = p00[x0], c001 = p00[x1], c010 = p01[x0], c011 = p01[x1];
    const float c100 = p10[x0], c101 = p10[x1], c110 = p11[x0], c111 = p11[x1];
    const float ux = 1.0f - tx, uy = 1.0f - ty, uz = 1.0f - tz;
    const float gx = uz * (uy * (c001 - c000) + ty * (c011 - c010)) + tz * (uy * (c101 - c100) + ty * (c111 - c110));
    const float gy = uz * (ux * (c010 - c000) + tx * (c011 - c001)) + tz * (ux * (c110 - c100) + tx * (c111 - c101));
    const float gz = uy * (ux * (c100 - c000) + tx * (c101 - c001)) + ty * (ux * (c110 - c010) + tx * (c111 - c011));
    const double G = 2.0 * ((double)dres[i] - fma((double)m[i], b.x, b.y));
    const double s = scale ? (double)scale[0] : 1.0;
    const double sg = s * G;
    grad[i] = (float)(sg * (double)gx);
    grad[N + i] = (float)(sg * (double)gy);
    grad[2 * N + i] = (float)(sg * (double)gz);
}

// The z adjoint fused with the gradient: a thread walks its column through
// a chunk of zchunk planes, keeping the in-range z window sum of the x-y
// adjoint t (see k_box_adjoint) as a running sum; the end planes take the
// clamp's folded offsets by a direct sum. The gradient then follows at each
// voxel without B(beta), B(gamma) going through memory.
__global__ __launch_bounds__(BX* BY) void k_ssd_grad_z(const float* __restrict__ ct,
                                                      const float* __restrict__ r,
                                                      const float* __restrict__ m,
                                                      const float* __restrict__ dres,
                                                      const double2* __restrict__ t,
                                                      const float* __restrict__ scale,
                                                      float* __restrict__ grad, int nx, int ny,
                                                      int nz, int R, int zchunk)
{
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int za = blockIdx.z * zchunk, zb = min(nz, za + zchunk);
    if (x >= nx || y >= ny) return;
    const long plane = (long)nx * ny;
    const double2* col = t + (long)y * nx + x;
    double s1 = 0.0, s2 = 0.0;
    for (int zz = max(0, za - R); zz <= min(nz - 1, za + R); ++zz) {
        const double2 v = col[zz * plane];
        s1 += v.x;
        s2 += v.y;
    }
    for (int z = za; z < zb; ++z) {
        if (z > za) {
            if (z + R <= nz - 1) {
                const double2 v = col[(z + R) * plane];
                s1 += v.x;
                s2 += v.y;
            }
            if (z - 1 - R >= 0) {
                const double2 v = col[(z - 1 - R) * plane];
                s1 -= v.x;
                s2 -= v.y;
            }
        }
        double2 b = make_double2(s1, s2);
        if (z == 0 || z == nz - 1) {
            b = make_double2(0.0, 0.0);
            for (int zz = max(0, z - R); zz <= min(nz - 1, z + R); ++zz) {
                const int c = fold_count(z, zz, nz, R);
                const double2 v = col[zz * plane];
                b.x = fma((double)c, v.x, b.x);
                b.y = fma((double)c, v.y, b.y);
            }
        }
        grad_at(ct, r, m, dres, scale, grad, x, y, z, nx, ny, nz, b);
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
    // about 8 planes per chunk: enough workgroups, short window warm-ups
    const int chunks = std::max(1, (d.nz + 7) / 8);
    const int zchunk = (d.nz + chunks - 1) / chunks;
    const dim3 g((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + zchunk - 1) / zchunk);
    hipLaunchKernelGGL(k_ssd_grad_z, g, dim3(BX, BY), 0, st, ct, r, m, dres, t, scale, grad, d.nx, d.ny, d.nz,
                       R, zchunk);
    return hipGetLastError();
}

hipError_t launch_ssd_finish(const double* partial, int n, double* loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_ssd_finish, dim3(1), dim3(256), 0, st, partial, n, loss);
    return hipGetLastError();
}

}  // namespace disc
