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
// offsets that the clamp folds onto them.
template <int AXIS>
__global__ __launch_bounds__(BX* BY) void k_box_adjoint(const double2* __restrict__ in,
                                                       double2* __restrict__ out, int nx, int ny,
                                                       int nz, int R)
{
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const long i = ((long)z * ny + y) * nx + x;
    const int j = AXIS == 0 ? x : (AXIS == 1 ? y : z);
    const int len = AXIS == 0 ? nx : (AXIS == 1 ? ny : nz);
    const long st = AXIS == 0 ? 1L : (AXIS == 1 ? (long)nx : (long)nx * ny);
    const double2* line = in + (i - (long)j * st);
    const int lo = max(0, j - R), hi = min(len - 1, j + R);
    double s1 = 0.0, s2 = 0.0;
    for (int xx = lo; xx <= hi; ++xx) {
        int c = 1;
        if (len == 1)
            c = 2 * R + 1;
        else if (j == 0)
            c = R - xx + 1;  // offsets k <= -xx
        else if (j == len - 1)
            c = R - (len - 1 - xx) + 1;  // offsets k >= len - 1 - xx
        const double2 v = line[(long)xx * st];
        s1 = fma((double)c, v.x, s1);
        s2 = fma((double)c, v.y, s2);
    }
    out[i] = make_double2(s1, s2);
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
                const int c = nz == 1 ? 2 * R + 1 : (z == 0 ? R - zz + 1 : R - (nz - 1 - zz) + 1);
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
    const dim3 g = grid_for(d), b(BX, BY);
    if (axis == 0)
        hipLaunchKernelGGL(k_box_adjoint<0>, g, b, 0, st, in, out, d.nx, d.ny, d.nz, R);
    else if (axis == 1)
        hipLaunchKernelGGL(k_box_adjoint<1>, g, b, 0, st, in, out, d.nx, d.ny, d.nz, R);
    else
        hipLaunchKernelGGL(k_box_adjoint<2>, g, b, 0, st, in, out, d.nx, d.ny, d.nz, R);
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
