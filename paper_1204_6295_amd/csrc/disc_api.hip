// C ABI of libdisc: argument validation, workspace layout, the Algorithm A1
// level schedule and per-kernel event timing. Kernels live in the other
// translation units; this file only decides what to launch.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "disc.h"
#include "kernels.h"

using disc::Dims;

namespace {

thread_local std::string g_thread_err;

enum KernelId { K_WARP = 0, K_CORRECT = 1, K_FORCE_XY = 2, K_SMOOTH_Z = 3, K_UPSAMPLE = 4, K_COUNT = 5 };

struct TimingRec {
    int kid;
    int level;
    double voxels;
};

}  // namespace

struct disc_ctx {
    disc_params p;
    disc::GaussTaps taps;
    int L = 0;
    Dims dims[DISC_MAX_LEVELS];
    const float* ct[DISC_MAX_LEVELS] = {};
    float* s[DISC_MAX_LEVELS] = {};
    float* ys[DISC_MAX_LEVELS] = {};
    float* r[2] = {};
    float* m = nullptr;
    float* f = nullptr;
    void* scratch = nullptr;
    int cur = 0;
    int level = 0;
    int it = 0;
    bool ready = false;
    bool f_valid = false;
    std::string err;
    // event timing
    int max_rec = 0;
    std::vector<hipEvent_t> ev;
    std::vector<TimingRec> rec;
};

namespace {

int fail(disc_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

int fail(disc_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_thread_err = buf;
    return code;
}

int hip_fail(disc_ctx* c, hipError_t e, const char* what)
{
    return fail(c, DISC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_patch(const int patch[3])
{
    for (int d = 0; d < 3; ++d)
        if (patch[d] < 1 || patch[d] % 2 == 0) return false;
    return patch[0] <= 2 * disc::kMaxPatchRxy + 1 && patch[1] <= 2 * disc::kMaxPatchRxy + 1 &&
           patch[2] <= disc::kMaxPatchZ;
}

bool valid_dims(int nx, int ny, int nz)
{
    if (nx < 1 || ny < 1 || nz < 1 || nz > 65535) return false;
    return (long)nx * ny * nz < (1L << 31);
}

int check_params(disc_ctx* c, const disc_params* p)
{
    if (!p) return fail(c, DISC_EINVAL, "params is NULL");
    if (!valid_patch(p->patch))
        return fail(c, DISC_EINVAL, "patch (%d,%d,%d): extents must be odd, px,py <= 31, pz <= 15",
                    p->patch[0], p->patch[1], p->patch[2]);
    disc::GaussTaps t;
    if (!disc::make_gauss_taps(p->sigma, &t))
        return fail(c, DISC_EINVAL, "sigma %g outside (0, %g]", (double)p->sigma,
                    disc::kMaxGaussR / 3.0);
    if (p->levels < 1 || p->levels > DISC_MAX_LEVELS)
        return fail(c, DISC_EINVAL, "levels %d outside 1..%d", p->levels, DISC_MAX_LEVELS);
    for (int l = 0; l < p->levels; ++l)
        if (p->iters[l] < 0) return fail(c, DISC_EINVAL, "iters[%d] is negative", l);
    if (p->global_shift != 0 && p->global_shift != 1)
        return fail(c, DISC_EINVAL, "global_shift must be 0 or 1");
    if (!(p->var_floor >= 0.0f) || !std::isfinite(p->var_floor))
        return fail(c, DISC_EINVAL, "var_floor must be finite and >= 0");
    if (!(p->diff_floor >= 0.0f) || !std::isfinite(p->diff_floor))
        return fail(c, DISC_EINVAL, "diff_floor must be finite and >= 0");
    return DISC_OK;
}

void level_dims(int L, int nx, int ny, int nz, Dims* dims)
{
    dims[L - 1] = Dims{nx, ny, nz};
    for (int l = L - 2; l >= 0; --l)
        dims[l] = Dims{(dims[l + 1].nx + 1) / 2, (dims[l + 1].ny + 1) / 2, (dims[l + 1].nz + 1) / 2};
}

// Workspace carve-up, shared by disc_workspace_bytes and disc_set_volumes.
struct Carver {
    char* base;
    size_t off = 0;
    void* take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

size_t carve(disc_ctx* c, char* base, int L, const Dims* dims)
{
    Carver cv{base};
    const size_t nf = (size_t)dims[L - 1].n();
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)dims[l].n();
        float* s = (float*)cv.take(n * 4);
        float* ys = (float*)cv.take(n * 4);
        float* ctw = l < L - 1 ? (float*)cv.take(n * 4) : nullptr;
        if (c) {
            c->s[l] = s;
            c->ys[l] = ys;
            if (l < L - 1) c->ct[l] = ctw;
        }
    }
    float* r0 = (float*)cv.take(3 * nf * 4);
    float* r1 = (float*)cv.take(3 * nf * 4);
    float* m = (float*)cv.take(nf * 4);
    float* f = (float*)cv.take(nf * 4);
    void* sc = cv.take(disc::shift_scratch_bytes());
    if (c) {
        c->r[0] = r0;
        c->r[1] = r1;
        c->m = m;
        c->f = f;
        c->scratch = sc;
    }
    return (cv.off + 255) & ~(size_t)255;
}

// Event bracketing of one launch (no-op unless timing is enabled).
struct Timed {
    disc_ctx* c;
    hipStream_t st;
    int slot = -1;
    Timed(disc_ctx* cc, hipStream_t s, int kid, int level, double vox) : c(cc), st(s)
    {
        if (c->max_rec > 0 && (int)c->rec.size() < c->max_rec) {
            slot = (int)c->rec.size();
            c->rec.push_back(TimingRec{kid, level, vox});
            (void)hipEventRecord(c->ev[2 * slot], st);
        }
    }
    ~Timed()
    {
        if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], st);
    }
};

int one_iteration(disc_ctx* c, hipStream_t st)
{
    hipError_t e;
    if (c->it >= c->p.iters[c->level] && c->level < c->L - 1) {
        const Dims dc = c->dims[c->level], df = c->dims[c->level + 1];
        {
            Timed tm(c, st, K_UPSAMPLE, c->level + 1, (double)df.n());
            e = disc::launch_upsample_field(c->r[c->cur], dc, c->r[1 - c->cur], df, st);
        }
        if (e != hipSuccess) return hip_fail(c, e, "upsample_field");
        c->cur ^= 1;
        c->level += 1;
        c->it = 0;
        c->f_valid = false;
    }
    const int l = c->level;
    const Dims d = c->dims[l];
    const double vox = (double)d.n();
    float* r = c->r[c->cur];
    float* q = c->r[1 - c->cur];
    {
        Timed tm(c, st, K_WARP, l, vox);
        e = disc::launch_warp(c->ct[l], r, c->m, d, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "warp");
    {
        Timed tm(c, st, K_CORRECT, l, vox);
        e = disc::launch_correct(c->m, c->ys[l], c->f, d, c->p.patch, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "correct");
    {
        Timed tm(c, st, K_FORCE_XY, l, vox);
        e = disc::launch_force_xy(c->m, c->f, r, q, nullptr, d, c->p.diff_floor, c->taps, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "force + xy smoothing");
    {
        Timed tm(c, st, K_SMOOTH_Z, l, vox);
        e = disc::launch_smooth_z(q, r, d, c->taps, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "z smoothing");
    c->it += 1;
    c->f_valid = true;
    return DISC_OK;
}

int remaining(const disc_ctx* c)
{
    int left = c->p.iters[c->level] - c->it;
    if (left < 0) left = 0;
    for (int l = c->level + 1; l < c->L; ++l) left += c->p.iters[l];
    return left;
}

}  // namespace

extern "C" {

int disc_params_default(disc_params* p)
{
    if (!p) return fail(nullptr, DISC_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->patch[0] = p->patch[1] = p->patch[2] = 11;
    p->sigma = 2.0f;
    p->levels = 3;
    p->iters[0] = p->iters[1] = p->iters[2] = 100;
    p->global_shift = 1;
    p->var_floor = 1e-2f;
    p->diff_floor = 1e-3f;
    return DISC_OK;
}

int disc_create(const disc_params* p, disc_ctx** out)
{
    if (!out) return fail(nullptr, DISC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(nullptr, p);
    if (rc != DISC_OK) return rc;
    disc_ctx* c = new disc_ctx();
    c->p = *p;
    disc::make_gauss_taps(p->sigma, &c->taps);
    c->L = p->levels;
    *out = c;
    return DISC_OK;
}

void disc_destroy(disc_ctx* c)
{
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

const char* disc_last_error(const disc_ctx* c)
{
    return c ? c->err.c_str() : g_thread_err.c_str();
}

size_t disc_workspace_bytes(const disc_params* p, int nx, int ny, int nz)
{
    if (check_params(nullptr, p) != DISC_OK || !valid_dims(nx, ny, nz)) return 0;
    Dims dims[DISC_MAX_LEVELS];
    level_dims(p->levels, nx, ny, nz, dims);
    return carve(nullptr, nullptr, p->levels, dims);
}

int disc_set_volumes(disc_ctx* c, const float* ct_dev, const float* cbct_dev, int nx, int ny,
                     int nz, void* workspace_dev, size_t workspace_bytes, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!ct_dev || !cbct_dev || !workspace_dev)
        return fail(c, DISC_EINVAL, "ct, cbct and workspace must be device pointers");
    if (!valid_dims(nx, ny, nz))
        return fail(c, DISC_EINVAL, "dims (%d,%d,%d): need >= 1, nz <= 65535, N < 2^31", nx, ny, nz);
    if (((uintptr_t)workspace_dev & 255) != 0)
        return fail(c, DISC_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = disc_workspace_bytes(&c->p, nx, ny, nz);
    if (workspace_bytes < need)
        return fail(c, DISC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    c->ready = false;
    level_dims(c->L, nx, ny, nz, c->dims);
    carve(c, (char*)workspace_dev, c->L, c->dims);
    const int L = c->L;
    const Dims fin = c->dims[L - 1];
    c->ct[L - 1] = ct_dev;
    hipError_t e;
    if (c->p.global_shift) {
        e = disc::launch_shift(ct_dev, cbct_dev, fin.n(), c->s[L - 1], nullptr, c->scratch, st);
        if (e != hipSuccess) return hip_fail(c, e, "global shift");
    } else {
        e = hipMemcpyAsync(c->s[L - 1], cbct_dev, (size_t)fin.n() * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(c, e, "copy cbct");
    }
    for (int l = L - 2; l >= 0; --l) {
        e = disc::launch_downsample(c->ct[l + 1], (float*)c->ct[l], c->dims[l + 1], st);
        if (e != hipSuccess) return hip_fail(c, e, "downsample ct");
        e = disc::launch_downsample(c->s[l + 1], c->s[l], c->dims[l + 1], st);
        if (e != hipSuccess) return hip_fail(c, e, "downsample cbct");
    }
    for (int l = 0; l < L; ++l) {
        e = disc::launch_static_stats(c->s[l], c->ys[l], c->dims[l], c->p.patch, c->p.var_floor, st);
        if (e != hipSuccess) return hip_fail(c, e, "static patch moments");
    }
    e = disc::launch_fill(c->r[0], 3 * c->dims[0].n(), 0.0f, st);
    if (e != hipSuccess) return hip_fail(c, e, "zero field");
    c->cur = 0;
    c->level = 0;
    c->it = 0;
    c->f_valid = false;
    c->ready = true;
    return DISC_OK;
}

int disc_iterate(disc_ctx* c, int n, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (n < 0) return fail(c, DISC_EINVAL, "n is negative");
    for (int k = 0; k < n; ++k) {
        int rc = one_iteration(c, (hipStream_t)stream);
        if (rc != DISC_OK) return rc;
    }
    return DISC_OK;
}

int disc_run(disc_ctx* c, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    return disc_iterate(c, remaining(c), stream);
}

int disc_state(const disc_ctx* c, int* level, int* iter_in_level, int dims[3])
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(const_cast<disc_ctx*>(c), DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (level) *level = c->level;
    if (iter_in_level) *iter_in_level = c->it;
    if (dims) {
        dims[0] = c->dims[c->level].nx;
        dims[1] = c->dims[c->level].ny;
        dims[2] = c->dims[c->level].nz;
    }
    return DISC_OK;
}

int disc_get_field(disc_ctx* c, float* out_dev, int dims_out[3], void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (!out_dev) return fail(c, DISC_EINVAL, "out is NULL");
    const Dims d = c->dims[c->level];
    hipError_t e = hipMemcpyAsync(out_dev, c->r[c->cur], (size_t)d.n() * 12, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy field");
    if (dims_out) {
        dims_out[0] = d.nx;
        dims_out[1] = d.ny;
        dims_out[2] = d.nz;
    }
    return DISC_OK;
}

int disc_set_field(disc_ctx* c, const float* r_dev, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (!r_dev) return fail(c, DISC_EINVAL, "field is NULL");
    const Dims d = c->dims[c->level];
    hipError_t e = hipMemcpyAsync(c->r[c->cur], r_dev, (size_t)d.n() * 12, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy field");
    return DISC_OK;
}

int disc_get_corrected(disc_ctx* c, float* out_dev, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (!out_dev) return fail(c, DISC_EINVAL, "out is NULL");
    if (!c->f_valid) return fail(c, DISC_ESTATE, "no iteration has run at the current level");
    const Dims d = c->dims[c->level];
    hipError_t e = hipMemcpyAsync(out_dev, c->f, (size_t)d.n() * 4, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy corrected image");
    return DISC_OK;
}

// ---- single steps -----------------------------------------------------------

#define DISC_CHECK_DIMS(nx, ny, nz)                                                        \
    if (!valid_dims(nx, ny, nz))                                                           \
        return fail(nullptr, DISC_EINVAL, "dims (%d,%d,%d): need >= 1, nz <= 65535, N < 2^31", \
                    nx, ny, nz)

int disc_step_warp(const float* ct_dev, const float* r_dev, int nx, int ny, int nz, float* m_dev,
                   void* stream)
{
    if (!ct_dev || !r_dev || !m_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    hipError_t e = disc::launch_warp(ct_dev, r_dev, m_dev, Dims{nx, ny, nz}, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "warp");
}

int disc_step_static_stats(const float* s_dev, int nx, int ny, int nz, const int patch[3],
                           float var_floor, float* ys_dev, void* stream)
{
    if (!s_dev || !ys_dev || !patch) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!valid_patch(patch)) return fail(nullptr, DISC_EINVAL, "invalid patch");
    if (!(var_floor >= 0.0f) || !std::isfinite(var_floor))
        return fail(nullptr, DISC_EINVAL, "var_floor must be finite and >= 0");
    hipError_t e = disc::launch_static_stats(s_dev, ys_dev, Dims{nx, ny, nz}, patch, var_floor,
                                             (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "static patch moments");
}

int disc_step_correct(const float* m_dev, const float* ys_dev, int nx, int ny, int nz,
                      const int patch[3], float* f_dev, void* stream)
{
    if (!m_dev || !ys_dev || !f_dev || !patch) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!valid_patch(patch)) return fail(nullptr, DISC_EINVAL, "invalid patch");
    hipError_t e = disc::launch_correct(m_dev, ys_dev, f_dev, Dims{nx, ny, nz}, patch,
                                        (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "correct");
}

int disc_step_force_smooth(const float* m_dev, const float* f_dev, const float* r_dev, int nx,
                           int ny, int nz, float sigma, float diff_floor, float* q_dev,
                           float* r_out_dev, float* rt_dev, void* stream)
{
    if (!m_dev || !f_dev || !r_dev || !q_dev || !r_out_dev)
        return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!(diff_floor >= 0.0f) || !std::isfinite(diff_floor))
        return fail(nullptr, DISC_EINVAL, "diff_floor must be finite and >= 0");
    disc::GaussTaps t;
    if (!disc::make_gauss_taps(sigma, &t)) return fail(nullptr, DISC_EINVAL, "invalid sigma");
    const Dims d{nx, ny, nz};
    hipError_t e = disc::launch_force_xy(m_dev, f_dev, r_dev, q_dev, rt_dev, d, diff_floor, t,
                                         (hipStream_t)stream);
    if (e == hipSuccess) e = disc::launch_smooth_z(q_dev, r_out_dev, d, t, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "force + smoothing");
}

int disc_step_smooth(const float* rt_dev, int nx, int ny, int nz, float sigma, float* q_dev,
                     float* r_dev, void* stream)
{
    if (!rt_dev || !q_dev || !r_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    disc::GaussTaps t;
    if (!disc::make_gauss_taps(sigma, &t)) return fail(nullptr, DISC_EINVAL, "invalid sigma");
    const Dims d{nx, ny, nz};
    hipError_t e = disc::launch_smooth_xy(rt_dev, q_dev, d, t, (hipStream_t)stream);
    if (e == hipSuccess) e = disc::launch_smooth_z(q_dev, r_dev, d, t, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "smooth");
}

size_t disc_step_shift_scratch_bytes(void)
{
    return disc::shift_scratch_bytes();
}

int disc_step_shift(const float* ct_dev, const float* cbct_dev, long n, float* s_dev,
                    double* dhu_dev, void* scratch_dev, size_t scratch_bytes, void* stream)
{
    if (!ct_dev || !cbct_dev || !s_dev || !scratch_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    if (n < 1 || n >= (1L << 31)) return fail(nullptr, DISC_EINVAL, "n must be in [1, 2^31)");
    if (scratch_bytes < disc::shift_scratch_bytes())
        return fail(nullptr, DISC_ENOMEM, "scratch too small");
    if (((uintptr_t)scratch_dev & 15) != 0) return fail(nullptr, DISC_EINVAL, "scratch must be 16-byte aligned");
    hipError_t e = disc::launch_shift(ct_dev, cbct_dev, n, s_dev, dhu_dev, scratch_dev, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "global shift");
}

int disc_step_downsample(const float* in_dev, int nx, int ny, int nz, float* out_dev, void* stream)
{
    if (!in_dev || !out_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    hipError_t e = disc::launch_downsample(in_dev, out_dev, Dims{nx, ny, nz}, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "downsample");
}

int disc_step_upsample_field(const float* rc_dev, int cnx, int cny, int cnz, float* rf_dev, int fnx,
                             int fny, int fnz, void* stream)
{
    if (!rc_dev || !rf_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(cnx, cny, cnz);
    DISC_CHECK_DIMS(fnx, fny, fnz);
    hipError_t e = disc::launch_upsample_field(rc_dev, Dims{cnx, cny, cnz}, rf_dev,
                                               Dims{fnx, fny, fnz}, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "upsample field");
}

int disc_copy_kernel(const void* src_dev, void* dst_dev, size_t bytes, void* stream)
{
    if (!src_dev || !dst_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    if ((bytes & 15) || ((uintptr_t)src_dev & 15) || ((uintptr_t)dst_dev & 15))
        return fail(nullptr, DISC_EINVAL, "copy needs 16-byte aligned pointers and size");
    hipError_t e = disc::launch_copy(src_dev, dst_dev, bytes, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "copy");
}

// ---- timing -------------------------------------------------------------------

int disc_timing_enable(disc_ctx* c, int max_records)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (max_records < 0) return fail(c, DISC_EINVAL, "max_records is negative");
    if ((int)c->ev.size() < 2 * max_records) {
        const size_t have = c->ev.size();
        c->ev.resize(2 * (size_t)max_records);
        for (size_t i = have; i < c->ev.size(); ++i) {
            hipError_t e = hipEventCreate(&c->ev[i]);
            if (e != hipSuccess) {
                c->ev.resize(i);
                return hip_fail(c, e, "event create");
            }
        }
    }
    c->max_rec = max_records;
    c->rec.clear();
    return DISC_OK;
}

int disc_timing_read(disc_ctx* c, int kernel_id, int level, int* launches, double* total_ms,
                     double* total_voxels)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (kernel_id < 0 || kernel_id >= K_COUNT) return fail(c, DISC_EINVAL, "unknown kernel id");
    int nl = 0;
    double ms = 0.0, vox = 0.0;
    for (size_t i = 0; i < c->rec.size(); ++i) {
        if (c->rec[i].kid != kernel_id || (level >= 0 && c->rec[i].level != level)) continue;
        hipError_t e = hipEventSynchronize(c->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "event synchronize");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "event elapsed");
        nl += 1;
        ms += t;
        vox += c->rec[i].voxels;
    }
    if (launches) *launches = nl;
    if (total_ms) *total_ms = ms;
    if (total_voxels) *total_voxels = vox;
    return DISC_OK;
}

}  // extern "C"
