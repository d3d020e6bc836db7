// C ABI of libdisc: argument validation, workspace layout, the Algorithm A1
// level schedule and per-kernel event timing. Kernels live in the other
// translation units; this file only decides what to launch.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "disc.h"
#include "kernels.h"

using disc::Dims;

namespace {

thread_local std::string g_thread_err;

enum KernelId { K_WARP = 0, K_CORRECT = 1, K_FORCE_XY = 2, K_SMOOTH_Z = 3, K_UPSAMPLE = 4, K_FILL = 5, K_COUNT = 6 };

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
    // Sec. 2.3 stopping rule: workgroup norm sums of the z pass, l^(k) per
    // level (hist_stride entries each), per level {stop flag, iterations run}
    double* norms = nullptr;
    double* hist = nullptr;
    int* flags = nullptr;
    int hist_stride = 1;
    int norm_parts = 0;
    // Eq. 7-10 (mask_mode 1): STD(S) per level, (a, b) and stamps (finest
    // size), per-pass counters, {HU_0, a_min, a_max, h, a_m}, Delta HU
    float* sd[DISC_MAX_LEVELS] = {};
    float2* ab = nullptr;
    unsigned char* stamp = nullptr;
    int* filled = nullptr;           // per pass: voxels filled
    disc::FillLists fl{};            // fill work lists
    long fl_clear = 0;               // floats to zero: queued, then wcount
    float* consts = nullptr;
    double* dhu = nullptr;
    void* med_scratch = nullptr;
    int cur = 0;
    int level = 0;
    int it = 0;
    bool ready = false;
    bool f_valid = false;
    bool m_ready = false;  // m holds CT(x + r(x)) for the current field
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
    return (long)nx * ny * nz < (1L << 30);
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
    if (p->force_mode != 0 && p->force_mode != 1)
        return fail(c, DISC_EINVAL, "force_mode must be 0 (static-gradient) or 1 (double force)");
    if (!(p->stop_eps >= 0.0f) || !std::isfinite(p->stop_eps))
        return fail(c, DISC_EINVAL, "stop_eps must be finite and >= 0");
    if (p->stop_eps > 0.0f && (p->stop_lag < 1 || p->stop_lag > 1000))
        return fail(c, DISC_EINVAL, "stop_lag must be in 1..1000");
    if (p->mask_mode != 0 && p->mask_mode != 1) return fail(c, DISC_EINVAL, "mask_mode must be 0 or 1");
    if (p->mask_mode == 1) {
        if (!std::isfinite(p->hu0) || !std::isfinite(p->fill_h))
            return fail(c, DISC_EINVAL, "hu0 and fill_h must be finite");
        if (!(p->a_lo >= 0.0f) || !(p->a_hi > p->a_lo) || !std::isfinite(p->a_hi))
            return fail(c, DISC_EINVAL, "need 0 <= a_lo < a_hi, finite");
        for (int d = 0; d < 3; ++d)
            if (p->fill_t[d] < 1 || p->fill_t[d] > 15 || p->fill_t[d] % 2 == 0)
                return fail(c, DISC_EINVAL, "fill_t extents must be odd, 1..15");
        if (p->fill_passes < 1 || p->fill_passes > 64)
            return fail(c, DISC_EINVAL, "fill_passes must be in 1..64");
    }
    if (p->check_finite != 0 && p->check_finite != 1) return fail(c, DISC_EINVAL, "check_finite must be 0 or 1");
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

size_t carve(disc_ctx* c, const disc_params* p, char* base, int L, const Dims* dims)
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
    int parts = 1, stride = 1;
    for (int l = 0; l < L; ++l) {
        parts = std::max(parts, disc::smooth_z_blocks(dims[l]));
        stride = std::max(stride, p->iters[l]);
    }
    double* norms = (double*)cv.take((size_t)parts * 2 * sizeof(double));
    // history and flags are contiguous: one fill clears both at set-up
    double* hist = (double*)cv.take((size_t)L * stride * sizeof(double) + (size_t)L * 2 * sizeof(int));
    if (p->mask_mode == 1) {
        for (int l = 0; l < L; ++l) {
            float* sdl = (float*)cv.take((size_t)dims[l].n() * 4);
            if (c) c->sd[l] = sdl;
        }
        float2* ab = (float2*)cv.take(nf * sizeof(float2));
        unsigned char* stamp = (unsigned char*)cv.take(nf);
        int* filled = (int*)cv.take((size_t)(p->fill_passes + 1) * sizeof(int));
        // queued and wcount are contiguous: one fill clears both
        const size_t ntl = (size_t)disc::fill_tiles(dims[L - 1]);
        int* queued = (int*)cv.take((ntl + (size_t)p->fill_passes + 2) * sizeof(int));
        int* wl = (int*)cv.take((size_t)(p->fill_passes + 1) * ntl * sizeof(int));
        float* consts = (float*)cv.take(8 * sizeof(float));
        double* dhu = (double*)cv.take(sizeof(double));
        void* med = cv.take(disc::median_scratch_bytes());
        if (c) {
            c->ab = ab;
            c->stamp = stamp;
            c->filled = filled;
            c->fl = disc::FillLists{queued, wl, queued + ntl};
            c->fl_clear = (long)(ntl + (size_t)p->fill_passes + 2);
            c->consts = consts;
            c->dhu = dhu;
            c->med_scratch = med;
        }
    }
    if (c) {
        c->r[0] = r0;
        c->r[1] = r1;
        c->m = m;
        c->f = f;
        c->scratch = sc;
        c->norms = norms;
        c->hist = hist;
        c->flags = hist ? reinterpret_cast<int*>(hist + (size_t)L * stride) : nullptr;
        c->hist_stride = stride;
        c->norm_parts = parts;
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
        c->m_ready = false;
    }
    const int l = c->level;
    const Dims d = c->dims[l];
    const double vox = (double)d.n();
    float* r = c->r[c->cur];
    float* q = c->r[1 - c->cur];
    // with the stopping rule on, every kernel of this level checks the
    // level's flag and the iteration becomes a no-op once it is set
    const bool rule = c->p.stop_eps > 0.0f;
    int* flags = rule ? c->flags + 2 * l : nullptr;
    // the history holds hist_stride >= iters[l] entries: iterations past the
    // schedule (finest level) run without evaluating the rule again
    const bool record = rule && c->it < c->hist_stride;
    // the z pass of the previous iteration has already warped the CT with
    // the field it produced; a standalone warp is needed only after set-up,
    // a level switch or disc_set_field
    if (!c->m_ready) {
        {
            Timed tm(c, st, K_WARP, l, vox);
            e = disc::launch_warp(c->ct[l], r, c->m, d, st, flags);
        }
        if (e != hipSuccess) return hip_fail(c, e, "warp");
    }
    if (c->p.mask_mode == 1) {
        {
            Timed tm(c, st, K_CORRECT, l, vox);
            e = disc::launch_fill(reinterpret_cast<float*>(c->filled), c->p.fill_passes + 1, 0.0f, st);
            if (e == hipSuccess)
                e = disc::launch_fill(reinterpret_cast<float*>(c->fl.queued), c->fl_clear, 0.0f, st);
            if (e == hipSuccess)
                e = disc::launch_mask_moments(c->m, c->ys[l], c->s[l], c->sd[l], c->ab, c->stamp, c->consts, d,
                                              c->p.patch, st, flags);
        }
        if (e != hipSuccess) return hip_fail(c, e, "correct (mask)");
        {
            Timed tm(c, st, K_FILL, l, vox);
            e = disc::launch_fill_seed(c->stamp, c->fl, d, c->p.fill_t, flags, st);
            for (int pass = 1; pass <= c->p.fill_passes && e == hipSuccess; ++pass)
                e = disc::launch_fill_pass(c->ab, c->stamp, c->s[l], c->consts, c->filled, c->fl, pass,
                                           c->p.fill_passes, d, c->p.fill_t, flags, st);
            if (e == hipSuccess) e = disc::launch_apply_ab(c->ab, c->s[l], c->f, d, flags, st);
        }
        if (e != hipSuccess) return hip_fail(c, e, "fill");
    } else {
        Timed tm(c, st, K_CORRECT, l, vox);
        e = disc::launch_correct(c->m, c->ys[l], c->f, d, c->p.patch, st, flags);
        if (e != hipSuccess) return hip_fail(c, e, "correct");
    }
    {
        Timed tm(c, st, K_FORCE_XY, l, vox);
        e = disc::launch_force_xy(c->m, c->f, r, q, nullptr, d, c->p.diff_floor, c->p.force_mode, c->taps,
                                  flags, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "force + xy smoothing");
    {
        Timed tm(c, st, K_SMOOTH_Z, l, vox);
        e = disc::launch_smooth_z(q, r, d, c->taps, flags, record ? c->norms : nullptr, st, c->ct[l], c->m);
    }
    if (e != hipSuccess) return hip_fail(c, e, "z smoothing");
    if (record) {
        e = disc::launch_stop_rule(c->norms, disc::smooth_z_blocks(d), c->hist + (size_t)l * c->hist_stride,
                                   flags, c->it, c->p.stop_lag, (double)c->p.stop_eps, st);
        if (e != hipSuccess) return hip_fail(c, e, "stopping rule");
    }
    c->it += 1;
    c->f_valid = true;
    c->m_ready = true;
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
    p->force_mode = 0;
    p->stop_eps = 0.0f;
    p->stop_lag = 10;
    p->mask_mode = 0;
    p->hu0 = 0.0f;
    p->a_lo = 0.5f;
    p->a_hi = 1.5f;
    p->fill_h = 0.0f;
    p->fill_t[0] = p->fill_t[1] = 7;
    p->fill_t[2] = 3;
    p->fill_passes = 10;
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
    return carve(nullptr, p, nullptr, p->levels, dims);
}

int disc_set_volumes(disc_ctx* c, const float* ct_dev, const float* cbct_dev, int nx, int ny,
                     int nz, void* workspace_dev, size_t workspace_bytes, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!ct_dev || !cbct_dev || !workspace_dev)
        return fail(c, DISC_EINVAL, "ct, cbct and workspace must be device pointers");
    if (!valid_dims(nx, ny, nz))
        return fail(c, DISC_EINVAL, "dims (%d,%d,%d): need >= 1, nz <= 65535, N < 2^30", nx, ny, nz);
    if (((uintptr_t)workspace_dev & 255) != 0)
        return fail(c, DISC_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = disc_workspace_bytes(&c->p, nx, ny, nz);
    if (workspace_bytes < need)
        return fail(c, DISC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    c->ready = false;
    level_dims(c->L, nx, ny, nz, c->dims);
    carve(c, &c->p, (char*)workspace_dev, c->L, c->dims);
    const int L = c->L;
    const Dims fin = c->dims[L - 1];
    c->ct[L - 1] = ct_dev;
    hipError_t e;
    if (c->p.check_finite) {
        // count NaN / Inf voxels into the first word of the shift scratch
        // (the shift below overwrites it) and wait for the answer
        int* cnt = static_cast<int*>(c->scratch);
        int host_cnt = 0;
        e = disc::launch_fill(reinterpret_cast<float*>(cnt), 1, 0.0f, st);
        if (e == hipSuccess) e = disc::launch_count_nonfinite(ct_dev, cbct_dev, fin.n(), cnt, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&host_cnt, cnt, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "finite check");
        if (host_cnt > 0)
            return fail(c, DISC_ENONFINITE, "ct and cbct hold %d NaN or Inf voxels", host_cnt);
    }
    const bool mask = c->p.mask_mode == 1;
    if (c->p.global_shift) {
        e = disc::launch_shift(ct_dev, cbct_dev, fin.n(), c->s[L - 1], mask ? c->dhu : nullptr, c->scratch, st);
        if (e != hipSuccess) return hip_fail(c, e, "global shift");
    } else {
        if (mask) {
            // Delta HU alone (HU_0 = 2 |Delta HU|); the shifted copy is scratch
            e = disc::launch_shift(ct_dev, cbct_dev, fin.n(), reinterpret_cast<float*>(c->ab), c->dhu, c->scratch, st);
            if (e != hipSuccess) return hip_fail(c, e, "mean difference");
        }
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
        e = disc::launch_static_stats(c->s[l], c->ys[l], c->dims[l], c->p.patch, c->p.var_floor, st,
                                      mask ? c->sd[l] : nullptr);
        if (e != hipSuccess) return hip_fail(c, e, "static patch moments");
    }
    if (mask) {
        // Sec. 2.3 rules on the initial finest images: a_m, then the Eq. 7
        // and Eq. 10 constants, all on the device (the a list is scratch in ab)
        float* avals = reinterpret_cast<float*>(c->ab);
        e = disc::launch_amed_values(ct_dev, c->ys[L - 1], c->sd[L - 1], avals, fin, c->p.patch, c->p.var_floor, st);
        if (e == hipSuccess)
            e = disc::launch_mask_consts(avals, fin.n(), c->dhu, c->p.hu0, c->p.a_lo, c->p.a_hi, c->p.fill_h,
                                         c->med_scratch, c->consts, st);
        if (e != hipSuccess) return hip_fail(c, e, "mask parameters");
    }
    e = disc::launch_fill(c->r[0], 3 * c->dims[0].n(), 0.0f, st);
    if (e != hipSuccess) return hip_fail(c, e, "zero field");
    // l^(k) history and stop flags (all-zero bits: 0.0 and 0)
    e = disc::launch_fill(reinterpret_cast<float*>(c->hist),
                          (long)(c->L * c->hist_stride * 2 + c->L * 2), 0.0f, st);
    if (e != hipSuccess) return hip_fail(c, e, "clear stopping-rule state");
    c->cur = 0;
    c->level = 0;
    c->it = 0;
    c->f_valid = false;
    c->m_ready = false;
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
    c->m_ready = false;
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

int disc_get_mask(disc_ctx* c, unsigned char* out_dev, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (!out_dev) return fail(c, DISC_EINVAL, "out is NULL");
    if (c->p.mask_mode != 1) return fail(c, DISC_ENOTSUP, "mask_mode is 0");
    if (!c->f_valid) return fail(c, DISC_ESTATE, "no iteration has run at the current level");
    const Dims d = c->dims[c->level];
    hipError_t e = hipMemcpyAsync(out_dev, c->stamp, (size_t)d.n(), hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : hip_fail(c, e, "copy mask");
}

// ---- single steps -----------------------------------------------------------

#define DISC_CHECK_DIMS(nx, ny, nz)                                                        \
    if (!valid_dims(nx, ny, nz))                                                           \
        return fail(nullptr, DISC_EINVAL, "dims (%d,%d,%d): need >= 1, nz <= 65535, N < 2^30", \
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
                           int ny, int nz, float sigma, float diff_floor, int force_mode, float* q_dev,
                           float* r_out_dev, float* rt_dev, const float* ct_dev, float* m_out_dev,
                           void* stream)
{
    if (!m_dev || !f_dev || !r_dev || !q_dev || !r_out_dev)
        return fail(nullptr, DISC_EINVAL, "null pointer");
    if ((ct_dev == nullptr) != (m_out_dev == nullptr))
        return fail(nullptr, DISC_EINVAL, "ct and m_out are both given or both NULL");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!(diff_floor >= 0.0f) || !std::isfinite(diff_floor))
        return fail(nullptr, DISC_EINVAL, "diff_floor must be finite and >= 0");
    disc::GaussTaps t;
    if (!disc::make_gauss_taps(sigma, &t)) return fail(nullptr, DISC_EINVAL, "invalid sigma");
    const Dims d{nx, ny, nz};
    if (force_mode != 0 && force_mode != 1) return fail(nullptr, DISC_EINVAL, "force_mode must be 0 or 1");
    hipError_t e = disc::launch_force_xy(m_dev, f_dev, r_dev, q_dev, rt_dev, d, diff_floor, force_mode, t,
                                         nullptr,
                                         (hipStream_t)stream);
    if (e == hipSuccess)
        e = disc::launch_smooth_z(q_dev, r_out_dev, d, t, nullptr, nullptr, (hipStream_t)stream, ct_dev, m_out_dev);
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
    if (e == hipSuccess) e = disc::launch_smooth_z(q_dev, r_dev, d, t, nullptr, nullptr, (hipStream_t)stream);
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
    if (n < 1 || n >= (1L << 30)) return fail(nullptr, DISC_EINVAL, "n must be in [1, 2^30)");
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

int disc_get_stats(disc_ctx* c, int level, int* iters_done, double* l_hist, int max_k, void* stream)
{
    if (!c) return fail(nullptr, DISC_EINVAL, "context is NULL");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (!(c->p.stop_eps > 0.0f)) return fail(c, DISC_ENOTSUP, "the stopping rule is off (stop_eps = 0)");
    if (level < 0 || level >= c->L) return fail(c, DISC_EINVAL, "level %d outside 0..%d", level, c->L - 1);
    if (max_k < 0 || (max_k > 0 && !l_hist)) return fail(c, DISC_EINVAL, "bad history buffer");
    hipStream_t st = (hipStream_t)stream;
    int fl[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(fl, c->flags + 2 * level, sizeof fl, hipMemcpyDeviceToHost, st);
    const int k = std::min(max_k, c->hist_stride);
    if (e == hipSuccess && k > 0)
        e = hipMemcpyAsync(l_hist, c->hist + (size_t)level * c->hist_stride, (size_t)k * sizeof(double),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "read stopping-rule state");
    if (iters_done) *iters_done = fl[1];
    return DISC_OK;
}

int disc_get_mask_params(disc_ctx* c, float out[5], void* stream)
{
    if (!c || !out) return fail(c, DISC_EINVAL, "null pointer");
    if (!c->ready) return fail(c, DISC_ESTATE, "disc_set_volumes has not succeeded");
    if (c->p.mask_mode != 1) return fail(c, DISC_ENOTSUP, "mask_mode is 0");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(out, c->consts, 5 * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? DISC_OK : hip_fail(c, e, "read mask parameters");
}

// ---- differentiable DISC: SSD loss and gradient ----------------------------

namespace {

// Scratch of the SSD calls: m, D (N floats each), two N-element double2
// buffers for the adjoint passes, the per-workgroup loss partials.
struct SsdScratch {
    float* m;
    float* dres;
    double2* a;
    double2* b;
    double* partial;
    size_t bytes;
};

// (base may be null: sizes only)
SsdScratch ssd_carve(char* base, Dims d)
{
    const size_t n = (size_t)d.n();
    Carver cv{base};
    SsdScratch s;
    s.m = static_cast<float*>(cv.take(n * sizeof(float)));
    s.dres = static_cast<float*>(cv.take(n * sizeof(float)));
    s.a = static_cast<double2*>(cv.take(n * sizeof(double2)));
    s.b = static_cast<double2*>(cv.take(n * sizeof(double2)));
    s.partial = static_cast<double*>(cv.take((size_t)disc::ssd_partial_count(d) * sizeof(double)));
    s.bytes = (cv.off + 255) & ~(size_t)255;
    return s;
}

int ssd_check(const float* ct, const float* ys, const float* r, int nx, int ny, int nz,
              const int patch[3], void* scratch, size_t scratch_bytes)
{
    if (!ct || !ys || !r || !patch || !scratch) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!valid_patch(patch)) return fail(nullptr, DISC_EINVAL, "invalid patch");
    if ((reinterpret_cast<uintptr_t>(scratch) & 255) != 0)
        return fail(nullptr, DISC_EINVAL, "scratch must be 256-byte aligned");
    const size_t need = ssd_carve(nullptr, Dims{nx, ny, nz}).bytes;
    if (scratch_bytes < need)
        return fail(nullptr, DISC_ENOMEM, "scratch of %zu bytes, need %zu", scratch_bytes, need);
    return DISC_OK;
}

}  // namespace

size_t disc_ssd_scratch_bytes(int nx, int ny, int nz)
{
    if (!valid_dims(nx, ny, nz)) return 0;
    return ssd_carve(nullptr, Dims{nx, ny, nz}).bytes;
}

int disc_ssd_loss(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny, int nz,
                  const int patch[3], double* loss_dev, void* scratch_dev, size_t scratch_bytes,
                  void* stream)
{
    if (!loss_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    int rc = ssd_check(ct_dev, ys_dev, r_dev, nx, ny, nz, patch, scratch_dev, scratch_bytes);
    if (rc != DISC_OK) return rc;
    const Dims d{nx, ny, nz};
    const hipStream_t st = (hipStream_t)stream;
    const SsdScratch s = ssd_carve(static_cast<char*>(scratch_dev), d);
    hipError_t e = disc::launch_warp(ct_dev, r_dev, s.m, d, st);
    if (e == hipSuccess) e = disc::launch_ssd_moments(s.m, ys_dev, s.dres, nullptr, s.partial, d, patch, st);
    if (e == hipSuccess) e = disc::launch_ssd_finish(s.partial, disc::ssd_partial_count(d), loss_dev, st);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "ssd loss");
}

int disc_ssd_grad(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny, int nz,
                  const int patch[3], const float* scale_dev, float* grad_dev, double* loss_dev,
                  void* scratch_dev, size_t scratch_bytes, void* stream)
{
    if (!grad_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    int rc = ssd_check(ct_dev, ys_dev, r_dev, nx, ny, nz, patch, scratch_dev, scratch_bytes);
    if (rc != DISC_OK) return rc;
    const Dims d{nx, ny, nz};
    const hipStream_t st = (hipStream_t)stream;
    const SsdScratch s = ssd_carve(static_cast<char*>(scratch_dev), d);
    hipError_t e = disc::launch_warp(ct_dev, r_dev, s.m, d, st);
    if (e == hipSuccess) e = disc::launch_ssd_moments(s.m, ys_dev, s.dres, s.a, s.partial, d, patch, st);
    if (e == hipSuccess) e = disc::launch_box_adjoint(s.a, s.b, d, 0, patch[0] / 2, st);
    if (e == hipSuccess) e = disc::launch_box_adjoint(s.b, s.a, d, 1, patch[1] / 2, st);
    if (e == hipSuccess)
        e = disc::launch_ssd_grad_z(ct_dev, r_dev, s.m, s.dres, s.a, scale_dev, grad_dev, d, patch[2] / 2, st);
    if (e == hipSuccess && loss_dev)
        e = disc::launch_ssd_finish(s.partial, disc::ssd_partial_count(d), loss_dev, st);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "ssd gradient");
}

}  // extern "C"

// ---- allocation-free SSD loss ------------------------------------------------
// The scratch of disc_ssd_loss_noalloc (m and the per-workgroup loss
// partials) is this fixed device array: every GPU the library runs on holds
// its own copy until the process ends. Host code never passes the array's
// name to a kernel (on the host it only stands for the symbol); it uses the
// device address hipGetSymbolAddress returns, looked up once per device.
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (current device).
int noalloc_scratch(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, DISC_ENOTSUP, "device %d: the allocation-free loss supports devices 0..%d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(nullptr, DISC_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DISC_OK;
}

}  // namespace

extern "C" {

int disc_ssd_loss_noalloc(const float* ct_dev, const float* ys_dev, const float* r_dev, int nx, int ny, int nz,
                          const int patch[3], double* loss_dev, void* stream)
{
    if (!ct_dev || !ys_dev || !r_dev || !patch || !loss_dev) return fail(nullptr, DISC_EINVAL, "null pointer");
    DISC_CHECK_DIMS(nx, ny, nz);
    if (!valid_patch(patch)) return fail(nullptr, DISC_EINVAL, "invalid patch");
    const Dims d{nx, ny, nz};
    // the loss uses the warped image m and the loss partials of the scratch
    const size_t m_bytes = ((size_t)d.n() * sizeof(float) + 255) & ~(size_t)255;
    const size_t need = m_bytes + (size_t)disc::ssd_partial_count(d) * sizeof(double);
    if (need > kNoAllocScratchBytes)
        return fail(nullptr, DISC_ENOMEM,
                    "volume of %ld voxels needs %zu bytes of scratch; the allocation-free loss holds %zu "
                    "(use disc_ssd_loss with a caller workspace)",
                    d.n(), need, kNoAllocScratchBytes);
    void* base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc != DISC_OK) return rc;
    float* m = static_cast<float*>(base);
    double* partial = reinterpret_cast<double*>(static_cast<char*>(base) + m_bytes);
    const hipStream_t st = (hipStream_t)stream;
    // every scratch element read below is written first by this call (m by
    // the warp, one partial per workgroup by the sweep): nothing is cleared
    hipError_t e = disc::launch_warp(ct_dev, r_dev, m, d, st);
    if (e == hipSuccess) e = disc::launch_ssd_moments(m, ys_dev, nullptr, nullptr, partial, d, patch, st);
    if (e == hipSuccess) e = disc::launch_ssd_finish(partial, disc::ssd_partial_count(d), loss_dev, st);
    return e == hipSuccess ? DISC_OK : hip_fail(nullptr, e, "ssd loss (allocation-free)");
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

// ---- batches of volumes ------------------------------------------------------

}  // extern "C"

struct disc_batch {
    disc_params p;
    disc::GaussTaps taps;
    disc::BatchTiles tiles;
    int n = 0;
    std::vector<Dims> dims;
    std::vector<disc::BatchVol> vols;
    std::vector<float*> s;
    void* shift_scratch = nullptr;
    int it = 0;
    bool ready = false;
    bool f_valid = false;
    bool m_ready = false;  // m holds CT(x + r(x)) for the current field
    std::string err;
    // captured iteration loop: graph_iters iterations, replayed by disc_batch_iterate
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_iters = 0;
};

namespace {

int bfail(disc_batch* b, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

int bfail(disc_batch* b, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b)
        b->err = buf;
    else
        g_thread_err = buf;
    return code;
}

void drop_graph(disc_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_iters = 0;
}

// One iteration of every pair. The z pass also warps the CT with the field
// it produces, so the standalone warp runs only when m is not yet current
// (after set-up).
hipError_t batch_once(disc_batch* b, hipStream_t st)
{
    const disc::BatchVol* v = b->vols.data();
    hipError_t e = hipSuccess;
    if (!b->m_ready) e = disc::launch_warp_batch(v, b->n, st);
    if (e == hipSuccess) e = disc::launch_correct_batch(v, b->n, b->p.patch, b->tiles, st);
    if (e == hipSuccess)
        e = disc::launch_force_xy_batch(v, b->n, b->p.diff_floor, b->p.force_mode, b->taps, b->tiles.plane_target, st);
    if (e == hipSuccess) e = disc::launch_smooth_z_batch(v, b->n, b->taps, b->tiles.z_target, true, st);
    if (e == hipSuccess) b->m_ready = true;
    return e;
}

size_t batch_bytes(const std::vector<Dims>& dims)
{
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = up(disc::shift_scratch_bytes());
    for (const Dims& d : dims) off += 10 * up((size_t)d.n() * sizeof(float));  // s ys m f + r q (3 each)
    return off;
}

}  // namespace

extern "C" {

int disc_batch_create(const disc_params* p, int n, const int* dims, disc_batch** out)
{
    if (!out) return bfail(nullptr, DISC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(nullptr, p);
    if (rc != DISC_OK) return rc;
    if (p->levels != 1)
        return bfail(nullptr, DISC_ENOTSUP, "batches run one resolution level (levels = 1)");
    if (p->stop_eps > 0.0f)
        return bfail(nullptr, DISC_ENOTSUP, "batches run fixed iteration counts (stop_eps = 0)");
    if (p->mask_mode != 0) return bfail(nullptr, DISC_ENOTSUP, "batches run without the Eq. 7-10 mask");
    if (n < 1 || n > DISC_MAX_BATCH) return bfail(nullptr, DISC_EINVAL, "batch size %d outside 1..%d", n, DISC_MAX_BATCH);
    if (!dims) return bfail(nullptr, DISC_EINVAL, "dims is NULL");
    disc_batch* b = new disc_batch();
    b->p = *p;
    disc::make_gauss_taps(p->sigma, &b->taps);
    b->n = n;
    for (int v = 0; v < n; ++v) {
        const int nx = dims[3 * v], ny = dims[3 * v + 1], nz = dims[3 * v + 2];
        if (!valid_dims(nx, ny, nz)) {
            delete b;
            return bfail(nullptr, DISC_EINVAL, "volume %d: dims (%d,%d,%d) invalid", v, nx, ny, nz);
        }
        b->dims.push_back(Dims{nx, ny, nz});
    }
    b->vols.resize(n);
    b->s.resize(n);
    b->tiles = disc::BatchTiles{32, 256, 256, 8192};
    *out = b;
    return DISC_OK;
}

void disc_batch_destroy(disc_batch* b)
{
    if (!b) return;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

const char* disc_batch_last_error(const disc_batch* b)
{
    return b ? b->err.c_str() : g_thread_err.c_str();
}

size_t disc_batch_workspace_bytes(const disc_batch* b)
{
    return b ? batch_bytes(b->dims) : 0;
}

int disc_batch_set_tiles(disc_batch* b, int mom_ts, int mom_target, int plane_target, int z_target)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    if ((mom_ts != 16 && mom_ts != 32) || mom_target < 1 || plane_target < 1 || z_target < 1)
        return bfail(b, DISC_EINVAL, "tiles: mom_ts 16 or 32, targets >= 1");
    b->tiles = disc::BatchTiles{mom_ts, mom_target, plane_target, z_target};
    drop_graph(b);
    return DISC_OK;
}

int disc_batch_set_volumes(disc_batch* b, const float* const* ct_dev, const float* const* cbct_dev,
                           void* workspace_dev, size_t workspace_bytes, void* stream)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    if (!ct_dev || !cbct_dev || !workspace_dev) return bfail(b, DISC_EINVAL, "null pointer");
    for (int v = 0; v < b->n; ++v)
        if (!ct_dev[v] || !cbct_dev[v]) return bfail(b, DISC_EINVAL, "volume %d: null pointer", v);
    if (((uintptr_t)workspace_dev & 255) != 0) return bfail(b, DISC_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = batch_bytes(b->dims);
    if (workspace_bytes < need)
        return bfail(b, DISC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    b->ready = false;
    drop_graph(b);
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* base = static_cast<char*>(workspace_dev);
    size_t off = 0;
    b->shift_scratch = base;
    off += up(disc::shift_scratch_bytes());
    for (int v = 0; v < b->n; ++v) {
        const Dims d = b->dims[v];
        const size_t sz = up((size_t)d.n() * sizeof(float));
        disc::BatchVol& bv = b->vols[v];
        b->s[v] = reinterpret_cast<float*>(base + off);
        off += sz;
        float* ys = reinterpret_cast<float*>(base + off);
        off += sz;
        bv.m = reinterpret_cast<float*>(base + off);
        off += sz;
        bv.f = reinterpret_cast<float*>(base + off);
        off += sz;
        bv.r = reinterpret_cast<float*>(base + off);
        off += 3 * sz;
        bv.q = reinterpret_cast<float*>(base + off);
        off += 3 * sz;
        bv.ct = ct_dev[v];
        bv.ys = ys;
        bv.d = d;
        hipError_t e;
        if (b->p.global_shift)
            e = disc::launch_shift(ct_dev[v], cbct_dev[v], d.n(), b->s[v], nullptr, b->shift_scratch, st);
        else
            e = hipMemcpyAsync(b->s[v], cbct_dev[v], (size_t)d.n() * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = disc::launch_static_stats(b->s[v], ys, d, b->p.patch, b->p.var_floor, st);
        if (e == hipSuccess) e = disc::launch_fill(bv.r, 3 * d.n(), 0.0f, st);
        if (e != hipSuccess)
            return bfail(b, DISC_EHIP, "set-up of volume %d: %s", v, hipGetErrorString(e));
    }
    b->it = 0;
    b->f_valid = false;
    b->m_ready = false;
    b->ready = true;
    return DISC_OK;
}

int disc_batch_iterate(disc_batch* b, int n, int use_graph, void* stream)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    if (!b->ready) return bfail(b, DISC_ESTATE, "disc_batch_set_volumes has not succeeded");
    if (n < 0) return bfail(b, DISC_EINVAL, "n must be >= 0");
    if (n == 0) return DISC_OK;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!use_graph) {
        for (int k = 0; k < n && e == hipSuccess; ++k) e = batch_once(b, st);
        if (e != hipSuccess) return bfail(b, DISC_EHIP, "batched iteration: %s", hipGetErrorString(e));
    } else {
        // the captured loop starts from a current m: warp once, eagerly, after set-up
        if (!b->m_ready) {
            e = disc::launch_warp_batch(b->vols.data(), b->n, st);
            if (e != hipSuccess) return bfail(b, DISC_EHIP, "batched warp: %s", hipGetErrorString(e));
            b->m_ready = true;
        }
        if (b->graph_iters != n) {
            drop_graph(b);
            if (!b->cap) {
                e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
                if (e != hipSuccess) return bfail(b, DISC_EHIP, "capture stream: %s", hipGetErrorString(e));
            }
            e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return bfail(b, DISC_EHIP, "begin capture: %s", hipGetErrorString(e));
            hipError_t le = hipSuccess;
            for (int k = 0; k < n && le == hipSuccess; ++k) le = batch_once(b, b->cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap, &g);
            if (le != hipSuccess || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(b, DISC_EHIP, "capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
            }
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return bfail(b, DISC_EHIP, "instantiate: %s", hipGetErrorString(e));
            }
            b->graph = g;
            b->exec = x;
            b->graph_iters = n;
        }
        e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return bfail(b, DISC_EHIP, "graph launch: %s", hipGetErrorString(e));
    }
    b->it += n;
    b->f_valid = true;
    return DISC_OK;
}

int disc_batch_run(disc_batch* b, int use_graph, void* stream)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    const int left = b->p.iters[0] - b->it;
    return disc_batch_iterate(b, left > 0 ? left : 0, use_graph, stream);
}

int disc_batch_get_field(disc_batch* b, int v, float* out_dev, void* stream)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    if (!b->ready) return bfail(b, DISC_ESTATE, "disc_batch_set_volumes has not succeeded");
    if (v < 0 || v >= b->n || !out_dev) return bfail(b, DISC_EINVAL, "bad volume index or null output");
    const hipError_t e = hipMemcpyAsync(out_dev, b->vols[v].r, (size_t)b->dims[v].n() * 12,
                                        hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : bfail(b, DISC_EHIP, "copy field: %s", hipGetErrorString(e));
}

int disc_batch_get_corrected(disc_batch* b, int v, float* out_dev, void* stream)
{
    if (!b) return bfail(nullptr, DISC_EINVAL, "batch is NULL");
    if (!b->ready || !b->f_valid) return bfail(b, DISC_ESTATE, "no iteration has run");
    if (v < 0 || v >= b->n || !out_dev) return bfail(b, DISC_EINVAL, "bad volume index or null output");
    const hipError_t e = hipMemcpyAsync(out_dev, b->vols[v].f, (size_t)b->dims[v].n() * 4,
                                        hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? DISC_OK : bfail(b, DISC_EHIP, "copy corrected: %s", hipGetErrorString(e));
}

}  // extern "C"
