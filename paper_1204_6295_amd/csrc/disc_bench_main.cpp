// disc_bench: native driver of the C ABI, for hardware-counter runs.
//
// Runs whole DISC registrations of a CT/CBCT pair read from raw float32
// files ([nz][ny][nx], x fastest) and, for counter calibration, one plain
// copy of a known number of bytes through disc_copy_kernel. Only the C ABI
// and the HIP runtime are used (no Python), so profilers that instrument
// dispatches see exactly the library's kernels.
//
// usage: disc_bench CT.f32 CBCT.f32 NX NY NZ PATCH SIGMA LEVELS ITERS STEPS COPY_MIB [VARIANT]
//   VARIANT 0 plain (default), 1 Eq. 7-10 mask and fill (default rules,
//   T = 7x7x3, 10 passes), 2 both Eq. 1 force terms, 3 the Sec. 2.3 stopping
//   rule (eps 1e-4, lag 10), 4 plain registrations followed by STEPS
//   evaluations of the differentiable path (SSD loss and gradient) at the
//   registered field.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "disc.h"

static bool read_raw(const char* path, std::vector<float>& v)
{
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    const size_t got = std::fread(v.data(), sizeof(float), v.size(), f);
    std::fclose(f);
    return got == v.size();
}

#define CHECK_HIP(x)                                                                 \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));             \
            return 1;                                                                \
        }                                                                            \
    } while (0)

#define CHECK_DISC(c, x)                                                             \
    do {                                                                             \
        int r_ = (x);                                                                \
        if (r_ != DISC_OK) {                                                         \
            std::fprintf(stderr, "%s: %d %s\n", #x, r_, disc_last_error(c));         \
            return 1;                                                                \
        }                                                                            \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 12 && argc != 13) {
        std::fprintf(stderr,
                     "usage: %s CT.f32 CBCT.f32 NX NY NZ PATCH SIGMA LEVELS ITERS STEPS COPY_MIB [VARIANT]\n",
                     argv[0]);
        return 2;
    }
    const int variant = argc == 13 ? std::atoi(argv[12]) : 0;
    const int nx = std::atoi(argv[3]), ny = std::atoi(argv[4]), nz = std::atoi(argv[5]);
    const int patch = std::atoi(argv[6]);
    const float sigma = (float)std::atof(argv[7]);
    const int levels = std::atoi(argv[8]), iters = std::atoi(argv[9]);
    const int steps = std::atoi(argv[10]);
    const size_t copy_bytes = (size_t)std::atol(argv[11]) << 20;
    if (nx < 1 || ny < 1 || nz < 1 || levels < 1 || levels > DISC_MAX_LEVELS || steps < 0 || variant < 0 ||
        variant > 4) {
        std::fprintf(stderr, "invalid sizes\n");
        return 2;
    }
    const size_t n = (size_t)nx * ny * nz;
    std::vector<float> ct(n), cb(n);
    if (!read_raw(argv[1], ct) || !read_raw(argv[2], cb)) {
        std::fprintf(stderr, "cannot read %zu floats from the input files\n", n);
        return 1;
    }

    disc_params p;
    disc_params_default(&p);
    p.patch[0] = p.patch[1] = p.patch[2] = patch;
    p.sigma = sigma;
    p.levels = levels;
    for (int l = 0; l < DISC_MAX_LEVELS; ++l) p.iters[l] = l < levels ? iters : 0;
    if (variant == 1) p.mask_mode = 1;
    if (variant == 2) p.force_mode = 1;
    if (variant == 3) {
        p.stop_eps = 1e-4f;
        p.stop_lag = 10;
    }
    disc_ctx* c = nullptr;
    CHECK_DISC(nullptr, disc_create(&p, &c));
    const size_t ws_bytes = disc_workspace_bytes(&p, nx, ny, nz);
    float *d_ct = nullptr, *d_cb = nullptr;
    void* d_ws = nullptr;
    CHECK_HIP(hipMalloc(&d_ct, n * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_cb, n * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_ws, ws_bytes));
    CHECK_HIP(hipMemcpy(d_ct, ct.data(), n * sizeof(float), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_cb, cb.data(), n * sizeof(float), hipMemcpyHostToDevice));
    hipStream_t st;
    CHECK_HIP(hipStreamCreate(&st));

    const auto t0 = std::chrono::steady_clock::now();
    for (int s = 0; s < steps; ++s) {
        CHECK_DISC(c, disc_set_volumes(c, d_ct, d_cb, nx, ny, nz, d_ws, ws_bytes, st));
        CHECK_DISC(c, disc_run(c, st));
    }
    CHECK_HIP(hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::printf("registrations: %d in %.3f ms (%.3f ms each)\n", steps, ms, steps ? ms / steps : 0.0);

    if (variant == 4) {
        // loss + gradient at the registered finest-level field
        const int pt[3] = {patch, patch, patch};
        float *d_s = nullptr, *d_ys = nullptr, *d_r = nullptr, *d_g = nullptr;
        double* d_loss = nullptr;
        void *d_sc = nullptr, *d_ssc = nullptr;
        const size_t sc_bytes = disc_ssd_scratch_bytes(nx, ny, nz);
        const size_t ssc_bytes = disc_step_shift_scratch_bytes();
        CHECK_HIP(hipMalloc(&d_s, n * sizeof(float)));
        CHECK_HIP(hipMalloc(&d_ys, n * sizeof(float)));
        CHECK_HIP(hipMalloc(&d_r, 3 * n * sizeof(float)));
        CHECK_HIP(hipMalloc(&d_g, 3 * n * sizeof(float)));
        CHECK_HIP(hipMalloc(&d_loss, sizeof(double)));
        CHECK_HIP(hipMalloc(&d_sc, sc_bytes));
        CHECK_HIP(hipMalloc(&d_ssc, ssc_bytes));
        CHECK_DISC(c, disc_get_field(c, d_r, nullptr, st));
        CHECK_DISC(nullptr, disc_step_shift(d_ct, d_cb, (long)n, d_s, nullptr, d_ssc, ssc_bytes, st));
        CHECK_DISC(nullptr, disc_step_static_stats(d_s, nx, ny, nz, pt, p.var_floor, d_ys, st));
        const auto t1 = std::chrono::steady_clock::now();
        for (int s = 0; s < steps; ++s)
            CHECK_DISC(nullptr, disc_ssd_grad(d_ct, d_ys, d_r, nx, ny, nz, pt, nullptr, d_g, d_loss, d_sc, sc_bytes, st));
        CHECK_HIP(hipStreamSynchronize(st));
        const double ms1 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
        double loss = 0.0;
        CHECK_HIP(hipMemcpy(&loss, d_loss, sizeof(double), hipMemcpyDeviceToHost));
        std::printf("loss + gradient: %d in %.3f ms (%.3f ms each), loss %.6g\n", steps, ms1, steps ? ms1 / steps : 0.0,
                    loss);
        for (void* q : {(void*)d_s, (void*)d_ys, (void*)d_r, (void*)d_g, (void*)d_loss, d_sc, d_ssc})
            CHECK_HIP(hipFree(q));
    }

    if (copy_bytes) {
        void *a = nullptr, *b = nullptr;
        CHECK_HIP(hipMalloc(&a, copy_bytes));
        CHECK_HIP(hipMalloc(&b, copy_bytes));
        CHECK_HIP(hipMemsetAsync(a, 0, copy_bytes, st));
        CHECK_DISC(nullptr, disc_copy_kernel(a, b, copy_bytes, st));
        CHECK_HIP(hipStreamSynchronize(st));
        std::printf("copy kernel: %zu bytes read, %zu bytes written\n", copy_bytes, copy_bytes);
        CHECK_HIP(hipFree(a));
        CHECK_HIP(hipFree(b));
    }
    disc_destroy(c);
    CHECK_HIP(hipFree(d_ct));
    CHECK_HIP(hipFree(d_cb));
    CHECK_HIP(hipFree(d_ws));
    CHECK_HIP(hipStreamDestroy(st));
    return 0;
}
