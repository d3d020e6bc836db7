/*
 * Host-side argument and state checks of the C ABI (include/disc.h), for a
 * build of the library's host code with AddressSanitizer and
 * UndefinedBehaviorSanitizer (the CPU test suite compiles and runs it). No
 * call here reaches the GPU: every one is rejected, or answered, before any
 * device work. Exits 0 when every call returns the documented code.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "disc.h"

#define EXPECT(call, code)                                                           \
    do {                                                                             \
        int rc_ = (call);                                                            \
        if (rc_ != (code)) {                                                         \
            fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, rc_, (code)); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

int main(void)
{
    float* fake = (float*)(uintptr_t)(1u << 20);
    double* loss = (double*)(uintptr_t)(1u << 21);
    void* ws = (void*)(uintptr_t)(1u << 22);
    const int patch[3] = {5, 5, 5}, bad[3] = {5, 4, 5};

    disc_params p;
    EXPECT(disc_params_default(&p), DISC_OK);
    EXPECT(disc_params_default(NULL), DISC_EINVAL);

    /* invalid parameters are rejected, with a message */
    disc_ctx* c = NULL;
    disc_params q = p;
    q.patch[0] = 4;
    EXPECT(disc_create(&q, &c), DISC_EINVAL);
    if (c || !strstr(disc_last_error(NULL), "odd")) return 1;
    q = p;
    q.sigma = NAN;
    EXPECT(disc_create(&q, &c), DISC_EINVAL);
    q = p;
    q.levels = 0;
    EXPECT(disc_create(&q, &c), DISC_EINVAL);
    q = p;
    q.mask_mode = 1;
    q.fill_t[1] = 6;
    EXPECT(disc_create(&q, &c), DISC_EINVAL);
    EXPECT(disc_create(NULL, &c), DISC_EINVAL);

    /* sizes */
    if (disc_workspace_bytes(&p, 256, 256, 96) < (size_t)40 * 256 * 256 * 96) return 1;
    if (disc_workspace_bytes(&p, 0, 5, 5) != 0 || disc_workspace_bytes(NULL, 5, 5, 5) != 0) return 1;
    if (disc_ssd_scratch_bytes(16, 16, 16) < (size_t)40 * 16 * 16 * 16 || disc_ssd_scratch_bytes(16, 16, 0) != 0)
        return 1;
    if (disc_step_shift_scratch_bytes() < 16 * 1024) return 1;

    /* a context answers out-of-order calls and argument errors on the host */
    EXPECT(disc_create(&p, &c), DISC_OK);
    EXPECT(disc_iterate(c, 1, NULL), DISC_ESTATE);
    EXPECT(disc_run(c, NULL), DISC_ESTATE);
    EXPECT(disc_get_corrected(c, fake, NULL), DISC_ESTATE);
    EXPECT(disc_state(c, NULL, NULL, NULL), DISC_ESTATE);
    EXPECT(disc_set_volumes(c, NULL, fake, 8, 8, 8, ws, (size_t)1 << 30, NULL), DISC_EINVAL);
    EXPECT(disc_set_volumes(c, fake, fake, 0, 8, 8, ws, (size_t)1 << 30, NULL), DISC_EINVAL);
    EXPECT(disc_set_volumes(c, fake, fake, 8, 8, 8, (char*)ws + 16, (size_t)1 << 30, NULL), DISC_EINVAL);
    EXPECT(disc_set_volumes(c, fake, fake, 64, 64, 64, ws, 1000, NULL), DISC_ENOMEM);
    if (!strstr(disc_last_error(c), "needs")) return 1;
    EXPECT(disc_timing_enable(c, -1), DISC_EINVAL);
    EXPECT(disc_get_stats(c, 0, NULL, NULL, 0, NULL), DISC_ESTATE);
    disc_destroy(c);
    disc_destroy(NULL);

    /* step entry points */
    EXPECT(disc_step_warp(NULL, fake, 4, 4, 4, fake, NULL), DISC_EINVAL);
    EXPECT(disc_step_warp(fake, fake, 4, 4, 70000, fake, NULL), DISC_EINVAL);
    EXPECT(disc_step_correct(fake, fake, 4, 4, 4, bad, fake, NULL), DISC_EINVAL);
    EXPECT(disc_step_static_stats(fake, 4, 4, 4, patch, -1.0f, fake, NULL), DISC_EINVAL);
    EXPECT(disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0f, INFINITY, 0, fake, fake, NULL, NULL, NULL,
                                  NULL),
           DISC_EINVAL);
    EXPECT(disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0f, 1e-3f, 0, fake, fake, NULL, fake, NULL, NULL),
           DISC_EINVAL);
    EXPECT(disc_step_smooth(fake, 4, 4, 4, 3.0f, fake, fake, NULL), DISC_EINVAL);
    EXPECT(disc_step_shift(fake, fake, 10, fake, NULL, ws, 8, NULL), DISC_ENOMEM);
    EXPECT(disc_step_upsample_field(fake, 0, 1, 1, fake, 2, 2, 2, NULL), DISC_EINVAL);
    EXPECT(disc_copy_kernel(fake, fake, 10, NULL), DISC_EINVAL);

    /* differentiable path */
    const size_t need = disc_ssd_scratch_bytes(16, 16, 16);
    EXPECT(disc_ssd_loss(fake, fake, fake, 16, 16, 16, bad, loss, ws, need, NULL), DISC_EINVAL);
    EXPECT(disc_ssd_loss(fake, fake, fake, 16, 16, 16, patch, loss, ws, need - 1, NULL), DISC_ENOMEM);
    EXPECT(disc_ssd_grad(fake, fake, fake, 16, 16, 16, patch, NULL, NULL, NULL, ws, need, NULL), DISC_EINVAL);
    EXPECT(disc_ssd_loss_noalloc(fake, fake, fake, 512, 512, 160, patch, loss, NULL), DISC_ENOMEM);

    /* batches */
    disc_params pb = p;
    pb.patch[0] = pb.patch[1] = pb.patch[2] = 5;
    pb.sigma = 1.5f;
    pb.levels = 1;
    pb.iters[0] = 10;
    const int dims[6] = {40, 30, 20, 33, 17, 9};
    disc_batch* b = NULL;
    EXPECT(disc_batch_create(&pb, 2, dims, &b), DISC_OK);
    const size_t bws = disc_batch_workspace_bytes(b);
    if (bws < (size_t)40 * (40 * 30 * 20 + 33 * 17 * 9)) return 1;
    EXPECT(disc_batch_set_tiles(b, 24, 256, 512, 2048), DISC_EINVAL);
    EXPECT(disc_batch_iterate(b, 1, 1, NULL), DISC_ESTATE);
    const float* vols[2] = {fake, fake + 1024};
    EXPECT(disc_batch_set_volumes(b, vols, vols, ws, bws - 1, NULL), DISC_ENOMEM);
    if (!strstr(disc_batch_last_error(b), "needs") && !strstr(disc_batch_last_error(b), "bytes")) return 1;
    disc_batch_destroy(b);
    EXPECT(disc_batch_create(&pb, 17, dims, &b), DISC_EINVAL);
    disc_batch_destroy(NULL);

    printf("abi host checks: ok\n");
    return 0;
}
