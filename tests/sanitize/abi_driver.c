/* Drives the argument validation of libimagegs's C ABI (include/imagegs.h) for a host build under
 * AddressSanitizer and UndefinedBehaviorSanitizer: size queries with good and bad arguments, and
 * every compute entry point with arguments that must be rejected before any device work (so no
 * GPU is needed).  Test infrastructure only: exits 0 when every call returned what it should. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "imagegs.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main(void) {
    size_t ws = 0, sv = 0;
    CHECK(igs_abi_version() == 3);
    for (int s = -5; s <= 0; ++s) CHECK(igs_status_string(s) != NULL);
    CHECK(igs_render_buffer_sizes(1000, 3, 256, 256, 10, 16, 16, 20000, &ws, &sv) == IGS_OK);
    CHECK(ws > 0 && sv > 0);
    CHECK(igs_render_buffer_sizes(1000, 3, 256, 256, 33, 16, 16, 20000, &ws, &sv) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_render_buffer_sizes(1000, 0, 256, 256, 10, 16, 16, 20000, &ws, &sv) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_render_buffer_sizes(-1, 3, 256, 256, 10, 16, 16, 20000, &ws, &sv) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_render_buffer_sizes(1000, 3, 256, 256, 10, 8, 8, 20000, &ws, &sv) ==
          IGS_ERR_UNSUPPORTED);
    CHECK(igs_render_buffer_sizes(1000, 3, 256, 256, 10, 16, 16, 0, &ws, &sv) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_render_buffer_sizes(1000, 3, 256, 256, 10, 16, 16, 100, NULL, &sv) ==
          IGS_ERR_INVALID_ARG);
    int64_t off[6];
    CHECK(igs_saved_offsets(1000, 3, 256, 256, 10, 16, 16, 20000, off) == IGS_OK);
    CHECK(off[0] == 0 && off[5] == (int64_t)sv);
    size_t qws = 0, lws = 0, sws = 0, pws = 0;
    CHECK(igs_query_workspace_size(1000, 500, 3, 64, 64, &qws) == IGS_OK);
    CHECK(igs_query_workspace_size(-1, 500, 3, 64, 64, &qws) == IGS_ERR_INVALID_ARG);
    CHECK(igs_query_workspace_size(1000, 500, 0, 64, 64, &qws) == IGS_ERR_INVALID_ARG);
    CHECK(igs_l1_workspace_size(3 * 64 * 64, &lws) == IGS_OK);
    CHECK(igs_l1_ssim_workspace_size(3, 100, 70, &sws) == IGS_OK);
    CHECK(igs_l1_ssim_workspace_size(0, 100, 70, &sws) == IGS_ERR_INVALID_ARG);
    CHECK(igs_place_workspace_size(64, 64, &pws) == IGS_OK);
    /* compute entry points: rejected before any HIP call (the fake pointer is never read) */
    void *fake = (void *)0x1000;
    CHECK(igs_render(NULL, 0, 3, 16, 16, 10, 16, 16, 100, NULL, NULL, 0, NULL, 0, NULL) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_render(fake, 10, 3, 16, 16, 10, 8, 8, 100, fake, NULL, 0, fake, 1 << 20, NULL) ==
          IGS_ERR_UNSUPPORTED);
    CHECK(igs_render(fake, 10, 3, 16, 16, 10, 16, 16, 100, fake, NULL, 0, fake, 16, NULL) ==
          IGS_ERR_WORKSPACE);
    CHECK(igs_render_backward(NULL, 5, 3, 16, 16, 10, 16, 16, 100, NULL, NULL, NULL, 0, NULL, NULL,
                              0, NULL) == IGS_ERR_INVALID_ARG);
    CHECK(igs_render_l1_grad(fake, 10, 17, 16, 16, 10, 16, 16, 100, fake, fake, fake, fake,
                             1 << 20, fake, 1 << 20, NULL) == IGS_ERR_UNSUPPORTED);
    CHECK(igs_render_l1_grad_noalloc(fake, 10, 3, 16, 16, 10, 16, 16, 100, NULL, fake, fake, fake,
                                     1 << 20, NULL) == IGS_ERR_INVALID_ARG);
    CHECK(igs_render_l1_grad_noalloc(fake, 10, 3, 64, 64, 10, 16, 16, (int64_t)1 << 24, fake,
                                     fake, fake, fake, 1 << 20, NULL) == IGS_ERR_WORKSPACE);
    CHECK(igs_l1_loss_grad(NULL, NULL, 3, 4, 4, NULL, NULL, NULL, 0, NULL) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_l1_ssim_loss_grad(NULL, fake, 3, 8, 8, 0.1, fake, fake, fake, 1 << 20, NULL) ==
          IGS_ERR_INVALID_ARG);
    CHECK(igs_adam_step(NULL, NULL, NULL, NULL, NULL, NULL, NULL, 4, 3, 8, 8, 1e-3f, 1e-3f, 1e-3f,
                        1e-3f, 0.9f, 0.999f, 1e-8f, 0.1f, 4.0f, NULL) == IGS_ERR_INVALID_ARG);
    CHECK(igs_fit_to_render(NULL, NULL, 4, 0, 8, 8, NULL) == IGS_ERR_INVALID_ARG);
    CHECK(igs_grad_to_fit(NULL, NULL, NULL, 4, 3, 8, 8, NULL) == IGS_ERR_INVALID_ARG);
    /* batches: descriptors written on the host, then checked */
    int32_t Hs[3] = {256, 17, 512}, Ws[3] = {64, 33, 512}, Ns[3] = {100, 0, 5000};
    igs_image_desc d[3];
    int64_t totals[4];
    CHECK(igs_batch_describe(3, 3, Hs, Ws, Ns, d, totals) == IGS_OK);
    CHECK(totals[0] == 5100 && totals[2] == 256 * 64 + 17 * 33 + 512 * 512);
    CHECK(igs_batch_buffer_sizes(d, 3, 3, 10, 50000, &ws, &sv) == IGS_OK);
    int64_t boff[7];
    CHECK(igs_batch_saved_offsets(d, 3, 3, 10, 50000, boff) == IGS_OK);
    igs_image_desc bad[3];
    memcpy(bad, d, sizeof(d));
    bad[1].gauss_off += 1;
    CHECK(igs_batch_buffer_sizes(bad, 3, 3, 10, 50000, &ws, &sv) == IGS_ERR_INVALID_ARG);
    Hs[1] = 0;
    CHECK(igs_batch_describe(3, 3, Hs, Ws, Ns, d, totals) == IGS_ERR_INVALID_ARG);
    igs_launch_config cfg;
    CHECK(igs_get_launch_config(&cfg) == IGS_OK);
    CHECK(igs_set_launch_config(NULL) == IGS_ERR_INVALID_ARG);
    printf("abi driver ok\n");
    return 0;
}
