/* Drives every entry point of the FP64 oracle (oracle/oracle.c) on small seeded inputs and with
 * invalid arguments, for a build under AddressSanitizer and UndefinedBehaviorSanitizer.  Test
 * infrastructure only: exits 0 when every call returned what it should. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_num_tiles(int H, int W, int th, int tw);
int orc_tile_lists(const double *params, int N, int n, int H, int W, int th, int tw,
                   const int32_t *tiles, int ntiles, int64_t *counts, int32_t *lists,
                   int64_t lists_cap);
int orc_render_tiles(const double *params, int N, int n, int H, int W, int K, int th, int tw,
                     const int32_t *tiles, int ntiles, double *img, int32_t *topk, double *qsel,
                     const double *grad_img, double *grad_params, double *grad_abs, int nthreads,
                     double gamma, double *margin);
int orc_render_dense(const double *params, int N, int n, int H, int W, int K, int th, int tw,
                     double *img, int nthreads);
int orc_rank_pixel(const double *params, int N, int n, int H, int W, int th, int tw, int h, int w,
                   int32_t *idx, double *q, double *mb, int cap);
int orc_blend_set(const double *params, int N, int n, int h, int w, const int32_t *ids, int k,
                  double *out);

static uint64_t state = 88172645463325252ull;
static double uniform(void) { /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main(void) {
    const int H = 37, W = 45, n = 3, N = 60, th = 16, tw = 16;
    double *p = malloc(sizeof(double) * (5 + n) * N);
    for (int i = 0; i < N; ++i) {
        p[0 * N + i] = uniform() * W;
        p[1 * N + i] = uniform() * H;
        p[2 * N + i] = uniform() * 3.14159;
        p[3 * N + i] = 1.0 + 8.0 * uniform();
        p[4 * N + i] = 1.0 + 8.0 * uniform();
        for (int c = 0; c < n; ++c) p[(5 + c) * N + i] = uniform();
    }
    const int T = orc_num_tiles(H, W, th, tw);
    CHECK(T == 9);
    int32_t tiles[9];
    for (int t = 0; t < T; ++t) tiles[t] = t;
    int64_t counts[9];
    CHECK(orc_tile_lists(p, N, n, H, W, th, tw, tiles, T, counts, NULL, 0) == 0);
    int64_t total = 0;
    for (int t = 0; t < T; ++t) total += counts[t];
    int32_t *lists = malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    CHECK(orc_tile_lists(p, N, n, H, W, th, tw, tiles, T, counts, lists, total) == 0);
    CHECK(orc_tile_lists(p, N, n, H, W, th, tw, tiles, T, counts, lists, total - 1) != 0);
    for (int K = 1; K <= 12; K += 11) {
        double *img = calloc((size_t)T * n * th * tw, sizeof(double));
        int32_t *topk = calloc((size_t)T * th * tw * K, sizeof(int32_t));
        double *qsel = calloc((size_t)T * th * tw * (K + 1), sizeof(double));
        double *margin = calloc((size_t)T * th * tw, sizeof(double));
        double *g = malloc(sizeof(double) * n * H * W);
        for (int e = 0; e < n * H * W; ++e) g[e] = uniform() - 0.5;
        double *grad = calloc((size_t)(5 + n) * N, sizeof(double));
        double *gabs = calloc((size_t)(5 + n) * N, sizeof(double));
        CHECK(orc_render_tiles(p, N, n, H, W, K, th, tw, tiles, T, img, topk, qsel, g, grad, gabs,
                               2, 16.0 * 5.9604644775390625e-8, margin) == 0);
        for (int e = 0; e < (5 + n) * N; ++e) CHECK(isfinite(grad[e]) && gabs[e] >= 0.0);
        double *dense = calloc((size_t)n * H * W, sizeof(double));
        CHECK(orc_render_dense(p, N, n, H, W, K, th, tw, dense, 2) == 0);
        free(img); free(topk); free(qsel); free(margin); free(g); free(grad); free(gabs);
        free(dense);
    }
    int32_t idx[60];
    double q[60], mb[60];
    const int m = orc_rank_pixel(p, N, n, H, W, th, tw, 20, 30, idx, q, mb, 60);
    CHECK(m >= 0 && m <= N);
    for (int a = 1; a < m; ++a) CHECK(q[a - 1] <= q[a]);
    double out[3];
    CHECK(orc_blend_set(p, N, n, 20, 30, idx, m < 5 ? m : 5, out) == 0);
    /* invalid arguments are rejected before any access */
    CHECK(orc_num_tiles(0, W, th, tw) < 0);
    int32_t bad_tile = T;
    CHECK(orc_tile_lists(p, N, n, H, W, th, tw, &bad_tile, 1, counts, NULL, 0) != 0);
    CHECK(orc_render_tiles(p, N, n, H, W, 0, th, tw, tiles, T, NULL, NULL, NULL, NULL, NULL, NULL,
                           1, 0.0, NULL) != 0);
    CHECK(orc_rank_pixel(p, N, n, H, W, th, tw, H, 0, idx, q, mb, 60) < 0);
    int32_t bad_id = N;
    CHECK(orc_blend_set(p, N, n, 0, 0, &bad_id, 1, out) != 0);
    free(lists);
    free(p);
    printf("oracle driver ok\n");
    return 0;
}
