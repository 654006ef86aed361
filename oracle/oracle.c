/*
 * FP64 CPU oracle for the Image-GS tile-based top-K renderer and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link, load or call this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code with the HIP implementation.
 *
 * What it computes (paper: "Image-GS", Sec. 3.1-3.3):
 *   - Gaussian value G_i(x) = exp(-q_i(x)/2), q_i(x) = (x-mu_i)^T Sigma_i^{-1} (x-mu_i)     (Eq. 1)
 *   - Sigma_i = R(theta_i) S_i S_i^T R(theta_i)^T, S_i = diag(s_1, s_2)                     (Eq. 2)
 *     so q = e1^2/s1^2 + e2^2/s2^2 with e = R^T (x - mu).
 *   - parameter vector p_i = (mu_x, mu_y, theta, s_1, s_2, c_0..c_{n-1})                    (Eq. 3)
 *   - tiles of tile_w x tile_h pixels; S_j = Gaussians whose 3-sigma enclosing circle
 *     (radius 3*max(s1,s2)) meets tile j; per pixel the top K of S_j by value; normalized
 *     blend over those K                                                                   (Sec. 3.2, Eq. 5)
 *   - gradients flow only through the K retained Gaussians; the selection itself is held
 *     constant                                                                              (Sec. 3.3)
 *
 * Readings where the paper is silent (each is listed with its reason in the design notes):
 *   - pixel (h, w) has centre (w + 1/2, h + 1/2); the image spans [0,W] x [0,H] in pixels;
 *   - tile j covers the closed rectangle [x0, min(x0+tile_w, W)] x [y0, min(y0+tile_h, H)];
 *     the circle test is  dx = mu_x - clamp(mu_x, x0, x1), dy likewise,
 *     (dx*dx + dy*dy) <= (3*max(s1,s2))^2, evaluated in double with each product and sum rounded
 *     separately (this file must be compiled with -ffp-contract=off), tangency counts;
 *   - ranking by q ascending (= G descending), equal q broken by the lower Gaussian index;
 *   - fewer than K candidates: all of S_j are kept; empty S_j: the pixel is 0 and gets no gradient;
 *   - the blend uses w_i = exp(-(q_i - q_min)/2), an exact identity of Eq. 5 that avoids underflow;
 *     no epsilon is added to the denominator.
 *
 * Everything is evaluated by brute force: S_j is built by testing every Gaussian against the
 * tile, and every member of S_j is evaluated and ranked at every pixel of the tile.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Row r of the [5+n][N] parameter array. */
#define P(params, N, r, i) ((params)[(size_t)(r) * (size_t)(N) + (size_t)(i)])

typedef struct {
    double q;
    double mb; /* rounding scale of q, see rank_scale */
    int32_t idx;
} cand_t;

static int cand_cmp(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->q < y->q) return -1;
    if (x->q > y->q) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Tile rectangle of tile t (row-major tile numbering, tiles_x = ceil(W / tw)). */
static void tile_rect(int t, int H, int W, int th, int tw, int *x0, int *x1, int *y0, int *y1) {
    int tiles_x = (W + tw - 1) / tw;
    int tx = t % tiles_x, ty = t / tiles_x;
    *x0 = tx * tw;
    *y0 = ty * th;
    *x1 = (*x0 + tw < W) ? *x0 + tw : W;
    *y1 = (*y0 + th < H) ? *y0 + th : H;
}

/* Sec. 3.2: does the enclosing circle of Gaussian i's 3-sigma ellipse meet the rectangle? */
static int circle_meets_rect(double mx, double my, double s1, double s2,
                             double x0, double x1, double y0, double y1) {
    double r = 3.0 * (s1 > s2 ? s1 : s2);
    double dx = mx - clampd(mx, x0, x1);
    double dy = my - clampd(my, y0, y1);
    double d2 = dx * dx + dy * dy;
    double r2 = r * r;
    return d2 <= r2;
}

/* Eq. 1-2: Mahalanobis form q and the rotated offsets e1, e2 at pixel centre (px, py). */
static double quad_form(double mx, double my, double th, double s1, double s2, double px, double py,
                        double *e1_out, double *e2_out) {
    double c = cos(th), s = sin(th);
    double dx = px - mx, dy = py - my;
    double e1 = c * dx + s * dy;
    double e2 = -s * dx + c * dy;
    if (e1_out) *e1_out = e1;
    if (e2_out) *e2_out = e2;
    return e1 * e1 / (s1 * s1) + e2 * e2 / (s2 * s2);
}

/*
 * Scale of the rounding error of q when it is evaluated in a narrower format as |e|^2 with
 * e = (cos dx + sin dy, -sin dx + cos dy) / s: the same squares taken over the magnitudes of the
 * products before they cancel, M = (|cos dx| + |sin dy|)^2 / s1^2 + (|sin dx| + |cos dy|)^2 / s2^2
 * (M >= q).  Each product, sum and input rounding perturbs e_a by a few units of the last place of
 * |cos dx| + |sin dy| (resp. |sin dx| + |cos dy|), so such an evaluation of q is accurate to a small
 * multiple of the unit roundoff times M; the tests use it to tell a selection that a float32
 * ranking decides for certain from a near tie, where either answer is correct (Sec. 3.2 ranks by
 * value; which of two nearly equal values is larger is then a rounding matter).
 */
static double rank_scale(double th, double s1, double s2, double px, double py, double mx,
                         double my) {
    double c = cos(th), s = sin(th);
    double dx = px - mx, dy = py - my;
    double a = fabs(c * dx) + fabs(s * dy);
    double b = fabs(s * dx) + fabs(c * dy);
    return a * a / (s1 * s1) + b * b / (s2 * s2);
}

int orc_num_tiles(int H, int W, int th, int tw) {
    if (H < 1 || W < 1 || th < 1 || tw < 1) return ORC_EINVAL;
    return ((H + th - 1) / th) * ((W + tw - 1) / tw);
}

/*
 * Tile hit sets S_j (Sec. 3.2) for the listed tiles.  counts[t] = |S_{tiles[t]}|.  If lists is not
 * NULL the members of each listed tile are written consecutively in ascending Gaussian index,
 * provided the total fits lists_cap (else ORC_ENOMEM and only counts are valid).
 */
int orc_tile_lists(const double *params, int N, int n, int H, int W, int th, int tw,
                   const int32_t *tiles, int ntiles, int64_t *counts, int32_t *lists, int64_t lists_cap) {
    (void)n;
    if (N < 0 || H < 1 || W < 1 || th < 1 || tw < 1 || ntiles < 0) return ORC_EINVAL;
    int T = orc_num_tiles(H, W, th, tw);
    for (int t = 0; t < ntiles; ++t)
        if (tiles[t] < 0 || tiles[t] >= T) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < ntiles; ++t) {
        int x0, x1, y0, y1;
        tile_rect(tiles[t], H, W, th, tw, &x0, &x1, &y0, &y1);
        int64_t c = 0;
        for (int i = 0; i < N; ++i)
            c += circle_meets_rect(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 3, i),
                                   P(params, N, 4, i), x0, x1, y0, y1);
        counts[t] = c;
    }
    if (!lists) return ORC_OK;
    int64_t total = 0;
    for (int t = 0; t < ntiles; ++t) total += counts[t];
    if (total > lists_cap) return ORC_ENOMEM;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntiles + 1));
    if (!start) return ORC_ENOMEM;
    start[0] = 0;
    for (int t = 0; t < ntiles; ++t) start[t + 1] = start[t] + counts[t];
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < ntiles; ++t) {
        int x0, x1, y0, y1;
        tile_rect(tiles[t], H, W, th, tw, &x0, &x1, &y0, &y1);
        int64_t o = start[t];
        for (int i = 0; i < N; ++i)
            if (circle_meets_rect(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 3, i),
                                  P(params, N, 4, i), x0, x1, y0, y1))
                lists[o++] = i;
    }
    free(start);
    return ORC_OK;
}

/*
 * Render (Eq. 5) the listed tiles and optionally accumulate the adjoint.
 *
 * Outputs are compact per listed tile, pixel p = ly*tw + lx within the tile:
 *   img   [ntiles][n][th*tw]   rendered colour (0 for pixels outside the image or with empty S_j)
 *   topk  [ntiles][th*tw][K]   Gaussian indices of S_j^K(x) in rank order, -1 where unused
 *   qsel  [ntiles][th*tw][K+1] q of the ranked candidates 1..K+1 (+inf where absent); the gap
 *                              q_(K+1) - q_(K) measures how close the selection is to a tie
 *   margin [ntiles][th*tw]     with gamma: min over the members j left out of
 *                              (q_j - gamma M_j) minus max over the retained i of
 *                              (q_i + gamma M_i) (M: rank_scale); +inf when every member is kept.
 *                              If each member's q is known only to within gamma M, a positive
 *                              margin means the retained set is still determined
 * Adjoint (Sec. 3.3): with g = grad_img[:, h, w] (full-size planar [n][H][W]) the contributions of
 * the listed tiles' pixels are added into grad_params [5+n][N] (caller zeroes it).  Gradients are
 * taken with S_j and S_j^K(x) held fixed.
 * grad_abs [5+n][N] (optional, caller zeroes it) receives the conditioning of each gradient sum:
 * the sum over pixels of the magnitudes of the terms before they cancel, i.e. |alpha g_c| for a
 * colour and (1/2) alpha (|g.c_i| + |g.c_r|) |dq/dp| for a geometry parameter.  A float32
 * evaluation of the same sums is accurate to a small multiple of eps32 times this value.
 * Any output pointer may be NULL.  nthreads <= 0 uses the OpenMP default.
 */
int orc_render_tiles(const double *params, int N, int n, int H, int W, int K, int th, int tw,
                     const int32_t *tiles, int ntiles, double *img, int32_t *topk, double *qsel,
                     const double *grad_img, double *grad_params, double *grad_abs, int nthreads,
                     double gamma, double *margin) {
    if (N < 0 || n < 1 || H < 1 || W < 1 || K < 1 || th < 1 || tw < 1 || ntiles < 0) return ORC_EINVAL;
    int T = orc_num_tiles(H, W, th, tw);
    for (int t = 0; t < ntiles; ++t)
        if (tiles[t] < 0 || tiles[t] >= T) return ORC_EINVAL;
    const int tp = th * tw;
    const int R = 5 + n;
    int do_grad = (grad_img != NULL && grad_params != NULL);
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif

#pragma omp parallel num_threads(nthreads)
    {
        int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
        cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
        double *gloc = NULL, *aloc = NULL;
        if (do_grad) gloc = (double *)calloc((size_t)R * (size_t)(N > 0 ? N : 1), sizeof(double));
        if (do_grad && grad_abs) aloc = (double *)calloc((size_t)R * (size_t)(N > 0 ? N : 1), sizeof(double));
        double *cr = (double *)malloc(sizeof(double) * (size_t)n);
        double *wts = (double *)malloc(sizeof(double) * (size_t)K);
        int ok = members && cand && cr && wts && (!do_grad || gloc) && (!(do_grad && grad_abs) || aloc);
        if (!ok) {
#pragma omp atomic write
            status = ORC_ENOMEM;
        }

#pragma omp for schedule(dynamic)
        for (int t = 0; t < ntiles; ++t) {
            if (!ok) continue;
            int x0, x1, y0, y1;
            tile_rect(tiles[t], H, W, th, tw, &x0, &x1, &y0, &y1);
            /* S_j by testing every Gaussian (Sec. 3.2), kept in ascending index */
            int m = 0;
            for (int i = 0; i < N; ++i)
                if (circle_meets_rect(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 3, i),
                                      P(params, N, 4, i), x0, x1, y0, y1))
                    members[m++] = i;
            for (int p = 0; p < tp; ++p) {
                int lx = p % tw, ly = p / tw;
                int w = x0 + lx, h = y0 + ly;
                int inside = (w < x1) && (h < y1);
                if (img)
                    for (int ch = 0; ch < n; ++ch) img[((size_t)t * n + ch) * tp + p] = 0.0;
                if (topk)
                    for (int k = 0; k < K; ++k) topk[((size_t)t * tp + p) * K + k] = -1;
                if (qsel)
                    for (int k = 0; k <= K; ++k) qsel[((size_t)t * tp + p) * (K + 1) + k] = INFINITY;
                if (margin) margin[(size_t)t * tp + p] = INFINITY;
                if (!inside || m == 0) continue;
                double px = w + 0.5, py = h + 0.5;
                /* rank every member of S_j at this pixel by (q, index) and keep the first K */
                for (int a = 0; a < m; ++a) {
                    int i = members[a];
                    cand[a].q = quad_form(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 2, i),
                                          P(params, N, 3, i), P(params, N, 4, i), px, py, NULL, NULL);
                    cand[a].idx = i;
                    cand[a].mb = margin ? rank_scale(P(params, N, 2, i), P(params, N, 3, i),
                                                     P(params, N, 4, i), px, py, P(params, N, 0, i),
                                                     P(params, N, 1, i))
                                        : 0.0;
                }
                qsort(cand, (size_t)m, sizeof(cand_t), cand_cmp);
                int keff = m < K ? m : K;
                if (margin && m > K) {
                    double hi_in = -INFINITY, lo_out = INFINITY;
                    for (int a = 0; a < m; ++a) {
                        if (a < keff) {
                            double v = cand[a].q + gamma * cand[a].mb;
                            if (v > hi_in) hi_in = v;
                        } else {
                            double v = cand[a].q - gamma * cand[a].mb;
                            if (v < lo_out) lo_out = v;
                        }
                    }
                    margin[(size_t)t * tp + p] = lo_out - hi_in;
                }
                if (topk)
                    for (int k = 0; k < keff; ++k) topk[((size_t)t * tp + p) * K + k] = cand[k].idx;
                if (qsel)
                    for (int k = 0; k <= K && k < m; ++k) qsel[((size_t)t * tp + p) * (K + 1) + k] = cand[k].q;
                /* Eq. 5: normalized blend over the retained K */
                double qmin = cand[0].q, Z = 0.0;
                for (int ch = 0; ch < n; ++ch) cr[ch] = 0.0;
                for (int k = 0; k < keff; ++k) {
                    wts[k] = exp(-0.5 * (cand[k].q - qmin));
                    Z += wts[k];
                    for (int ch = 0; ch < n; ++ch) cr[ch] += wts[k] * P(params, N, 5 + ch, cand[k].idx);
                }
                for (int ch = 0; ch < n; ++ch) cr[ch] /= Z;
                if (img)
                    for (int ch = 0; ch < n; ++ch) img[((size_t)t * n + ch) * tp + p] = cr[ch];
                if (!do_grad) continue;
                /* adjoint of Eq. 5 through the retained K (Sec. 3.3) */
                for (int k = 0; k < keff; ++k) {
                    int i = cand[k].idx;
                    double alpha = wts[k] / Z;
                    double dot = 0.0, gci = 0.0, gcr = 0.0;
                    for (int ch = 0; ch < n; ++ch) {
                        double g = grad_img[((size_t)ch * H + h) * W + w];
                        gloc[(size_t)(5 + ch) * N + i] += alpha * g;
                        dot += g * (P(params, N, 5 + ch, i) - cr[ch]);
                        gci += g * P(params, N, 5 + ch, i);
                        gcr += g * cr[ch];
                        if (aloc) aloc[(size_t)(5 + ch) * N + i] += fabs(alpha * g);
                    }
                    double dLdq = -0.5 * alpha * dot;
                    double dmag = 0.5 * alpha * (fabs(gci) + fabs(gcr));
                    double mx = P(params, N, 0, i), my = P(params, N, 1, i), thv = P(params, N, 2, i);
                    double s1 = P(params, N, 3, i), s2 = P(params, N, 4, i);
                    double e1, e2;
                    quad_form(mx, my, thv, s1, s2, px, py, &e1, &e2);
                    double c = cos(thv), s = sin(thv);
                    double i1 = 1.0 / (s1 * s1), i2 = 1.0 / (s2 * s2);
                    double dq_dmx = -2.0 * c * e1 * i1 + 2.0 * s * e2 * i2;
                    double dq_dmy = -2.0 * s * e1 * i1 - 2.0 * c * e2 * i2;
                    double dq_dth = 2.0 * e1 * e2 * (i1 - i2);
                    double dq_ds1 = -2.0 * e1 * e1 * i1 / s1;
                    double dq_ds2 = -2.0 * e2 * e2 * i2 / s2;
                    gloc[(size_t)0 * N + i] += dLdq * dq_dmx;
                    gloc[(size_t)1 * N + i] += dLdq * dq_dmy;
                    gloc[(size_t)2 * N + i] += dLdq * dq_dth;
                    gloc[(size_t)3 * N + i] += dLdq * dq_ds1;
                    gloc[(size_t)4 * N + i] += dLdq * dq_ds2;
                    if (aloc) {
                        aloc[(size_t)0 * N + i] += dmag * fabs(dq_dmx);
                        aloc[(size_t)1 * N + i] += dmag * fabs(dq_dmy);
                        aloc[(size_t)2 * N + i] += dmag * fabs(dq_dth);
                        aloc[(size_t)3 * N + i] += dmag * fabs(dq_ds1);
                        aloc[(size_t)4 * N + i] += dmag * fabs(dq_ds2);
                    }
                }
            }
        }
        if (do_grad && ok) {
#pragma omp critical
            {
                for (size_t e = 0; e < (size_t)R * (size_t)N; ++e) grad_params[e] += gloc[e];
                if (aloc)
                    for (size_t e = 0; e < (size_t)R * (size_t)N; ++e) grad_abs[e] += aloc[e];
            }
        }
        free(members);
        free(cand);
        free(gloc);
        free(aloc);
        free(cr);
        free(wts);
    }
    return status;
}

/*
 * Same definition, evaluated the dense way of Eq. 4-5: at every pixel every one of the N Gaussians
 * is evaluated, non-members of the pixel's S_j are then discarded, and the survivors are ranked.
 * Produces the image only ([n][H][W]).  Used as the "dense" timing mode and as a cross-check.
 */
int orc_render_dense(const double *params, int N, int n, int H, int W, int K, int th, int tw,
                     double *img, int nthreads) {
    if (N < 0 || n < 1 || H < 1 || W < 1 || K < 1 || th < 1 || tw < 1) return ORC_EINVAL;
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    const int tiles_x = (W + tw - 1) / tw;
#pragma omp parallel num_threads(nthreads)
    {
        cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
        if (!cand) {
#pragma omp atomic write
            status = ORC_ENOMEM;
        }
#pragma omp for schedule(dynamic)
        for (int h = 0; h < H; ++h) {
            if (!cand) continue;
            for (int w = 0; w < W; ++w) {
                int t = (h / th) * tiles_x + (w / tw);
                int x0, x1, y0, y1;
                tile_rect(t, H, W, th, tw, &x0, &x1, &y0, &y1);
                double px = w + 0.5, py = h + 0.5;
                int m = 0;
                for (int i = 0; i < N; ++i) {
                    double q = quad_form(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 2, i),
                                         P(params, N, 3, i), P(params, N, 4, i), px, py, NULL, NULL);
                    if (circle_meets_rect(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 3, i),
                                          P(params, N, 4, i), x0, x1, y0, y1)) {
                        cand[m].q = q;
                        cand[m].idx = i;
                        ++m;
                    }
                }
                for (int ch = 0; ch < n; ++ch) img[((size_t)ch * H + h) * W + w] = 0.0;
                if (m == 0) continue;
                qsort(cand, (size_t)m, sizeof(cand_t), cand_cmp);
                int keff = m < K ? m : K;
                double qmin = cand[0].q, Z = 0.0;
                for (int k = 0; k < keff; ++k) Z += exp(-0.5 * (cand[k].q - qmin));
                for (int ch = 0; ch < n; ++ch) {
                    double acc = 0.0;
                    for (int k = 0; k < keff; ++k)
                        acc += exp(-0.5 * (cand[k].q - qmin)) * P(params, N, 5 + ch, cand[k].idx);
                    img[((size_t)ch * H + h) * W + w] = acc / Z;
                }
            }
        }
        free(cand);
    }
    return status;
}

/*
 * Every member of the hit set S_j of the tile holding pixel (h, w), ranked at the pixel centre by
 * (q, index) as in orc_render_tiles: idx, q and M (rank_scale) of each, in rank order.  Returns
 * |S_j| (only the first cap entries are written) or a negative error.
 */
int orc_rank_pixel(const double *params, int N, int n, int H, int W, int th, int tw, int h, int w,
                   int32_t *idx, double *q, double *mb, int cap) {
    (void)n;
    if (N < 0 || H < 1 || W < 1 || th < 1 || tw < 1 || h < 0 || h >= H || w < 0 || w >= W ||
        cap < 0)
        return ORC_EINVAL;
    int tiles_x = (W + tw - 1) / tw;
    int x0, x1, y0, y1;
    tile_rect((h / th) * tiles_x + w / tw, H, W, th, tw, &x0, &x1, &y0, &y1);
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
    if (!cand) return ORC_ENOMEM;
    double px = w + 0.5, py = h + 0.5;
    int m = 0;
    for (int i = 0; i < N; ++i) {
        double mx = P(params, N, 0, i), my = P(params, N, 1, i), thv = P(params, N, 2, i);
        double s1 = P(params, N, 3, i), s2 = P(params, N, 4, i);
        if (!circle_meets_rect(mx, my, s1, s2, x0, x1, y0, y1)) continue;
        cand[m].q = quad_form(mx, my, thv, s1, s2, px, py, NULL, NULL);
        cand[m].mb = rank_scale(thv, s1, s2, px, py, mx, my);
        cand[m].idx = i;
        ++m;
    }
    qsort(cand, (size_t)m, sizeof(cand_t), cand_cmp);
    for (int a = 0; a < m && a < cap; ++a) {
        idx[a] = cand[a].idx;
        q[a] = cand[a].q;
        mb[a] = cand[a].mb;
    }
    free(cand);
    return m;
}

/*
 * Eq. 5 over a given set of Gaussians at the pixel centre (w + 1/2, h + 1/2): the normalized blend
 * sum_k exp(-(q_k - q_min)/2) c_k / sum_k exp(-(q_k - q_min)/2) into out[n] (0 for an empty set).
 */
int orc_blend_set(const double *params, int N, int n, int h, int w, const int32_t *ids, int k,
                  double *out) {
    if (N < 0 || n < 1 || k < 0) return ORC_EINVAL;
    for (int a = 0; a < k; ++a)
        if (ids[a] < 0 || ids[a] >= N) return ORC_EINVAL;
    for (int ch = 0; ch < n; ++ch) out[ch] = 0.0;
    if (k == 0) return ORC_OK;
    double px = w + 0.5, py = h + 0.5, qmin = INFINITY;
    double *qs = (double *)malloc(sizeof(double) * (size_t)k);
    if (!qs) return ORC_ENOMEM;
    for (int a = 0; a < k; ++a) {
        int i = ids[a];
        qs[a] = quad_form(P(params, N, 0, i), P(params, N, 1, i), P(params, N, 2, i),
                          P(params, N, 3, i), P(params, N, 4, i), px, py, NULL, NULL);
        if (qs[a] < qmin) qmin = qs[a];
    }
    double Z = 0.0;
    for (int a = 0; a < k; ++a) {
        double wt = exp(-0.5 * (qs[a] - qmin));
        Z += wt;
        for (int ch = 0; ch < n; ++ch) out[ch] += wt * P(params, N, 5 + ch, ids[a]);
    }
    for (int ch = 0; ch < n; ++ch) out[ch] /= Z;
    free(qs);
    return ORC_OK;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
