/*
 * imagegs.h - C ABI of libimagegs.so, the gfx950 (MI355X) implementation of the Image-GS
 * differentiable renderer (anisotropic coloured 2D Gaussians, tile-based top-K normalized blend)
 * and its adjoint.
 *
 * Paper: "Image-GS: Content-Adaptive Image Representation via 2D Gaussians", arXiv 2407.01866.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every buffer argument is a DEVICE pointer owned by the caller.  The library never allocates
 *    or frees device memory and never synchronizes: all work is enqueued on `stream`
 *    (a hipStream_t passed as void*; NULL = the default stream), so results are ready only once
 *    the caller synchronizes that stream.
 *  - Argument checks are synchronous and return an igs_status; nothing throws across the ABI.
 *  - Data-dependent failures (too many tile/Gaussian pairs for `pair_capacity`, a tile list too
 *    long for 16-bit slots) are detected on the device and reported in the status block, an
 *    int64_t[8] array at byte offset 0 of `saved` (or of `workspace` when `saved` is NULL):
 *        status[0]  P, the number of (tile, Gaussian) pairs the render required
 *        status[1]  1 if P exceeded pair_capacity: nothing past the capacity was written, the
 *                   image is NOT valid and the caller must retry with pair_capacity >= P
 *        status[2]  the largest tile hit-set size |S_j|
 *        status[3]  1 if some |S_j| exceeded 65535: the image is valid but the saved top-K slots
 *                   are not, so igs_render_backward must not be called on this state
 *        status[4]  E_fwd = sum over tiles of |S_j| times the tile's pixel count: the (pixel,
 *                   candidate) evaluations the render performed
 *        status[5]  E_bwd = sum over pixels of the number of retained Gaussians, min(K, |S_j|)
 *        status[6]  1 if a gradient derived from this render must not be applied: status[1] is
 *                   set, or the call saved 16-bit top-K slots for a separate adjoint (igs_render
 *                   with `saved`, igs_render_l1 and their batched forms) and status[3] is set.
 *                   igs_render_l1_grad keeps its slots on chip at full width, so a long hit set
 *                   does not set it there.  Meant as the skip_flag of igs_adam_step.
 *    The caller reads it asynchronously (e.g. a copy to pinned memory) before trusting outputs.
 *  - Parameters are float32 structure-of-arrays [5+n][N] (Eq. 3: p_i = (mu, theta, s, c)),
 *    rows in this order:
 *        0 mu_x, 1 mu_y   mean in pixel units; the image spans [0,W] x [0,H] and pixel (h, w)
 *                         has its centre at (w + 1/2, h + 1/2)
 *        2 theta          rotation angle in radians (any value; Sigma is pi-periodic)
 *        3 s_1, 4 s_2     scales in pixels, > 0 (Eq. 2: Sigma = R(theta) S S^T R(theta)^T)
 *        5 .. 4+n         colour c in R^n
 *    Non-finite or non-positive scales give unspecified pixel values but never unsafe memory
 *    access; a Gaussian whose mean or scale is not finite hits no tile.
 *  - Images (render output, targets, image gradients) are float32 planar [n][H][W].
 *  - Only 16 x 16 tiles (the paper's tile size, Sec. 4.1) are supported: tile_h = tile_w = 16.
 */
#ifndef IMAGEGS_H
#define IMAGEGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t igs_status;

#define IGS_OK 0
#define IGS_ERR_INVALID_ARG (-1) /* a size, pointer or hyper-parameter is out of range          */
#define IGS_ERR_WORKSPACE (-2)   /* workspace / saved buffer smaller than the size query said    */
#define IGS_ERR_HIP (-3)         /* a HIP runtime call or kernel launch failed                   */
#define IGS_ERR_UNSUPPORTED (-4) /* valid request this build does not implement (e.g. tile 8x8) */

#define IGS_MAX_K 32          /* largest top-K                                                  */
#define IGS_MAX_CHANNELS 32   /* largest colour dimension n                                     */
#define IGS_TILE 16           /* tile side in pixels                                            */
#define IGS_STATUS_WORDS 8    /* int64 words of the device status block                        */

/* ABI revision; bumped on any incompatible change. */
int32_t igs_abi_version(void);

/* Human-readable name of a status code (static storage). */
const char *igs_status_string(igs_status s);

/* Bounds-checked build only (libimagegs_debug.so, the same sources compiled with
 * IGS_BOUNDS_CHECK): in that build the kernels validate their indices into the LDS batches
 * (forward staging, retained slots, the adjoint's counters, items and chunks) and into the pair
 * arrays (emission, sort scatter, sorted emit indices) against the buffer sizes; an index out of
 * range sets the bit of its site and is replaced by 0, so no access leaves its buffer.  Writes
 * to *out the OR of the sites met since the previous call and clears them (synchronizes the
 * device); 0 means no violation.  The normal build has no checks: *out = 0 and the call returns
 * IGS_ERR_UNSUPPORTED.  Errors: IGS_ERR_INVALID_ARG (out NULL), IGS_ERR_HIP. */
igs_status igs_bounds_violations(uint32_t *out);

/*
 * Buffer sizes for igs_render / igs_render_backward with these dimensions.
 *   pair_capacity: how many (tile, Gaussian) pairs the binning may hold (>= 1, < 2^31).  P, the
 *                  number needed, is data dependent (Sec. 3.2: one pair per tile a Gaussian's
 *                  3-sigma circle meets); the status block reports it.
 *   *saved_bytes:  state the forward leaves for the adjoint (status, tile ranges, sorted hit
 *                  lists, per-Gaussian geometry, per-pixel top-K slots and blend normalizers).
 *   *ws_bytes:     scratch needed by either call when `saved` is given; a forward without saved
 *                  state needs ws_bytes + saved_bytes of workspace.
 * Errors: IGS_ERR_INVALID_ARG (N < 0, n or K or H or W out of range, NULL out pointers),
 *         IGS_ERR_UNSUPPORTED (tile size other than 16 x 16).
 */
igs_status igs_render_buffer_sizes(int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                                   int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                                   size_t *ws_bytes, size_t *saved_bytes);

/*
 * Byte offsets of the parts of the saved state, for inspection (e.g. to compare the tile hit sets
 * and top-K selection with a reference).  out[0] status block; out[1] tile ranges, int32[T][2]
 * (start, end) into the sorted list, tiles numbered row-major, T = ceil(H/16) * ceil(W/16);
 * out[2] sorted Gaussian indices uint32[pair_capacity]: S_j is entries start..end-1 of tile j, in
 * ascending index; out[3] top-K slots uint16[K][H][W], the rank-ordered positions of the retained
 * Gaussians within their tile's S_j (0xFFFF = unused); out[4] per-pixel float32[H][W][2]
 * (blend shift, 1/sum of weights); out[5] total bytes.
 * Errors: as igs_render_buffer_sizes.
 */
igs_status igs_saved_offsets(int32_t N, int32_t n, int32_t H, int32_t W, int32_t K, int32_t tile_h,
                             int32_t tile_w, int64_t pair_capacity, int64_t out[6]);

/*
 * Forward render, Sec. 3.2 / Eq. 5.  For each Gaussian: the radius r = 3 max(s_1, s_2) of the
 * circle enclosing its 3-sigma ellipse; tile hit sets S_j = Gaussians whose circle meets the
 * closed tile rectangle (clipped to the image), ordered by ascending Gaussian index; for every
 * pixel x of tile j the K members of S_j with the largest G_i(x) (smallest Mahalanobis form q,
 * equal q broken by the lower index); and c_r(x) = sum_K G_i c_i / sum_K G_i.  Pixels whose tile
 * has an empty S_j are 0.
 *   params   [5+n][N] float32 (see the conventions above), N >= 0 (N = 0 renders zeros)
 *   image    [n][H][W] float32 output, fully overwritten
 *   saved    NULL for inference only, else saved_bytes of state kept for igs_render_backward
 *   workspace / ws_bytes: scratch of at least the queried ws_bytes (+ saved_bytes if saved is
 *            NULL); 256-byte aligned pointers are required for saved and workspace.
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_UNSUPPORTED, IGS_ERR_WORKSPACE, IGS_ERR_HIP.
 */
igs_status igs_render(const float *params, int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                      int32_t tile_h, int32_t tile_w, int64_t pair_capacity, float *image,
                      void *saved, size_t saved_bytes, void *workspace, size_t ws_bytes,
                      void *stream);

/*
 * Adjoint of igs_render (Sec. 3.3): gradients flow through the K retained Gaussians of every
 * pixel while the tile hit sets and the top-K selection saved by the forward are held fixed.
 *   params, N, n, H, W, K, tile sizes, pair_capacity: exactly as passed to the forward
 *   image       the forward's output [n][H][W]
 *   grad_image  dL/dc_r, [n][H][W] float32
 *   saved       the state written by the forward (its status block must show no overflow)
 *   grad_params [5+n][N] float32 output, overwritten (not accumulated): dL/d(mu_x, mu_y, theta,
 *               s_1, s_2, c) in the units of `params`
 *   workspace   scratch of at least ws_bytes
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_UNSUPPORTED, IGS_ERR_WORKSPACE, IGS_ERR_HIP.
 */
igs_status igs_render_backward(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                               int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                               const float *image, const float *grad_image, const void *saved,
                               size_t saved_bytes, float *grad_params, void *workspace,
                               size_t ws_bytes, void *stream);

/*
 * Forward render fused with the L1 term of the fitting loss (Sec. 3.2 / Eq. 5 and Sec. 3.3,
 * Sec. 4.1), for a fitting iteration whose loss is the mean absolute error.  Renders exactly as
 * igs_render, and in the same pass compares every pixel with the target:
 *   target    [n][H][W] float32
 *   image     [n][H][W] float32 output, identical to igs_render's
 *   loss_out  device double[2]: [0] mean |image - target|, [1] mean (image - target)^2 (as
 *             igs_l1_loss_grad; sums are taken per tile, then over tiles in a fixed order)
 *   saved     required: besides igs_render's state it receives, per pixel, the signs of
 *             image - target and g . c_r with g = sign(image - target) / (n*H*W), which is all
 *             igs_render_backward_l1 needs from the loss
 *   workspace / sizes: as igs_render (igs_render_buffer_sizes covers this call)
 * n must be <= 16 (two bits per channel in the per-pixel record).
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_UNSUPPORTED (n > 16 or tile size), IGS_ERR_WORKSPACE,
 *         IGS_ERR_HIP.
 */
igs_status igs_render_l1(const float *params, int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                         int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                         const float *target, float *image, double *loss_out, void *saved,
                         size_t saved_bytes, void *workspace, size_t ws_bytes, void *stream);

/*
 * Adjoint of igs_render_l1 (Sec. 3.3): the gradient of the mean absolute error with respect to
 * the parameters, through the K retained Gaussians, with the selection held fixed.  Gives the
 * same result as igs_l1_loss_grad followed by igs_render_backward, without the gradient image.
 *   saved        the state written by igs_render_l1 (not igs_render) for the same arguments
 *   grad_params  [5+n][N] float32 output, overwritten
 * Errors: as igs_render_l1.
 */
igs_status igs_render_backward_l1(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                                  int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                                  const void *saved, size_t saved_bytes, float *grad_params,
                                  void *workspace, size_t ws_bytes, void *stream);

/*
 * One fitting evaluation of the L1 loss in a single rasterization pass (Sec. 3.2 Eq. 5, Sec. 3.3,
 * loss of Sec. 4.1): binning as igs_render, then one kernel in which each tile's workgroup
 * renders the tile, compares it with the target and runs the adjoint of that comparison, keeping
 * every per-pixel quantity on chip.  The loss and the gradient are bit for bit those of
 * igs_render_l1 followed by igs_render_backward_l1; no image is produced.
 *   target       [n][H][W] float32
 *   loss_out     device double[2]: mean |image - target|, mean (image - target)^2
 *   grad_params  [5+n][N] float32 output, overwritten: dL/dparams of the mean absolute error
 *   saved        required, saved_bytes as igs_render's: receives the binning state and the status
 *                block (on pair-capacity overflow the loss is that of an all-zero image and
 *                grad_params is zero, as in the two-pass path)
 *   workspace / sizes: as igs_render (igs_render_buffer_sizes covers this call)
 * n must be <= 16.
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_UNSUPPORTED (n > 16 or tile size), IGS_ERR_WORKSPACE,
 *         IGS_ERR_HIP.
 */
igs_status igs_render_l1_grad(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                              int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                              const float *target, double *loss_out, float *grad_params,
                              void *saved, size_t saved_bytes, void *workspace, size_t ws_bytes,
                              void *stream);

/*
 * igs_render_l1_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or fitting loops, harnesses that forbid hipMalloc): the same kernels and
 * results, bit for bit, with the workspace taken from a static device array of
 * IGS_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on until the process
 * ends.  The caller still provides every input and output, `saved` included.  No device memory
 * is allocated or freed by the call.
 *   arguments: as igs_render_l1_grad without workspace / ws_bytes
 * The workspace igs_render_buffer_sizes reports for these arguments must fit the array (64 MiB:
 * e.g. a 1024 x 1024 x 3 fit with 20,000 Gaussians and a few hundred thousand pairs); otherwise
 * IGS_ERR_WORKSPACE and nothing is launched.  All calls on one device share its array: calls that
 * overlap on a device (other streams, threads) race and give undefined results; calls in one
 * stream order are safe.  The array keeps the last call's contents; the kernels read nothing from
 * it that the same call did not write.
 * Errors: as igs_render_l1_grad; IGS_ERR_WORKSPACE when the workspace would exceed the array.
 */
#define IGS_NOALLOC_SCRATCH_BYTES (64ull << 20)
igs_status igs_render_l1_grad_noalloc(const float *params, int32_t N, int32_t n, int32_t H,
                                      int32_t W, int32_t K, int32_t tile_h, int32_t tile_w,
                                      int64_t pair_capacity, const float *target, double *loss_out,
                                      float *grad_params, void *saved, size_t saved_bytes,
                                      void *stream);

/*
 * Binning alone (Sec. 3.2): the footprint bound, pair emission, sort and tile ranges of
 * igs_render, written into `saved` without rasterizing, for decoders that answer point queries
 * (igs_query).  Arguments, sizes, status block and errors as igs_render (image not needed).
 */
igs_status igs_bin(const float *params, int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                   int32_t tile_h, int32_t tile_w, int64_t pair_capacity, void *saved,
                   size_t saved_bytes, void *workspace, size_t ws_bytes, void *stream);

/* Scratch bytes igs_query needs for M points and N Gaussians of n channels on an H x W image:
 * the sort of the points by tile, and one packed record per Gaussian (its ranking and blend
 * geometry and colours, 128 bytes for n <= 16), so that a query reads one record per hit-set
 * member instead of gathering from n + 3 arrays.  Errors: IGS_ERR_INVALID_ARG. */
igs_status igs_query_workspace_size(int32_t M, int32_t N, int32_t n, int32_t H, int32_t W,
                                    size_t *ws_bytes);

/*
 * Random access (Sec. 1, Sec. 3.2): the colour of the representation at M arbitrary points of
 * the image plane, each evaluated on its own by Eq. 5: the point (x, y) belongs to tile
 * (floor(x/16), floor(y/16)), every member of that tile's S_j is ranked by q at the point (then
 * by index) and the top K are blended.  The ranking and blend are igs_render's operations, so at
 * a pixel centre (w + 1/2, h + 1/2) the result equals the rendered pixel bit for bit.
 *   params, N, n, H, W, K, tiles, pair_capacity: as the igs_bin or igs_render call that wrote
 *          `saved` (whose status block must report no overflow)
 *   points [M][2] float32 device: (x, y) of each point, in pixels; points outside [0,W) x [0,H)
 *          or not finite give 0
 *   out    [M][n] float32 device output: the n channels of each point together
 *   workspace  NULL: the points are evaluated in input order (right when they are already
 *          grouped by tile, e.g. in scanline order), reading the Gaussians' data where `saved`
 *          and `params` hold it; else device scratch of at least igs_query_workspace_size
 *          bytes, 256-byte aligned, used to sort the points by tile first (a stable sort, so
 *          results do not depend on it) so that neighbouring lanes share a hit set, and to pack
 *          each Gaussian's data into one record (the results are the same either way)
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_UNSUPPORTED (tile size), IGS_ERR_WORKSPACE (saved or
 * workspace too small or misaligned), IGS_ERR_HIP.
 */
igs_status igs_query(const float *params, int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                     int32_t tile_h, int32_t tile_w, int64_t pair_capacity, const void *saved,
                     size_t saved_bytes, const float *points, int32_t M, float *out,
                     void *workspace, size_t ws_bytes, void *stream);

/*
 * Float16 storage (Sec. 4.1: the trained attributes are quantized to float16): every value of
 * a [5+n][N] float32 array (normally the fitter's parameters: normalized mean, rotation, inverse
 * scales, colour) rounded to IEEE binary16, nearest with ties to even, as uint16 bit patterns.
 */
igs_status igs_params_to_fp16(const float *params, int32_t N, int32_t n, uint16_t *out,
                              void *stream);

/*
 * Decoding of stored float16 fitter parameters [5+n][N_stored] into igs_render's float32 units
 * for the first N_prefix Gaussians (a level of detail: the error-guided schedule appends
 * Gaussians, so each of its stages is a prefix): mean x W and x H, rotation, scale =
 * 1 / inverse scale, colour.  render_params is [5+n][N_prefix].
 * Errors: IGS_ERR_INVALID_ARG (N_prefix > N_stored, shapes), IGS_ERR_HIP.
 */
igs_status igs_decode_fp16(const uint16_t *stored, int32_t N_stored, int32_t n, int32_t N_prefix,
                           int32_t H, int32_t W, float *render_params, void *stream);

/* Scratch bytes igs_l1_loss_grad needs for an image of count = n*H*W values. */
igs_status igs_l1_workspace_size(int64_t count, size_t *ws_bytes);

/*
 * L1 term of the fitting loss (Sec. 3.3, Sec. 4.1), taken as the mean over all n*H*W values:
 *   grad_image = sign(image - target) / (n*H*W)  (sign(0) = 0), [n][H][W] float32
 *   loss_out   device double[2]: [0] mean |image - target|, [1] mean (image - target)^2 (for PSNR)
 * Reductions are deterministic (fixed order).  Errors: IGS_ERR_INVALID_ARG, IGS_ERR_WORKSPACE,
 * IGS_ERR_HIP.
 */
igs_status igs_l1_loss_grad(const float *image, const float *target, int32_t n, int32_t H,
                            int32_t W, float *grad_image, double *loss_out, void *workspace,
                            size_t ws_bytes, void *stream);

/* Scratch bytes igs_l1_ssim_loss_grad needs for an [n][H][W] image. */
igs_status igs_l1_ssim_workspace_size(int32_t n, int32_t H, int32_t W, size_t *ws_bytes);

/*
 * The paper's fitting loss with its SSIM term (Sec. 3.3, Sec. 4.1: L1 + 0.1 L_SSIM), taken as
 *   L = mean|image - target| + ssim_weight * (1 - SSIM)
 * where SSIM is the mean, over all n*H*W positions (every channel on its own), of the
 * structural-similarity map of Wang et al. with an 11 x 11 Gaussian window (sigma 1.5, weights
 * summing to 1), the images extended by zeros outside [0,H) x [0,W) (one map value per pixel),
 * C1 = 0.01^2 and C2 = 0.03^2 (values in [0, 1] units).  Local means and second moments are
 * accumulated in fp64.
 *   image, target  [n][H][W] float32 device
 *   ssim_weight    weight of 1 - SSIM (the paper uses 0.1), finite and >= 0
 *   grad_image     [n][H][W] float32 device output: dL/d(image), overwritten
 *   loss_out       device double[4] output: L, mean |image - target|, mean squared error, SSIM
 *   workspace      device scratch of at least igs_l1_ssim_workspace_size bytes (three fp32
 *                  partial-derivative maps and the per-block sums)
 * Deterministic (fixed-order reductions).  Errors: IGS_ERR_INVALID_ARG, IGS_ERR_WORKSPACE,
 * IGS_ERR_HIP.
 */
igs_status igs_l1_ssim_loss_grad(const float *image, const float *target, int32_t n, int32_t H,
                                 int32_t W, double ssim_weight, float *grad_image,
                                 double *loss_out, void *workspace, size_t ws_bytes,
                                 void *stream);

/* Scratch bytes igs_init_gaussians / igs_add_gaussians need for an H x W image. */
igs_status igs_place_workspace_size(int32_t H, int32_t W, size_t *ws_bytes);

/*
 * Content-adaptive initialization (Sec. 3.3, Eq. 6; Sec. 4.1): draws `count` pixels, each
 * independently with probability
 *   P(x) = (1 - lambda_init) |grad I(x)| / sum_x |grad I| + lambda_init / (H W)
 * where grad I is the per-channel central difference of the target inside the image and the
 * one-sided difference at its border (zero along an axis of length 1) and |.| the Euclidean norm
 * over both directions and all channels (uniform if the target has no gradient).  Pixel i is the
 * first pixel, in row-major order, whose cumulative probability exceeds uniforms[i].  The new
 * Gaussian j = first + i sits at the pixel centre (w + 1/2, h + 1/2) with rotation 0, both
 * scales `scale` pixels (the paper uses 5) and the target's colour at that pixel.
 *   target         [n][H][W] float32 device
 *   lambda_init    in [0, 1] (the paper uses 0.3)
 *   uniforms       device float32[count], each in [0, 1) (the caller's random numbers)
 *   render_params  [5+n][N_total] float32 device: columns [first, first + count) are written in
 *                  igs_render's units; other columns are untouched
 *   fit_params     NULL, or [5+n][N_total] float32 device: the same columns in the fitter's
 *                  parameterization (mean / (W, H), 1 / scale), as igs_adam_step keeps them
 *   workspace      device scratch of at least igs_place_workspace_size bytes
 * Deterministic.  Errors: IGS_ERR_INVALID_ARG (shapes, first + count > N_total, scale <= 0,
 * lambda outside [0, 1]), IGS_ERR_WORKSPACE, IGS_ERR_HIP.
 */
igs_status igs_init_gaussians(const float *target, int32_t n, int32_t H, int32_t W,
                              double lambda_init, const float *uniforms, int32_t count,
                              float scale, float *render_params, float *fit_params,
                              int32_t N_total, int32_t first, void *workspace, size_t ws_bytes,
                              void *stream);

/*
 * Error-guided addition of Gaussians (Sec. 3.3, Eq. 7; Sec. 4.1): as igs_init_gaussians, with
 * pixels drawn with probability P(x) = e(x) / sum_x e, e(x) = sum over channels of
 * |image - target| (uniform if the image equals the target); new Gaussians are initialized like
 * the content-adaptive ones (pixel centre, rotation 0, `scale` pixels, the target's colour).
 *   image  [n][H][W] float32 device: the current render
 * Errors: as igs_init_gaussians.
 */
igs_status igs_add_gaussians(const float *image, const float *target, int32_t n, int32_t H,
                             int32_t W, const float *uniforms, int32_t count, float scale,
                             float *render_params, float *fit_params, int32_t N_total,
                             int32_t first, void *workspace, size_t ws_bytes, void *stream);

/*
 * One Adam step (Sec. 4.1: Adam with constant per-group learning rates) in the fitter's
 * parameterization, fused with the chain rules from the renderer's units and the clipping of
 * Sec. 3.1:
 *   fit_params    [5+n][N] in/out: rows mu_x/W, mu_y/H (Sec. 4.1 maps the image to [0,1]^2),
 *                 theta, 1/s_1, 1/s_2 (inverse scales, Sec. 3.3 footnote and Sec. 4.1), colour
 *   render_params [5+n][N] out: the same parameters converted to igs_render's units
 *   grad_render   [5+n][N] in: dL/d(render params), e.g. igs_render_backward's output
 *   m, v          [5+n][N] in/out: Adam moments (zero before the first step)
 *   step          device int32[1] in/out: steps taken so far; incremented on the device after
 *                 the update
 *   skip_flag     device int64 or NULL: when non-NULL and non-zero at execution time the whole
 *                 step is a no-op (parameters, moments and step unchanged); pass the overflow
 *                 word of the render's status block so that an iteration whose render overflowed
 *                 the pair buffer changes nothing
 *   lr_mu, lr_theta, lr_inv_scale, lr_color: learning rates of the four groups
 *   beta1, beta2, eps: Adam constants; theta is clipped to [0, pi] and 1/s to
 *   [inv_scale_lo, inv_scale_hi] after the update.
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_HIP.
 */
igs_status igs_adam_step(float *fit_params, float *render_params, const float *grad_render,
                         float *m, float *v, int32_t *step, const int64_t *skip_flag, int32_t N,
                         int32_t n, int32_t H,
                         int32_t W, float lr_mu, float lr_theta, float lr_inv_scale,
                         float lr_color, float beta1, float beta2, float eps, float inv_scale_lo,
                         float inv_scale_hi, void *stream);

/*
 * Convert fitter parameters (see igs_adam_step) to render parameters without an update.
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_HIP.
 */
igs_status igs_fit_to_render(const float *fit_params, float *render_params, int32_t N, int32_t n,
                             int32_t H, int32_t W, void *stream);

/*
 * Chain rule from the renderer's units to the fitter's (the same rule igs_adam_step applies
 * before its update): for the [5+n][N] gradient grad_render with respect to render parameters,
 * writes grad_fit [5+n][N], the gradient with respect to fit_params (layout of igs_adam_step):
 * rows mu_x/W and mu_y/H get W and H times the mean rows, theta and colour rows are copied, and
 * the inverse-scale rows u = 1/s get -dL/ds / u^2.  grad_fit may not alias the inputs.
 * Errors: IGS_ERR_INVALID_ARG, IGS_ERR_HIP.
 */
igs_status igs_grad_to_fit(const float *fit_params, const float *grad_render, float *grad_fit,
                           int32_t N, int32_t n, int32_t H, int32_t W, void *stream);

/* ------------------------------------------------------------------------------------------
 * Batches: many images of uneven size and Gaussian count rendered, differentiated and optimized
 * by one launch per phase.  The images are concatenated: the parameter array is [5+n][Ntot]
 * (image b's Gaussians are columns gauss_off .. gauss_off+N-1), images/targets/gradients are
 * concatenated planar blocks (image b occupies floats n*pix_off .. n*(pix_off+H*W)-1 as
 * [n][H][W]).  Tiles of all images share one global numbering and one sort; the forward builds a
 * queue of all tiles ordered by decreasing |S_j| (stable), kept in the saved state, and both
 * raster passes take their tiles from it, so long tile lists start first.  Images are
 * independent: a Gaussian only bins into its own image's tiles, so every image renders exactly as
 * igs_render would render it alone.
 * Every batched entry point takes the descriptor array twice: on the host (sizes and validation)
 * and in device memory (read by the kernels; same bytes, caller-owned).
 * ------------------------------------------------------------------------------------------ */
typedef struct igs_image_desc {
  int32_t H, W, N, tiles_x;
  int32_t tiles_y, tile_off, gauss_off, l1_block_off;
  int64_t pix_off, ssim_block_off;  /* first workgroup of the image in the batched SSIM grid */
} igs_image_desc;

/*
 * Fill B descriptors for images H[b] x W[b] with N[b] Gaussians and n channels, in order.
 * totals_out: [0] total Gaussians, [1] total tiles, [2] total pixels, [3] loss blocks.
 * Errors: IGS_ERR_INVALID_ARG (sizes out of range, totals beyond 2^31 Gaussians or 2^24 tiles).
 */
igs_status igs_batch_describe(int32_t B, int32_t n, const int32_t *H, const int32_t *W,
                              const int32_t *N, igs_image_desc *descs_out, int64_t totals_out[4]);

/* As igs_render_buffer_sizes / igs_saved_offsets for a batch (out[6]: the tile queue, int32[T]). */
igs_status igs_batch_buffer_sizes(const igs_image_desc *descs, int32_t B, int32_t n, int32_t K,
                                  int64_t pair_capacity, size_t *ws_bytes, size_t *saved_bytes);
igs_status igs_batch_saved_offsets(const igs_image_desc *descs, int32_t B, int32_t n, int32_t K,
                                   int64_t pair_capacity, int64_t out[7]);

/* igs_render for a batch (Sec. 3.2, Eq. 5 per image); pair_capacity bounds the pairs of all
   images together.  Errors: as igs_render. */
igs_status igs_render_batched(const float *params, const igs_image_desc *descs_host,
                              const igs_image_desc *descs_dev, int32_t B, int32_t n, int32_t K,
                              int64_t pair_capacity, float *images, void *saved,
                              size_t saved_bytes, void *workspace, size_t ws_bytes, void *stream);

/* igs_render_backward for a batch (Sec. 3.3).  grad_params [5+n][Ntot] is overwritten. */
igs_status igs_render_backward_batched(const float *params, const igs_image_desc *descs_host,
                                       const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                       int32_t K, int64_t pair_capacity, const float *images,
                                       const float *grad_images, const void *saved,
                                       size_t saved_bytes, float *grad_params, void *workspace,
                                       size_t ws_bytes, void *stream);

/*
 * igs_render_l1 for a batch: targets are concatenated like the images; loss_out is device
 * double[B][2] (per image: mean |d| and mean d^2 over its own n*H_b*W_b values, d = image -
 * target), and the gradient of image b's loss is normalized by its own n*H_b*W_b, so each image
 * is fitted exactly as it would be alone.  n <= 16.
 */
igs_status igs_render_l1_batched(const float *params, const igs_image_desc *descs_host,
                                 const igs_image_desc *descs_dev, int32_t B, int32_t n, int32_t K,
                                 int64_t pair_capacity, const float *targets, float *images,
                                 double *loss_out, void *saved, size_t saved_bytes,
                                 void *workspace, size_t ws_bytes, void *stream);

/* Adjoint of igs_render_l1_batched; grad_params [5+n][Ntot] is overwritten. */
igs_status igs_render_backward_l1_batched(const float *params, const igs_image_desc *descs_host,
                                          const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                          int32_t K, int64_t pair_capacity, const void *saved,
                                          size_t saved_bytes, float *grad_params, void *workspace,
                                          size_t ws_bytes, void *stream);

/* igs_render_l1_grad for a batch: per-image loss and gradient normalization as
   igs_render_l1_batched; tiles are taken largest hit set first.  n <= 16. */
igs_status igs_render_l1_grad_batched(const float *params, const igs_image_desc *descs_host,
                                      const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                      int32_t K, int64_t pair_capacity, const float *targets,
                                      double *loss_out, float *grad_params, void *saved,
                                      size_t saved_bytes, void *workspace, size_t ws_bytes,
                                      void *stream);

/* L1 term per image (each normalized by its own n*H*W); loss_out is device double[B][2]
   (mean |d|, mean d^2 per image).  Deterministic.  Errors: as igs_l1_loss_grad. */
igs_status igs_l1_batched_workspace_size(const igs_image_desc *descs, int32_t B, int32_t n,
                                         size_t *ws_bytes);
igs_status igs_l1_loss_grad_batched(const float *images, const float *targets,
                                    const igs_image_desc *descs_host,
                                    const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                    float *grad_images, double *loss_out, void *workspace,
                                    size_t ws_bytes, void *stream);

/* Scratch bytes igs_l1_ssim_loss_grad_batched needs for the batch. */
igs_status igs_l1_ssim_batched_workspace_size(const igs_image_desc *descs, int32_t B, int32_t n,
                                              size_t *ws_bytes);

/*
 * igs_l1_ssim_loss_grad for every image of a batch in one launch per stencil pass: each image's
 * loss, SSIM and gradient are those igs_l1_ssim_loss_grad gives for that image alone (gradients
 * bit for bit; the loss sums in another order).  Strip s of a channel plane belongs to the last
 * image whose ssim_block_off <= s (igs_batch_describe sets it).
 *   images, targets, grad_images: concatenated [n][H][W] blocks as for the batched render
 *   loss_out  device double[B][4]: per image L, mean |image - target|, MSE, SSIM
 * Errors: as igs_l1_ssim_loss_grad, and IGS_ERR_INVALID_ARG for inconsistent descriptors.
 */
igs_status igs_l1_ssim_loss_grad_batched(const float *images, const float *targets,
                                         const igs_image_desc *descs_host,
                                         const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                         double ssim_weight, float *grad_images, double *loss_out,
                                         void *workspace, size_t ws_bytes, void *stream);

/* igs_adam_step for a batch: each Gaussian's mean is normalized by its own image's W and H and
   its inverse scales are clipped to [1/max(H,W), inv_scale_hi] of its image. */
igs_status igs_adam_step_batched(float *fit_params, float *render_params,
                                 const float *grad_render, float *m, float *v, int32_t *step,
                                 const int64_t *skip_flag, const igs_image_desc *descs_host,
                                 const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                 float lr_mu, float lr_theta, float lr_inv_scale, float lr_color,
                                 float beta1, float beta2, float eps, float inv_scale_hi,
                                 void *stream);
igs_status igs_fit_to_render_batched(const float *fit_params, float *render_params,
                                     const igs_image_desc *descs_host,
                                     const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                     void *stream);

/*
 * Launch settings of the raster kernels, per host thread (every thread starts from the
 * defaults); they apply to calls the thread issues afterwards (a captured graph keeps the
 * settings it was captured with), so callers that interleave work tuned differently set theirs
 * before enqueueing it.  No setting changes any output bit; they only trade scheduling and
 * blocking strategies, which is what an autotuner may choose among:
 *   persistent  0: one workgroup per tile (default); 1: a resident grid of wgs_per_cu workgroups
 *               per CU pulls tiles from per-XCD queues in the same order (the queues live in the
 *               workspace and are cleared by a kernel before each launch, so capture is safe);
 *               applies to the forward, adjoint and single-pass raster kernels
 *   wgs_per_cu  persistent grid size per CU, 0..64 (0 = as many as the kernel's resources allow)
 *   fwd_cull    1 (default): the forward visits candidates in ascending order of a lower bound of
 *               the Mahalanobis form over the tile and skips, per wave, candidates that cannot
 *               enter any of the wave's lists; 0: every candidate is ranked at every pixel
 *   fwd_batch   members of S_j the forward stages in LDS at a time, a multiple of 32 in
 *               [64, 256] (0 = 192); a tile whose S_j fits one batch also keeps its members'
 *               blend data there
 *   k_unroll    length of the forward's register-resident sorted list: the smallest compiled
 *               length (1, 2, 4, 8, 10, 16, 32) >= max(K, k_unroll), 0 = the smallest >= K; its
 *               first K entries are the top-K whatever its length (keys are unique)
 * Errors: IGS_ERR_INVALID_ARG (NULL or out-of-range fields).
 */
typedef struct {
  int32_t persistent;
  int32_t wgs_per_cu;
  int32_t fwd_cull;
  int32_t fwd_batch;
  int32_t k_unroll;
} igs_launch_config;
igs_status igs_set_launch_config(const igs_launch_config *cfg);
igs_status igs_get_launch_config(igs_launch_config *cfg);

/*
 * Kernel timers (measurement aid, off by default).  While enabled, every entry point records a
 * pair of HIP events on its stream around each of its phases; igs_timing_read waits for the
 * recorded events, returns the accumulated milliseconds and call counts per phase and, if reset is
 * non-zero, clears them.  Phases: IGS_PHASE_BINNING (footprint bound, scan, pair emission, sort
 * and tile ranges), IGS_PHASE_RASTER_FWD (the forward raster kernel, with the fused L1 epilogue
 * when called through igs_render_l1), IGS_PHASE_RASTER_BWD (the adjoint raster kernel),
 * IGS_PHASE_GRAD_REDUCE (the adjoint's per-Gaussian reduction), IGS_PHASE_LOSS (the loss
 * kernels, or the fused forward's final loss reduction), IGS_PHASE_ADAM, IGS_PHASE_RASTER_FIT (the
 * single-pass kernel of igs_render_l1_grad).  At most 65536 event
 * pairs are kept between reads; further phases go untimed.  Not thread-safe; do not enable during
 * graph capture.
 */
#define IGS_PHASE_BINNING 0
#define IGS_PHASE_RASTER_FWD 1
#define IGS_PHASE_RASTER_BWD 2
#define IGS_PHASE_LOSS 3
#define IGS_PHASE_ADAM 4
#define IGS_PHASE_GRAD_REDUCE 5
#define IGS_PHASE_RASTER_FIT 6
#define IGS_NUM_PHASES 7
igs_status igs_timing_enable(int32_t on);
igs_status igs_timing_read(double ms_out[IGS_NUM_PHASES], int64_t calls_out[IGS_NUM_PHASES],
                           int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* IMAGEGS_H */
