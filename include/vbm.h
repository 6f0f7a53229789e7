/*
 * vbm.h -- C ABI of the MI355X (gfx950) Variable Basis Mapping library, libvbm.so.
 *
 * Variable Basis Mapping (VBM) turns a volume into a 3D Gaussian Splatting scene: a transfer
 * function maps the scalar field to RGBA (Sec. 3), a J-level 3D DWT decomposes it (Sec. 3,
 * Sec. 4.3 eq. mul_wavelet_coff), every kept coefficient becomes one Gaussian by a lookup in the
 * Wavelet-to-Gaussian Transition Bank (Sec. 4.2, Sec. 4.3), and an image-space fine-tuning loop
 * refines the Gaussians against direct-volume-rendered images (Sec. 4.4).  This library runs that
 * path on the GPU: vbm_dwt3d, vbm_build_gaussians, vbm_render_fwd, vbm_render_bwd, plus the loss,
 * optimiser and supervision-renderer kernels of the fine-tuning loop.
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless the parameter name ends in "_host".
 *   - The caller owns all memory.  The library never allocates device memory: each call that
 *     needs scratch space takes a workspace sized by the matching *_workspace_size() function or
 *     by vbm_plan_make().
 *   - Every call enqueues on the given HIP stream (a hipStream_t passed as void*, NULL = the null
 *     stream) and returns without synchronising, except vbm_render_fwd in VBM_MODE_EXACT, which
 *     synchronises once to read the pair count.
 *   - Argument checks run on the host before anything is enqueued, so a call that returns an
 *     error has launched nothing.  vbm_last_error() returns a thread-local message.
 *   - Conditions found on the device (pair-list overflow) are reported through caller-provided
 *     device flags, never by aborting.
 *   - Volumes are float32 [z][y][x] (x fastest), G^3 values, covering [-1, 1]^3 with voxel i
 *     centred at -1 + (2/G)(i + 1/2).
 */
#ifndef VBM_H
#define VBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vbm_status;
#define VBM_OK 0
#define VBM_ERR_INVALID (-1)     /* bad argument (null pointer, size, range) */
#define VBM_ERR_UNSUPPORTED (-2) /* wavelet, tile size or device not supported */
#define VBM_ERR_WORKSPACE (-3)   /* workspace smaller than required */
#define VBM_ERR_HIP (-4)         /* a HIP runtime call failed */
#define VBM_ERR_CAPACITY (-5)    /* a fixed capacity was exceeded (host-detected) */

#define VBM_WAVELET_HAAR 0   /* Haar, the paper's ablation basis (Sec. 5.4) */
#define VBM_WAVELET_BIOR44 1 /* biorthogonal 4.4 = CDF 9/7, the paper's default (Sec. 4.2) */

const char* vbm_version(void);
const char* vbm_last_error(void);

/* ------------------------------------------------------------------------------------------
 * Transfer function (Sec. 3, Transfer Function): RF = TF(F), scalar -> RGBA.  Piecewise linear
 * through n_points ascending control points x[i] with values rgba[i][0..3]; constant beyond the
 * end points.  Host struct, passed by pointer, copied at call time.
 * ------------------------------------------------------------------------------------------ */
#define VBM_TF_MAX_POINTS 16
typedef struct {
  int32_t n_points;
  float x[VBM_TF_MAX_POINTS];
  float rgba[VBM_TF_MAX_POINTS][4];
} vbm_tf;

/* ------------------------------------------------------------------------------------------
 * vbm_dwt3d -- RGBA wavelet coefficients A_{j,o,k,c} of TF(vol) (Sec. 4.3, eq. mul_wavelet_coff).
 *
 *   vol     float32 [G][G][G] scalar field (tf != NULL), or float32 [4][G^3] planar RGBA (tf == NULL)
 *   G, J    grid size and levels; G % 2^J == 0, 2 <= G/2^J, 1 <= J <= 10, G <= 1024
 *   wavelet VBM_WAVELET_HAAR or VBM_WAVELET_BIOR44; periodised separable analysis, x then y then z
 *           per level, the next level on LLL
 *   coeffs  float32 [4][G^3] output, per channel in the packed subband layout
 *           [LLL_J][level J: o=1..7][level J-1: o=1..7]...[level 1: o=1..7],
 *           block (j, o) = [n^3] in [kz][ky][kx] order, n = G/2^j; orientation o has bit d set
 *           when the high-pass was taken along axis d (bit 0 = x, 1 = y, 2 = z)
 *   ws      workspace of vbm_dwt3d_workspace_size(G, J) bytes
 * Errors: VBM_ERR_INVALID on null pointers or sizes, VBM_ERR_UNSUPPORTED on an unknown wavelet
 * or more than VBM_TF_MAX_POINTS control points, VBM_ERR_WORKSPACE if ws_bytes is too small.
 * ------------------------------------------------------------------------------------------ */
size_t vbm_dwt3d_workspace_size(int32_t G, int32_t J);
vbm_status vbm_dwt3d(const float* vol, int32_t G, int32_t J, int32_t wavelet, const vbm_tf* tf_host,
                     float* coeffs, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * Transition bank (Sec. 4.2: eq. canonical_wavelet, eq. roi, eq. moment, eq. canonical_gaussian,
 * eq. ridge_regression), computed on the host in double precision.  One entry per subband in the
 * packed block order above: 7J + 1 entries (seven orientations per level plus the final LLL).
 *   u      centroid of the dominant lobe, voxel-index units relative to the impulse origin 2^j k
 *   sigma  weighted covariance over the ROI {W > tau max W}: xx, yy, zz, xy, xz, yz
 *   w      ridge-regression amplitude <G,|Y|> / (<G,G> + lambda)
 *   scale, quat  sigma = R(quat) diag(scale^2) R(quat)^T; quat (w, x, y, z), w >= 0; identity and
 *          scale = sqrt(diag sigma) when sigma is diagonal
 * vbm_bank_pack writes VBM_BANK_FLOATS floats per entry (w, u[3], scale[3], quat[4], pad) into
 * host memory; the caller uploads them for vbm_build_gaussians.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t j, o, roi_size, pad;
  double w;
  double u[3];
  double sigma[6];
  double scale[3];
  double quat[4];
} vbm_bank_entry;

#define VBM_BANK_FLOATS 12
int32_t vbm_bank_size(int32_t J);
vbm_status vbm_bank_build(int32_t wavelet, int32_t J, double tau, double lambda, vbm_bank_entry* out_host);
vbm_status vbm_bank_pack(const vbm_bank_entry* entries_host, int32_t n_entries, float* out_host);

/* ------------------------------------------------------------------------------------------
 * Gaussian parameter sets.  Structure of arrays, float32, one plane per component with plane
 * stride `stride` (>= number of Gaussians):
 *   means [3][stride] world x, y, z         scales  [3][stride] > 0 (activated)
 *   quats [4][stride] w, x, y, z (any norm) opacity [stride] in (0, 1) (activated)
 *   rgb   [3][stride]
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* rgb;
  int64_t stride;
} vbm_gaussians;

typedef struct {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* rgb;
  int64_t stride;
} vbm_gaussians_c;

/* ------------------------------------------------------------------------------------------
 * vbm_build_gaussians -- joint-norm top-K selection and analytical construction (Sec. 4.3:
 * eq. per_location_weight, eq. wavelet_gaussian_kernel, eq. translation_operator; joint norm of
 * Supp. A).  Keeps the K locations with the largest float32 joint norm
 * sqrt(((R^2 + G^2) + B^2) + A^2) (ties to the lower packed index) and emits them in ascending
 * packed-index order, one Gaussian each:
 *   mean  = -1 + h (u_{j,o} + 2^j k + delta), h = 2/G;  scale = h scale_{j,o};  quat = quat_{j,o}
 *   amp   = s_j |A_{j,o,k,:}| w_{j,o}, s_j = 2^{-3j/2} (s_mode 0) or 1 (s_mode 1)
 *   opacity = clamp(amp_A, opacity_min, opacity_max), rgb = clamp(amp_RGB, 0, 1)
 *   coeffs      float32 [4][G^3] as written by vbm_dwt3d
 *   bank_dev    VBM_BANK_FLOATS * (7J+1) floats from vbm_bank_pack
 *   kept_index  optional int64 [K] output of the kept packed indices (NULL to skip)
 * Errors: VBM_ERR_INVALID for K < 1 or K > G^3, null pointers or bad opts.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t s_mode;
  float delta;
  float opacity_min;
  float opacity_max;
  /* Ablation variants (Sec. 5): isotropic = 1 replaces every covariance by sigma_iso^2 I (scales
   * sigma_iso, identity rotation) with sigma_iso the mean over the built Gaussians of the mean of
   * their three bank scales (the full model's average extent, summed in float64 in a fixed order);
   * unit_weight = 1 sets w_{j,o} = 1 (no energy projection).  Both 0 for the method itself. */
  int32_t isotropic;
  int32_t unit_weight;
} vbm_build_opts;

size_t vbm_build_workspace_size(int32_t G, int32_t J);
vbm_status vbm_build_gaussians(const float* coeffs, int32_t G, int32_t J, const float* bank_dev, int64_t K,
                               const vbm_build_opts* opts_host, vbm_gaussians out, int64_t* kept_index, void* ws,
                               size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_adaptive_select -- adaptive per-subband selection (Supp. A: global budget allocation
 * across subbands, joint multi-channel sparsification, robust MAD-based thresholding, top-K
 * selection under sparsity constraints).  For every subband of the packed layout (the LLL block
 * and the seven detail blocks of each level, 7J+1 subbands):
 *   E = sum_k A_{j,o,k,ref}^2 (float64), N = #k, S = E^alpha N^beta,
 *   K_{j,o} = max(min_band, floor(K_tot S / sum S))        (sum S = 0 gives 0)
 *   v = sqrt(((R^2 + G^2) + B^2) + A^2) in float32 (the vbm_build_gaussians key)
 *   MAD = median |v - median(v)|, medians of an even count = (a + b) * 0.5 (float32),
 *   sigma = MAD / 0.6745, T = lambda sigma (float32)
 *   K = min(K_{j,o}, #(v >= T)); keep v >= max(T, v_(K)) (all ties with v_(K); none if K = 0)
 * The kept packed indices are written in ascending order to kept_index[0 .. capacity) (device,
 * int64) and their total to *count_dev (device, int64); a total above capacity means the list was
 * cut at capacity.  band_stats (device, optional) receives VBM_ADAPTIVE_STATS doubles per subband:
 * E, N, K_tot S / sum S, K_{j,o}, median, MAD, sigma, T, #(v >= T), K, v_(K), kept count.
 * The total can exceed K_tot when the per-band minimum applies.  Enqueues only (no host sync).
 * Errors: VBM_ERR_INVALID for bad G/J, K_tot outside 1..G^3, negative alpha/beta/lambda,
 * ref_channel outside 0..3, null pointers; VBM_ERR_WORKSPACE if ws_bytes is too small.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int64_t K_tot;       /* global budget */
  double alpha, beta;  /* S = E^alpha N^beta */
  float lambda;        /* T = lambda sigma */
  int32_t ref_channel; /* 0..3 (R, G, B, A); the supplement's typical choice is A */
  int64_t min_band;    /* per-subband minimum budget (10 in the supplement) */
} vbm_adaptive_opts;

#define VBM_ADAPTIVE_STATS 12
size_t vbm_adaptive_workspace_size(int32_t G, int32_t J);
vbm_status vbm_adaptive_select(const float* coeffs, int32_t G, int32_t J, const vbm_adaptive_opts* opts_host,
                               int64_t capacity, int64_t* kept_index, int64_t* count_dev, double* band_stats,
                               void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_construct_gaussians -- the construction of vbm_build_gaussians (Sec. 4.3) for a given list
 * of n packed indices (device, int64), one Gaussian per entry in list order; an entry outside
 * [0, G^3) leaves its output slot untouched.  Enqueues only.  Errors: VBM_ERR_INVALID for bad G/J, n < 0, out.stride < n, null pointers or
 * bad opts.
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_construct_gaussians(const float* coeffs, int32_t G, int32_t J, const float* bank_dev,
                                   const int64_t* kept_index, int64_t n, const vbm_build_opts* opts_host,
                                   vbm_gaussians out, void* stream);

/* ------------------------------------------------------------------------------------------
 * Rendering batches.  A batch renders n_views views; view v shows scene `scene` of a
 * concatenated Gaussian set whose scene s occupies Gaussians [scene_offsets[s], scene_offsets[s+1]).
 * Pinhole camera, OpenCV axes (x right, y down, z forward); viewmat is world->camera [R|t],
 * 3x4 row-major; pixel (i, j) samples the image plane at (i + 0.5, j + 0.5).
 *
 * Rasteriser (the paper cites 3DGS for it, Sec. 4.4): EWA projection with 0.3 px dilation and
 * a 1.3x field-of-view clamp in the Jacobian, near-plane cull, 3-sigma tile rectangles, pairs in
 * ascending (global tile, float32 depth bits, item) order, front-to-back compositing per pixel with
 * alpha = min(0.99, o exp(power)), skip alpha < 1/255, stop before adding once T would drop below
 * 1e-4.  Images are planar float32 [3][H][W] per view, concatenated in view order;
 * final_T and n_contrib are [H][W] per view, concatenated: final_T is the transmittance left after
 * compositing, n_contrib (int32) the number of entries of the pixel's tile list that its
 * compositing took into account -- the list position of the Gaussian that would have taken T below
 * 1e-4 (that Gaussian excluded), or the whole list length when that never happens; the backward
 * reads both.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t scene;
  int32_t width, height;
  int32_t pad;
  float fx, fy, cx, cy;
  float near_plane;
  float viewmat[12];
  float bg[3];
} vbm_view;

#define VBM_MODE_BATCHED 0 /* counts stay on the device: no host sync, graph-capturable */
#define VBM_MODE_EXACT 1   /* one host sync per call to read the pair count; sort sized exactly */

typedef struct {
  int32_t tile;          /* tile edge in pixels: 8, 16 or 32 */
  int32_t sort_bits;     /* radix digit width for the tile sort: 4..8 */
  int64_t pair_capacity; /* pair slots reserved in the workspace, in [1, 2^30) */
  int32_t mode;          /* VBM_MODE_BATCHED or VBM_MODE_EXACT */
  int32_t lds_batch;     /* record staging of the forward compositing: 0 = each record through the
                          * scalar cache into registers; 32 or 64 = the tile's list staged in LDS
                          * batches of that many entries (8x8 and 16x16 tiles only).  Results are
                          * identical. */
  int32_t lds_batch_bwd; /* the same choice for the backward compositing */
  int32_t pad0;
} vbm_schedule;

#define VBM_WS_REGIONS 24
typedef struct {
  int32_t n_views, n_scenes, tile, mode;
  int32_t sort_bits, tile_key_bits, lds_batch, lds_batch_bwd;
  int64_t n_gaussians, n_items, n_tiles, n_pixels, pair_capacity;
  size_t view_table_bytes; /* device view table written by vbm_plan_make into view_table_host */
  size_t ws_bytes;         /* workspace needed by vbm_render_fwd + vbm_render_bwd */
  size_t region_offset[VBM_WS_REGIONS];
  size_t region_bytes[VBM_WS_REGIONS];
} vbm_plan;

/* Workspace regions a test may read back after vbm_render_fwd (offsets into ws). */
#define VBM_REGION_COUNTERS 0    /* uint32 [16]: [0] visible items, [1] pairs, [2] overflow, [4..5]
                                  * uint64 ballot words taken by large footprints */
#define VBM_REGION_ITEM_DEPTH 1  /* float32 [n_items] camera depth (0 when culled) */
#define VBM_REGION_ITEM_RECT 2   /* uint32 [n_items][4], the binning entry of each item:
                                  * [0] x0 | x1 << 16 and [1] y0 | y1 << 16, the candidate
                                  * rectangle in tiles (12 bits each; with 16x16 tiles bits
                                  * 12..13 and 28..29 of [1] hold the first row band the footprint
                                  * can reach in tile row y0 and the last in tile row y1 - 1),
                                  * [2] the reached-tile mask of a rectangle of at most 32 tiles
                                  * (row-major) or the first ballot word of a larger one
                                  * (0xFFFFFFFF when the word buffer was full), [3] the number of
                                  * reached tiles */
#define VBM_REGION_ITEM_NTILES 3 /* uint32 [n_items] */
#define VBM_REGION_ITEM_REC 4    /* float32 [n_items][4]: conic.abc, opacity (mean2d is in
                                  * VBM_REGION_ITEM_COEF) */
#define VBM_REGION_ITEM_BLUE 5   /* float32 [n_items]: blue */
#define VBM_REGION_PAIR_TILE 6   /* uint32 [pair_capacity]: sorted global tile of each pair */
#define VBM_REGION_PAIR_ITEM 7   /* uint32 [pair_capacity]: sorted item of each pair in bits 0..26;
                                  * bit 27 + k is set when the footprint can reach lane group k of
                                  * the tile (with 16x16 tiles pixel rows 4k .. 4k + 3; every group
                                  * with other tiles); bit 31 is 0.  With 8x8 and 16x16 tiles
                                  * vbm_render_fwd keeps a copy elsewhere in ws with bit 27 + k set
                                  * when it evaluated lane group k (pixel rows k*64/tile .. of the
                                  * tile) of the pair, which vbm_render_bwd reads */
#define VBM_REGION_RANGES 8      /* uint32 [n_tiles][2]: [start, end) of each tile's list */
#define VBM_REGION_GRAD2D 9      /* float32 [n_items][16] after vbm_render_bwd: columns 0..5 hold the
                                  * sums over the item's pixels of dL/dpower times dx, dy, dx^2,
                                  * dx dy, dy^2 and 1 (d = mean2d - pixel centre), columns 6..8
                                  * drgb; with the item's conic (A, B, C) and opacity o the 2D
                                  * gradients are dmean2d = -(A m0 + B m1, B m0 + C m1), dconic =
                                  * (-m2/2, -m3, -m4/2), dopacity = m5 / o.  Rows of items never
                                  * binned stay 0; columns 9..15 are padding */
#define VBM_REGION_ITEM_COEF 19  /* float32 [n_items][8]: compositing record mean2d.xy, -A/2 log2e,
                                  * -B log2e, -C/2 log2e, log2(opacity), r, g (conic A, B, C) */

/* Plans a batch (host only).  scene_offsets_host is int64 [n_scenes + 1].  If view_table_host
 * is not NULL it receives plan->view_table_bytes bytes that the caller copies to the device and
 * passes as view_table_dev.  Item i of view v is Gaussian scene_offsets[scene_v] + (i - item_offset_v).
 * Limits (VBM_ERR_INVALID beyond them): 1..4096 views and scenes, images up to 16384 x 16384, fewer
 * than 2^27 items (sum over views of the scene's Gaussian count) and 2^31 tiles, Gaussians and image
 * values in the batch. */
vbm_status vbm_plan_make(const vbm_view* views_host, int32_t n_views, const int64_t* scene_offsets_host,
                         int32_t n_scenes, const vbm_schedule* sched_host, vbm_plan* plan_out,
                         void* view_table_host);

/* ------------------------------------------------------------------------------------------
 * vbm_render_fwd -- project (all views), bin, depth-sort, tile-sort and composite.
 *   status    device int32 [4]: [0] set to 1 if the pair list overflowed pair_capacity (the images
 *             are then incomplete; re-plan with a larger capacity), [1] pair count, [2] visible items,
 *             [3] incremented when this forward overflowed (a count over the forwards that share the
 *             buffer, so that a loop without host syncs can check once; the caller resets it)
 *   ws        plan->ws_bytes; holds the state vbm_render_bwd needs, keep it unchanged between
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_render_fwd(const vbm_plan* plan_host, const void* view_table_dev, vbm_gaussians_c g, float* image,
                          float* final_T, int32_t* n_contrib, int32_t* status, void* ws, size_t ws_bytes,
                          void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_render_bwd -- gradient of sum <dL_dimg, image> w.r.t. the activated parameters, by
 * reverse-order compositing that recomputes each pixel's transmittance from final_T by division,
 * then the chain through the EWA projection, summed over views.
 *   grads       same SoA layout as the parameters; written (accumulate = 0) or added to (1)
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_render_bwd(const vbm_plan* plan_host, const void* view_table_dev, vbm_gaussians_c g,
                          const float* dL_dimg, const float* final_T, const int32_t* n_contrib, vbm_gaussians grads,
                          int32_t accumulate, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_image_loss -- fine-tuning loss (Sec. 4.4, "as in 3DGS") and its gradient w.r.t. the image.
 *   kind 0: L1 = mean |I - I_ref| over all views, channels and pixels
 *   kind 1: (1 - lambda) L1 + lambda (1 - SSIM), SSIM per channel with an 11x11 Gaussian window
 *           (sigma 1.5), zero-padded "same" filtering, C1 = 0.01^2, C2 = 0.03^2, averaged over all
 *           views, channels and pixels
 *   view_dims_host int32 [n_views][2] = (width, height); images laid out as for vbm_render_fwd
 *   dL_dimg  written; loss_dev float32 [1] written
 * ------------------------------------------------------------------------------------------ */
size_t vbm_image_loss_workspace_size(const int32_t* view_dims_host, int32_t n_views, int32_t kind);
vbm_status vbm_image_loss(const float* image, const float* target, const int32_t* view_dims_host, int32_t n_views,
                          int32_t kind, float lambda, float* dL_dimg, float* loss_dev, void* ws, size_t ws_bytes,
                          void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_image_loss_static -- vbm_image_loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the same loss, gradient
 * and kernels, with the scratch space taken from a fixed device array inside the library instead of
 * a workspace argument.  Nothing is allocated by the call.
 *   Arguments as vbm_image_loss without ws / ws_bytes.
 *   Limit: the call needs vbm_image_loss_workspace_size(view_dims, n_views, kind) <=
 *   VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES (64 MiB): any size for L1 (kind 0, about 8 KiB), and about
 *   1.8 million pixels in all views for L1 + D-SSIM (kind 1, 36 bytes per pixel).  Larger calls
 *   return VBM_ERR_CAPACITY and launch nothing.
 *   Each GPU holds one copy of the array (64 MiB, until the process ends), looked up at the first
 *   call on that device.  Every call on a GPU uses that GPU's copy: calls that overlap on one GPU
 *   (on different streams or threads without ordering) race and give wrong results; calls ordered
 *   on one stream are fine.  Nothing in the array needs clearing between calls.
 * Errors: those of vbm_image_loss, VBM_ERR_CAPACITY beyond the limit, VBM_ERR_HIP if the array's
 * device address cannot be looked up.
 * ------------------------------------------------------------------------------------------ */
#define VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES (64u << 20)
vbm_status vbm_image_loss_static(const float* image, const float* target, const int32_t* view_dims_host,
                                 int32_t n_views, int32_t kind, float lambda, float* dL_dimg, float* loss_dev,
                                 void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_adam_step -- Adam (Sec. 5, Implementation Details) on the raw parameters.
 *   raw, m, v  float32 [14][stride]: rows 0-2 means, 3-5 log scales, 6-9 quats, 10 logit opacity,
 *              11-13 rgb
 *   grads      activated-parameter gradients (from vbm_render_bwd), chained through
 *              scale = exp(raw) and opacity = sigmoid(raw) inside the kernel
 *   act        written with the updated activated parameters
 *   lr         per group: means, log scales, quats, logit opacity, rgb
 *   step_dev   optional device int32 step counter: when non-NULL the call first increments it and the
 *              kernel reads the step from it (so a captured graph replays with advancing steps);
 *              when NULL, opts->step (1-based) is used
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  float lr[5];
  float beta1, beta2, eps;
  int32_t step; /* 1-based step count */
  int32_t pad;
} vbm_adam_opts;

vbm_status vbm_adam_step(int64_t n, int64_t stride, float* raw, float* m, float* v, vbm_gaussians_c grads,
                         vbm_gaussians act, const vbm_adam_opts* opts_host, int32_t* step_dev, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_adam_init -- the optimiser state at the start of fine-tuning (Sec. 5, Implementation
 * Details: Adam; the raw parameters of vbm_adam_step).  For Gaussians 0..n-1:
 *   raw rows 0-2 = means, 3-5 = log(scales), 6-9 = quats, 10 = log(o / (1 - o)), 11-13 = rgb
 *   m = v = 0 on all 14 rows
 *   act        activated parameters (stride act.stride >= n), read only
 *   raw, m, v  float32 [14][stride], stride >= n, written (columns >= n untouched)
 * There is no clamp: a scale <= 0 or an opacity outside (0, 1) gives a non-finite raw value, as the
 * map itself does (the construction's opacities lie in [opacity_min, opacity_max] inside (0, 1)).
 * Enqueues only.  Errors: VBM_ERR_INVALID for null pointers, n < 0, stride < n or act.stride < n.
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_adam_init(int64_t n, int64_t stride, vbm_gaussians_c act, float* raw, float* m, float* v, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_dvr_render -- supervision images by ray marching (Sec. 4.4: the method fine-tunes against
 * volume-rendered images).  One ray per pixel centre, clipped to [-1,1]^3, a sample every
 * step_vox voxels from the entry point, trilinear interpolation of the scalar field, the transfer
 * function after interpolation, opacity corrected to the step (1 - (1 - a)^step_vox),
 * front-to-back until T < 1e-4, background bg.  Output layout as vbm_render_fwd's image.
 * The marching runs in float64 (volume and control points are float32 values); the images are
 * rounded to float32 once at the end.
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_dvr_render(const float* vol, int32_t G, const vbm_tf* tf_host, const vbm_view* views_host,
                          int32_t n_views, float step_vox, float* image, void* stream);

/* ------------------------------------------------------------------------------------------
 * vbm_profile_events -- measurement aid: hipEvent_t handles (passed as void*) that later
 * vbm_render_fwd / vbm_render_bwd calls record on their stream immediately before and after the
 * compositing kernel launch, so a caller can time that kernel alone with hipEventElapsedTime.
 * Process-wide setting; NULL handles disable the recording.  Not for use inside graph capture.
 * ------------------------------------------------------------------------------------------ */
vbm_status vbm_profile_events(void* composite_fwd_begin, void* composite_fwd_end, void* composite_bwd_begin,
                              void* composite_bwd_end);

/* vbm_profile_counters -- measurement aid: when dev_counters (device uint64 [4], zeroed by the caller)
 * is non-NULL, later compositing launches add the number of (pixel, Gaussian) evaluations and of
 * contributing evaluations: [0] forward evaluated, [1] forward contributing, [2] backward evaluated,
 * [3] backward contributing.  Process-wide; NULL disables it (the default). */
vbm_status vbm_profile_counters(void* dev_counters);

#ifdef __cplusplus
}
#endif
#endif /* VBM_H */
