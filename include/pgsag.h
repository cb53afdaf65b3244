/*
 * pgsag.h -- C ABI of a masked, tile-based, differentiable 3D Gaussian
 * splatting rasterizer for AMD Instinct MI355X (gfx950).
 *
 * The operation is the per-sub-region rendering step of PG-SAG
 * (arXiv 2501.01677): Gaussians with position, anisotropic covariance,
 * spherical-harmonics colour and opacity are projected to 2D Gaussians,
 * assigned to image tiles, depth sorted and alpha blended (Sec. 3.1, Eq. 1);
 * the camera-frame Gaussian normals (Eq. 2) and plane distances (Eq. 3) are
 * blended the same way and turned into an unbiased depth by intersecting
 * every pixel ray with the blended plane (Eq. 4).  Only pixels inside the
 * building mask are rendered (Sec. 1, Sec. 4.1, Sec. 5.3), and many
 * sub-regions and views are rendered in one batch (Sec. 4.1, Sec. 4.4).
 * The backward pass returns gradients of a scalar loss with respect to the
 * raw Gaussian parameters (differentiable rendering, Sec. 3.1).
 *
 * Conventions
 *  - All floating point is FP32, counts are int32, masks uint8 (0 / non-0).
 *  - Every array is planar (structure of arrays), row-major images [H][W].
 *  - World to camera: x_c = R x_w + t, R row-major; the camera looks along
 *    +z, image x to the right, image y down.  Pixel (u, v) samples the image
 *    plane at (u + 0.5, v + 0.5).  Intrinsics fx, fy, cx, cy.
 *  - Raw parameters of a Gaussian set of n Gaussians:
 *      means [3][n], log_scales [3][n] (natural log of the axis scales),
 *      quats [4][n] as (w, x, y, z), any non-zero norm (normalised inside),
 *      opacity_logits [n] (opacity = sigmoid(logit)),
 *      sh [(deg+1)^2][3][n]  (real orthonormal SH with the Condon-Shortley
 *      phase, coefficient index l*l + l + m; colour = sum + 0.5, clamped at
 *      0, evaluated on the world-frame direction camera centre -> mean).
 *  - Outputs per render, for masked pixels (0 elsewhere):
 *      rgb [3][H][W] (Eq. 1 plus background times final transmittance),
 *      normal [3][H][W] (Eq. 2, camera frame, not normalised),
 *      dist [H][W] (Eq. 3, blended signed plane distance n_c . t_c),
 *      depth [H][W] (Eq. 4: dist / (normal . K^-1 p~), 0 unless the
 *                    denominator is below -1e-6),
 *      alpha [H][W] (1 - final transmittance),
 *      n_contrib [H][W] (number of blended Gaussians, the g_i of Eq. 9).
 *  - Constants (see pgsag_config): fragments with alpha < alpha_min are
 *    skipped; blending stops before a fragment would take the transmittance
 *    below t_min; alpha = min(alpha_max, o * exp(-q/2)); +dilation px^2 on
 *    the projected covariance diagonal; Gaussians with FP32 camera depth
 *    <= z_near or logit < logit_min are culled; the depth order key is the
 *    FP32 camera depth ((R20*x + R21*y) + R22*z) + t2 with every operation
 *    rounded separately, ties by Gaussian index.
 *
 * Ownership: the caller owns every buffer -- parameters, outputs,
 * gradients, the workspace and the device copy of the descriptor.  The
 * library never allocates or frees device memory and keeps no global
 * mutable state except the thread-local error string and the static
 * scratch array of pgsag_dbscan_static (held per GPU by the library).  Work is enqueued on
 * the caller's HIP stream (passed as void*, a hipStream_t; NULL = the null
 * stream); no call synchronises except pgsag_read_status.  pgsag_forward
 * and pgsag_backward are capturable into a HIP graph.
 *
 * Errors: every call returns a pgsag_status_code; on failure
 * pgsag_last_error() (thread-local, valid until the next call on the same
 * thread) describes it.  A pair-capacity overflow is detected on the
 * device: emission stops at the capacity, the status word records the
 * pairs that were needed and the outputs of that forward are invalid; read
 * it with pgsag_read_status and plan again with a larger capacity.
 */
#ifndef PGSAG_H
#define PGSAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PGSAG_ABI_VERSION 3
#define PGSAG_NUM_STAGES 8

typedef enum pgsag_status_code {
  PGSAG_OK = 0,
  PGSAG_INVALID_ARGUMENT = 1,    /* null required pointer, bad size, bad tile */
  PGSAG_WORKSPACE_TOO_SMALL = 2, /* workspace or descriptor buffer too small */
  PGSAG_UNSUPPORTED = 3,         /* valid but not implemented combination */
  PGSAG_HIP_ERROR = 4            /* a HIP launch or copy failed */
} pgsag_status_code;

/* Stages timed when an event array is passed to forward/backward
 * (events[2*s] recorded before stage s, events[2*s+1] after it). */
typedef enum pgsag_stage {
  PGSAG_STAGE_TILE_MASK = 0,  /* per-tile masked-pixel counts, active-tile row prefix */
  PGSAG_STAGE_PREPROCESS = 1, /* projection, SH colour, normal, support rect */
  PGSAG_STAGE_DEPTH_SORT = 2, /* compaction + radix sort of visible records */
  PGSAG_STAGE_EMIT = 3,       /* pair-count scan + (tile, record) emission */
  PGSAG_STAGE_TILE_SORT = 4,  /* stable radix sort of pairs by tile, ranges, queue */
  PGSAG_STAGE_COMPOSITE = 5,  /* forward compositing + depth epilogue */
  PGSAG_STAGE_BACKWARD_COMPOSITE = 6, /* backward compositing (2D gradients) */
  PGSAG_STAGE_BACKWARD_PREPROCESS = 7 /* chain rule to raw parameters */
} pgsag_stage;

typedef struct pgsag_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9]; /* world -> camera rotation, row-major */
  float t[3]; /* x_c = R x_w + t */
} pgsag_camera;

typedef struct pgsag_gaussians {
  int64_t n;         /* number of Gaussians, >= 0 */
  int32_t sh_degree; /* 0..3 */
  int32_t reserved;
  const float *means, *log_scales, *quats, *opacity_logits, *sh; /* device */
} pgsag_gaussians;

/* Gradients with respect to the raw parameters of one set, same layouts as
 * pgsag_gaussians; overwritten (not accumulated) by pgsag_backward, summed
 * over every render of the set.  Any pointer may be NULL (not wanted). */
typedef struct pgsag_grads {
  float *means, *log_scales, *quats, *opacity_logits, *sh;
} pgsag_grads;

/* Device output planes of one render; NULL = not wanted, except alpha-free
 * operation: the backward needs nothing here, but the depth gradient needs
 * normal and dist, which must then be non-NULL. */
typedef struct pgsag_outputs {
  float *rgb, *normal, *dist, *depth, *alpha;
  int32_t *n_contrib;
} pgsag_outputs;

/* Device dL/d(output) planes, same layouts as pgsag_outputs; NULL = zero.
 * Values at unmasked pixels are ignored.  count: dL/ds [H][W] for the soft
 * contributor count s = sum of alpha over the fragments blended at the
 * pixel -- the differentiable stand-in for the integer count g_i of Eq. 9
 * (Sec. 4.3), through which the balance-load term's gradient flows; s
 * itself is not an output. */
typedef struct pgsag_grad_outputs {
  const float *rgb, *normal, *dist, *depth, *alpha, *count;
} pgsag_grad_outputs;

typedef struct pgsag_render {
  int32_t set; /* index of the Gaussian set this render draws */
  int32_t reserved;
  pgsag_camera cam;
  const uint8_t *mask; /* device [H][W], non-zero = building pixel; NULL = all */
  pgsag_outputs out;
  pgsag_grad_outputs gout;
} pgsag_render;

typedef struct pgsag_config {
  int32_t tile;        /* 8, 16 or 32 (pixels per tile side) */
  int32_t persistent;  /* 1: persistent workgroups pulling an LPT tile queue */
  int32_t queue_chunk; /* tiles fetched per queue pop (1..64) */
  int32_t workgroups_per_cu; /* persistent grid = 256 CUs x this (1..16) */
  float alpha_min;  /* 1/255 */
  float t_min;      /* 1e-4 */
  float alpha_max;  /* 0.99 */
  float dilation;   /* 0.3 */
  float z_near;     /* 0.2 */
  float fov_clamp;  /* 1.3 */
  float logit_min;  /* float32(-ln 254) */
  float depth_guard; /* 1e-6 */
  float bg[3];      /* 0, 0, 0 */
  /* How the backward compositing pass sums each record's 13 per-pixel
     gradient terms over a wave (same sums, different speed):
     0: matrix cores -- the wave buffers 8 records' per-pixel weights in LDS
        and contracts them with the pixels' features in FP32 MFMA steps
        (fewer instructions per record; best for long tile lists);
     1: lane exchanges -- each record is reduced at once across the wave
        (less work per tile, twice the resident workgroups; best for short
        tile lists).  Any other value is an error. */
  int32_t bwd_reduce;
  /* 0: the backward compositing pass adds each wave's per-record sums to
        the record's 2D-gradient slot with float atomics, so the gradients
        can differ in the last bits from run to run (addition order);
     1: deterministic -- every (tile pair, wave) writes its sums to a slot of
        its own, and a segmented reduction then adds each record's slots in
        a fixed order (its tiles in row-major order, waves in index order).
        Gradients are then bit-identical from run to run, between a batch
        and the same renders launched one by one, and between the plain and
        the persistent launch.  Costs workspace (4 + 64 x (tile/8)^2 bytes
        per pair of capacity) and about twice the backward time.
     Any other value is an error. */
  int32_t deterministic;
} pgsag_config;

typedef struct pgsag_plan_info {
  uint64_t workspace_bytes; /* device workspace the batch needs */
  uint64_t desc_bytes;      /* size of the packed descriptor */
  uint64_t n_records;       /* sum over renders of the set size */
  uint64_t n_tiles;         /* sum over renders of tiles_x * tiles_y */
  uint64_t n_pixels;        /* sum over renders of W * H */
  uint64_t pair_capacity;   /* (tile, Gaussian) pairs the workspace holds */
  int32_t tile_bits;        /* bits of the global tile id */
  int32_t reserved;
} pgsag_plan_info;

/* Byte offsets of the workspace regions (for inspection by tests). */
typedef struct pgsag_layout {
  uint64_t status;     /* uint64 pairs_needed, uint32 overflow, uint32 n_visible */
  uint64_t tile_count; /* uint32 [n_tiles] masked pixels per tile */
  uint64_t sat;        /* uint32 per-tile-row prefix counts of active tiles */
  uint64_t ranges;     /* uint32 [n_tiles][2] [start, end) into the pairs */
  uint64_t queue;      /* uint32 [n_tiles] tile work queue (LPT order) */
  uint64_t records;    /* float [n_records][16] projected records */
  uint64_t depth_key;  /* uint32 [n_records] FP32 depth key bits */
  uint64_t rect;       /* uint16 [n_records][4] tile rect x0, y0, x1, y1 */
  uint64_t n_active;   /* uint32 [n_records] active tiles in the rect */
  uint64_t pair_tile;  /* uint32 [capacity] sorted pair tile ids */
  uint64_t pair_record; /* uint32 [capacity] sorted pair record ids */
  uint64_t pixel_T;    /* float [n_pixels] final transmittance */
  uint64_t pixel_last; /* int32 [n_pixels] last blended pair index, -1 none */
  uint64_t grad2d;     /* float [n_records][16] per-record pixel sums of the backward compositing pass */
  uint64_t work;       /* uint32 [n_tiles][(tile/8)^2][3] per (tile, 8x8-pixel wave): list entries the
                          forward compositing evaluated, entries the backward evaluated, and backward
                          entries with at least one contributing pixel (each entry is evaluated for all
                          64 pixels of the wave); written by every forward / backward */
  uint64_t end;
} pgsag_layout;

typedef struct pgsag_status {
  uint64_t pairs_needed; /* pairs the last forward/binning emitted or needed */
  uint32_t overflow;     /* 1 if pairs_needed > capacity (outputs invalid) */
  uint32_t n_visible;    /* records with at least one active tile */
  uint32_t error;        /* non-zero if a single-pass scan of the binning gave
                            up waiting for a predecessor's prefix (a bounded
                            wait): that pass's outputs are invalid */
  uint32_t reserved;
} pgsag_status;

/* PGSAG_ABI_VERSION of the loaded library. */
int pgsag_version(void);

/* Thread-local description of the last failure on this thread. */
const char *pgsag_last_error(void);

/* Fills *cfg with the defaults listed in pgsag_config. */
void pgsag_default_config(pgsag_config *cfg);

/* Sizes the workspace and descriptor of a batch (host only, no device
 * work).  sets[n_sets] and renders[n_renders] are read for their sizes;
 * pair_capacity is the maximum number of (tile, Gaussian) pairs (1..2^30-1).
 * Returns INVALID_ARGUMENT for n_sets < 1, n_renders < 1, a render whose set
 * index is out of range, width/height < 1 or > 65535 pixels, sh_degree
 * outside 0..3, tile not in {8,16,32}, bwd_reduce or deterministic not 0/1,
 * n < 0; UNSUPPORTED for more than 4096 renders, more than 64 renders of
 * one set, 2^30 or more records or 2^32-1 or more tiles in the batch. */
int pgsag_plan(const pgsag_config *cfg, const pgsag_gaussians *sets, int32_t n_sets,
               const pgsag_render *renders, int32_t n_renders, uint64_t pair_capacity,
               pgsag_plan_info *out);

/* Packs the batch into host_desc[desc_bytes] (host memory).  The caller
 * copies these bytes to a device buffer (dev_desc) before forward/backward;
 * device pointers inside stay valid for as long as the caller keeps the
 * buffers alive, so a captured graph may replay with the same descriptor.
 * set_grads may be NULL (no backward).  Same validation as pgsag_plan, plus
 * non-NULL parameter pointers for n > 0 and depth gradients requiring the
 * normal and dist outputs. */
int pgsag_pack(const pgsag_config *cfg, const pgsag_gaussians *sets,
               const pgsag_grads *set_grads, int32_t n_sets, const pgsag_render *renders,
               int32_t n_renders, uint64_t pair_capacity, void *host_desc,
               size_t desc_bytes);

/* Workspace byte offsets of a packed batch. */
int pgsag_layout_of(const void *host_desc, pgsag_layout *out);

/* Forward pass (Sec. 3.1, Eq. 1-4) of every render of the batch: tile-mask
 * reduce, projection, depth sort, tile binning, tile sort, compositing and
 * the depth epilogue.  host_desc: the packed bytes (host); dev_desc: their
 * device copy; workspace: device buffer of at least workspace_bytes, left
 * untouched by the caller until pgsag_backward; stream: hipStream_t or NULL;
 * events: NULL or 2*PGSAG_NUM_STAGES hipEvent_t recorded around the stages. */
int pgsag_forward(const void *host_desc, const void *dev_desc, void *workspace,
                  size_t workspace_bytes, void *stream, void **events);

/* Backward pass: gradients of L = sum over renders, masked pixels and
 * channels of gout * output with respect to the raw parameters of every set
 * (overwritten, summed over the set's renders).  Must follow the forward of
 * the same batch on the same workspace; recomputes the per-pixel blending
 * state from the saved final transmittance and last index instead of storing
 * per-fragment alphas. */
int pgsag_backward(const void *host_desc, const void *dev_desc, void *workspace,
                   size_t workspace_bytes, void *stream, void **events);

/* Tile binning alone (the integer stages of Sec. 3.1: tile assignment and
 * sorting): reads per-record tile rects, depth keys and validity that the
 * caller has written into the workspace (layout: rect, depth_key, and
 * n_active != 0 meaning valid), recounts active tiles from the masks,
 * compacts, depth sorts, emits pairs, tile sorts and builds the ranges.
 * For testing the binning against a reference on chosen inputs. */
int pgsag_binning(const void *host_desc, const void *dev_desc, void *workspace,
                  size_t workspace_bytes, void *stream);

/* Copies the status word of the last forward (or binning) to *out and
 * synchronises the stream.  The outputs of that pass are valid only when
 * both out->overflow and out->error are 0. */
int pgsag_read_status(const void *host_desc, const void *workspace, pgsag_status *out,
                      void *stream);

/* Fused Adam update over n floats (device pointers, any alignment of 4
 * bytes): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * step >= 1.  (The paper does not name its optimiser; this is the one the
 * 3DGS family uses.) */
int pgsag_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                    float lr, float b1, float b2, float eps, int32_t step, void *stream);

/* The same update with the step count kept on the device, for a training
 * step captured once in a HIP graph and replayed: state is device int32[4]
 * owned by the caller, state[0] = steps taken so far (0 before the first;
 * incremented by this call before the update), state[1..2] receive the
 * step's bias corrections 1/(1 - b1^t), 1/(1 - b2^t) as floats. */
int pgsag_adam_step_device(float *params, const float *grads, float *m, float *v, int64_t n, float lr, float b1,
                           float b2, float eps, int32_t *state, void *stream);

/* Adam folded into the backward pass (see pgsag_backward_adam). */
typedef struct pgsag_adam_config {
  float lr, b1, b2, eps;   /* as for pgsag_adam_step */
  int32_t *step_state;     /* device int32[4], as for pgsag_adam_step_device */
  int64_t m_offset;        /* first moment of every parameter array: its gradient pointer + m_offset floats */
  int64_t v_offset;        /* second moment: gradient pointer + v_offset floats */
  int32_t write_grads;     /* non-zero: also store the gradients at the gradient pointers */
  int32_t reserved;
} pgsag_adam_config;

/* pgsag_backward followed, inside the backward projection kernel, by the
 * Adam update of pgsag_adam_step_device applied to every raw-parameter array
 * that has a gradient pointer in the descriptor: the parameters are updated
 * IN PLACE (the descriptor's parameter pointers are written), the moments
 * live at the gradient pointer plus m_offset / v_offset floats (the same
 * layout as the gradients, e.g. three equal slices of one buffer), and the
 * gradients themselves are stored only with write_grads.  Saves the
 * gradient round trip through memory and a second read of the parameters
 * (the separate update reads p, g, m, v and writes p, m, v).  Same stream,
 * capture and ownership rules as pgsag_backward. */
int pgsag_backward_adam(const void *host_desc, const void *dev_desc, void *workspace, size_t workspace_bytes,
                        const pgsag_adam_config *adam, void *stream, void **events);

/* Balance-load statistics of the last forward (Sec. 4.3, Eq. 9): per
 * render, over tiles with at least one masked pixel, the mean and the
 * population variance of the per-tile pair counts, and over masked pixels
 * the mean and population standard deviation of n_contrib / w where
 * w = pixel_weight (device [H][W] per render, NULL = 1).  out: device float
 * [n_renders][4] = {tile mean, tile variance, pixel mean, pixel std}. */
int pgsag_load_stats(const void *host_desc, const void *dev_desc, const void *workspace,
                     const float *const *pixel_weight, float *out, void *stream);

/* Weights of the training losses on the rendered outputs (Sec. 4.2 Eq. 8,
 * Sec. 4.3 Eq. 11).  Defaults from pgsag_default_loss_config. */
typedef struct pgsag_loss_config {
  float lambda_rgb;      /* weight of the masked L1 colour term: 1 */
  float lambda_normal;   /* weight of the boundary-aware normal term: 0.01 */
  float boundary_weight; /* normal-term weight on mask-boundary pixels: 0.1 */
  float lambda_load;     /* lambda of Eq. 11 (balance-load share): 0 */
  int32_t normal_norm;   /* 1 = L1 (default), 2 = squared L2 (Eq. 8 as printed) */
  float normal_eps;      /* rendered normals with |N| <= eps take no part: 1e-6 */
  int32_t load_term;     /* the balance-load term L_load of Eq. 11:
                            0 (default): variance of the pair counts over tiles
                              holding masked pixels, a value only;
                            1: the GC-load of Eq. 9, std over masked pixels of
                              n_contrib / w, with its gradient taken through the
                              soft count (see pgsag_grad_outputs.count) */
  int32_t reserved;
} pgsag_loss_config;

void pgsag_default_loss_config(pgsag_loss_config *lc);

/* Loss of the last forward of the batch and its gradient with respect to
 * the rendered planes (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 11).  Per render, with
 * M its masked pixels:
 *   L_rgb = (1/3M) sum over masked pixels and channels |rgb - gt|
 *   L_ban = (1/M) sum over masked pixels where both normals exist of
 *           w * ||n_depth - N/|N|||  (L1 or squared L2), w = boundary_weight
 *           on masked pixels with an unmasked 4-neighbour inside the image,
 *           1 elsewhere; n_depth = normalize(dPy x dPx) from the points
 *           depth * K^-1 p~ of masked pixels with depth > 0, central
 *           differences along x and y with a missing neighbour replaced by
 *           the pixel itself; it exists where the pixel has a neighbour
 *           along each axis; N is used where |N| > normal_eps
 *   L     = (1 - lambda_load)(lambda_rgb L_rgb + lambda_normal L_ban)
 *           + lambda_load * L_load
 *   L_load = (load_term 0) Var(pair counts over tiles holding masked
 *           pixels), a value only: zero gradient;
 *           (load_term 1) the GC-load of Eq. 9: sigma = population std over
 *           masked pixels of x = n_contrib / w, w = pixel_weight[r] (NULL
 *           array or entry = 1; e.g. pgsag_luminance_weights).  Its gradient
 *           is taken through the soft count s (straight through the integer
 *           count): dL/ds = lambda_load (x - mean x) / (M sigma w), 0 when
 *           sigma = 0.
 * Reads each render's rgb, normal and depth outputs (required; n_contrib
 * too with load_term 1) and gt_rgb[r] (host array of n_renders device
 * pointers to [3][H][W]).  Writes dL/d(rgb, normal, depth) into the
 * render's grad-output planes (required; the descriptor's const pointers
 * are written here), 0 into its dist and alpha grad-output planes if
 * present, and dL/ds into its count plane (required with load_term 1;
 * written 0 with load_term 0 if present), at masked pixels only: other
 * pixels are left as they are (the backward ignores them).  loss: device
 * float [n_renders][4] = {L, L_rgb, L_ban, L_load}.  Needs the workspace of
 * the preceding pgsag_forward.  Capturable. */
int pgsag_loss(const pgsag_loss_config *lc, const void *host_desc, const void *dev_desc, void *workspace,
               uint64_t workspace_bytes, const float *const *gt_rgb, const float *const *pixel_weight, float *loss,
               void *stream);

/* Per-pixel weights w_i of the gradient-constrained balance-load term
 * (Sec. 4.3 Eq. 9), a reading of its "gradient-dependent weight":
 * w = 0.1 + |grad Y| / mean over masked pixels of |grad Y|, Y = 0.299 R +
 * 0.587 G + 0.114 B of the ground truth (device [3][H][W] of render
 * `render`), gradients by central differences inside the image and
 * one-sided differences on its border; w = 1 everywhere when that mean is
 * 0.  weight: device float [H][W], every pixel written.  Feed it to
 * pgsag_load_stats and pgsag_loss as pixel_weight.  Uses the workspace's loss
 * accumulators of that render. */
int pgsag_luminance_weights(const void *host_desc, const void *dev_desc, void *workspace, uint64_t workspace_bytes,
                            int32_t render, const float *gt_rgb, float *weight, void *stream);

/* ------------------------------------------------------------------------
 * Building-point voting (Sec. 4.1, "Reliability-scored Multi-view Voting
 * Filter", Eq. 6-7).  SfM sparse points are re-projected into every coarsely
 * masked view.  Point p is in Image_j when its camera-frame depth exceeds
 * z_near and its projection lies inside the image, and in M_j when it is in
 * Image_j and the mask pixel under the projection is non-zero:
 *   votes(p) = sum_j I(p in M_j)                  (Eq. 6: potential building
 *                                                  point iff votes > 0)
 *   US(p)    = sum_j I(p in Image_j \ M_j)        (Eq. 7: unreliability score)
 *   flags(p) = bit 0: votes > 0; bit 1: votes > 0 and US < tau (reliable).
 * The projection is taken in FP32 with every operation rounded on its own,
 * in this order: xc = ((R00 x + R01 y) + R02 z) + t0 (likewise yc, zc);
 * in front iff zc > z_near; u = fx (xc / zc) + cx, v = fy (yc / zc) + cy
 * (correctly rounded division); inside iff 0 <= u < W and 0 <= v < H; the
 * pixel is (floor u, floor v).  No occlusion test. */
typedef struct pgsag_vote_view {
  pgsag_camera cam;
  const uint8_t *mask; /* device [H][W], non-zero = building pixel; NULL = every pixel */
} pgsag_vote_view;

/* host_views and dev_views hold the same n_views views (the host copy is
 * read for validation, the device copy by the kernel; the caller uploads
 * it).  points: device float [3][n_points] (planar x, y, z).  votes, us:
 * device uint16 [n_points] or NULL (not wanted); flags: device uint8
 * [n_points], required.  1 <= n_views <= 65535 (the counts are 16-bit),
 * n_points >= 0, tau >= 0, z_near > 0, image sizes 1..65535.  Every output
 * element is written.  No allocation, no synchronisation; capturable. */
int pgsag_vote(const pgsag_vote_view *host_views, const pgsag_vote_view *dev_views, int32_t n_views,
               const float *points, int64_t n_points, float z_near, int32_t tau, uint16_t *votes,
               uint16_t *us, uint8_t *flags, void *stream);

/* ------------------------------------------------------------------------
 * Building grouping (Sec. 4.1, "Building Grouping"): DBSCAN (the clustering
 * the paper names) over the ground-plane coordinates (x, y) of the points
 * that take part -- e.g. the reliable building points of pgsag_vote -- and
 * the views each group keeps.
 *   N(p)    = points q taking part with d2 = dx*dx + dy*dy <= eps*eps, in
 *             FP32 with every operation rounded on its own (dx = px - qx,
 *             dy = py - qy); p itself included
 *   core    = |N(p)| >= min_pts
 *   cluster = connected component of core points joined within eps, named
 *             by its smallest core point index
 *   border  = non-core point with a core neighbour: it takes the smallest
 *             name among its core neighbours' clusters (DBSCAN leaves the
 *             choice to the visiting order; this rule makes it unique)
 *   noise   = label -1; points that take no part also get -1 (and count 0) */

/* Device workspace bytes for pgsag_dbscan over n_points points
 * (0 <= n_points <= 2^23). */
int pgsag_dbscan_workspace(int64_t n_points, uint64_t *bytes);

/* points: device float [3][n_points] (x, y used; planar).  A point takes
 * part when flags is NULL or (flags[i] & flag_mask) != 0 (flags: device
 * uint8 [n_points], e.g. pgsag_vote's flags with flag_mask 2 = reliable).
 * eps > 0 (finite), min_pts >= 1.  Outputs (device, every element written):
 * count int32 [n] = |N(p)| (0 for points taking no part; NULL = not
 * wanted), label int32 [n] = cluster name or -1, cluster int32 [n] =
 * compact id 0..k-1 in ascending order of the names or -1 (NULL = not
 * wanted), n_clusters uint32 [1] = k.  workspace: device buffer of
 * pgsag_dbscan_workspace bytes, owned by the caller, scratch only (no state
 * kept between calls).  No allocation, no synchronisation; capturable. */
int pgsag_dbscan(const float *points, int64_t n_points, const uint8_t *flags, uint32_t flag_mask, float eps,
                 int32_t min_pts, int32_t *count, int32_t *label, int32_t *cluster, uint32_t *n_clusters,
                 void *workspace, uint64_t workspace_bytes, void *stream);

/* The scratch of pgsag_dbscan_static: up to this many points. */
#define PGSAG_DBSCAN_STATIC_MAX_POINTS (1 << 19)

/* pgsag_dbscan without a workspace argument, for callers that cannot
 * allocate device memory (work under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * validation as pgsag_dbscan, with n_points limited to
 * PGSAG_DBSCAN_STATIC_MAX_POINTS (more: INVALID_ARGUMENT, nothing
 * launched).  The scratch is a static device array of the library
 * (23,609,600 bytes) that each GPU it runs on holds from its first call there until the
 * process ends; its device address is looked up on that first call, on the
 * current device, which must be the device of `stream`.  Every call on one
 * GPU shares that GPU's array (the kernels rewrite what they read in each
 * call): calls that overlap on one GPU -- on different streams or from
 * different threads -- race and give wrong results.  No allocation, no
 * synchronisation. */
int pgsag_dbscan_static(const float *points, int64_t n_points, const uint8_t *flags, uint32_t flag_mask, float eps,
                        int32_t min_pts, int32_t *count, int32_t *label, int32_t *cluster, uint32_t *n_clusters,
                        void *stream);

/* Views of each group ("subgroups that each contain the ... original
 * images", Sec. 4.1): hits[c][j] = points with cluster id c that land inside
 * view j's building mask, with the projection of pgsag_vote; assigned[c][j]
 * = hits >= min_hits.  cluster: device int32 [n_points] compact ids (< 0 =
 * none; ids >= max_clusters are ignored, so size max_clusters from
 * pgsag_dbscan's n_clusters).  hits: device uint32 [max_clusters][n_views];
 * assigned: device uint8 [max_clusters][n_views] or NULL.  Views as for
 * pgsag_vote.  No allocation, no synchronisation; capturable. */
int pgsag_group_views(const pgsag_vote_view *host_views, const pgsag_vote_view *dev_views, int32_t n_views,
                      const float *points, int64_t n_points, const int32_t *cluster, int32_t max_clusters,
                      float z_near, uint32_t min_hits, uint32_t *hits, uint8_t *assigned, void *stream);

/* ------------------------------------------------------------------------
 * Depth fusion and TSDF integration (Sec. 4.4, "Mesh Extraction and
 * Merge"): the depth maps several groups render from one view (the depth
 * output of pgsag_forward) are merged by their mean where they overlap, and
 * the fused maps of many views are integrated into a truncated signed
 * distance volume (the TSDF method the paper cites).  Meshing itself is not
 * part of this library. */

/* Mean fusion of n_maps (1..64) depth maps of one view: for every pixel,
 * over the maps with depth > 0 in their given order, s = s + depth (FP32,
 * each addition rounded), fused = s / (their number) (one rounded
 * division), 0 where none has a depth.  depths: host array of n_maps device
 * pointers to float [height][width]; fused: device float [height][width];
 * count: device uint8 [height][width] (maps with a depth) or NULL.  Every
 * element written.  No allocation, no synchronisation; capturable. */
int pgsag_fuse_depth(const float *const *depths, int32_t n_maps, int32_t width, int32_t height, float *fused,
                     uint8_t *count, void *stream);

typedef struct pgsag_volume {
  float origin[3]; /* world position of the volume's corner */
  float voxel;     /* voxel side (> 0) */
  int32_t nx, ny, nz; /* voxels per side (0..2^23); storage [nz][ny][nx] */
  float trunc;     /* truncation distance (> 0) */
} pgsag_volume;

typedef struct pgsag_depth_view {
  pgsag_camera cam;
  const float *depth; /* device float [H][W] (e.g. a fused map), 0 = no depth */
} pgsag_depth_view;

/* Projective TSDF with unit weights over n_views (0..65535) views.  Voxel
 * (i, j, k) has the centre c = ((i + 0.5) voxel + origin_x, ...) (FP32, each
 * operation rounded).  A view sees c when, with the projection of
 * pgsag_vote, c is in front (zc > z_near) and inside the image, the depth D
 * at its pixel is > 0 and sdf = D - zc >= -trunc; it then adds
 * min(1, sdf / trunc) with weight 1.  accumulate = 0: tsdf = (sum of the
 * added values) / W and weight = W (the number of views that saw the
 * voxel), tsdf = 1 and weight = 0 where none did.  accumulate = 1: a running
 * average continuing from the values already in tsdf and weight, tsdf =
 * (W0 tsdf0 + sum) / (W0 + W), weight = W0 + W (voxels no view saw keep
 * theirs).  tsdf, weight: device float [nz][ny][nx].  host_views and
 * dev_views hold the same views (host copy validated, device copy read).
 * No allocation, no synchronisation; capturable. */
int pgsag_tsdf_integrate(const pgsag_volume *vol, const pgsag_depth_view *host_views,
                         const pgsag_depth_view *dev_views, int32_t n_views, float z_near, float *tsdf,
                         float *weight, int32_t accumulate, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PGSAG_H */
