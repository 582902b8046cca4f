/*
 * rogs.h -- C ABI of librogs, differentiable tile-based splatting of meshgrid
 * Gaussian surfels (RoGs, arXiv 2405.14342) on AMD MI355X (gfx950).
 *
 * The library renders 2D Gaussian surfels (Sec. 3.1, Eq. 1-3: covariance
 * R S S^T R^T with s_z = 0) into camera images with the EWA projection of
 * Eq. 5, sorts them by view depth and alpha-composites colour, semantic
 * logits, depth and alpha front to back (Eq. 6), evaluates the masked L1 and
 * cross-entropy losses with per-camera exposure (Eq. 7-9, Eq. 12), runs the
 * adjoint of all of that, and applies Adam (Sec. 4.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  Every array argument is a DEVICE pointer owned by the caller,
 *    except the structs themselves and `rogs_camera` arrays, which live in
 *    host memory and are read during the call.  The library allocates no
 *    device memory in these calls: scratch space is one caller-provided
 *    workspace whose size `rogs_workspace_size` returns.  The context owns
 *    a small pinned host buffer and a few events.
 *  - Streams.  `stream` is a hipStream_t (NULL = the null stream).  Calls
 *    enqueue work and return without waiting, except where a flag asks for
 *    a host read-back (ROGS_SYNC_COUNT).
 *  - Errors.  Every call returns ROGS_OK (0) or a negative status; the text
 *    of the last error is kept in the context (`rogs_last_error`).  No
 *    exception crosses the ABI.  A context is used by one host thread at a
 *    time.  Invalid arguments are rejected before any GPU work is enqueued.
 *  - Parameter layout.  Surfel parameters are structure-of-arrays FP32,
 *    component-major: q[4][N] (w, x, y, z), s[2][N], rgb[3][N], sem[C][N].
 *  - Packed parameter block (gradients and Adam): K = 11 + C rows of N
 *    floats each, in the row order
 *        0 z | 1-4 q(w,x,y,z) | 5-6 s (log-scale for Adam) |
 *        7 alpha (logit for Adam) | 8-10 rgb | 11.. 11+C-1 sem
 *  - Image layout.  Views of a batch are packed one after another; view v
 *    starts at pixel offset P_v = sum_{u<v} W_u H_u.  A per-pixel image with
 *    K channels stores channel c of pixel (x, y) of view v at
 *        K * P_v + c * W_v * H_v + y * W_v + x.
 *    Rendered images have K = 5 + C channels: R, G, B, sem[0..C-1], D, A.
 *
 * Key contract
 * ------------
 * Everything that decides an integer (culling, tile rectangles, the depth
 * sort key, whether a pixel is touched by a surfel) follows this sequence on
 * every implementation.  The projection is computed in IEEE binary64 from the
 * binary32 inputs (promoted exactly), round to nearest even, without fused
 * multiply-add, with correctly rounded division and square root, exactly in
 * this order ("a*b + c*d" means round(round(a*b) + round(c*d))):
 *
 *   tx = ((R0*x + R1*y) + R2*z) + t0,  ty, tz likewise with rows 1, 2
 *   visible needs tz >= z_near; if cull_lat > 0 also, with dx = x - o0,
 *     dy = y - o1: |dx*ex0 + dy*ex1| <= cull_lat and
 *     0 <= dx*ez0 + dy*ez1 <= cull_fwd     (ground rectangle, supp. Sec. 2.1)
 *   nn = ((qw*qw + qx*qx) + qy*qy) + qz*qz > 0;  n = sqrt(nn);
 *   w = qw/n, a = qx/n, b = qy/n, c = qz/n
 *   r1 = (1 - 2*(b*b + c*c), 2*(a*b + w*c), 2*(a*c - w*b))
 *   r2 = (2*(a*b - w*c), 1 - 2*(a*a + c*c), 2*(b*c + w*a))
 *   T1 = s_x*r1, T2 = s_y*r2;  c1_k = (Rk0*T1_0 + Rk1*T1_1) + Rk2*T1_2, c2 likewise
 *   pinhole: limx = (0.65*W)/fx, limy = (0.65*H)/fy, xr = tx/tz, yr = ty/tz,
 *            xc = min(max(xr, -limx), limx), yc likewise,
 *            j00 = fx/tz, j11 = fy/tz, j02 = -(j00*xc), j12 = -(j11*yc),
 *            u = fx*xr + cx, v = fy*yr + cy
 *   ortho:   j00 = fx, j11 = fy, j02 = j12 = 0, u = fx*tx + cx, v = fy*ty + cy
 *   m00 = j00*c1_0 + j02*c1_2, m01 = j00*c2_0 + j02*c2_2,
 *   m10 = j11*c1_1 + j12*c1_2, m11 = j11*c2_1 + j12*c2_2
 *   g0 = m00*m00 + m01*m01, g1 = m10*m10 + m11*m11,
 *   s00 = g0 + eps, s11 = g1 + eps, s01 = m00*m10 + m01*m11,
 *   dm = m00*m11 - m01*m10, det = (dm*dm + eps*(g0 + g1)) + eps*eps > 0
 *   conic A = s11/det, B = -(s01/det), C = s00/det
 *   hx = sqrt(q_cut*s00) + 1, hy = sqrt(q_cut*s11) + 1
 *   tile rect: x0 = floor((u - hx)/tile_w), x1 = floor((u + hx)/tile_w) + 1,
 *              y0, y1 likewise; each clamped to [0, tiles]; needs x0<x1, y0<y1
 *              (and u, v, hx, hy, A, B, C finite)
 * The record keeps binary32 roundings: u_hi = f32(u), u_lo = f32(u - u_hi),
 * v_hi, v_lo likewise, A, B, C = f32(A), ..., t_z = f32(tz).
 *   sort key  = (global tile index << 32) | bit pattern of f32(tz), ties by id
 * Tiles of a slot: in each rectangle row ty, the tiles [lo, hi) whose pixel
 * columns the ellipse q <= q_cut * (1 + 2^-18 / (1 - rho)), rho = |B| /
 * sqrt(A C), reaches over the row's pixel-centre rows (binary64 from the
 * record, one rounding per step): a = (ty*tile_h + 0.5) - v, b = (min((ty +
 * 1)*tile_h, h) - 0.5) - v clipped to +-dym, dym = sqrt((A*qe)/det), det =
 * A*C - B*B; the extreme points dy* = +-B*sqrt(qe/(C*det)) clamped to [a, b];
 * x = u + (-(B*dy*) -+ sqrt(max(0, A*qe - det*dy*^2)))/A; columns ceil(xl -
 * 0.5) .. floor(xr - 0.5) clipped to the image; tiles by integer division,
 * clipped to [x0, x1).  A conic with 1 - rho < 2^-16 or det <= 0 keeps the
 * whole rectangle row.
 * Per pixel, in binary32: dx = ((px + 0.5) - u_hi) - u_lo, dy likewise,
 *   q32 = fma(dx, fma(A, dx, (2*B)*dy), (C*dy)*dy); the pixel is touched iff
 *   q32 <= q_cut.
 *
 * Values (Eq. 6): for touched pixels g = exp(-q/2), a = min(alpha*g,
 * alpha_max), w = a*T, O += w*f for f in (rgb, sem, tz), T *= 1 - a; a pixel
 * stops after the surfel that takes T below t_eps; A = 1 - T.
 */
#ifndef ROGS_H
#define ROGS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ROGS_API __attribute__((visibility("default")))
#else
#define ROGS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status */
#define ROGS_OK          0
#define ROGS_NOT_READY   1   /* serve poll: result not finished yet */
#define ROGS_EINVAL     -1   /* invalid argument (nothing enqueued) */
#define ROGS_ENOMEM     -2   /* workspace or arena too small */
#define ROGS_ECAPACITY  -3   /* pair buffer too small; needed size reported */
#define ROGS_EHIP       -4   /* a HIP runtime call failed */
#define ROGS_EREJECT    -5   /* serve admission rejected the request */
#define ROGS_ESTATE     -6   /* call out of order (e.g. bin_sort before project) */

#define ROGS_PINHOLE 0
#define ROGS_ORTHO   1

/* flags */
#define ROGS_SYNC_COUNT   1u  /* rogs_bin_sort: read the pair count back (host sync) */
#define ROGS_ACCUMULATE   2u  /* rogs_render_bwd: add into grads instead of overwriting */

typedef struct rogs_ctx rogs_ctx;

/* Surfel parameters in the render domain (activated s and alpha), device SoA.
 * Eq. 3: Theta = {(x, y, z), (r, g, b), (s_x, s_y), alpha, R, Sem}; x, y are
 * the fixed grid vertices (Sec. 3.1, meshgrid layout), the rest learnable. */
typedef struct {
  int32_t n;            /* number of surfels N (>= 1) */
  int32_t n_sem;        /* semantic classes C (1..8 or 16) */
  const float* x;       /* [N] grid vertex x (m) */
  const float* y;       /* [N] grid vertex y (m) */
  const float* z;       /* [N] height (m) */
  const float* q;       /* [4][N] rotation quaternion w, x, y, z (not necessarily unit) */
  const float* s;       /* [2][N] scales s_x, s_y > 0 (m) */
  const float* alpha;   /* [N] opacity in (0, 1) */
  const float* rgb;     /* [3][N] colour */
  const float* sem;     /* [C][N] semantic logits */
} rogs_surfels;

/* One view (host memory).  OpenCV camera: x right, y down, z forward;
 * camera-space point t = R_cw * mu + t_cw.  Pinhole: fx, fy, cx, cy in
 * pixels.  Orthographic (Sec. 3.3.1, J = identity): fx, fy in pixels per
 * metre.  The ground cull rectangle (supp. Sec. 2.1) is given by its origin
 * (camera centre xy), unit ground directions of the camera x and z axes, a
 * half-width and a forward length; cull_lat <= 0 disables it.
 * tile: 0 renders the view in the options' tile shape; otherwise
 * tile_w | tile_h << 16 gives this view its own shape, of the same area
 * (tile_w * tile_h) as the options' and with tile_w dividing 64
 * (ROGS_EINVAL otherwise).  Every shape renders the same values; rogs_autotune
 * chooses shapes per resolution class this way. */
typedef struct {
  int32_t w, h;         /* image size, 1..16384 */
  int32_t model;        /* ROGS_PINHOLE or ROGS_ORTHO */
  int32_t tile;         /* 0, or this view's tile_w | tile_h << 16 */
  float fx, fy, cx, cy;
  float R_cw[9];        /* row-major */
  float t_cw[3];
  float z_near;
  float cull_o[2], cull_ex[2], cull_ez[2];
  float cull_lat, cull_fwd;
} rogs_camera;

typedef struct {
  int32_t tile_w, tile_h;  /* tile shape; tile_w in {1,2,...,64} dividing 64 and
                              tile_w*tile_h in {64, 128, 256}; default 16 x 16 */
  float eps2d;             /* EWA low-pass added to Sigma' (px^2), default 0.3 */
  float q_cut;             /* Mahalanobis cut, default 9 (3 sigma) */
  float alpha_max;         /* opacity clamp, default 0.99 */
  float t_eps;             /* termination threshold on T, default 1e-6 */
  int32_t stage;           /* list entries the compositing waves stage in LDS per
                              batch: 16, 32 or 64 (0 means 32, the default).
                              Values are the same for each; only speed differs. */
} rogs_render_opts;

/* Loss targets of a batch (Eq. 8, 9), device arrays in the image layout. */
typedef struct {
  const float* rgb;        /* [3 channels per view] target colour */
  const uint8_t* label;    /* [1 channel per view] class index < C */
  const uint8_t* mask;     /* [1 channel per view] 1 = road pixel (M), 0 = ignored */
  const float* exposure;   /* [V][2] per-view (a, b) of Eq. 7 */
  float lambda_c;          /* Eq. 12 weight of L_c (paper: 1) */
  float lambda_s;          /* Eq. 12 weight of L_s (paper: 0.06) */
  float view_scale;        /* multiplies every view's loss (1 / total views) */
  /* Grid-side terms of Eq. 12, applied by rogs_step_fused (the plain path
   * calls rogs_elev_loss); rogs_loss ignores them. */
  const int32_t* nbr;      /* [4][N] neighbour table of Eq. 10 (up, down, left, right;
                              own index where there is none; symmetric), or NULL */
  const float* zbar;       /* [N] LiDAR elevation targets of Eq. 11, or NULL */
  float lambda_smooth;     /* Eq. 12 weight of L_smooth (paper: 0.003; 1 with LiDAR) */
  float lambda_z;          /* Eq. 12 weight of L_z (paper: 0.02) */
} rogs_targets;

/* Per-group Adam learning rates (Sec. 4.2). */
typedef struct {
  float z, q, s, alpha, rgb, sem, exposure;
} rogs_lr;

/* Optimiser settings (Sec. 4.2): per-group rates, and the height rate
 * z(t) = z_start (z_end / z_start)^t, t = (step - 1) / (total_steps - 1)
 * clamped to [0, 1] (log-linear from z_start to z_end over the run; the
 * paper sets it proportional to the scene size, 1.6e-4 to 1.6e-6 of it);
 * total_steps = 1 uses z_start, total_steps = 0 the constant lr.z.
 * beta1, beta2 in [0, 1), eps > 0. */
typedef struct {
  rogs_lr lr;            /* per-group rates (lr.z used only when total_steps == 0) */
  float z_start, z_end;  /* height rate at the first and at the last step (> 0) */
  int64_t total_steps;   /* length of the height schedule; 0 = constant lr.z */
  float beta1, beta2, eps;
} rogs_optim;

/* ------------------------------------------------------ context */
ROGS_API int rogs_create(rogs_ctx** ctx);
ROGS_API void rogs_destroy(rogs_ctx* ctx);
ROGS_API const char* rogs_last_error(const rogs_ctx* ctx);
/* Fills opts with the defaults listed above. */
ROGS_API void rogs_default_opts(rogs_render_opts* opts);

/* Bytes of workspace for a batch of n_views cameras over s->n surfels with
 * room for pair_capacity (surfel, tile) pairs and slot_capacity visible
 * (view, surfel) slots (0 = pair_capacity; at most pair_capacity, since
 * every visible slot has at least one pair).  Host-only computation.  Kernels
 * that wait for a count kept on the device are sized by these capacities, so
 * capacities close to the real counts launch fewer idle blocks. */
ROGS_API int rogs_workspace_size(const rogs_surfels* s, const rogs_camera* cams, int32_t n_views,
                        const rogs_render_opts* opts, int64_t pair_capacity,
                        int64_t slot_capacity, size_t* bytes);

/* a1-a2, Eq. 5 + supp. Sec. 2.1.  Starts a batch: uploads the view table into
 * the workspace, culls and projects every (view, surfel) with the key
 * contract, counts tiles per surfel and scans the counts.  The batch state
 * (layout, views) is kept in ctx for the calls below, which must pass the
 * same workspace. */
ROGS_API int rogs_project(rogs_ctx* ctx, const rogs_surfels* s, const rogs_camera* cams, int32_t n_views,
                 const rogs_render_opts* opts, void* ws, size_t ws_bytes, int64_t pair_capacity,
                 int64_t slot_capacity, void* stream);

/* a3-a5, Sec. 3.3.1 ("ascending order of original depth").  Emits one pair
 * per covered tile and orders the pairs by (tile, depth), ties by surfel id
 * (the order a stable sort of (tile, depth) keys in surfel-id order gives),
 * and writes per-tile ranges ((0, 0) for an empty tile).  With ROGS_SYNC_COUNT the pair
 * count P is read back first (host sync): if P > pair_capacity or the
 * visible-slot count exceeds slot_capacity the call returns ROGS_ECAPACITY
 * with *n_pairs_out = P and enqueues nothing more (rogs_batch_stats gives
 * both counts).
 * Without it the count stays on the device; an overflow is flagged on the
 * device and reported by rogs_overflow(). n_pairs_out may be NULL. */
ROGS_API int rogs_bin_sort(rogs_ctx* ctx, void* ws, int64_t* n_pairs_out, uint32_t flags, void* stream);

/* Reads the device pair count and overflow flag of the current batch (host sync). */
ROGS_API int rogs_pair_count(rogs_ctx* ctx, void* ws, int64_t* n_pairs, int32_t* overflow, void* stream);

/* Channel sets.  Planes of a rendered view: RGB (3), SEM (the C semantic
 * logits, composited like colour, Sec. 3.3.1), D (sum w t_z), A (1 - T);
 * ELEV (serving and BEV export) is formed from D and A. */
#define ROGS_CH_RGB  1u
#define ROGS_CH_SEM  2u
#define ROGS_CH_D    4u
#define ROGS_CH_A    8u
#define ROGS_CH_ELEV 16u
#define ROGS_CH_ALL  31u

/* a6, Eq. 6.  Front-to-back compositing of R, G, B, sem[C], D = sum w t_z and
 * A = 1 - T into out_images (5 + C channels, image layout above).  Only the
 * planes selected by channel_mask (a non-empty OR of ROGS_CH_*; ELEV selects D
 * and A) are composited and written; the others are left untouched, and the
 * per-pixel sums they would need are not formed (an RGB-only render skips the
 * C semantic accumulations).  The selected planes are bitwise the same as in
 * an all-plane render.  Only a render of every plane (ROGS_CH_ALL) keeps
 * T_final, the number of list entries each pixel visited and the relative
 * depth sum in the workspace for rogs_render_bwd. */
ROGS_API int rogs_render_fwd(rogs_ctx* ctx, const rogs_surfels* s, void* ws, float* out_images,
                    uint32_t channel_mask, void* stream);

/* a7, Eq. 7, 8, 9, 12.  For every pixel of the batch: c' = e^a c + b,
 * masked L1 over the three colour channels and masked cross-entropy of the
 * composited logits against the label, each divided by the view's mask
 * count |M_v|, weighted by lambda_c / lambda_s and view_scale.  Writes
 * dL/d(out) into dL_dout (5 + C channels; D and A rows are 0), adds the loss
 * to loss_out[0] and dL/d(a, b) to d_exposure[V][2] (device, accumulate). */
ROGS_API int rogs_loss(rogs_ctx* ctx, void* ws, const float* out_images, const rogs_targets* t,
              float* dL_dout, float* loss_out, float* d_exposure, void* stream);

/* a8-a9, adjoint of Eq. 5-6.  Given the forward images and dL/d(out) of
 * the current batch (after a rogs_render_fwd of every plane, else
 * ROGS_ESTATE), writes dL/d(surfel parameters) into the packed block
 * grads[11 + C][N] (rows: z, q, s, alpha, rgb, sem; w.r.t. the activated
 * s and alpha), summed over the batch's views.  ROGS_ACCUMULATE adds. */
ROGS_API int rogs_render_bwd(rogs_ctx* ctx, const rogs_surfels* s, void* ws, const float* out_images,
                    const float* dL_dout, float* grads, uint32_t flags, void* stream);

/* a10, Adam (Sec. 4.2) with torch semantics (bias correction, dense update)
 * on the packed raw block params[11 + C][N] (rows 5-6 log-scales, row 7
 * opacity logit) with moments m, v of the same shape; grads are w.r.t. the
 * activated values and are chained through exp / sigmoid using the current
 * s_act and alpha_act.  The height row's rate for this step comes from the
 * schedule in optim.  Writes the refreshed activated scales s_act[2][N] =
 * exp(log s) and opacity alpha_act[N] = sigmoid(logit).  When exposure !=
 * NULL also steps exposure[n_views][2] with d_exposure and its moments m_exp,
 * v_exp (rate lr.exposure).  step >= 1; n_sem 1..8 or 16. */
ROGS_API int rogs_adam_step(rogs_ctx* ctx, int32_t n, int32_t n_sem, float* params, const float* grads,
                   float* m, float* v, float* s_act, float* alpha_act, const rogs_optim* optim,
                   int64_t step, float* exposure, const float* d_exposure, float* m_exp,
                   float* v_exp, int32_t n_views, void* stream);

/* ------------------------------------------------------ fused step
 * The whole training step (a1-a10) over all views of a batch in one graph:
 * cull + projection, emission, binning and ranges with the pair count kept
 * on the device; then one kernel per tile that composites the forward, forms
 * the loss and its per-pixel seed dL/dO in registers and runs the backward
 * pass over the same list (neither the images nor the seed are written to
 * memory); then the projection adjoint fused with Adam.  The step number
 * lives on the device (step_state), so no host value changes between steps.
 *
 * The sequence is captured into a hipGraph on the first call and replayed by
 * later calls with the same arguments (same pointers, sizes, options, view
 * resolutions and per-view tile shapes; camera poses may change: each call copies the camera
 * table from one of two pinned buffers ahead of the graph).  Two steps stay
 * in flight: each call first waits for the step launched two calls before,
 * then launches, so the device runs the previous step meanwhile.  A step
 * that overflowed pair_capacity made no update (parameters, moments and
 * step count untouched); unless that was already seen through
 * rogs_fused_status, the call that waits for it returns ROGS_ECAPACITY
 * without launching.  Read the needed count with rogs_fused_status, grow
 * the workspace and call again. */
typedef struct {
  int32_t n, n_sem;
  const float* x;        /* [N] fixed grid vertices */
  const float* y;
  float* params;         /* [11 + C][N] raw block (row layout above) */
  float* m;              /* Adam moments, same shape */
  float* v;
  float* s_act;          /* [2][N] activated scales; refreshed by every step */
  float* alpha_act;      /* [N] activated opacity; refreshed by every step */
  float* exposure;       /* [V][2] per-view (a, b) of Eq. 7; updated by Adam */
  float* m_exp;          /* its moments */
  float* v_exp;
  float* d_exposure;     /* [V][2] output: dL/d(a, b) of the last step */
  float* grads;          /* optional [11 + C][N] output of the step's gradients, or NULL */
  void* step_state;      /* 64 bytes of device memory, zeroed before the first step:
                            step count, skipped steps, last loss (16-byte aligned) */
} rogs_train_state;

#define ROGS_FUSED_EAGER 4u   /* run the same kernels without graph capture */

ROGS_API int rogs_fused_workspace_size(const rogs_train_state* t, const rogs_camera* cams,
                                       int32_t n_views, const rogs_render_opts* opts,
                                       int64_t pair_capacity, int64_t slot_capacity,
                                       size_t* bytes);
ROGS_API int rogs_step_fused(rogs_ctx* ctx, const rogs_train_state* t, const rogs_camera* cams,
                             int32_t n_views, const rogs_render_opts* opts,
                             const rogs_targets* targets, const rogs_optim* optim, void* ws,
                             size_t ws_bytes, int64_t pair_capacity, int64_t slot_capacity,
                             uint32_t flags, void* stream);
/* Waits for the fused steps in flight and reports, for the last one,
 * stats[0] pairs P, [1] overflow,
 * [2] visible slots, [3] steps applied, [4] steps skipped, [5] pixels,
 * [6] tiles, [7] slots; *loss = loss of the last applied step (nullable). */
ROGS_API int rogs_fused_status(rogs_ctx* ctx, int64_t* stats, float* loss);

/* ------------------------------------------------------ grid-side terms
 * Elevation smoothness (Eq. 10) over the four grid neighbours and the LiDAR
 * elevation loss (Eq. 11), per surfel:
 *   L = lambda_smooth / 4 * sum_i sum_{j in N(i)} (z_i - z_j)^2
 *     + lambda_z * sum_i (z_i - zbar_i)^2
 * nbr[4][n] must be symmetric (j = up(i) implies i = down(j), likewise
 * left/right; a surfel is its own neighbour where it has none), which makes
 * dL/dz_i = lambda_smooth * sum_d (z_i - z_{nbr[d][i]}) + 2 lambda_z (z_i - zbar_i).
 * Adds the gradient into dz[n] and the loss into loss_out[0] (device).  Either
 * term may be off (nbr or zbar NULL).  scratch: device memory of
 * rogs_elev_scratch_bytes(n) bytes (block partial sums, summed in a fixed
 * order). */
ROGS_API size_t rogs_elev_scratch_bytes(int32_t n);
ROGS_API int rogs_elev_loss(rogs_ctx* ctx, int32_t n, const float* z, const int32_t* nbr,
                            float lambda_smooth, const float* zbar, float lambda_z, float* dz,
                            float* loss_out, void* scratch, size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as rogs_elev_loss, without a scratch argument.  The
 * block partial sums live in a fixed device array of the library, sized for
 * n <= ROGS_ELEV_STATIC_MAX_N (256 KiB per GPU, held until the process ends);
 * larger n returns ROGS_EINVAL.  The call allocates nothing.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller. */
#define ROGS_ELEV_STATIC_MAX_N 16777216
ROGS_API int rogs_elev_loss_static(rogs_ctx* ctx, int32_t n, const float* z, const int32_t* nbr,
                                   float lambda_smooth, const float* zbar, float lambda_z,
                                   float* dz, float* loss_out, void* stream);

/* LiDAR targets of Eq. 11: zbar[i] = pz of the point nearest to (x_i, y_i) in
 * the xy-plane (squared distance in binary64 of the binary32 inputs, ties to
 * the lower point index: the brute-force result), idx[i] its index
 * (nullable).  The points are bucketed into a uniform grid of about 2m cells
 * over the bounding box of surfels and points, and each surfel searches
 * rings of cells outward until no unvisited cell can hold a nearer point:
 * O(n + m) work for points spread like road returns.  Device arrays; 1 <= m <=
 * 2^29.  scratch: caller-owned device memory, 256-byte aligned, of
 * rogs_lidar_scratch_bytes(n, m) bytes (the grid, the points in cell order). */
ROGS_API size_t rogs_lidar_scratch_bytes(int32_t n, int32_t m);
ROGS_API int rogs_lidar_targets(rogs_ctx* ctx, int32_t n, const float* x, const float* y,
                                int32_t m, const float* px, const float* py, const float* pz,
                                float* zbar, int32_t* idx, void* scratch, size_t scratch_bytes,
                                void* stream);

/* Meshgrid layout and pose-based initialisation (Sec. 3.1, Eq. 4; supp.
 * Sec. 1 and 3.3).  A raster of W x H cells of `spacing` metres with cell
 * (col, row) centred at (x0 + col * spacing, y0 + row * spacing); each pose's
 * position falls in cell (floor((x - x0)/spacing + 1/2), likewise for y);
 * the road mask is the disk dilation of those cells by radius_px cells
 * (dx^2 + dy^2 <= r^2).  Surfels sit at the road cells, indexed by a running
 * count in row-major order (idx[H][W], -1 off the road); per surfel: x, y
 * (binary32 of the binary64 cell position), neighbours nbr[4][cap] (cells
 * above, below, left, right; own index off the road), and from the pose
 * nearest in the xy-plane (binary64 squared distance, ties to the lower
 * index): z = z_v - (n31 (x - x_v) + n32 (y - y_v)) / n33 with n3 the third
 * column of R_v (Eq. 4, binary64), and q = R_v as a unit quaternion (w >= 0).
 * Writes the count to *n_out (host sync).  If it exceeds capacity the
 * per-surfel arrays are not written and the call returns ROGS_ECAPACITY
 * (capacity 0 with NULL arrays is a size query and returns ROGS_OK).
 * poses: device array; scratch: rogs_meshgrid_scratch_bytes(W, H, n_poses). */
typedef struct {
  float x, y, z;           /* rear-axle ground point (m) */
  float R[9];              /* row-major world-from-vehicle rotation: columns forward, left, up */
} rogs_pose;
ROGS_API size_t rogs_meshgrid_scratch_bytes(int32_t W, int32_t H, int32_t n_poses);
ROGS_API int rogs_meshgrid_layout(rogs_ctx* ctx, const rogs_pose* poses, int32_t n_poses,
                                  double x0, double y0, float spacing, int32_t W, int32_t H,
                                  int32_t radius_px, int32_t* idx, int64_t capacity, float* x,
                                  float* y, float* z, float* q, int32_t* nbr, int64_t* n_out,
                                  void* scratch, size_t scratch_bytes, void* stream);

/* ------------------------------------------------------ BEV export
 * Chunked orthographic top-down export (the paper renders its BEV maps in
 * chunks of 2000 x 2000 pixels at 0.05 m/px and stitches them).  The stitched
 * image has W x H pixels of m_per_px metres; pixel (col, row) is centred at
 * (x0 + (col + 1/2) m, y0 + (H - row - 1/2) m), so row 0 is the image's
 * northern edge.  Every chunk of chunk_px x chunk_px pixels (smaller at the
 * right and bottom edges) is one orthographic camera looking straight down
 * from `height` (rogs_bev_camera), rendered with rogs_project + rogs_bin_sort
 * (host count, one sync per chunk) + rogs_render_fwd and copied into `out`:
 * the planes selected by `channels` (ROGS_CH_* as for serving, in the order
 * RGB, SEM, D, A, ELEV, each W x H floats; ELEV = height - D / A, NaN where
 * A = 0).  ws: device workspace of rogs_bev_workspace_size bytes for the
 * given pair capacity; a chunk with more pairs stops the export with
 * ROGS_ECAPACITY and *n_pairs_max (nullable) = the largest pair count seen. */
ROGS_API void rogs_bev_camera(double x0, double y0, int32_t W, int32_t H, float m_per_px,
                              int32_t ox, int32_t oy, int32_t cw, int32_t ch, float height,
                              rogs_camera* cam);
ROGS_API int rogs_bev_workspace_size(const rogs_surfels* s, int32_t chunk_px,
                                     const rogs_render_opts* opts, int64_t pair_capacity,
                                     size_t* bytes);
ROGS_API int rogs_bev_export(rogs_ctx* ctx, const rogs_surfels* s, const rogs_render_opts* opts,
                             double x0, double y0, int32_t W, int32_t H, float m_per_px,
                             int32_t chunk_px, float height, uint32_t channels, float* out,
                             void* ws, size_t ws_bytes, int64_t pair_capacity,
                             int64_t* n_pairs_max, void* stream);

/* ------------------------------------------------------ autotuner
 * Chooses the launch configuration for a workload: the tile shape (which
 * also sets the pixels per lane, tile_w * tile_h / 64), the LDS staging depth
 * (opts->stage) and a tile shape per resolution class.  Every configuration
 * renders the same values, since the per-pixel rule does not depend on it
 * (Sec. 3.3.1 with the 3-sigma cut); they differ in the number of (surfel,
 * tile) pairs, in the work each wave rejects and in LDS occupancy.  One run
 * is rogs_project + rogs_bin_sort (device count) + rogs_render_fwd +
 * rogs_render_bwd with dL/d(out) = 1 over the given surfels and views; each
 * configuration is sized with one counted run and then timed over `reps`
 * runs after one warm-up.  The search is a descent: (1) every shape with
 * tile_w in {4, 8, 16, 32, 64} and tile_w * tile_h in {64, 128, 256}, all
 * views alike, staging depth 32; (2) staging depth 16, 32, 64 at that shape;
 * (3) with more than one resolution class (views of equal w, h and model),
 * each class in turn tries the other shapes of the same area while the rest
 * keep theirs.  With step != NULL the timed run is instead one fused
 * training step (rogs_step_fused with ROGS_FUSED_EAGER) on copies of
 * step->state that the call makes and restores before each configuration,
 * so the caller's state is only read; each configuration's capacities come
 * from one untimed step.  The result goes to opts->tile_w / tile_h / stage (other
 * fields kept) and, when view_tiles is not null, view_tiles[v] receives the
 * rogs_camera.tile code of view v (0 where the view keeps the options'
 * shape); pass those codes in the cameras of later calls.  *ms_out
 * (nullable) receives the time per run of the result.
 * cache_json (nullable): path of a JSON cache keyed by the workload (what
 * is timed, n, n_sem, every view's size, model and fx).  A cached entry, which lists the
 * shape of each class, is returned without timing; a new result is added to
 * the file, which this call rewrites whole.  A file not written by this call
 * is rejected (ROGS_EINVAL) and left untouched.  The cameras' own tile fields
 * are ignored.  In step mode the context's fused-step status is reset: it
 * holds no step of the caller afterwards (read it first if needed).
 * Unlike the calls above this one allocates (hipMalloc: workspace, images,
 * gradients) and frees before returning, synchronises the stream, and leaves
 * the context's batch state at the last shape timed (call rogs_project
 * again before rogs_bin_sort / render). */
typedef struct {
  const rogs_train_state* state;   /* read only; targets->exposure == state->exposure */
  const rogs_targets* targets;
  const rogs_optim* optim;
} rogs_tune_step;

ROGS_API int rogs_autotune(rogs_ctx* ctx, const rogs_surfels* s, const rogs_camera* cams,
                           int32_t n_views, rogs_render_opts* opts, int32_t* view_tiles,
                           const rogs_tune_step* step, const char* cache_json, int32_t reps,
                           float* ms_out, void* stream);

/* ------------------------------------------------------ serving
 * Render server over a resident map (the served form of a6: forward only).
 * Requests are single views with a channel set; worker lanes owned by the
 * server batch whatever is queued whenever one is idle (continuous
 * batching, up to max_views views per batch and what a lane's arena holds),
 * renders the batch with rogs_project + rogs_bin_sort (pair count on the
 * device) + rogs_render_fwd, and copies each request's channels into its
 * buffer.  A batch that overflows the pair capacity the arena leaves is split
 * in two and rerun; a single view that still does not fit completes with
 * status ROGS_ECAPACITY.  Every view is rendered independently of the rest
 * of its batch, so a request's output is bitwise the same alone or batched.
 *
 * Output planes (each W x H floats, row-major), in this order for the bits
 * set: RGB (3 planes), SEM (C), D, A, ELEV.  ELEV = elev_ref - D / A (for an
 * orthographic camera looking straight down from height elev_ref this is the
 * surface height: D / A is the opacity-weighted depth); NaN where A = 0. */
typedef struct rogs_server rogs_server;

typedef struct {
  rogs_camera cam;       /* the view (host copy taken at submit) */
  uint32_t channels;     /* OR of ROGS_CH_* (non-zero) */
  float elev_ref;        /* reference height for ROGS_CH_ELEV */
  float* out;            /* DEVICE buffer of (planes * w * h) floats, caller-owned; must
                            stay valid until the request's poll returns ROGS_OK */
} rogs_request;

typedef struct {
  int32_t status;        /* ROGS_OK or the request's error (ROGS_ECAPACITY, ROGS_EHIP) */
  int32_t batch_views;   /* views in the batch that rendered it */
  int64_t t_arrive_ns;   /* steady-clock time of submit */
  int64_t t_start_ns;    /* its batch started */
  int64_t t_done_ns;     /* its output was complete on the device */
} rogs_result;

/* map: device surfel arrays that stay valid and unchanged while the server
 * lives.  arena: caller-owned device memory (256-byte aligned) holding the
 * batch workspaces and images; the server allocates no device memory.
 * lanes (1..8): worker threads, each with its own stream and an equal share
 * of the arena; an idle lane takes the queued requests, so batches on
 * different lanes overlap on the device.  device: HIP device ordinal.
 * Returns ROGS_EINVAL for bad arguments. */
ROGS_API int rogs_server_create(rogs_server** srv, const rogs_surfels* map,
                                const rogs_render_opts* opts, void* arena, size_t arena_bytes,
                                int32_t max_views, int32_t lanes, int32_t device);
/* Thread-safe.  Queues one request and returns its ticket.  ROGS_EINVAL: bad
 * camera, channels or buffer; ROGS_EREJECT: the view alone cannot fit a
 * lane's arena share, or the queue is full (65536 requests); ROGS_ESTATE:
 * the server is shutting down. */
ROGS_API int rogs_serve_submit(rogs_server* srv, const rogs_request* req, uint64_t* ticket);
/* Thread-safe, non-blocking.  ROGS_NOT_READY while the request is queued or
 * rendering (res gets t_arrive_ns); ROGS_OK once done: res filled, the ticket
 * is released (a second poll returns ROGS_EINVAL).  res->status carries the
 * request's own outcome. */
ROGS_API int rogs_serve_poll(rogs_server* srv, uint64_t ticket, rogs_result* res);
/* stats[7]: batches, views rendered, batch splits, largest batch, views that
 * failed with ROGS_ECAPACITY, requests queued now, most batches in flight at
 * once (over all lanes). */
ROGS_API int rogs_server_stats(rogs_server* srv, int64_t* stats);
/* Stops accepting requests, renders everything still queued, joins the
 * worker and frees the server (not the arena). */
ROGS_API void rogs_server_destroy(rogs_server* srv);

/* Batch statistics (host sync): stats[0] pairs P, [1] overflow flag,
 * [2] visible (view, surfel) slots, [3] pixels, [4] tiles, [5] slots V*N. */
ROGS_API int rogs_batch_stats(rogs_ctx* ctx, void* ws, int64_t* stats, void* stream);

/* Kernel timing.  While enabled, every launch group of the context is
 * bracketed by two HIP events on its stream.  rogs_prof_read waits for the
 * recorded events, returns the summed milliseconds and launch counts per group
 * (arrays of ROGS_PROF_GROUPS entries; n must be >= ROGS_PROF_GROUPS) since
 * the previous read, and resets them.  Group names: rogs_prof_name.  In
 * the fused step, group "fused_graph" times the whole graph launch (the
 * kernels inside a graph carry no events; ROGS_FUSED_EAGER times them), and
 * "render_step" its combined forward + loss + backward compositing. */
#define ROGS_PROF_GROUPS 12
ROGS_API int rogs_prof_enable(rogs_ctx* ctx, int32_t on);
ROGS_API int rogs_prof_read(rogs_ctx* ctx, double* ms, int64_t* launches, int32_t n);
ROGS_API const char* rogs_prof_name(int32_t group);

/* Read-back helpers for tests (host sync): copy the sorted keys, surfel ids
 * and per-tile ranges of the current batch to host buffers of the given
 * capacity. */
ROGS_API int rogs_debug_pairs(rogs_ctx* ctx, void* ws, uint64_t* keys, int32_t* surfel_ids,
                     int32_t* views, int64_t cap, uint32_t* ranges, int64_t n_tiles,
                     void* stream);
/* Work counts of the current batch after rogs_render_fwd (host sync): over
 * all pixels, *evaluated = list entries visited front to back up to each
 * pixel's termination, *contributing = those whose 3-sigma test passed
 * (q32 <= q_cut).  The compositing kernels' arithmetic is proportional to
 * these counts. */
ROGS_API int rogs_debug_work(rogs_ctx* ctx, void* ws, int64_t* evaluated, int64_t* contributing,
                             void* stream);
/* Copy the per-(view, surfel) projection records of the current batch:
 * rec[V][N][8] = u_hi v_hi u_lo v_lo A B C t_z, rect[V][N][4] = x0 x1 y0 y1,
 * count[V][N] = tiles reached (the row spans; 0 = culled or no tile reached, then
 * rec and rect read as zero). */
ROGS_API int rogs_debug_records(rogs_ctx* ctx, void* ws, float* rec, int32_t* rect, uint32_t* count,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ROGS_H */
