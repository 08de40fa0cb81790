/*
 * ddvr.h -- C ABI of the MI355X (gfx950) differentiable direct volume renderer.
 *
 * What is computed (Weiss & Westermann, "DiffDVR", arXiv 2107.12672):
 *   forward  -- Sec. 4.1, Alg. 1 (Direct Volume Rendering Algorithm): one ray
 *               per pixel, x_i = x_o + i*dt*omega for i = 0..N-1, trilinear
 *               density (Sec. 3.1 vertex grid), piecewise-linear transfer
 *               function with R regularly spaced knots (Sec. 3.1), Beer-Lambert
 *               opacity alpha_i = 1 - exp(-dt*tau) and front-to-back blending
 *               (Sec. 3.1; eq. blend-forward, Sec. 4.4).
 *   adjoint  -- Sec. 4.3, Alg. 2 (Adjoint Code of the DVR Algorithm), run with
 *               the inversion trick of Sec. 4.4 (eq. inv-blend-forward): the
 *               ray is re-traversed back to front and the blended state is
 *               recovered analytically instead of being stored, so memory is
 *               O(pixels), independent of the number of samples.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the comment says (host).  The caller
 *     owns all memory; the render calls never allocate.
 *   - Every call returns an int status (ddvr_status): 0 on success, < 0 on
 *     error.  Arguments are validated on the host before any launch; on a
 *     validation error nothing is launched and nothing is written.  No C++
 *     exception crosses this boundary.  ddvr_last_error() describes the last
 *     failure of the calling thread.
 *   - Work is enqueued on the given HIP stream (NULL = the null stream) and
 *     is asynchronous, except where a (host) output is requested.
 *   - Gradients ACCUMULATE (+=), as the "+=" of Alg. 2; zero them first.
 *   - NaN / Inf inside device data are not checked; they propagate.
 *
 * Geometry (the paper leaves the camera intrinsics open, Sec. 4.1 / 5.1):
 *   - volume: scalar densities at the vertices of an nx*ny*nz grid, stored
 *     [nz][ny][nx] (x fastest).  Isotropic spacing h = 2/(max(n)-1); the grid
 *     is centred at the origin, so its longest axis spans [-1, 1].
 *   - camera: pinhole.  Pixel (px, py), py = 0 the top row, has
 *     u = 2(px+1/2)/W - 1, v = 1 - 2(py+1/2)/H and direction
 *     omega = normalize(fwd + u*right + v*up); right/up are pre-scaled by
 *     tan(fovy/2)*W/H and tan(fovy/2).  The ray starts at the box entry point
 *     x_o = eye + t0*omega (t0 = 0 if the eye is inside the box) and takes
 *     N = ceil(L/dt) samples, L the chord length inside the box.
 *   - transfer function (emission-absorption model): table [R][4] of
 *     (r, g, b, tau), knots at k/(R-1); density clamped to [0,1] first.  The
 *     emission of a segment is premultiplied, c_i = alpha_i * rgb_i.
 *   - absorption-only model: tau(d) = d per world unit, no TF, no emission.
 *   - images: [H][W][4] float32 premultiplied (r, g, b, alpha) for the
 *     emission-absorption model, [H][W] float32 alpha for absorption-only.
 *     Background is transparent black; rays that miss the grid give exactly 0.
 *   - transmittance: [H][W] float32, T_N = 1 - alpha, saved by the forward
 *     pass for the adjoint (1 - alpha loses T_N in float32 once T_N is tiny).
 */
#ifndef DDVR_H
#define DDVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDVR_ABI_VERSION 5

typedef enum {
  DDVR_OK = 0,
  DDVR_ERR_NULL = -1,        /* a required pointer is NULL */
  DDVR_ERR_SHAPE = -2,       /* a size is out of range (grid < 2, R < 2, W/H <= 0, ...) */
  DDVR_ERR_DTYPE = -3,       /* unknown storage type */
  DDVR_ERR_VALUE = -4,       /* a scalar is out of range (step <= 0, non-finite, ...) */
  DDVR_ERR_HIP = -5,         /* the HIP runtime reported an error (also a pending
                                asynchronous error of an earlier launch) */
  DDVR_ERR_UNSUPPORTED = -6, /* valid request the library does not handle */
  DDVR_ERR_WORKSPACE = -7    /* workspace missing or too small */
} ddvr_status;

typedef enum { DDVR_F32 = 0, DDVR_F16 = 1, DDVR_BF16 = 2 } ddvr_dtype;

/* Models.
 *   ABSORPTION              tau(d) = d, image = alpha only.
 *   EMISSION_ABSORPTION     scalar density through the transfer function.
 *   COLOR                   pre-shaded colour volume: every vertex holds
 *                           (r, g, b, tau), data -> [nz][ny][nx][4] of the
 *                           volume's dtype (16-byte aligned for f32, 8-byte for
 *                           f16/bf16), each channel interpolated trilinearly,
 *                           then the emission-absorption segment and blend;
 *                           no TF (tf may be NULL), d_volume is
 *                           [nz][ny][nx][4] float32, images as
 *                           emission-absorption.  Single views, batches
 *                           (one storage type, not PLAIN, not RESIDUAL, one
 *                           workgroup per 16x16 tile in list order) and
 *                           render_tangent (direct gathers). */
typedef enum {
  DDVR_ABSORPTION = 0,
  DDVR_EMISSION_ABSORPTION = 1,
  DDVR_COLOR = 2
} ddvr_model;

/* Adjoint mode (low bits of `flags`).
 *   AUTO       absorption-only: the inversion of Sec. 4.4 carried out in closed
 *              form (see render_adjoint); emission-absorption: T-form inversion
 *              T^(i) = T^(i+1)/e_i, and rays whose saved T_N < 2^-100 (where
 *              float32 inversion breaks down, Sec. 4.4 "alpha < 1") are handed
 *              to the segment-checkpoint fallback.
 *   INVERT_T   T-form inversion for every ray, no fallback.
 *   INVERT_ALPHA  the paper's alpha-form, eq. (inv-blend-forward).  Its
 *              recovered T^(i) carries a relative error ~ 2^-24 / T_N, so rays
 *              with T_N < 2^-10 take the checkpoint fallback (needs workspace).
 *   CHECKPOINT segment checkpointing for every ray (the stored-state
 *              alternative; needs workspace).
 *   RESIDUAL   colour model only: every ray runs its adjoint in forward order
 *              with alpha_hat^(i+1) T^(i+1) = g_alpha T_N - (C_N - C^(i+1)).C_hat
 *              (no division, no workspace).
 * The colour model takes AUTO (T-form inversion; rays with T_N < 2^-100 use
 * the RESIDUAL form in the same launch, no workspace), INVERT_T or RESIDUAL;
 * the other models reject RESIDUAL, the colour model INVERT_ALPHA and
 * CHECKPOINT (DDVR_ERR_UNSUPPORTED). */
#define DDVR_ADJ_AUTO 0
#define DDVR_ADJ_INVERT_T 1
#define DDVR_ADJ_INVERT_ALPHA 2
#define DDVR_ADJ_CHECKPOINT 3
#define DDVR_ADJ_RESIDUAL 4
#define DDVR_ADJ_MODE_MASK 0xF
/* Launch strategy (bit flags, OR-ed into `flags`).
 *   PLAIN      one thread per ray with direct global gathers and global atomics
 *              for the density gradient (no LDS staging).  Same results up to
 *              float rounding; kept as the straightforward baseline.  (The
 *              colour model always gathers directly; it ignores PLAIN.) */
#define DDVR_LAUNCH_PLAIN 0x10
/* Loss of the fused passes (render_fused_l2, batch pass 2):
 *   LOSS_L1    loss = loss_scale * sum |image - target|, upstream gradient
 *              loss_scale * sign(image - target) (0 where equal): the L1 image
 *              loss of eq. (tf-loss) with loss_scale = 1/(N W H).  Without it
 *              the loss is L2, loss_scale * sum (image - target)^2.  Other
 *              passes ignore the bit. */
#define DDVR_LOSS_L1 0x20

/* A scalar grid: data -> [nz][ny][nx] values of `dtype` (device). */
typedef struct {
  const void* data;
  int32_t dtype;   /* ddvr_dtype */
  int32_t nx, ny, nz;
} ddvr_volume;

/* Transfer function: rgba_tau -> [R][4] float32 (device), R >= 2.
 * Ignored (may be {NULL, 0}) for the absorption-only model. */
typedef struct {
  const float* rgba_tau;
  int32_t R;
} ddvr_tf;

/* Camera frame (host struct): eye, unit forward, right*tan(fovy/2)*W/H,
 * up*tan(fovy/2), image size. */
typedef struct {
  float eye[3], fwd[3], right[3], up[3];
  int32_t width, height;
} ddvr_camera;

/* Gradient outputs (device pointers, each may be NULL = not requested).
 *   d_volume  [nz][ny][nx] float32 (the gradient of the float32 master copy,
 *             also when the grid is stored as f16/bf16)
 *   d_tf      [R][4] float32
 *   d_camera  [12] float32 in the order eye, fwd, right, up of ddvr_camera
 *   d_step    [1] float32 (per world unit) */
typedef struct {
  float* d_volume;
  float* d_tf;
  float* d_camera;
  float* d_step;
} ddvr_grads;

/* Launch shape of the render kernels (process-wide default, captured by a
 * batch when it is created).
 *   waves      waves per workgroup: 1 (8x8-pixel tiles), 2 (16x8) or 4 (16x16)
 *   lds_cap    voxels per LDS brick (64..16384, default 7168); the forward stages the grid
 *              values of each slab's brick, the adjoint accumulates the density
 *              gradient of the brick before one global atomic per voxel
 *   slab_k     initial samples per ray in a slab (>= 4); the kernel halves it
 *              while a slab's brick exceeds lds_cap and doubles it after small
 *              bricks, up to slab_kmax (<= 4096).
 *   cell_acc   1: keep a ray's density gradient for its current cell in
 *              registers and add it to the brick when the ray leaves the cell
 *              (Sec. 4.4, "on exit of the current cell"); 0: add every sample.
 *   lane_map   lane -> pixel map of the forward / adjoint passes: a wave
 *              takes an 8x8 block of adjacent pixels ("compact") or an 8x8
 *              lattice of every other pixel of the tile ("interleaved").
 *              0 compact / compact, 1 interleaved / interleaved, 2 compact /
 *              interleaved (the fused pass hands each ray's transmittance and
 *              upstream gradient to the adjoint's lane through LDS), 3
 *              interleaved / compact.
 *   schedule   batches only: 0 auto (2 when views differ in image size or grid,
 *              else 1), 1 one workgroup per tile with contiguous tile ranges
 *              per XCD, 2 persistent workgroups popping tiles from a queue
 *              ordered by estimated samples, longest first.  Batches whose
 *              grids mix storage types always use 2.
 *   slab_axis  density and absorption-only grids: 1 (default) slabs between
 *              planes of the grid axis closest to the tile's centre ray, whose
 *              bricks stay tight at any view angle; 0 shells of constant
 *              sample distance from the tile's earliest entry point.  A tile
 *              where some ray does not advance along that axis, and every
 *              launch without bricks, use shells.
 * Results do not depend on the tuning beyond float32 summation order. */
typedef struct {
  int32_t waves;
  int32_t lds_cap;
  int32_t slab_k;
  int32_t slab_kmax;
  int32_t cell_acc;
  int32_t lane_map;
  int32_t schedule;
  int32_t slab_axis;
} ddvr_tuning;

/* Set / read the process-wide launch shape (no paper counterpart).  set:
 * DDVR_ERR_NULL for NULL, DDVR_ERR_VALUE outside the ranges above. */
int ddvr_set_tuning(const ddvr_tuning* t);
int ddvr_get_tuning(ddvr_tuning* t);

/* Version of this ABI (DDVR_ABI_VERSION; no paper counterpart). */
int ddvr_abi_version(void);

/* Description of the last error of the calling thread (static storage, valid
 * until the next call on this thread; no paper counterpart).  Never NULL. */
const char* ddvr_last_error(void);

/* Camera on a sphere around the grid centre, facing it (Sec. 5.1: longitude /
 * latitude parameterisation), up = +y.  Angles in RADIANS:
 * eye = dist*(cos(pitch)cos(yaw), sin(pitch), cos(pitch)sin(yaw)).
 * out (host).  |pitch| must be < pi/2 (the frame is degenerate at the poles). */
int ddvr_camera_from_sphere(float yaw, float pitch, float dist, float fovy, int32_t width,
                            int32_t height, ddvr_camera* out);

/* Chain rule from a frame gradient d_frame[12] (host, layout of
 * ddvr_grads.d_camera) to d_sphere[4] (host) = d/d(yaw, pitch, dist, fovy)
 * (Sec. 5.1: gradients w.r.t. the viewpoint's longitude, latitude, distance). */
int ddvr_camera_grad_to_sphere(float yaw, float pitch, float dist, float fovy, int32_t width,
                               int32_t height, const float* d_frame, float* d_sphere);

/* Storage copy of a float32 master grid (form of the grid the kernels read; no
 * paper counterpart: reduced-precision storage is this implementation's):
 * dst[i] = round_to_nearest_even(src[i]) in `dtype` (f32: plain copy), for
 * i < n.  src, dst device; may not overlap. */
int ddvr_cast_volume(const float* src, void* dst, int32_t dtype, int64_t n, void* hip_stream);

/* Forward pass (Alg. 1) of one view.
 *   step_world  dt > 0 in world units (a step of s voxels is s*h).
 *   image       [H][W][4] (EA) or [H][W] (AO) float32, written.
 *   transmittance [H][W] float32, written; may be NULL (the adjoint needs it).
 *   flags       0 or DDVR_LAUNCH_PLAIN. */
int ddvr_render_forward(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, float* image, float* transmittance,
                        int32_t flags, void* hip_stream);

/* Storage of the segment-checkpoint fallback (Sec. 4.4: the inversion needs
 * none, but it fails as alpha -> 1; the fallback stores the transmittance at
 * segment starts, a square-root share of the tape of Sec. 4.3).
 * Bytes of workspace render_adjoint / render_fused_l2 need for `flags`
 * (0 unless a checkpoint path can run: emission-absorption AUTO,
 * INVERT_ALPHA and CHECKPOINT).  The size depends on the pixel count and on
 * sqrt(samples per ray), not on the samples themselves.  bytes (host). */
int ddvr_adjoint_workspace_size(const ddvr_volume* vol, const ddvr_camera* cam, float step_world,
                                int32_t model, int32_t flags, size_t* bytes);

/* Adjoint pass (Alg. 2 with the inversion trick, Sec. 4.4) of one view.
 *   image, transmittance  the forward outputs for the same inputs.
 *   d_image     dLoss/dimage, layout of `image`.
 *   grads       (host struct) gradients to accumulate into.
 *   flags       adjoint mode | launch flags.
 *   workspace   device scratch of >= ddvr_adjoint_workspace_size bytes (may be
 *               NULL when that size is 0).
 *   n_fallback_rays (host, may be NULL): if given, the call synchronises the
 *               stream and returns how many rays took the checkpoint path.
 * The colour model's default (slab) route re-marches the forward in the same
 * kernel for the start of each ray's inversion and the scale of its
 * fixed-point gradient brick; it reads d_image only (image and transmittance
 * must still be given, as for every model). */
int ddvr_render_adjoint(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, const float* image,
                        const float* transmittance, const float* d_image,
                        const ddvr_grads* grads, int32_t flags, void* workspace,
                        size_t workspace_bytes, int32_t* n_fallback_rays, void* hip_stream);

/* ddvr_render_adjoint without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Nothing is allocated: the
 * checkpoint fallback's ray queue and slots live in a static 64 MiB device
 * array of the library, one per device, held until the process ends (its
 * address is looked up once per device on the first call there).  Same
 * arguments, results and errors as ddvr_render_adjoint otherwise; fewer
 * concurrent checkpoint slots may run when the view is large.
 *   - DDVR_ERR_WORKSPACE if the view's queue (8 bytes per pixel) and at least
 *     256 checkpoint slots (4 (2 ceil(sqrt(samples per ray)) + 4) bytes each,
 *     rounded up to 256) exceed 64 MiB, e.g. above ~2800x2800 pixels.
 *   - Calls on one device share the array: calls that overlap on one device
 *     (other streams, other threads) race and must be serialised by the
 *     caller.  Each call clears what it needs (the queue length) itself. */
int ddvr_render_adjoint_noalloc(const ddvr_volume* vol, const ddvr_tf* tf,
                                const ddvr_camera* cam, float step_world, int32_t model,
                                const float* image, const float* transmittance,
                                const float* d_image, const ddvr_grads* grads, int32_t flags,
                                int32_t* n_fallback_rays, void* hip_stream);

/* Alg. 1, then Alg. 2 seeded by the image loss's gradient (its first line,
 * here computed in the kernel from the L2 loss, or the L1 image loss of eq.
 * (tf-loss)), in one launch: the forward's state stays in registers.
 * Fused forward -> loss gradient -> adjoint of one view, one launch
 * (pixel-local loss only).  loss = loss_scale * sum((image - target)^2), or
 * loss_scale * sum |image - target| with DDVR_LOSS_L1 in flags.
 *   target      layout of `image`.
 *   image, transmittance  written as by render_forward (transmittance may be
 *               NULL unless the fallback path is possible).
 *   loss_out    (device, may be NULL) one double, += loss. */
int ddvr_render_fused_l2(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                         float step_world, int32_t model, const float* target, float loss_scale,
                         float* image, float* transmittance, const ddvr_grads* grads,
                         int32_t flags, void* workspace, size_t workspace_bytes,
                         int32_t* n_fallback_rays, double* loss_out, void* hip_stream);

/* ------------------------------------------------------------------------
 * Forward-mode derivatives (Sec. 4.2, forward differentiation with forward
 * variables; Sec. 5.1 compares "forward-immediate" and "forward-delayed").
 * ------------------------------------------------------------------------ */
#define DDVR_MAX_DIRECTIONS 4
/* A direction in (camera frame, step) space: d_frame in the layout of
 * ddvr_grads.d_camera (eye, fwd, right, up), d_step per world unit. */
typedef struct {
  float d_frame[12];
  float d_step;
} ddvr_direction;

/* Forward pass of one view carrying, for every sample, the derivatives of
 * its state along ndir (1..DDVR_MAX_DIRECTIONS) directions -- the paper's
 * forward variables with p = ndir parameters (Sec. 4.2).  Cost grows with
 * ndir; it suits the few camera / step parameters of viewpoint optimisation.
 * The sample count N is piecewise constant in the camera and the step and is
 * not differentiated (as in the adjoint).
 *   dirs        (host) [ndir] directions.
 *   image       layout of render_forward's image, written; may be NULL.
 *   image_dot   [ndir][H][W][C] float32, d image / d direction_k, written
 *               ("forward-immediate": the caller contracts later); may be NULL.
 *   d_image, d_dir  "forward-delayed": d_dir[k] (device, ndir floats) +=
 *               sum over pixels and channels of d_image * image_dot_k, reduced
 *               in the same pass; both NULL, or both given.
 *   flags       0 or DDVR_LAUNCH_PLAIN.
 * At least one of image, image_dot, d_dir must be given.  The tangent
 * launch always uses 16x16-pixel tiles (4 waves); the brick capacity and slab
 * lengths follow the tuning. */
int ddvr_render_tangent(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, const ddvr_direction* dirs,
                        int32_t ndir, float* image, float* image_dot, const float* d_image,
                        float* d_dir, int32_t flags, void* hip_stream);

/* Directions of the sphere camera's parameters: d_frame[k*12 + j] (host,
 * [4][12]) = d frame_j / d (yaw, pitch, dist, fovy)_k, angles in radians --
 * the tangent inputs that make render_tangent differentiate w.r.t. the
 * viewpoint (the transpose of ddvr_camera_grad_to_sphere; Sec. 5.1, forward
 * mode). */
int ddvr_camera_sphere_tangents(float yaw, float pitch, float dist, float fovy, int32_t width,
                                int32_t height, float* d_frame);

/* ------------------------------------------------------------------------
 * Density from colour (Sec. 5.4, second stage of the reconstruction
 * pipeline): a density grid whose TF colours match a pre-shaded colour volume.
 * ------------------------------------------------------------------------ */
/* One estimation sweep.  For every voxel, ncand candidate densities drawn
 * uniformly from [0, 1) are mapped through the TF, and the one of least cost
 *   C(d) = ||C_T - C(d)||^2 + alpha log(1 + |tau_T - tau(d)|)
 *          + beta sum over the 6-neighbourhood (d - d_i)^2
 * is kept (ties: the lowest candidate index).  (C_T, tau_T) is the voxel's
 * entry of `color`; d_i are the previous estimate's grid neighbours (absent
 * outside the grid).  The sweep is Jacobi: every voxel reads d_prev only.
 *   color       colour volume (data [nz][ny][nx][4], as the DDVR_COLOR model).
 *   tf          [R][4] float32 (r, g, b, tau), knots at k/(R-1), 2 <= R <= 4096.
 *   d_prev      [nz][ny][nx] float32 (device) or NULL: no neighbour term (the
 *               first sweep).  Must not alias d_out.
 *   alpha, beta finite weights (the paper: alpha = 1/max(tau_T), beta = 1;
 *               see ddvr_color_tau_max).
 *   seed, sweep candidates are outputs (sweep*nvox + voxel)*ncand + k of the
 *               SplitMix64 stream of `seed` (Steele, Lea and Flood 2014), top
 *               24 bits times 2^-24; sweep >= 0 numbers the iterations.
 *   ncand       candidates per voxel, 1..65536 (the paper: 256).
 *   d_out       [nz][ny][nx] float32, written.
 *   cost_out    [nz][ny][nx] float32 cost of the kept candidate, or NULL.
 *   n_changed   (device, one uint32, or NULL) += voxels whose estimate differs
 *               from d_prev (the paper's stopping test). */
int ddvr_density_from_color(const ddvr_volume* color, const ddvr_tf* tf, const float* d_prev,
                            float alpha, float beta, uint64_t seed, int32_t sweep,
                            int32_t ncand, float* d_out, float* cost_out, uint32_t* n_changed,
                            void* hip_stream);

/* Largest extinction (channel 3) of a colour volume (Sec. 5.4 colour volume;
 * no paper counterpart for the reduction): *out (device, one float) is written
 * (-inf for an empty volume). */
int ddvr_color_tau_max(const ddvr_volume* color, float* out, void* hip_stream);

/* ------------------------------------------------------------------------
 * The reconstruction loop around the renderer (Sec. 5.1-5.3): priors, the
 * opacity entropy, the optimiser and the multi-resolution resampling.  All
 * pointers are device pointers; gradients and losses ACCUMULATE (+=).
 * ------------------------------------------------------------------------ */
/* TF smoothing prior of eq. (tf-loss): loss_out (one double, or NULL) +=
 * lambda/(4(R-1)) sum_c sum_r (T[r+1][c] - T[r][c])^2, d_tf ([R][4], or NULL)
 * += its gradient.  tf [R][4], 2 <= R <= 2^24. */
int ddvr_tf_prior(const float* tf, int32_t R, float lambda, float* d_tf, double* loss_out,
                  void* hip_stream);

/* The same prior on a density grid in 3D (Sec. 5.3): loss_out += lambda times
 * the mean over all pairs of grid neighbours along x, y and z of the squared
 * difference; d_volume += its gradient.  volume, d_volume [nz][ny][nx]
 * float32 (the master copy); sizes >= 1 with at least one pair. */
int ddvr_volume_prior(const float* volume, int32_t nx, int32_t ny, int32_t nz, float lambda,
                      float* d_volume, double* loss_out, void* hip_stream);

/* Opacity entropy of Sec. 5.1, OE = H(alpha) over the npix alphas of an
 * image, with H the normalised entropy H(x) = -1/log2(N) sum p_i log2 p_i,
 * p_i = x_i / sum x (0 log 0 = 0), in [0, 1].  (The paper prints H without
 * the minus sign, yet reports positive entropies that viewpoint selection
 * maximises; the sign is read as lost.)
 *   image     [npix][channels] float32, channels 4 (alpha = channel 3) or 1.
 *   work      two doubles of scratch (overwritten).
 *   value_out one double, written (or NULL).
 *   d_image   layout of image, or NULL: += scale * dOE/dalpha on the alpha
 *             channel; pixels with alpha = 0 (unbounded derivative) get none.
 * The alphas must not all be zero (the entropy is then undefined). */
int ddvr_opacity_entropy(const float* image, int64_t npix, int32_t channels, double* work,
                         double* value_out, float* d_image, float scale, void* hip_stream);

/* One Adam step (Kingma and Ba 2014; the optimiser of the Sec. 5.2-5.3
 * reconstructions) on n float32 parameters, step t >= 1:
 *   m = beta1 m + (1-beta1) g;  v = beta2 v + (1-beta2) g^2;
 *   param -= lr (m/(1-beta1^t)) / (sqrt(v/(1-beta2^t)) + eps), then clamped to
 *   [lo, hi] (pass -inf / +inf for none).
 * Fused into the same pass: store (or NULL) gets the new parameters in
 * store_dtype (round to nearest even, as ddvr_cast_volume), and grad is
 * zeroed when zero_grad != 0. */
int ddvr_adam_step(float* param, float* grad, float* m, float* v, int64_t n, int32_t t,
                   float lr, float beta1, float beta2, float eps, float lo, float hi, void* store,
                   int32_t store_dtype, int32_t zero_grad, void* hip_stream);

/* Trilinear resampling of a vertex grid onto another spanning the same box
 * (the multi-resolution schedule of Sec. 5.3): destination vertex i of an
 * axis sits at i (s-1)/(d-1) source grid units.  src [sz][sy][sx], dst
 * [dz][dy][dx] float32; every size >= 2; src and dst must not overlap. */
int ddvr_resample_volume(const float* src, int32_t sx, int32_t sy, int32_t sz, float* dst,
                         int32_t dx, int32_t dy, int32_t dz, void* hip_stream);

/* The same on a grid of `channels` (1..4) interleaved float32 values per
 * vertex, src [sz][sy][sx][channels], dst [dz][dy][dx][channels], each channel
 * resampled on its own (the colour volume of Sec. 5.4 under the same
 * multi-resolution schedule).  ddvr_resample_volume is channels = 1. */
int ddvr_resample_channels(const float* src, int32_t channels, int32_t sx, int32_t sy,
                           int32_t sz, float* dst, int32_t dx, int32_t dy, int32_t dz,
                           void* hip_stream);

/* ------------------------------------------------------------------------
 * Batches: many views of one or several grids in ONE launch (no paper
 * counterpart: the paper renders its views one after another, Sec. 5; the
 * per-view work is Alg. 1 / Alg. 2 as above).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t volume;          /* index into the batch's volume array */
  int32_t tf;              /* index into the batch's TF array (-1 for AO) */
  ddvr_camera cam;
  float step_world;
  float* image;            /* [H][W][C] */
  float* transmittance;    /* [H][W] or NULL */
  const float* d_image;    /* adjoint input, or NULL */
  const float* target;     /* fused-L2 target, or NULL */
  float* d_camera;         /* [12] or NULL */
  float* d_step;           /* [1] or NULL */
} ddvr_view;

typedef struct ddvr_batch ddvr_batch;

/* Build a batch (no paper counterpart; host-side planning + a small device
 * buffer of view descriptors and a cost-ordered tile queue, owned by the
 * batch).
 *   d_volumes[nvol], d_tfs[ntf]: per-volume / per-TF gradient outputs (device,
 *   entries or the arrays themselves may be NULL).
 *   The pointers inside are captured; rebuild the batch if they change. */
int ddvr_batch_create(const ddvr_volume* vols, int32_t nvol, const ddvr_tf* tfs, int32_t ntf,
                      const ddvr_view* views, int32_t nview, int32_t model, int32_t flags,
                      float* const* d_volumes, float* const* d_tfs, void* hip_stream,
                      ddvr_batch** out);
/* Free a batch and its device buffers (NULL is ignored; no paper counterpart). */
void ddvr_batch_destroy(ddvr_batch* b);
/* Workspace bytes of the batch's adjoint (checkpoint queue and slots; no paper
 * counterpart), and one pass of the batch (per view Alg. 1 / Alg. 2): pass 0 =
 * forward, 1 = adjoint (views need d_image), 2 = fused forward+L2+adjoint
 * (views need target). loss_out as in render_fused_l2.  Workspace as for a
 * single view, sized by ddvr_batch_workspace_size. */
int ddvr_batch_workspace_size(const ddvr_batch* b, size_t* bytes);
int ddvr_batch_run(ddvr_batch* b, int32_t pass, float loss_scale, double* loss_out,
                   void* workspace, size_t workspace_bytes, void* hip_stream);
/* Record pass `pass` of the batch into a HIP graph and replay it (no paper
 * counterpart).  The batch
 * keeps one recorded graph per pass, keyed on (loss_scale, loss_out,
 * workspace, workspace_bytes): a call with the same arguments as the pass's
 * last recording replays it, other arguments re-record that pass only (after
 * waiting for the stream).  Alternating passes therefore replay. */
int ddvr_batch_run_graph(ddvr_batch* b, int32_t pass, float loss_scale, double* loss_out,
                         void* workspace, size_t workspace_bytes, void* hip_stream);
/* Graphs recorded and instantiated by ddvr_batch_run_graph so far (host; no
 * paper counterpart). */
int ddvr_batch_graph_builds(const ddvr_batch* b, int64_t* builds);
/* Samples (sum over rays of N, Alg. 1's sample count) the batch's views take;
 * host output. */
int ddvr_batch_sample_count(const ddvr_batch* b, int64_t* samples);

/* ------------------------------------------------------------------------
 * Step plans (no paper counterpart: the batched form of one optimisation
 * step).  A plan records the WHOLE step of a batch -- forward, loss gradient,
 * adjoint and the checkpoint fallback -- into one HIP graph when it is created;
 * ddvr_plan_execute replays it.  The batch must outlive the plan, and the
 * buffers the batch and the plan captured must stay valid and unchanged in
 * address.
 * ------------------------------------------------------------------------ */
/* adjoint seeded by the views' d_image as the caller wrote it (forward, then
 * adjoint) */
#define DDVR_PLAN_LOSS_GIVEN 0
/* L2 against each view's target (L1 with DDVR_LOSS_L1 in the batch's flags),
 * the fused pass: one launch */
#define DDVR_PLAN_LOSS_FUSED 1
/* minus the opacity entropy of every view's image (Sec. 5.1, the objective
 * of viewpoint selection; OE as ddvr_opacity_entropy): loss = -loss_scale *
 * sum over views of OE_v.  The plan WRITES every element of each view's
 * d_image (the alpha channel -loss_scale dOE_v/dalpha, 0 where alpha = 0,
 * colour channels 0) between the forward and the adjoint. */
#define DDVR_PLAN_LOSS_NEG_ENTROPY 2
typedef struct ddvr_plan ddvr_plan;
/* Record a batch's whole step into one HIP graph (no paper counterpart):
 *   loss        one of DDVR_PLAN_LOSS_*.
 *   loss_scale  weight of the loss (fused: as render_fused_l2).
 *   loss_out    (device, one double, may be NULL) += the step's loss on every
 *               replay.
 *   workspace   as for ddvr_batch_run, sized by ddvr_batch_workspace_size.
 *   hip_stream  unused at creation (recording launches nothing).
 * The plan owns its graph and, for the entropy, 3 doubles per view. */
int ddvr_plan_create(ddvr_batch* b, int32_t loss, float loss_scale, double* loss_out,
                     void* workspace, size_t workspace_bytes, void* hip_stream, ddvr_plan** out);
/* Replay the recorded step on hip_stream (no paper counterpart). */
int ddvr_plan_execute(ddvr_plan* p, void* hip_stream);
/* Entropy plans: OE of every view at the last replay (Sec. 5.1's opacity
 * entropy), out (host) [n], n the number of views; synchronises hip_stream. */

int ddvr_plan_loss_terms(const ddvr_plan* p, double* out, int32_t n, void* hip_stream);
/* Free a plan and its graph (NULL is ignored; no paper counterpart). */
void ddvr_plan_destroy(ddvr_plan* p);

/* ------------------------------------------------------------------------
 * Measurement (no paper counterpart): the sustained VALU issue rate of the
 * device, the ceiling of the render kernels' ALU roofline.
 * ------------------------------------------------------------------------ */
/* One launch of `blocks` workgroups of 256 lanes; every lane runs `iters`
 * rounds of 16 independent chains of one VALU operation each -- non-packed
 * float32 FMA (mode 0), 32-bit integer add (mode 1), the two alternating over
 * the chains (mode 2), FMA alternating with the hardware exp2 (mode 3), or
 * two dependent instructions per chain: a float32 multiply then a max (mode
 * 4), a shift then an xor (mode 5), an FMA then a max (mode 6); or multiplies
 * and maxes on alternating chains (mode 7) -- built with the library's own
 * compiler flags.  out [blocks*256] float32 (device) receives a checksum per
 * lane; *lane_ops (host) = blocks*256*iters*16 instructions (times 2 for modes
 * 4 to 6).  Modes outside 0..7: DDVR_ERR_VALUE. */
int ddvr_valu_probe(int32_t mode, int32_t blocks, int32_t iters, float* out, int64_t* lane_ops,
                    void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DDVR_H */
