/*
 * gs3tr.h -- C ABI of the MI355X (gfx950) implementation of one optimizer
 * iteration of 3DGS^2-TR: a second-order trust-region method for 3D Gaussian
 * Splatting (tile rasteriser forward and backward, Gauss-Newton Hutchinson
 * diagonal, Hellinger-clipped update) and its Adam baseline.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns gs3_status; GS3_OK is 0 and errors are
 *   negative.  gs3_last_error() returns a thread-local message for the last
 *   failing call on the calling thread.  Arguments are validated before any
 *   work is enqueued, so GS3_EINVAL leaves the scene untouched.
 * Streams: all work is enqueued on the caller's hipStream_t (NULL = the
 *   default stream); no call waits for the whole device.  Functions that must know the number of (Gaussian,
 *   tile) pairs of a view before launching the blend block the calling
 *   thread once per view until the stream has run up to that view's pair
 *   count (a pinned host word written by the binning scan; the stream is
 *   not drained); the others are asynchronous.  A scene must not be used
 *   from two host threads or two streams at once; different scenes may run
 *   concurrently on different streams.
 * Ownership: a scene owns its device copies of the parameters, the training
 *   targets, the optimizer state and all scratch.  Pointers passed in are
 *   borrowed for the duration of the call only.  Output pointers are
 *   caller-owned device buffers of the documented size.
 * Layout: the parameter vector x and every vector of its shape (gradient,
 *   Hessian diagonal, trust-region radius) is structure-of-arrays
 *   float[P][N]: P = 11 + 3K rows, K = (d+1)^2, N Gaussians.  Rows: mean
 *   x, y, z; log-scale 0..2; quaternion q_x, q_y, q_z, q_w (unnormalised);
 *   opacity logit; then SH coefficient k of channel c at row 11 + 3k + c.
 *   Images are float[H][W][3], row-major, pixel (i, j) centred at
 *   (j + 1/2, i + 1/2).  Cameras are OpenCV pinholes (x right, y down, z
 *   forward) with a world-to-camera rotation R (row-major) and translation t.
 *
 * Paper: "3DGS^2-TR: Scalable Second-Order Trust-Region Method for 3D
 * Gaussian Splatting" (Hsiao et al.).  Each function cites the passage that
 * defines what it computes.
 */
#ifndef GS3TR_H
#define GS3TR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs3_status;
enum {
  GS3_OK = 0,
  GS3_EINVAL = -1,      /* bad argument: NULL, size, index or range        */
  GS3_ENOMEM = -2,      /* a device allocation failed                      */
  GS3_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed      */
  GS3_ENONFINITE = -4,  /* an update met a non-finite gradient entry or
                           produced a non-finite parameter (gs3_scene_sync) */
  GS3_ESTATE = -5,      /* the scene is not in a state that allows the call */
  GS3_ENOTIMPL = -6     /* the requested variant is not implemented        */
};

/* Scene flags: reserved; gs3_scene_desc.flags must be GS3_FLAG_NONE
 * (anything else is EINVAL).  Method variants are chosen per call
 * (gs3_tr_hparams.variant). */
enum {
  GS3_FLAG_NONE = 0u
};

typedef struct gs3_scene gs3_scene; /* opaque */

typedef struct {
  int32_t width, height;   /* pixels; both in [1, 16368]                    */
  float fx, fy, cx, cy;    /* pinhole intrinsics in pixels                  */
  float R[9];              /* world-to-camera rotation, row-major           */
  float t[3];              /* world-to-camera translation                   */
} gs3_camera;

typedef struct {
  int64_t n_gaussians;       /* N >= 1                                      */
  int32_t sh_degree;         /* d in 0..3                                   */
  int32_t n_cameras;         /* M >= 1, number of training views            */
  const gs3_camera* cameras; /* host array of n_cameras cameras             */
  float background[3];       /* colour added with the final transmittance   */
  float lambda_dssim;        /* lambda of the L1 / D-SSIM mix, in [0, 1]    */
  uint32_t flags;            /* reserved, must be GS3_FLAG_NONE             */
  const uint8_t* train_mask; /* host, n_cameras entries: nonzero marks a
                                training view (the M images of the
                                objective); NULL = every camera trains.
                                Held-out views are rendered and scored only. */
} gs3_scene_desc;

/* Trust-region radius variants (gs3_tr_hparams.variant, bit flags).  0 is
 * the radius exactly as the appendix prints it.
 * GS3_TR_MEAN_EXACT: the mean radius uses 1 / (Sigma^-1)_cc in place of
 *   Sigma_cc (the printed form is exact only for an axis-aligned Sigma).
 * GS3_TR_SECOND_ORDER: the scale, quaternion, opacity and colour radii use
 *   the constants 8/3, 16, 8, 8 in place of 2, 8, 4, 4, so that each spends
 *   the whole budget epsilon to second order (the printed Taylor steps are
 *   conservative by factors 0.75, 0.5, 0.5, 0.5). */
#define GS3_TR_MEAN_EXACT 1u
#define GS3_TR_SECOND_ORDER 2u
/* GS3_TR_SH_JOINT: the view-dependent SH coefficients (k >= 1) of channel c
 *   share the radius eta_C / S_d, S_d the maximum over directions of
 *   sum_{k>=1} |Y_k| at degree d, so that moving all of them at once changes
 *   the colour by at most eta_C in any direction; the DC coefficient keeps
 *   eta_C / C0.  Without it every coefficient gets eta_C / C0. */
#define GS3_TR_SH_JOINT 4u

typedef struct {
  float theta1;     /* EMA decay of the gradient, in [0, 1)               */
  float theta2;     /* EMA decay of the Hessian diagonal, in [0, 1)       */
  float epsilon;    /* Hellinger trust-region budget, > 0                 */
  uint32_t variant; /* GS3_TR_* bits; other bits are rejected (EINVAL)    */
} gs3_tr_hparams;

/* Number of rows P = 11 + 3 (d+1)^2 of the parameter layout; -1 if d is not 0..3. */
int32_t gs3_n_params(int32_t sh_degree);

/* Library version string (static storage). */
const char* gs3_version(void);

/* Create a scene: copies params_dev (float[P][N], device) and the training
 * targets targets_dev (device; camera j's float[H_j][W_j][3] images stored
 * back to back in camera order) on `stream` and returns the handle in *out.
 * The optimizer state (gradient EMA, Hessian-diagonal EMA, Adam moments,
 * the fused iteration's buffers) is created, zeroed, by the first call that
 * needs it, so a scene holds only its method's state.  Setting: the least-squares problem of Eq. objective, whose
 * M images are the given cameras.  Errors: EINVAL (NULL or bad sizes),
 * ENOMEM, EDEVICE.  The scene must be released with gs3_scene_destroy. */
gs3_status gs3_scene_create(const gs3_scene_desc* desc, const float* params_dev, const float* targets_dev,
                            hipStream_t stream, gs3_scene** out);

/* Release the scene.  Waits for the work the scene has enqueued (its own
 * completion event, recorded by every call on that call's stream) and for
 * nothing else; its device blocks go to a process-wide cache that later
 * scenes draw from (see gs3_trim_cache), so tearing one scene down does not
 * stall the streams of others. */
gs3_status gs3_scene_destroy(gs3_scene* scene);

/* Borrowed device pointer to the scene's parameters float[P][N]; valid
 * until the scene is destroyed or the next gs3_tr_iteration (which swaps
 * the two parameter buffers); updated in place by tr_step / adam_step. */
gs3_status gs3_scene_params(gs3_scene* scene, float** params_dev);

/* Overwrite the scene's parameters from params_dev (float[P][N], device). */
gs3_status gs3_scene_set_params(gs3_scene* scene, const float* params_dev, hipStream_t stream);

/* Resident bytes (targets, parameters and the trust-region method's state:
 * six float[P][N] buffers and the radius scratch, where Adam needs three
 * buffers) and the peak scratch of a scene described by desc: two slots of
 * per-Gaussian and per-pixel buffers and pair buffers reserved for 12
 * (Gaussian, tile) pairs per Gaussian with 25% slack (slot 0, allocated at
 * creation, and the slot of the probe entry that a gs3_tr_iteration with one
 * Hutchinson view and probe adds).  A view with more pairs grows the pair
 * buffers (stream-ordered, without waiting for the device), and batches of
 * more views or probes add slots; gs3_scene_device_bytes reports what a
 * scene holds.  Used to admit scenes under an HBM budget.  No device work. */
gs3_status gs3_scene_bytes(const gs3_scene_desc* desc, int64_t* resident, int64_t* peak_scratch);

/* Device bytes the scene holds now: everything gs3_scene_bytes counts
 * (optimizer state only once created) plus any growth of its pair buffers. */
gs3_status gs3_scene_device_bytes(gs3_scene* scene, int64_t* bytes);

/* Release the device blocks that destroyed scenes left in the process-wide
 * cache (waiting for the device).  The cache keeps at most 16 GiB; blocks
 * beyond that are released when they are given back. */
gs3_status gs3_trim_cache(void);

/* Wait for all work the scene enqueued; reports deferred device errors, and
 * GS3_ENONFINITE (once, then cleared) if an update since the last sync read
 * a non-finite gradient entry or wrote a non-finite parameter (the trust-
 * region and Adam updates check every row they write). */
gs3_status gs3_scene_sync(gs3_scene* scene);

/* Render camera `cam` (0 <= cam < n_cameras) of the scene's current
 * parameters into rgb_dev (float[H][W][3], device).  Tile rasteriser of the
 * Background section: project, tile keys, sort, front-to-back alpha blend
 * C = sum_i c_i abar_i T_i + T_final * background. */
gs3_status gs3_render(gs3_scene* scene, int32_t cam, float* rgb_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gs3_render
 * without a scene.  Renders params_dev (float[P][N], device, read only; N =
 * n_gaussians, P from sh_degree) from *camera (host) into rgb_dev
 * (float[H][W][3], device) with background[3] (host; NULL = black), with the
 * same kernels as gs3_render, so the image is bit-identical to a scene's.
 * Every scratch buffer is carved from one library-owned static device array
 * of 128 MiB per GPU (held by each GPU the library runs on until the process
 * ends); the call performs no device or pinned-host allocation and no free.
 * Limits: the per-Gaussian and per-pixel buffers (88 B per Gaussian, 8 B
 * per pixel, 12 B per tile) must fit, and the view's (Gaussian, tile) pairs
 * must fit the rest (about 33 B per pair: some 3.5M pairs for 100k Gaussians
 * at 800x800); EINVAL otherwise, before any work for the size check and
 * after the binning for the pair count.  Synchronises the stream once (to read
 * the pair count).  Calls that overlap on one GPU share the array and race:
 * serialise them (every call rewrites the parts it reads; nothing needs to
 * start at zero). */
gs3_status gs3_render_noalloc(int64_t n_gaussians, int32_t sh_degree, const float* params_dev,
                              const gs3_camera* camera, const float background[3], float* rgb_dev,
                              hipStream_t stream);

/* Bin camera `cam` (Background, "Review of Gaussian Splatting": splats are
 * bucketed per 16x16 tile and sorted by depth).  A splat is paired with the
 * tiles of its 3-sigma screen rectangle whose block of pixel centres its skip
 * ellipse (alpha exp(power) >= 1/255, widened for float32 rounding) can
 * reach, in row-major order; a splat that reaches no tile is culled.  Writes
 * the sorted 64-bit keys ((tile << 32) | float bits of depth) and the
 * Gaussian index of every (Gaussian, tile) pair into
 * keys_dev / gids_dev (capacity entries each, device; either may be NULL),
 * each tile's [start, end) into ranges_dev (uint32[tiles][2], device, may be
 * NULL) and the pair count into *n_pairs (host).  Fails with EINVAL when the
 * pair count exceeds capacity (n_pairs is still set).  Every call that bins
 * a view (render, grad, hvp_diag, ...) fails with EINVAL for a view of
 * 2^32 - 2 or more pairs.  Synchronises. */
gs3_status gs3_bin(gs3_scene* scene, int32_t cam, uint64_t* keys_dev, uint32_t* gids_dev, uint32_t* ranges_dev,
                   int64_t capacity, int64_t* n_pairs, hipStream_t stream);

/* Stochastic gradient of Methodology / Algorithm 1:
 *   g_t = (1/m) (M/|S1|) sum_{j in S1} J_j^T f_j
 * with f_j the square roots of image j's loss components (Eq. pixel_loss,
 * Eq. objective) and S1 = cams[0..n_cams); the views go in batches of up to
 * 8, each batch one blend-forward, one blend-backward and one projection-
 * backward launch over all its views.  Writes grad_dev (float[P][N],
 * device).  If loss_out is not NULL it receives
 * 1/(2m) sum_{j in S1} sum_k l_jk (host double; synchronises). */
gs3_status gs3_grad(gs3_scene* scene, const int32_t* cams, int32_t n_cams, float* grad_dev, double* loss_out,
                    hipStream_t stream);

/* Hutchinson estimate of the Gauss-Newton diagonal (Methodology):
 *   D_t = (1/m) (M/|S2|) (1/nu) sum_{i<nu} z_i (.) sum_{j in S2} J_j^T J_j z_i
 * with Rademacher probes z_i: entry k = row * N + gaussian is +1 when the
 * top bit of SplitMix64(SplitMix64(seed ^ i) ^ k) is clear, else -1.
 * J_j^T J_j z is formed as an image JVP, the loss Jacobian with Gauss-Newton
 * weights 1/(4 max(l, 1e-6)) and an image VJP.  Writes D_dev (float[P][N]).
 * The (view, probe) entries go in batches of up to 8: each view is binned
 * once per batch, and one JVP blend launch, one backward launch and one
 * projection backward cover every entry of the batch. */
gs3_status gs3_hvp_diag(gs3_scene* scene, const int32_t* cams, int32_t n_cams, int32_t nu, uint64_t seed,
                        float* D_dev, hipStream_t stream);

/* The update of Algorithm 1: ghat = theta1 ghat + (1-theta1) g; if D_dev is
 * not NULL (a Hutchinson iteration) Dhat = theta2 Dhat + (1-theta2) D;
 * dx = -ghat / Dhat (where Dhat <= 0: -sign(ghat) eta, or 0 if eta is
 * infinite); eta = SHD(x, epsilon), the parameter-wise Hellinger radius;
 * x += clip(dx, -eta, eta).  grad_dev and D_dev are float[P][N] device
 * buffers; eta_out_dev and dx_out_dev (nullable, float[P][N]) receive eta
 * (+inf where unconstrained) and the clipped step. */
gs3_status gs3_tr_step(gs3_scene* scene, const float* grad_dev, const float* D_dev, const gs3_tr_hparams* hp,
                       float* eta_out_dev, float* dx_out_dev, hipStream_t stream);

/* One whole iteration of Algorithm 1 in one call: if n2 > 0 (a Hutchinson
 * iteration) D_t over the views cams2[0..n2) with nu probes of `seed` (as
 * gs3_hvp_diag); the stochastic gradient over cams1[0..n1) (as gs3_grad);
 * then the update of gs3_tr_step with D_t on Hutchinson iterations.  The
 * update is fused into the projection backward of the last gradient view,
 * so the gradient of that view never goes through memory; when the n2 * nu
 * Hutchinson entries and the n1 views fit one batch (n1 + n2 * nu <= 8) the
 * same launch also forms D_t, which then never goes through memory either
 * (the entries take their own view slots: a Hutchinson iteration holds n1 +
 * n2 * nu slots of per-view scratch, and the probe entries run on a second
 * stream the scene creates, forked from `stream` and joined to it before
 * the update, so the call still completes in `stream` order).  The parameters are double-buffered
 * (the update reads one copy and writes the other), so a pointer from
 * gs3_scene_params is not valid after this call.  A D_t of a larger batch
 * and the other views' gradient live in scene-owned buffers.  loss_out (nullable,
 * host) receives the mini-batch objective as in gs3_grad.  Same results as
 * gs3_hvp_diag + gs3_grad + gs3_tr_step on the same views. */
gs3_status gs3_tr_iteration(gs3_scene* scene, const int32_t* cams1, int32_t n1, const int32_t* cams2, int32_t n2,
                            int32_t nu, uint64_t seed, const gs3_tr_hparams* hp, double* loss_out,
                            hipStream_t stream);

/* The ADAM baseline of the Evaluations section (the first-order method the
 * paper compares against, run with the original 3DGS training settings):
 * Adam (Kingma and Ba) with bias correction, betas (0.9, 0.999),
 * eps 1e-15 and one learning rate per parameter group:
 * lr_per_group = {mean, SH DC, SH rest, opacity, scale, rotation} (host).
 * `step` is the 1-based Adam step count. */
gs3_status gs3_adam_step(gs3_scene* scene, const float* grad_dev, const float* lr_per_group, int32_t step,
                         hipStream_t stream);

/* ADAM-TR, the ablation of the Evaluations section: the Adam step clipped
 * by the parameter-wise Hellinger radius eta = SHD(x, epsilon). */
gs3_status gs3_adam_tr_step(gs3_scene* scene, const float* grad_dev, const float* lr_per_group, int32_t step,
                            float epsilon, hipStream_t stream);

/* PSNR 10 log10(1/MSE) of camera `cam`'s render against its target (host
 * double; synchronises): the reconstruction metric the Evaluations section
 * reports on held-out views (the 3DGS train/test split). */
gs3_status gs3_psnr(gs3_scene* scene, int32_t cam, double* psnr_out, hipStream_t stream);

/* Image-space VJP for autograd: grad_dev (float[P][N]) = J_img^T cot_dev,
 * cot_dev = dL/dC of camera cam (float[H][W][3], device). */
gs3_status gs3_render_vjp(gs3_scene* scene, int32_t cam, const float* cot_dev, float* grad_dev,
                          hipStream_t stream);

/* Image-space JVP for forward-mode autograd: rgb_dev and tan_dev
 * (float[H][W][3]) receive C(x) and J_img tangent_dev (tangent float[P][N]). */
gs3_status gs3_render_jvp(gs3_scene* scene, int32_t cam, const float* tangent_dev, float* rgb_dev, float* tan_dev,
                          hipStream_t stream);

/* Copy the optimizer state out (device buffers float[P][N] each; any may be
 * NULL): parameters, gradient EMA, Hessian-diagonal EMA, Adam m and v (zeros
 * for state not created yet). */
gs3_status gs3_scene_export(gs3_scene* scene, float* x, float* ghat, float* Dhat, float* adam_m, float* adam_v,
                            hipStream_t stream);

/* Restore the optimizer state exported by gs3_scene_export (NULL = keep;
 * creates the state it writes). */
gs3_status gs3_scene_import(gs3_scene* scene, const float* x, const float* ghat, const float* Dhat,
                            const float* adam_m, const float* adam_v, hipStream_t stream);

/* Measurement.  gs3_profile_enable(names) brackets every later launch of the
 * named stages with HIP events on the stream each runs on.  Stage names
 * (comma separated; "all" = every stage; NULL or "" disables): project_fwd,
 * depth_sort, scan, emit_pairs, pair_sort, blend_fwd, blend_jvp, blend_bwd,
 * pair_sums (each Gaussian's backward partials summed), project_bwd (the
 * chain rule into a gradient or Hutchinson diagonal), tr_update (the chain
 * rule fused with the update in gs3_tr_iteration), project_jvp, loss,
 * tr_step, adam_step.  Blend stages also
 * count their work on the device, with instrumented instances of their
 * kernels, unless gs3_profile_count(0) has switched counting off (then the
 * bracketed launches are the uninstrumented kernels every other call runs;
 * counting is on initially).  gs3_profile_read(name, ...) waits for the
 * recorded events and returns the number of bracketed launches, their summed
 * duration in milliseconds and two work counters: for blend stages the
 * (pixel, splat) evaluations and the contributing evaluations, for tr_step
 * and adam_step the Gaussians and the parameters updated, else 0 (any output
 * pointer may be NULL; the blend counters read 0 for launches made with
 * counting off).  gs3_profile_reset() forgets every record.  All four are
 * serialised by a process-wide lock. */
gs3_status gs3_profile_enable(const char* names);
gs3_status gs3_profile_count(int32_t on);
gs3_status gs3_profile_read(const char* name, int64_t* launches, double* total_ms, int64_t* work0,
                            int64_t* work1);
gs3_status gs3_profile_reset(void);

/* Message of the last failing call on this thread ("" if none). */
const char* gs3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS3TR_H */
