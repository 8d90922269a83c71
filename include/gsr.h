/*
 * gsr.h -- C ABI of libgsr.so, a differentiable tile rasterizer for 3D
 * Gaussian Splatting on AMD Instinct MI355X (gfx950).
 *
 * It computes the rendering step of DROID-Splat's mapper (Sec. 3.3
 * "Differentiable Rendering"): Gaussians with mean P, rotation r, scale s,
 * density sigma and SH colour are rendered at keyframe poses by front-to-back
 * alpha compositing, C = sum_i c_i a_i prod_{j<i} (1 - a_j), with
 * a_i = sigma_i G(R, t, P_i, r_i, s_i) (eqn:rendering), producing an image
 * and a depth map per keyframe; gradients flow to every Gaussian parameter
 * and, for pose refinement, to each keyframe pose (Sec. 3.3, last paragraph;
 * supplementary S1.3).  The mapper renders a batch of keyframes per
 * iteration (supplementary S1.2): one call renders F frames of any sizes.
 *
 * Conventions
 *  - All tensor arguments are device pointers to contiguous FP32 arrays owned
 *    by the caller (the Python binding passes PyTorch storage); `cams` and
 *    `settings` are host structs.  Pointers must be 4-byte aligned.
 *  - Parameters: means [n,3]; log_scales [n,3] (s = exp); quats [n,4] as
 *    (w, x, y, z), normalised inside; opacity_logits [n] (sigma = 1/(1+e^-o));
 *    sh [n, (d+1)^2, 3] real SH coefficients, coefficient-major, colour =
 *    max(0, sum_k sh_k Y_k(dir) + 1/2), dir the unit vector from the camera
 *    centre to the mean.
 *  - poses [F,3,4] world->camera [R | t], OpenCV axes (x right, y down,
 *    z forward); pixel (i, j) samples the point (i, j) of the pinhole image
 *    u = fx x/z + cx, v = fy y/z + cy.
 *  - Outputs are packed over frames in order: rgb holds, per frame, a [3,H,W]
 *    block; depth and alpha hold a [H,W] block per frame.  depth is the
 *    alpha-blended view depth sum_i z_i a_i T_i (or, with
 *    GSR_FLAG_MEDIAN_DEPTH, the median depth); alpha = 1 - T_final;
 *    rgb = sum_i c_i a_i T_i + T_final * background.
 *  - Culling and thresholds: keep a Gaussian in a frame iff z > near, the
 *    projected 2x2 covariance (+0.3 px^2) is positive definite and its
 *    3-sigma pixel square [ceil(u-r), floor(u+r)] x [ceil(v-r), floor(v+r)],
 *    r = 3 sqrt(lambda_max), meets the image.  A Gaussian contributes to a
 *    pixel only inside its square (so results do not depend on the tile
 *    shape); a = min(0.99, sigma exp(-q/2)); entries with a < 1/255 are
 *    skipped; a pixel stops before the entry that would take T below 1e-4.
 *    A Gaussian with a non-finite parameter (NaN or +-Inf in its mean,
 *    scales, quaternion, opacity logit or an SH coefficient of the rendered
 *    degree) is culled in every frame; a Gaussian that no frame keeps gets
 *    gradients of exactly 0.
 *  - Cameras: width, height in [1, 65535]; fx, fy > 0 and finite; cx, cy
 *    finite; near_z > 0 and finite (GSR_ERR_INVALID_ARGUMENT otherwise).
 *  - The pose gradient g_twist [F,6] = dL/dxi at xi = 0 for the left
 *    perturbation T_f <- Exp(xi) T_f, xi = (rho, phi), translation first.
 *  - Gradient outputs are overwritten, never accumulated.
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls are
 *    asynchronous unless stated; one context serves one stream at a time.
 *
 * Errors: every call returns a gsr_status; no exception or abort crosses the
 * ABI.  Arguments are validated on the host before any launch.  A HIP error
 * returns GSR_ERR_HIP; gsr_last_error() gives the message.  n == 0 or a
 * frame that nothing reaches is not an error (background, 0, 0).
 */
#ifndef GSR_H
#define GSR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsr_status;
#define GSR_OK 0
#define GSR_ERR_INVALID_ARGUMENT 1
#define GSR_ERR_CAPACITY 2      /* more (tile, Gaussian) keys than key_capacity */
#define GSR_ERR_OUT_OF_MEMORY 3
#define GSR_ERR_HIP 4
#define GSR_ERR_STATE 5         /* backward without a matching forward */
#define GSR_ERR_UNSUPPORTED 6   /* e.g. a tile shape without a kernel */

/* One pinhole camera per frame (host struct). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float near_z; /* cull depth, 0.2 in the workloads */
} gsr_camera;

/* Render settings (host struct). */
typedef struct {
  int32_t sh_degree;      /* 0..3 */
  float background[3];
  int32_t tile_w, tile_h; /* 16x16, 8x8, 32x8, 16x8 or 32x16 */
  int32_t lds_batch;      /* Gaussians staged per LDS round by the 3D compositing kernels:
                             32, 64, 128; 0 = 64 (the surfel kernels always stage 64) */
  int64_t key_capacity;   /* 0: the library sizes the key buffers from the
                             exact count (one 8-byte device->host read per
                             forward); > 0: fixed capacity, no host read, and
                             an overflow is reported by gsr_check_overflow */
  uint32_t flags;         /* GSR_FLAG_* */
} gsr_settings;

#define GSR_FLAG_NO_XCD_REMAP 1u /* map workgroup i to tile i (default: each
                                    XCD gets a contiguous run of tiles) */
#define GSR_FLAG_TIMING 2u       /* record HIP events around every stage on the
                                    call's stream; read with gsr_debug_timings */
#define GSR_FLAG_COUNT_PAIRS 4u  /* count evaluated (pixel, entry) pairs in the
                                    forward compositing; see gsr_stats.n_pairs */
#define GSR_FLAG_MEDIAN_DEPTH 8u /* depth output = the median depth, the depth mode
                                    Sec. 3.3 names (after MonoGS): the z of the
                                    first blended entry after which the pixel's
                                    transmittance is below 1/2, 0 where it never
                                    is; gsr_backward then takes g_depth as the
                                    gradient of that depth, which reaches that
                                    entry's z only (the choice of entry is
                                    piecewise constant).  Default: alpha-blended
                                    depth sum_i z_i a_i T_i */

/* Stages timed under GSR_FLAG_TIMING (index into gsr_debug_timings). */
#define GSR_STAGE_PREPROCESS 0
#define GSR_STAGE_DEPTH_SORT 1
#define GSR_STAGE_OFFSETS 2
#define GSR_STAGE_KEYGEN 3
#define GSR_STAGE_TILE_SORT 4
#define GSR_STAGE_RANGES 5
#define GSR_STAGE_COMPOSITE_FWD 6
#define GSR_STAGE_LOSS 7
#define GSR_STAGE_COMPOSITE_BWD 8
#define GSR_STAGE_PREPROCESS_BWD 9
#define GSR_N_STAGES 10

typedef struct gsr_context gsr_context;

/* Creates a context bound to HIP device `device`.  *out receives it. */
gsr_status gsr_create(gsr_context** out, int32_t device);
/* Frees the context and its workspace (synchronises the device first). */
gsr_status gsr_destroy(gsr_context* ctx);
/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* gsr_last_error(const gsr_context* ctx);

/* Forward render of F frames (rows A0-A6 of the method: preprocess, depth
 * sort, keys, tile sort, ranges, compositing).  Saves what the backward
 * needs in the context; the caller keeps every input unchanged until the
 * matching gsr_backward has been enqueued. */
gsr_status gsr_forward(gsr_context* ctx, const gsr_settings* settings, int64_t n,
                       const float* means, const float* log_scales, const float* quats,
                       const float* opacity_logits, const float* sh, int32_t n_frames,
                       const gsr_camera* cams, const float* poses, float* rgb, float* depth,
                       float* alpha, void* stream);

/* Forward render of F frames with 2D Gaussian surfels instead of 3D
 * Gaussians (the primitive Sec. 3.3 and tab:renderer compare, after the 2DGS
 * method the paper cites).  A surfel is a flat disk: means [n,3], log_scales
 * [n,2] (its two in-plane scales), quats [n,4] (w, x, y, z; the first two
 * rotated axes span the disk, the third is its normal), opacity logits and
 * SH colour as for gsr_forward.  Each pixel's ray is intersected with the
 * disk: with M = K [s_u R_f t_u | s_v R_f t_v | R_f mu + t_f] (rows M0..M2),
 * (u, v) = (p0/p2, p1/p2), p = (x M2 - M0) x (y M2 - M1); G = exp(-(u^2 +
 * v^2)/2), the screen-space low-pass G_lp = exp(-|(x, y) - c|^2) around the
 * projected centre c, alpha = min(0.99, sigma max(G, G_lp)); compositing,
 * thresholds and order as gsr_forward (by the centre's depth).  Outputs rgb,
 * depth (sum_i w_i z_i with z_i = M2 . (u, v, 1), the centre's depth where
 * G_lp is the larger), alpha, normal [sum_f 3 H_f W_f] (CHW per frame,
 * sum_i w_i n_i, n_i the disk normal in the camera frame turned to face the
 * camera) and dist [sum_f H_f W_f], the depth distortion of the surfel
 * objective (the L_dist term the supplementary's Rendering settings add for
 * 2D Gaussian Splatting): per pixel the sum over pairs i < j of blended
 * entries of w_i w_j (z_i - z_j)^2.  A surfel covers the bounding box of
 * the image of the disk |(u, v)| <= sqrt(2 ln(255 sigma)) united with the
 * square of half width sqrt(ln(255 sigma)) around c, and is culled when
 * sigma <= 1/255 or the centre or the disk's nearest point is not beyond
 * the near plane.
 * GSR_FLAG_COUNT_PAIRS counts the (pixel, surfel) pairs whose box test
 * passes before the pixel stops; GSR_FLAG_MEDIAN_DEPTH is not supported
 * (GSR_ERR_UNSUPPORTED).  All output pointers are device memory, 4-byte
 * aligned; GSR_ERR_INVALID_ARGUMENT if normal or dist is NULL.  gsr_backward
 * after this forward returns GSR_ERR_STATE; use gsr_backward_surfel. */
gsr_status gsr_forward_surfel(gsr_context* ctx, const gsr_settings* settings, int64_t n,
                              const float* means, const float* log_scales, const float* quats,
                              const float* opacity_logits, const float* sh, int32_t n_frames,
                              const gsr_camera* cams, const float* poses, float* rgb,
                              float* depth, float* alpha, float* normal, float* dist,
                              void* stream);

/* Backward of the last gsr_forward_surfel on ctx (same method as
 * gsr_backward, for the surfel primitive of Sec. 3.3 / tab:renderer) for
 * upstream gradients of its five outputs, packed like them: g_rgb, g_depth,
 * g_alpha, g_normal [sum 3HW], g_dist [sum HW] (device, non-NULL; pass
 * zeros for an unused output).  Writes g_means [n,3], g_log_scales [n,2],
 * g_quats [n,4], g_opacity_logits [n], g_sh [n,(d+1)^2,3] (summed over
 * frames) and g_twist [F,6] (the left-perturbation pose twist (rho, phi) of
 * each frame).  The forward's inputs must be unchanged.  GSR_ERR_STATE if
 * the last forward was not a surfel forward. */
gsr_status gsr_backward_surfel(gsr_context* ctx, const float* g_rgb, const float* g_depth,
                               const float* g_alpha, const float* g_normal,
                               const float* g_dist, float* g_means, float* g_log_scales,
                               float* g_quats, float* g_opacity_logits, float* g_sh,
                               float* g_twist, void* stream);

/* The normal-consistency term of the surfel objective (the L_normal that the
 * supplementary's Rendering settings add for 2D Gaussian Splatting) on F
 * frames of rendered depth, alpha [sum_f H_f W_f] and normal [sum_f 3 H_f
 * W_f] (packed like the gsr_forward_surfel outputs; any images of that
 * layout).  Per frame, with the points P = D K^-1 (x, y, 1) and on interior
 * pixels (1 <= x <= W-2, 1 <= y <= H-2), N = v/|v|, v = dP_y x dP_x from the
 * central differences dP_x = P(x+1, y) - P(x-1, y), dP_y = P(x, y+1) -
 * P(x, y-1); a pixel's sum_i w_i (1 - n_i . N) is alpha - normal . N; the
 * frame's term is its mean over the (W-2)(H-2) interior pixels (0 where
 * v = 0).  Writes *loss = weight * sum_f term_f (device float) and ADDS the
 * gradient of *loss to g_depth, g_alpha and g_normal (device, packed like
 * the images), so that it stacks on the gradients of other terms.  Uses
 * only cams' width, height, fx, fy, cx, cy.  Does not touch the saved
 * forward.  Arithmetic in FP64 from the FP32 images. */
gsr_status gsr_normal_consistency(gsr_context* ctx, int32_t n_frames, const gsr_camera* cams,
                                  const float* depth, const float* alpha, const float* normal,
                                  float weight, float* loss, float* g_depth, float* g_alpha,
                                  float* g_normal, void* stream);

/* Backward of the last forward on ctx for upstream gradients g_rgb, g_depth,
 * g_alpha (packed like the outputs).  Writes g_means [n,3], g_log_scales
 * [n,3], g_quats [n,4], g_opacity_logits [n], g_sh [n,(d+1)^2,3] (summed
 * over frames) and g_twist [F,6].  GSR_ERR_STATE if no forward preceded. */
gsr_status gsr_backward(gsr_context* ctx, const float* g_rgb, const float* g_depth,
                        const float* g_alpha, float* g_means, float* g_log_scales,
                        float* g_quats, float* g_opacity_logits, float* g_sh, float* g_twist,
                        void* stream);

/* L1 loss of the last forward's outputs against targets (packed like them):
 * *loss = sum_f [ mean |rgb - target_rgb| + depth_weight * mean over
 * {target_depth > 0} |depth - target_depth| ] (the L1 terms of the paper's
 * rendering loss), and its gradients g_rgb, g_depth, g_alpha (= 0), ready
 * for gsr_backward.  `loss` is a device float.  The images are read from
 * the rgb and depth buffers that last forward wrote, by the pointers it was
 * given: the caller keeps those buffers allocated and unchanged until this
 * call has run on the stream. */
gsr_status gsr_loss_l1(gsr_context* ctx, const float* target_rgb, const float* target_depth,
                       float depth_weight, float* loss, float* g_rgb, float* g_depth,
                       float* g_alpha, void* stream);

/* gsr_loss_l1 for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and error behaviour, but it allocates nothing.
 * Its per-block partial sums and per-frame scale factors live in a static
 * device array of 1 MiB (one copy per GPU, resolved by gsr_create and held
 * until the process ends), which limits it to F * ceil(max W*H / 2048) * 24
 * + 8 F <= 1 MiB bytes (e.g. 43 frames of 1920x1080); a larger last forward
 * returns GSR_ERR_UNSUPPORTED without launching anything.  All calls on one
 * GPU share that array: calls that overlap on one GPU (any streams or
 * contexts) race; run them in sequence.  Every scratch value a call reads is
 * written by that call first. */
gsr_status gsr_loss_l1_noalloc(gsr_context* ctx, const float* target_rgb,
                               const float* target_depth, float depth_weight, float* loss,
                               float* g_rgb, float* g_depth, float* g_alpha, void* stream);

/* One mapping step: gsr_forward, gsr_loss_l1 and gsr_backward in sequence,
 * with the upstream gradients held in the context. */
gsr_status gsr_step_l1(gsr_context* ctx, const gsr_settings* settings, int64_t n,
                       const float* means, const float* log_scales, const float* quats,
                       const float* opacity_logits, const float* sh, int32_t n_frames,
                       const gsr_camera* cams, const float* poses, const float* target_rgb,
                       const float* target_depth, float depth_weight, float* rgb, float* depth,
                       float* alpha, float* loss, float* g_means, float* g_log_scales,
                       float* g_quats, float* g_opacity_logits, float* g_sh, float* g_twist,
                       void* stream);

/* The paper's full rendering loss (eqn rnd_loss, Sec. 3.3; lambda2 = 0.2 and
 * lambda1 = 0.8 or 0.9 in supplementary S1.2) of images laid out like the
 * last forward's outputs (frame sizes and packing of that forward):
 *   *loss = sum_f ( lambda1 [ (1 - lambda2) mean |rgb - target_rgb|
 *                             + lambda2 (1 - SSIM_f) ]
 *                   + (1 - lambda1) mean over {target_depth > 0} |depth - target_depth| ),
 * SSIM_f = the mean over the 3 channels and all pixels of frame f of Wang et
 * al.'s SSIM map (11x11 Gaussian window of standard deviation 1.5, weights
 * summing to 1; C1 = 0.01^2, C2 = 0.03^2; window sums with zero padding), and
 * its gradients g_rgb, g_depth and g_alpha (= 0), ready for gsr_backward.
 * A frame with no valid target depth has no depth term.  rgb, depth and the
 * targets are device arrays packed like gsr_forward's outputs (the forward's
 * own output buffers may be passed); `loss` is a device float; `ssim`, if
 * not NULL, receives SSIM_f [n_frames] (device floats).  lambda1 and
 * lambda2 must lie in [0, 1] (GSR_ERR_INVALID_ARGUMENT otherwise);
 * GSR_ERR_STATE if no forward preceded.  The SSIM map is evaluated in FP64;
 * the workspace grows by 72 bytes per pixel. */
gsr_status gsr_loss_render(gsr_context* ctx, const float* rgb, const float* depth,
                           const float* target_rgb, const float* target_depth, float lambda1,
                           float lambda2, float* loss, float* ssim, float* g_rgb,
                           float* g_depth, float* g_alpha, void* stream);

/* One mapping step with the full rendering loss: gsr_forward,
 * gsr_loss_render on the forward's outputs and gsr_backward in sequence,
 * with the upstream gradients held in the context.  `ssim` may be NULL. */
gsr_status gsr_step_render(gsr_context* ctx, const gsr_settings* settings, int64_t n,
                           const float* means, const float* log_scales, const float* quats,
                           const float* opacity_logits, const float* sh, int32_t n_frames,
                           const gsr_camera* cams, const float* poses, const float* target_rgb,
                           const float* target_depth, float lambda1, float lambda2, float* rgb,
                           float* depth, float* alpha, float* loss, float* ssim,
                           float* g_means, float* g_log_scales, float* g_quats,
                           float* g_opacity_logits, float* g_sh, float* g_twist, void* stream);

/* Densification statistics (the adaptive density control of the 3DGS
 * lineage that Sec. 3.3 describes: Gaussians are split and cloned by their
 * size and positional gradient).  For every Gaussian g, adds to
 * grad_accum[g] the sum over the frames f where (g, f) was kept by the last
 * forward of |dL/d(u, v)|_2, the norm of the last backward's gradient with
 * respect to the projected mean (pixel units), and adds the number of those
 * frames to count[g].  grad_accum and count [n] are caller-owned device
 * floats, accumulated into (zero them to start).  GSR_ERR_STATE unless a
 * forward and its backward preceded. */
gsr_status gsr_densify_stats(gsr_context* ctx, float* grad_accum, float* count, void* stream);

/* MCMC densification, position noise (Sec. 3.3 and supplementary S1.2, which
 * sets lr_noise = 1e4; the MCMC method the paper cites):
 *   means[g] += scale * gate(o_g) * Sigma_g eps[g],
 * Sigma_g = R_g diag(s_g^2) R_g^T the Gaussian's covariance (s = exp of the
 * log-scales, R from the normalised quaternion), o_g = sigmoid(logit),
 * gate(o) = 1 / (1 + exp(100 (o - 0.995))).  eps [n,3] are the caller's
 * standard normal draws and scale = lr_noise x the current position learning
 * rate.  Evaluated in FP64; means are updated in place. */
gsr_status gsr_mcmc_noise(gsr_context* ctx, int64_t n, float* means, const float* log_scales,
                          const float* quats, const float* opacity_logits, const float* eps,
                          float scale, void* stream);

/* MCMC densification, relocation of dead Gaussians.  src [n] (device int32)
 * gives for each dead Gaussian g the live source i it moves to, and -1 for
 * every other Gaussian (the caller samples the sources, in the method in
 * proportion to opacity, among Gaussians with src = -1; a source must not be
 * dead itself).  A source chosen c times becomes N = c + 1 copies at its
 * place: opacity o' = 1 - (1 - o)^(1/N) (N copies over each other give back
 * o), scales multiplied by o / sum_{m=1}^{N} C(N, m) (-1)^(m-1) o'^m /
 * sqrt(m) (the composited opacity integrates along a line through the
 * centre to the source's), means, quaternion and SH copied to the dead
 * slots.  Entries of src outside [0, n) count as -1; N above 1024 is taken
 * as 1024.  Parameters are updated in place; optimiser moments of the moved
 * Gaussians are the caller's to reset.  Uses 36 bytes of workspace per
 * Gaussian. */
gsr_status gsr_mcmc_relocate(gsr_context* ctx, int64_t n, int32_t sh_degree, float* means,
                             float* log_scales, float* quats, float* opacity_logits, float* sh,
                             const int32_t* src, void* stream);

/* Autotuner: runs gsr_step_l1 with every supported tile shape (16x16, 8x8,
 * 32x8, 16x8, 32x16) and every LDS batch (32, 64, 128 Gaussians staged per
 * round) on the given inputs: one untimed sizing run per tile shape, then
 * `reps` runs per (shape, batch) timed with HIP events on `stream`.  Writes
 * the fastest settings to *chosen (base settings with tile_w, tile_h and
 * lds_batch replaced and a fixed key_capacity 5% above the measured count);
 * on the fastest shape the default batch of 64 is kept when its time is
 * within 1% of the fastest batch's, so that run-to-run noise does not flip
 * between batches that differ by less than it.
 * ms[GSR_TUNE_BATCHES * i + j] receives the median step time of shape i with
 * batch j in the orders above (array of GSR_TUNE_TILES * GSR_TUNE_BATCHES;
 * NULL allowed).  Results do not depend on the choice: images are bitwise
 * the same for every shape and batch.  The choice is cached in the context
 * per (multiset of frame sizes, n rounded up to a power of two, SH degree);
 * a cached choice is returned without measuring (ms all -1) unless `force`.
 * The library owns the scratch outputs it renders into. */
#define GSR_TUNE_TILES 5
#define GSR_TUNE_BATCHES 3
gsr_status gsr_autotune(gsr_context* ctx, const gsr_settings* base, int64_t n, const float* means,
                        const float* log_scales, const float* quats,
                        const float* opacity_logits, const float* sh, int32_t n_frames,
                        const gsr_camera* cams, const float* poses, const float* target_rgb,
                        const float* target_depth, float depth_weight, int32_t reps,
                        int32_t force, gsr_settings* chosen, float* ms, void* stream);

/* Optimiser step of the mapping loop (one launch sequence): Adam on the means
 * (lr_means) and the SH coefficients (lr_sh), and Adam on each frame's pose
 * twist (lr_pose) followed by the fold T_f <- Exp(xi_f) T_f in FP64 (left
 * perturbation, xi = (rho, phi), Exp = [R(phi), V(phi) rho]).  Log-scales,
 * quaternions and opacities are not updated.  m_* / v_* are caller-owned
 * first/second moment buffers shaped like their parameters (zero before the
 * first step); *step (device int32, 0 before the first step) is the number of
 * steps taken and is incremented on the device, so a captured iteration
 * advances it on every replay.  Bias correction uses step + 1.  n_frames is at
 * most 1024. */
gsr_status gsr_adam_step(gsr_context* ctx, int64_t n, int32_t sh_degree, float* means,
                         const float* g_means, float* m_means, float* v_means, float* sh,
                         const float* g_sh, float* m_sh, float* v_sh, int32_t n_frames,
                         float* poses, const float* g_twist, float* m_twist, float* v_twist,
                         float lr_means, float lr_sh, float lr_pose, float beta1, float beta2,
                         float eps, int32_t* step, void* stream);

/* Synchronises `stream` and returns GSR_ERR_CAPACITY if a fixed-capacity
 * forward since the last check had more keys than key_capacity (its outputs
 * are then undefined), else GSR_OK.  Clears the flag. */
gsr_status gsr_check_overflow(gsr_context* ctx, void* stream);

typedef struct {
  int64_t n_records;    /* n * F */
  int64_t n_keys;       /* (tile, Gaussian) keys of the last forward */
  int64_t n_tiles;      /* tiles over all frames */
  int64_t n_pixels;
  int64_t key_capacity; /* allocated key slots */
  uint32_t epoch;       /* backward calls so far */
  int32_t tile_w, tile_h;
  int64_t n_pairs;      /* evaluated (pixel, entry) pairs of the last forward
                           with GSR_FLAG_COUNT_PAIRS, else -1 */
  int64_t n_culled;     /* (Gaussian, frame) records the last forward culled:
                           behind the near plane, not positive definite,
                           outside the image, too faint, or non-finite */
  int64_t n_nonfinite;  /* Gaussians with a non-finite parameter (means,
                           log-scales, quaternion, opacity logit or an SH
                           coefficient of the rendered degree); each is culled
                           in every frame and its gradients are 0 */
} gsr_stats;

/* Statistics of the last forward (synchronises `stream`).  n_culled and
 * n_nonfinite are counted on the device from the forward's parameter buffers,
 * which must still hold the forward's inputs. */
gsr_status gsr_debug_stats(gsr_context* ctx, gsr_stats* out, void* stream);

/* Per-stage GPU time of every call made with GSR_FLAG_TIMING since the last
 * read: ms[s] = total milliseconds, calls[s] = number of timed launches of
 * stage s (arrays of GSR_N_STAGES).  Synchronises on the recorded events and
 * clears them. */
gsr_status gsr_debug_timings(gsr_context* ctx, double* ms, int64_t* calls);

/* Copies the last forward's integer artefacts to host arrays (synchronises
 * `stream`); any pointer may be NULL.  Record r = f*n + g:
 *   ntiles [n*F]     tiles covered (0 = culled)
 *   depth_key [n*F]  bits of fp32(z) (0xffffffff = culled)
 *   square [n*F*2]   pixel bounds of kept records, x_lo | x_hi << 16,
 *                    y_lo | y_hi << 16: the 3-sigma square clipped to the
 *                    box where alpha can reach 1/255
 *   tile_keys [K], tile_vals [K]  sorted global tile ids and record ids
 *   ranges [T*2]     [start, end) of each tile in the sorted keys
 *   n_last [P]       per pixel, list position after its last blended entry
 *   t_final [P]      per pixel, final transmittance */
gsr_status gsr_debug_lists(gsr_context* ctx, uint32_t* ntiles, uint32_t* depth_key,
                           uint32_t* square, uint32_t* tile_keys, uint32_t* tile_vals,
                           uint32_t* ranges, int32_t* n_last, float* t_final, void* stream);

/* Copies the per-record screen-space gradients of the last backward,
 * [n*F][10] doubles, record r = f*n + g: dL/du, dL/dv, dL/dSigma'_xx,
 * dL/dSigma'_xy, dL/dSigma'_yy (gradient of the symmetric 2x2 projected
 * covariance, off-diagonal counted once), dL/dopacity (of alpha =
 * opacity * G), dL/dcolour[3], dL/dz.  Synchronises `stream`;
 * GSR_ERR_STATE before the first backward. */
gsr_status gsr_debug_grad2d(gsr_context* ctx, double* out, void* stream);

/* Measurement aid: a plain device copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned, device memory, no overlap), one 16-byte element
 * per thread, enqueued on `stream`.  Copies of >= 2 GB give the achievable
 * HBM bandwidth that the sort's bandwidth fraction is reported against. */
gsr_status gsr_debug_copy(gsr_context* ctx, const void* src, void* dst, uint64_t bytes,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif
