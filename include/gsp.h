/*
 * gsp.h -- C ABI of the MI355X (gfx950) pose-differentiable 3D Gaussian
 * splatting rasterizer.
 *
 * The library implements the hot path of "Look Gauss, No Pose"
 * (arXiv 2410.08743): render a view of a Gaussian set from a camera with
 * intrinsics K and world-to-camera extrinsics T = (R_c, t_c) (Sec. III-A,
 * Eq. (1)-(4)), and back-propagate an image gradient to the Gaussian
 * parameters and to the camera pose, the latter as a gradient on the se(3)
 * tangent vector tau (Sec. III-B, Eq. (5)-(13)).
 *
 * Conventions shared by every call:
 *  - All pointers marked "device" are HIP device (or managed) memory on the
 *    context's device; pointers marked "host" are ordinary host memory that
 *    the call reads before returning.  The caller owns every buffer.  The
 *    library allocates no device memory after gsp_create.
 *  - Work is enqueued on the given HIP stream (NULL = the default stream) and
 *    calls return without synchronising, except gsp_instances and
 *    gsp_list_pairs.
 *  - Every call returns a gsp_status.  Argument errors return GSP_EINVAL
 *    before anything is enqueued; gsp_last_error() then describes the
 *    problem (thread-local, valid until the next call on the same thread).
 *  - Floats are IEEE binary32.  Poses are world->camera [R | t], row-major
 *    3 x 4.  Quaternions are (w, x, y, z) and need not be normalised; the
 *    library normalises them and differentiates through the normalisation.
 *  - Images are CHW binary32 per view, 3 x roi_h x roi_w; each view's image
 *    and image gradient are passed by their own device pointer (host arrays
 *    of V pointers), so requests of different sizes can share a launch
 *    without being packed.  Per-pixel workspace arrays (T_final, counts) are
 *    packed one view after another in view order.
 *  - The pose gradient is the left-perturbation twist: for T(tau) =
 *    Exp(tau) T with tau = (rho, phi) (translation first), d[V][6] holds
 *    dL/dtau at tau = 0.  Under this convention the camera centre moves by
 *    -R_c^T rho and not at all under phi, which is how the colour term of
 *    Eq. (7) enters (the paper's Eq. (11) prints a mixed convention).
 *  - Rasterizer constants not stated in the paper (16 x 16 tiles, near plane
 *    0.2, covariance dilation 0.3 px^2, Jacobian clamp 1.3 x tan(fov/2),
 *    3-sigma radius, alpha <= 0.99, skip alpha < 1/255, stop before the
 *    transmittance falls below 1e-4) are fixed at build time.
 */
#ifndef GSP_H
#define GSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSP_OK = 0,
    GSP_EINVAL = 1,        /* bad argument; nothing was enqueued */
    GSP_ECAPACITY = 2,     /* more (Gaussian, tile) instances than capacity */
    GSP_ENOMEM = 3,        /* workspace too small for the request */
    GSP_EHIP = 4,          /* a HIP runtime call failed */
    GSP_EUNSUPPORTED = 5   /* not available on this device / build */
} gsp_status;

typedef struct gsp_ctx gsp_ctx;   /* opaque; one per device */

/* Maximum number of views rendered by one call. */
#define GSP_MAX_VIEWS 32

/* Gaussian set G of Sec. III-A.  Device pointers, structure-of-arrays:
 * means [n][3]; scales [n][3] (activated, > 0); quats [n][4] (w, x, y, z,
 * nonzero); opacities [n] (activated, in (0, 1)); sh [n][S][3] with
 * S = (sh_degree + 1)^2, colour = max(0, sum_k sh[k] Y_k(d) + 1/2) where Y is
 * the real spherical-harmonic basis (Condon-Shortley phase, m = -l..l). */
typedef struct {
    const float *means;
    const float *scales;
    const float *quats;
    const float *opacities;
    const float *sh;
    int64_t n;            /* 0 <= n < 2^31 / views */
    int32_t sh_degree;    /* 0..3 */
} gsp_gaussians;

/* One camera (host struct).  Pixel (i, j) of the full image is sampled at
 * continuous coordinates (i + 1/2, j + 1/2); projection is
 * x = fx * X / Z + cx.  The rendered region of interest starts at a multiple
 * of 16 pixels (roi_x, roi_y), lies inside the image and may have any size;
 * it equals the corresponding crop of the full-image render exactly. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    int32_t roi_x, roi_y, roi_w, roi_h;
    float bg[3];          /* background colour, blended with weight T_final */
} gsp_view;

/* Gradient outputs of gsp_render_bwd (device pointers, same layouts as
 * gsp_gaussians).  A NULL member is not computed; when every Gaussian member
 * is NULL only the pose gradient is produced.  Gaussian gradients are summed
 * over the call's views.  pose: device [V][6], may be NULL. */
typedef struct {
    float *means;
    float *scales;
    float *quats;
    float *opacities;
    float *sh;
    float *pose;
} gsp_grads;

/* Flags for gsp_render_bwd. */
#define GSP_ACCUMULATE 1u  /* add into the gradient buffers instead of overwriting */

/* Hyper-parameters of the tangent-space Adam step (gsp_pose_adam).  The
 * learning rate follows a cosine decay from lr_start to lr_end over
 * total_steps steps (constant when they are equal).  parametrization
 * selects the group the step moves in: GSP_POSE_SE3 (the paper's, Sec.
 * III-B: poses in SE(3), update retracted on the left) or GSP_POSE_T_SO3
 * (the decoupled alternative the paper leaves to future work, Sec. IV-A:
 * camera centre c in R^3 and rotation in SO(3) separately; the twist
 * gradient (rho, phi) maps to dL/dc = -R^T dL/drho and dL/dphi, the step
 * moves c <- c + delta_c and R <- Exp(delta_phi) R, i.e. rotates about the
 * camera centre). */
#define GSP_POSE_SE3 0
#define GSP_POSE_T_SO3 1
typedef struct {
    float lr_start, lr_end;
    int32_t total_steps;
    float beta1, beta2, eps;
    int32_t parametrization;
} gsp_adam_params;

/* Creates a context on HIP device `device` (validates that it is gfx950). */
gsp_status gsp_create(int device, gsp_ctx **out);
gsp_status gsp_destroy(gsp_ctx *ctx);

/* Bytes of device workspace that a render of V views of n Gaussians with room
 * for `instance_capacity` (Gaussian, tile) pairs needs.  The same workspace
 * carries the forward state (projected splats, sorted instances, tile ranges,
 * per-pixel T_final and contributor counts) to the backward. */
gsp_status gsp_workspace_size(int64_t n, int32_t sh_degree, int32_t V, const gsp_view *views,
                              int64_t instance_capacity, size_t *bytes);

/* Forward render (Sec. III-A): projection and EWA covariance (Eq. (1)-(2)),
 * SH colour, tile binning, the (tile, depth, index) order of the instances
 * (the order a stable sort on the 64-bit key tile << 32 | depth bits gives),
 * per-tile ranges and front-to-back compositing (Eq. (3)-(4)).
 *   g          Gaussians (device arrays)
 *   V, views   1..GSP_MAX_VIEWS host view descriptors
 *   poses      device [V][3][4] world->camera
 *   images     host array of V device pointers; images[v] receives view v,
 *              3 x roi_h x roi_w
 *   alphas     NULL, or a host array of V device pointers (entries may be
 *              NULL); alphas[v] receives 1 - T_final, roi_h x roi_w
 *   workspace  device, ws_bytes >= gsp_workspace_size(..., instance_capacity)
 * When the number of instances M exceeds instance_capacity the excess work is
 * skipped on the device and the outputs are undefined; gsp_instances then
 * reports the overflow and the M needed.  Returns GSP_OK once enqueued. */
gsp_status gsp_render_fwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                          const float *poses, float *const *images, float *const *alphas,
                          void *workspace, size_t ws_bytes, int64_t instance_capacity,
                          void *stream);

/* Backward of the last gsp_render_fwd made with this workspace and the same
 * g, views, poses and capacity.  dl_dimages: host array of V device pointers,
 * dl_dimages[v] laid out like images[v].
 * The per-pixel lists are recomputed back to front from T_final and the
 * contributor count instead of being stored; gradients of the 2D splats are
 * reduced per (tile, Gaussian) and then per Gaussian in a fixed order, and
 * the per-view pose gradient (Eq. (7)-(13)) is reduced with wavefront
 * shuffles and block reductions in a fixed order, so results are
 * bit-reproducible run to run. */
gsp_status gsp_render_bwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                          const float *poses, const float *const *dl_dimages,
                          void *workspace, size_t ws_bytes, int64_t instance_capacity,
                          const gsp_grads *grads, uint32_t flags, void *stream);

/* One pose-solve iteration's backward and update (Sec. III-B): the pose-only
 * gsp_render_bwd (grads->pose = dpose, no Gaussian gradient, no flags)
 * followed by gsp_pose_adam(V, poses, dpose, m, v, steps, params,
 * guard_workspace = workspace), in the same launches as the backward alone:
 * the kernel that sums each view's pose gradient also applies its Adam
 * step.  Results are bit-identical to the two calls.  poses is read by the
 * backward (the poses of the forward) and then updated in place; dpose
 * [V][6], m, v [V][6], steps [V]: device.  Argument errors as the two
 * calls; an overflowed render skips the step on the device. */
gsp_status gsp_render_bwd_pose_step(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                    const gsp_view *views, float *poses,
                                    const float *const *dl_dimages, void *workspace, size_t ws_bytes,
                                    int64_t instance_capacity, float *dpose, float *m, float *v,
                                    int32_t *steps, const gsp_adam_params *params, void *stream);

/* Render and L1 photometric loss in one pass (the pose-estimation objective
 * of Sec. III-B with the L1 term of Eq. (16)): renders exactly as
 * gsp_render_fwd, and in place of each image writes into dl_dimages[v] the
 * gradient gsp_loss_l1 would compute from that image and targets[v]:
 * sign(image - target) / (3 roi_h roi_w), 0 where equal -- bit for bit the
 * same.  The images themselves are not stored.  The workspace then holds
 * this forward for gsp_render_bwd exactly as after gsp_render_fwd.
 *   targets, dl_dimages  host arrays of V device pointers, CHW FP32 like
 *                        the images (targets read, dl_dimages written)
 *   loss                 device float [V] or NULL: mean |image - target| of
 *                        each view, summed in FP64 in a fixed order (tile by
 *                        tile; bit-reproducible, though its last bits may
 *                        differ from gsp_loss_l1's block order)
 * Other arguments and errors as gsp_render_fwd. */
gsp_status gsp_render_fwd_l1(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                             const gsp_view *views, const float *poses,
                             const float *const *targets, float *const *dl_dimages,
                             float *const *alphas, float *loss, void *workspace, size_t ws_bytes,
                             int64_t instance_capacity, void *stream);

/* Stored-list mode (the alternative to recomputation in the backward).
 * The backward of Eq. (3)-(4) needs, for every pixel, the alpha_i of its
 * blended splats and the transmittance T_i in front of each.  gsp_render_bwd
 * recomputes them back to front from T_final (T_i = T_{i+1} / (1 - alpha_i)),
 * which keeps only 8 bytes of per-pixel state.  This mode stores them
 * instead: gsp_render_fwd_store renders exactly as gsp_render_fwd and then
 * writes, for each pixel and each blended splat front to back, a 12-byte
 * record (list position in the pixel's tile, alpha_i negated when the 0.99
 * clamp is active, T_i) into a caller buffer `lists`; gsp_render_bwd_stored
 * is gsp_render_bwd reading those records instead of recomputing them
 * (same outputs, to FP32 rounding of the recovered transmittances).
 *   lists          device, lists_bytes >= gsp_lists_bytes(V, views,
 *                  pair_capacity); the same buffer and capacity must reach
 *                  the backward.  Layout: a 64-byte header (uint32 [0], [1]
 *                  low and high words of the number of stored pairs of the
 *                  last forward, [2] nonzero when it exceeded pair_capacity,
 *                  [3] nonzero when any forward did since the caller zeroed
 *                  the buffer), then per-pixel counts and offsets and the
 *                  records.
 *   pair_capacity  records the buffer holds (0 .. 2^32 - 2).
 * When a forward's pairs exceed pair_capacity its records are not written
 * and the stored backward of it produces zero gradients; gsp_list_pairs
 * reports the overflow and the count needed.  Errors as gsp_render_fwd /
 * gsp_render_bwd, plus GSP_EINVAL for a NULL `lists` and GSP_ENOMEM for a
 * buffer smaller than gsp_lists_bytes.  gsp_lists_bytes returns 0 for
 * invalid views or capacity. */
size_t gsp_lists_bytes(int32_t V, const gsp_view *views, int64_t pair_capacity);
gsp_status gsp_render_fwd_store(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                const gsp_view *views, const float *poses, float *const *images,
                                float *const *alphas, void *workspace, size_t ws_bytes,
                                int64_t instance_capacity, void *lists, size_t lists_bytes,
                                int64_t pair_capacity, void *stream);
gsp_status gsp_render_bwd_stored(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                 const gsp_view *views, const float *poses,
                                 const float *const *dl_dimages, void *workspace, size_t ws_bytes,
                                 int64_t instance_capacity, const void *lists, size_t lists_bytes,
                                 int64_t pair_capacity, const gsp_grads *grads, uint32_t flags,
                                 void *stream);
/* Synchronises `stream` and reports the pairs stored by the last forward in
 * `lists` and whether that or any earlier forward (since the caller zeroed
 * the buffer) exceeded its pair capacity. */
gsp_status gsp_list_pairs(gsp_ctx *ctx, const void *lists, void *stream, int64_t *pairs_out,
                          int32_t *overflow_out);

/* Synchronises `stream` and reports the instance count M of the last forward
 * in `workspace`, and whether that forward or any earlier one on the same
 * workspace (since the caller zero-filled it) exceeded its capacity.  The
 * workspace keeps these counters in its first 64 bytes, as uint32: [0], [1]
 * the low and high words of M, [2] nonzero when the last forward overflowed,
 * [4] nonzero when any forward did; a caller may copy them asynchronously
 * instead of calling this function. */
gsp_status gsp_instances(gsp_ctx *ctx, const void *workspace, void *stream,
                         int64_t *m_out, int32_t *overflow_out);

/* Mean absolute error (the L1 part of Eq. (16)) of each view:
 * loss[v] = mean |pred[v] - target[v]| over its 3 x roi_h x roi_w values,
 * grad[v] = sign(pred[v] - target[v]) / (3 roi_h roi_w) (0 where equal), so
 * that a view's loss and gradient do not depend on the other views of the
 * call.  pred, target, grad: host arrays of V device pointers.  loss: device
 * float [V] or NULL; when it is given, scratch must be device memory of
 * gsp_loss_l1_scratch_bytes(V, views) bytes, and each loss is reduced in a
 * fixed order (bit-reproducible). */
gsp_status gsp_loss_l1(gsp_ctx *ctx, int32_t V, const gsp_view *views, const float *const *pred,
                       const float *const *target, float *const *grad, float *loss,
                       void *scratch, void *stream);
size_t gsp_loss_l1_scratch_bytes(int32_t V, const gsp_view *views);

/* gsp_loss_l1 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and results, bit for bit, without the scratch argument.
 * The per-block partial sums of the losses go to a fixed array inside the
 * library (GSP_NOALLOC_SCRATCH_BYTES per GPU, held by each GPU the library
 * runs on until the process ends), so with `loss` non-NULL the views of a
 * call may total at most 2^15 blocks of 4096 values (134,217,728 values, e.g.
 * 32 views of 2048 x 2048); larger calls return GSP_EINVAL before anything is
 * enqueued (without `loss` there is no limit).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, threads or
 * contexts) race on it and must be serialised by the caller.  The call
 * allocates nothing. */
#define GSP_NOALLOC_SCRATCH_BYTES (256 * 1024)
gsp_status gsp_loss_l1_noalloc(gsp_ctx *ctx, int32_t V, const gsp_view *views,
                               const float *const *pred, const float *const *target,
                               float *const *grad, float *loss, void *stream);

/* One tangent-space Adam step per view (Sec. III-B: pose T = Exp(tau) with
 * the update retracted on the left): for each v, steps[v] += 1,
 * m, v moments updated with dpose[v], delta = -lr mhat / (sqrt(vhat) + eps),
 * poses[v] <- Exp(delta) poses[v].  poses [V][12], dpose/m/v [V][6],
 * steps [V] int32: device.  V >= 1, no upper limit.  guard_workspace: NULL,
 * or the workspace of the render that produced dpose; when that render
 * overflowed its instance capacity the step is skipped on the device (poses,
 * moments and steps unchanged), so that a caller who learns of the overflow
 * later can repeat the iteration. */
gsp_status gsp_pose_adam(gsp_ctx *ctx, int32_t V, float *poses, const float *dpose,
                         float *m, float *v, int32_t *steps, const gsp_adam_params *params,
                         const void *guard_workspace, void *stream);

/* The pose a twist moves to, and the gradient on the twist itself (Sec.
 * III-B: T(tau) = Exp(tau) T with the left perturbation, tau = (rho, phi)).
 * gsp_twist_apply: out[v] = Exp(tau[v]) poses[v] (tau [V][6], poses and out
 * [V][12] world->camera, device; out may alias poses).  gsp_twist_chain:
 * given dpose[v], the twist gradient that gsp_render_bwd returns at the pose
 * Exp(tau[v]) poses[v], writes dtau[v] = dL/dtau[v] = J(tau[v])^T dpose[v],
 * J the left Jacobian of SE(3) (Exp(tau + delta) = Exp(J delta) Exp(tau) to
 * first order; J = I at tau = 0); dtau must not alias dpose.  V >= 1; FP64
 * inside, FP32 stored. */
gsp_status gsp_twist_apply(gsp_ctx *ctx, int32_t V, const float *tau, const float *poses,
                           float *out, void *stream);
gsp_status gsp_twist_chain(gsp_ctx *ctx, int32_t V, const float *tau, const float *dpose,
                           float *dtau, void *stream);

/* Image loss of the joint refinement, L_RGB of Eq. (16), per view:
 *   loss[v] = (1 - beta) mean |pred - target| + beta (1 - mean SSIM(pred, target))
 * over the 3 x roi_h x roi_w values of view v, and grad[v] = dloss[v]/dpred[v]
 * (the L1 part as in gsp_loss_l1).  SSIM is evaluated per channel at every
 * pixel with an 11 x 11 Gaussian window of standard deviation 1.5 (weights
 * normalised), C1 = 0.01^2, C2 = 0.03^2, and zero padding outside the image
 * (the formulation of the 3DGS loss that Sec. III-C adopts).  Values are
 * expected in [0, 1].  pred, target, grad: host arrays of V device pointers
 * (grad may not alias pred or target).  loss: device float [V] or NULL.
 * scratch: device memory of at least gsp_loss_rgb_scratch_bytes(V, views)
 * bytes (the per-pixel SSIM derivatives and per-tile partial sums); it is
 * needed with or without loss.  Losses are reduced in a fixed order
 * (bit-reproducible), and a view's results do not depend on the other views
 * of the call. */
gsp_status gsp_loss_rgb(gsp_ctx *ctx, int32_t V, const gsp_view *views, const float *const *pred,
                        const float *const *target, float *const *grad, float *loss, float beta,
                        void *scratch, size_t scratch_bytes, void *stream);
size_t gsp_loss_rgb_scratch_bytes(int32_t V, const gsp_view *views);

/* Raw Gaussian parameters of the joint refinement (device, updated in place
 * by gsp_gaussian_adam): means [n][3], log_scales [n][3] (scales =
 * exp(log_scales)), quats [n][4] (raw; normalised by the renderer),
 * logit_opacities [n] (opacities = sigmoid(logit)), sh [n][S][3]. */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *logit_opacities;
    float *sh;
} gsp_gaussian_params;

/* Hyper-parameters of gsp_gaussian_adam (double, so that decimal values
 * such as beta2 = 0.999 reach the update unrounded).  The means' learning
 * rate decays
 * log-linearly from lr_means_start at step 1 to lr_means_end at step
 * total_steps (held after it); the SH degree-0 coefficients use lr_sh_dc,
 * the higher ones lr_sh_rest.  aniso_r is the ratio r of Eq. (17) and
 * aniso_weight its weight in the objective (Eq. (15): 1; 0 turns it off). */
typedef struct {
    double lr_means_start, lr_means_end;
    int32_t total_steps;
    double lr_sh_dc, lr_sh_rest, lr_opacities, lr_scales, lr_quats;
    double beta1, beta2, eps;
    double aniso_r, aniso_weight;
} gsp_gaussian_adam_params;

/* One Adam step (step = 1, 2, ...; bias-corrected) on the raw Gaussian
 * parameters, given `grads` (means, scales, quats, opacities, sh all
 * non-NULL) from gsp_render_bwd, i.e. gradients with respect to the
 * activated parameters: the kernel applies the activations' chain rule and
 * adds aniso_weight * dL_An/dscales (Eq. (17); for tied scales the first
 * index is the max, resp. min).  m, v: device float arrays of n (11 + 3 S)
 * moments each, laid out group after group in the order of
 * gsp_gaussian_params.  scales_out [n][3], opacities_out [n]: device, receive
 * exp(log_scales) and sigmoid(logit_opacities) after the step (the arrays a
 * gsp_gaussians for the next render points at, with means, quats and sh
 * taken from `params`).  aniso_loss: device float or NULL; receives L_An of
 * the parameters before the step, and then needs scratch of
 * gsp_gaussian_adam_scratch_bytes(n) bytes.  guard_workspace as for
 * gsp_pose_adam (on overflow nothing is written). */
gsp_status gsp_gaussian_adam(gsp_ctx *ctx, int64_t n, int32_t sh_degree,
                             const gsp_gaussian_params *params, const gsp_grads *grads, float *m,
                             float *v, int32_t step, const gsp_gaussian_adam_params *hp,
                             float *scales_out, float *opacities_out, float *aniso_loss,
                             void *scratch, const void *guard_workspace, void *stream);
size_t gsp_gaussian_adam_scratch_bytes(int64_t n);

/* Relative pose estimation between frames t and t+1 (Sec. III-D).
 *
 * gsp_unproject: the scene of frame t from its depth map.  Pixels
 * (stride i, stride j) of the view's region of interest, i < ceil(roi_w /
 * stride), j < ceil(roi_h / stride), become Gaussian k = j * ceil(roi_w /
 * stride) + i at the point of camera-frame depth depth[y][x] on the ray
 * through the pixel's centre (frame t's camera is the world frame), with
 * identity rotation, logit opacity log(opacity / (1 - opacity)), SH
 * degree-0 coefficient (c - 1/2) / Y_0 from the pixel colour c (higher
 * coefficients 0), and isotropic log scale log of the mean distance to its
 * three nearest neighbours (fewer if there are fewer; 0.01 with none).  A
 * pixel whose depth is not a positive finite number gives a Gaussian at
 * depth 1 with logit -30 (it never blends) that is nobody's neighbour.
 *   depth [roi_h][roi_w], image [3][roi_h][roi_w]: device FP32
 *   out: raw parameters of gsp_unproject_count(...) Gaussians (device; sh
 *        [n][(sh_degree+1)^2][3])
 *   scratch: device, gsp_unproject_scratch_bytes(view, stride) bytes
 * The neighbours are found by brute force (n^2 distance tests), so n is
 * limited to 2^18 points (GSP_EINVAL beyond: choose a larger stride). */
gsp_status gsp_unproject_count(const gsp_view *view, int32_t stride, int64_t *n);
size_t gsp_unproject_scratch_bytes(const gsp_view *view, int32_t stride);
gsp_status gsp_unproject(gsp_ctx *ctx, const gsp_view *view, const float *depth,
                         const float *image, int32_t stride, float opacity, int32_t sh_degree,
                         const gsp_gaussian_params *out, void *scratch, size_t scratch_bytes,
                         void *stream);

/* Confidence-masked L1 of Eq. (21) per view: loss[v] = sum over the pixels
 * and channels of M |pred - target| and grad[v] = M sign(pred - target)
 * (0 where equal), with the mask of Eq. (20) M = [alpha > 0.99], alpha the
 * accumulated opacity 1 - T_final that gsp_render_fwd writes (decided in
 * FP64 on the FP32 value).  pred, target, alpha, grad: host arrays of V
 * device pointers; loss: device float [V] or NULL (then scratch may be
 * NULL), else scratch of gsp_loss_masked_l1_scratch_bytes(V, views) bytes;
 * fixed-order reduction. */
gsp_status gsp_loss_masked_l1(gsp_ctx *ctx, int32_t V, const gsp_view *views,
                              const float *const *pred, const float *const *target,
                              const float *const *alpha, float *const *grad, float *loss,
                              void *scratch, void *stream);
size_t gsp_loss_masked_l1_scratch_bytes(int32_t V, const gsp_view *views);

/* Workspace introspection for tests: device pointer and element count of an
 * intermediate array of the last forward/backward.  Names: "geom" (float4
 * pairs per view-Gaussian: u_hi v_hi u_lo v_lo | A2 B2 C2 log2(o), with
 * the conic [[A, B], [B, C]] stored as (A2, B2, C2) = -log2(e) (A/2, B, C/2)),
 * "color" (float4),
 * "rect" (uint16 x0 y0 x1 y1), "depth" (uint32 float bits), "tiles"
 * (uint32 count), "offsets" (uint32 first emission position, i.e. gradient
 * slot, of each view-Gaussian, in index order),
 * "keys" (uint32 global tile id of each sorted instance; the depth part of
 * the 64-bit key is "depth" of its value), "values" (uint32 sorted),
 * "ranges" (uint32 pairs per tile), "tfinal" (float per pixel),
 * "ncontrib" (uint32 per pixel), "neval", "nblend" (uint32 per pixel, see
 * GSP_PROFILE_COUNTS), "grad2d" (float [V*n][9]: du dv dA dB dC
 * do dr dg db; do is zero after a backward that asked for no opacity
 * gradient), "counters" (uint32: M, overflow). */
gsp_status gsp_inspect(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                       void *workspace, size_t ws_bytes, int64_t instance_capacity,
                       const char *name, void **ptr, int64_t *count);

/* Measurement modes (bit mask for gsp_profile_enable).
 * GSP_PROFILE_TIMING: every stage of gsp_render_fwd / gsp_render_bwd
 * (preprocess, duplicate, tile_sort, ranges, depth_order, raster_fwd, raster_bwd,
 * preprocess_bwd) and the gsp_loss_l1, gsp_loss_rgb, gsp_pose_adam and
 * gsp_gaussian_adam kernels are
 * bracketed by HIP events recorded on the call's stream.
 * GSP_PROFILE_COUNTS: the forward rasterizer also counts, per pixel, the
 * (pixel, splat) pairs it evaluated and blended (gsp_inspect "neval",
 * "nblend"); a slower variant, meant for a separate measurement pass.
 * gsp_profile_read waits for the recorded events and returns, for up to
 * max_stages stages, the stage name (NUL-terminated, < 32 chars), the number
 * of launches and the summed milliseconds since the previous read; *n_out is
 * the number of stages written.  Not thread-safe per context. */
#define GSP_PROFILE_TIMING 1
#define GSP_PROFILE_COUNTS 2
gsp_status gsp_profile_enable(gsp_ctx *ctx, int mode);
gsp_status gsp_profile_read(gsp_ctx *ctx, int32_t max_stages, char *names /* [max][32] */,
                            int64_t *counts, double *ms, int32_t *n_out);

const char *gsp_status_string(gsp_status s);
const char *gsp_last_error(void);
int gsp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GSP_H */
