/*
 * gso.h -- FP64 CPU oracle of the pose-differentiable 3D Gaussian splatting
 * rasterizer of "Look Gauss, No Pose" (arXiv 2410.08743).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; it is
 * loaded by the tests, by __graft_entry__.smoke() and by the cpu_baseline leg
 * of bench.py, and by nothing else.  It shares no source, header, constant or
 * helper with the GPU library (paper_2410_08743_amd/csrc), and neither side
 * includes or links the other.
 *
 * Every computation is in double precision.  Inputs arrive as doubles (the
 * callers widen FP32 data exactly).  The only non-FP64 quantity is the sort
 * key's depth, which the method quantises to float32 (see gso_splat).
 *
 * Where the paper is silent (thresholds, tile size, dilation, ...), the
 * constants below are the readings recorded in the design notes; they are
 * written here by value, independently of the GPU side.
 */
#ifndef GSO_H
#define GSO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Camera intrinsics and render region.  Pixel (i, j) is evaluated at
 * continuous image coordinates (i + 1/2, j + 1/2); the region of interest
 * (ROI) must start on a multiple of the 16-pixel tile. */
typedef struct {
    int32_t width, height;          /* full image size (drives the J clamp) */
    double fx, fy, cx, cy;          /* pinhole intrinsics, full-image pixels */
    int32_t roi_x, roi_y, roi_w, roi_h;
    double bg[3];                   /* background colour */
} gso_view;

/* Gaussian set G (Sec. III-A): mean, activated scale (> 0), raw quaternion
 * (w, x, y, z), activated opacity in (0, 1), SH coefficients [n][S][3]. */
typedef struct {
    int64_t n;
    int32_t sh_degree;              /* 0..3, S = (sh_degree + 1)^2 */
    const double *means;            /* [n][3] */
    const double *scales;           /* [n][3] */
    const double *quats;            /* [n][4] */
    const double *opacities;        /* [n]    */
    const double *sh;               /* [n][S][3] */
} gso_gaussians;

/* Per-Gaussian projected splat for one view. */
typedef struct {
    double u, v;                    /* projected mean, pixel-index coordinates */
    double cov[3];                  /* dilated 2D covariance (a, b, c) */
    double conic[3];                /* its inverse (A, B, C) */
    double color[3];                /* SH colour after +1/2 and clamp at 0 */
    double p[3];                    /* mean in the camera frame */
    double opacity;
    float depth_key;                /* float32(p_z), the sort key's depth */
    int32_t radius;                 /* ceil(3 sqrt(lambda_max)) */
    int32_t rect[4];                /* tile rect x0, y0, x1, y1 (ROI tiles, half-open) */
    int32_t rendered;               /* 1 when the splat reaches binning */
    int32_t fragile;                /* 1 when a discrete decision is within margin */
    int32_t color_clamped[3];
    int32_t jclamp[2];              /* 1 when x/z (resp. y/z) hit the J clamp */
} gso_splat;

/* Gradient outputs of gso_backward.  NULL members are not written. */
typedef struct {
    double *means;                  /* [n][3] */
    double *scales;                 /* [n][3] */
    double *quats;                  /* [n][4] */
    double *opacities;              /* [n]    */
    double *sh;                     /* [n][S][3] */
    double *splat2d;                /* [n][9]: du dv dA dB dC do dr dg db */
    double *pose;                   /* [6]: (rho, phi), left twist */
    double *pose_parts;             /* [18]: sum g, sum p x g, sum G_W (3x3), sum h */
} gso_grads;

/* One evaluated (pixel, splat) pair, for invariant checks. */
typedef struct {
    int32_t gaussian;
    int32_t position;               /* index in the tile list */
    int32_t blended;                /* 1 blended, 0 skipped */
    int32_t alpha_clamped;
    double power, alpha, T_before;
} gso_trace_entry;

/* Frozen constants. */
#define GSO_TILE        16
#define GSO_NEAR        0.2
#define GSO_DILATION    0.3
#define GSO_JCLAMP      1.3
#define GSO_LAMBDA_MIN  0.1
#define GSO_ALPHA_MAX   0.99
#define GSO_ALPHA_MIN   (1.0 / 255.0)
#define GSO_T_MIN       1e-4

/* Straddle margins for decisions that FP32 and FP64 can take differently. */
#define GSO_MARGIN_INT   1e-9       /* absolute, on a value about to be floor/ceil'd */
#define GSO_MARGIN_NEAR  1e-9       /* absolute, on p_z - near */
/* FP32 bounds the margins cover: a splat's alpha at a pixel carries a
 * relative error of about 1e-6 (conic rounded once, pixel offsets formed from
 * an (hi, lo) centre, one exp), and the transmittance after ~70 blends one of
 * at most ~1.2e-5; 2e-5 covers both. */
#define GSO_MARGIN_ALPHA 2e-5       /* relative, on o*exp(power) vs 1/255 */
#define GSO_MARGIN_T     2e-5       /* relative, on T(1-alpha) vs 1e-4 */
#define GSO_SIGNIFICANT_T 1e-3      /* an alpha straddle below this T is harmless */

int gso_version(void);

/* OpenMP threads the oracle's parallel loops use. */
int gso_max_threads(void);
/* Sets the number of OpenMP threads later calls use (n >= 1). */
void gso_set_threads(int n);

/* Real spherical harmonics up to degree 3 (Condon-Shortley phase, order
 * m = -l..l) at direction d; writes (degree+1)^2 values and, if grad is not
 * NULL, their partial derivatives [(degree+1)^2][3] as polynomials in d. */
void gso_sh_basis(int degree, const double d[3], double *Y, double *grad);

/* Rotation matrix (row-major) of q / |q|, q = (w, x, y, z). */
void gso_quat_to_rotmat(const double q[4], double R[9]);

/* SE(3) exponential of tau = (rho, phi); T = [R | t] row-major 3x4. */
void gso_se3_exp(const double tau[6], double T[12]);

/* Left retraction T <- Exp(delta) T. */
void gso_se3_retract(const double delta[6], double T[12]);

/* Projection of every Gaussian for one view (pose = world->camera [R|t]). */
int gso_preprocess(const gso_gaussians *g, const gso_view *view,
                   const double pose[12], gso_splat *out);

/* Number of (Gaussian, tile) instances over V views. */
int64_t gso_count_instances(int32_t V, int64_t n, const gso_splat *const *splats);

/* Binning + sort over V views: keys (tile << 32 | depth bits) with tile ids
 * offset by the previous views' tile counts, values v * n + i.  Writes the
 * sorted arrays; returns M, or -1 if M exceeds capacity. */
int64_t gso_bin_sort(int32_t V, int64_t n, const gso_splat *const *splats,
                     const int32_t *tiles_x, const int32_t *tiles_y,
                     int64_t capacity, uint64_t *keys, uint32_t *values);

/* Per-tile [start, end) of sorted keys; tiles without instances get [0, 0). */
void gso_tile_ranges(int64_t M, const uint64_t *keys, int64_t ntiles,
                     uint32_t *ranges);

/* Forward render of one view.  image [3][roi_h][roi_w]; T_final and
 * n_contrib [roi_h][roi_w]; straddle (may be NULL) flags pixels whose result
 * depends on a decision within margin; signature (may be NULL) receives a
 * hash of every discrete decision (cull, rects, order, blended sets, stops,
 * clamps).  Returns 0 on success. */
int gso_render(const gso_gaussians *g, const gso_view *view, const double pose[12],
               double *image, double *T_final, int32_t *n_contrib,
               uint8_t *straddle, uint64_t *signature);

/* The same image from the per-pixel definition: every rendered splat whose
 * tile rect contains the pixel's tile, ordered by (depth_key, index), with no
 * tile lists or sorted instance arrays. */
int gso_render_brute(const gso_gaussians *g, const gso_view *view,
                     const double pose[12], double *image, double *T_final);

/* Evaluated pairs of one pixel (absolute coordinates), front to back. */
int gso_pixel_trace(const gso_gaussians *g, const gso_view *view,
                    const double pose[12], int32_t px, int32_t py,
                    gso_trace_entry *entries, int32_t max_entries);

/* Exact derivative of gso_render's image with upstream dl_dimage
 * [3][roi_h][roi_w].  Gradients are written (not accumulated). */
int gso_backward(const gso_gaussians *g, const gso_view *view, const double pose[12],
                 const double *dl_dimage, gso_grads *out);

/* Mean absolute error over count values and its gradient w.r.t. a
 * (sign(a - b) / count, 0 where equal).  grad may be NULL. */
double gso_l1(int64_t count, const double *a, const double *b, double *grad);

/* Masked L1 (sum over pixels with 1 - T_final > 0.99 of |a - b|), per-pixel
 * mask applied to all 3 channels of [3][h][w] images. */
double gso_masked_l1(int64_t pixels, const double *a, const double *b,
                     const double *T_final, double *grad);

/* One tangent-space Adam step on a pose: moments m, v in R^6 are updated with
 * gradient g at step k (1-based); delta = -lr mhat / (sqrt(vhat) + eps);
 * T <- Exp(delta) T.  delta_out (may be NULL) receives delta. */
void gso_pose_adam(double T[12], double m[6], double v[6], const double g[6],
                   int32_t k, double lr, double beta1, double beta2, double eps,
                   double delta_out[6]);

#ifdef __cplusplus
}
#endif
#endif
