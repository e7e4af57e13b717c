/*
 * gso.c -- FP64 CPU oracle of the pose-differentiable Gaussian splatting
 * rasterizer of "Look Gauss, No Pose" (arXiv 2410.08743).
 *
 * TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library.  It is independent of the
 * HIP library: no shared source, header, table or helper.
 *
 * Paper passages followed (Sec. = section of the paper):
 *   Sec. III-A, Eq. (1)  3D covariance from quaternion and scale
 *   Sec. III-A           pinhole projection pi(K T mu)
 *   Sec. III-A, Eq. (2)  EWA 2D covariance J R_c Sigma R_c^T J^T
 *   Sec. III-A, Eq. (3)  splat opacity alpha = o exp(-1/2 d^T Sigma^-1 d)
 *   Sec. III-A           SH colour from the viewing direction (mu - o_c)
 *   Sec. III-A, Eq. (4)  depth-sorted front-to-back alpha compositing
 *   Sec. III-B, Eq. (5)-(6)  left-perturbation Lie differential
 *   Sec. III-B, Eq. (7)  pose gradient: 2D mean, 2D covariance and colour terms
 *   Sec. III-B, Eq. (8)/(10) d(T x)/d tau = (I | -[y]x)
 *   Sec. III-B, Eq. (12)-(13) dR_c/d phi_k = [e_k]x R_c
 *   Sec. III-D, Eq. (20)-(21) alpha mask and masked L1
 * The paper leaves the rasterizer's thresholds, tile size and dilation to the
 * 3DGS rasterizer it extends; the constants in gso.h are those readings.
 *
 * Eq. (11) of the paper writes the colour term as dc/dmu (R_c | [o_c]x R_c);
 * under the left perturbation that Eq. (8), (10) and (13) use, the camera
 * centre moves by -R_c^T rho and not at all under phi, so the colour term
 * enters the pose gradient only through rho.  Central differences of
 * gso_render decide between the two (tests/test_oracle_gradients.py).
 */
#include "gso.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int gso_version(void) { return 1; }

int gso_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void gso_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3 (Sec. III-A: c = SH(f, d)).          */
/* ------------------------------------------------------------------------ */

void gso_sh_basis(int degree, const double d[3], double *Y, double *grad)
{
    const double x = d[0], y = d[1], z = d[2];
    const double rpi = sqrt(M_PI);
    const double k0 = 1.0 / (2.0 * rpi);
    const double k1 = sqrt(3.0) / (2.0 * rpi);
    const double k2a = sqrt(15.0) / (2.0 * rpi);
    const double k2b = sqrt(5.0) / (4.0 * rpi);
    const double k2c = sqrt(15.0) / (4.0 * rpi);
    const double k3a = sqrt(35.0 / 2.0) / (4.0 * rpi);
    const double k3b = sqrt(105.0) / (2.0 * rpi);
    const double k3c = sqrt(21.0 / 2.0) / (4.0 * rpi);
    const double k3d = sqrt(7.0) / (4.0 * rpi);
    const double k3e = sqrt(105.0) / (4.0 * rpi);
    double G[16][3];
    memset(G, 0, sizeof G);

    Y[0] = k0;
    if (degree >= 1) {
        Y[1] = -k1 * y;  G[1][1] = -k1;
        Y[2] = k1 * z;   G[2][2] = k1;
        Y[3] = -k1 * x;  G[3][0] = -k1;
    }
    if (degree >= 2) {
        Y[4] = k2a * x * y;                    G[4][0] = k2a * y;  G[4][1] = k2a * x;
        Y[5] = -k2a * y * z;                   G[5][1] = -k2a * z; G[5][2] = -k2a * y;
        Y[6] = k2b * (2 * z * z - x * x - y * y);
        G[6][0] = -2 * k2b * x; G[6][1] = -2 * k2b * y; G[6][2] = 4 * k2b * z;
        Y[7] = -k2a * x * z;                   G[7][0] = -k2a * z; G[7][2] = -k2a * x;
        Y[8] = k2c * (x * x - y * y);          G[8][0] = 2 * k2c * x; G[8][1] = -2 * k2c * y;
    }
    if (degree >= 3) {
        Y[9] = -k3a * y * (3 * x * x - y * y);
        G[9][0] = -6 * k3a * x * y; G[9][1] = -k3a * (3 * x * x - 3 * y * y);
        Y[10] = k3b * x * y * z;
        G[10][0] = k3b * y * z; G[10][1] = k3b * x * z; G[10][2] = k3b * x * y;
        Y[11] = -k3c * y * (4 * z * z - x * x - y * y);
        G[11][0] = 2 * k3c * x * y; G[11][1] = -k3c * (4 * z * z - x * x - 3 * y * y);
        G[11][2] = -8 * k3c * y * z;
        Y[12] = k3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
        G[12][0] = -6 * k3d * x * z; G[12][1] = -6 * k3d * y * z;
        G[12][2] = k3d * (6 * z * z - 3 * x * x - 3 * y * y);
        Y[13] = -k3c * x * (4 * z * z - x * x - y * y);
        G[13][0] = -k3c * (4 * z * z - 3 * x * x - y * y); G[13][1] = 2 * k3c * x * y;
        G[13][2] = -8 * k3c * x * z;
        Y[14] = k3e * z * (x * x - y * y);
        G[14][0] = 2 * k3e * x * z; G[14][1] = -2 * k3e * y * z; G[14][2] = k3e * (x * x - y * y);
        Y[15] = -k3a * x * (x * x - 3 * y * y);
        G[15][0] = -k3a * (3 * x * x - 3 * y * y); G[15][1] = 6 * k3a * x * y;
    }
    if (grad) {
        const int S = (degree + 1) * (degree + 1);
        for (int k = 0; k < S; k++)
            for (int c = 0; c < 3; c++) grad[3 * k + c] = G[k][c];
    }
}

/* ------------------------------------------------------------------------ */
/* Rotations and SE(3) (Sec. III-A Eq. (1); Sec. III-B).                     */
/* ------------------------------------------------------------------------ */

void gso_quat_to_rotmat(const double q[4], double R[9])
{
    const double nrm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nrm, x = q[1] / nrm, y = q[2] / nrm, z = q[3] / nrm;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* d R(qhat) / d qhat_c for c = w, x, y, z (unit quaternion entries). */
static void rotmat_dq(const double qh[4], double dR[4][9])
{
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    double Dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    double Dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    double Dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    double Dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    memcpy(dR[0], Dw, sizeof Dw);
    memcpy(dR[1], Dx, sizeof Dx);
    memcpy(dR[2], Dy, sizeof Dy);
    memcpy(dR[3], Dz, sizeof Dz);
}

static void skew(const double a[3], double S[9])
{
    S[0] = 0;     S[1] = -a[2]; S[2] = a[1];
    S[3] = a[2];  S[4] = 0;     S[5] = -a[0];
    S[6] = -a[1]; S[7] = a[0];  S[8] = 0;
}

static void mat3_mul(const double A[9], const double B[9], double C[9])
{
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

void gso_se3_exp(const double tau[6], double T[12])
{
    const double *rho = tau, *phi = tau + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double a, b, c; /* sin(t)/t, (1-cos t)/t^2, (t - sin t)/t^3 */
    if (th < 1e-4) {
        a = 1 - th2 / 6 + th2 * th2 / 120;
        b = 0.5 - th2 / 24 + th2 * th2 / 720;
        c = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040;
    } else {
        a = sin(th) / th;
        b = (1 - cos(th)) / th2;
        c = (th - sin(th)) / (th2 * th);
    }
    double K[9], K2[9], R[9], V[9];
    skew(phi, K);
    mat3_mul(K, K, K2);
    for (int i = 0; i < 9; i++) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + a * K[i] + b * K2[i];
        V[i] = I + b * K[i] + c * K2[i];
    }
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) T[4 * i + j] = R[3 * i + j];
        T[4 * i + 3] = V[3 * i] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
    }
}

void gso_se3_retract(const double delta[6], double T[12])
{
    double E[12], out[12];
    gso_se3_exp(delta, E);
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 4; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += E[4 * i + k] * T[4 * k + j];
            if (j == 3) s += E[4 * i + 3];
            out[4 * i + j] = s;
        }
    }
    memcpy(T, out, sizeof out);
}

/* ------------------------------------------------------------------------ */
/* Preprocess: projection, EWA covariance, radius, tile rect, colour.        */
/* ------------------------------------------------------------------------ */

static int near_integer(double x)
{
    return fabs(x - nearbyint(x)) <= GSO_MARGIN_INT;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void view_tiles(const gso_view *vw, int *gw, int *gh, int *ox, int *oy)
{
    *gw = (vw->roi_w + GSO_TILE - 1) / GSO_TILE;
    *gh = (vw->roi_h + GSO_TILE - 1) / GSO_TILE;
    *ox = vw->roi_x / GSO_TILE;
    *oy = vw->roi_y / GSO_TILE;
}

/* Quantities of one Gaussian that the forward and the backward share. */
typedef struct {
    double p[3], z;
    double W[9];          /* camera rotation R_c */
    double Rq[9];         /* rotation of the Gaussian */
    double Sigma[9];      /* 3D covariance, Eq. (1) */
    double J[6];          /* clamped projection Jacobian, 2x3 */
    double T2[6];         /* J W */
    double cov[3], det;
    double xz, yz;        /* clamped x/z, y/z */
    double dir[3], dist;  /* viewing direction and |mu - o_c| */
    double Y[16], dY[48];
} gso_geom;

static void camera_point(const double pose[12], const double mu[3], double p[3])
{
    for (int k = 0; k < 3; k++)
        p[k] = fma(pose[4 * k + 2], mu[2],
                   fma(pose[4 * k + 1], mu[1], fma(pose[4 * k + 0], mu[0], pose[4 * k + 3])));
}

/* Returns 1 when the Gaussian passes the near-plane and determinant tests. */
static int geometry(const gso_gaussians *g, int64_t i, const gso_view *vw,
                    const double pose[12], gso_geom *G, gso_splat *s)
{
    const double *mu = g->means + 3 * i;
    camera_point(pose, mu, G->p);
    G->z = G->p[2];
    s->p[0] = G->p[0]; s->p[1] = G->p[1]; s->p[2] = G->p[2];
    s->depth_key = (float)G->p[2];
    s->opacity = g->opacities[i];
    if (fabs(G->z - GSO_NEAR) <= GSO_MARGIN_NEAR) s->fragile = 1;
    if (!(G->z > GSO_NEAR)) return 0;

    const double z = G->z;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) G->W[3 * r + c] = pose[4 * r + c];

    /* Sec. III-A: mu_hat = pi(K T mu), pixel-index coordinates. */
    s->u = vw->fx * G->p[0] / z + vw->cx - 0.5;
    s->v = vw->fy * G->p[1] / z + vw->cy - 0.5;

    /* Jacobian of the perspective map, with the view-frustum clamp. */
    const double limx = GSO_JCLAMP * 0.5 * vw->width / vw->fx;
    const double limy = GSO_JCLAMP * 0.5 * vw->height / vw->fy;
    double xz = G->p[0] / z, yz = G->p[1] / z;
    if (xz < -limx || xz > limx) { s->jclamp[0] = 1; xz = xz < 0 ? -limx : limx; }
    if (yz < -limy || yz > limy) { s->jclamp[1] = 1; yz = yz < 0 ? -limy : limy; }
    G->xz = xz; G->yz = yz;
    G->J[0] = vw->fx / z; G->J[1] = 0;            G->J[2] = -vw->fx * xz / z;
    G->J[3] = 0;          G->J[4] = vw->fy / z;   G->J[5] = -vw->fy * yz / z;

    /* Eq. (1): Sigma = R(q) diag(s) diag(s)^T R(q)^T. */
    const double *sc = g->scales + 3 * i;
    gso_quat_to_rotmat(g->quats + 4 * i, G->Rq);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += G->Rq[3 * r + k] * sc[k] * sc[k] * G->Rq[3 * c + k];
            G->Sigma[3 * r + c] = acc;
        }

    /* Eq. (2): Sigma_hat = [J R_c Sigma R_c^T J^T]_2x2, plus the dilation. */
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += G->J[3 * r + k] * G->W[3 * k + c];
            G->T2[3 * r + c] = acc;
        }
    double cv[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            cv[0] += G->T2[a] * G->Sigma[3 * a + b] * G->T2[b];
            cv[1] += G->T2[a] * G->Sigma[3 * a + b] * G->T2[3 + b];
            cv[2] += G->T2[3 + a] * G->Sigma[3 * a + b] * G->T2[3 + b];
        }
    cv[0] += GSO_DILATION;
    cv[2] += GSO_DILATION;
    G->cov[0] = cv[0]; G->cov[1] = cv[1]; G->cov[2] = cv[2];
    G->det = cv[0] * cv[2] - cv[1] * cv[1];
    s->cov[0] = cv[0]; s->cov[1] = cv[1]; s->cov[2] = cv[2];
    if (!(G->det > 0)) return 0;
    s->conic[0] = cv[2] / G->det;
    s->conic[1] = -cv[1] / G->det;
    s->conic[2] = cv[0] / G->det;

    /* Sec. III-A colour: direction from the camera centre o_c = -R_c^T t_c. */
    double oc[3];
    for (int k = 0; k < 3; k++)
        oc[k] = -(pose[k] * pose[3] + pose[4 + k] * pose[7] + pose[8 + k] * pose[11]);
    double w[3] = {mu[0] - oc[0], mu[1] - oc[1], mu[2] - oc[2]};
    G->dist = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int k = 0; k < 3; k++) G->dir[k] = w[k] / G->dist;
    gso_sh_basis(g->sh_degree, G->dir, G->Y, G->dY);
    const int S = (g->sh_degree + 1) * (g->sh_degree + 1);
    const double *f = g->sh + (int64_t)3 * S * i;
    for (int c = 0; c < 3; c++) {
        double acc = 0;
        for (int k = 0; k < S; k++) acc += f[3 * k + c] * G->Y[k];
        acc += 0.5;
        if (acc < 0) { s->color_clamped[c] = 1; acc = 0; }
        s->color[c] = acc;
    }
    return 1;
}

static void preprocess_one(const gso_gaussians *g, int64_t i, const gso_view *vw,
                           const double pose[12], gso_splat *s, gso_geom *G)
{
    memset(s, 0, sizeof *s);
    if (!geometry(g, i, vw, pose, G, s)) return;

    /* 3-sigma radius from the larger eigenvalue of Sigma_hat. */
    const double mid = 0.5 * (G->cov[0] + G->cov[2]);
    const double disc = mid * mid - G->det;
    const double lam = mid + sqrt(disc > GSO_LAMBDA_MIN ? disc : GSO_LAMBDA_MIN);
    const double r3 = 3.0 * sqrt(lam);
    if (near_integer(r3)) s->fragile = 1;
    const int r = (int)ceil(r3);
    s->radius = r;

    /* Tile rect, clamped to the region of interest's tile grid. */
    int gw, gh, ox, oy;
    view_tiles(vw, &gw, &gh, &ox, &oy);
    const double bx0 = (s->u - r) / GSO_TILE, bx1 = (s->u + r + GSO_TILE - 1) / GSO_TILE;
    const double by0 = (s->v - r) / GSO_TILE, by1 = (s->v + r + GSO_TILE - 1) / GSO_TILE;
    if (near_integer(bx0) || near_integer(bx1) || near_integer(by0) || near_integer(by1))
        s->fragile = 1;
    s->rect[0] = clampi((int)floor(bx0) - ox, 0, gw);
    s->rect[1] = clampi((int)floor(by0) - oy, 0, gh);
    s->rect[2] = clampi((int)floor(bx1) - ox, 0, gw);
    s->rect[3] = clampi((int)floor(by1) - oy, 0, gh);
    s->rendered = (s->rect[2] - s->rect[0]) * (s->rect[3] - s->rect[1]) > 0;
}

int gso_preprocess(const gso_gaussians *g, const gso_view *view, const double pose[12],
                   gso_splat *out)
{
    if (!g || !view || !pose || !out || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) {
        gso_geom G;
        preprocess_one(g, i, view, pose, out + i, &G);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Binning, sort, tile ranges.                                                */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; uint32_t value; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->value != y->value) return x->value < y->value ? -1 : 1;
    return 0;
}

static uint32_t float_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

int64_t gso_count_instances(int32_t V, int64_t n, const gso_splat *const *splats)
{
    int64_t M = 0;
    for (int32_t v = 0; v < V; v++)
        for (int64_t i = 0; i < n; i++) {
            const gso_splat *s = splats[v] + i;
            if (s->rendered) M += (int64_t)(s->rect[2] - s->rect[0]) * (s->rect[3] - s->rect[1]);
        }
    return M;
}

int64_t gso_bin_sort(int32_t V, int64_t n, const gso_splat *const *splats,
                     const int32_t *tiles_x, const int32_t *tiles_y,
                     int64_t capacity, uint64_t *keys, uint32_t *values)
{
    const int64_t M = gso_count_instances(V, n, splats);
    if (M > capacity) return -1;
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (size_t)(M > 0 ? M : 1));
    if (!kv) return -1;
    int64_t m = 0, base = 0;
    for (int32_t v = 0; v < V; v++) {
        for (int64_t i = 0; i < n; i++) {
            const gso_splat *s = splats[v] + i;
            if (!s->rendered) continue;
            const uint64_t dbits = float_bits(s->depth_key);
            for (int ty = s->rect[1]; ty < s->rect[3]; ty++)
                for (int tx = s->rect[0]; tx < s->rect[2]; tx++) {
                    const uint64_t tile = (uint64_t)(base + (int64_t)ty * tiles_x[v] + tx);
                    kv[m].key = (tile << 32) | dbits;
                    kv[m].value = (uint32_t)(v * n + i);
                    m++;
                }
        }
        base += (int64_t)tiles_x[v] * tiles_y[v];
    }
    qsort(kv, (size_t)M, sizeof(kv_t), kv_cmp);
    for (int64_t k = 0; k < M; k++) { keys[k] = kv[k].key; values[k] = kv[k].value; }
    free(kv);
    return M;
}

void gso_tile_ranges(int64_t M, const uint64_t *keys, int64_t ntiles, uint32_t *ranges)
{
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)ntiles);
    for (int64_t k = 0; k < M; k++) {
        const uint64_t t = keys[k] >> 32;
        if (k == 0 || (keys[k - 1] >> 32) != t) ranges[2 * t] = (uint32_t)k;
        if (k == M - 1 || (keys[k + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(k + 1);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing (Eq. (3)-(4)).                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t pos;          /* list position */
    int32_t gauss;
    int32_t clamped;
    double alpha, T, power, dx, dy;
} blend_rec;

static uint64_t fnv(uint64_t h, uint64_t v)
{
    for (int b = 0; b < 8; b++) {
        h ^= (v >> (8 * b)) & 0xff;
        h *= 1099511628211ULL;
    }
    return h;
}

/* Composites list[0..len) at pixel (px, py).  Returns n_contrib (one past
 * the last blended list position). */
static int composite(const gso_splat *sp, const uint32_t *list, int len,
                     double px, double py, const double bg[3],
                     double rgb[3], double *T_out, int *straddle, uint64_t *hash,
                     blend_rec *rec, int *nrec,
                     gso_trace_entry *trace, int *ntrace, int max_trace)
{
    double T = 1.0, C[3] = {0, 0, 0};
    int last = 0, nb = 0, nt = 0, stop = -1;
    uint64_t h = 1469598103934665603ULL;
    for (int k = 0; k < len; k++) {
        const gso_splat *s = sp + list[k];
        const double dx = s->u - px, dy = s->v - py;
        const double power = -0.5 * (s->conic[0] * dx * dx + s->conic[2] * dy * dy)
                             - s->conic[1] * dx * dy;
        if (straddle && fabs(power) <= 1e-12) *straddle = 1;
        if (power > 0) continue;
        const double a_pre = s->opacity * exp(power);
        if (straddle && T > GSO_SIGNIFICANT_T &&
            fabs(a_pre - GSO_ALPHA_MIN) <= GSO_MARGIN_ALPHA * GSO_ALPHA_MIN)
            *straddle = 1;
        const int clamped = a_pre > GSO_ALPHA_MAX;
        const double alpha = clamped ? GSO_ALPHA_MAX : a_pre;
        const int blended_ok = alpha >= GSO_ALPHA_MIN;
        double testT = T * (1.0 - alpha);
        if (blended_ok && straddle && fabs(testT - GSO_T_MIN) <= GSO_MARGIN_T * GSO_T_MIN)
            *straddle = 1;
        const int stops = blended_ok && testT < GSO_T_MIN;
        const int blends = blended_ok && !stops;
        if (trace && nt < max_trace) {
            trace[nt].gaussian = (int32_t)list[k];
            trace[nt].position = k;
            trace[nt].blended = blends;
            trace[nt].alpha_clamped = clamped;
            trace[nt].power = power;
            trace[nt].alpha = alpha;
            trace[nt].T_before = T;
            nt++;
        }
        if (!blended_ok) continue;
        if (stops) { stop = k; break; }
        if (rec) {
            rec[nb].pos = k; rec[nb].gauss = (int32_t)list[k]; rec[nb].clamped = clamped;
            rec[nb].alpha = alpha; rec[nb].T = T; rec[nb].power = power;
            rec[nb].dx = dx; rec[nb].dy = dy;
        }
        nb++;
        if (hash) h = fnv(fnv(h, list[k]), (uint64_t)clamped);
        for (int c = 0; c < 3; c++) C[c] += s->color[c] * alpha * T;
        T = testT;
        last = k + 1;
    }
    for (int c = 0; c < 3; c++) rgb[c] = C[c] + T * bg[c];
    *T_out = T;
    if (nrec) *nrec = nb;
    if (ntrace) *ntrace = nt;
    if (hash) *hash = fnv(fnv(h, (uint64_t)(int64_t)stop), (uint64_t)last);
    return last;
}

/* ------------------------------------------------------------------------ */
/* Tiled render.                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    gso_splat *sp;
    uint64_t *keys;
    uint32_t *vals;
    uint32_t *ranges;
    int64_t M;
    int gw, gh, ox, oy;
    int maxlen;
} raster_state;

static void state_free(raster_state *st)
{
    free(st->sp); free(st->keys); free(st->vals); free(st->ranges);
    memset(st, 0, sizeof *st);
}

static int state_build(const gso_gaussians *g, const gso_view *vw, const double pose[12],
                       raster_state *st)
{
    memset(st, 0, sizeof *st);
    if (!g || !vw || !pose || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return -1;
    if (vw->roi_x % GSO_TILE || vw->roi_y % GSO_TILE || vw->roi_w <= 0 || vw->roi_h <= 0 ||
        vw->roi_x < 0 || vw->roi_y < 0 || vw->roi_x + vw->roi_w > vw->width ||
        vw->roi_y + vw->roi_h > vw->height)
        return -1;
    view_tiles(vw, &st->gw, &st->gh, &st->ox, &st->oy);
    st->sp = (gso_splat *)malloc(sizeof(gso_splat) * (size_t)(g->n > 0 ? g->n : 1));
    if (!st->sp) return -1;
    gso_preprocess(g, vw, pose, st->sp);
    const gso_splat *const views[1] = {st->sp};
    st->M = gso_count_instances(1, g->n, views);
    st->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(st->M > 0 ? st->M : 1));
    st->vals = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(st->M > 0 ? st->M : 1));
    const int64_t ntiles = (int64_t)st->gw * st->gh;
    st->ranges = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)ntiles);
    if (!st->keys || !st->vals || !st->ranges) { state_free(st); return -1; }
    const int32_t tx = st->gw, ty = st->gh;
    gso_bin_sort(1, g->n, views, &tx, &ty, st->M, st->keys, st->vals);
    gso_tile_ranges(st->M, st->keys, ntiles, st->ranges);
    st->maxlen = 0;
    for (int64_t t = 0; t < ntiles; t++) {
        const int len = (int)(st->ranges[2 * t + 1] - st->ranges[2 * t]);
        if (len > st->maxlen) st->maxlen = len;
    }
    return 0;
}

/* Marks tiles near a fragile Gaussian's rect: their pixels straddle. */
static void fragile_tiles(const gso_gaussians *g, const raster_state *st, uint8_t *tile_flag)
{
    const int64_t ntiles = (int64_t)st->gw * st->gh;
    memset(tile_flag, 0, (size_t)ntiles);
    for (int64_t i = 0; i < g->n; i++) {
        const gso_splat *s = st->sp + i;
        if (!s->fragile) continue;
        if (s->radius == 0) { memset(tile_flag, 1, (size_t)ntiles); return; }
        for (int ty = s->rect[1] - 1; ty <= s->rect[3]; ty++)
            for (int tx = s->rect[0] - 1; tx <= s->rect[2]; tx++)
                if (tx >= 0 && ty >= 0 && tx < st->gw && ty < st->gh)
                    tile_flag[(int64_t)ty * st->gw + tx] = 1;
    }
}

int gso_render(const gso_gaussians *g, const gso_view *vw, const double pose[12],
               double *image, double *T_final, int32_t *n_contrib,
               uint8_t *straddle, uint64_t *signature)
{
    raster_state st;
    if (state_build(g, vw, pose, &st)) return -1;
    const int w = vw->roi_w, hgt = vw->roi_h;
    const int64_t P = (int64_t)w * hgt;
    const int64_t ntiles = (int64_t)st.gw * st.gh;
    uint8_t *tflag = (uint8_t *)malloc((size_t)ntiles);
    uint64_t *phash = signature ? (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P) : NULL;
    if (!tflag || (signature && !phash)) { free(tflag); free(phash); state_free(&st); return -1; }
    fragile_tiles(g, &st, tflag);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < ntiles; t++) {
        const int tx = (int)(t % st.gw), ty = (int)(t / st.gw);
        const uint32_t start = st.ranges[2 * t], end = st.ranges[2 * t + 1];
        uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(end - start + 1));
        for (uint32_t k = start; k < end; k++) list[k - start] = st.vals[k];
        for (int ly = 0; ly < GSO_TILE; ly++)
            for (int lx = 0; lx < GSO_TILE; lx++) {
                const int rx = tx * GSO_TILE + lx, ry = ty * GSO_TILE + ly;
                if (rx >= w || ry >= hgt) continue;
                const int64_t pix = (int64_t)ry * w + rx;
                double rgb[3], T;
                int strad = tflag[t];
                uint64_t hh = 0;
                const int nc = composite(st.sp, list, (int)(end - start),
                                         (double)(vw->roi_x + rx), (double)(vw->roi_y + ry),
                                         vw->bg, rgb, &T, &strad, signature ? &hh : NULL,
                                         NULL, NULL, NULL, NULL, 0);
                if (image)
                    for (int c = 0; c < 3; c++) image[(int64_t)c * P + pix] = rgb[c];
                if (T_final) T_final[pix] = T;
                if (n_contrib) n_contrib[pix] = nc;
                if (straddle) straddle[pix] = (uint8_t)strad;
                if (phash) phash[pix] = hh;
            }
        free(list);
    }

    if (signature) {
        uint64_t h = 1469598103934665603ULL;
        for (int64_t i = 0; i < g->n; i++) {
            const gso_splat *s = st.sp + i;
            h = fnv(h, (uint64_t)s->rendered);
            if (!s->rendered) continue;
            for (int k = 0; k < 4; k++) h = fnv(h, (uint64_t)s->rect[k]);
            h = fnv(h, (uint64_t)s->radius);
            for (int k = 0; k < 3; k++) h = fnv(h, (uint64_t)s->color_clamped[k]);
            h = fnv(h, (uint64_t)(s->jclamp[0] * 2 + s->jclamp[1]));
        }
        for (int64_t k = 0; k < st.M; k++) h = fnv(h, st.vals[k]);
        for (int64_t p = 0; p < P; p++) h = fnv(h, phash[p]);
        *signature = h;
    }
    free(tflag);
    free(phash);
    state_free(&st);
    return 0;
}

static int cmp_depth_index(const void *a, const void *b, const gso_splat *sp)
{
    const uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    const uint32_t di = float_bits(sp[i].depth_key), dj = float_bits(sp[j].depth_key);
    if (di != dj) return di < dj ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

int gso_render_brute(const gso_gaussians *g, const gso_view *vw, const double pose[12],
                     double *image, double *T_final)
{
    if (!g || !vw || !pose || g->n < 0) return -1;
    if (vw->roi_x % GSO_TILE || vw->roi_y % GSO_TILE || vw->roi_w <= 0 || vw->roi_h <= 0)
        return -1;
    gso_splat *sp = (gso_splat *)malloc(sizeof(gso_splat) * (size_t)(g->n > 0 ? g->n : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->n > 0 ? g->n : 1));
    if (!sp || !list) { free(sp); free(list); return -1; }
    gso_preprocess(g, vw, pose, sp);
    const int w = vw->roi_w, hgt = vw->roi_h;
    const int64_t P = (int64_t)w * hgt;
    for (int ry = 0; ry < hgt; ry++)
        for (int rx = 0; rx < w; rx++) {
            const int tx = rx / GSO_TILE, ty = ry / GSO_TILE;
            int len = 0;
            for (int64_t i = 0; i < g->n; i++) {
                const gso_splat *s = sp + i;
                if (s->rendered && tx >= s->rect[0] && tx < s->rect[2] &&
                    ty >= s->rect[1] && ty < s->rect[3])
                    list[len++] = (uint32_t)i;
            }
            /* insertion sort by (depth_key, index): plain and stable */
            for (int a = 1; a < len; a++) {
                const uint32_t x = list[a];
                int b = a - 1;
                while (b >= 0 && cmp_depth_index(&list[b], &x, sp) > 0) { list[b + 1] = list[b]; b--; }
                list[b + 1] = x;
            }
            double rgb[3], T;
            composite(sp, list, len, (double)(vw->roi_x + rx), (double)(vw->roi_y + ry), vw->bg,
                      rgb, &T, NULL, NULL, NULL, NULL, NULL, NULL, 0);
            const int64_t pix = (int64_t)ry * w + rx;
            if (image)
                for (int c = 0; c < 3; c++) image[(int64_t)c * P + pix] = rgb[c];
            if (T_final) T_final[pix] = T;
        }
    free(sp);
    free(list);
    return 0;
}

int gso_pixel_trace(const gso_gaussians *g, const gso_view *vw, const double pose[12],
                    int32_t px, int32_t py, gso_trace_entry *entries, int32_t max_entries)
{
    raster_state st;
    if (state_build(g, vw, pose, &st)) return -1;
    const int rx = px - vw->roi_x, ry = py - vw->roi_y;
    if (rx < 0 || ry < 0 || rx >= vw->roi_w || ry >= vw->roi_h) { state_free(&st); return -1; }
    const int64_t t = (int64_t)(ry / GSO_TILE) * st.gw + rx / GSO_TILE;
    const uint32_t start = st.ranges[2 * t], end = st.ranges[2 * t + 1];
    double rgb[3], T;
    int nt = 0;
    composite(st.sp, st.vals + start, (int)(end - start), (double)px, (double)py, vw->bg,
              rgb, &T, NULL, NULL, NULL, NULL, entries, &nt, max_entries);
    state_free(&st);
    return nt;
}

/* ------------------------------------------------------------------------ */
/* Backward: exact derivative of gso_render.                                  */
/* ------------------------------------------------------------------------ */

/* Chain rule from the splat gradient (du dv dA dB dC do dr dg db) to the 3D
 * parameters, plus this Gaussian's pose contribution (Eq. (7)). */
static void backward_one(const gso_gaussians *g, int64_t i, const gso_view *vw,
                         const double pose[12], const double d2[9],
                         double dmu[3], double dsc[3], double dq[4], double *dop,
                         double *dsh, double parts[18])
{
    gso_splat s;
    gso_geom G;
    memset(&s, 0, sizeof s);
    const int S = (g->sh_degree + 1) * (g->sh_degree + 1);
    memset(dmu, 0, 3 * sizeof(double));
    memset(dsc, 0, 3 * sizeof(double));
    memset(dq, 0, 4 * sizeof(double));
    *dop = 0;
    if (dsh) memset(dsh, 0, sizeof(double) * 3 * (size_t)S);
    memset(parts, 0, 18 * sizeof(double));
    if (!geometry(g, i, vw, pose, &G, &s)) return;

    const double a = G.cov[0], b = G.cov[1], c = G.cov[2], det = G.det, det2 = det * det;
    const double dA = d2[2], dB = d2[3], dC = d2[4];
    /* conic = inverse(cov): derivative of the 2x2 inverse */
    const double da = (-c * c * dA + b * c * dB - b * b * dC) / det2;
    const double db = (2 * b * c * dA - (a * c + b * b) * dB + 2 * a * b * dC) / det2;
    const double dc = (-b * b * dA + a * b * dB - a * a * dC) / det2;
    const double Gh[4] = {da, 0.5 * db, 0.5 * db, dc};  /* dL/dSigma_hat, symmetric */

    /* dL/dT2 = 2 Gh T2 Sigma ; dL/dSigma = T2^T Gh T2 */
    double GhT2[6], GT2[6], GSig[9];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            GhT2[3 * r + k] = Gh[2 * r] * G.T2[k] + Gh[2 * r + 1] * G.T2[3 + k];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int m = 0; m < 3; m++) acc += GhT2[3 * r + m] * G.Sigma[3 * m + k];
            GT2[3 * r + k] = 2 * acc;
        }
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            GSig[3 * r + k] = G.T2[r] * GhT2[k] + G.T2[3 + r] * GhT2[3 + k];

    /* T2 = J W : dL/dJ = dL/dT2 W^T ; dL/dW = J^T dL/dT2 */
    double GJ[6], GW[9];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int m = 0; m < 3; m++) acc += GT2[3 * r + m] * G.W[3 * k + m];
            GJ[3 * r + k] = acc;
        }
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            GW[3 * r + k] = G.J[r] * GT2[k] + G.J[3 + r] * GT2[3 + k];

    /* J -> p, through the clamp */
    const double z = G.z, x = G.p[0], y = G.p[1];
    const double fx = vw->fx, fy = vw->fy;
    double gp[3] = {0, 0, 0};
    gp[2] += GJ[0] * (-fx / (z * z)) + GJ[4] * (-fy / (z * z));
    if (!s.jclamp[0]) {
        gp[0] += GJ[2] * (-fx / (z * z));
        gp[2] += GJ[2] * (2 * fx * x / (z * z * z));
    } else {
        gp[2] += GJ[2] * (fx * G.xz / (z * z));
    }
    if (!s.jclamp[1]) {
        gp[1] += GJ[5] * (-fy / (z * z));
        gp[2] += GJ[5] * (2 * fy * y / (z * z * z));
    } else {
        gp[2] += GJ[5] * (fy * G.yz / (z * z));
    }
    /* projected mean -> p */
    const double du = d2[0], dv = d2[1];
    gp[0] += du * fx / z;
    gp[1] += dv * fy / z;
    gp[2] += -du * fx * x / (z * z) - dv * fy * y / (z * z);

    /* p = R_c mu + t_c -> mu */
    for (int k = 0; k < 3; k++)
        dmu[k] = G.W[k] * gp[0] + G.W[3 + k] * gp[1] + G.W[6 + k] * gp[2];

    /* Sigma = M M^T, M = R_q diag(s) */
    const double *sc = g->scales + 3 * i;
    double Mm[9], GM[9], GRq[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) Mm[3 * r + k] = G.Rq[3 * r + k] * sc[k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int m = 0; m < 3; m++) acc += GSig[3 * r + m] * Mm[3 * m + k];
            GM[3 * r + k] = 2 * acc;
        }
    for (int k = 0; k < 3; k++) {
        double acc = 0;
        for (int r = 0; r < 3; r++) acc += GM[3 * r + k] * G.Rq[3 * r + k];
        dsc[k] = acc;
    }
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) GRq[3 * r + k] = GM[3 * r + k] * sc[k];
    const double *q = g->quats + 4 * i;
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double dR[4][9], dqh[4];
    rotmat_dq(qh, dR);
    for (int k = 0; k < 4; k++) {
        double acc = 0;
        for (int e = 0; e < 9; e++) acc += GRq[e] * dR[k][e];
        dqh[k] = acc;
    }
    const double proj = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
    for (int k = 0; k < 4; k++) dq[k] = (dqh[k] - qh[k] * proj) / qn;

    *dop = d2[5];

    /* colour: SH coefficients and the viewing direction */
    const double *f = g->sh + (int64_t)3 * S * i;
    double ddir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ch++) {
        if (s.color_clamped[ch]) continue;
        const double gc = d2[6 + ch];
        for (int k = 0; k < S; k++) {
            if (dsh) dsh[3 * k + ch] = gc * G.Y[k];
            for (int e = 0; e < 3; e++) ddir[e] += gc * f[3 * k + ch] * G.dY[3 * k + e];
        }
    }
    const double dd = ddir[0] * G.dir[0] + ddir[1] * G.dir[1] + ddir[2] * G.dir[2];
    double dw[3];
    for (int e = 0; e < 3; e++) dw[e] = (ddir[e] - G.dir[e] * dd) / G.dist;
    for (int e = 0; e < 3; e++) dmu[e] += dw[e];

    /* pose parts: g, p x g, dL/dW, h = dL/do_c = -dw */
    parts[0] = gp[0]; parts[1] = gp[1]; parts[2] = gp[2];
    parts[3] = G.p[1] * gp[2] - G.p[2] * gp[1];
    parts[4] = G.p[2] * gp[0] - G.p[0] * gp[2];
    parts[5] = G.p[0] * gp[1] - G.p[1] * gp[0];
    for (int e = 0; e < 9; e++) parts[6 + e] = GW[e];
    for (int e = 0; e < 3; e++) parts[15 + e] = -dw[e];
}

int gso_backward(const gso_gaussians *g, const gso_view *vw, const double pose[12],
                 const double *dl_dimage, gso_grads *out)
{
    raster_state st;
    if (!dl_dimage || !out) return -1;
    if (state_build(g, vw, pose, &st)) return -1;
    const int w = vw->roi_w, hgt = vw->roi_h;
    const int64_t P = (int64_t)w * hgt;
    const int64_t ntiles = (int64_t)st.gw * st.gh;
    const int64_t n = g->n;
    const int S = (g->sh_degree + 1) * (g->sh_degree + 1);

    /* per-instance slots keep the accumulation order independent of threads */
    double *slot = (double *)calloc((size_t)(st.M > 0 ? st.M : 1) * 9, sizeof(double));
    double *d2 = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    if (!slot || !d2) { free(slot); free(d2); state_free(&st); return -1; }

#pragma omp parallel
    {
        blend_rec *rec = (blend_rec *)malloc(sizeof(blend_rec) * (size_t)(st.maxlen + 1));
        double *suf = (double *)malloc(sizeof(double) * 3);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < ntiles; t++) {
            const int tx = (int)(t % st.gw), ty = (int)(t / st.gw);
            const uint32_t start = st.ranges[2 * t], end = st.ranges[2 * t + 1];
            const uint32_t *list = st.vals + start;
            for (int ly = 0; ly < GSO_TILE; ly++)
                for (int lx = 0; lx < GSO_TILE; lx++) {
                    const int rx = tx * GSO_TILE + lx, ry = ty * GSO_TILE + ly;
                    if (rx >= w || ry >= hgt) continue;
                    const int64_t pix = (int64_t)ry * w + rx;
                    double rgb[3], Tf;
                    int nb = 0;
                    composite(st.sp, list, (int)(end - start), (double)(vw->roi_x + rx),
                              (double)(vw->roi_y + ry), vw->bg, rgb, &Tf, NULL, NULL,
                              rec, &nb, NULL, NULL, 0);
                    const double G0 = dl_dimage[pix], G1 = dl_dimage[P + pix],
                                 G2 = dl_dimage[2 * P + pix];
                    const double Gc[3] = {G0, G1, G2};
                    /* suffix: colour blended behind entry k, plus background */
                    for (int ch = 0; ch < 3; ch++) suf[ch] = Tf * vw->bg[ch];
                    for (int e = nb - 1; e >= 0; e--) {
                        const blend_rec *r = rec + e;
                        const gso_splat *s = st.sp + r->gauss;
                        double *o = slot + 9 * (size_t)(start + (uint32_t)r->pos);
                        double dalpha = 0;
                        for (int ch = 0; ch < 3; ch++) {
                            o[6 + ch] += Gc[ch] * r->alpha * r->T;
                            dalpha += Gc[ch] * (s->color[ch] * r->T - suf[ch] / (1.0 - r->alpha));
                        }
                        for (int ch = 0; ch < 3; ch++) suf[ch] += s->color[ch] * r->alpha * r->T;
                        if (r->clamped) continue;
                        const double ep = exp(r->power);
                        o[5] += dalpha * ep;
                        const double dpow = dalpha * s->opacity * ep;
                        const double A = s->conic[0], B = s->conic[1], C = s->conic[2];
                        o[0] += dpow * (-(A * r->dx + B * r->dy));
                        o[1] += dpow * (-(C * r->dy + B * r->dx));
                        o[2] += dpow * (-0.5 * r->dx * r->dx);
                        o[3] += dpow * (-r->dx * r->dy);
                        o[4] += dpow * (-0.5 * r->dy * r->dy);
                    }
                }
        }
        free(rec);
        free(suf);
    }
    for (int64_t k = 0; k < st.M; k++) {
        double *dst = d2 + 9 * (size_t)st.vals[k];
        const double *src = slot + 9 * (size_t)k;
        for (int e = 0; e < 9; e++) dst[e] += src[e];
    }
    free(slot);

    double *parts_all = (double *)calloc((size_t)(n > 0 ? n : 1) * 18, sizeof(double));
    if (!parts_all) { free(d2); state_free(&st); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double dmu[3], dsc[3], dq[4], dop;
        double *dsh = out->sh ? out->sh + (int64_t)3 * S * i : NULL;
        backward_one(g, i, vw, pose, d2 + 9 * i, dmu, dsc, dq, &dop, dsh, parts_all + 18 * i);
        if (out->means) memcpy(out->means + 3 * i, dmu, sizeof dmu);
        if (out->scales) memcpy(out->scales + 3 * i, dsc, sizeof dsc);
        if (out->quats) memcpy(out->quats + 4 * i, dq, sizeof dq);
        if (out->opacities) out->opacities[i] = dop;
    }
    if (out->splat2d) memcpy(out->splat2d, d2, sizeof(double) * 9 * (size_t)n);

    double parts[18] = {0};
    for (int64_t i = 0; i < n; i++)
        for (int e = 0; e < 18; e++) parts[e] += parts_all[18 * i + e];
    if (out->pose_parts) memcpy(out->pose_parts, parts, sizeof parts);
    if (out->pose) {
        /* rho: sum g - R_c sum h ; phi: sum p x g + vee(sum dL/dW R_c^T) */
        double Rc[9], B[9];
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < 3; k++) Rc[3 * r + k] = pose[4 * r + k];
        for (int r = 0; r < 3; r++) {
            out->pose[r] = parts[r] - (Rc[3 * r] * parts[15] + Rc[3 * r + 1] * parts[16] +
                                       Rc[3 * r + 2] * parts[17]);
        }
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < 3; k++) {
                double acc = 0;
                for (int m = 0; m < 3; m++) acc += parts[6 + 3 * r + m] * Rc[3 * k + m];
                B[3 * r + k] = acc;
            }
        out->pose[3] = parts[3] + B[7] - B[5];
        out->pose[4] = parts[4] + B[2] - B[6];
        out->pose[5] = parts[5] + B[3] - B[1];
    }
    free(parts_all);
    free(d2);
    state_free(&st);
    (void)P;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Losses (Eq. (16) L1 part; Eq. (20)-(21)) and the pose Adam step.           */
/* ------------------------------------------------------------------------ */

double gso_l1(int64_t count, const double *a, const double *b, double *grad)
{
    double acc = 0;
    for (int64_t k = 0; k < count; k++) {
        const double r = a[k] - b[k];
        acc += fabs(r);
        if (grad) grad[k] = (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) / (double)count;
    }
    return count > 0 ? acc / (double)count : 0.0;
}

double gso_masked_l1(int64_t pixels, const double *a, const double *b,
                     const double *T_final, double *grad)
{
    double acc = 0;
    for (int64_t k = 0; k < pixels; k++) {
        const int m = (1.0 - T_final[k]) > 0.99;
        for (int c = 0; c < 3; c++) {
            const int64_t e = (int64_t)c * pixels + k;
            const double r = a[e] - b[e];
            if (m) acc += fabs(r);
            if (grad) grad[e] = m ? (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) : 0.0;
        }
    }
    return acc;
}

void gso_pose_adam(double T[12], double m[6], double v[6], const double g[6],
                   int32_t k, double lr, double beta1, double beta2, double eps,
                   double delta_out[6])
{
    double delta[6];
    const double c1 = 1.0 - pow(beta1, k), c2 = 1.0 - pow(beta2, k);
    for (int e = 0; e < 6; e++) {
        m[e] = beta1 * m[e] + (1 - beta1) * g[e];
        v[e] = beta2 * v[e] + (1 - beta2) * g[e] * g[e];
        const double mh = m[e] / c1, vh = v[e] / c2;
        delta[e] = -lr * mh / (sqrt(vh) + eps);
    }
    if (delta_out) memcpy(delta_out, delta, sizeof delta);
    gso_se3_retract(delta, T);
}
