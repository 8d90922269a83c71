/*
 * gsr_ref.c -- plain FP64 CPU oracle of the differentiable tile rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY (see gsr_ref.h).  Nothing here is shared with the
 * HIP path.  The code follows the method step by step, with no blocking,
 * fusion or reordering beyond what the definitions state:
 *
 *   1. activations and world covariance     (Sec. 3.3: P, r, s, sigma, SH)
 *   2. view transform, near cull            (Sec. 3.1: g_i in SE(3), pinhole Pi_c)
 *   3. EWA projection, conic, 3-sigma square (alpha_i = sigma_i * G(R,t,P,r,s))
 *   4. tile lists sorted by (depth, index)   (tile-based rasterizer, 3DGS lineage)
 *   5. SH colour                             (c "converted from SH")
 *   6. front-to-back compositing             (eqn:rendering, alpha >= 1/255,
 *                                             stop when T < 1e-4)
 *   7. reverse-order analytic backward       (gradients of every parameter)
 *   8. chain rule to parameters and pose twist (Sec. 3.3: poses optimised
 *                                             through the rendering objective)
 *
 * Pins: tests/test_oracle_*.py (brute force, closed forms, library routines,
 * invariants, central finite differences).
 */
#include "gsr_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Thresholds are the FP32-rounded values, widened (the GPU compares in FP32). */
#define A_MIN ((double)(1.0f / 255.0f))
#define A_MAX ((double)0.99f)
#define T_MIN ((double)1e-4f)
/* EWA low-pass variance (px^2), Jacobian guard factor, 3-sigma extent. */
#define LOWPASS 0.3
#define JGUARD 1.3
#define EXTENT 3.0
/* Relative half-width of the threshold-sensitivity bands (minimum), and the
 * FP32 unit roundoff used to widen them where FP32 evaluation is worse. */
#define BAND 1e-4
#define EPS32 5.9604644775390625e-08

typedef struct {
  int keep;
  int32_t x_lo, x_hi, y_lo, y_hi;
  int32_t bx_lo, bx_hi, by_lo, by_hi; /* square clipped to the alpha box */
  int32_t tx_lo, tx_hi, ty_lo, ty_hi, n_tiles;
  uint32_t depth_bits;
  double t[3];
  double u, v, z;
  double cov[3]; /* s_xx, s_xy, s_yy (with low-pass) */
  double det;
  double conic[3]; /* A, B, C */
  double lmax, radius;
  double opacity;
  double raw[3], color[3];
  double dir[3], dist;
  double J[6];  /* 2x3 row-major */
  double Sc[9]; /* R_f Sigma R_f^T */
  int clamp_x, clamp_y;
} rec_t;

struct ref_state {
  ref_settings set;
  int64_t n;
  int32_t F;
  int32_t K_sh; /* (d+1)^2 */
  ref_camera* cams;
  double* poses; /* F x 12 */
  double *means, *log_scales, *quats, *opac, *sh; /* private FP64 copies of the inputs */
  rec_t* rec;                                            /* F*n */
  int64_t* tile_off;  /* F+1 global tile offsets */
  int32_t* grid_x;    /* tiles per row per frame */
  int64_t* pix_off;   /* F+1 pixel offsets */
  int64_t T;          /* total tiles */
  int64_t K;
  int64_t* tile_start; /* T+1 */
  int32_t* tile_g;     /* K */
  uint8_t* flags;      /* P */
  int32_t* n_last;     /* P */
  double* t_final;     /* P */
  int64_t pairs;
  uint64_t hash;
  double* g2d; /* F*n x 10 screen-space gradients of the last backward, or NULL */
};

/* ------------------------------------------------------------------ */
/* small linear algebra                                                */
/* ------------------------------------------------------------------ */

static void mat3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}
static void mat3_mul_bt(const double* A, const double* B, double* C) { /* A B^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[j * 3 + k];
      C[i * 3 + j] = s;
    }
}
static void mat3_mul_at(const double* A, const double* B, double* C) { /* A^T B */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[k * 3 + i] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}

/* Unit-quaternion rotation matrix, q = (w, x, y, z), already normalised. */
void ref_quat_to_rotmat(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dL/dq (unit quaternion components) from dL/dR, differentiating the entries
 * of ref_quat_to_rotmat one by one. */
static void rotmat_grad_to_quat(const double* q, const double* dR, double* dq) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  /* d R_ij / d(w,x,y,z) */
  const double d[9][4] = {
      {0.0, 0.0, -4.0 * y, -4.0 * z},           /* R00 */
      {-2.0 * z, 2.0 * y, 2.0 * x, -2.0 * w},    /* R01 */
      {2.0 * y, 2.0 * z, 2.0 * w, 2.0 * x},      /* R02 */
      {2.0 * z, 2.0 * y, 2.0 * x, 2.0 * w},      /* R10 */
      {0.0, -4.0 * x, 0.0, -4.0 * z},           /* R11 */
      {-2.0 * x, -2.0 * w, 2.0 * z, 2.0 * y},    /* R12 */
      {-2.0 * y, 2.0 * z, -2.0 * w, 2.0 * x},    /* R20 */
      {2.0 * x, 2.0 * w, 2.0 * z, 2.0 * y},      /* R21 */
      {0.0, -4.0 * x, -4.0 * y, 0.0}};          /* R22 */
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int e = 0; e < 9; ++e) s += dR[e] * d[e][k];
    dq[k] = s;
  }
}

/* ------------------------------------------------------------------ */
/* real spherical harmonics, degree <= 3, order (l,m), m = -l..l,      */
/* with the (-1)^|m| phase                                             */
/* ------------------------------------------------------------------ */

void ref_sh_basis(int32_t degree, const double* dir, double* Y) {
  const double x = dir[0], y = dir[1], z = dir[2];
  const double pi = M_PI;
  Y[0] = 0.5 * sqrt(1.0 / pi);
  if (degree < 1) return;
  const double k1 = sqrt(3.0 / (4.0 * pi));
  Y[1] = -k1 * y;
  Y[2] = k1 * z;
  Y[3] = -k1 * x;
  if (degree < 2) return;
  const double k2a = 0.5 * sqrt(15.0 / pi);
  const double k2b = 0.25 * sqrt(5.0 / pi);
  const double k2c = 0.25 * sqrt(15.0 / pi);
  Y[4] = k2a * x * y;
  Y[5] = -k2a * y * z;
  Y[6] = k2b * (2.0 * z * z - x * x - y * y);
  Y[7] = -k2a * x * z;
  Y[8] = k2c * (x * x - y * y);
  if (degree < 3) return;
  const double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  const double k3b = 0.5 * sqrt(105.0 / pi);
  const double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  const double k3d = 0.25 * sqrt(7.0 / pi);
  const double k3e = 0.25 * sqrt(105.0 / pi);
  Y[9] = -k3a * y * (3.0 * x * x - y * y);
  Y[10] = k3b * x * y * z;
  Y[11] = -k3c * y * (4.0 * z * z - x * x - y * y);
  Y[12] = k3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  Y[13] = -k3c * x * (4.0 * z * z - x * x - y * y);
  Y[14] = k3e * z * (x * x - y * y);
  Y[15] = -k3a * x * (x * x - 3.0 * y * y);
}

/* Gradient of each basis polynomial with respect to (x, y, z), the direction
 * components taken as independent variables: out[k*3 + a]. */
void ref_sh_basis_grad(int32_t degree, const double* dir, double* g) {
  const double x = dir[0], y = dir[1], z = dir[2];
  const double pi = M_PI;
  const int nb = (degree + 1) * (degree + 1);
  for (int i = 0; i < nb * 3; ++i) g[i] = 0.0;
  if (degree < 1) return;
  const double k1 = sqrt(3.0 / (4.0 * pi));
  g[1 * 3 + 1] = -k1;
  g[2 * 3 + 2] = k1;
  g[3 * 3 + 0] = -k1;
  if (degree < 2) return;
  const double k2a = 0.5 * sqrt(15.0 / pi);
  const double k2b = 0.25 * sqrt(5.0 / pi);
  const double k2c = 0.25 * sqrt(15.0 / pi);
  g[4 * 3 + 0] = k2a * y;  g[4 * 3 + 1] = k2a * x;
  g[5 * 3 + 1] = -k2a * z; g[5 * 3 + 2] = -k2a * y;
  g[6 * 3 + 0] = -2.0 * k2b * x; g[6 * 3 + 1] = -2.0 * k2b * y; g[6 * 3 + 2] = 4.0 * k2b * z;
  g[7 * 3 + 0] = -k2a * z; g[7 * 3 + 2] = -k2a * x;
  g[8 * 3 + 0] = 2.0 * k2c * x; g[8 * 3 + 1] = -2.0 * k2c * y;
  if (degree < 3) return;
  const double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  const double k3b = 0.5 * sqrt(105.0 / pi);
  const double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  const double k3d = 0.25 * sqrt(7.0 / pi);
  const double k3e = 0.25 * sqrt(105.0 / pi);
  /* Y9 = -k3a (3x^2 y - y^3) */
  g[9 * 3 + 0] = -6.0 * k3a * x * y;
  g[9 * 3 + 1] = -k3a * (3.0 * x * x - 3.0 * y * y);
  /* Y10 = k3b x y z */
  g[10 * 3 + 0] = k3b * y * z; g[10 * 3 + 1] = k3b * x * z; g[10 * 3 + 2] = k3b * x * y;
  /* Y11 = -k3c (4 y z^2 - x^2 y - y^3) */
  g[11 * 3 + 0] = 2.0 * k3c * x * y;
  g[11 * 3 + 1] = -k3c * (4.0 * z * z - x * x - 3.0 * y * y);
  g[11 * 3 + 2] = -8.0 * k3c * y * z;
  /* Y12 = k3d (2 z^3 - 3 x^2 z - 3 y^2 z) */
  g[12 * 3 + 0] = -6.0 * k3d * x * z;
  g[12 * 3 + 1] = -6.0 * k3d * y * z;
  g[12 * 3 + 2] = k3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  /* Y13 = -k3c (4 x z^2 - x^3 - x y^2) */
  g[13 * 3 + 0] = -k3c * (4.0 * z * z - 3.0 * x * x - y * y);
  g[13 * 3 + 1] = 2.0 * k3c * x * y;
  g[13 * 3 + 2] = -8.0 * k3c * x * z;
  /* Y14 = k3e z (x^2 - y^2) */
  g[14 * 3 + 0] = 2.0 * k3e * x * z;
  g[14 * 3 + 1] = -2.0 * k3e * y * z;
  g[14 * 3 + 2] = k3e * (x * x - y * y);
  /* Y15 = -k3a (x^3 - 3 x y^2) */
  g[15 * 3 + 0] = -k3a * (3.0 * x * x - 3.0 * y * y);
  g[15 * 3 + 1] = 6.0 * k3a * x * y;
}

/* ------------------------------------------------------------------ */
/* step 1-5: per (Gaussian, frame) record                              */
/* ------------------------------------------------------------------ */

typedef struct {
  double s[3];   /* scales */
  double qn;     /* |q| */
  double qh[4];  /* unit quaternion */
  double R[9];
  double Sigma[9];
  double opacity;
} gauss_t;

static void gaussian_setup(const ref_state* st, int64_t g, gauss_t* G) {
  for (int a = 0; a < 3; ++a) G->s[a] = exp(st->log_scales[g * 3 + a]);
  double q[4];
  for (int a = 0; a < 4; ++a) q[a] = st->quats[g * 4 + a];
  G->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int a = 0; a < 4; ++a) G->qh[a] = q[a] / G->qn;
  ref_quat_to_rotmat(G->qh, G->R);
  /* Sigma = R diag(s^2) R^T */
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = G->R[i * 3 + j] * G->s[j];
  mat3_mul_bt(M, M, G->Sigma);
  G->opacity = 1.0 / (1.0 + exp(-st->opac[g]));
}

/* A Gaussian takes part only if every one of its parameters is a finite
 * number: means, log-scales, quaternion, opacity logit and the SH
 * coefficients of the rendered degree (the paper is silent; a non-finite
 * parameter would otherwise reach the images through the colour or through
 * an infinite depth). */
static int params_finite(const ref_state* st, int64_t g) {
  for (int a = 0; a < 3; ++a)
    if (!isfinite(st->means[g * 3 + a]) || !isfinite(st->log_scales[g * 3 + a])) return 0;
  for (int a = 0; a < 4; ++a)
    if (!isfinite(st->quats[g * 4 + a])) return 0;
  if (!isfinite(st->opac[g])) return 0;
  for (int i = 0; i < st->K_sh * 3; ++i)
    if (!isfinite(st->sh[g * st->K_sh * 3 + i])) return 0;
  return 1;
}

static void build_record(const ref_state* st, int f, int64_t g, rec_t* r) {
  memset(r, 0, sizeof(*r));
  if (!params_finite(st, g)) return;
  const ref_camera* cam = &st->cams[f];
  const double* P = &st->poses[f * 12];
  const double W[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]};
  const double tf[3] = {P[3], P[7], P[11]};
  const double mu[3] = {st->means[g * 3 + 0], st->means[g * 3 + 1],
                        st->means[g * 3 + 2]};
  /* step 2: t = W mu + t_f, near cull */
  for (int i = 0; i < 3; ++i)
    r->t[i] = W[i * 3 + 0] * mu[0] + W[i * 3 + 1] * mu[1] + W[i * 3 + 2] * mu[2] + tf[i];
  const double tx = r->t[0], ty = r->t[1], tz = r->t[2];
  if (!(tz > (double)cam->near_z)) return;
  const double fx = cam->fx, fy = cam->fy, cx = cam->cx, cy = cam->cy;
  /* step 3: projection of the mean and EWA covariance */
  r->u = fx * tx / tz + cx;
  r->v = fy * ty / tz + cy;
  r->z = tz;
  gauss_t G;
  gaussian_setup(st, g, &G);
  r->opacity = G.opacity;
  const double limx = JGUARD * (double)cam->width / (2.0 * fx);
  const double limy = JGUARD * (double)cam->height / (2.0 * fy);
  double rx = tx / tz, ry = ty / tz;
  r->clamp_x = 0;
  r->clamp_y = 0;
  if (rx < -limx) { rx = -limx; r->clamp_x = -1; }
  if (rx > limx) { rx = limx; r->clamp_x = 1; }
  if (ry < -limy) { ry = -limy; r->clamp_y = -1; }
  if (ry > limy) { ry = limy; r->clamp_y = 1; }
  const double txc = tz * rx, tyc = tz * ry;
  r->J[0] = fx / tz; r->J[1] = 0.0; r->J[2] = -fx * txc / (tz * tz);
  r->J[3] = 0.0; r->J[4] = fy / tz; r->J[5] = -fy * tyc / (tz * tz);
  double tmp[9];
  mat3_mul(W, G.Sigma, tmp);
  mat3_mul_bt(tmp, W, r->Sc);
  /* Sigma' = J Sc J^T + lowpass I */
  double JS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += r->J[i * 3 + k] * r->Sc[k * 3 + j];
      JS[i * 3 + j] = s;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += JS[i * 3 + k] * r->J[j * 3 + k];
      S2[i * 2 + j] = s;
    }
  r->cov[0] = S2[0] + LOWPASS;
  r->cov[1] = S2[1];
  r->cov[2] = S2[3] + LOWPASS;
  r->det = r->cov[0] * r->cov[2] - r->cov[1] * r->cov[1];
  if (!(r->det > 0.0)) return;
  r->conic[0] = r->cov[2] / r->det;
  r->conic[1] = -r->cov[1] / r->det;
  r->conic[2] = r->cov[0] / r->det;
  const double mid = 0.5 * (r->cov[0] + r->cov[2]);
  const double hd = 0.5 * (r->cov[0] - r->cov[2]);
  r->lmax = mid + sqrt(hd * hd + r->cov[1] * r->cov[1]);
  r->radius = EXTENT * sqrt(r->lmax);
  /* pixel square [ceil(u-r), floor(u+r)] clipped to the image */
  const double xa = ceil(r->u - r->radius), xb = floor(r->u + r->radius);
  const double ya = ceil(r->v - r->radius), yb = floor(r->v + r->radius);
  const double Wm1 = (double)(cam->width - 1), Hm1 = (double)(cam->height - 1);
  if (!(xa <= Wm1 && xb >= 0.0 && xa <= xb)) return;
  if (!(ya <= Hm1 && yb >= 0.0 && ya <= yb)) return;
  r->x_lo = (int32_t)(xa > 0.0 ? xa : 0.0);
  r->x_hi = (int32_t)(xb < Wm1 ? xb : Wm1);
  r->y_lo = (int32_t)(ya > 0.0 ? ya : 0.0);
  r->y_hi = (int32_t)(yb < Hm1 ? yb : Hm1);
  /* Tile rect: tiles of the square clipped to the bounding box of the region
   * where alpha can reach A_MIN, {q <= Qa}, Qa = 2 ln(opacity / A_MIN); its
   * half-widths are sqrt(Qa s_xx), sqrt(Qa s_yy).  Pixels outside it have
   * alpha < A_MIN and are skipped anyway, so the images are unchanged; a
   * Gaussian that can reach A_MIN at no pixel of its square is culled. */
  const double Qa = 2.0 * log(r->opacity / A_MIN) * (1.0 + 1e-9);
  if (!(Qa > 0.0)) return;
  const double hx = sqrt(Qa * r->cov[0]), hy = sqrt(Qa * r->cov[2]);
  const double ba = ceil(r->u - hx), bb = floor(r->u + hx);
  const double ca = ceil(r->v - hy), cb = floor(r->v + hy);
  r->bx_lo = ba > (double)r->x_lo ? (int32_t)ba : r->x_lo;
  r->bx_hi = bb < (double)r->x_hi ? (int32_t)bb : r->x_hi;
  r->by_lo = ca > (double)r->y_lo ? (int32_t)ca : r->y_lo;
  r->by_hi = cb < (double)r->y_hi ? (int32_t)cb : r->y_hi;
  if (!(r->bx_lo <= r->bx_hi && r->by_lo <= r->by_hi)) return;
  const int tw = st->set.tile_w, th = st->set.tile_h;
  r->tx_lo = r->bx_lo / tw; r->tx_hi = r->bx_hi / tw;
  r->ty_lo = r->by_lo / th; r->ty_hi = r->by_hi / th;
  r->n_tiles = (r->tx_hi - r->tx_lo + 1) * (r->ty_hi - r->ty_lo + 1);
  /* depth key: fp32(z), round to nearest even, compared as IEEE bits */
  float zf = (float)tz;
  memcpy(&r->depth_bits, &zf, 4);
  /* step 5: colour from SH at the unit direction from the camera centre */
  double C[3];
  for (int i = 0; i < 3; ++i)
    C[i] = -(W[0 * 3 + i] * tf[0] + W[1 * 3 + i] * tf[1] + W[2 * 3 + i] * tf[2]);
  double d[3] = {mu[0] - C[0], mu[1] - C[1], mu[2] - C[2]};
  r->dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) r->dir[i] = d[i] / r->dist;
  double Y[16];
  ref_sh_basis(st->set.sh_degree, r->dir, Y);
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int k = 0; k < st->K_sh; ++k)
      s += st->sh[(g * st->K_sh + k) * 3 + c] * Y[k];
    r->raw[c] = s + 0.5;
    r->color[c] = r->raw[c] > 0.0 ? r->raw[c] : 0.0;
  }
  r->keep = 1;
}

/* ------------------------------------------------------------------ */
/* step 4: per-tile lists sorted by (depth bits, g)                    */
/* ------------------------------------------------------------------ */

static const rec_t* g_sort_rec; /* frame base for the comparator */
static int cmp_entry(const void* a, const void* b) {
  const int32_t ga = *(const int32_t*)a, gb = *(const int32_t*)b;
  const uint32_t da = g_sort_rec[ga].depth_bits, db = g_sort_rec[gb].depth_bits;
  if (da != db) return da < db ? -1 : 1;
  return ga < gb ? -1 : (ga > gb ? 1 : 0);
}

/* ------------------------------------------------------------------ */
/* step 6: compositing of one pixel                                    */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t g;
  int32_t pos;    /* position in the tile list */
  double a, G, araw, Ti, dx, dy;
} blend_t;

/* Walks the tile list of pixel (px, py) of frame f.  Fills out[] with the
 * blended entries (if out != NULL), returns their number; writes T_final,
 * the stop position n_last, the accumulated colour/depth, the median entry
 * (*med: index among the blended entries of the first one after which T is
 * below 1/2, -1 if none; *zmed its depth), the flags and the count of
 * (pixel, entry) square hits. */
static int walk_pixel(const ref_state* st, int f, int px, int py, blend_t* out,
                      double* T_out, int32_t* nlast_out, double* S, double* Sz,
                      int* med, double* zmed, uint8_t* flags, int64_t* hits) {
  const int tw = st->set.tile_w, th = st->set.tile_h;
  const int64_t tile = st->tile_off[f] + (int64_t)(py / th) * st->grid_x[f] + px / tw;
  const int64_t s0 = st->tile_start[tile], s1 = st->tile_start[tile + 1];
  const rec_t* base = &st->rec[(int64_t)f * st->n];
  double T = 1.0;
  int nb = 0;
  int32_t nlast = 0;
  uint8_t fl = 0;
  S[0] = S[1] = S[2] = 0.0;
  *Sz = 0.0;
  *med = -1;
  *zmed = 0.0;
  const int median = st->set.depth_mode == REF_DEPTH_MEDIAN;
  for (int64_t k = s0; k < s1; ++k) {
    const int32_t g = st->tile_g[k];
    const rec_t* r = &base[g];
    if (px < r->x_lo || px > r->x_hi || py < r->y_lo || py > r->y_hi) continue;
    /* work statistic: pixels inside the alpha box (the only ones that can pass) */
    if (px >= r->bx_lo && px <= r->bx_hi && py >= r->by_lo && py <= r->by_hi) ++*hits;
    const double dx = r->u - (double)px, dy = r->v - (double)py;
    const double q = r->conic[0] * dx * dx + 2.0 * r->conic[1] * dx * dy +
                     r->conic[2] * dy * dy;
    const double G = exp(-0.5 * q);
    const double araw = r->opacity * G;
    const double a = araw < A_MAX ? araw : A_MAX;
    /* Sensitivity bands: the larger of BAND and the FP32 error bound of the
     * quantity, relative.  An FP32 evaluation of q errs by up to a few
     * eps32 * (A dx^2 + 2|B dx dy| + C dy^2), which exceeds q by the
     * anisotropy of elongated Gaussians; alpha inherits half of it.  T after
     * n blends carries up to ~n eps32. */
    const double qabs = r->conic[0] * dx * dx + 2.0 * fabs(r->conic[1] * dx * dy) +
                        r->conic[2] * dy * dy;
    const double band_a = fmax(BAND, 8.0 * EPS32 * qabs);
    if (fabs(a - A_MIN) < band_a * A_MIN) fl |= REF_FLAG_ALPHA_BAND;
    if (a < A_MIN) continue;
    const double Tn = T * (1.0 - a);
    const double band_t = fmax(BAND, 4.0 * EPS32 * (double)(nb + 1));
    if (fabs(Tn - T_MIN) < band_t * T_MIN) fl |= REF_FLAG_T_BAND;
    if (Tn < T_MIN) break;
    if (fabs(araw - A_MAX) < BAND * A_MAX) fl |= REF_FLAG_CLAMP_BAND;
    /* median depth: the first blended entry after which T is below 1/2 */
    if (median) {
      if (fabs(Tn - 0.5) < band_t * 0.5) fl |= REF_FLAG_MEDIAN_BAND;
      if (*med < 0 && Tn < 0.5) {
        *med = nb;
        *zmed = r->z;
      }
    }
    const double w = a * T;
    for (int c = 0; c < 3; ++c) S[c] += r->color[c] * w;
    *Sz += r->z * w;
    if (out) {
      blend_t* b = &out[nb];
      b->g = g; b->pos = (int32_t)(k - s0);
      b->a = a; b->G = G; b->araw = araw; b->Ti = T; b->dx = dx; b->dy = dy;
    }
    ++nb;
    T = Tn;
    nlast = (int32_t)(k - s0 + 1);
  }
  *T_out = T;
  *nlast_out = nlast;
  *flags = fl;
  return nb;
}

/* ------------------------------------------------------------------ */
/* forward                                                              */
/* ------------------------------------------------------------------ */

static uint64_t fnv(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xffu;
    h *= 1099511628211ull;
  }
  return h;
}

static int validate(const ref_settings* s, int64_t n, const float* means,
                    const float* log_scales, const float* quats, const float* opac,
                    const float* sh, int32_t F, const ref_camera* cams,
                    const float* poses) {
  if (!s || n < 0 || F < 1 || !cams || !poses) return REF_ERR_INVALID_ARGUMENT;
  if (s->sh_degree < 0 || s->sh_degree > 3) return REF_ERR_INVALID_ARGUMENT;
  if (s->tile_w < 1 || s->tile_h < 1) return REF_ERR_INVALID_ARGUMENT;
  if (n > 0 && (!means || !log_scales || !quats || !opac || !sh))
    return REF_ERR_INVALID_ARGUMENT;
  for (int f = 0; f < F; ++f)
    if (cams[f].width < 1 || cams[f].height < 1) return REF_ERR_INVALID_ARGUMENT;
  return REF_OK;
}

static int forward_impl(const ref_settings* s, int64_t n, double* means,
                        double* log_scales, double* quats, double* opac, double* sh,
                        int32_t F, const ref_camera* cams, double* poses, double* rgb,
                        double* depth, double* alpha, ref_state** out) {
  /* takes ownership of the six FP64 arrays */
  ref_state* st = (ref_state*)calloc(1, sizeof(ref_state));
  if (!st) return REF_ERR_OUT_OF_MEMORY;
  st->set = *s;
  st->n = n;
  st->F = F;
  st->K_sh = (s->sh_degree + 1) * (s->sh_degree + 1);
  st->cams = (ref_camera*)malloc(sizeof(ref_camera) * F);
  memcpy(st->cams, cams, sizeof(ref_camera) * F);
  st->poses = poses;
  st->means = means; st->log_scales = log_scales; st->quats = quats;
  st->opac = opac; st->sh = sh;
  const int nthr = s->n_threads > 0 ? s->n_threads : 1;
  /* frame layout */
  st->tile_off = (int64_t*)malloc(sizeof(int64_t) * (F + 1));
  st->pix_off = (int64_t*)malloc(sizeof(int64_t) * (F + 1));
  st->grid_x = (int32_t*)malloc(sizeof(int32_t) * F);
  st->tile_off[0] = 0;
  st->pix_off[0] = 0;
  for (int f = 0; f < F; ++f) {
    const int gx = (cams[f].width + s->tile_w - 1) / s->tile_w;
    const int gy = (cams[f].height + s->tile_h - 1) / s->tile_h;
    st->grid_x[f] = gx;
    st->tile_off[f + 1] = st->tile_off[f] + (int64_t)gx * gy;
    st->pix_off[f + 1] = st->pix_off[f] + (int64_t)cams[f].width * cams[f].height;
  }
  st->T = st->tile_off[F];
  const int64_t P = st->pix_off[F];

  /* steps 1-3, 5 */
  const int64_t M = (int64_t)F * n;
  st->rec = (rec_t*)malloc(sizeof(rec_t) * (M > 0 ? M : 1));
#pragma omp parallel for num_threads(nthr) schedule(static)
  for (int64_t r = 0; r < M; ++r) build_record(st, (int)(r / (n ? n : 1)), r % (n ? n : 1), &st->rec[r]);

  /* step 4: tile lists (CSR by global tile id), each sorted by (depth, g) */
  st->tile_start = (int64_t*)calloc((size_t)st->T + 1, sizeof(int64_t));
  for (int f = 0; f < F; ++f)
    for (int64_t g = 0; g < n; ++g) {
      const rec_t* r = &st->rec[(int64_t)f * n + g];
      if (!r->keep) continue;
      for (int ty = r->ty_lo; ty <= r->ty_hi; ++ty)
        for (int tx = r->tx_lo; tx <= r->tx_hi; ++tx)
          st->tile_start[st->tile_off[f] + (int64_t)ty * st->grid_x[f] + tx + 1]++;
    }
  for (int64_t t = 0; t < st->T; ++t) st->tile_start[t + 1] += st->tile_start[t];
  st->K = st->tile_start[st->T];
  st->tile_g = (int32_t*)malloc(sizeof(int32_t) * (st->K > 0 ? st->K : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (st->T > 0 ? st->T : 1));
  memcpy(fill, st->tile_start, sizeof(int64_t) * st->T);
  for (int f = 0; f < F; ++f)
    for (int64_t g = 0; g < n; ++g) {
      const rec_t* r = &st->rec[(int64_t)f * n + g];
      if (!r->keep) continue;
      for (int ty = r->ty_lo; ty <= r->ty_hi; ++ty)
        for (int tx = r->tx_lo; tx <= r->tx_hi; ++tx)
          st->tile_g[fill[st->tile_off[f] + (int64_t)ty * st->grid_x[f] + tx]++] = (int32_t)g;
    }
  free(fill);
  for (int f = 0; f < F; ++f) {
    g_sort_rec = &st->rec[(int64_t)f * n];
    for (int64_t t = st->tile_off[f]; t < st->tile_off[f + 1]; ++t)
      qsort(&st->tile_g[st->tile_start[t]], (size_t)(st->tile_start[t + 1] - st->tile_start[t]),
            sizeof(int32_t), cmp_entry);
  }

  /* step 6: per-pixel compositing */
  st->flags = (uint8_t*)calloc((size_t)(P > 0 ? P : 1), 1);
  st->n_last = (int32_t*)calloc((size_t)(P > 0 ? P : 1), sizeof(int32_t));
  st->t_final = (double*)calloc((size_t)(P > 0 ? P : 1), sizeof(double));
  uint64_t* phash = (uint64_t*)calloc((size_t)(P > 0 ? P : 1), sizeof(uint64_t));
  int64_t pairs = 0;
  for (int f = 0; f < F; ++f) {
    const int Wf = cams[f].width, Hf = cams[f].height;
    const int64_t p0 = st->pix_off[f];
    int64_t maxlen = 1;
    for (int64_t t = st->tile_off[f]; t < st->tile_off[f + 1]; ++t)
      if (st->tile_start[t + 1] - st->tile_start[t] > maxlen)
        maxlen = st->tile_start[t + 1] - st->tile_start[t];
#pragma omp parallel num_threads(nthr) reduction(+ : pairs)
    {
      blend_t* buf = (blend_t*)malloc(sizeof(blend_t) * maxlen);
#pragma omp for schedule(dynamic, 16)
      for (int py = 0; py < Hf; ++py)
        for (int px = 0; px < Wf; ++px) {
          double S[3], Sz, T;
          int32_t nl;
          uint8_t fl;
          int med;
          double zmed;
          const int nb =
              walk_pixel(st, f, px, py, buf, &T, &nl, S, &Sz, &med, &zmed, &fl, &pairs);
          const int64_t p = p0 + (int64_t)py * Wf + px;
          const int64_t plane = (int64_t)Wf * Hf;
          for (int c = 0; c < 3; ++c)
            rgb[3 * p0 + c * plane + (int64_t)py * Wf + px] = S[c] + T * (double)s->background[c];
          depth[p] = s->depth_mode == REF_DEPTH_MEDIAN ? zmed : Sz;
          alpha[p] = 1.0 - T;
          st->flags[p] = fl;
          st->n_last[p] = nl;
          st->t_final[p] = T;
          uint64_t h = 1469598103934665603ull;
          h = fnv(h, (uint64_t)nl);
          h = fnv(h, (uint64_t)(int64_t)med);
          for (int i = 0; i < nb; ++i) {
            h = fnv(h, (uint64_t)buf[i].pos);
            h = fnv(h, (uint64_t)(buf[i].araw > A_MAX));
          }
          phash[p] = h;
        }
      free(buf);
    }
  }
  st->pairs = pairs;
  /* decision hash */
  uint64_t h = 1469598103934665603ull;
  for (int64_t r = 0; r < M; ++r) {
    const rec_t* q = &st->rec[r];
    h = fnv(h, (uint64_t)q->keep);
    if (!q->keep) continue;
    h = fnv(h, ((uint64_t)(uint32_t)q->x_lo << 32) | (uint32_t)q->x_hi);
    h = fnv(h, ((uint64_t)(uint32_t)q->y_lo << 32) | (uint32_t)q->y_hi);
    h = fnv(h, (uint64_t)(q->clamp_x + 2) * 16 + (uint64_t)(q->clamp_y + 2));
    h = fnv(h, (uint64_t)((q->raw[0] > 0) | (q->raw[1] > 0) << 1 | (q->raw[2] > 0) << 2));
  }
  for (int64_t k = 0; k < st->K; ++k) h = fnv(h, (uint64_t)st->tile_g[k]);
  for (int64_t p = 0; p < P; ++p) h = fnv(h, phash[p]);
  st->hash = h;
  free(phash);
  *out = st;
  return REF_OK;
}

static double* widen(const float* a, int64_t m) {
  double* d = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
  for (int64_t i = 0; i < m; ++i) d[i] = (double)a[i];
  return d;
}
static double* copy64(const double* a, int64_t m) {
  double* d = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
  if (m > 0) memcpy(d, a, sizeof(double) * m);
  return d;
}

int ref_forward(const ref_settings* s, int64_t n, const float* means,
                const float* log_scales, const float* quats,
                const float* opacity_logits, const float* sh, int32_t F,
                const ref_camera* cams, const float* poses, double* rgb,
                double* depth, double* alpha, ref_state** out) {
  if (!out) return REF_ERR_INVALID_ARGUMENT;
  *out = NULL;
  int rc = validate(s, n, means, log_scales, quats, opacity_logits, sh, F, cams, poses);
  if (rc) return rc;
  const int64_t K = (s->sh_degree + 1) * (s->sh_degree + 1);
  return forward_impl(s, n, widen(means, 3 * n), widen(log_scales, 3 * n), widen(quats, 4 * n),
                      widen(opacity_logits, n), widen(sh, 3 * K * n), F, cams,
                      widen(poses, 12 * (int64_t)F), rgb, depth, alpha, out);
}

int ref_forward_f64(const ref_settings* s, int64_t n, const double* means,
                    const double* log_scales, const double* quats,
                    const double* opacity_logits, const double* sh, int32_t F,
                    const ref_camera* cams, const double* poses, double* rgb,
                    double* depth, double* alpha, ref_state** out) {
  if (!out) return REF_ERR_INVALID_ARGUMENT;
  *out = NULL;
  int rc = validate(s, n, (const float*)means, (const float*)log_scales, (const float*)quats,
                    (const float*)opacity_logits, (const float*)sh, F, cams, (const float*)poses);
  if (rc) return rc;
  const int64_t K = (s->sh_degree + 1) * (s->sh_degree + 1);
  return forward_impl(s, n, copy64(means, 3 * n), copy64(log_scales, 3 * n), copy64(quats, 4 * n),
                      copy64(opacity_logits, n), copy64(sh, 3 * K * n), F, cams,
                      copy64(poses, 12 * (int64_t)F), rgb, depth, alpha, out);
}

/* ------------------------------------------------------------------ */
/* backward                                                             */
/* ------------------------------------------------------------------ */

/* per-record screen-space gradient: du, dv, dA, dB, dC, dsigma, dc0..2, dz */
#define NG2 10

int ref_backward(ref_state* st, const double* g_rgb, const double* g_depth,
                 const double* g_alpha, double* g_means, double* g_log_scales,
                 double* g_quats, double* g_opac, double* g_sh, double* g_twist) {
  if (!st) return REF_ERR_STATE;
  const int64_t n = st->n;
  const int F = st->F;
  const int64_t M = (int64_t)F * n;
  const int Ksh = st->K_sh;
  if (n > 0 && (!g_means || !g_log_scales || !g_quats || !g_opac || !g_sh))
    return REF_ERR_INVALID_ARGUMENT;
  if (!g_twist || !g_rgb || !g_depth || !g_alpha) return REF_ERR_INVALID_ARGUMENT;
  int nthr = st->set.n_threads > 0 ? st->set.n_threads : 1;
  /* per-thread accumulators of the per-record screen-space gradients */
  double* acc = (double*)calloc((size_t)nthr * (M > 0 ? M : 1) * NG2, sizeof(double));
  if (!acc) return REF_ERR_OUT_OF_MEMORY;
  const double bg[3] = {st->set.background[0], st->set.background[1], st->set.background[2]};
  int64_t dummy_hits = 0;
  for (int f = 0; f < F; ++f) {
    const int Wf = st->cams[f].width, Hf = st->cams[f].height;
    const int64_t p0 = st->pix_off[f];
    const int64_t plane = (int64_t)Wf * Hf;
    int64_t maxlen = 1;
    for (int64_t t = st->tile_off[f]; t < st->tile_off[f + 1]; ++t)
      if (st->tile_start[t + 1] - st->tile_start[t] > maxlen)
        maxlen = st->tile_start[t + 1] - st->tile_start[t];
#pragma omp parallel num_threads(nthr) reduction(+ : dummy_hits)
    {
#ifdef _OPENMP
      const int tid = omp_get_thread_num();
#else
      const int tid = 0;
#endif
      double* my = acc + (size_t)tid * M * NG2;
      blend_t* buf = (blend_t*)malloc(sizeof(blend_t) * maxlen);
#pragma omp for schedule(dynamic, 16)
      for (int py = 0; py < Hf; ++py)
        for (int px = 0; px < Wf; ++px) {
          double S[3], Sz, Tf;
          int32_t nl;
          uint8_t fl;
          int med;
          double zmed;
          const int nb = walk_pixel(st, f, px, py, buf, &Tf, &nl, S, &Sz, &med, &zmed, &fl,
                                    &dummy_hits);
          const int median = st->set.depth_mode == REF_DEPTH_MEDIAN;
          const int64_t p = p0 + (int64_t)py * Wf + px;
          double GC[3];
          for (int c = 0; c < 3; ++c) GC[c] = g_rgb[3 * p0 + c * plane + (int64_t)py * Wf + px];
          const double GD = g_depth[p], GA = g_alpha[p];
          /* suffix sums: sum_{j>i} c_j w_j + T_final bg, sum_{j>i} z_j w_j */
          double accc[3] = {Tf * bg[0], Tf * bg[1], Tf * bg[2]};
          double accz = 0.0;
          for (int i = nb - 1; i >= 0; --i) {
            const blend_t* b = &buf[i];
            const rec_t* r = &st->rec[(int64_t)f * n + b->g];
            double* gr = &my[((int64_t)f * n + b->g) * NG2];
            const double w = b->a * b->Ti;
            const double om = 1.0 - b->a;
            double dLda = 0.0;
            for (int c = 0; c < 3; ++c) {
              dLda += GC[c] * (r->color[c] * b->Ti - accc[c] / om);
              gr[6 + c] += GC[c] * w;
            }
            if (median) {
              /* D = z of the median entry: no dependence on any alpha */
              if (i == med) gr[9] += GD;
            } else {
              dLda += GD * (r->z * b->Ti - accz / om);
              gr[9] += GD * w;
            }
            dLda += GA * (Tf / om);
            for (int c = 0; c < 3; ++c) accc[c] += r->color[c] * w;
            accz += r->z * w;
            if (b->araw > A_MAX) continue; /* clamped: alpha does not move */
            gr[5] += dLda * b->G;
            const double dLdq = -0.5 * b->a * dLda;
            const double A = r->conic[0], B = r->conic[1], C = r->conic[2];
            gr[0] += dLdq * 2.0 * (A * b->dx + B * b->dy);
            gr[1] += dLdq * 2.0 * (B * b->dx + C * b->dy);
            gr[2] += dLdq * b->dx * b->dx;
            gr[3] += dLdq * 2.0 * b->dx * b->dy;
            gr[4] += dLdq * b->dy * b->dy;
          }
        }
      free(buf);
    }
  }
  for (int t = 1; t < nthr; ++t)
    for (int64_t i = 0; i < M * NG2; ++i) acc[i] += acc[(size_t)t * M * NG2 + i];
  free(st->g2d);
  st->g2d = (double*)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1) * NG2);
  if (st->g2d && M > 0) memcpy(st->g2d, acc, sizeof(double) * (size_t)M * NG2);

  /* step 8: chain rule per record, summed over frames per Gaussian */
  double* twist_thr = (double*)calloc((size_t)nthr * F * 6, sizeof(double));
#pragma omp parallel num_threads(nthr)
  {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    double* tw = twist_thr + (size_t)tid * F * 6;
#pragma omp for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
      gauss_t G;
      gaussian_setup(st, g, &G);
      double dmu[3] = {0, 0, 0}, dSigma[9] = {0}, dsig = 0.0;
      double* dsh = &g_sh[g * Ksh * 3];
      for (int i = 0; i < Ksh * 3; ++i) dsh[i] = 0.0;
      const double mu[3] = {st->means[g * 3], st->means[g * 3 + 1], st->means[g * 3 + 2]};
      int kept = 0;
      for (int f = 0; f < F; ++f) {
        const rec_t* r = &st->rec[(int64_t)f * n + g];
        if (!r->keep) continue;
        kept = 1;
        const double* gr = &acc[((int64_t)f * n + g) * NG2];
        const ref_camera* cam = &st->cams[f];
        const double* P = &st->poses[f * 12];
        const double W[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]};
        const double fx = cam->fx, fy = cam->fy;
        const double tx = r->t[0], ty = r->t[1], tz = r->t[2];
        double dt[3] = {0, 0, 0};
        /* (u, v, z) -> t */
        dt[0] += gr[0] * fx / tz;
        dt[2] += -gr[0] * fx * tx / (tz * tz);
        dt[1] += gr[1] * fy / tz;
        dt[2] += -gr[1] * fy * ty / (tz * tz);
        dt[2] += gr[9];
        /* opacity */
        dsig += gr[5];
        /* conic -> Sigma' : dL/dSigma' = -Q G_Q Q with G_Q = [[dA, dB/2],[dB/2, dC]] */
        const double Q[4] = {r->conic[0], r->conic[1], r->conic[1], r->conic[2]};
        const double GQ[4] = {gr[2], 0.5 * gr[3], 0.5 * gr[3], gr[4]};
        double t1[4], GS[4];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            t1[i * 2 + j] = Q[i * 2 + 0] * GQ[0 * 2 + j] + Q[i * 2 + 1] * GQ[1 * 2 + j];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            GS[i * 2 + j] = -(t1[i * 2 + 0] * Q[0 * 2 + j] + t1[i * 2 + 1] * Q[1 * 2 + j]);
        /* Sigma' = J Sc J^T + lowpass: G_J = 2 GS J Sc, G_Sc = J^T GS J */
        double JSc[6];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += r->J[i * 3 + k] * r->Sc[k * 3 + j];
            JSc[i * 3 + j] = s;
          }
        double GJ[6];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 3; ++j)
            GJ[i * 3 + j] = 2.0 * (GS[i * 2 + 0] * JSc[0 * 3 + j] + GS[i * 2 + 1] * JSc[1 * 3 + j]);
        double GSc[9];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < 2; ++i)
              for (int j = 0; j < 2; ++j) s += r->J[i * 3 + a] * GS[i * 2 + j] * r->J[j * 3 + b];
            GSc[a * 3 + b] = s;
          }
        /* J -> t.  J00 = fx/tz, J11 = fy/tz, J02 = -fx txc/tz^2, J12 = -fy tyc/tz^2
         * with txc = tz * clamp(tx/tz); where the clamp is active txc = tz*lim. */
        dt[2] += GJ[0] * (-fx / (tz * tz));
        dt[2] += GJ[4] * (-fy / (tz * tz));
        if (r->clamp_x == 0) {
          dt[0] += GJ[2] * (-fx / (tz * tz));
          dt[2] += GJ[2] * (2.0 * fx * tx / (tz * tz * tz));
        } else {
          const double txc = tz * (r->clamp_x * JGUARD * (double)cam->width / (2.0 * fx));
          dt[2] += GJ[2] * (fx * txc / (tz * tz * tz));
        }
        if (r->clamp_y == 0) {
          dt[1] += GJ[5] * (-fy / (tz * tz));
          dt[2] += GJ[5] * (2.0 * fy * ty / (tz * tz * tz));
        } else {
          const double tyc = tz * (r->clamp_y * JGUARD * (double)cam->height / (2.0 * fy));
          dt[2] += GJ[5] * (fy * tyc / (tz * tz * tz));
        }
        /* Sc = W Sigma W^T  ->  G_Sigma += W^T G_Sc W */
        double tmp[9], GSig[9];
        mat3_mul_at(W, GSc, tmp);
        mat3_mul(tmp, W, GSig);
        for (int i = 0; i < 9; ++i) dSigma[i] += GSig[i];
        /* colour: c = max(raw, 0), raw = sum_k sh_k Y_k(dir) + 0.5 */
        double Y[16], dY[48];
        ref_sh_basis(st->set.sh_degree, r->dir, Y);
        ref_sh_basis_grad(st->set.sh_degree, r->dir, dY);
        double draw[3];
        for (int c = 0; c < 3; ++c) draw[c] = r->raw[c] > 0.0 ? gr[6 + c] : 0.0;
        double ddir[3] = {0, 0, 0};
        for (int k = 0; k < Ksh; ++k)
          for (int c = 0; c < 3; ++c) {
            dsh[k * 3 + c] += Y[k] * draw[c];
            const double s = st->sh[(g * Ksh + k) * 3 + c] * draw[c];
            for (int a = 0; a < 3; ++a) ddir[a] += s * dY[k * 3 + a];
          }
        /* dir = d/|d|, d = mu - C_f  ->  dd = (I - dir dir^T) ddir / |d| */
        const double dd0 = r->dir[0] * ddir[0] + r->dir[1] * ddir[1] + r->dir[2] * ddir[2];
        double dd[3];
        for (int a = 0; a < 3; ++a) dd[a] = (ddir[a] - r->dir[a] * dd0) / r->dist;
        /* t = W mu + t_f */
        for (int a = 0; a < 3; ++a) {
          dmu[a] += W[0 * 3 + a] * dt[0] + W[1 * 3 + a] * dt[1] + W[2 * 3 + a] * dt[2];
          dmu[a] += dd[a];
        }
        /* pose twist, left perturbation T <- Exp(xi) T at xi = 0, xi = (rho, phi):
         *   dt = rho + phi x t;  dSc = [phi]x Sc - Sc [phi]x;  dC = -W^T rho. */
        double* twf = &tw[f * 6];
        for (int a = 0; a < 3; ++a) twf[a] += dt[a];
        twf[3] += ty * dt[2] - tz * dt[1];
        twf[4] += tz * dt[0] - tx * dt[2];
        twf[5] += tx * dt[1] - ty * dt[0];
        /* dC/drho = -W^T, dd = -dC  =>  dL/drho += W (dL/dd) */
        for (int a = 0; a < 3; ++a)
          twf[a] += W[a * 3 + 0] * dd[0] + W[a * 3 + 1] * dd[1] + W[a * 3 + 2] * dd[2];
        for (int k = 0; k < 3; ++k) {
          double E[9] = {0};
          /* [e_k]x */
          if (k == 0) { E[5] = -1; E[7] = 1; }
          if (k == 1) { E[2] = 1; E[6] = -1; }
          if (k == 2) { E[1] = -1; E[3] = 1; }
          double ES[9], SE[9];
          mat3_mul(E, r->Sc, ES);
          mat3_mul(r->Sc, E, SE);
          double s = 0.0;
          for (int i = 0; i < 9; ++i) s += GSc[i] * (ES[i] - SE[i]);
          twf[3 + k] += s;
        }
        (void)mu;
      }
      if (!kept) { /* no frame sees it: every gradient is exactly 0 */
        for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = g_log_scales[g * 3 + a] = 0.0;
        for (int a = 0; a < 4; ++a) g_quats[g * 4 + a] = 0.0;
        g_opac[g] = 0.0;
        continue;
      }
      /* Sigma = M M^T with M = R diag(s):  G_M = 2 G_Sigma M (G_Sigma symmetric) */
      double Gs[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gs[i * 3 + j] = 0.5 * (dSigma[i * 3 + j] + dSigma[j * 3 + i]);
      double Mm[9], GM[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mm[i * 3 + j] = G.R[i * 3 + j] * G.s[j];
      mat3_mul(Gs, Mm, GM);
      for (int i = 0; i < 9; ++i) GM[i] *= 2.0;
      double dR[9], ds[3] = {0, 0, 0};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          dR[i * 3 + j] = GM[i * 3 + j] * G.s[j];
          ds[j] += GM[i * 3 + j] * G.R[i * 3 + j];
        }
      for (int a = 0; a < 3; ++a) g_log_scales[g * 3 + a] = ds[a] * G.s[a];
      double dqh[4];
      rotmat_grad_to_quat(G.qh, dR, dqh);
      const double proj = dqh[0] * G.qh[0] + dqh[1] * G.qh[1] + dqh[2] * G.qh[2] + dqh[3] * G.qh[3];
      for (int a = 0; a < 4; ++a) g_quats[g * 4 + a] = (dqh[a] - G.qh[a] * proj) / G.qn;
      for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = dmu[a];
      g_opac[g] = dsig * G.opacity * (1.0 - G.opacity);
    }
  }
  for (int i = 0; i < F * 6; ++i) {
    double s = 0.0;
    for (int t = 0; t < nthr; ++t) s += twist_thr[(size_t)t * F * 6 + i];
    g_twist[i] = s;
  }
  free(twist_thr);
  free(acc);
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* accessors                                                            */
/* ------------------------------------------------------------------ */

void ref_free(ref_state* st) {
  if (!st) return;
  free(st->cams); free(st->poses);
  free(st->means); free(st->log_scales); free(st->quats); free(st->opac); free(st->sh);
  free(st->rec); free(st->tile_off); free(st->grid_x); free(st->pix_off);
  free(st->tile_start); free(st->tile_g);
  free(st->flags); free(st->n_last); free(st->t_final); free(st->g2d);
  free(st);
}

int64_t ref_num_keys(const ref_state* st) { return st ? st->K : -1; }
int64_t ref_num_tiles(const ref_state* st) { return st ? st->T : -1; }
int64_t ref_num_pixels(const ref_state* st) { return st ? st->pix_off[st->F] : -1; }
int64_t ref_pairs_evaluated(const ref_state* st) { return st ? st->pairs : -1; }
uint64_t ref_decision_hash(const ref_state* st) { return st ? st->hash : 0; }

void ref_records(const ref_state* st, int32_t* ints, uint32_t* depth_bits, double* vals) {
  const int64_t M = (int64_t)st->F * st->n;
  for (int64_t r = 0; r < M; ++r) {
    const rec_t* q = &st->rec[r];
    if (ints) {
      int32_t* o = &ints[r * 14];
      o[0] = q->keep; o[1] = q->x_lo; o[2] = q->x_hi; o[3] = q->y_lo; o[4] = q->y_hi;
      o[5] = q->tx_lo; o[6] = q->tx_hi; o[7] = q->ty_lo; o[8] = q->ty_hi; o[9] = q->n_tiles;
      o[10] = q->bx_lo; o[11] = q->bx_hi; o[12] = q->by_lo; o[13] = q->by_hi;
    }
    if (depth_bits) depth_bits[r] = q->keep ? q->depth_bits : 0u;
    if (vals) {
      double* o = &vals[r * 20];
      o[0] = q->u; o[1] = q->v; o[2] = q->z;
      o[3] = q->conic[0]; o[4] = q->conic[1]; o[5] = q->conic[2];
      o[6] = q->cov[0]; o[7] = q->cov[1]; o[8] = q->cov[2];
      o[9] = q->lmax; o[10] = q->radius; o[11] = q->opacity;
      o[12] = q->color[0]; o[13] = q->color[1]; o[14] = q->color[2];
      o[15] = q->raw[0]; o[16] = q->raw[1]; o[17] = q->raw[2];
      o[18] = q->det; o[19] = q->t[2];
    }
  }
}

void ref_tile_lists(const ref_state* st, int64_t* tile_start, int32_t* entries) {
  if (tile_start) memcpy(tile_start, st->tile_start, sizeof(int64_t) * (st->T + 1));
  if (entries && st->K > 0) memcpy(entries, st->tile_g, sizeof(int32_t) * st->K);
}

int ref_screen_grads(const ref_state* st, double* out) {
  if (!st || !st->g2d) return REF_ERR_STATE;
  const int64_t M = (int64_t)st->F * st->n;
  if (M > 0) memcpy(out, st->g2d, sizeof(double) * (size_t)M * NG2);
  return REF_OK;
}

void ref_pixel_info(const ref_state* st, uint8_t* flags, int32_t* n_last, double* t_final) {
  const int64_t P = st->pix_off[st->F];
  if (flags) memcpy(flags, st->flags, P);
  if (n_last) memcpy(n_last, st->n_last, sizeof(int32_t) * P);
  if (t_final) memcpy(t_final, st->t_final, sizeof(double) * P);
}
