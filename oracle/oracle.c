/*
 * CPU FP64 reference ("oracle") for the differentiable Gaussian-splatting renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code with the GPU library.
 *
 * What it computes, and where that comes from
 * -------------------------------------------
 * The paper (CL-Splats) builds its local optimisation on the standard 3D Gaussian
 * Splatting renderer with default settings (Supp. Sec. "Implementation Details") and
 * modifies that renderer's kernels (Supp. "Local Optimization Kernel", Table
 * tab:timings).  It does not restate the renderer's equations, so this file writes
 * the forward model out from first principles:
 *   - EWA splatting of an anisotropic 3D Gaussian (covariance R diag(s^2) R^T from a
 *     log-scale and a quaternion) through a pinhole camera, with a 0.3 px^2 low-pass
 *     added to the 2D covariance;
 *   - view-dependent colour from real spherical harmonics of degree <= 3, plus 0.5,
 *     clamped at 0;
 *   - front-to-back alpha compositing per pixel in depth order, with alpha clamped at
 *     0.99, contributions below 1/255 skipped, and compositing stopped before the
 *     Gaussian that would take the transmittance below 1e-4.
 * The paper's local kernel (Sec. 3.3 "Local Optimization Kernel"; Supp. items 1-3:
 * a tile render mask from the changed Gaussians, rendering only masked tiles, and
 * preprocess-backward only for the changed Gaussians) claims the changed Gaussians
 * receive exactly the gradients of a full-scene step.  Tiles are pure culling, so the
 * oracle renders every requested pixel by brute force over ALL Gaussians in global
 * depth order, without tiles, and differentiates that definition exactly.
 *
 * Conventions fixed here (the paper leaves them open):
 *   - pixel (px, py) samples the point (px + 0.5, py + 0.5);
 *   - camera: p = R mu + t (OpenCV axes), u = fx X/Z + cx, v = fy Y/Z + cy;
 *   - depth order key: the float32 value z32 = fma(R20, x, fma(R21, y, fma(R22, z, t2)))
 *     evaluated on the float32 inputs, ties broken by Gaussian index; Gaussians with
 *     z32 <= 0.2f are culled (near plane);
 *   - the Jacobian uses X/Z and Y/Z clamped to 1.3 times the half-image tangent
 *     (W/2)/fx and (H/2)/fy;
 *   - quaternions are (w, x, y, z) and normalised; a zero quaternion is culled;
 *   - opacity below 1/255 is culled (no pixel can pass the alpha test);
 *   - real SH basis without the Condon-Shortley phase, index k = l^2 + l + m.
 *
 * Everything except the depth key and the near-plane test is evaluated in double.
 *
 * Near-threshold flags: a pixel is flagged when one of its discrete decisions sits
 * within 1e-5 (relative) of its threshold, so a float32 evaluation may legitimately
 * decide it the other way.  Gaussian-level decisions (SH clamp, Jacobian clamp,
 * opacity cut) are flagged the same way.  Comparisons excuse flagged items.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

#define NEAR_REL 1e-5

/* ------------------------------------------------------------------ SH basis */
/* Real spherical harmonics up to degree 3 evaluated on a unit direction d.
 * Y_{l,m} with k = l*l + l + m, no Condon-Shortley phase. */
static const double SH_C0 = 0.28209479177387814;  /* 1/(2 sqrt(pi)) */
static const double SH_C1 = 0.4886025119029199;   /* sqrt(3/(4 pi)) */
static const double SH_C2A = 1.0925484305920792;  /* sqrt(15/pi)/2 */
static const double SH_C2B = 0.31539156525252005; /* sqrt(5/pi)/4 */
static const double SH_C2C = 0.5462742152960396;  /* sqrt(15/pi)/4 */
static const double SH_C3A = 0.5900435899266435;  /* sqrt(35/(2 pi))/4 */
static const double SH_C3B = 2.890611442640554;   /* sqrt(105/pi)/2 */
static const double SH_C3C = 0.4570457994644658;  /* sqrt(21/(2 pi))/4 */
static const double SH_C3D = 0.3731763325901154;  /* sqrt(7/pi)/4 */
static const double SH_C3E = 1.445305721320277;   /* sqrt(105/pi)/4 */

void orc_sh_basis(const double d[3], double Y[16]) {
  const double x = d[0], y = d[1], z = d[2];
  Y[0] = SH_C0;
  Y[1] = SH_C1 * y;
  Y[2] = SH_C1 * z;
  Y[3] = SH_C1 * x;
  Y[4] = SH_C2A * x * y;
  Y[5] = SH_C2A * y * z;
  Y[6] = SH_C2B * (3.0 * z * z - 1.0);
  Y[7] = SH_C2A * x * z;
  Y[8] = SH_C2C * (x * x - y * y);
  Y[9] = SH_C3A * y * (3.0 * x * x - y * y);
  Y[10] = SH_C3B * x * y * z;
  Y[11] = SH_C3C * y * (5.0 * z * z - 1.0);
  Y[12] = SH_C3D * z * (5.0 * z * z - 3.0);
  Y[13] = SH_C3C * x * (5.0 * z * z - 1.0);
  Y[14] = SH_C3E * z * (x * x - y * y);
  Y[15] = SH_C3A * x * (x * x - 3.0 * y * y);
}

/* Magnitude of each basis polynomial above: its constant times the sum of the absolute
 * values of its monomials.  A float32 evaluation of Y_k can be wrong by a few ulp of
 * this magnitude (cancellation near the zeros of Y_k); it scales the error bounds. */
static void sh_basis_mag(const double d[3], double M[16]) {
  const double x = fabs(d[0]), y = fabs(d[1]), z = fabs(d[2]);
  M[0] = SH_C0;
  M[1] = SH_C1 * y;
  M[2] = SH_C1 * z;
  M[3] = SH_C1 * x;
  M[4] = SH_C2A * x * y;
  M[5] = SH_C2A * y * z;
  M[6] = SH_C2B * (3.0 * z * z + 1.0);
  M[7] = SH_C2A * x * z;
  M[8] = SH_C2C * (x * x + y * y);
  M[9] = SH_C3A * y * (3.0 * x * x + y * y);
  M[10] = SH_C3B * x * y * z;
  M[11] = SH_C3C * y * (5.0 * z * z + 1.0);
  M[12] = SH_C3D * z * (5.0 * z * z + 3.0);
  M[13] = SH_C3C * x * (5.0 * z * z + 1.0);
  M[14] = SH_C3E * z * (x * x + y * y);
  M[15] = SH_C3A * x * (x * x + 3.0 * y * y);
}

/* Gradient of each basis polynomial above with respect to (x, y, z), as written. */
static void sh_basis_grad(const double d[3], double G[16][3]) {
  const double x = d[0], y = d[1], z = d[2];
  memset(G, 0, sizeof(double) * 48);
  G[1][1] = SH_C1;
  G[2][2] = SH_C1;
  G[3][0] = SH_C1;
  G[4][0] = SH_C2A * y; G[4][1] = SH_C2A * x;
  G[5][1] = SH_C2A * z; G[5][2] = SH_C2A * y;
  G[6][2] = SH_C2B * 6.0 * z;
  G[7][0] = SH_C2A * z; G[7][2] = SH_C2A * x;
  G[8][0] = SH_C2C * 2.0 * x; G[8][1] = -SH_C2C * 2.0 * y;
  G[9][0] = SH_C3A * 6.0 * x * y; G[9][1] = SH_C3A * (3.0 * x * x - 3.0 * y * y);
  G[10][0] = SH_C3B * y * z; G[10][1] = SH_C3B * x * z; G[10][2] = SH_C3B * x * y;
  G[11][1] = SH_C3C * (5.0 * z * z - 1.0); G[11][2] = SH_C3C * 10.0 * y * z;
  G[12][2] = SH_C3D * (15.0 * z * z - 3.0);
  G[13][0] = SH_C3C * (5.0 * z * z - 1.0); G[13][2] = SH_C3C * 10.0 * x * z;
  G[14][0] = SH_C3E * 2.0 * x * z; G[14][1] = -SH_C3E * 2.0 * y * z; G[14][2] = SH_C3E * (x * x - y * y);
  G[15][0] = SH_C3A * (3.0 * x * x - 3.0 * y * y); G[15][1] = -SH_C3A * 6.0 * x * y;
}

/* ------------------------------------------------------------------ inputs */
typedef struct {
  int64_t n;
  int sh_degree;
  const double *means;     /* [3][n] */
  const double *log_scales;/* [3][n] */
  const double *quats;     /* [4][n] (w, x, y, z) */
  const double *opac;      /* [n] logits */
  const double *sh;        /* [K][3][n] */
} scene_t;

typedef struct {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H;
} cam_t;

static void load_cam(const double *c, cam_t *cam) {
  memcpy(cam->R, c, 9 * sizeof(double));
  memcpy(cam->t, c + 9, 3 * sizeof(double));
  cam->fx = c[12]; cam->fy = c[13]; cam->cx = c[14]; cam->cy = c[15];
  cam->W = (int)c[16]; cam->H = (int)c[17];
}

/* Per-Gaussian forward state for one camera. */
typedef struct {
  int visible;
  int flags;             /* ORC_F_* bits */
  float z32;
  double p[3];           /* camera-space centre */
  double u, v;
  double cov2[3];        /* a, b, c of the 2x2 screen covariance (with low-pass) */
  double conic[3];       /* A, B, C of its inverse */
  double o;              /* opacity */
  double pre[3];         /* colour before the clamp */
  double rgb[3];
  double rx, ry;         /* half extents of the alpha >= 1/255 ellipse box */
  /* saved for the backward */
  double s[3], qn[4], qnorm, Rq[9], Sigma[9], J[6], M[6], dir[3], dist, Xt, Yt;
  double limx, limy;
  /* first-order bounds on the error of a float32 evaluation of the quantities above
   * (not part of the method: they size the comparison bar, see err_bounds()) */
  double e_u, e_v;       /* absolute error of u, v (pixels) */
  double e_K;            /* absolute error of each conic entry */
  double e_cov;          /* absolute error of each screen-covariance entry */
  double e_det;          /* relative error of the conic from its inversion's rounding */
  double e_rgb[3];       /* absolute error of each colour channel */
} gstate_t;

#define ORC_F_VISIBLE 1
#define ORC_F_CLAMPX 2
#define ORC_F_CLAMPY 4
#define ORC_F_SHCLAMP_R 8
#define ORC_F_SHCLAMP_G 16
#define ORC_F_SHCLAMP_B 32
#define ORC_F_NEAR 64          /* some Gaussian-level decision is near its threshold */

static int near_rel(double x, double thr) { return fabs(x - thr) <= NEAR_REL * fabs(thr); }
/* x (> 0) within a factor exp(max(NEAR_REL, rel)) of thr (> 0): rel bounds the error of
 * ln x in a float32 evaluation of x, so the decision x vs thr may go either way there */
static int near_band(double x, double thr, double rel) {
  const double r = fmax(NEAR_REL, rel), q = x / thr;
  if (r < 0.5 && (q < 0.5 || q > 2.0)) return 0;   /* |ln q| > ln 2 > r: no logarithm needed */
  return fabs(log(q)) <= r;
}

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dR_ij / dq_m for the formula above; out[m][9]. */
static void quat_to_rot_grad(const double q[4], double dR[4][9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  /* d/dw */
  double Dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  /* d/dx */
  double Dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  /* d/dy */
  double Dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  /* d/dz */
  double Dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  memcpy(dR[0], Dw, sizeof Dw);
  memcpy(dR[1], Dx, sizeof Dx);
  memcpy(dR[2], Dy, sizeof Dy);
  memcpy(dR[3], Dz, sizeof Dz);
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

static void err_bounds(const scene_t *sc, int64_t i, const cam_t *cam, const double mu[3], gstate_t *g);

/* Forward geometry and colour of Gaussian i for one camera. */
static void project_one(const scene_t *sc, int64_t i, const cam_t *cam, gstate_t *g) {
  const int64_t n = sc->n;
  memset(g, 0, sizeof *g);
  const double mu[3] = {sc->means[i], sc->means[n + i], sc->means[2 * n + i]};

  /* depth key on float32 inputs with a fixed fused chain */
  {
    const float mx = (float)mu[0], my = (float)mu[1], mz = (float)mu[2];
    g->z32 = fmaf((float)cam->R[6], mx, fmaf((float)cam->R[7], my, fmaf((float)cam->R[8], mz, (float)cam->t[2])));
  }

  double q[4];
  for (int k = 0; k < 4; ++k) q[k] = sc->quats[k * n + i];
  g->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(g->qnorm > 0.0)) return;
  if (!((double)g->z32 > (double)0.2f)) return;

  g->o = sigmoid(sc->opac[i]);
  if (near_rel(g->o, 1.0 / 255.0)) g->flags |= ORC_F_NEAR;
  if (g->o < 1.0 / 255.0) return;

  for (int k = 0; k < 4; ++k) g->qn[k] = q[k] / g->qnorm;
  for (int k = 0; k < 3; ++k) g->s[k] = exp(sc->log_scales[k * n + i]);
  quat_to_rot(g->qn, g->Rq);
  /* Sigma = Rq diag(s^2) Rq^T */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += g->Rq[3 * a + k] * g->s[k] * g->s[k] * g->Rq[3 * b + k];
      g->Sigma[3 * a + b] = acc;
    }

  /* camera transform */
  for (int a = 0; a < 3; ++a)
    g->p[a] = cam->R[3 * a] * mu[0] + cam->R[3 * a + 1] * mu[1] + cam->R[3 * a + 2] * mu[2] + cam->t[a];
  const double X = g->p[0], Y = g->p[1], Z = g->p[2];
  g->u = cam->fx * X / Z + cam->cx;
  g->v = cam->fy * Y / Z + cam->cy;

  /* Jacobian of the perspective map with clamped lateral ratios */
  g->limx = 1.3 * (0.5 * cam->W) / cam->fx;
  g->limy = 1.3 * (0.5 * cam->H) / cam->fy;
  double rxz = X / Z, ryz = Y / Z;
  if (near_rel(fabs(rxz), g->limx) || near_rel(fabs(ryz), g->limy)) g->flags |= ORC_F_NEAR;
  if (rxz > g->limx) { rxz = g->limx; g->flags |= ORC_F_CLAMPX; }
  if (rxz < -g->limx) { rxz = -g->limx; g->flags |= ORC_F_CLAMPX; }
  if (ryz > g->limy) { ryz = g->limy; g->flags |= ORC_F_CLAMPY; }
  if (ryz < -g->limy) { ryz = -g->limy; g->flags |= ORC_F_CLAMPY; }
  g->Xt = Z * rxz;
  g->Yt = Z * ryz;
  g->J[0] = cam->fx / Z; g->J[1] = 0.0;         g->J[2] = -cam->fx * g->Xt / (Z * Z);
  g->J[3] = 0.0;         g->J[4] = cam->fy / Z; g->J[5] = -cam->fy * g->Yt / (Z * Z);
  /* M = J Rcam (2x3) */
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += g->J[3 * a + k] * cam->R[3 * k + b];
      g->M[3 * a + b] = acc;
    }
  /* cov2 = M Sigma M^T + 0.3 I */
  double MS[6];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += g->M[3 * a + k] * g->Sigma[3 * k + b];
      MS[3 * a + b] = acc;
    }
  double C2[4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += MS[3 * a + k] * g->M[3 * b + k];
      C2[2 * a + b] = acc;
    }
  g->cov2[0] = C2[0] + 0.3;
  g->cov2[1] = 0.5 * (C2[1] + C2[2]);
  g->cov2[2] = C2[3] + 0.3;
  const double det = g->cov2[0] * g->cov2[2] - g->cov2[1] * g->cov2[1];
  if (!(det > 0.0)) return;
  g->conic[0] = g->cov2[2] / det;
  g->conic[1] = -g->cov2[1] / det;
  g->conic[2] = g->cov2[0] / det;

  /* colour */
  const double campos[3] = {
      -(cam->R[0] * cam->t[0] + cam->R[3] * cam->t[1] + cam->R[6] * cam->t[2]),
      -(cam->R[1] * cam->t[0] + cam->R[4] * cam->t[1] + cam->R[7] * cam->t[2]),
      -(cam->R[2] * cam->t[0] + cam->R[5] * cam->t[1] + cam->R[8] * cam->t[2])};
  double dv[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
  g->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int a = 0; a < 3; ++a) g->dir[a] = dv[a] / g->dist;
  double Yb[16];
  orc_sh_basis(g->dir, Yb);
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5, mag = 0.5;
    for (int k = 0; k < K; ++k) {
      const double term = sc->sh[((int64_t)k * 3 + ch) * n + i] * Yb[k];
      acc += term;
      mag += fabs(term);
    }
    g->pre[ch] = acc;
    if (fabs(acc) <= NEAR_REL * mag) g->flags |= ORC_F_NEAR;
    if (acc < 0.0) {
      g->rgb[ch] = 0.0;
      g->flags |= (ORC_F_SHCLAMP_R << ch);
    } else {
      g->rgb[ch] = acc;
    }
  }

  /* extent: alpha >= 1/255 needs d^T conic d <= 2 ln(255 o); the box of that ellipse
   * has half widths sqrt(2 ln(255 o) a) and sqrt(2 ln(255 o) c).  A relative margin of
   * 2^-12 keeps a float32 evaluation of the same box conservative. */
  const double kappa = 2.0 * log(255.0 * g->o);
  g->rx = sqrt(kappa * g->cov2[0]) * (1.0 + 1.0 / 4096.0);
  g->ry = sqrt(kappa * g->cov2[2]) * (1.0 + 1.0 / 4096.0);
  err_bounds(sc, i, cam, mu, g);
  g->visible = 1;
  g->flags |= ORC_F_VISIBLE;
}

/* ------------------------------------------------------------------ float32 error model
 * Not part of the method: it sizes the comparison bar for a float32 evaluation of the
 * same definition.  Per Gaussian and view, first-order bounds on the error of each
 * projected quantity when evaluated in float32 (unit roundoff U32 = 2^-24), each
 * operation of a chain counted once with its operands' magnitudes:
 *   - camera-space centre: a coordinate is a 3-term fused dot product plus a
 *     translation, error <= 3 U32 times the sum of the absolute values of its terms
 *     (mX, mY, mZ);
 *   - u = fx X/Z + cx: the errors of X and Z carried through the quotient (3 U32 each),
 *     the rounding of the reciprocal and product (3 U32 |u - cx|), the final sum
 *     (2 U32 |u|);
 *   - screen covariance M Sigma M^T + 0.3 I with Sigma = Rq diag(s^2) Rq^T, M = J Rcam:
 *     the roundings of the normalised quaternion, the rotation entries, the scales'
 *     exponentials and the Jacobian's reciprocal depth move Sigma by ~8 U32 s_max^2 and
 *     M by a few U32 of its rows, so every entry is wrong by at most
 *     E_cov = 8 U32 s_max^2 (|M_0| + |M_1|)^2 plus 2 U32 (a + c) for its own sums; the
 *     conic K = cov^-1 then by 2 E_cov / lambda_min^2 (the derivative of an inverse is
 *     -K dS K, of norm ||K||^2 ||dS||) plus 4 U32 of its largest entry;
 *   - opacity: the logistic function in float32, 4 U32 relative;
 *   - colour: the spherical-harmonic sum is rounded relative to the sum of the
 *     magnitudes of its terms (each basis polynomial by the magnitude of its monomials,
 *     8 U32), and the unit view direction carries an error of ~8 U32 (|c| + |mu|)/dist,
 *     which moves each basis value by at most its gradient's size times that. */
#define U32 (1.0 / 16777216.0)
static void err_bounds(const scene_t *sc, int64_t i, const cam_t *cam, const double mu[3], gstate_t *g) {
  const int64_t n = sc->n;
  double m[3];
  for (int a = 0; a < 3; ++a)
    m[a] = fabs(cam->R[3 * a] * mu[0]) + fabs(cam->R[3 * a + 1] * mu[1]) + fabs(cam->R[3 * a + 2] * mu[2]) +
           fabs(cam->t[a]);
  const double X = g->p[0], Y = g->p[1], Z = g->p[2];
  g->e_u = U32 * (3.0 * cam->fx / Z * (m[0] + fabs(X) * m[2] / Z) + 3.0 * fabs(g->u - cam->cx) + 2.0 * fabs(g->u));
  g->e_v = U32 * (3.0 * cam->fy / Z * (m[1] + fabs(Y) * m[2] / Z) + 3.0 * fabs(g->v - cam->cy) + 2.0 * fabs(g->v));
  /* rows of M = J Rcam and the largest scale */
  double nM[2];
  for (int r = 0; r < 2; ++r)
    nM[r] = sqrt(g->M[3 * r] * g->M[3 * r] + g->M[3 * r + 1] * g->M[3 * r + 1] + g->M[3 * r + 2] * g->M[3 * r + 2]);
  double smax = g->s[0];
  if (g->s[1] > smax) smax = g->s[1];
  if (g->s[2] > smax) smax = g->s[2];
  const double a = g->cov2[0], b = g->cov2[1], c = g->cov2[2];
  const double Ecov = 8.0 * U32 * smax * smax * (nM[0] + nM[1]) * (nM[0] + nM[1]) + 2.0 * U32 * (a + c);
  const double lmin = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
  double Kmax = fabs(g->conic[0]);
  if (fabs(g->conic[1]) > Kmax) Kmax = fabs(g->conic[1]);
  if (fabs(g->conic[2]) > Kmax) Kmax = fabs(g->conic[2]);
  g->e_K = 4.0 * U32 * Kmax + 2.0 * Ecov / (lmin * lmin);
  /* the inversion K = (c, -b, a) / (ac - b^2) rounds the determinant relative to
   * (|ac| + b^2) / |ac - b^2| (cancellation for elongated footprints), then the
   * reciprocal and the products */
  g->e_cov = Ecov;
  g->e_det = 2.0 * U32 * (fabs(a * c) + b * b) / fabs(a * c - b * b) + 3.0 * U32;
  /* colour */
  double cp[3];
  for (int a2 = 0; a2 < 3; ++a2)
    cp[a2] = -(cam->R[a2] * cam->t[0] + cam->R[3 + a2] * cam->t[1] + cam->R[6 + a2] * cam->t[2]);
  const double rdir = 8.0 * U32 * (sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]) +
                                   sqrt(mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2])) / g->dist;
  double Mb[16], dY[16][3];
  sh_basis_mag(g->dir, Mb);
  sh_basis_grad(g->dir, dY);
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double mag = 0.5, dmag = 0.0;
    for (int k = 0; k < K; ++k) {
      const double f = fabs(sc->sh[((int64_t)k * 3 + ch) * n + i]);
      mag += f * Mb[k];
      dmag += f * (fabs(dY[k][0]) + fabs(dY[k][1]) + fabs(dY[k][2]));
    }
    g->e_rgb[ch] = 8.0 * U32 * mag + rdir * dmag;
  }
}

static void make_scene(scene_t *sc, int64_t n, int sh_degree, const double *means, const double *log_scales,
                       const double *quats, const double *opac, const double *sh) {
  sc->n = n; sc->sh_degree = sh_degree;
  sc->means = means; sc->log_scales = log_scales; sc->quats = quats; sc->opac = opac; sc->sh = sh;
}

/* out per Gaussian (stride 16): u, v, A, B, C, o, r, g, b, rx, ry, a, b, c, z32, 0 */
int orc_preprocess(int64_t n, int sh_degree, const double *means, const double *log_scales, const double *quats,
                   const double *opac, const double *sh, const double *camv, double *out, float *z32,
                   int32_t *flags) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3) return ORC_EINVAL;
  scene_t sc; make_scene(&sc, n, sh_degree, means, log_scales, quats, opac, sh);
  cam_t cam; load_cam(camv, &cam);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    gstate_t g;
    project_one(&sc, i, &cam, &g);
    double *o = out + 16 * i;
    o[0] = g.u; o[1] = g.v; o[2] = g.conic[0]; o[3] = g.conic[1]; o[4] = g.conic[2]; o[5] = g.o;
    o[6] = g.rgb[0]; o[7] = g.rgb[1]; o[8] = g.rgb[2]; o[9] = g.rx; o[10] = g.ry;
    o[11] = g.cov2[0]; o[12] = g.cov2[1]; o[13] = g.cov2[2]; o[14] = (double)g.z32; o[15] = 0.0;
    z32[i] = g.z32;
    flags[i] = g.flags;
  }
  return ORC_OK;
}

/* The float32 error bounds of err_bounds() per Gaussian (stride 8): e_u, e_v, e_K,
 * e_rgb[3], e_cov, e_det; zero for culled Gaussians. */
int orc_error_bounds(int64_t n, int sh_degree, const double *means, const double *log_scales, const double *quats,
                     const double *opac, const double *sh, const double *camv, double *out) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3) return ORC_EINVAL;
  scene_t sc; make_scene(&sc, n, sh_degree, means, log_scales, quats, opac, sh);
  cam_t cam; load_cam(camv, &cam);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    gstate_t g;
    project_one(&sc, i, &cam, &g);
    double *o = out + 8 * i;
    if (!g.visible) { for (int k = 0; k < 8; ++k) o[k] = 0.0; continue; }
    o[0] = g.e_u; o[1] = g.e_v; o[2] = g.e_K; o[3] = g.e_rgb[0]; o[4] = g.e_rgb[1]; o[5] = g.e_rgb[2];
    o[6] = g.e_cov; o[7] = g.e_det;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ depth order */
typedef struct { float z; int64_t id; } zkey_t;
static int cmp_zkey(const void *a, const void *b) {
  const zkey_t *x = (const zkey_t *)a, *y = (const zkey_t *)b;
  if (x->z < y->z) return -1;
  if (x->z > y->z) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* ------------------------------------------------------------------ render + backward */
/* What the per-pixel walk needs of each Gaussian. */
typedef struct {
  double u, v, conic[3], o, rgb[3];
  int flags;
  int visible;
  float z32;
  double e_u, e_v, e_K, e_rgb[3];   /* float32 error bounds (err_bounds) */
  double e_cov, e_det;
} rstate_t;

typedef struct {
  int64_t id;
  double alpha, T, G, dx, dy;
  int clamped;
} contrib_t;

/*
 * Render the pixels pix[0..npix) (pairs px, py) of one camera by brute force over all
 * Gaussians in depth order.  Outputs colour (rgb + T*bg), final transmittance, the
 * number of blended Gaussians and a near-threshold flag per pixel.
 *
 * If dL_dC is given ([npix][3], the upstream gradient of the loss with respect to the
 * pixel colours), also accumulates the exact derivative of the loss with respect to
 * each Gaussian's screen-space quantities into grad2d ([n][9]: u, v, A, B, C, opacity,
 * r, g, b) and the sum of absolute per-pixel terms into s2d ([n][9]).  gflag[n] is set
 * for Gaussians blended at (or decided near a threshold at) a flagged pixel.
 *
 * pert ([n][9], optional, entries in [-1, 1]) perturbs each Gaussian's projected
 * quantities u, v, A, B, C, opacity, r, g, b by that fraction of their float32 error
 * bounds (err_bounds; the opacity by 4 U32 relative) before rendering: rendering with a
 * few random sign patterns shows how far a float32 evaluation's gradient can move,
 * with the pixels' contributions combined with their signs, as they are in the sum.
 *
 * e2d ([n][9], optional) receives the part of the float32 error that such
 * perturbations do not model: the rounding of the compositing chains themselves (the
 * transmittance as a running product, or rebuilt backwards by division, and the colour
 * sums), 4 U32 per blended Gaussian of the pixel plus 16 U32, relative to each
 * partial's magnitude with dL/dalpha taken as sum |g| (T c + S/(1 - alpha)), before its
 * two parts cancel.
 */
int orc_render(int64_t n, int sh_degree, const double *means, const double *log_scales, const double *quats,
               const double *opac, const double *sh, const double *camv, const double *bg, int64_t npix,
               const int32_t *pix, double *out_rgb, double *out_T, int32_t *out_ncontrib, int32_t *out_flag,
               const double *dL_dC, double *grad2d, double *s2d, int32_t *gflag, double *e2d,
               const double *pert) {
  if (n < 0 || npix < 0 || sh_degree < 0 || sh_degree > 3) return ORC_EINVAL;
  scene_t sc; make_scene(&sc, n, sh_degree, means, log_scales, quats, opac, sh);
  cam_t cam; load_cam(camv, &cam);

  rstate_t *gs = (rstate_t *)malloc(sizeof(rstate_t) * (size_t)(n > 0 ? n : 1));
  zkey_t *order = (zkey_t *)malloc(sizeof(zkey_t) * (size_t)(n > 0 ? n : 1));
  if (!gs || !order) { free(gs); free(order); return ORC_ENOMEM; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    gstate_t g;
    project_one(&sc, i, &cam, &g);
    rstate_t *r = &gs[i];
    r->u = g.u; r->v = g.v;
    for (int k = 0; k < 3; ++k) { r->conic[k] = g.conic[k]; r->rgb[k] = g.rgb[k]; }
    r->o = g.o; r->flags = g.flags; r->visible = g.visible; r->z32 = g.z32;
    r->e_u = g.e_u; r->e_v = g.e_v; r->e_K = g.e_K; r->e_cov = g.e_cov; r->e_det = g.e_det;
    for (int k = 0; k < 3; ++k) r->e_rgb[k] = g.e_rgb[k];
    if (pert && r->visible) {
      const double *x = pert + 9 * i;
      r->u += x[0] * g.e_u;
      r->v += x[1] * g.e_v;
      for (int k = 0; k < 3; ++k) r->conic[k] += x[2 + k] * g.e_K;
      r->o *= 1.0 + x[5] * 4.0 * U32;
      for (int k = 0; k < 3; ++k)
        if (r->rgb[k] > 0.0) r->rgb[k] = fmax(0.0, r->rgb[k] + x[6 + k] * g.e_rgb[k]);
    }
  }
  int64_t nv = 0;
  for (int64_t i = 0; i < n; ++i)
    if (gs[i].visible) { order[nv].z = gs[i].z32; order[nv].id = i; ++nv; }
  qsort(order, (size_t)nv, sizeof(zkey_t), cmp_zkey);

  const double a_min = 1.0 / 255.0, a_max = 0.99, t_stop = 1e-4;
  int err = 0;

#pragma omp parallel
  {
    size_t cap = 256;
    contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * cap);
    int64_t *near_ids = (int64_t *)malloc(sizeof(int64_t) * 64);
    size_t near_cap = 64;
    if (!list || !near_ids) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
      if (err) continue;
      const double px = pix[2 * p] + 0.5, py = pix[2 * p + 1] + 0.5;
      double T = 1.0, C[3] = {0.0, 0.0, 0.0};
      double relT = 0.0;   /* bound on the relative float32 error of T */
      size_t nc = 0, nn = 0;
      int flag = 0;
      for (int64_t r = 0; r < nv && !err; ++r) {
        const rstate_t *g = &gs[order[r].id];
        const double dx = px - g->u, dy = py - g->v;
        const double A = g->conic[0], B = g->conic[1], Cc = g->conic[2];
        const double qf = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
        const double qabs = fabs(A * dx * dx) + 2.0 * fabs(B * dx * dy) + fabs(Cc * dy * dy);
        /* decision 1: a positive exponent (possible only through cancellation) is skipped */
        int near = (qf < NEAR_REL * qabs);
        const double power = -0.5 * qf;
        int action; /* 0 skip, 1 blend, 2 stop */
        double G = 0.0, alpha = 0.0, Tn = T, relTn = relT;
        int clamped = 0;
        if (power > 0.0) {
          action = 0;
        } else {
          G = exp(power);
          const double oG = g->o * G;
          /* float32 error of ln(o G) = ln o + power: the centre's error bounds times
           * |d power/d (u, v)| = |K d|; the covariance's, through the inverse (d power =
           * (K d)^T dS (K d) / 2, |dS| <= 2 e_cov), |K d|^2 e_cov; the inversion's
           * rounding, |power| e_det; the evaluation of the quadratic form (4 U32 of the
           * sum of its absolute terms); the opacity and the exponential (4 U32 each) */
          const double Ku = A * dx + B * dy, Kv = B * dx + Cc * dy;
          const double rel_a = fabs(Ku) * g->e_u + fabs(Kv) * g->e_v + (Ku * Ku + Kv * Kv) * g->e_cov +
                               0.5 * qf * g->e_det + 4.0 * U32 * qabs + 8.0 * U32;
          /* decision 2: alpha clamp; decision 3: alpha skip; decision 4: stop; each
           * flagged when its value lies within its float32 error of the threshold */
          if (near_band(oG, a_max, rel_a)) near = 1;
          clamped = !(oG < a_max);
          alpha = clamped ? a_max : oG;
          if (near_band(alpha, a_min, rel_a)) near = 1;
          if (alpha < a_min) {
            action = 0;
          } else {
            Tn = T * (1.0 - alpha);
            /* T' = T (1 - alpha): the relative error of 1 - alpha is alpha/(1 - alpha)
             * times alpha's (to first order), plus the product's rounding */
            relTn = relT + (clamped ? 0.0 : alpha / (1.0 - alpha) * rel_a) + 2.0 * U32;
            if (near_band(Tn, t_stop, relTn)) near = 1;
            action = (Tn < t_stop) ? 2 : 1;
          }
        }
        if (near) {
          flag = 1;
          if (nn == near_cap) {
            near_cap *= 2;
            int64_t *nw = (int64_t *)realloc(near_ids, sizeof(int64_t) * near_cap);
            if (!nw) { err = 1; break; }
            near_ids = nw;
          }
          near_ids[nn++] = order[r].id;
        }
        if (action == 0) continue;
        if (action == 2) break;
        if (nc == cap) {
          cap *= 2;
          contrib_t *nl = (contrib_t *)realloc(list, sizeof(contrib_t) * cap);
          if (!nl) { err = 1; break; }
          list = nl;
        }
        list[nc].id = order[r].id; list[nc].alpha = alpha; list[nc].T = T; list[nc].G = G;
        list[nc].dx = dx; list[nc].dy = dy; list[nc].clamped = clamped;
        ++nc;
        for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * g->rgb[ch];
        T = Tn;
        relT = relTn;
      }
      for (int ch = 0; ch < 3; ++ch) out_rgb[3 * p + ch] = C[ch] + T * bg[ch];
      out_T[p] = T;
      out_ncontrib[p] = (int32_t)nc;
      out_flag[p] = flag;

      if (gflag) {
        for (size_t j = 0; j < nc; ++j)
          if (gs[list[j].id].flags & ORC_F_NEAR) {
#pragma omp atomic write
            gflag[list[j].id] = 1;
          }
      }
      if (gflag && flag) {
        for (size_t j = 0; j < nc; ++j) {
#pragma omp atomic write
          gflag[list[j].id] = 1;
        }
        for (size_t j = 0; j < nn; ++j) {
#pragma omp atomic write
          gflag[near_ids[j]] = 1;
        }
      }

      if (dL_dC && grad2d) {
        const double gC[3] = {dL_dC[3 * p], dL_dC[3 * p + 1], dL_dC[3 * p + 2]};
        /* suffix colour S_j = sum_{k>j} alpha_k T_k c_k + T_final bg, built back to front */
        double S[3] = {T * bg[0], T * bg[1], T * bg[2]};
        /* chain rounding (see the function comment) */
        const double rho = 4.0 * U32 * (double)nc + 16.0 * U32;
        for (size_t jj = nc; jj-- > 0;) {
          const contrib_t *c = &list[jj];
          const rstate_t *g = &gs[c->id];
          if (e2d) {
            const double om = 1.0 - c->alpha;
            double ma = 0.0;
            for (int ch = 0; ch < 3; ++ch) ma += fabs(gC[ch]) * (c->T * g->rgb[ch] + S[ch] / om);
            double e[9];
            for (int k = 0; k < 9; ++k) e[k] = 0.0;
            if (!c->clamped) {
              const double A = g->conic[0], B = g->conic[1], Cc = g->conic[2];
              const double mdp = rho * c->alpha * ma;
              e[0] = mdp * fabs(A * c->dx + B * c->dy);
              e[1] = mdp * fabs(B * c->dx + Cc * c->dy);
              e[2] = mdp * 0.5 * c->dx * c->dx;
              e[3] = mdp * fabs(c->dx * c->dy);
              e[4] = mdp * 0.5 * c->dy * c->dy;
              e[5] = rho * c->G * ma;
            }
            for (int ch = 0; ch < 3; ++ch) e[6 + ch] = rho * fabs(gC[ch]) * c->alpha * c->T;
            for (int k = 0; k < 9; ++k) {
#pragma omp atomic
              e2d[9 * c->id + k] += e[k];
            }
          }
          double d2[9];
          double dL_dalpha = 0.0;
          for (int ch = 0; ch < 3; ++ch) {
            d2[6 + ch] = gC[ch] * c->alpha * c->T;
            dL_dalpha += gC[ch] * (c->T * g->rgb[ch] - S[ch] / (1.0 - c->alpha));
          }
          double dL_dpower = 0.0, dL_do = 0.0;
          if (!c->clamped) {
            dL_do = dL_dalpha * c->G;
            dL_dpower = dL_dalpha * c->alpha;
          }
          const double A = g->conic[0], B = g->conic[1], Cc = g->conic[2];
          d2[0] = dL_dpower * (A * c->dx + B * c->dy);
          d2[1] = dL_dpower * (B * c->dx + Cc * c->dy);
          d2[2] = dL_dpower * (-0.5 * c->dx * c->dx);
          d2[3] = dL_dpower * (-c->dx * c->dy);
          d2[4] = dL_dpower * (-0.5 * c->dy * c->dy);
          d2[5] = dL_do;
          for (int k = 0; k < 9; ++k) {
#pragma omp atomic
            grad2d[9 * c->id + k] += d2[k];
            if (s2d) {
#pragma omp atomic
              s2d[9 * c->id + k] += fabs(d2[k]);
            }
          }
          for (int ch = 0; ch < 3; ++ch) S[ch] += c->alpha * c->T * g->rgb[ch];
        }
      }
    }
    free(list);
    free(near_ids);
  }
  free(gs);
  free(order);
  return err ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------ preprocess backward */
/* Chain rule from the screen-space gradient d2[9] (u, v, A, B, C, o, r, g, b) of
 * Gaussian i to its raw parameters: means(3), log_scales(3), quats(4), opacity
 * logit(1), sh[k][ch] (3K), written to out[].
 *
 * With magnitude != 0 the same chain is evaluated on absolute values: every factor of
 * every product and every term of every sum is replaced by its absolute value (each SH
 * basis value by the magnitude of its monomials).  That is the size of the terms a
 * float32 evaluation of the chain rounds, in any order, before they cancel: for an
 * isotropic Gaussian, for instance, the quaternion gradient is exactly zero, yet a
 * float32 evaluation leaves a residue of a few U32 of these terms. */
#define AB(x) (magnitude ? fabs(x) : (x))
static void backward_one(const scene_t *sc, int64_t i, const cam_t *cam, const gstate_t *g, const double d2[9],
                         double *out, int magnitude) {
  const int64_t n = sc->n;
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  const int P = 11 + 3 * K;
  const double sg = magnitude ? 1.0 : -1.0;   /* the sign of a subtracted term */
  for (int k = 0; k < P; ++k) out[k] = 0.0;
  if (!g->visible) return;
  double dmu[3] = {0, 0, 0};

  /* colour -> SH coefficients and view direction */
  {
    double Yb[16], dY[16][3];
    if (magnitude) sh_basis_mag(g->dir, Yb); else orc_sh_basis(g->dir, Yb);
    sh_basis_grad(g->dir, dY);
    double ddir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      const double gp = (g->pre[ch] < 0.0) ? 0.0 : AB(d2[6 + ch]);
      for (int k = 0; k < K; ++k) {
        out[11 + 3 * k + ch] = gp * Yb[k];
        const double f = AB(sc->sh[((int64_t)k * 3 + ch) * n + i]);
        for (int a = 0; a < 3; ++a) ddir[a] += gp * f * AB(dY[k][a]);
      }
    }
    double dd = 0.0;
    for (int a = 0; a < 3; ++a) dd += AB(g->dir[a]) * ddir[a];
    for (int a = 0; a < 3; ++a) dmu[a] += (ddir[a] + sg * AB(g->dir[a]) * dd) / g->dist;
  }

  /* opacity */
  out[10] = AB(d2[5]) * g->o * (1.0 - g->o);

  /* conic -> screen covariance: dL/dcov2 = -K GK K, with GK symmetric and the
   * off-diagonal conic entry B appearing twice */
  const double Kc[4] = {AB(g->conic[0]), AB(g->conic[1]), AB(g->conic[1]), AB(g->conic[2])};
  const double GK[4] = {AB(d2[2]), 0.5 * AB(d2[3]), 0.5 * AB(d2[3]), AB(d2[4])};
  double KG[4], GC2[4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) KG[2 * a + b] = Kc[2 * a] * GK[b] + Kc[2 * a + 1] * GK[2 + b];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) GC2[2 * a + b] = sg * (KG[2 * a] * Kc[b] + KG[2 * a + 1] * Kc[2 + b]);

  /* cov2 = M Sigma M^T + 0.3 I:  dSigma = M^T GC2 M,  dM = 2 GC2 M Sigma */
  double GSig[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) acc += AB(g->M[3 * r + a]) * GC2[2 * r + c] * AB(g->M[3 * c + b]);
      GSig[3 * a + b] = acc;
    }
  double GM[6];
  for (int r = 0; r < 2; ++r)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int c = 0; c < 2; ++c)
        for (int k = 0; k < 3; ++k) acc += 2.0 * GC2[2 * r + c] * AB(g->M[3 * c + k]) * AB(g->Sigma[3 * k + b]);
      GM[3 * r + b] = acc;
    }
  /* M = J Rcam:  dJ = dM Rcam^T */
  double GJ[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int b = 0; b < 3; ++b) acc += GM[3 * r + b] * AB(cam->R[3 * k + b]);
      GJ[3 * r + k] = acc;
    }
  /* J -> camera-space centre */
  const double X = g->p[0], Y = g->p[1], Z = g->p[2];
  const double fx = cam->fx, fy = cam->fy;
  double dX = 0, dY_ = 0, dZ = 0, dXt = 0, dYt = 0;
  dZ += GJ[0] * AB(-fx / (Z * Z));
  dXt += GJ[2] * AB(-fx / (Z * Z));
  dZ += GJ[2] * AB(2.0 * fx * g->Xt / (Z * Z * Z));
  dZ += GJ[4] * AB(-fy / (Z * Z));
  dYt += GJ[5] * AB(-fy / (Z * Z));
  dZ += GJ[5] * AB(2.0 * fy * g->Yt / (Z * Z * Z));
  if (g->flags & ORC_F_CLAMPX) dZ += dXt * AB(g->Xt / Z); else dX += dXt;
  if (g->flags & ORC_F_CLAMPY) dZ += dYt * AB(g->Yt / Z); else dY_ += dYt;
  /* projected centre */
  dX += AB(d2[0]) * fx / Z;
  dZ += AB(d2[0]) * AB(-fx * X / (Z * Z));
  dY_ += AB(d2[1]) * fy / Z;
  dZ += AB(d2[1]) * AB(-fy * Y / (Z * Z));
  /* p = Rcam mu + t */
  const double dp[3] = {dX, dY_, dZ};
  for (int a = 0; a < 3; ++a)
    dmu[a] += AB(cam->R[a]) * dp[0] + AB(cam->R[3 + a]) * dp[1] + AB(cam->R[6 + a]) * dp[2];
  for (int a = 0; a < 3; ++a) out[a] = dmu[a];

  /* Sigma = Rq diag(s^2) Rq^T */
  for (int k = 0; k < 3; ++k) {
    double quad = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) quad += AB(g->Rq[3 * a + k]) * GSig[3 * a + b] * AB(g->Rq[3 * b + k]);
    const double ds = 2.0 * g->s[k] * quad;
    out[3 + k] = ds * g->s[k]; /* d/dlog_scale */
  }
  double GR[9];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int b = 0; b < 3; ++b) acc += 2.0 * GSig[3 * a + b] * AB(g->Rq[3 * b + k]) * g->s[k] * g->s[k];
      GR[3 * a + k] = acc;
    }
  double dR[4][9], dqn[4];
  quat_to_rot_grad(g->qn, dR);
  for (int m = 0; m < 4; ++m) {
    double acc = 0.0;
    for (int e = 0; e < 9; ++e) acc += GR[e] * AB(dR[m][e]);
    dqn[m] = acc;
  }
  double dot = 0.0;
  for (int m = 0; m < 4; ++m) dot += AB(g->qn[m]) * dqn[m];
  for (int m = 0; m < 4; ++m) out[6 + m] = (dqn[m] + sg * AB(g->qn[m]) * dot) / g->qnorm;
}
#undef AB

/*
 * grads[n][P] = chain rule of grad2d[n][9] (P = 11 + 3K raw parameters per Gaussian).
 * If s2d and s_raw are given, s_raw[n][P] carries s2d[n][9] to the raw parameters
 * column by column: with abs_chain != 0 through the chain rule evaluated on absolute
 * values (backward_one with magnitude != 0), an upper bound on the sum of the absolute
 * values of the terms each raw-parameter gradient is summed and chained from, which
 * scales its float32 rounding; with abs_chain == 0 through the absolute values of the
 * exact Jacobian, which carries a bound on the error of the screen-space gradient
 * (first order) to the raw parameters.
 */
int orc_preprocess_backward(int64_t n, int sh_degree, const double *means, const double *log_scales,
                            const double *quats, const double *opac, const double *sh, const double *camv,
                            const double *grad2d, const double *s2d, double *grads, double *s_raw, int abs_chain) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3) return ORC_EINVAL;
  scene_t sc; make_scene(&sc, n, sh_degree, means, log_scales, quats, opac, sh);
  cam_t cam; load_cam(camv, &cam);
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const int P = 11 + 3 * K;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    gstate_t g;
    project_one(&sc, i, &cam, &g);
    backward_one(&sc, i, &cam, &g, grad2d + 9 * i, grads + (int64_t)P * i, 0);
    if (s2d && s_raw) {
      double col[59];
      double *sr = s_raw + (int64_t)P * i;
      for (int k = 0; k < P; ++k) sr[k] = 0.0;
      for (int c = 0; c < 9; ++c) {
        double e[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        e[c] = 1.0;
        backward_one(&sc, i, &cam, &g, e, col, abs_chain ? 1 : 0);
        for (int k = 0; k < P; ++k) sr[k] += fabs(col[k]) * s2d[9 * i + c];
      }
    }
  }
  return ORC_OK;
}
