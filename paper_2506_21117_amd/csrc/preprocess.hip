// Per-Gaussian preprocess: projection, colour, extent, tile rectangle (forward), and
// the chain rule from screen-space gradients to raw parameters for the changed
// Gaussians only (Supp. "Local Optimization Kernel", item 3).
//
// One thread per Gaussian; raw parameters are component-major so every load of a
// component is coalesced across the wave.  The projected record is written as three
// 16-byte stores so the rasteriser can gather it with three 16-byte loads.
#include "internal.hpp"

namespace clsp {
namespace {

// Real SH basis up to degree 3 (no Condon-Shortley phase, k = l^2 + l + m).
constexpr float SH0 = 0.28209479177387814f;
constexpr float SH1 = 0.4886025119029199f;
constexpr float SH2A = 1.0925484305920792f;
constexpr float SH2B = 0.31539156525252005f;
constexpr float SH2C = 0.5462742152960396f;
constexpr float SH3A = 0.5900435899266435f;
constexpr float SH3B = 2.890611442640554f;
constexpr float SH3C = 0.4570457994644658f;
constexpr float SH3D = 0.3731763325901154f;
constexpr float SH3E = 1.445305721320277f;

__device__ __forceinline__ void sh_eval(float x, float y, float z, int K, float* Y) {
  Y[0] = SH0;
  if (K > 1) {
    Y[1] = SH1 * y;
    Y[2] = SH1 * z;
    Y[3] = SH1 * x;
  }
  if (K > 4) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH2A * x * y;
    Y[5] = SH2A * y * z;
    Y[6] = SH2B * (3.0f * zz - 1.0f);
    Y[7] = SH2A * x * z;
    Y[8] = SH2C * (xx - yy);
    if (K > 9) {
      Y[9] = SH3A * y * (3.0f * xx - yy);
      Y[10] = SH3B * x * y * z;
      Y[11] = SH3C * y * (5.0f * zz - 1.0f);
      Y[12] = SH3D * z * (5.0f * zz - 3.0f);
      Y[13] = SH3C * x * (5.0f * zz - 1.0f);
      Y[14] = SH3E * z * (xx - yy);
      Y[15] = SH3A * x * (xx - 3.0f * yy);
    }
  }
}

// d(sum_k c_k Y_k)/d(x, y, z) for coefficients c (one colour channel).
__device__ __forceinline__ void sh_eval_grad(float x, float y, float z, int K, const float* c, float& gx, float& gy,
                                             float& gz) {
  gx = gy = gz = 0.0f;
  if (K > 1) {
    gy += SH1 * c[1];
    gz += SH1 * c[2];
    gx += SH1 * c[3];
  }
  if (K > 4) {
    gx += SH2A * y * c[4];
    gy += SH2A * x * c[4];
    gy += SH2A * z * c[5];
    gz += SH2A * y * c[5];
    gz += SH2B * 6.0f * z * c[6];
    gx += SH2A * z * c[7];
    gz += SH2A * x * c[7];
    gx += SH2C * 2.0f * x * c[8];
    gy -= SH2C * 2.0f * y * c[8];
    if (K > 9) {
      const float xx = x * x, yy = y * y, zz = z * z;
      gx += SH3A * 6.0f * x * y * c[9];
      gy += SH3A * 3.0f * (xx - yy) * c[9];
      gx += SH3B * y * z * c[10];
      gy += SH3B * x * z * c[10];
      gz += SH3B * x * y * c[10];
      gy += SH3C * (5.0f * zz - 1.0f) * c[11];
      gz += SH3C * 10.0f * y * z * c[11];
      gz += SH3D * (15.0f * zz - 3.0f) * c[12];
      gx += SH3C * (5.0f * zz - 1.0f) * c[13];
      gz += SH3C * 10.0f * x * z * c[13];
      gx += SH3E * 2.0f * x * z * c[14];
      gy -= SH3E * 2.0f * y * z * c[14];
      gz += SH3E * (xx - yy) * c[14];
      gx += SH3A * 3.0f * (xx - yy) * c[15];
      gy -= SH3A * 6.0f * x * y * c[15];
    }
  }
}

__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R) {
  R[0] = 1.0f - 2.0f * (y * y + z * z);
  R[1] = 2.0f * (x * y - w * z);
  R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);
  R[4] = 1.0f - 2.0f * (x * x + z * z);
  R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);
  R[7] = 2.0f * (y * z + w * x);
  R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Forward geometry shared by the two kernels.  Everything the backward needs is kept.
struct Geo {
  float mu[3];
  float z32;
  float X, Y, Z, invZ;
  float tx, ty;          // lateral ratios after the clamp
  float qn[4], qinv;     // normalised quaternion and 1/|q|
  float Rq[9];
  float s[3];
  float M[6];            // J * Rcam
  float U[6];            // M * Rq * diag(s): cov2 = U U^T + 0.3 I
  float a, b, c;         // cov2 with low-pass
  float A, B, C;         // conic
  float o;
  uint32_t flags;
  bool ok;
};

__device__ __forceinline__ void load_geo(const RawParams& g, int64_t row, const DevCam& cam, Geo& q) {
  const int64_t nr = g.n_rows;
  q.mu[0] = g.means[row];
  q.mu[1] = g.means[nr + row];
  q.mu[2] = g.means[2 * nr + row];
  q.z32 = __fmaf_rn(cam.R[6], q.mu[0], __fmaf_rn(cam.R[7], q.mu[1], __fmaf_rn(cam.R[8], q.mu[2], cam.t[2])));
  q.ok = false;
  q.flags = 0;
  const float qw = g.quats[row], qx = g.quats[nr + row], qy = g.quats[2 * nr + row], qz = g.quats[3 * nr + row];
  const float qq = qw * qw + qx * qx + qy * qy + qz * qz;
  if (!(qq > 0.0f)) return;
  if (!(q.z32 > NEAR_Z)) return;
  q.o = 1.0f / (1.0f + __expf(-g.opac[row]));
  if (q.o < ALPHA_MIN) return;

  q.qinv = rsqrtf(qq);
  q.qn[0] = qw * q.qinv;
  q.qn[1] = qx * q.qinv;
  q.qn[2] = qy * q.qinv;
  q.qn[3] = qz * q.qinv;
  quat_to_rot(q.qn[0], q.qn[1], q.qn[2], q.qn[3], q.Rq);
  for (int k = 0; k < 3; ++k) q.s[k] = __expf(g.log_scales[k * nr + row]);

  q.X = fmaf(cam.R[0], q.mu[0], fmaf(cam.R[1], q.mu[1], fmaf(cam.R[2], q.mu[2], cam.t[0])));
  q.Y = fmaf(cam.R[3], q.mu[0], fmaf(cam.R[4], q.mu[1], fmaf(cam.R[5], q.mu[2], cam.t[1])));
  q.Z = q.z32;
  q.invZ = 1.0f / q.Z;
  float tx = q.X * q.invZ, ty = q.Y * q.invZ;
  if (tx > cam.limx) { tx = cam.limx; q.flags |= CLSP_FLAG_CLAMP_X; }
  if (tx < -cam.limx) { tx = -cam.limx; q.flags |= CLSP_FLAG_CLAMP_X; }
  if (ty > cam.limy) { ty = cam.limy; q.flags |= CLSP_FLAG_CLAMP_Y; }
  if (ty < -cam.limy) { ty = -cam.limy; q.flags |= CLSP_FLAG_CLAMP_Y; }
  q.tx = tx;
  q.ty = ty;
  // J = [[fx/Z, 0, -fx tx/Z], [0, fy/Z, -fy ty/Z]];  M = J Rcam
  const float j00 = cam.fx * q.invZ, j02 = -cam.fx * tx * q.invZ;
  const float j11 = cam.fy * q.invZ, j12 = -cam.fy * ty * q.invZ;
  for (int k = 0; k < 3; ++k) {
    q.M[k] = j00 * cam.R[k] + j02 * cam.R[6 + k];
    q.M[3 + k] = j11 * cam.R[3 + k] + j12 * cam.R[6 + k];
  }
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      q.U[3 * r + k] = (q.M[3 * r] * q.Rq[k] + q.M[3 * r + 1] * q.Rq[3 + k] + q.M[3 * r + 2] * q.Rq[6 + k]) * q.s[k];
  q.a = q.U[0] * q.U[0] + q.U[1] * q.U[1] + q.U[2] * q.U[2] + LOWPASS;
  q.b = q.U[0] * q.U[3] + q.U[1] * q.U[4] + q.U[2] * q.U[5];
  q.c = q.U[3] * q.U[3] + q.U[4] * q.U[4] + q.U[5] * q.U[5] + LOWPASS;
  const float det = q.a * q.c - q.b * q.b;
  if (!(det > 0.0f)) return;
  const float id = 1.0f / det;
  q.A = q.c * id;
  q.B = -q.b * id;
  q.C = q.a * id;
  q.ok = true;
}

__device__ __forceinline__ void view_dir(const Geo& q, const DevCam& cam, float* d, float& dist) {
  const float dx = q.mu[0] - cam.campos[0], dy = q.mu[1] - cam.campos[1], dz = q.mu[2] - cam.campos[2];
  const float d2 = dx * dx + dy * dy + dz * dz;
  const float inv = rsqrtf(d2);
  dist = d2 * inv;
  d[0] = dx * inv;
  d[1] = dy * inv;
  d[2] = dz * inv;
}

__global__ void __launch_bounds__(256) preprocess_kernel(RawParams g, DevCam cam, int view, int64_t r0, int64_t r1,
                                                         float* __restrict__ splat, float* __restrict__ depth,
                                                         uint2* __restrict__ rect, uint32_t* __restrict__ flags) {
  const int64_t i = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  const int64_t row = g.gather ? (int64_t)g.gather[i] : i;
  const int64_t e = (int64_t)view * g.n + i;
  Geo q;
  load_geo(g, row, cam, q);
  float4* out = reinterpret_cast<float4*>(splat + e * SPLAT_STRIDE);
  depth[e] = q.z32;
  if (!q.ok) {
    out[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    rect[e] = make_uint2(0u, 0u);
    flags[e] = 0u;
    return;
  }
  const float u = cam.fx * q.X * q.invZ + cam.cx;
  const float v = cam.fy * q.Y * q.invZ + cam.cy;

  // colour
  const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
  float d[3], dist;
  view_dir(q, cam, d, dist);
  float Yb[16];
  sh_eval(d[0], d[1], d[2], K, Yb);
  float rgb[3];
  uint32_t fl = q.flags | CLSP_FLAG_VISIBLE;
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
    for (int k = 0; k < K; ++k) acc = fmaf(g.sh[((int64_t)k * 3 + ch) * g.n_rows + row], Yb[k], acc);
    if (acc < 0.0f) {
      acc = 0.0f;
      fl |= (CLSP_FLAG_SHCLAMP_R << ch);
    }
    rgb[ch] = acc;
  }

  // extent of the ellipse alpha >= 1/255, and its tile rectangle, evaluated from the
  // rounded extents that are stored: no contraction here, or u + rx would be fused
  // with rx's last product into an fma and round differently from the stored values
  float rx, ry, fx0, fx1, fy0, fy1;
  {
#pragma clang fp contract(off)
    const float kappa = 2.0f * (__logf(q.o) + 5.541263545158426f);  // 2 ln(255 o)
    const float kap = fmaxf(kappa, 0.0f);
    rx = sqrtf(kap * q.a) * EXTENT_MARGIN;
    ry = sqrtf(kap * q.c) * EXTENT_MARGIN;
    fx0 = floorf(((u - rx) - 0.5f) * 0.0625f);
    fx1 = floorf(((u + rx) - 0.5f) * 0.0625f) + 1.0f;
    fy0 = floorf(((v - ry) - 0.5f) * 0.0625f);
    fy1 = floorf(((v + ry) - 0.5f) * 0.0625f) + 1.0f;
  }
  const uint32_t x0 = (uint32_t)fminf(fmaxf(fx0, 0.0f), (float)cam.TX);
  const uint32_t x1 = (uint32_t)fminf(fmaxf(fx1, 0.0f), (float)cam.TX);
  const uint32_t y0 = (uint32_t)fminf(fmaxf(fy0, 0.0f), (float)cam.TY);
  const uint32_t y1 = (uint32_t)fminf(fmaxf(fy1, 0.0f), (float)cam.TY);

  out[0] = make_float4(u, v, q.A, q.B);
  out[1] = make_float4(q.C, q.o, rgb[0], rgb[1]);
  out[2] = make_float4(rgb[2], rx, ry, 0.0f);
  rect[e] = make_uint2(x0 | (x1 << 16), y0 | (y1 << 16));
  flags[e] = fl;
}

// Chain rule for changed Gaussian i (in [a0, a1)) of one view: hands each parameter
// component's gradient to put(c, value) once, c over the flat list means[3],
// log_scales[3], quats[4], opacity, sh[3K] (sh coefficient k of channel ch is
// 11 + 3k + ch); components without a gradient (invisible, clamped channel, no
// screen-space gradient) are not handed over.
template <int KD = -1, class Put>
__device__ __forceinline__ void backward_row(const RawParams& g, const DevCam& cam, int view, int64_t i, int64_t a0,
                                             int64_t a1, const uint32_t* __restrict__ flags,
                                             const float* __restrict__ grad2d, Put put) {
  const int64_t e = (int64_t)view * g.n + i;
  const uint32_t fl = flags[e];
  if (!(fl & CLSP_FLAG_VISIBLE)) return;
  const float4* gp = reinterpret_cast<const float4*>(grad2d + ((int64_t)view * (a1 - a0) + (i - a0)) * G2D_STRIDE);
  const float4 g0 = gp[0], g1 = gp[1], g2 = gp[2];
  const float gu = g0.x, gv = g0.y, gA = g0.z, gB = g0.w, gC = g1.x, go = g1.y;
  const float gcol[3] = {g1.z, g1.w, g2.x};
  if (gu == 0.f && gv == 0.f && gA == 0.f && gB == 0.f && gC == 0.f && go == 0.f && gcol[0] == 0.f &&
      gcol[1] == 0.f && gcol[2] == 0.f)
    return;

  const int64_t row = i;  // gradients are produced for the un-gathered parameter layout
  Geo q;
  load_geo(g, row, cam, q);
  const int64_t nr = g.n_rows;
  // (KD: the SH degree when the caller fixes it at compile time, so that every component
  // index handed to put is a constant)
  const int K = KD >= 0 ? (KD + 1) * (KD + 1) : (g.sh_degree + 1) * (g.sh_degree + 1);

  float dmu[3] = {0.f, 0.f, 0.f};

  // colour: SH coefficients and the view direction (clamped channels pass nothing)
  {
    float d[3], dist;
    view_dir(q, cam, d, dist);
    float Yb[16];
    sh_eval(d[0], d[1], d[2], K, Yb);
    float gd[3] = {0.f, 0.f, 0.f};
    for (int ch = 0; ch < 3; ++ch) {
      const float gpre = (fl & (CLSP_FLAG_SHCLAMP_R << ch)) ? 0.0f : gcol[ch];
      if (gpre == 0.0f) continue;
      float coef[16];
      for (int k = 0; k < K; ++k) {
        coef[k] = g.sh[((int64_t)k * 3 + ch) * nr + row];
        put(11 + k * 3 + ch, gpre * Yb[k]);
      }
      float gx, gy, gz;
      sh_eval_grad(d[0], d[1], d[2], K, coef, gx, gy, gz);
      gd[0] += gpre * gx;
      gd[1] += gpre * gy;
      gd[2] += gpre * gz;
    }
    const float dd = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
    const float invd = 1.0f / dist;
    for (int k = 0; k < 3; ++k) dmu[k] += (gd[k] - d[k] * dd) * invd;
  }

  // opacity
  put(10, go * q.o * (1.0f - q.o));

  // conic -> screen covariance: G2 = -K GK K with GK = [[gA, gB/2], [gB/2, gC]]
  const float h = 0.5f * gB;
  const float k00 = q.A * gA + q.B * h, k01 = q.A * h + q.B * gC;
  const float k10 = q.B * gA + q.C * h, k11 = q.B * h + q.C * gC;
  const float G00 = -(k00 * q.A + k01 * q.B);
  const float G01 = -(k00 * q.B + k01 * q.C);
  const float G11 = -(k10 * q.B + k11 * q.C);
  // cov2 = U U^T (+0.3 I), U = M Rq diag(s):  dU = 2 G2 U
  float gU[6];
  for (int k = 0; k < 3; ++k) {
    gU[k] = 2.0f * (G00 * q.U[k] + G01 * q.U[3 + k]);
    gU[3 + k] = 2.0f * (G01 * q.U[k] + G11 * q.U[3 + k]);
  }
  // U = M W with W = Rq diag(s): dM = dU W^T ; dW = M^T dU
  float W[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) W[3 * r + k] = q.Rq[3 * r + k] * q.s[k];
  float gM[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) gM[3 * r + c] = gU[3 * r] * W[3 * c] + gU[3 * r + 1] * W[3 * c + 1] + gU[3 * r + 2] * W[3 * c + 2];
  float gW[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) gW[3 * r + k] = q.M[r] * gU[k] + q.M[3 + r] * gU[3 + k];
  // W = Rq diag(s): d log s_k = s_k * sum_r dW[r][k] Rq[r][k];  dRq[r][k] = dW[r][k] s_k
  float gR[9];
  for (int k = 0; k < 3; ++k) {
    const float acc = gW[k] * q.Rq[k] + gW[3 + k] * q.Rq[3 + k] + gW[6 + k] * q.Rq[6 + k];
    put(3 + k, acc * q.s[k]);
    gR[k] = gW[k] * q.s[k];
    gR[3 + k] = gW[3 + k] * q.s[k];
    gR[6 + k] = gW[6 + k] * q.s[k];
  }
  // Rq(qn) -> qn
  {
    const float w = q.qn[0], x = q.qn[1], y = q.qn[2], z = q.qn[3];
    const float gw = 2.0f * (z * (gR[3] - gR[1]) + y * (gR[2] - gR[6]) + x * (gR[7] - gR[5]));
    const float gx = 2.0f * (y * (gR[1] + gR[3]) + z * (gR[2] + gR[6]) + w * (gR[7] - gR[5])) - 4.0f * x * (gR[4] + gR[8]);
    const float gy = 2.0f * (x * (gR[1] + gR[3]) + w * (gR[2] - gR[6]) + z * (gR[5] + gR[7])) - 4.0f * y * (gR[0] + gR[8]);
    const float gz = 2.0f * (w * (gR[3] - gR[1]) + x * (gR[2] + gR[6]) + y * (gR[5] + gR[7])) - 4.0f * z * (gR[0] + gR[4]);
    const float dot = w * gw + x * gx + y * gy + z * gz;
    put(6, (gw - w * dot) * q.qinv);
    put(7, (gx - x * dot) * q.qinv);
    put(8, (gy - y * dot) * q.qinv);
    put(9, (gz - z * dot) * q.qinv);
  }
  // M = J Rcam: dJ = dM Rcam^T (only the four non-zero entries of J matter)
  const float gJ00 = gM[0] * cam.R[0] + gM[1] * cam.R[1] + gM[2] * cam.R[2];
  const float gJ02 = gM[0] * cam.R[6] + gM[1] * cam.R[7] + gM[2] * cam.R[8];
  const float gJ11 = gM[3] * cam.R[3] + gM[4] * cam.R[4] + gM[5] * cam.R[5];
  const float gJ12 = gM[3] * cam.R[6] + gM[4] * cam.R[7] + gM[5] * cam.R[8];
  // J entries as functions of (X, Y, Z); with t = X/Z (or its clamp):
  // j00 = fx/Z, j02 = -fx t/Z, j11 = fy/Z, j12 = -fy ty/Z
  const float iz = q.invZ, iz2 = iz * iz;
  float gX = 0.f, gY = 0.f, gZ = 0.f;
  gZ += -cam.fx * iz2 * gJ00 - cam.fy * iz2 * gJ11;
  {
    // j02 = -fx Xt / Z^2 with Xt = X unclamped, Xt = +-lim Z clamped
    const float Xt = q.tx * q.Z;
    gZ += 2.0f * cam.fx * Xt * iz2 * iz * gJ02;
    const float gXt = -cam.fx * iz2 * gJ02;
    if (fl & CLSP_FLAG_CLAMP_X) gZ += gXt * q.tx; else gX += gXt;
    const float Yt = q.ty * q.Z;
    gZ += 2.0f * cam.fy * Yt * iz2 * iz * gJ12;
    const float gYt = -cam.fy * iz2 * gJ12;
    if (fl & CLSP_FLAG_CLAMP_Y) gZ += gYt * q.ty; else gY += gYt;
  }
  // projected centre
  gX += gu * cam.fx * iz;
  gY += gv * cam.fy * iz;
  gZ -= (gu * cam.fx * q.X + gv * cam.fy * q.Y) * iz2;
  // p = Rcam mu + t
  for (int k = 0; k < 3; ++k) dmu[k] += cam.R[k] * gX + cam.R[3 + k] * gY + cam.R[6 + k] * gZ;
  put(0, dmu[0]);
  put(1, dmu[1]);
  put(2, dmu[2]);
}

// Component c of row i of a parameter set (the flat order of backward_row).
__device__ __forceinline__ float* param_comp(const MutParams& X, int c, int64_t i) {
  const int64_t n = X.n;
  if (c < 3) return X.means + c * n + i;
  if (c < 6) return X.log_scales + (c - 3) * n + i;
  if (c < 10) return X.quats + (c - 6) * n + i;
  if (c == 10) return X.opac + i;
  return X.sh + (int64_t)(c - 11) * n + i;
}

// Chain rule for the changed Gaussians [a0, a1) of one view; adds into grads.
__global__ void __launch_bounds__(128) preprocess_backward_kernel(RawParams g, DevCam cam, int view, int64_t a0,
                                                                  int64_t a1, const uint32_t* __restrict__ flags,
                                                                  const float* __restrict__ grad2d, MutParams out,
                                                                  const uint32_t* __restrict__ skip) {
  const int64_t i = a0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a1 || (skip && *skip)) return;
  backward_row(g, cam, view, i, a0, a1, flags, grad2d, [&](int c, float v) { *param_comp(out, c, i) += v; });
}

// The same for a single view, followed by one Adam step of the row with those
// gradients (the rest zero), exactly as zeroed gradients + the kernel above + the Adam
// kernel would do it.  D: the SH degree.  The row's gradients are collected first (every
// component index a constant), then every component gets the same Adam update, sixteen
// at a time with their moments and parameters all read before any is written (the
// arrays may alias as far as the compiler knows); the first sixteen are read before the
// gradients are computed, together with the step's skip flag and count.
template <int D>
__device__ __forceinline__ void backward_adam_row(const RawParams& g, const DevCam& cam, int64_t a0, int64_t a1,
                                                  const uint32_t* __restrict__ flags,
                                                  const float* __restrict__ grad2d, const FusedAdam& A, int64_t i) {
  constexpr int C = 11 + 3 * (D + 1) * (D + 1), G = 16, G0 = C < G ? C : G;
  float m0[G0], v0[G0], p0[G0];
#pragma unroll
  for (int c = 0; c < G0; ++c) {
    m0[c] = *param_comp(A.M, c, i);
    v0[c] = *param_comp(A.V, c, i);
    p0[c] = *param_comp(A.P, c, i);
  }
  // a step whose lists ran out of pair capacity updates nothing (the raster backward
  // wrote no gradient either, so the workspace is still zero)
  if (A.skip && *A.skip) return;
  float bc1 = A.bc1, bc2 = A.bc2;
  if (A.step_dev) {
    const float t = (float)max(*A.step_dev, 1);
    bc1 = 1.0f - powf(A.b1, t);
    bc2 = 1.0f - powf(A.b2, t);
  }
  float gr[C];
#pragma unroll
  for (int c = 0; c < C; ++c) gr[c] = 0.0f;
  // the gradient as the separate calls see it: 0 + v
  backward_row<D>(g, cam, 0, i, a0, a1, flags, grad2d, [&](int c, float v) { gr[c] = 0.0f + v; });
  auto update = [&](int c, float m, float v, float p, float gg) {
    const int grp = c < 3 ? 0 : c < 6 ? 1 : c < 10 ? 2 : c == 10 ? 3 : c < 14 ? 4 : 5;
    const float mm = A.b1 * m + (1.0f - A.b1) * gg;
    const float vv = A.b2 * v + (1.0f - A.b2) * gg * gg;
    *param_comp(A.M, c, i) = mm;
    *param_comp(A.V, c, i) = vv;
    *param_comp(A.P, c, i) = p - A.lr[grp] * (mm / bc1) / (sqrtf(vv / bc2) + A.eps);
  };
#pragma unroll
  for (int c = 0; c < G0; ++c) update(c, m0[c], v0[c], p0[c], gr[c]);
#pragma unroll
  for (int c0 = G; c0 < C; c0 += G) {
    float mv[G], vv[G], pv[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (c0 + u < C) {
        mv[u] = *param_comp(A.M, c0 + u, i);
        vv[u] = *param_comp(A.V, c0 + u, i);
        pv[u] = *param_comp(A.P, c0 + u, i);
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (c0 + u < C) update(c0 + u, mv[u], vv[u], pv[u], gr[c0 + u]);
  }
  // leave the row's screen-space gradient zero for the next call, which then needs no
  // clearing launch (rows never reached here were never written)
  float4* gp = reinterpret_cast<float4*>(const_cast<float*>(grad2d) + (i - a0) * G2D_STRIDE);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  gp[0] = z;
  gp[1] = z;
  gp[2] = z;
}

__global__ void __launch_bounds__(128) preprocess_backward_adam_kernel(RawParams g, DevCam cam, int64_t a0,
                                                                       int64_t a1, const uint32_t* __restrict__ flags,
                                                                       const float* __restrict__ grad2d, FusedAdam A) {
  const int64_t i = a0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a1) return;
  switch (A.P.sh_degree) {
    case 0: backward_adam_row<0>(g, cam, a0, a1, flags, grad2d, A, i); break;
    case 1: backward_adam_row<1>(g, cam, a0, a1, flags, grad2d, A, i); break;
    case 2: backward_adam_row<2>(g, cam, a0, a1, flags, grad2d, A, i); break;
    default: backward_adam_row<3>(g, cam, a0, a1, flags, grad2d, A, i); break;
  }
}

}  // namespace

hipError_t launch_preprocess(const RawParams& g, const DevCam& cam, int view, int64_t r0, int64_t r1, float* splat,
                             float* depth, uint32_t* rect, uint32_t* flags, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const int blocks = ceil_div(r1 - r0, 256);
  hipLaunchKernelGGL(preprocess_kernel, dim3(blocks), dim3(256), 0, s, g, cam, view, r0, r1, splat, depth,
                     reinterpret_cast<uint2*>(rect), flags);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward_adam(const RawParams& g, const DevCam& cam, int64_t a0, int64_t a1,
                                           const uint32_t* flags, const float* grad2d, const FusedAdam& A,
                                           hipStream_t s) {
  if (a1 <= a0) return hipSuccess;
  hipLaunchKernelGGL(preprocess_backward_adam_kernel, dim3(ceil_div(a1 - a0, 128)), dim3(128), 0, s, g, cam, a0, a1,
                     flags, grad2d, A);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(const RawParams& g, const DevCam& cam, int view, int64_t a0, int64_t a1,
                                      const uint32_t* flags, const float* grad2d, const MutParams& grads,
                                      const uint32_t* skip, hipStream_t s) {
  if (a1 <= a0) return hipSuccess;
  const int blocks = ceil_div(a1 - a0, 128);
  hipLaunchKernelGGL(preprocess_backward_kernel, dim3(blocks), dim3(128), 0, s, g, cam, view, a0, a1, flags, grad2d,
                     grads, skip);
  return hipGetLastError();
}

}  // namespace clsp
