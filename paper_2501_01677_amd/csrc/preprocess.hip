// Per-Gaussian projection (forward) and its chain rule (backward).
//
// Forward, one thread per Gaussian of a set, looping over the views that
// draw the set so the raw parameters are read once per step (Sec. 3.1:
// each 3D Gaussian becomes a 2D Gaussian per viewing direction):
//   scale = exp(log_scale), unit quaternion, opacity = sigmoid(logit)
//   t = R_c mean + t_c;  EWA covariance  J R_c R S^2 R^T R_c^T J^T + 0.3 I
//   conic = inverse covariance, 2D mean, SH colour (+0.5, clamped at 0),
//   camera-frame normal of the smallest-scale axis facing the camera
//   (Eq. 2) and the plane distance n_c . t (Eq. 3), the FP32 depth key and
//   the support rectangle in tiles with its number of active tiles.
// Backward, same thread shape: reads the per-view 2D gradients written by
// the backward compositing and applies the chain rule to the raw
// parameters, summing over views, and overwrites the gradient arrays.
#include "internal.h"

namespace pgsag {
namespace {

// Real SH basis (orthonormal, Condon-Shortley phase) as polynomials of the
// unit direction; coefficients are the closed forms
//   sqrt(1/(4pi)), sqrt(3/(4pi)), sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4,
//   sqrt(35/(2pi))/4, sqrt(105/pi)/2, sqrt(21/(2pi))/4, sqrt(7/pi)/4,
//   sqrt(105/pi)/4.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.54627421529603959f;
constexpr float kY3a = 0.59004358992664352f;
constexpr float kY3b = 2.8906114426405538f;
constexpr float kY3c = 0.45704579946446572f;
constexpr float kY3d = 0.37317633259011540f;
constexpr float kY3e = 1.4453057213202769f;

__device__ inline void sh_basis(int deg, float x, float y, float z, float *B) {
  B[0] = kY0;
  if (deg < 1) return;
  B[1] = -kY1 * y;
  B[2] = kY1 * z;
  B[3] = -kY1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  B[4] = kY2a * x * y;
  B[5] = -kY2a * y * z;
  B[6] = kY2b * (3.f * zz - 1.f);
  B[7] = -kY2a * x * z;
  B[8] = kY2c * (xx - yy);
  if (deg < 3) return;
  B[9] = -kY3a * y * (3.f * xx - yy);
  B[10] = kY3b * x * y * z;
  B[11] = -kY3c * y * (5.f * zz - 1.f);
  B[12] = kY3d * z * (5.f * zz - 3.f);
  B[13] = -kY3c * x * (5.f * zz - 1.f);
  B[14] = kY3e * z * (xx - yy);
  B[15] = -kY3a * x * (xx - 3.f * yy);
}

// d(sum_j w_j B_j)/d(x,y,z) for weights w (the polynomial extension of the
// basis off the sphere; only its tangential part is used).
__device__ inline void sh_basis_grad(int deg, float x, float y, float z, const float *w,
                                     float &gx, float &gy, float &gz) {
  gx = gy = gz = 0.f;
  if (deg < 1) return;
  gy += -kY1 * w[1];
  gz += kY1 * w[2];
  gx += -kY1 * w[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += kY2a * y * w[4];
  gy += kY2a * x * w[4];
  gy += -kY2a * z * w[5];
  gz += -kY2a * y * w[5];
  gz += 6.f * kY2b * z * w[6];
  gx += -kY2a * z * w[7];
  gz += -kY2a * x * w[7];
  gx += 2.f * kY2c * x * w[8];
  gy += -2.f * kY2c * y * w[8];
  if (deg < 3) return;
  gx += -kY3a * 6.f * x * y * w[9];
  gy += -kY3a * 3.f * (xx - yy) * w[9];
  gx += kY3b * y * z * w[10];
  gy += kY3b * x * z * w[10];
  gz += kY3b * x * y * w[10];
  gy += -kY3c * (5.f * zz - 1.f) * w[11];
  gz += -kY3c * 10.f * y * z * w[11];
  gz += kY3d * (15.f * zz - 3.f) * w[12];
  gx += -kY3c * (5.f * zz - 1.f) * w[13];
  gz += -kY3c * 10.f * x * z * w[13];
  gx += 2.f * kY3e * x * z * w[14];
  gy += -2.f * kY3e * y * z * w[14];
  gz += kY3e * (xx - yy) * w[14];
  gx += -kY3a * 3.f * (xx - yy) * w[15];
  gy += kY3a * 6.f * x * y * w[15];
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ inline void quat_rot(float w, float x, float y, float z, float *M) {
  M[0] = 1.f - 2.f * (y * y + z * z);
  M[1] = 2.f * (x * y - w * z);
  M[2] = 2.f * (x * z + w * y);
  M[3] = 2.f * (x * y + w * z);
  M[4] = 1.f - 2.f * (x * x + z * z);
  M[5] = 2.f * (y * z - w * x);
  M[6] = 2.f * (x * z - w * y);
  M[7] = 2.f * (y * z + w * x);
  M[8] = 1.f - 2.f * (x * x + y * y);
}

// Gradient of sum_ij G_ij M_ij(q) with respect to the unit quaternion.
__device__ inline void quat_rot_vjp(float w, float x, float y, float z, const float *G,
                                    float &gw, float &gx, float &gy, float &gz) {
  gw = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  gx = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
              2.f * x * G[8]);
  gy = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
              2.f * y * G[8]);
  gz = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] +
              x * G[6] + y * G[7]);
}

struct Raw {
  float mx, my, mz;
  float ls[3], s[3];
  float qw, qx, qy, qz, qn;  // normalised quaternion and the input norm
  float logit, o;
  float M[9];  // rotation of the Gaussian
  int jstar;
  float ax, ay, az;  // column jstar of M (the Gaussian normal, world frame)
};

__device__ inline void load_raw(const DevSet &S, int64_t i, Raw &g) {
  const int64_t n = S.n;
  g.mx = S.means[i];
  g.my = S.means[n + i];
  g.mz = S.means[2 * n + i];
  for (int k = 0; k < 3; ++k) {
    g.ls[k] = S.log_scales[k * n + i];
    g.s[k] = __expf(g.ls[k]);
  }
  float qw = S.quats[i], qx = S.quats[n + i], qy = S.quats[2 * n + i], qz = S.quats[3 * n + i];
  float nn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  float inv = 1.f / nn;
  g.qn = nn;
  g.qw = qw * inv; g.qx = qx * inv; g.qy = qy * inv; g.qz = qz * inv;
  g.logit = S.logits[i];
  g.o = 1.f / (1.f + __expf(-g.logit));
  quat_rot(g.qw, g.qx, g.qy, g.qz, g.M);
  int j = 0;
  if (g.ls[1] < g.ls[j]) j = 1;
  if (g.ls[2] < g.ls[j]) j = 2;
  g.jstar = j;
  // arithmetic selection keeps M in registers (no addressable array)
  const float e0 = j == 0 ? 1.f : 0.f, e1 = j == 1 ? 1.f : 0.f, e2 = j == 2 ? 1.f : 0.f;
  g.ax = e0 * g.M[0] + e1 * g.M[1] + e2 * g.M[2];
  g.ay = e0 * g.M[3] + e1 * g.M[4] + e2 * g.M[5];
  g.az = e0 * g.M[6] + e1 * g.M[7] + e2 * g.M[8];
}

// FP32 depth key of the mean: ((R20 x + R21 y) + R22 z) + t2, each operation
// rounded on its own (no contraction), so every implementation agrees on it.
// hipcc contracts a*b + c into an FMA by default (also inside the
// __fmul_rn/__fadd_rn helpers), which would change the rounding; the
// operations are written here with contraction switched off.
__device__ inline float depth_key(const DevCamera &c, const Raw &g) {
#pragma clang fp contract(off)
  const float a = c.R[6] * g.mx;
  const float b = c.R[7] * g.my;
  const float d = c.R[8] * g.mz;
  const float ab = a + b;
  const float abd = ab + d;
  return abd + c.t[2];
}

// View-dependent projection shared by forward and backward.
struct View {
  float tx, ty, tz;        // camera-frame mean
  float xt, yt;            // clamped lateral coordinates used in J
  bool clx, cly;           // clamp active
  float T[6];              // J * R_c (2x3)
  float U[6];              // T * M * diag(s) (2x3)
  float cxx, cxy, cyy;     // covariance incl. dilation
  float ca, cb, cc;        // conic
  float mx, my;            // 2D mean
  float n[3];              // camera-frame normal (flipped)
  float sgn;               // +1 / -1 flip
  float d;                 // plane distance
  float dir[3];            // unit view direction (world)
  float vlen;              // |mean - centre|
};

__device__ inline void project_view(const DevCamera &c, const Header &h, const Raw &g, View &v) {
  const float *R = c.R;
  v.tx = R[0] * g.mx + R[1] * g.my + R[2] * g.mz + c.t[0];
  v.ty = R[3] * g.mx + R[4] * g.my + R[5] * g.mz + c.t[1];
  v.tz = R[6] * g.mx + R[7] * g.my + R[8] * g.mz + c.t[2];
  const float iz = 1.f / v.tz;
  const float rx = v.tx * iz, ry = v.ty * iz;
  v.clx = (rx < -c.limx) || (rx > c.limx);
  v.cly = (ry < -c.limy) || (ry > c.limy);
  v.xt = fminf(fmaxf(rx, -c.limx), c.limx) * v.tz;
  v.yt = fminf(fmaxf(ry, -c.limy), c.limy) * v.tz;
  const float j00 = c.fx * iz, j02 = -c.fx * v.xt * iz * iz;
  const float j11 = c.fy * iz, j12 = -c.fy * v.yt * iz * iz;
  for (int k = 0; k < 3; ++k) {
    v.T[k] = j00 * R[k] + j02 * R[6 + k];
    v.T[3 + k] = j11 * R[3 + k] + j12 * R[6 + k];
  }
  // U = T * M * diag(s)
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      v.U[3 * r + k] = (v.T[3 * r] * g.M[k] + v.T[3 * r + 1] * g.M[3 + k] + v.T[3 * r + 2] * g.M[6 + k]) * g.s[k];
  v.cxx = v.U[0] * v.U[0] + v.U[1] * v.U[1] + v.U[2] * v.U[2] + h.cfg.dilation;
  v.cxy = v.U[0] * v.U[3] + v.U[1] * v.U[4] + v.U[2] * v.U[5];
  v.cyy = v.U[3] * v.U[3] + v.U[4] * v.U[4] + v.U[5] * v.U[5] + h.cfg.dilation;
  const float det = v.cxx * v.cyy - v.cxy * v.cxy;
  const float idet = 1.f / det;
  v.ca = v.cyy * idet;
  v.cb = -v.cxy * idet;
  v.cc = v.cxx * idet;
  v.mx = c.fx * rx + c.cx;
  v.my = c.fy * ry + c.cy;
  // normal: axis j* of the Gaussian rotation, into the camera frame
  const float ax = g.ax, ay = g.ay, az = g.az;
  float n0 = R[0] * ax + R[1] * ay + R[2] * az;
  float n1 = R[3] * ax + R[4] * ay + R[5] * az;
  float n2 = R[6] * ax + R[7] * ay + R[8] * az;
  const float dt = n0 * v.tx + n1 * v.ty + n2 * v.tz;
  v.sgn = dt > 0.f ? -1.f : 1.f;
  v.n[0] = v.sgn * n0; v.n[1] = v.sgn * n1; v.n[2] = v.sgn * n2;
  v.d = v.n[0] * v.tx + v.n[1] * v.ty + v.n[2] * v.tz;
  const float dx = g.mx - c.centre[0], dy = g.my - c.centre[1], dz = g.mz - c.centre[2];
  v.vlen = sqrtf(dx * dx + dy * dy + dz * dz);
  const float il = 1.f / v.vlen;
  v.dir[0] = dx * il; v.dir[1] = dy * il; v.dir[2] = dz * il;
}

// Thread -> (set, Gaussian) for the sets of SH degree D.
template <int D>
__device__ inline bool locate(const void *desc, const DevSet *&S, int64_t &i) {
  const Header &h = *header(desc);
  const int32_t *ids = deg_ids_of(desc, D);
  const uint32_t *starts = deg_starts_of(desc, D);
  const int k = upper_index(starts, h.deg_count[D], (uint32_t)blockIdx.x);
  S = sets_of(desc) + ids[k];
  i = (int64_t)(blockIdx.x - starts[k]) * blockDim.x + threadIdx.x;
  return i < S->n;
}

// Active tiles of a tile rectangle from the per-row prefix of active flags;
// four rows' loads are issued together.
__device__ inline uint32_t count_active(const uint32_t *rowsat, uint32_t pitch, uint32_t x0, uint32_t y0, uint32_t x1,
                                        uint32_t y1) {
  uint32_t c = 0;
  uint32_t y = y0;
  for (; y + 4 <= y1; y += 4) {
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hi[k] = rowsat[(y + k) * pitch + x1];
      lo[k] = rowsat[(y + k) * pitch + x0];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) c += hi[k] - lo[k];
  }
  for (; y < y1; ++y) c += rowsat[y * pitch + x1] - rowsat[y * pitch + x0];
  return c;
}

template <int D>
__global__ void __launch_bounds__(256) preprocess_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  constexpr int K = (D + 1) * (D + 1);
  const Header &h = *header(desc);
  const DevSet *Sp;
  int64_t i;
  if (!locate<D>(desc, Sp, i)) return;
  const DevSet &S = *Sp;
  const DevRender *rends = renders_of(desc);
  const int64_t n = S.n;
  Raw g;
  load_raw(S, i, g);
  // The SH coefficients (most of the bytes) are loaded once per Gaussian,
  // with the other parameters, and serve every view below.
  float shc[3 * K];
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) shc[j] = S.sh[j * n + i];
  float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  uint32_t *dkey = ws_ptr<uint32_t>(ws, h.ws.depth_key);
  uint2 *rect = ws_ptr<uint2>(ws, h.ws.rect);
  uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  const uint32_t *sat = ws_ptr<uint32_t>(ws, h.ws.sat);
  const int tile = h.cfg.tile;
  const bool opaque_enough = g.logit >= h.cfg.logit_min;

  for (int vi = 0; vi < S.n_renders; ++vi) {
    const DevRender &rd = rends[S.renders[vi]];
    const DevCamera &c = rd.cam;
    const uint64_t r = rd.record_offset + (uint64_t)i;
    const float key = depth_key(c, g);
    uint32_t count = 0;
    uint2 rr = make_uint2(0u, 0u);
    if (key > h.cfg.z_near && opaque_enough) {
      // Colour first: it needs only the view direction, so its arithmetic
      // overlaps the projection's.
      float col[3];
      {
        const float dx = g.mx - c.centre[0], dy = g.my - c.centre[1], dz = g.mz - c.centre[2];
        const float il = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        float B[16];
        sh_basis(D, dx * il, dy * il, dz * il, B);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          float a = 0.5f;
#pragma unroll
          for (int j = 0; j < K; ++j) a += B[j] * shc[3 * j + k];
          col[k] = fmaxf(a, 0.f);
        }
      }
      View v;
      project_view(c, h, g, v);
      // support: q <= 2 ln(o / alpha_min), with a small outward margin
      const float qmax = 2.f * __logf(g.o / h.cfg.alpha_min);
      if (qmax > 0.f && v.tz > 0.f) {
        const float hx = sqrtf(qmax * v.cxx) * 1.0001f + 1e-3f;
        const float hy = sqrtf(qmax * v.cyy) * 1.0001f + 1e-3f;
        // pixel centres u + 0.5 inside [mx - hx, mx + hx]
        const float fu0 = fminf(fmaxf(ceilf(v.mx - hx - 0.5f), 0.f), (float)c.W);
        const float fu1 = fminf(fmaxf(floorf(v.mx + hx - 0.5f), -1.f), (float)(c.W - 1));
        const float fv0 = fminf(fmaxf(ceilf(v.my - hy - 0.5f), 0.f), (float)c.H);
        const float fv1 = fminf(fmaxf(floorf(v.my + hy - 0.5f), -1.f), (float)(c.H - 1));
        const int u0 = (int)fu0, u1 = (int)fu1, w0 = (int)fv0, w1 = (int)fv1;
        if (u0 <= u1 && w0 <= w1) {
          const uint32_t x0 = u0 / tile, x1 = u1 / tile + 1, y0 = w0 / tile, y1 = w1 / tile + 1;
          count = count_active(sat + rd.sat_offset, rd.tiles_x + 1, x0, y0, x1, y1);
          rr = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
        }
        if (count > 0) {
          rec4[r * 4 + 0] = make_float4(v.mx, v.my, v.ca, v.cb);
          rec4[r * 4 + 1] = make_float4(v.cc, g.o, col[0], col[1]);
          rec4[r * 4 + 2] = make_float4(col[2], v.n[0], v.n[1], v.n[2]);
          rec4[r * 4 + 3] = make_float4(v.d, 1.f / g.o, hx, __log2f(g.o));
        }
      }
    }
    dkey[r] = __float_as_uint(key);
    rect[r] = rr;
    nact[r] = count;
  }
}

// ------------------------------------------------------------ backward

// Final value of one raw-parameter gradient: stored, and with Adam enabled
// also used to update that parameter and its moments in place.
template <bool ADAM>
__device__ __forceinline__ void put_grad(float *gp, const float *param, uint64_t idx, float g, const AdamArgs &A,
                                         float c1, float c2) {
  if constexpr (!ADAM) {
    gp[idx] = g;
    return;
  }
  if (A.write_grads) gp[idx] = g;
  float *pm = gp + A.m_off, *pv = gp + A.v_off;
  float *pp = const_cast<float *>(param);
  float m = pm[idx], v = pv[idx], p = pp[idx];
  m = A.b1 * m + (1.f - A.b1) * g;
  v = A.b2 * v + (1.f - A.b2) * g * g;
  p -= A.lr * (m * c1) / (sqrtf(v * c2) + A.eps);
  pm[idx] = m;
  pv[idx] = v;
  pp[idx] = p;
}

// The same for G parameters at idx + k * stride. With Adam, every
// parameter and moment of the group is loaded before any is stored: the
// stores may alias later loads as far as the compiler knows, so one
// parameter at a time would cost a memory round trip each.
template <bool ADAM, int G>
__device__ __forceinline__ void put_grads(float *gp, const float *param, uint64_t idx, uint64_t stride, const float *g,
                                          const AdamArgs &A, float c1, float c2) {
  if constexpr (!ADAM) {
#pragma unroll
    for (int k = 0; k < G; ++k) gp[idx + k * stride] = g[k];
    return;
  }
  float *pm = gp + A.m_off, *pv = gp + A.v_off;
  float *pp = const_cast<float *>(param);
  float m[G], v[G], p[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    m[k] = pm[idx + k * stride];
    v[k] = pv[idx + k * stride];
    p[k] = pp[idx + k * stride];
  }
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const uint64_t e = idx + k * stride;
    if (A.write_grads) gp[e] = g[k];
    m[k] = A.b1 * m[k] + (1.f - A.b1) * g[k];
    v[k] = A.b2 * v[k] + (1.f - A.b2) * g[k] * g[k];
    p[k] -= A.lr * (m[k] * c1) / (sqrtf(v[k] * c2) + A.eps);
    pm[e] = m[k];
    pv[e] = v[k];
    pp[e] = p[k];
  }
}

// With Adam folded in, degree 3 would take 184 VGPRs (2 waves per SIMD);
// 3 waves fit in 166 without spilling.
template <int D, bool ADAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) backward_preprocess_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                                  AdamArgs A) {
  constexpr int K = (D + 1) * (D + 1);
  const Header &h = *header(desc);
  const DevSet *Sp;
  int64_t i;
  if (!locate<D>(desc, Sp, i)) return;
  const DevSet &S = *Sp;
  const DevRender *rends = renders_of(desc);
  const int64_t n = S.n;
  Raw g;
  load_raw(S, i, g);
  const float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  const float4 *g2 = ws_ptr<float4>(ws, h.ws.g2);

  float gmean[3] = {0.f, 0.f, 0.f};
  float gs[3] = {0.f, 0.f, 0.f};     // dL/ds
  float gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // dL/dM (Gaussian rotation)
  float go = 0.f;
  float gsh[3 * K];
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) gsh[j] = 0.f;

  for (int vi = 0; vi < S.n_renders; ++vi) {
    const DevRender &rd = rends[S.renders[vi]];
    const DevCamera &c = rd.cam;
    const uint64_t r = rd.record_offset + (uint64_t)i;
    if (nact[r] == 0) continue;
    const float4 a0 = g2[r * 4 + 0], a1 = g2[r * 4 + 1], a2 = g2[r * 4 + 2], a3 = g2[r * 4 + 3];
    // the pixel sums of the compositing pass times the record's conic and
    // 1/o (as blended: the record's stored values)
    const float4 q0 = rec4[r * 4 + 0];
    const float inv_o = rec4[r * 4 + 3].y;
    const float d_mx = -2.f * (q0.z * a0.x + q0.w * a0.y);
    const float d_my = -2.f * (q0.w * a0.x + rec4[r * 4 + 1].x * a0.y);
    const float d_ca = a0.z, d_cb = 2.f * a0.w;
    const float d_cc = a1.x, d_o = a1.y * inv_o;
    const float d_col[3] = {a1.z, a1.w, a2.x};
    float d_n[3] = {a2.y, a2.z, a2.w};
    const float d_d = a3.x;

    View v;
    project_view(c, h, g, v);
    const float *R = c.R;
    float gt[3] = {0.f, 0.f, 0.f};  // dL/dt (camera-frame mean)

    // opacity
    go += d_o;

    // colour -> SH coefficients and view direction; the clamp at 0 is
    // read back from the stored (clamped) colour
    {
      float B[16];
      sh_basis(D, v.dir[0], v.dir[1], v.dir[2], B);
      const float4 c1 = rec4[r * 4 + 1], c2 = rec4[r * 4 + 2];
      const float dc[3] = {c1.z > 0.f ? d_col[0] : 0.f, c1.w > 0.f ? d_col[1] : 0.f,
                           c2.x > 0.f ? d_col[2] : 0.f};
      float w[16];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        w[j] = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          gsh[3 * j + k] += B[j] * dc[k];
          w[j] += dc[k] * S.sh[(3 * j + k) * n + i];
        }
      }
      float gx, gy, gz;
      sh_basis_grad(D, v.dir[0], v.dir[1], v.dir[2], w, gx, gy, gz);
      const float dd = gx * v.dir[0] + gy * v.dir[1] + gz * v.dir[2];
      const float il = 1.f / v.vlen;
      gmean[0] += (gx - dd * v.dir[0]) * il;
      gmean[1] += (gy - dd * v.dir[1]) * il;
      gmean[2] += (gz - dd * v.dir[2]) * il;
    }

    // plane distance d = n . t and normal n = sgn R_c M[:, j*]
    for (int k = 0; k < 3; ++k) {
      gt[k] += d_d * v.n[k];
      d_n[k] += d_d * (k == 0 ? v.tx : (k == 1 ? v.ty : v.tz));
    }
    {
      // dL/d(axis) = sgn R_c^T dL/dn
      const float ga0 = v.sgn * (R[0] * d_n[0] + R[3] * d_n[1] + R[6] * d_n[2]);
      const float ga1 = v.sgn * (R[1] * d_n[0] + R[4] * d_n[1] + R[7] * d_n[2]);
      const float ga2 = v.sgn * (R[2] * d_n[0] + R[5] * d_n[1] + R[8] * d_n[2]);
      const int j = g.jstar;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float sel = c == j ? 1.f : 0.f;
        gM[c] += sel * ga0;
        gM[3 + c] += sel * ga1;
        gM[6 + c] += sel * ga2;
      }
    }

    // 2D mean = (fx tx / tz + cx, fy ty / tz + cy)
    const float iz = 1.f / v.tz;
    gt[0] += d_mx * c.fx * iz;
    gt[1] += d_my * c.fy * iz;
    gt[2] += -(d_mx * c.fx * v.tx + d_my * c.fy * v.ty) * iz * iz;

    // conic = inverse(cov): dL/dcov = -K G K with G = [[ga, gb/2], [gb/2, gc]]
    const float Ka = v.ca, Kb = v.cb, Kc = v.cc;
    const float Ga = d_ca, Gb = 0.5f * d_cb, Gc = d_cc;
    // P = K G
    const float p00 = Ka * Ga + Kb * Gb, p01 = Ka * Gb + Kb * Gc;
    const float p10 = Kb * Ga + Kc * Gb, p11 = Kb * Gb + Kc * Gc;
    // H = -(P K)  (symmetric)
    const float H00 = -(p00 * Ka + p01 * Kb);
    const float H01 = -(p00 * Kb + p01 * Kc);
    const float H11 = -(p10 * Kb + p11 * Kc);
    // cov = U U^T + dil I: dL/dU = 2 H U
    float gU[6];
    for (int k = 0; k < 3; ++k) {
      gU[k] = 2.f * (H00 * v.U[k] + H01 * v.U[3 + k]);
      gU[3 + k] = 2.f * (H01 * v.U[k] + H11 * v.U[3 + k]);
    }
    // U = T A with A = M diag(s); dL/dT = gU A^T, dL/dA = T^T gU
    float gT[6];
    for (int rr = 0; rr < 2; ++rr)
      for (int k = 0; k < 3; ++k) {
        float acc = 0.f;
        for (int m = 0; m < 3; ++m) acc += gU[3 * rr + m] * g.M[3 * k + m] * g.s[m];
        gT[3 * rr + k] = acc;
      }
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m) {
        const float gA = v.T[k] * gU[m] + v.T[3 + k] * gU[3 + m];  // dL/dA_km
        gM[3 * k + m] += gA * g.s[m];
        gs[m] += gA * g.M[3 * k + m];
      }
    // T = J R_c, J = [[fx/tz, 0, -fx xt/tz^2], [0, fy/tz, -fy yt/tz^2]]
    float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
    for (int k = 0; k < 3; ++k) {
      gJ00 += gT[k] * R[k];
      gJ02 += gT[k] * R[6 + k];
      gJ11 += gT[3 + k] * R[3 + k];
      gJ12 += gT[3 + k] * R[6 + k];
    }
    const float iz2 = iz * iz, iz3 = iz2 * iz;
    gt[2] += -c.fx * iz2 * gJ00 + 2.f * c.fx * v.xt * iz3 * gJ02 - c.fy * iz2 * gJ11 +
             2.f * c.fy * v.yt * iz3 * gJ12;
    const float gxt = -c.fx * iz2 * gJ02;
    const float gyt = -c.fy * iz2 * gJ12;
    // xt = clamp(tx/tz) tz: d/dtx = 1 (free) or 0 (clamped); d/dtz = 0 or +-lim
    if (v.clx) gt[2] += gxt * (v.tx * iz > 0.f ? c.limx : -c.limx);
    else gt[0] += gxt;
    if (v.cly) gt[2] += gyt * (v.ty * iz > 0.f ? c.limy : -c.limy);
    else gt[1] += gyt;

    // t = R_c mean + t_c
    for (int k = 0; k < 3; ++k) gmean[k] += R[k] * gt[0] + R[3 + k] * gt[1] + R[6 + k] * gt[2];
  }

  float *gm = S.g_means, *gl = S.g_log_scales, *gq = S.g_quats, *go_ = S.g_logits, *gsh_ = S.g_sh;
  // A Gaussian seen by no view keeps every accumulator at zero, and the
  // expressions below then give exact zeros: all lanes share one store
  // sequence, so each gradient cache line is written once (a separate
  // zero-writing branch made every line of a mixed wave be written twice).
  const float c1 = ADAM ? A.coef[0] : 1.f, c2 = ADAM ? A.coef[1] : 1.f;
  if (gm) put_grads<ADAM, 3>(gm, S.means, i, n, gmean, A, c1, c2);
  if (gl) {
    const float v[3] = {gs[0] * g.s[0], gs[1] * g.s[1], gs[2] * g.s[2]};
    put_grads<ADAM, 3>(gl, S.log_scales, i, n, v, A, c1, c2);
  }
  if (gq) {
    float gw, gx, gy, gz;
    quat_rot_vjp(g.qw, g.qx, g.qy, g.qz, gM, gw, gx, gy, gz);
    // through q / |q|
    const float dot = gw * g.qw + gx * g.qx + gy * g.qy + gz * g.qz;
    const float inv = 1.f / g.qn;
    const float v[4] = {(gw - dot * g.qw) * inv, (gx - dot * g.qx) * inv, (gy - dot * g.qy) * inv,
                        (gz - dot * g.qz) * inv};
    put_grads<ADAM, 4>(gq, S.quats, i, n, v, A, c1, c2);
  }
  if (go_) put_grad<ADAM>(go_, S.logits, i, go * g.o * (1.f - g.o), A, c1, c2);
  if (gsh_) {
    constexpr int G = (3 * K) % 8 == 0 ? 8 : 3;
#pragma unroll
    for (int j = 0; j < 3 * K; j += G) put_grads<ADAM, G>(gsh_, S.sh, (uint64_t)j * n + i, n, gsh + j, A, c1, c2);
  }
}

}  // namespace

void launch_preprocess(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.deg_blocks[0]) hipLaunchKernelGGL(preprocess_kernel<0>, dim3(h.deg_blocks[0]), dim3(256), 0, s, d_desc, ws);
  if (h.deg_blocks[1]) hipLaunchKernelGGL(preprocess_kernel<1>, dim3(h.deg_blocks[1]), dim3(256), 0, s, d_desc, ws);
  if (h.deg_blocks[2]) hipLaunchKernelGGL(preprocess_kernel<2>, dim3(h.deg_blocks[2]), dim3(256), 0, s, d_desc, ws);
  if (h.deg_blocks[3]) hipLaunchKernelGGL(preprocess_kernel<3>, dim3(h.deg_blocks[3]), dim3(256), 0, s, d_desc, ws);
}

template <bool ADAM>
void launch_bwd_pre(const void *d_desc, const Header &h, void *ws, const AdamArgs &A, hipStream_t s) {
  if (h.deg_blocks[0])
    hipLaunchKernelGGL((backward_preprocess_kernel<0, ADAM>), dim3(h.deg_blocks[0]), dim3(256), 0, s, d_desc, ws, A);
  if (h.deg_blocks[1])
    hipLaunchKernelGGL((backward_preprocess_kernel<1, ADAM>), dim3(h.deg_blocks[1]), dim3(256), 0, s, d_desc, ws, A);
  if (h.deg_blocks[2])
    hipLaunchKernelGGL((backward_preprocess_kernel<2, ADAM>), dim3(h.deg_blocks[2]), dim3(256), 0, s, d_desc, ws, A);
  if (h.deg_blocks[3])
    hipLaunchKernelGGL((backward_preprocess_kernel<3, ADAM>), dim3(h.deg_blocks[3]), dim3(256), 0, s, d_desc, ws, A);
}

void launch_backward_preprocess(const void *d_desc, const Header &h, void *ws, const AdamArgs &A, hipStream_t s) {
  if (A.enabled)
    launch_bwd_pre<true>(d_desc, h, ws, A, s);
  else
    launch_bwd_pre<false>(d_desc, h, ws, A, s);
}

}  // namespace pgsag
