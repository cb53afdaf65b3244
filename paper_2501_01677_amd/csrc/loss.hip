// Training losses on the rendered outputs of a batch and their gradients
// with respect to the rendered rgb, normal and depth planes (Sec. 4.2 Eq. 8,
// Sec. 4.3 Eq. 9-11).  The gradients are written into each render's
// grad-output planes, so the backward pass consumes them directly.
//
// Per render, M = masked pixels:
//   L_rgb = (1 / 3M) sum over masked pixels and channels |rgb - gt|
//   L_ban = (1 / M) sum over masked pixels with both normals
//           w * || n_depth - N / |N| ||  (L1, or squared L2),
//           w = boundary weight on the mask boundary, 1 elsewhere
//   L     = (1 - lambda_load) (lambda_rgb L_rgb + lambda_normal L_ban)
//           + lambda_load L_load
//   L_load: load_term 0: Var(pairs per active tile)   (value only)
//           load_term 1: GC-load of Eq. 9, std over masked pixels of
//           x = n_contrib / w; its gradient goes to the soft count (the sum
//           of the blended alphas): dL/ds = lambda_load (x - mean) / (M std w)
// n_depth: pixels inside the mask with a positive depth are back-projected,
// P = depth K^-1 p~; dPx = P(u+1) - P(u-1) and dPy = P(v+1) - P(v-1), a
// neighbour that is not such a pixel being replaced by the pixel itself;
// n_depth = normalize(dPy x dPx) (faces the camera).  The mask boundary is
// the set of masked pixels with an unmasked 4-neighbour inside the image.
//
// Kernels, all bounded by HBM traffic (41 bytes read and 28 written per
// masked pixel):
//   loss_tiles   per render: masked-pixel count and the pair-count moments
//                over active tiles (from the forward's tile counts/ranges)
//   loss_pixels  16 x 16 pixel blocks staged with a 2-pixel halo in LDS:
//                depth normals and their gradients are formed once per cell
//                of the 18 x 18 ring, then every pixel gathers the depth
//                gradient from the up-to-five normals its point enters
//   loss_final   per render: sum of the block partials, the four loss values
//   gc_grad      per render, GC-load only: dL/d(soft count) at masked pixels
// plus the luminance weights of Eq. 9 (weights_grad, weights_final).
#include "internal.h"

namespace pgsag {
namespace {

constexpr int kLB = 16;                 // output block side
constexpr int kHalo = 2;
constexpr int kSX = kLB + 2 * kHalo;    // staged cells per side
constexpr int kGX = kLB + 2;            // cells whose normal gradients are formed
constexpr int kAcc = 8;                 // doubles per render
constexpr int kSlots = 64;              // partial-sum slots per render (blocks add into slot block % 64)

struct LossParams {
  float lambda_rgb, lambda_normal, boundary_weight, lambda_load, eps;
  int norm, load_term;
};
constexpr int kPart = 4;  // doubles per partial-sum slot: |rgb - gt|, w e, sum x, sum x^2

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum of one double per thread over a 256-thread block (valid in thread 0).
__device__ inline double block_sum_d(double x) {
  __shared__ double part[4];
  x = wave_sum_d(x);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  const double t = part[0] + part[1] + part[2] + part[3];
  __syncthreads();
  return t;
}

__global__ void fill_f64_kernel(double *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// acc[0] masked pixels, [1] active tiles, [2] sum of pair counts over active
// tiles, [3] sum of their squares.  grid (blocks, n_renders).
__global__ void __launch_bounds__(256) loss_tiles_kernel(const void *__restrict__ desc, const void *__restrict__ ws,
                                                         double *__restrict__ acc_all) {
  const Header &h = *header(desc);
  const int r = blockIdx.y;
  const DevRender &rd = renders_of(desc)[r];
  const uint64_t ntile = (uint64_t)rd.tiles_x * rd.tiles_y;
  const uint32_t *tc = ws_ptr<const uint32_t>(const_cast<void *>(ws), h.ws.tile_count) + rd.tile_offset;
  const uint2 *rg = ws_ptr<const uint2>(const_cast<void *>(ws), h.ws.ranges) + rd.tile_offset;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntile; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t c = tc[t];
    a0 += (double)c;
    if (c > 0) {
      const double k = (double)(rg[t].y - rg[t].x);
      a1 += 1.0;
      a2 += k;
      a3 += k * k;
    }
  }
  a0 = block_sum_d(a0);
  a1 = block_sum_d(a1);
  a2 = block_sum_d(a2);
  a3 = block_sum_d(a3);
  if (threadIdx.x == 0) {
    double *acc = acc_all + kAcc * r;
    atomicAdd(&acc[0], a0);
    atomicAdd(&acc[1], a1);
    atomicAdd(&acc[2], a2);
    atomicAdd(&acc[3], a3);
  }
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// Per block: partial sums of |rgb - gt| and of w e, added into one of the
// render's 64 partial-sum slots (block index mod 64: no address sees more
// than 1/64 of the blocks).  One block per 16 x 16 pixels.
__global__ void __launch_bounds__(256) loss_pixels_kernel(const void *__restrict__ desc, void *__restrict__ ws, int r,
                                                          const float *__restrict__ gt,
                                                          const float *__restrict__ weight, LossParams lp) {
  const Header &h = *header(desc);
  const DevRender &rd = renders_of(desc)[r];
  const int W = rd.cam.W, H = rd.cam.H;
  const int bpr = (W + kLB - 1) / kLB;
  const int x0 = (blockIdx.x % bpr) * kLB, y0 = (blockIdx.x / bpr) * kLB;
  const double *acc = ws_ptr<double>(ws, h.ws.loss) + kAcc * r;
  double *part = ws_ptr<double>(ws, h.ws.loss_part) + kPart * ((uint64_t)r * kSlots + blockIdx.x % kSlots);
  const uint64_t plane = (uint64_t)W * H;

  __shared__ float sP[3][kSX * kSX];
  __shared__ uint8_t sF[kSX * kSX];   // bit0 valid (masked, depth > 0), bit1 masked, bit2 inside the image
  __shared__ float sG[6][kGX * kGX];  // dL/d(dPx), dL/d(dPy)

  const float fx = rd.cam.fx, fy = rd.cam.fy, cx = rd.cam.cx, cy = rd.cam.cy;
  int any = 0;
  for (int k = threadIdx.x; k < kSX * kSX; k += 256) {
    const int u = x0 - kHalo + k % kSX, v = y0 - kHalo + k / kSX;
    uint32_t f = 0;
    float px = 0.f, py = 0.f, pz = 0.f;
    if (u >= 0 && u < W && v >= 0 && v < H) {
      f = 4;
      const uint64_t p = (uint64_t)v * W + u;
      // depth is read together with the mask (not after it), and used only
      // where the pixel is masked
      const float d = rd.o_depth[p];
      const bool m = rd.mask == nullptr || rd.mask[p];
      const float dm = m ? d : 0.f;
      if (m) f |= 2;
      if (dm > 0.f) {
        f |= 1;
        px = dm * (((float)u + 0.5f - cx) / fx);
        py = dm * (((float)v + 0.5f - cy) / fy);
        pz = dm;
      }
      const int iu = u - x0, iv = v - y0;
      if (m && iu >= 0 && iu < kLB && iv >= 0 && iv < kLB) any = 1;
    }
    sF[k] = (uint8_t)f;
    sP[0][k] = px;
    sP[1][k] = py;
    sP[2][k] = pz;
  }
  if (__syncthreads_or(any) == 0) return;  // no masked pixel in this block

  const double Md = acc[0];
  const float inv_m = Md > 0.0 ? (float)(1.0 / Md) : 0.f;
  const float kn = (1.f - lp.lambda_load) * lp.lambda_normal * inv_m;
  const float kr = (1.f - lp.lambda_load) * lp.lambda_rgb * inv_m * (1.f / 3.f);
  float e_sum = 0.f;

  // normal term on the 18 x 18 ring: values (inner cells), rendered-normal
  // gradients (inner cells) and dL/d(dPx), dL/d(dPy) (every cell).  A thread
  // covers at most two cells: both cells' rendered normals are loaded before
  // any gradient is stored, and the stores wait until after both.
  static_assert(kGX * kGX <= 2 * 256, "two cells per thread");
  float Nc[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int k = threadIdx.x + 256 * it;
    if (k < kGX * kGX) {
      const int gx = k % kGX, gy = k / kGX;
      if (sF[(gy + 1) * kSX + (gx + 1)] & 1) {
        const uint64_t p = (uint64_t)(y0 - 1 + gy) * W + (x0 - 1 + gx);
        Nc[it][0] = rd.o_normal[p];
        Nc[it][1] = rd.o_normal[plane + p];
        Nc[it][2] = rd.o_normal[2 * plane + p];
      }
    }
  }
  float gNs[2][3];
  uint64_t pst[2];
  bool st[2] = {false, false};
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int k = threadIdx.x + 256 * it;
    if (k >= kGX * kGX) break;
    const int gx = k % kGX, gy = k / kGX;
    const int s = (gy + 1) * kSX + (gx + 1);
    const int u = x0 - 1 + gx, v = y0 - 1 + gy;
    const bool inner = gx >= 1 && gx <= kLB && gy >= 1 && gy <= kLB;
    float G[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float gN[3] = {0.f, 0.f, 0.f};
    const uint32_t f = sF[s];
    if (f & 1) {
      const bool vxp = sF[s + 1] & 1, vxm = sF[s - 1] & 1, vyp = sF[s + kSX] & 1, vym = sF[s - kSX] & 1;
      if ((vxp || vxm) && (vyp || vym)) {
        float ax[3], ay[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float pc = sP[c][s];
          ax[c] = (vxp ? sP[c][s + 1] : pc) - (vxm ? sP[c][s - 1] : pc);
          ay[c] = (vyp ? sP[c][s + kSX] : pc) - (vym ? sP[c][s - kSX] : pc);
        }
        // c = dPy x dPx
        const float c0 = ay[1] * ax[2] - ay[2] * ax[1];
        const float c1 = ay[2] * ax[0] - ay[0] * ax[2];
        const float c2 = ay[0] * ax[1] - ay[1] * ax[0];
        const float cl2 = c0 * c0 + c1 * c1 + c2 * c2;
        const float N0 = Nc[it][0], N1 = Nc[it][1], N2 = Nc[it][2];
        const float nl = sqrtf(N0 * N0 + N1 * N1 + N2 * N2);
        if (cl2 > 0.f && nl > lp.eps) {
          const float il = 1.f / sqrtf(cl2), inl = 1.f / nl;
          const float nd[3] = {c0 * il, c1 * il, c2 * il};
          const float nr[3] = {N0 * inl, N1 * inl, N2 * inl};
          // mask boundary: an unmasked neighbour inside the image
          const auto unmasked = [&](int q) { return (sF[q] & 6) == 4; };
          const bool mb = unmasked(s + 1) || unmasked(s - 1) || unmasked(s + kSX) || unmasked(s - kSX);
          const float w = mb ? lp.boundary_weight : 1.f;
          float e = 0.f, g[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float df = nd[c] - nr[c];
            if (lp.norm == 1) {
              e += fabsf(df);
              g[c] = sgnf(df);
            } else {
              e += df * df;
              g[c] = 2.f * df;
            }
            g[c] *= w * kn;  // dL/d n_depth; dL/d n_rendered = -g
          }
          if (inner) {
            e_sum += w * e;
            const float dot = -(g[0] * nr[0] + g[1] * nr[1] + g[2] * nr[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) gN[c] = (-g[c] - nr[c] * dot) * inl;
          }
          // through n_depth = c / |c|, then c = dPy x dPx
          const float dn = g[0] * nd[0] + g[1] * nd[1] + g[2] * nd[2];
          const float gc[3] = {(g[0] - nd[0] * dn) * il, (g[1] - nd[1] * dn) * il, (g[2] - nd[2] * dn) * il};
          // dL/d(dPx) = gc x dPy ; dL/d(dPy) = dPx x gc
          G[0] = gc[1] * ay[2] - gc[2] * ay[1];
          G[1] = gc[2] * ay[0] - gc[0] * ay[2];
          G[2] = gc[0] * ay[1] - gc[1] * ay[0];
          G[3] = ax[1] * gc[2] - ax[2] * gc[1];
          G[4] = ax[2] * gc[0] - ax[0] * gc[2];
          G[5] = ax[0] * gc[1] - ax[1] * gc[0];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sG[c][k] = G[c];
    st[it] = inner && (f & 2);
    pst[it] = (uint64_t)v * W + u;
#pragma unroll
    for (int c = 0; c < 3; ++c) gNs[it][c] = gN[c];
  }
  {
    float *gn = const_cast<float *>(rd.g_normal);
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (st[it]) {
        gn[pst[it]] = gNs[it][0];
        gn[plane + pst[it]] = gNs[it][1];
        gn[2 * plane + pst[it]] = gNs[it][2];
      }
  }
  __syncthreads();

  // one pixel per thread: colour term, depth gradient, GC-load moments
  float r_sum = 0.f;
  double x_sum = 0.0, x_sq = 0.0;
  {
    const int iu = threadIdx.x % kLB, iv = threadIdx.x / kLB;
    const int u = x0 + iu, v = y0 + iv;
    const int s = (iv + kHalo) * kSX + (iu + kHalo);
    const uint32_t f = sF[s];
    if (f & 2) {
      const uint64_t p = (uint64_t)v * W + u;
      float *grgb = const_cast<float *>(rd.g_rgb);
      float orgb[3], trgb[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        orgb[c] = rd.o_rgb[c * plane + p];
        trgb[c] = gt[c * plane + p];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float df = orgb[c] - trgb[c];
        r_sum += fabsf(df);
        grgb[c * plane + p] = sgnf(df) * kr;
      }
      float gd = 0.f;
      if (f & 1) {
        const int g = (iv + 1) * kGX + (iu + 1);
        const float wxp = (sF[s + 1] & 1) ? 0.f : 1.f, wxm = (sF[s - 1] & 1) ? 0.f : 1.f;
        const float wyp = (sF[s + kSX] & 1) ? 0.f : 1.f, wym = (sF[s - kSX] & 1) ? 0.f : 1.f;
        float gP[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
          gP[c] = sG[c][g - 1] - sG[c][g + 1] + sG[3 + c][g - kGX] - sG[3 + c][g + kGX] +
                  (wxp - wxm) * sG[c][g] + (wyp - wym) * sG[3 + c][g];
        gd = gP[0] * (((float)u + 0.5f - cx) / fx) + gP[1] * (((float)v + 0.5f - cy) / fy) + gP[2];
      }
      const_cast<float *>(rd.g_depth)[p] = gd;
      if (rd.g_dist) const_cast<float *>(rd.g_dist)[p] = 0.f;
      if (rd.g_alpha) const_cast<float *>(rd.g_alpha)[p] = 0.f;
      if (lp.load_term == 1) {
        const float x = (float)rd.o_ncontrib[p] / (weight ? weight[p] : 1.f);
        x_sum = (double)x;
        x_sq = (double)x * (double)x;
      } else if (rd.g_count) {
        const_cast<float *>(rd.g_count)[p] = 0.f;  // the tile-variance term has no gradient
      }
    }
  }
  const double a = block_sum_d((double)r_sum);
  const double b = block_sum_d((double)e_sum);
  double c = 0.0, d = 0.0;
  if (lp.load_term == 1) {
    c = block_sum_d(x_sum);
    d = block_sum_d(x_sq);
  }
  if (threadIdx.x == 0) {
    atomicAdd(&part[0], a);
    atomicAdd(&part[1], b);
    if (lp.load_term == 1) {
      atomicAdd(&part[2], c);
      atomicAdd(&part[3], d);
    }
  }
}

// One wave per render: sum the render's partial-sum slots, then the four
// loss values; for the GC-load term also the mean of x and the factor
// lambda_load / (M std) of its gradient (acc[4], acc[5]).
__global__ void __launch_bounds__(64) loss_final_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                        LossParams lp, float *__restrict__ out) {
  const Header &h = *header(desc);
  const int r = blockIdx.x;
  const double *part = ws_ptr<const double>(ws, h.ws.loss_part) + kPart * (uint64_t)r * kSlots;
  const double s_rgb = wave_sum_d(part[kPart * threadIdx.x]);
  const double s_n = wave_sum_d(part[kPart * threadIdx.x + 1]);
  const double s_x = wave_sum_d(part[kPart * threadIdx.x + 2]);
  const double s_xx = wave_sum_d(part[kPart * threadIdx.x + 3]);
  if (threadIdx.x != 0) return;
  double *acc = ws_ptr<double>(ws, h.ws.loss) + kAcc * r;
  const double M = acc[0] > 0 ? acc[0] : 1.0;
  const double l_rgb = s_rgb / (3.0 * M), l_ban = s_n / M;
  double load;
  if (lp.load_term == 1) {
    const double mean = s_x / M;
    double var = s_xx / M - mean * mean;
    if (var < 0) var = 0;
    load = sqrt(var);
    acc[4] = mean;
    acc[5] = load > 0 && acc[0] > 0 ? (double)lp.lambda_load / (acc[0] * load) : 0.0;
  } else {
    const double nt = acc[1] > 0 ? acc[1] : 1.0;
    const double mean = acc[2] / nt;
    double var = acc[3] / nt - mean * mean;
    if (var < 0) var = 0;
    load = var;
  }
  const double geo = (double)lp.lambda_rgb * l_rgb + (double)lp.lambda_normal * l_ban;
  out[4 * r + 0] = (float)((1.0 - (double)lp.lambda_load) * geo + (double)lp.lambda_load * load);
  out[4 * r + 1] = (float)l_rgb;
  out[4 * r + 2] = (float)l_ban;
  out[4 * r + 3] = (float)load;
}

// GC-load gradient at the masked pixels of render r:
// dL/ds = lambda_load (x - mean) / (M std w), x = n_contrib / w.
__global__ void __launch_bounds__(256) gc_grad_kernel(const void *__restrict__ desc, const void *__restrict__ ws,
                                                      int r, const float *__restrict__ weight) {
  const Header &h = *header(desc);
  const DevRender &rd = renders_of(desc)[r];
  const uint64_t plane = (uint64_t)rd.cam.W * rd.cam.H;
  const double *acc = ws_ptr<const double>(ws, h.ws.loss) + kAcc * r;
  const float mean = (float)acc[4], k = (float)acc[5];
  float *gc = const_cast<float *>(rd.g_count);
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (uint64_t)gridDim.x * blockDim.x) {
    if (rd.mask != nullptr && rd.mask[p] == 0) continue;
    const float w = weight ? weight[p] : 1.f;
    const float x = (float)rd.o_ncontrib[p] / w;
    gc[p] = k * (x - mean) / w;
  }
}

// Eq. 9 weights.  Pass 1: |grad Y| per pixel (central differences inside,
// one-sided at the border) into weight[], and its sum and count over masked
// pixels into acc[6], acc[7].
__device__ __forceinline__ float lum(const float *g, uint64_t plane, uint64_t p) {
  return 0.299f * g[p] + 0.587f * g[plane + p] + 0.114f * g[2 * plane + p];
}

__global__ void __launch_bounds__(256) weights_grad_kernel(const void *__restrict__ desc, void *__restrict__ ws, int r,
                                                           const float *__restrict__ gt, float *__restrict__ weight) {
  const Header &h = *header(desc);
  const DevRender &rd = renders_of(desc)[r];
  const int W = rd.cam.W, H = rd.cam.H;
  const uint64_t plane = (uint64_t)W * H;
  double s = 0.0, n = 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (uint64_t)gridDim.x * blockDim.x) {
    const int u = (int)(p % W), v = (int)(p / W);
    float gx = 0.f, gy = 0.f;
    if (W > 1) {
      const int a = u + 1 < W ? u + 1 : u, b = u > 0 ? u - 1 : u;
      gx = (lum(gt, plane, p + (a - u)) - lum(gt, plane, p - (u - b))) / (float)(a - b);
    }
    if (H > 1) {
      const int a = v + 1 < H ? v + 1 : v, b = v > 0 ? v - 1 : v;
      gy = (lum(gt, plane, p + (uint64_t)(a - v) * W) - lum(gt, plane, p - (uint64_t)(v - b) * W)) / (float)(a - b);
    }
    const float mag = sqrtf(gx * gx + gy * gy);
    weight[p] = mag;
    if (rd.mask == nullptr || rd.mask[p]) {
      s += mag;
      n += 1.0;
    }
  }
  s = block_sum_d(s);
  n = block_sum_d(n);
  if (threadIdx.x == 0) {
    double *acc = ws_ptr<double>(ws, h.ws.loss) + kAcc * r;
    atomicAdd(&acc[6], s);
    atomicAdd(&acc[7], n);
  }
}

__global__ void __launch_bounds__(256) weights_final_kernel(const void *__restrict__ desc, const void *__restrict__ ws,
                                                            int r, float *__restrict__ weight) {
  const Header &h = *header(desc);
  const DevRender &rd = renders_of(desc)[r];
  const uint64_t plane = (uint64_t)rd.cam.W * rd.cam.H;
  const double *acc = ws_ptr<const double>(const_cast<void *>(ws), h.ws.loss) + kAcc * r;
  const double mean = acc[7] > 0 ? acc[6] / acc[7] : 0.0;
  const float im = mean > 0 ? (float)(1.0 / mean) : 0.f;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (uint64_t)gridDim.x * blockDim.x)
    weight[p] = mean > 0 ? 0.1f + weight[p] * im : 1.f;
}

LossParams params_of(const pgsag_loss_config &lc) {
  LossParams p;
  p.lambda_rgb = lc.lambda_rgb;
  p.lambda_normal = lc.lambda_normal;
  p.boundary_weight = lc.boundary_weight;
  p.lambda_load = lc.lambda_load;
  p.eps = lc.normal_eps;
  p.norm = lc.normal_norm;
  p.load_term = lc.load_term;
  return p;
}

unsigned grid_for(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (unsigned)(b < 512 ? (b ? b : 1) : 512);
}

}  // namespace

void launch_loss(const void *d_desc, const void *h_desc, void *ws, const pgsag_loss_config &lc,
                 const float *const *gt, const float *const *weight, float *out, hipStream_t s) {
  const Header &h = *header(h_desc);
  const DevRender *rd = renders_of(h_desc);
  double *acc = ws_ptr<double>(ws, h.ws.loss);
  // the accumulators and the partial sums (laid out one after the other)
  // cleared by one launch
  const int np = h.n_renders * kSlots * kPart;
  const int n = (int)((h.ws.loss_part - h.ws.loss) / sizeof(double)) + np;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, acc, n);
  uint64_t max_tiles = 1;
  for (int r = 0; r < h.n_renders; ++r) {
    const uint64_t t = (uint64_t)rd[r].tiles_x * rd[r].tiles_y;
    max_tiles = t > max_tiles ? t : max_tiles;
  }
  unsigned tb = (unsigned)((max_tiles + 255) / 256);
  tb = tb > 16 ? 16 : tb;
  hipLaunchKernelGGL(loss_tiles_kernel, dim3(tb, h.n_renders), dim3(256), 0, s, d_desc, (const void *)ws, acc);
  const LossParams lp = params_of(lc);
  for (int r = 0; r < h.n_renders; ++r) {
    const unsigned blocks = (unsigned)(((rd[r].cam.W + kLB - 1) / kLB) * ((rd[r].cam.H + kLB - 1) / kLB));
    if (blocks)
      hipLaunchKernelGGL(loss_pixels_kernel, dim3(blocks), dim3(256), 0, s, d_desc, ws, r, gt[r],
                         weight ? weight[r] : nullptr, lp);
  }
  hipLaunchKernelGGL(loss_final_kernel, dim3(h.n_renders), dim3(64), 0, s, d_desc, ws, lp, out);
  if (lc.load_term == 1)
    for (int r = 0; r < h.n_renders; ++r) {
      const uint64_t plane = (uint64_t)rd[r].cam.W * rd[r].cam.H;
      hipLaunchKernelGGL(gc_grad_kernel, dim3(grid_for(plane)), dim3(256), 0, s, d_desc, (const void *)ws, r,
                         weight ? weight[r] : nullptr);
    }
}

void launch_luminance_weights(const void *d_desc, const void *h_desc, void *ws, int r, const float *gt,
                              float *weight, hipStream_t s) {
  const Header &h = *header(h_desc);
  const DevRender &rd = renders_of(h_desc)[r];
  double *acc = ws_ptr<double>(ws, h.ws.loss) + kAcc * r;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, s, acc + 6, 2);
  const uint64_t plane = (uint64_t)rd.cam.W * rd.cam.H;
  hipLaunchKernelGGL(weights_grad_kernel, dim3(grid_for(plane)), dim3(256), 0, s, d_desc, ws, r, gt, weight);
  hipLaunchKernelGGL(weights_final_kernel, dim3(grid_for(plane)), dim3(256), 0, s, d_desc, (const void *)ws, r,
                     weight);
}

}  // namespace pgsag
