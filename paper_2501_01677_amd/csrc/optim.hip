// Fused Adam update and the balance-load statistics of a rendered batch.
//
// Adam (the paper names no optimiser; 3DGS-family training uses Adam):
// one pass reads p, g, m, v and writes p, m, v -- 28 bytes per parameter,
// vectorised to 16-byte accesses when every pointer is 16-byte aligned.
//
// Balance-load statistics (Sec. 4.3, Eq. 9): per render, the mean and
// population variance of the per-tile pair counts over tiles holding masked
// pixels, and the mean and population standard deviation over masked pixels
// of g_i / w_i, g_i the number of Gaussians blended at pixel i (n_contrib).
#include "internal.h"

namespace pgsag {
namespace {

__device__ __forceinline__ void adam1(float &p, float g, float &m, float &v, float lr, float b1, float b2,
                                      float eps, float c1, float c2) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  p -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Bias corrections 1/(1 - b^t) either as arguments or, for the device-step
// form, from the two floats the coefficient kernel wrote.
__device__ __forceinline__ void corrections(const float *coef, float &c1, float &c2) {
  if (coef) {
    c1 = coef[0];
    c2 = coef[1];
  }
}

__global__ void __launch_bounds__(256) adam_vec_kernel(float4 *__restrict__ p, const float4 *__restrict__ g,
                                                       float4 *__restrict__ m, float4 *__restrict__ v, int64_t n4,
                                                       float lr, float b1, float b2, float eps, float c1, float c2,
                                                       const float *__restrict__ coef) {
  corrections(coef, c1, c2);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n4; i += stride) {
    float4 pp = p[i], gg = g[i], mm = m[i], vv = v[i];
    adam1(pp.x, gg.x, mm.x, vv.x, lr, b1, b2, eps, c1, c2);
    adam1(pp.y, gg.y, mm.y, vv.y, lr, b1, b2, eps, c1, c2);
    adam1(pp.z, gg.z, mm.z, vv.z, lr, b1, b2, eps, c1, c2);
    adam1(pp.w, gg.w, mm.w, vv.w, lr, b1, b2, eps, c1, c2);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

__global__ void __launch_bounds__(256) adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, int64_t lo,
                                                   int64_t n, float lr, float b1, float b2, float eps, float c1,
                                                   float c2, const float *__restrict__ coef) {
  corrections(coef, c1, c2);
  int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float pp = p[i], mm = m[i], vv = v[i];
    adam1(pp, g[i], mm, vv, lr, b1, b2, eps, c1, c2);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

// Device step counter: state[0] += 1, then the bias corrections of that
// step into state[1], state[2] (as floats), computed in double.
__global__ void adam_coef_kernel(int32_t *__restrict__ state, float b1, float b2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int32_t t = state[0] + 1;
  state[0] = t;
  float *coef = reinterpret_cast<float *>(state + 1);
  coef[0] = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
  coef[1] = (float)(1.0 / (1.0 - pow((double)b2, (double)t)));
}

// Sums over one render: [0] active tiles, [1] sum of counts, [2] sum of
// squared counts, [3] masked pixels, [4] sum of g/w, [5] sum of (g/w)^2.
__global__ void __launch_bounds__(256) load_sums_kernel(const void *__restrict__ desc, const void *__restrict__ ws,
                                                        int r, const float *__restrict__ weight,
                                                        double *__restrict__ sums) {
  const Header &h = *header(desc);
  const DevRender &rd = renders_of(desc)[r];
  const uint64_t ntile = (uint64_t)rd.tiles_x * rd.tiles_y;
  const uint64_t npix = (uint64_t)rd.cam.W * rd.cam.H;
  const uint32_t *tc = ws_ptr<uint32_t>(ws, h.ws.tile_count) + rd.tile_offset;
  const uint2 *rg = ws_ptr<uint2>(ws, h.ws.ranges) + rd.tile_offset;
  double a[6] = {0, 0, 0, 0, 0, 0};
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntile; t += stride) {
    if (tc[t] > 0) {
      const double c = (double)(rg[t].y - rg[t].x);
      a[0] += 1.0;
      a[1] += c;
      a[2] += c * c;
    }
  }
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
    const bool m = rd.mask == nullptr || rd.mask[p] != 0;
    if (m) {
      const double w = weight ? (double)weight[p] : 1.0;
      const double x = (double)rd.o_ncontrib[p] / w;
      a[3] += 1.0;
      a[4] += x;
      a[5] += x * x;
    }
  }
  __shared__ double part[6][4];
  for (int k = 0; k < 6; ++k) {
    double x = a[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) part[k][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 6) atomicAdd(&sums[threadIdx.x], part[threadIdx.x][0] + part[threadIdx.x][1] +
                                                        part[threadIdx.x][2] + part[threadIdx.x][3]);
}

__global__ void load_final_kernel(const double *__restrict__ sums, float *__restrict__ out) {
  if (threadIdx.x != 0) return;
  const double nt = sums[0] > 0 ? sums[0] : 1.0;
  const double mt = sums[1] / nt;
  const double vt = sums[2] / nt - mt * mt;
  const double np = sums[3] > 0 ? sums[3] : 1.0;
  const double mp = sums[4] / np;
  const double vp = sums[5] / np - mp * mp;
  out[0] = (float)mt;
  out[1] = (float)(vt > 0 ? vt : 0.0);
  out[2] = (float)mp;
  out[3] = (float)sqrt(vp > 0 ? vp : 0.0);
}

__global__ void zero_f64_kernel(double *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

}  // namespace

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t step, int32_t *state, hipStream_t s) {
  const float *coef = nullptr;
  if (state) {
    hipLaunchKernelGGL(adam_coef_kernel, dim3(1), dim3(64), 0, s, state, b1, b2);
    coef = reinterpret_cast<const float *>(state + 1);
  }
  if (n <= 0) return;
  const double c1 = state ? 1.0 : 1.0 / (1.0 - pow((double)b1, (double)step));
  const double c2 = state ? 1.0 : 1.0 / (1.0 - pow((double)b2, (double)step));
  const bool aligned = (((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) & 15u) == 0;
  int64_t done = 0;
  if (aligned && n >= 4) {
    const int64_t n4 = n / 4;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(adam_vec_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (float4 *)p, (const float4 *)g,
                       (float4 *)m, (float4 *)v, n4, lr, b1, b2, eps, (float)c1, (float)c2, coef);
    done = n4 * 4;
  }
  if (done < n) {
    int64_t blocks = (n - done + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, done, n, lr, b1, b2, eps,
                       (float)c1, (float)c2, coef);
  }
}

void launch_adam_coef(int32_t *state, float b1, float b2, hipStream_t s) {
  hipLaunchKernelGGL(adam_coef_kernel, dim3(1), dim3(64), 0, s, state, b1, b2);
}

void launch_load_stats(const void *d_desc, const Header &h, const void *ws, int r, const float *pixel_weight,
                       float *out, hipStream_t s) {
  double *sums = reinterpret_cast<double *>(static_cast<char *>(const_cast<void *>(ws)) + h.ws.stats) + 8 * r;
  hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, s, sums, 8);
  hipLaunchKernelGGL(load_sums_kernel, dim3(256), dim3(256), 0, s, d_desc, ws, r, pixel_weight, sums);
  hipLaunchKernelGGL(load_final_kernel, dim3(1), dim3(64), 0, s, sums, out + 4 * r);
}

}  // namespace pgsag
