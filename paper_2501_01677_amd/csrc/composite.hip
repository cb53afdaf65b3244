// Per-tile alpha compositing at building-mask pixels (Sec. 3.1, Eq. 1-4)
// and its backward pass.
//
// Shape: one workgroup per tile of T x T pixels, one lane per pixel (each
// pixel is a GPU thread, Sec. 4.3); a wave covers an 8 x 8 sub-block.  The
// tile's depth-ordered list of projected records is staged through LDS in
// batches of T*T records (one coalesced 64-byte record load per lane).
// Before touching a record a wave compares the record's support box with
// its 8 x 8 pixel block and skips it as a whole if they do not meet; lanes
// whose pixel is unmasked or whose transmittance has stopped idle, and the
// workgroup leaves the tile when no lane is alive (__syncthreads_count).
//
// The backward pass walks the same list back to front from the tile's
// largest last-blended index, recovering each pixel's transmittance before a
// fragment as T_i = T_{i+1} / (1 - alpha_i) from the saved final T, keeps the
// suffix sums of the blended features, and reduces the 13 per-fragment 2D
// gradients across the wave before one float atomic per value per wave.
//
// In persistent mode a grid of (CUs x occupancy) workgroups pulls chunks of
// tiles from an LPT-ordered queue with an atomic counter; every workgroup
// leaves once the counter passes the end of the queue.
#include "internal.h"

namespace pgsag {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

// Records staged per LDS batch: one per lane, at most 512 (32 KB).
template <int T>
constexpr int batch_of() { return T * T < 512 ? T * T : 512; }

// alpha of a record at pixel centre (px, py); the same instruction sequence
// is used by the forward and backward kernels so they take identical
// skip decisions.
__device__ __forceinline__ float eval_alpha(float px, float py, const float4 &r0, float cc, float o,
                                            float amax, float &dx, float &dy, float &G, float &raw) {
#pragma clang fp contract(off)
  dx = px - r0.x;
  dy = py - r0.y;
  const float dxy = dx * dy;
  const float dxx = dx * dx;
  const float dyy = dy * dy;
  const float b2 = 2.f * r0.w;
  const float cross = b2 * dxy;
  const float q = __builtin_fmaf(cc, dyy, __builtin_fmaf(r0.z, dxx, cross));
  const float arg = (-0.5f * kLog2e) * q;
  G = __builtin_amdgcn_exp2f(arg);
  raw = o * G;
  return fminf(amax, raw);
}

__device__ __forceinline__ bool wave_culls(const float4 &r0, const float4 &r3, float wx0, float wx1, float wy0,
                                           float wy1) {
  return (r0.x + r3.y < wx0) || (r0.x - r3.y > wx1) || (r0.y + r3.z < wy0) || (r0.y - r3.z > wy1);
}

struct TileGeom {
  const DevRender *rd;
  int px, py;       // pixel of this lane
  bool inside;
  float wx0, wx1, wy0, wy1;  // pixel-centre box of this lane's wave
};

template <int T>
__device__ __forceinline__ void tile_geom(const void *desc, const Header &h, uint32_t tile, TileGeom &g) {
  const int r = upper_index(tile_starts_of(desc), h.n_renders, tile);
  const DevRender &rd = renders_of(desc)[r];
  g.rd = &rd;
  const uint32_t local = tile - rd.tile_offset;
  const int tx = (int)(local % (uint32_t)rd.tiles_x), ty = (int)(local / (uint32_t)rd.tiles_x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int SB = T / 8;  // 8x8 sub-blocks per tile side
  const int sbx = wave % SB, sby = wave / SB;
  const int bx = tx * T + sbx * 8, by = ty * T + sby * 8;
  g.px = bx + (lane & 7);
  g.py = by + (lane >> 3);
  g.inside = g.px < rd.cam.W && g.py < rd.cam.H;
  g.wx0 = bx + 0.5f;
  g.wx1 = bx + 7.5f;
  g.wy0 = by + 0.5f;
  g.wy1 = by + 7.5f;
}

template <int T>
__device__ void forward_tile(const void *__restrict__ desc, const Header &h, void *__restrict__ ws, uint32_t tile,
                             float4 (*srec)[4], const uint32_t *__restrict__ vals) {
  constexpr int NT = batch_of<T>();
  TileGeom g;
  tile_geom<T>(desc, h, tile, g);
  const DevRender &rd = *g.rd;
  const int W = rd.cam.W;
  const uint64_t pix = (uint64_t)g.py * W + g.px;
  const bool masked = g.inside && (rd.mask == nullptr || rd.mask[pix] != 0);
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[tile];
  const float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  const float amin = h.cfg.alpha_min, amax = h.cfg.alpha_max, tmin = h.cfg.t_min;
  const float fx = g.px + 0.5f, fy = g.py + 0.5f;
  bool done = !masked;
  float Tr = 1.f;
  float F[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int32_t n = 0, last = -1;
  for (uint32_t b = rg.x; b < rg.y; b += NT) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t j = b + threadIdx.x;
    if (threadIdx.x < NT && j < rg.y) {
      const uint64_t rid = vals[j];
      const float4 *src = rec4 + rid * 4;
      srec[threadIdx.x][0] = src[0];
      srec[threadIdx.x][1] = src[1];
      srec[threadIdx.x][2] = src[2];
      srec[threadIdx.x][3] = src[3];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, rg.y - b);
    if (__ballot(!done) != 0ull) {
      for (int k = 0; k < cnt; ++k) {
        const float4 r0 = srec[k][0];
        const float4 r3 = srec[k][3];
        if (wave_culls(r0, r3, g.wx0, g.wx1, g.wy0, g.wy1)) continue;
        if (!done) {
          const float4 r1 = srec[k][1];
          float dx, dy, G, raw;
          const float a = eval_alpha(fx, fy, r0, r1.x, r1.y, amax, dx, dy, G, raw);
          if (a >= amin) {
            const float Tn = Tr * (1.f - a);
            if (Tn < tmin) {
              done = true;
            } else {
              const float4 r2 = srec[k][2];
              const float w = a * Tr;
              F[0] = fmaf(w, r1.z, F[0]);
              F[1] = fmaf(w, r1.w, F[1]);
              F[2] = fmaf(w, r2.x, F[2]);
              F[3] = fmaf(w, r2.y, F[3]);
              F[4] = fmaf(w, r2.z, F[4]);
              F[5] = fmaf(w, r2.w, F[5]);
              F[6] = fmaf(w, r3.x, F[6]);
              Tr = Tn;
              ++n;
              last = (int32_t)(b + k);
            }
          }
        }
        if ((k & 7) == 7 && __ballot(!done) == 0ull) break;
      }
    }
  }
  if (!g.inside) return;
  const uint64_t HW = (uint64_t)rd.cam.H * W;
  float rgb0 = 0.f, rgb1 = 0.f, rgb2 = 0.f, alpha = 0.f, depth = 0.f;
  if (masked) {
    rgb0 = F[0] + Tr * h.cfg.bg[0];
    rgb1 = F[1] + Tr * h.cfg.bg[1];
    rgb2 = F[2] + Tr * h.cfg.bg[2];
    alpha = 1.f - Tr;
    const float rx = (fx - rd.cam.cx) / rd.cam.fx, ry = (fy - rd.cam.cy) / rd.cam.fy;
    const float den = F[3] * rx + F[4] * ry + F[5];
    depth = den < -h.cfg.depth_guard ? F[6] / den : 0.f;
  } else {
    for (int c = 0; c < 7; ++c) F[c] = 0.f;
  }
  if (rd.o_rgb) {
    rd.o_rgb[pix] = rgb0;
    rd.o_rgb[HW + pix] = rgb1;
    rd.o_rgb[2 * HW + pix] = rgb2;
  }
  if (rd.o_normal) {
    rd.o_normal[pix] = F[3];
    rd.o_normal[HW + pix] = F[4];
    rd.o_normal[2 * HW + pix] = F[5];
  }
  if (rd.o_dist) rd.o_dist[pix] = F[6];
  if (rd.o_depth) rd.o_depth[pix] = depth;
  if (rd.o_alpha) rd.o_alpha[pix] = alpha;
  if (rd.o_ncontrib) rd.o_ncontrib[pix] = masked ? n : 0;
  ws_ptr<float>(ws, h.ws.pix_T)[rd.pixel_offset + pix] = Tr;
  ws_ptr<int32_t>(ws, h.ws.pix_last)[rd.pixel_offset + pix] = masked ? last : -1;
}

// Sum of v[0..15] over the 64 lanes of a wave by recursive halving: after
// the call lane L holds the total of value (L >> 2) & 15.
__device__ __forceinline__ float wave_reduce16(float v[16]) {
  const int lane = threadIdx.x & 63;
  float w8[8], w4[4], w2[2];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float mine = hi ? v[8 + s] : v[s];
      const float send = hi ? v[s] : v[8 + s];
      w8[s] = mine + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float mine = hi ? w8[4 + s] : w8[s];
      const float send = hi ? w8[s] : w8[4 + s];
      w4[s] = mine + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float mine = hi ? w4[2 + s] : w4[s];
      const float send = hi ? w4[s] : w4[2 + s];
      w2[s] = mine + __shfl_xor(send, 8, 64);
    }
  }
  const bool hi = lane & 4;
  float x = (hi ? w2[1] : w2[0]) + __shfl_xor(hi ? w2[0] : w2[1], 4, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  return x;
}

template <int T>
__device__ void backward_tile(const void *__restrict__ desc, const Header &h, void *__restrict__ ws, uint32_t tile,
                              float4 (*srec)[4], uint32_t *sid, int *smax, const uint32_t *__restrict__ vals) {
  constexpr int NT = batch_of<T>();
  TileGeom g;
  tile_geom<T>(desc, h, tile, g);
  const DevRender &rd = *g.rd;
  const int W = rd.cam.W;
  const uint64_t pix = (uint64_t)g.py * W + g.px;
  const uint64_t HW = (uint64_t)rd.cam.H * W;
  const bool masked = g.inside && (rd.mask == nullptr || rd.mask[pix] != 0);
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[tile];
  const float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  float *g2 = ws_ptr<float>(ws, h.ws.g2);
  const float amin = h.cfg.alpha_min, amax = h.cfg.alpha_max;
  const float fx = g.px + 0.5f, fy = g.py + 0.5f;

  int32_t last = -1;
  float Tr = 1.f, Tf = 1.f;
  float gch[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float ga = 0.f;
  float S[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (masked) {
    last = ws_ptr<int32_t>(ws, h.ws.pix_last)[rd.pixel_offset + pix];
    Tf = ws_ptr<float>(ws, h.ws.pix_T)[rd.pixel_offset + pix];
    Tr = Tf;
    if (rd.g_rgb) {
      gch[0] = rd.g_rgb[pix];
      gch[1] = rd.g_rgb[HW + pix];
      gch[2] = rd.g_rgb[2 * HW + pix];
    }
    if (rd.g_normal) {
      gch[3] = rd.g_normal[pix];
      gch[4] = rd.g_normal[HW + pix];
      gch[5] = rd.g_normal[2 * HW + pix];
    }
    if (rd.g_dist) gch[6] = rd.g_dist[pix];
    if (rd.g_alpha) ga = rd.g_alpha[pix];
    if (rd.g_depth) {
      // depth = D / (N . r): fold its gradient into D and N
      const float gd = rd.g_depth[pix];
      const float N0 = rd.o_normal[pix], N1 = rd.o_normal[HW + pix], N2 = rd.o_normal[2 * HW + pix];
      const float D = rd.o_dist[pix];
      const float rx = (fx - rd.cam.cx) / rd.cam.fx, ry = (fy - rd.cam.cy) / rd.cam.fy;
      const float den = N0 * rx + N1 * ry + N2;
      if (den < -h.cfg.depth_guard) {
        const float iden = 1.f / den;
        gch[6] += gd * iden;
        const float k = -gd * D * iden * iden;
        gch[3] += k * rx;
        gch[4] += k * ry;
        gch[5] += k;
      }
    }
    S[0] = h.cfg.bg[0] * Tf;
    S[1] = h.cfg.bg[1] * Tf;
    S[2] = h.cfg.bg[2] * Tf;
  }
  if (threadIdx.x == 0) *smax = -1;
  __syncthreads();
  if (last >= 0) atomicMax(smax, last);
  __syncthreads();
  const int maxlast = *smax;
  if (maxlast < (int)rg.x) return;  // uniform: no pixel blended anything
  const uint32_t end = (uint32_t)maxlast + 1;
  const int lane = threadIdx.x & 63;
  for (int64_t bend = end; bend > (int64_t)rg.x; bend -= NT) {
    const uint32_t bstart = (uint32_t)max((int64_t)rg.x, bend - NT);
    __syncthreads();
    const uint32_t j = bstart + threadIdx.x;
    if (threadIdx.x < NT && j < (uint32_t)bend) {
      const uint32_t rid = vals[j];
      const float4 *src = rec4 + (uint64_t)rid * 4;
      srec[threadIdx.x][0] = src[0];
      srec[threadIdx.x][1] = src[1];
      srec[threadIdx.x][2] = src[2];
      srec[threadIdx.x][3] = src[3];
      sid[threadIdx.x] = rid;
    }
    __syncthreads();
    const int cnt = (int)((uint32_t)bend - bstart);
    if (__ballot(last >= (int32_t)bstart) == 0ull) continue;
    for (int k = cnt - 1; k >= 0; --k) {
      const float4 r0 = srec[k][0];
      const float4 r3 = srec[k][3];
      if (wave_culls(r0, r3, g.wx0, g.wx1, g.wy0, g.wy1)) continue;
      const int32_t idx = (int32_t)(bstart + k);
      float v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = 0.f;
      bool contrib = false;
      if (idx <= last) {
        const float4 r1 = srec[k][1];
        float dx, dy, G, raw;
        const float a = eval_alpha(fx, fy, r0, r1.x, r1.y, amax, dx, dy, G, raw);
        if (a >= amin) {
          contrib = true;
          const float4 r2 = srec[k][2];
          const float f[7] = {r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
          const float om = 1.f - a;
          const float iom = 1.f / om;
          const float Tp = Tr * iom;
          const float w = a * Tp;
          float dLda = ga * Tf * iom;
#pragma unroll
          for (int c = 0; c < 7; ++c) {
            dLda += gch[c] * (Tp * f[c] - S[c] * iom);
            v[6 + c] = w * gch[c];
            S[c] = fmaf(w, f[c], S[c]);
          }
          Tr = Tp;
          if (raw <= amax) {
            v[G_O] = dLda * G;
            const float dLdq = -0.5f * a * dLda;
            v[G_MX] = -2.f * dLdq * (r0.z * dx + r0.w * dy);
            v[G_MY] = -2.f * dLdq * (r0.w * dx + r1.x * dy);
            v[G_CA] = dLdq * dx * dx;
            v[G_CB] = 2.f * dLdq * dx * dy;
            v[G_CC] = dLdq * dy * dy;
          }
        }
      }
      if (__ballot(contrib) == 0ull) continue;
      const float tot = wave_reduce16(v);
      const int which = (lane >> 2) & 15;
      if ((lane & 3) == 0 && which < 13) unsafeAtomicAdd(g2 + (uint64_t)sid[k] * kG2 + which, tot);
    }
  }
}

template <int T>
__global__ void __launch_bounds__(T *T) forward_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                        const uint32_t *__restrict__ vals) {
  __shared__ float4 srec[batch_of<T>()][4];
  __shared__ uint32_t s_item;
  const Header &h = *header(desc);
  if (!h.cfg.persistent) {
    forward_tile<T>(desc, h, ws, blockIdx.x, srec, vals);
    return;
  }
  uint32_t *ctr = ws_ptr<uint32_t>(ws, h.ws.status) + S_QUEUE_FWD;
  const uint32_t *queue = ws_ptr<uint32_t>(ws, h.ws.queue);
  const uint32_t chunk = (uint32_t)h.cfg.queue_chunk;
  const uint32_t ntiles = (uint32_t)h.n_tiles;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(ctr, chunk);
    __syncthreads();
    const uint32_t base = s_item;
    if (base >= ntiles) break;
    const uint32_t stop = min(ntiles, base + chunk);
    for (uint32_t it = base; it < stop; ++it) {
      __syncthreads();
      forward_tile<T>(desc, h, ws, queue[it], srec, vals);
    }
  }
}

template <int T>
__global__ void __launch_bounds__(T *T) backward_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                         const uint32_t *__restrict__ vals) {
  __shared__ float4 srec[batch_of<T>()][4];
  __shared__ uint32_t sid[batch_of<T>()];
  __shared__ int smax;
  __shared__ uint32_t s_item;
  const Header &h = *header(desc);
  if (!h.cfg.persistent) {
    backward_tile<T>(desc, h, ws, blockIdx.x, srec, sid, &smax, vals);
    return;
  }
  uint32_t *ctr = ws_ptr<uint32_t>(ws, h.ws.status) + S_QUEUE_BWD;
  const uint32_t *queue = ws_ptr<uint32_t>(ws, h.ws.queue);
  const uint32_t chunk = (uint32_t)h.cfg.queue_chunk;
  const uint32_t ntiles = (uint32_t)h.n_tiles;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(ctr, chunk);
    __syncthreads();
    const uint32_t base = s_item;
    if (base >= ntiles) break;
    const uint32_t stop = min(ntiles, base + chunk);
    for (uint32_t it = base; it < stop; ++it) {
      __syncthreads();
      backward_tile<T>(desc, h, ws, queue[it], srec, sid, &smax, vals);
    }
  }
}

unsigned persistent_grid(const Header &h) {
  uint64_t g = 256ull * (uint64_t)h.cfg.workgroups_per_cu;
  return (unsigned)(g < h.n_tiles ? g : (h.n_tiles ? h.n_tiles : 1));
}

template <int T>
void launch_fwd_t(const void *d, const Header &h, void *ws, hipStream_t s) {
  const uint32_t *vals = ws_ptr<uint32_t>(ws, h.ws.sorted_val);
  const unsigned grid = h.cfg.persistent ? persistent_grid(h) : (unsigned)h.n_tiles;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(forward_kernel<T>), dim3(grid), dim3(T * T), 0, s, d, ws, vals);
}

template <int T>
void launch_bwd_t(const void *d, const Header &h, void *ws, hipStream_t s) {
  const uint32_t *vals = ws_ptr<uint32_t>(ws, h.ws.sorted_val);
  const unsigned grid = h.cfg.persistent ? persistent_grid(h) : (unsigned)h.n_tiles;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(backward_kernel<T>), dim3(grid), dim3(T * T), 0, s, d, ws, vals);
}

}  // namespace

void launch_composite(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_tiles == 0) return;
  switch (h.cfg.tile) {
    case 8: launch_fwd_t<8>(d_desc, h, ws, s); break;
    case 16: launch_fwd_t<16>(d_desc, h, ws, s); break;
    default: launch_fwd_t<32>(d_desc, h, ws, s); break;
  }
}

void launch_backward_composite(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_tiles == 0) return;
  switch (h.cfg.tile) {
    case 8: launch_bwd_t<8>(d_desc, h, ws, s); break;
    case 16: launch_bwd_t<16>(d_desc, h, ws, s); break;
    default: launch_bwd_t<32>(d_desc, h, ws, s); break;
  }
}

}  // namespace pgsag
