// Building-point voting over many masked views (Sec. 4.1, "Reliability-scored
// Multi-view Voting Filter", Eq. 6-7): every SfM sparse point is projected
// into every view; it scores a vote where it lands on a coarse building-mask
// pixel (Eq. 6) and an unreliability count where it lands inside the image
// but off the mask (Eq. 7).  Reliable = at least one vote and fewer than tau
// unreliable sightings.
//
// One thread per point, the views in the inner loop: a workgroup stages up
// to 64 views' cameras in LDS, every thread loads its point once (planar
// x, y, z: coalesced) and gathers one mask byte per view it lands in.  The
// gathers dominate: the kernel is bound by how many distinct mask lines a
// wave's points touch, not by the 12 + 5 bytes per point it streams.
//
// The projection decides integers (inside or not, which pixel), so it is
// taken in FP32 with one fixed operation order and no contraction: every
// multiply, add and the (correctly rounded) division rounds on its own.
#include "internal.h"

namespace pgsag {
namespace {

constexpr int kVoteBlock = 256;
constexpr int kViewChunk = 64;
constexpr int kViewFloats = 18;  // R 9, t 3, fx fy cx cy, W, H (as floats)

__global__ void __launch_bounds__(kVoteBlock)
    vote_kernel(const pgsag_vote_view *__restrict__ views, int n_views, const float *__restrict__ pts, int64_t n,
                float z_near, int tau, uint16_t *__restrict__ votes, uint16_t *__restrict__ us,
                uint8_t *__restrict__ flags) {
  __shared__ float sv[kViewChunk][kViewFloats];
  __shared__ const uint8_t *smask[kViewChunk];
  __shared__ int sw[kViewChunk];
  const int64_t i = (int64_t)blockIdx.x * kVoteBlock + threadIdx.x;
  const bool valid = i < n;
  const float x = valid ? pts[i] : 0.f;
  const float y = valid ? pts[n + i] : 0.f;
  const float z = valid ? pts[2 * n + i] : 0.f;
  uint32_t nv = 0, nu = 0;
  for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int cnt = n_views - v0 < kViewChunk ? n_views - v0 : kViewChunk;
    __syncthreads();
    for (int k = threadIdx.x; k < cnt * kViewFloats; k += kVoteBlock) {
      const int j = k / kViewFloats, f = k % kViewFloats;
      const pgsag_camera &c = views[v0 + j].cam;
      float val;
      if (f < 9) val = c.R[f];
      else if (f < 12) val = c.t[f - 9];
      else if (f == 12) val = c.fx;
      else if (f == 13) val = c.fy;
      else if (f == 14) val = c.cx;
      else if (f == 15) val = c.cy;
      else if (f == 16) val = (float)c.width;
      else val = (float)c.height;
      sv[j][f] = val;
    }
    if ((int)threadIdx.x < cnt) {
      smask[threadIdx.x] = views[v0 + threadIdx.x].mask;
      sw[threadIdx.x] = views[v0 + threadIdx.x].cam.width;
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < cnt; ++j) {
#pragma clang fp contract(off)
      const float *c = sv[j];
      const float xc = ((c[0] * x + c[1] * y) + c[2] * z) + c[9];
      const float yc = ((c[3] * x + c[4] * y) + c[5] * z) + c[10];
      const float zc = ((c[6] * x + c[7] * y) + c[8] * z) + c[11];
      const float u = c[12] * (xc / zc) + c[14];
      const float v = c[13] * (yc / zc) + c[15];
      const bool inside = zc > z_near && u >= 0.f && u < c[16] && v >= 0.f && v < c[17];
      if (inside) {
        const uint8_t *m = smask[j];
        const bool hit = m == nullptr || m[(uint64_t)(uint32_t)v * (uint32_t)sw[j] + (uint32_t)u] != 0;
        nv += hit ? 1u : 0u;
        nu += hit ? 0u : 1u;
      }
    }
  }
  if (!valid) return;
  if (votes) votes[i] = (uint16_t)nv;
  if (us) us[i] = (uint16_t)nu;
  const uint8_t potential = nv > 0 ? 1 : 0;
  const uint8_t reliable = (potential && nu < (uint32_t)tau) ? 2 : 0;
  flags[i] = potential | reliable;
}

}  // namespace
}  // namespace pgsag

using namespace pgsag;

extern "C" {

int pgsag_vote(const pgsag_vote_view *host_views, const pgsag_vote_view *dev_views, int32_t n_views,
               const float *points, int64_t n_points, float z_near, int32_t tau, uint16_t *votes, uint16_t *us,
               uint8_t *flags, void *stream) {
  if (!host_views || !dev_views) return set_error(PGSAG_INVALID_ARGUMENT, "null view array");
  if (n_views < 1 || n_views > 65535) return set_error(PGSAG_INVALID_ARGUMENT, "n_views must be in 1..65535");
  if (n_points < 0) return set_error(PGSAG_INVALID_ARGUMENT, "n_points < 0");
  if (n_points > 0 && (!points || !flags)) return set_error(PGSAG_INVALID_ARGUMENT, "null points or flags");
  if (!(z_near > 0.f)) return set_error(PGSAG_INVALID_ARGUMENT, "z_near must be > 0");
  if (tau < 0) return set_error(PGSAG_INVALID_ARGUMENT, "tau must be >= 0");
  for (int j = 0; j < n_views; ++j) {
    const pgsag_camera &c = host_views[j].cam;
    if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
      return set_error(PGSAG_INVALID_ARGUMENT, "view %d: image size must be 1..65535", j);
  }
  if (n_points == 0) return PGSAG_OK;
  const int64_t blocks = (n_points + kVoteBlock - 1) / kVoteBlock;
  if (blocks > 0x7fffffff) return set_error(PGSAG_UNSUPPORTED, "too many points");
  hipLaunchKernelGGL(vote_kernel, dim3((unsigned)blocks), dim3(kVoteBlock), 0, static_cast<hipStream_t>(stream),
                     dev_views, (int)n_views, points, n_points, z_near, (int)tau, votes, us, flags);
  return hip_status("vote");
}

}  // extern "C"
