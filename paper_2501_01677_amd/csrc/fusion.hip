// Depth fusion and TSDF volume integration (Sec. 4.4, "Mesh Extraction and
// Merge"): the depth maps that several groups render from one view are
// merged by their mean where they overlap, and the fused maps of many views
// are integrated into a truncated signed distance volume (the running
// average of projective signed distances with unit weights).
//
// fuse_kernel:  elementwise over the pixels of one view, 4 pixels per thread
//               (16-byte loads and stores when the planes allow): bound by
//               HBM traffic, K x 4 bytes read and 4 (+1) written per pixel.
// tsdf_kernel:  one thread per voxel, x fastest (coalesced stores), the
//               views' cameras staged in LDS and looped over inside; per
//               (voxel, view) an FP32 projection in the fixed operation
//               order, one depth gather and the truncated update.  The
//               correctly rounded divisions of the projection make it
//               bound by ALU issue rather than by its 8 (or 16) bytes per
//               voxel.
#include <cmath>

#include "internal.h"

namespace pgsag {
namespace {

constexpr int kMaxMaps = 64;

struct MapList {
  const float *p[kMaxMaps];
};

__global__ void __launch_bounds__(256) fuse_kernel(MapList maps, int k, uint64_t n, float *__restrict__ fused,
                                                   uint8_t *__restrict__ count, int vec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (vec) {
    const uint64_t n4 = n / 4;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
      float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
      uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
      for (int m = 0; m < k; ++m) {
        const float4 d = reinterpret_cast<const float4 *>(maps.p[m])[q];
        if (d.x > 0.f) { s.x += d.x; ++c0; }
        if (d.y > 0.f) { s.y += d.y; ++c1; }
        if (d.z > 0.f) { s.z += d.z; ++c2; }
        if (d.w > 0.f) { s.w += d.w; ++c3; }
      }
      float4 o;
      o.x = c0 ? s.x / (float)c0 : 0.f;
      o.y = c1 ? s.y / (float)c1 : 0.f;
      o.z = c2 ? s.z / (float)c2 : 0.f;
      o.w = c3 ? s.w / (float)c3 : 0.f;
      reinterpret_cast<float4 *>(fused)[q] = o;
      if (count) {
        const uint32_t packed = c0 | (c1 << 8) | (c2 << 16) | (c3 << 24);
        reinterpret_cast<uint32_t *>(count)[q] = packed;
      }
    }
    for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
      float s = 0.f;
      uint32_t c = 0;
      for (int m = 0; m < k; ++m) {
        const float d = maps.p[m][i];
        if (d > 0.f) { s += d; ++c; }
      }
      fused[i] = c ? s / (float)c : 0.f;
      if (count) count[i] = (uint8_t)c;
    }
    return;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float s = 0.f;
    uint32_t c = 0;
    for (int m = 0; m < k; ++m) {
      const float d = maps.p[m][i];
      if (d > 0.f) { s += d; ++c; }
    }
    fused[i] = c ? s / (float)c : 0.f;
    if (count) count[i] = (uint8_t)c;
  }
}

constexpr int kTsdfBlock = 256;
constexpr int kViewChunk = 32;
constexpr int kViewFloats = 18;  // R 9, t 3, fx fy cx cy, W, H (as floats)

__global__ void __launch_bounds__(kTsdfBlock)
    tsdf_kernel(pgsag_volume vol, const pgsag_depth_view *__restrict__ views, int n_views, float z_near,
                float *__restrict__ tsdf, float *__restrict__ weight, int accumulate) {
  __shared__ float sv[kViewChunk][kViewFloats];
  __shared__ const float *sdep[kViewChunk];
  __shared__ int sw[kViewChunk];
  const uint64_t nxy = (uint64_t)vol.nx * vol.ny;
  const uint64_t nvox = nxy * vol.nz;
  const uint64_t idx = (uint64_t)blockIdx.x * kTsdfBlock + threadIdx.x;
  const bool valid = idx < nvox;
  float x, y, z;
  {
#pragma clang fp contract(off)
    const uint64_t k = idx / nxy, r = idx % nxy;
    const uint32_t j = (uint32_t)(r / vol.nx), i = (uint32_t)(r % vol.nx);
    x = ((float)i + 0.5f) * vol.voxel + vol.origin[0];
    y = ((float)j + 0.5f) * vol.voxel + vol.origin[1];
    z = ((float)k + 0.5f) * vol.voxel + vol.origin[2];
  }
  const float tr = vol.trunc;
  float sum = 0.f;
  uint32_t cnt = 0;
  for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int nv = n_views - v0 < kViewChunk ? n_views - v0 : kViewChunk;
    __syncthreads();
    for (int q = threadIdx.x; q < nv * kViewFloats; q += kTsdfBlock) {
      const int jv = q / kViewFloats, f = q % kViewFloats;
      const pgsag_camera &c = views[v0 + jv].cam;
      float val;
      if (f < 9) val = c.R[f];
      else if (f < 12) val = c.t[f - 9];
      else if (f == 12) val = c.fx;
      else if (f == 13) val = c.fy;
      else if (f == 14) val = c.cx;
      else if (f == 15) val = c.cy;
      else if (f == 16) val = (float)c.width;
      else val = (float)c.height;
      sv[jv][f] = val;
    }
    if ((int)threadIdx.x < nv) {
      sdep[threadIdx.x] = views[v0 + threadIdx.x].depth;
      sw[threadIdx.x] = views[v0 + threadIdx.x].cam.width;
    }
    __syncthreads();
    if (!valid) continue;
    for (int jv = 0; jv < nv; ++jv) {
#pragma clang fp contract(off)
      const float *c = sv[jv];
      const float xc = ((c[0] * x + c[1] * y) + c[2] * z) + c[9];
      const float yc = ((c[3] * x + c[4] * y) + c[5] * z) + c[10];
      const float zc = ((c[6] * x + c[7] * y) + c[8] * z) + c[11];
      const float u = c[12] * (xc / zc) + c[14];
      const float v = c[13] * (yc / zc) + c[15];
      if (zc > z_near && u >= 0.f && u < c[16] && v >= 0.f && v < c[17]) {
        const float d = sdep[jv][(uint64_t)(uint32_t)v * (uint32_t)sw[jv] + (uint32_t)u];
        const float sdf = d - zc;
        if (d > 0.f && sdf >= -tr) {
          const float t = sdf / tr;
          sum += t < 1.f ? t : 1.f;
          ++cnt;
        }
      }
    }
  }
  if (!valid) return;
  if (accumulate) {
    if (cnt == 0) return;  // no view saw the voxel: it keeps its values
    const float w0 = weight[idx];
    const float t0 = tsdf[idx];
    const float w1 = w0 + (float)cnt;
    tsdf[idx] = w1 > 0.f ? (w0 * t0 + sum) / w1 : 1.f;
    weight[idx] = w1;
  } else {
    tsdf[idx] = cnt ? sum / (float)cnt : 1.f;
    weight[idx] = (float)cnt;
  }
}

}  // namespace
}  // namespace pgsag

using namespace pgsag;

extern "C" {

int pgsag_fuse_depth(const float *const *depths, int32_t n_maps, int32_t width, int32_t height, float *fused,
                     uint8_t *count, void *stream) {
  if (!depths) return set_error(PGSAG_INVALID_ARGUMENT, "null depth-map array");
  if (n_maps < 1 || n_maps > kMaxMaps) return set_error(PGSAG_INVALID_ARGUMENT, "n_maps must be in 1..%d", kMaxMaps);
  if (width < 0 || height < 0) return set_error(PGSAG_INVALID_ARGUMENT, "negative image size");
  const uint64_t n = (uint64_t)width * (uint64_t)height;
  if (n == 0) return PGSAG_OK;
  if (!fused) return set_error(PGSAG_INVALID_ARGUMENT, "null fused output");
  MapList ml{};
  uintptr_t align = (uintptr_t)fused | (count ? (uintptr_t)count : 0);
  for (int m = 0; m < n_maps; ++m) {
    if (!depths[m]) return set_error(PGSAG_INVALID_ARGUMENT, "depth map %d is null", m);
    ml.p[m] = depths[m];
    align |= (uintptr_t)depths[m];
  }
  const int vec = (align & 15u) == 0 ? 1 : 0;
  uint64_t blocks = ((vec ? n / 4 : n) + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fuse_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), ml,
                     (int)n_maps, n, fused, count, vec);
  return hip_status("fuse depth");
}

int pgsag_tsdf_integrate(const pgsag_volume *vol, const pgsag_depth_view *host_views,
                         const pgsag_depth_view *dev_views, int32_t n_views, float z_near, float *tsdf,
                         float *weight, int32_t accumulate, void *stream) {
  if (!vol) return set_error(PGSAG_INVALID_ARGUMENT, "null volume");
  if (vol->nx < 0 || vol->ny < 0 || vol->nz < 0) return set_error(PGSAG_INVALID_ARGUMENT, "negative volume size");
  if (!(vol->voxel > 0.f) || !std::isfinite(vol->voxel)) return set_error(PGSAG_INVALID_ARGUMENT, "voxel must be > 0");
  if (!(vol->trunc > 0.f) || !std::isfinite(vol->trunc)) return set_error(PGSAG_INVALID_ARGUMENT, "trunc must be > 0");
  if (vol->nx > (1 << 23) || vol->ny > (1 << 23) || vol->nz > (1 << 23))
    return set_error(PGSAG_INVALID_ARGUMENT, "volume sides must be at most 2^23 voxels");
  if (n_views < 0 || n_views > 65535) return set_error(PGSAG_INVALID_ARGUMENT, "n_views must be in 0..65535");
  if (n_views > 0 && (!host_views || !dev_views)) return set_error(PGSAG_INVALID_ARGUMENT, "null view array");
  if (!(z_near > 0.f)) return set_error(PGSAG_INVALID_ARGUMENT, "z_near must be > 0");
  if (accumulate != 0 && accumulate != 1) return set_error(PGSAG_INVALID_ARGUMENT, "accumulate must be 0 or 1");
  for (int j = 0; j < n_views; ++j) {
    const pgsag_camera &c = host_views[j].cam;
    if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
      return set_error(PGSAG_INVALID_ARGUMENT, "view %d: image size must be 1..65535", j);
    if (!host_views[j].depth) return set_error(PGSAG_INVALID_ARGUMENT, "view %d: null depth map", j);
  }
  const uint64_t nvox = (uint64_t)vol->nx * vol->ny * vol->nz;
  if (nvox == 0) return PGSAG_OK;
  if (!tsdf || !weight) return set_error(PGSAG_INVALID_ARGUMENT, "null tsdf or weight");
  const uint64_t blocks = (nvox + kTsdfBlock - 1) / kTsdfBlock;
  if (blocks > 0x7fffffffull) return set_error(PGSAG_UNSUPPORTED, "volume too large");
  hipLaunchKernelGGL(tsdf_kernel, dim3((unsigned)blocks), dim3(kTsdfBlock), 0, static_cast<hipStream_t>(stream), *vol,
                     dev_views, (int)n_views, z_near, tsdf, weight, (int)accumulate);
  return hip_status("tsdf integrate");
}

}  // extern "C"
