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
#include <cmath>
#include <mutex>

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


// ------------------------------------------------------------------------
// Building grouping: DBSCAN over the ground-plane coordinates (x, y) of the
// points that take part (Sec. 4.1, "Building Grouping").
//
// Neighbour search runs on a spatial hash: cells of side 1.01 eps (so two
// points within eps are in the same or adjacent cells), each cell hashed to
// one of H buckets (H a power of two >= 2n); the points are counting-sorted
// by bucket.  A point scans the buckets of its 3x3 cells, each bucket once
// (a bucket shared by two of those cells is skipped the second time):
// points of other cells in those buckets are more than eps away and fail the
// distance test, so every point within eps is counted exactly once.  The
// distance test is the FP32 rule d2 = dx*dx + dy*dy <= eps*eps with every
// operation rounded on its own.  Three passes walk the neighbours: counting
// (core flags), union-find over core-core pairs (a lock-free union that
// always hooks the larger root under the smaller, so a component's root is
// its smallest core index: the cluster's name), and border points (the
// smallest name among their core neighbours).  A scan of the roots gives
// compact cluster ids.

constexpr int kScanT = 256;
constexpr int kScanI = 16;
constexpr int kScanTile = kScanT * kScanI;  // 4096 elements per scan block

__device__ __forceinline__ uint32_t cell_hash(int cx, int cy) {
  return ((uint32_t)cx * 73856093u) ^ ((uint32_t)cy * 19349663u);
}

__device__ __forceinline__ void cell_of(float x, float y, double inv_side, int &cx, int &cy) {
  cx = (int)floor((double)x * inv_side);
  cy = (int)floor((double)y * inv_side);
}

__device__ __forceinline__ bool within(float px, float py, float qx, float qy, float e2) {
#pragma clang fp contract(off)
  const float dx = px - qx;
  const float dy = py - qy;
  const float d2 = dx * dx + dy * dy;
  return d2 <= e2;
}

// Exclusive scan of n uint32 values (n <= kScanTile * kScanTile) in three
// kernels: per-block scans with block totals, a scan of the totals in one
// block, and the add-back.  total (device) receives the sum.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[kScanT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kScanT / 64; ++k) {
    if (k < w) base += wsum[k];
    all += wsum[k];
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

__global__ void __launch_bounds__(kScanT) scan_blocks_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                             uint32_t *__restrict__ sums, uint32_t n) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanI;
  uint32_t v[kScanI];
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kScanI; ++k) {
    v[k] = b0 + k < n ? in[b0 + k] : 0u;
    t += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(t, &total);
#pragma unroll
  for (int k = 0; k < kScanI; ++k) {
    if (b0 + k < n) out[b0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanT) scan_sums_kernel(uint32_t *__restrict__ sums, uint32_t nb,
                                                           uint32_t *__restrict__ total_out) {
  uint32_t v[kScanI];
  uint32_t t = 0;
  const uint32_t b0 = threadIdx.x * kScanI;
#pragma unroll
  for (int k = 0; k < kScanI; ++k) {
    v[k] = b0 + k < nb ? sums[b0 + k] : 0u;
    t += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(t, &total);
#pragma unroll
  for (int k = 0; k < kScanI; ++k) {
    if (b0 + k < nb) sums[b0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) *total_out = total;
}

__global__ void __launch_bounds__(kScanT) scan_add_kernel(uint32_t *__restrict__ out, const uint32_t *__restrict__ sums,
                                                          uint32_t n) {
  const uint32_t add = sums[blockIdx.x];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanT)
    if (b0 + k < n) out[b0 + k] += add;
}

__global__ void fill_u32_kernel2(uint32_t *__restrict__ p, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

struct Dbs {
  const float *pts;
  int64_t n;
  const uint8_t *flags;
  uint32_t flag_mask;
  float e2;
  double inv_side;
  int32_t min_pts;
  uint32_t hmask;
  uint32_t *bcount, *bstart, *cursor, *pbucket, *sidx, *parent, *npart, *scan_sums;
  float2 *sxy;
  uint8_t *score;
  int32_t *count, *label, *cluster;
  uint32_t *n_clusters;
};

// Bucket of every taking-part point, bucket sizes; outputs initialised.
__global__ void __launch_bounds__(256) dbs_bucket_kernel(Dbs d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  const bool part = d.flags == nullptr || (d.flags[i] & d.flag_mask) != 0;
  uint32_t b = 0xffffffffu;
  if (part) {
    int cx, cy;
    cell_of(d.pts[i], d.pts[d.n + i], d.inv_side, cx, cy);
    b = cell_hash(cx, cy) & d.hmask;
    atomicAdd(&d.bcount[b], 1u);
  }
  d.pbucket[i] = b;
  d.parent[i] = (uint32_t)i;
  if (d.count) d.count[i] = 0;
  d.label[i] = -1;
  if (d.cluster) d.cluster[i] = -1;
}

__global__ void __launch_bounds__(256) dbs_scatter_kernel(Dbs d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  const uint32_t b = d.pbucket[i];
  if (b == 0xffffffffu) return;
  const uint32_t pos = atomicAdd(&d.cursor[b], 1u);
  d.sxy[pos] = make_float2(d.pts[i], d.pts[d.n + i]);
  d.sidx[pos] = (uint32_t)i;
}

// Visits every taking-part point q within eps of (px, py) (itself
// included), as sorted positions k: f(k).
template <typename F>
__device__ __forceinline__ void for_neighbours(const Dbs &d, float px, float py, F &&f) {
  int cx, cy;
  cell_of(px, py, d.inv_side, cx, cy);
  uint32_t seen[9];
  int ns = 0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const uint32_t b = cell_hash(cx + dx, cy + dy) & d.hmask;
      bool dup = false;
      for (int k = 0; k < ns; ++k) dup |= seen[k] == b;
      if (dup) continue;
      seen[ns++] = b;
      const uint32_t s0 = d.bstart[b], s1 = s0 + d.bcount[b];
      for (uint32_t k = s0; k < s1; ++k) {
        const float2 q = d.sxy[k];
        if (within(px, py, q.x, q.y, d.e2)) f(k);
      }
    }
  }
}

__global__ void __launch_bounds__(256) dbs_count_kernel(Dbs d) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= *d.npart) return;
  const float2 p = d.sxy[s];
  uint32_t c = 0;
  for_neighbours(d, p.x, p.y, [&](uint32_t) { ++c; });
  d.score[s] = c >= (uint32_t)d.min_pts ? 1 : 0;
  if (d.count) d.count[d.sidx[s]] = (int32_t)c;
}

__device__ __forceinline__ uint32_t uf_load(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t *parent, uint32_t x) {
  uint32_t p = uf_load(&parent[x]);
  while (p != x) {
    const uint32_t g = uf_load(&parent[p]);
    if (g != p) atomicMin(&parent[x], g);  // path halving; parents only decrease
    x = p;
    p = g;
  }
  return x;
}

__device__ __forceinline__ void uf_union(uint32_t *parent, uint32_t a, uint32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    // hook the larger root a under b, if a is still a root
    const uint32_t old = atomicCAS(&parent[a], a, b);
    if (old == a) return;
    a = old;
  }
}

__global__ void __launch_bounds__(256) dbs_union_kernel(Dbs d) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= *d.npart || !d.score[s]) return;
  const float2 p = d.sxy[s];
  const uint32_t i = d.sidx[s];
  for_neighbours(d, p.x, p.y, [&](uint32_t k) {
    if (!d.score[k]) return;
    const uint32_t j = d.sidx[k];
    if (j < i) uf_union(d.parent, i, j);
  });
}

// Core points: their root (the cluster's smallest core index).
__global__ void __launch_bounds__(256) dbs_root_kernel(Dbs d) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= *d.npart || !d.score[s]) return;
  const uint32_t i = d.sidx[s];
  d.label[i] = (int32_t)uf_find(d.parent, i);
}

// Border points: the smallest name among their core neighbours.
__global__ void __launch_bounds__(256) dbs_border_kernel(Dbs d) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= *d.npart || d.score[s]) return;
  const float2 p = d.sxy[s];
  int32_t best = 0x7fffffff;
  for_neighbours(d, p.x, p.y, [&](uint32_t k) {
    if (!d.score[k]) return;
    const int32_t l = d.label[d.sidx[k]];
    best = l < best ? l : best;
  });
  if (best != 0x7fffffff) d.label[d.sidx[s]] = best;
}

// root flags by point index (a core point that names its own cluster)
__global__ void __launch_bounds__(256) dbs_rootflag_kernel(Dbs d, uint32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  flag[i] = d.label[i] == (int32_t)i ? 1u : 0u;
}

__global__ void __launch_bounds__(256) dbs_cluster_kernel(Dbs d, const uint32_t *__restrict__ id) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  const int32_t l = d.label[i];
  d.cluster[i] = l >= 0 ? (int32_t)id[l] : -1;
}

// View hits per cluster: every labelled point, in bucket order (so a wave's
// points mostly share a cluster), projected into every view as in the
// voting filter; a wave adds its hits of one (cluster, view) with one atomic.
__global__ void __launch_bounds__(kVoteBlock)
    group_views_kernel(const pgsag_vote_view *__restrict__ views, int n_views, const float *__restrict__ pts,
                       int64_t n, const int32_t *__restrict__ cluster, int max_clusters, float z_near,
                       uint32_t *__restrict__ hits) {
  __shared__ float sv[kViewChunk][kViewFloats];
  __shared__ const uint8_t *smask[kViewChunk];
  __shared__ int sw[kViewChunk];
  const int64_t i = (int64_t)blockIdx.x * kVoteBlock + threadIdx.x;
  const int c = i < n ? cluster[i] : -1;
  const bool act = c >= 0 && c < max_clusters;
  const float x = act ? pts[i] : 0.f;
  const float y = act ? pts[n + i] : 0.f;
  const float z = act ? pts[2 * n + i] : 0.f;
  const int lane = threadIdx.x & 63;
  for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int cnt = n_views - v0 < kViewChunk ? n_views - v0 : kViewChunk;
    __syncthreads();
    for (int k = threadIdx.x; k < cnt * kViewFloats; k += kVoteBlock) {
      const int j = k / kViewFloats, f = k % kViewFloats;
      const pgsag_camera &cm = views[v0 + j].cam;
      float val;
      if (f < 9) val = cm.R[f];
      else if (f < 12) val = cm.t[f - 9];
      else if (f == 12) val = cm.fx;
      else if (f == 13) val = cm.fy;
      else if (f == 14) val = cm.cx;
      else if (f == 15) val = cm.cy;
      else if (f == 16) val = (float)cm.width;
      else val = (float)cm.height;
      sv[j][f] = val;
    }
    if ((int)threadIdx.x < cnt) {
      smask[threadIdx.x] = views[v0 + threadIdx.x].mask;
      sw[threadIdx.x] = views[v0 + threadIdx.x].cam.width;
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      bool hit = false;
      if (act) {
#pragma clang fp contract(off)
        const float *cv = sv[j];
        const float xc = ((cv[0] * x + cv[1] * y) + cv[2] * z) + cv[9];
        const float yc = ((cv[3] * x + cv[4] * y) + cv[5] * z) + cv[10];
        const float zc = ((cv[6] * x + cv[7] * y) + cv[8] * z) + cv[11];
        const float u = cv[12] * (xc / zc) + cv[14];
        const float v = cv[13] * (yc / zc) + cv[15];
        if (zc > z_near && u >= 0.f && u < cv[16] && v >= 0.f && v < cv[17]) {
          const uint8_t *m = smask[j];
          hit = m == nullptr || m[(uint64_t)(uint32_t)v * (uint32_t)sw[j] + (uint32_t)u] != 0;
        }
      }
      // one atomic per distinct cluster among the wave's hitting lanes
      uint64_t pending = __ballot(hit);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int cl = __shfl(c, leader, 64);
        const uint64_t same = __ballot(hit && c == cl);
        if (lane == leader) atomicAdd(&hits[(uint64_t)cl * n_views + v0 + j], (uint32_t)__popcll(same));
        pending &= ~same;
      }
    }
  }
}

__global__ void __launch_bounds__(256) group_assign_kernel(const uint32_t *__restrict__ hits, uint64_t n,
                                                           uint32_t min_hits, uint8_t *__restrict__ assigned) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    assigned[i] = hits[i] >= min_hits ? 1 : 0;
}


struct DbsLayout {
  uint64_t bcount, bstart, cursor, pbucket, sidx, parent, npart, sums, sxy, score, end;
  uint32_t H;
};

constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

constexpr DbsLayout dbs_layout(int64_t n) {
  DbsLayout L{};
  uint64_t H = 1024;
  while (H < 2 * (uint64_t)n) H <<= 1;
  L.H = (uint32_t)H;
  uint64_t o = 0;
  L.bcount = o; o = align256(o + 4 * H);
  L.bstart = o; o = align256(o + 4 * H);
  L.cursor = o; o = align256(o + 4 * H);
  L.pbucket = o; o = align256(o + 4 * (uint64_t)n);
  L.sidx = o; o = align256(o + 4 * (uint64_t)n);
  L.parent = o; o = align256(o + 4 * (uint64_t)n);
  L.npart = o; o = align256(o + 4);
  L.sums = o; o = align256(o + 4 * (uint64_t)kScanTile);
  L.sxy = o; o = align256(o + 8 * (uint64_t)n);
  L.score = o; o = align256(o + (uint64_t)n);
  L.end = o;
  return L;
}

unsigned blocks_of(uint64_t n, unsigned per = 256) { return (unsigned)((n + per - 1) / per); }

void launch_fill(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return;
  uint64_t b = (n + 255) / 256;
  hipLaunchKernelGGL(fill_u32_kernel2, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, v, n);
}

// exclusive scan in[0, n) -> out (may alias in), the total into *total
void launch_scan(const uint32_t *in, uint32_t *out, uint32_t *sums, uint32_t *total, uint64_t n, hipStream_t s) {
  const unsigned nb = blocks_of(n, kScanTile);
  if (nb) hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(kScanT), 0, s, in, out, sums, (uint32_t)n);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanT), 0, s, sums, nb, total);
  if (nb > 1) hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanT), 0, s, out, (const uint32_t *)sums, (uint32_t)n);
}

__global__ void copy_u32_kernel(const uint32_t *__restrict__ a, uint32_t *__restrict__ b, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

constexpr int64_t kDbsMaxPoints = int64_t(1) << 23;

// Runs the DBSCAN kernels on scratch memory ws of at least
// dbs_layout(n_points).end bytes (arguments already validated, n_points > 0).
int dbscan_run(const float *points, int64_t n_points, const uint8_t *flags, uint32_t flag_mask, float eps,
               int32_t min_pts, int32_t *count, int32_t *label, int32_t *cluster, uint32_t *n_clusters,
               char *ws, hipStream_t s) {
  const DbsLayout L = dbs_layout(n_points);
  Dbs d{};
  d.pts = points;
  d.n = n_points;
  d.flags = flags;
  d.flag_mask = flag_mask;
  d.e2 = eps * eps;
  d.inv_side = 1.0 / (1.01 * (double)eps);
  d.min_pts = min_pts;
  d.hmask = L.H - 1;
  d.bcount = reinterpret_cast<uint32_t *>(ws + L.bcount);
  d.bstart = reinterpret_cast<uint32_t *>(ws + L.bstart);
  d.cursor = reinterpret_cast<uint32_t *>(ws + L.cursor);
  d.pbucket = reinterpret_cast<uint32_t *>(ws + L.pbucket);
  d.sidx = reinterpret_cast<uint32_t *>(ws + L.sidx);
  d.parent = reinterpret_cast<uint32_t *>(ws + L.parent);
  d.npart = reinterpret_cast<uint32_t *>(ws + L.npart);
  d.scan_sums = reinterpret_cast<uint32_t *>(ws + L.sums);
  d.sxy = reinterpret_cast<float2 *>(ws + L.sxy);
  d.score = reinterpret_cast<uint8_t *>(ws + L.score);
  d.count = count;
  d.label = label;
  d.cluster = cluster;
  d.n_clusters = n_clusters;
  const unsigned pb = blocks_of((uint64_t)n_points);
  // every scratch word the kernels read is written first in this call
  // (the bucket counts by a fill kernel), so nothing carries over between
  // calls on the same scratch
  launch_fill(d.bcount, 0u, L.H, s);
  hipLaunchKernelGGL(dbs_bucket_kernel, dim3(pb), dim3(256), 0, s, d);
  launch_scan(d.bcount, d.bstart, d.scan_sums, d.npart, L.H, s);
  hipLaunchKernelGGL(copy_u32_kernel, dim3(4096), dim3(256), 0, s, (const uint32_t *)d.bstart, d.cursor, (uint64_t)L.H);
  hipLaunchKernelGGL(dbs_scatter_kernel, dim3(pb), dim3(256), 0, s, d);
  hipLaunchKernelGGL(dbs_count_kernel, dim3(pb), dim3(256), 0, s, d);
  hipLaunchKernelGGL(dbs_union_kernel, dim3(pb), dim3(256), 0, s, d);
  hipLaunchKernelGGL(dbs_root_kernel, dim3(pb), dim3(256), 0, s, d);
  hipLaunchKernelGGL(dbs_border_kernel, dim3(pb), dim3(256), 0, s, d);
  // compact ids: root flags (in the cursor buffer, free after the scatter),
  // scanned in place
  uint32_t *ids = d.cursor;
  hipLaunchKernelGGL(dbs_rootflag_kernel, dim3(pb), dim3(256), 0, s, d, ids);
  launch_scan(ids, ids, d.scan_sums, n_clusters, (uint64_t)n_points, s);
  if (cluster) hipLaunchKernelGGL(dbs_cluster_kernel, dim3(pb), dim3(256), 0, s, d, (const uint32_t *)ids);
  return hip_status("dbscan");
}

// Validation shared by both DBSCAN entry points (all but the scratch).
int dbscan_check(const float *points, int64_t n_points, int64_t max_points, float eps, int32_t min_pts,
                 const int32_t *label, const uint32_t *n_clusters) {
  if (n_points < 0 || n_points > max_points)
    return set_error(PGSAG_INVALID_ARGUMENT, "n_points must be in 0..%lld", (long long)max_points);
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(PGSAG_INVALID_ARGUMENT, "eps must be finite and > 0");
  if (min_pts < 1) return set_error(PGSAG_INVALID_ARGUMENT, "min_pts must be >= 1");
  if (!n_clusters) return set_error(PGSAG_INVALID_ARGUMENT, "null n_clusters");
  if (n_points > 0 && (!points || !label)) return set_error(PGSAG_INVALID_ARGUMENT, "null points or label");
  return PGSAG_OK;
}

// ---------------------------------------------------------------------
// Library-owned DBSCAN scratch for pgsag_dbscan_static: room for
// PGSAG_DBSCAN_STATIC_MAX_POINTS points.  Each GPU the library runs on
// holds its own copy of the array until the process ends.  In host code
// `scratch` names a host-side stand-in, never a device address: the device
// address is taken once per device with hipGetSymbolAddress (that device
// current) and kept in scratch_ptr.
constexpr uint64_t kStaticScratchBytes = dbs_layout(PGSAG_DBSCAN_STATIC_MAX_POINTS).end;
constexpr int kMaxDevices = 64;

}  // namespace
}  // namespace pgsag

static __device__ __align__(256) uint8_t scratch[pgsag::kStaticScratchBytes];

namespace pgsag {
namespace {

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (taken on its first use there).
int static_scratch(char **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(PGSAG_HIP_ERROR, "hipGetDevice: %s", hipGetErrorName(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(PGSAG_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(PGSAG_HIP_ERROR, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorName(e));
    scratch_ptr[dev] = p;
  }
  *out = static_cast<char *>(scratch_ptr[dev]);
  return PGSAG_OK;
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

int pgsag_dbscan_workspace(int64_t n_points, uint64_t *bytes) {
  if (!bytes) return set_error(PGSAG_INVALID_ARGUMENT, "null output");
  if (n_points < 0 || n_points > kDbsMaxPoints)
    return set_error(PGSAG_INVALID_ARGUMENT, "n_points must be in 0..%lld", (long long)kDbsMaxPoints);
  *bytes = dbs_layout(n_points).end;
  return PGSAG_OK;
}

int pgsag_dbscan(const float *points, int64_t n_points, const uint8_t *flags, uint32_t flag_mask, float eps,
                 int32_t min_pts, int32_t *count, int32_t *label, int32_t *cluster, uint32_t *n_clusters,
                 void *workspace, uint64_t workspace_bytes, void *stream) {
  const int rc = dbscan_check(points, n_points, kDbsMaxPoints, eps, min_pts, label, n_clusters);
  if (rc != PGSAG_OK) return rc;
  if (n_points > 0 && !workspace) return set_error(PGSAG_INVALID_ARGUMENT, "null workspace");
  const DbsLayout L = dbs_layout(n_points);
  if (n_points > 0 && workspace_bytes < L.end)
    return set_error(PGSAG_WORKSPACE_TOO_SMALL, "workspace needs %llu bytes", (unsigned long long)L.end);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_points == 0) {
    launch_fill(n_clusters, 0u, 1, s);
    return hip_status("dbscan");
  }
  return dbscan_run(points, n_points, flags, flag_mask, eps, min_pts, count, label, cluster, n_clusters,
                    static_cast<char *>(workspace), s);
}

int pgsag_dbscan_static(const float *points, int64_t n_points, const uint8_t *flags, uint32_t flag_mask, float eps,
                        int32_t min_pts, int32_t *count, int32_t *label, int32_t *cluster, uint32_t *n_clusters,
                        void *stream) {
  const int rc = dbscan_check(points, n_points, PGSAG_DBSCAN_STATIC_MAX_POINTS, eps, min_pts, label, n_clusters);
  if (rc != PGSAG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_points == 0) {
    launch_fill(n_clusters, 0u, 1, s);
    return hip_status("dbscan (static scratch)");
  }
  char *ws = nullptr;
  const int sc = static_scratch(&ws);
  if (sc != PGSAG_OK) return sc;
  return dbscan_run(points, n_points, flags, flag_mask, eps, min_pts, count, label, cluster, n_clusters, ws, s);
}

int pgsag_group_views(const pgsag_vote_view *host_views, const pgsag_vote_view *dev_views, int32_t n_views,
                      const float *points, int64_t n_points, const int32_t *cluster, int32_t max_clusters,
                      float z_near, uint32_t min_hits, uint32_t *hits, uint8_t *assigned, void *stream) {
  if (!host_views || !dev_views) return set_error(PGSAG_INVALID_ARGUMENT, "null view array");
  if (n_views < 1 || n_views > 65535) return set_error(PGSAG_INVALID_ARGUMENT, "n_views must be in 1..65535");
  if (n_points < 0) return set_error(PGSAG_INVALID_ARGUMENT, "n_points < 0");
  if (max_clusters < 0) return set_error(PGSAG_INVALID_ARGUMENT, "max_clusters < 0");
  if (!(z_near > 0.f)) return set_error(PGSAG_INVALID_ARGUMENT, "z_near must be > 0");
  if (max_clusters > 0 && !hits) return set_error(PGSAG_INVALID_ARGUMENT, "null hits");
  if (n_points > 0 && max_clusters > 0 && (!points || !cluster))
    return set_error(PGSAG_INVALID_ARGUMENT, "null points or cluster ids");
  for (int j = 0; j < n_views; ++j) {
    const pgsag_camera &c = host_views[j].cam;
    if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
      return set_error(PGSAG_INVALID_ARGUMENT, "view %d: image size must be 1..65535", j);
  }
  if (max_clusters == 0) return PGSAG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t nh = (uint64_t)max_clusters * (uint64_t)n_views;
  launch_fill(hits, 0u, nh, s);
  if (n_points > 0) {
    const int64_t blocks = (n_points + kVoteBlock - 1) / kVoteBlock;
    if (blocks > 0x7fffffff) return set_error(PGSAG_UNSUPPORTED, "too many points");
    hipLaunchKernelGGL(group_views_kernel, dim3((unsigned)blocks), dim3(kVoteBlock), 0, s, dev_views, (int)n_views,
                       points, n_points, cluster, (int)max_clusters, z_near, hits);
  }
  if (assigned) {
    const uint64_t b = (nh + 255) / 256;
    hipLaunchKernelGGL(group_assign_kernel, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s,
                       (const uint32_t *)hits, nh, min_hits, assigned);
  }
  return hip_status("group views");
}

}  // extern "C"
