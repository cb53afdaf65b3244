// Tile binning (Sec. 3.1: projected Gaussians are assigned to image tiles
// and sorted), restricted to tiles that hold building-mask pixels.
//
// Pipeline (all counts stay on the device; grids are sized from host bounds
// and blocks past the device count exit or contribute nothing):
//   tile_mask     masked pixels per tile and, per tile row, the prefix count
//                 of active tiles (one workgroup per tile row), so a support
//                 rectangle's active-tile count is two loads per tile row
//   compact       stable compaction of records with >= 1 active tile into
//                 (depth key, record) lists
//   radix sort    stable LSD sort of that list by the FP32 depth key
//   pair scan     exclusive scan of active-tile counts in depth order
//   emit          (global tile, record) pairs, depth order preserved
//   radix sort    stable LSD sort of the pairs by tile id -> every tile's list
//                 is in (depth, record) order
//   ranges        per tile [start, end) into the sorted pairs
//   queue         tiles ordered by decreasing list length (LPT) in buckets of
//                 log2(length), tiles without masked pixels last
#include "internal.h"

namespace pgsag {
namespace {

__device__ inline uint32_t *status_of(void *ws, const Header &h) {
  return ws_ptr<uint32_t>(ws, h.ws.status);
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

// -------------------------------------------------------------- scans

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread across a 256-thread block; returns
// the exclusive prefix and writes the block total to *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t s = wsum[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// ------------------------------------------------------------ tile mask

// Non-zero bytes of a 32-bit word.
__device__ inline uint32_t nonzero_bytes(uint32_t w) {
  uint32_t t = (w | (w >> 4)) & 0x0f0f0f0fu;
  t |= t >> 2;
  t = (t | (t >> 1)) & 0x01010101u;
  return __popc(t);
}

// Non-zero bytes of m[x0, x1).
__device__ inline uint32_t count_span(const uint8_t *m, int x0, int x1) {
  uint32_t c = 0;
  int x = x0;
  while (x < x1 && ((uintptr_t)(m + x) & 3u)) c += m[x++] != 0;
  for (; x + 4 <= x1; x += 4) c += nonzero_bytes(*reinterpret_cast<const uint32_t *>(m + x));
  while (x < x1) c += m[x++] != 0;
  return c;
}

// One workgroup per global tile row: masked (or, without a mask, in-image)
// pixels of every tile of the row, and the row prefix of active flags
// rowsat[ty][x] = number of active tiles among tiles 0..x-1 of row ty.
__global__ void __launch_bounds__(256) tile_mask_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t row = blockIdx.x;
  const int r = upper_index(row_starts_of(desc), h.n_renders, row);
  const DevRender &rd = renders_of(desc)[r];
  const int ty = (int)(row - row_starts_of(desc)[r]);
  const int tile = h.cfg.tile;
  const int W = rd.cam.W, H = rd.cam.H;
  const int tx_n = rd.tiles_x;
  __shared__ uint32_t cnt[65536 / 8 + 1];  // tiles_x <= 8192 for W <= 65535, tile >= 8
  for (int x = threadIdx.x; x < tx_n; x += blockDim.x) cnt[x] = 0;
  __syncthreads();
  const int y0 = ty * tile, y1 = min(H, y0 + tile);
  const int rows = y1 - y0;
  if (rd.mask == nullptr) {
    for (int x = threadIdx.x; x < tx_n; x += blockDim.x)
      cnt[x] = (uint32_t)((min(W, (x + 1) * tile) - x * tile) * rows);
  } else {
    // one work item per (tile, pixel row): count a tile-wide span
    for (int it = threadIdx.x; it < tx_n * rows; it += blockDim.x) {
      const int x = it % tx_n, y = y0 + it / tx_n;
      const int a = x * tile, b = min(W, a + tile);
      const uint32_t c = count_span(rd.mask + (uint64_t)y * W, a, b);
      if (c) atomicAdd(&cnt[x], c);
    }
  }
  __syncthreads();
  uint32_t *tc = ws_ptr<uint32_t>(ws, h.ws.tile_count) + rd.tile_offset + (uint64_t)ty * tx_n;
  uint32_t *rs = ws_ptr<uint32_t>(ws, h.ws.sat) + rd.sat_offset + (uint64_t)ty * (tx_n + 1);
  if (threadIdx.x == 0) rs[0] = 0;
  uint32_t running = 0;
  for (int base = 0; base < tx_n; base += blockDim.x) {
    const int x = base + threadIdx.x;
    uint32_t v = 0;
    if (x < tx_n) {
      tc[x] = cnt[x];
      v = cnt[x] > 0 ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, &tot);
    if (x < tx_n) rs[x + 1] = running + ex + v;
    running += tot;
  }
}

// Active tiles inside caller-provided rects (binning-only entry point).
__global__ void recount_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint64_t rec = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rec >= h.n_records) return;
  const int r = upper_index(rec_starts_of(desc), h.n_renders, rec);
  const DevRender &rd = renders_of(desc)[r];
  uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  if (nact[rec] == 0) return;
  const uint2 rr = ws_ptr<uint2>(ws, h.ws.rect)[rec];
  uint32_t x0 = rr.x & 0xffffu, y0 = rr.x >> 16, x1 = rr.y & 0xffffu, y1 = rr.y >> 16;
  x1 = min(x1, (uint32_t)rd.tiles_x);
  y1 = min(y1, (uint32_t)rd.tiles_y);
  uint32_t count = 0;
  if (x0 < x1 && y0 < y1) {
    const uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.sat) + rd.sat_offset;
    const uint32_t pitch = rd.tiles_x + 1;
    for (uint32_t y = y0; y < y1; ++y) count += st[y * pitch + x1] - st[y * pitch + x0];
  }
  nact[rec] = count;
}

__device__ inline uint64_t bounded_count(const uint32_t *n_dev, uint64_t n_bound) {
  if (n_dev == nullptr) return n_bound;
  const uint64_t d = *n_dev;
  return d < n_bound ? d : n_bound;
}

// Inputs of the scans.
struct InVisible {  // 1 for records with at least one active tile
  const uint32_t *nact;
  __device__ uint32_t operator()(uint64_t i) const { return nact[i] > 0 ? 1u : 0u; }
};
struct InPairs {  // active-tile count of the i-th record in depth order
  const uint32_t *nact, *order;
  __device__ uint32_t operator()(uint64_t i) const { return nact[order[i]]; }
};
struct InArray {
  const uint32_t *a;
  __device__ uint32_t operator()(uint64_t i) const { return a[i]; }
};

// Outputs of the scans: called for every i < n with its exclusive prefix.
struct OutCompact {
  const uint32_t *key_in;
  uint32_t *key_out, *val_out;
  __device__ void operator()(uint64_t i, uint32_t pos, uint32_t v) const {
    if (v) {
      key_out[pos] = key_in[i];
      val_out[pos] = (uint32_t)i;
    }
  }
};
struct OutArray {
  uint32_t *a;
  __device__ void operator()(uint64_t i, uint32_t pos, uint32_t) const { a[i] = pos; }
};

template <class In>
__global__ void __launch_bounds__(256) scan_reduce_kernel(In in, uint64_t n_bound, const uint32_t *n_dev, uint32_t *sums) {
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += in(i);
  }
  uint32_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of sums[0..nb) in place by one workgroup; the grand total
// goes to total_out[0] (and, as 64 bits, to total64 if given).
__global__ void __launch_bounds__(256) scan_top_kernel(uint32_t *sums, uint32_t nb, uint32_t *total_out,
                                                       uint32_t *total64) {
  uint64_t running = 0;
  for (uint32_t c = 0; c < nb; c += kScanChunk) {
    uint32_t v[kScanItems];
    uint32_t ts = 0;
    const uint32_t b = c + threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (b + k < nb) ? sums[b + k] : 0u;
      ts += v[k];
    }
    uint32_t tot;
    uint32_t off = block_exclusive_scan(ts, &tot);
    uint32_t acc = (uint32_t)running + off;
    for (int k = 0; k < kScanItems; ++k) {
      if (b + k < nb) sums[b + k] = acc;
      acc += v[k];
    }
    running += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (total_out) total_out[0] = (uint32_t)running;
    if (total64) {
      total64[0] = (uint32_t)running;
      total64[1] = (uint32_t)(running >> 32);
    }
  }
}

template <class In, class Out>
__global__ void __launch_bounds__(256) scan_down_kernel(In in, Out out, uint64_t n_bound, const uint32_t *n_dev,
                                                        const uint32_t *sums) {
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t ts = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    v[k] = i < n ? in(i) : 0u;
    ts += v[k];
  }
  uint32_t tot;
  uint32_t acc = block_exclusive_scan(ts, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    if (i < n) out(i, acc, v[k]);
    acc += v[k];
  }
}

template <class In, class Out>
void device_scan(In in, Out out, uint64_t n_bound, const uint32_t *n_dev, uint32_t *sums,
                 uint32_t *total_out, uint32_t *total64, hipStream_t s) {
  const uint32_t nb = (uint32_t)((n_bound + kScanChunk - 1) / kScanChunk);
  if (nb == 0) {
    // nothing to scan: still publish a zero total
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, 0u, total_out, total64);
    return;
  }
  hipLaunchKernelGGL(HIP_KERNEL_NAME(scan_reduce_kernel<In>), dim3(nb), dim3(kScanBlock), 0, s, in, n_bound, n_dev, sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, nb, total_out, total64);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(scan_down_kernel<In, Out>), dim3(nb), dim3(kScanBlock), 0, s, in, out, n_bound,
                     n_dev, sums);
}

// ------------------------------------------------------- radix sort

__global__ void __launch_bounds__(256) radix_hist_kernel(const uint32_t *__restrict__ keys, uint64_t n_bound,
                                                         const uint32_t *n_dev, int shift, uint32_t *hist,
                                                         uint32_t nblocks) {
  __shared__ uint32_t hs[kRadixBins];
  hs[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
  if (base < n) {
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
      if (i < n) atomicAdd(&hs[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
    }
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = hs[threadIdx.x];
}

// Stable scatter of one 8-bit digit.  The block's 4096 keys are taken in 16
// rounds of 256 consecutive keys; inside a round each wave ranks its keys
// among equal digits with ballots (lane order), the four waves are ordered by
// index, and every digit keeps a running base across rounds.
__global__ void __launch_bounds__(256) radix_scatter_kernel(const uint32_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin,
                                                            uint32_t *__restrict__ kout,
                                                            uint32_t *__restrict__ vout, uint64_t n_bound,
                                                            const uint32_t *n_dev, int shift,
                                                            const uint32_t *__restrict__ hist,
                                                            uint32_t nblocks) {
  __shared__ uint32_t base[kRadixBins];
  __shared__ uint32_t wcnt[4][kRadixBins];
  __shared__ uint32_t woff[4][kRadixBins];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t blk = (uint64_t)blockIdx.x * kScanChunk;
  if (blk >= n) return;
  base[tid] = hist[(uint64_t)tid * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int round = 0; round < kScanItems; ++round) {
    const uint64_t i = blk + (uint64_t)round * kScanBlock + tid;
    const bool valid = i < n;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t d = (key >> shift) & (kRadixBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    {
      const uint32_t c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
      const uint32_t b0 = base[tid];
      woff[0][tid] = b0;
      woff[1][tid] = b0 + c0;
      woff[2][tid] = b0 + c0 + c1;
      woff[3][tid] = b0 + c0 + c1 + c2;
      base[tid] = b0 + c0 + c1 + c2 + c3;
      wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = woff[wave][d] + rank;
      kout[pos] = key;
      vout[pos] = vin[i];
    }
  }
}

// Sorts (keys, vals) held in buffers [0] by `bits` low bits of the key;
// returns the index of the buffer holding the result.
int radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint64_t n_bound, const uint32_t *n_dev, int bits,
               uint32_t *hist, uint32_t *sums, hipStream_t s) {
  const uint32_t nb = (uint32_t)((n_bound + kScanChunk - 1) / kScanChunk);
  int cur = 0;
  if (nb == 0) return 0;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kScanBlock), 0, s, keys[cur], n_bound, n_dev, shift, hist, nb);
    device_scan(InArray{hist}, OutArray{hist}, (uint64_t)nb * kRadixBins, nullptr, sums, nullptr, nullptr, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kScanBlock), 0, s, keys[cur], vals[cur], keys[1 - cur],
                       vals[1 - cur], n_bound, n_dev, shift, hist, nb);
    cur = 1 - cur;
  }
  return cur;
}

// -------------------------------------------------------------- emission

__global__ void __launch_bounds__(256) emit_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                   const uint32_t *__restrict__ order,
                                                   uint32_t *__restrict__ key_out,
                                                   uint32_t *__restrict__ val_out) {
  const Header &h = *header(desc);
  const uint32_t *st = status_of(ws, h);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st[S_NVIS]) return;
  const uint32_t rec = order[i];
  uint64_t off = ws_ptr<uint32_t>(ws, h.ws.pair_off)[i];
  const uint64_t cap = h.pair_capacity;
  if (off >= cap) return;
  const int r = upper_index(rec_starts_of(desc), h.n_renders, (uint64_t)rec);
  const DevRender &rd = renders_of(desc)[r];
  const uint2 rr = ws_ptr<uint2>(ws, h.ws.rect)[rec];
  const uint32_t x0 = rr.x & 0xffffu, y0 = rr.x >> 16;
  const uint32_t x1 = min(rr.y & 0xffffu, (uint32_t)rd.tiles_x), y1 = min(rr.y >> 16, (uint32_t)rd.tiles_y);
  const uint32_t *tc = ws_ptr<uint32_t>(ws, h.ws.tile_count);
  for (uint32_t ty = y0; ty < y1; ++ty) {
    const uint32_t row = rd.tile_offset + ty * rd.tiles_x;
    for (uint32_t tx = x0; tx < x1; ++tx) {
      const uint32_t gt = row + tx;
      if (tc[gt] > 0) {
        if (off >= cap) return;
        key_out[off] = gt;
        val_out[off] = rec;
        ++off;
      }
    }
  }
}

// Pairs actually stored (min(needed, capacity)) and the overflow flag.
__global__ void pair_status_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint64_t need = (uint64_t)st[S_PAIRS_LO] | ((uint64_t)st[S_PAIRS_HI] << 32);
  const uint64_t cap = h.pair_capacity;
  st[S_OVERFLOW] = need > cap ? 1u : 0u;
  st[S_NPAIRS] = (uint32_t)(need > cap ? cap : need);
}

// ------------------------------------------------------------ ranges

__global__ void __launch_bounds__(256) ranges_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                     const uint32_t *__restrict__ tiles) {
  const Header &h = *header(desc);
  const uint32_t np = status_of(ws, h)[S_NPAIRS];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  uint2 *ranges = ws_ptr<uint2>(ws, h.ws.ranges);
  const uint32_t t = tiles[i];
  if (i == 0 || tiles[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i + 1 == np || tiles[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

// ------------------------------------------------------------- queue

__device__ inline uint32_t lpt_bucket(uint32_t masked, uint32_t len) {
  if (masked == 0) return 33;             // nothing to render: last
  if (len == 0) return 32;                // masked pixels but no Gaussian
  return (uint32_t)__clz(len);             // longer lists first (0 = longest)
}

__global__ void queue_count_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_tiles) return;
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[t];
  const uint32_t m = ws_ptr<uint32_t>(ws, h.ws.tile_count)[t];
  atomicAdd(ws_ptr<uint32_t>(ws, h.ws.bucket) + lpt_bucket(m, rg.y - rg.x), 1u);
}

__global__ void queue_offsets_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  if (threadIdx.x != 0) return;
  uint32_t *b = ws_ptr<uint32_t>(ws, h.ws.bucket);
  uint32_t acc = 0;
  for (int k = 0; k < 34; ++k) {
    const uint32_t c = b[k];
    b[k] = acc;
    acc += c;
  }
}

__global__ void queue_fill_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_tiles) return;
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[t];
  const uint32_t m = ws_ptr<uint32_t>(ws, h.ws.tile_count)[t];
  const uint32_t pos = atomicAdd(ws_ptr<uint32_t>(ws, h.ws.bucket) + lpt_bucket(m, rg.y - rg.x), 1u);
  ws_ptr<uint32_t>(ws, h.ws.queue)[pos] = (uint32_t)t;
}

inline unsigned blocks_for(uint64_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

uint64_t scan_scratch_words(uint64_t max_n) {
  // block sums of a scan over max_n elements, or over a radix histogram
  const uint64_t nb = (max_n + kScanChunk - 1) / kScanChunk;
  const uint64_t hb = (nb * kRadixBins + kScanChunk - 1) / kScanChunk;
  return (nb > hb ? nb : hb) + 64;
}

uint64_t radix_hist_words(uint64_t max_n) {
  const uint64_t nb = (max_n + kScanChunk - 1) / kScanChunk;
  return nb * kRadixBins + 64;
}

void launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t s) {
  if (n == 0) return;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, value, n);
}

void launch_tile_mask(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  hipLaunchKernelGGL(tile_mask_kernel, dim3(h.n_tile_rows), dim3(256), 0, s, d_desc, ws);
}

void launch_recount(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  hipLaunchKernelGGL(recount_kernel, dim3(blocks_for(h.n_records)), dim3(256), 0, s, d_desc, ws);
}

// Compaction of visible records + stable depth sort.  The sorted record
// ids end in vis_val[cur] (cur recorded in the header by the host: the
// number of passes is fixed, so it is known).
void launch_depth_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  uint32_t *sums = ws_ptr<uint32_t>(ws, h.ws.scan_sums);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_key[0]), ws_ptr<uint32_t>(ws, h.ws.vis_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_val[0]), ws_ptr<uint32_t>(ws, h.ws.vis_val[1])};
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  device_scan(InVisible{nact}, OutCompact{ws_ptr<uint32_t>(ws, h.ws.depth_key), keys[0], vals[0]}, h.n_records,
              nullptr, sums, st + S_NVIS, nullptr, s);
  radix_sort(keys, vals, h.n_records, st + S_NVIS, 32, ws_ptr<uint32_t>(ws, h.ws.hist), sums, s);
}

void launch_emit(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  uint32_t *sums = ws_ptr<uint32_t>(ws, h.ws.scan_sums);
  const uint32_t *order = ws_ptr<uint32_t>(ws, h.ws.vis_val[0]);  // 4 passes: back in buffer 0
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  device_scan(InPairs{nact, order}, OutArray{ws_ptr<uint32_t>(ws, h.ws.pair_off)}, h.n_records, st + S_NVIS, sums,
              nullptr, st + S_PAIRS_LO, s);
  hipLaunchKernelGGL(pair_status_kernel, dim3(1), dim3(1), 0, s, d_desc, ws);
  if (h.n_records == 0) return;
  hipLaunchKernelGGL(emit_kernel, dim3(blocks_for(h.n_records)), dim3(256), 0, s, d_desc, ws, order,
                     ws_ptr<uint32_t>(ws, h.ws.pair_key[0]), ws_ptr<uint32_t>(ws, h.ws.pair_val[0]));
}

void launch_tile_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_key[0]), ws_ptr<uint32_t>(ws, h.ws.pair_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_val[0]), ws_ptr<uint32_t>(ws, h.ws.pair_val[1])};
  const int cur = radix_sort(keys, vals, h.pair_capacity, st + S_NPAIRS, (int)h.tile_bits,
                             ws_ptr<uint32_t>(ws, h.ws.hist), ws_ptr<uint32_t>(ws, h.ws.scan_sums), s);
  launch_fill_u32(ws_ptr<uint32_t>(ws, h.ws.ranges), 0u, 2 * h.n_tiles, s);
  hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(h.pair_capacity)), dim3(256), 0, s, d_desc, ws, keys[cur]);
  if (h.cfg.persistent) {
    launch_fill_u32(ws_ptr<uint32_t>(ws, h.ws.bucket), 0u, 64, s);
    hipLaunchKernelGGL(queue_count_kernel, dim3(blocks_for(h.n_tiles)), dim3(256), 0, s, d_desc, ws);
    hipLaunchKernelGGL(queue_offsets_kernel, dim3(1), dim3(64), 0, s, d_desc, ws);
    hipLaunchKernelGGL(queue_fill_kernel, dim3(blocks_for(h.n_tiles)), dim3(256), 0, s, d_desc, ws);
  }
}

}  // namespace pgsag
