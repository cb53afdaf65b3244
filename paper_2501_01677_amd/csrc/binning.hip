// Tile binning (Sec. 3.1: projected Gaussians are assigned to image tiles
// and sorted), restricted to tiles that hold building-mask pixels.
//
// Pipeline (all counts stay on the device; grids are sized from host bounds
// and blocks past the device count exit):
//   tile_mask     masked pixels per tile and, per tile row, the prefix count
//                 of active tiles (one workgroup per tile row), so a support
//                 rectangle's active-tile count is two loads per tile row
//   compact       stable compaction of records with >= 1 active tile into
//                 (depth key, record) lists
//   radix sort    stable LSD sort of that list by the FP32 depth key; a pass
//                 whose digit is the same for every key is skipped
//   pair scan     exclusive scan of active-tile counts in depth order
//   emit          (global tile, record) pairs, depth order preserved
//   radix sort    stable LSD sort of the pairs by tile id -> every tile's list
//                 is in (depth, record) order
//   ranges        per tile [start, end) into the sorted pairs
//   queue         tiles ordered by decreasing list length (LPT) in buckets of
//                 log2(length), tiles without masked pixels last
//
// The scans and radix passes are single pass: each workgroup takes the next
// chunk index from an atomic counter (so every chunk before it belongs to a
// workgroup that is already running), publishes its chunk total, and looks
// back over its predecessors' published totals until it meets an inclusive
// prefix (decoupled look-back).  Waits only ever point backwards, to
// workgroups that are resident and do not wait on later ones, so they end;
// a bounded spin sets an error word instead of waiting forever.
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

// ------------------------------------------------------ look-back helpers

constexpr uint32_t kMaxSpins = 1u << 22;
constexpr uint64_t kAgg64 = 1ull << 62, kInc64 = 2ull << 62, kVal64 = (1ull << 62) - 1;
constexpr uint32_t kAgg32 = 1u << 30, kInc32 = 2u << 30, kVal32 = (1u << 30) - 1;

__device__ inline uint64_t ld64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ld32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chunk index of this workgroup, in launch order of the workgroups.
__device__ inline uint32_t virtual_block(uint32_t *ctr) {
  __shared__ uint32_t s_vid;
  if (threadIdx.x == 0) s_vid = atomicAdd(ctr, 1u);
  __syncthreads();
  return s_vid;
}

__device__ inline uint64_t wave_sum64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t olo = __shfl_xor(lo, o, 64), ohi = __shfl_xor(hi, o, 64);
    const uint32_t nlo = lo + olo;
    hi = hi + ohi + (nlo < lo ? 1u : 0u);
    lo = nlo;
  }
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive prefix of chunk `vid` whose own total is `agg`; called by the
// 64 lanes of one wave, which inspect 64 predecessors at a time.
__device__ uint64_t lookback64(uint64_t *st, uint32_t vid, uint64_t agg, uint32_t *err) {
  const int lane = threadIdx.x & 63;
  if (vid == 0) {
    if (lane == 0) st64(&st[0], kInc64 | agg);
    return 0;
  }
  if (lane == 0) st64(&st[vid], kAgg64 | agg);
  uint64_t excl = 0;
  int64_t hi = (int64_t)vid - 1;
  for (;;) {
    const int64_t idx = hi - lane;
    uint64_t w = kInc64;  // before chunk 0: an inclusive zero
    if (idx >= 0) {
      uint32_t spins = 0;
      for (;;) {
        w = ld64(&st[idx]);
        if ((w >> 62) != 0) break;
        if (++spins >= kMaxSpins) {
          atomicOr(err, 1u);
          w = kInc64;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const uint64_t inc = __ballot((w >> 62) == 2);
    const int first = inc ? (__ffsll((unsigned long long)inc) - 1) : 64;
    excl += wave_sum64(lane <= first ? (w & kVal64) : 0ull);
    if (inc) break;
    hi -= 64;
  }
  if (lane == 0) st64(&st[vid], kInc64 | (excl + agg));
  return excl;
}

// Per-digit exclusive prefix of chunk `vid` (one thread per digit).  The
// predecessors' words are read eight at a time so that a walk over chunks
// that have only published their own totals costs one memory round trip
// per eight chunks.
__device__ uint32_t lookback_digit(uint32_t *lb, uint32_t vid, int d, uint32_t agg, uint32_t *err) {
  if (vid == 0) {
    st32(&lb[d], kInc32 | agg);
    return 0;
  }
  st32(&lb[(uint64_t)vid * kRadixBins + d], kAgg32 | agg);
  uint32_t excl = 0;
  int64_t j = (int64_t)vid - 1;
  bool done = false;
  while (!done) {
    uint32_t w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = (j - u >= 0) ? ld32(&lb[(uint64_t)(j - u) * kRadixBins + d]) : kInc32;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (done) break;
      uint32_t x = w[u], spins = 0;
      while ((x >> 30) == 0) {  // not published yet: wait for it
        if (++spins >= kMaxSpins) {
          atomicOr(err, 1u);
          x = kInc32;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        x = ld32(&lb[(uint64_t)(j - u) * kRadixBins + d]);
      }
      excl += x & kVal32;
      if ((x >> 30) == 2) done = true;
    }
    j -= 8;
  }
  st32(&lb[(uint64_t)vid * kRadixBins + d], kInc32 | (excl + agg));
  return excl;
}

// ------------------------------------------------------------ compaction

// Records with at least one active tile, in record order, as (depth key,
// record id) -> vis_key[0], vis_val[0]; the count goes to the status word.
__global__ void __launch_bounds__(256) compact_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint64_t n = h.n_records;
  const uint32_t nb = (uint32_t)chunks_of(n);
  const uint32_t vid = virtual_block(st + S_CTR_COMPACT);
  if (vid >= nb) return;
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  const uint64_t base = (uint64_t)vid * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
  uint32_t f[kScanItems];
  uint32_t ts = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    f[k] = (i < n && nact[i] > 0) ? 1u : 0u;
    ts += f[k];
  }
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan(ts, &tot);
  __shared__ uint64_t s_prefix;
  if (threadIdx.x < 64) {
    const uint64_t p = lookback64(ws_ptr<uint64_t>(ws, h.ws.lb_compact), vid, tot, st + S_ERROR);
    if (threadIdx.x == 0) s_prefix = p;
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;
  if (vid == nb - 1 && threadIdx.x == 0) st[S_NVIS] = (uint32_t)(prefix + tot);
  const uint32_t *dkey = ws_ptr<uint32_t>(ws, h.ws.depth_key);
  uint32_t *ko = ws_ptr<uint32_t>(ws, h.ws.vis_key[0]);
  uint32_t *vo = ws_ptr<uint32_t>(ws, h.ws.vis_val[0]);
  uint64_t pos = prefix + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (f[k]) {
      const uint64_t i = base + k;
      ko[pos] = dkey[i];
      vo[pos] = (uint32_t)i;
      ++pos;
    }
  }
}

// ------------------------------------------------------- radix sort

// Digit histograms of every pass in one read of the keys.
__global__ void __launch_bounds__(256) digit_hist_kernel(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                         uint64_t n_bound, int passes, uint32_t *hist) {
  __shared__ uint32_t hs[4][kRadixBins];
  for (int p = 0; p < 4; ++p) hs[p][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t k = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&hs[p][(k >> (kRadixBits * p)) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (hs[p][threadIdx.x]) atomicAdd(&hist[p * kRadixBins + threadIdx.x], hs[p][threadIdx.x]);
}

// One stable LSD pass over the 8-bit digit `pass`.  With `dynamic`, passes
// whose digit is constant over all keys are skipped (every workgroup of such
// a pass returns at once) and the ping-pong buffer of each pass follows the
// number of non-skipped passes before it; the buffer holding the final
// order is published in status[cur_word].
__global__ void __launch_bounds__(256) onesweep_kernel(uint32_t *keys0, uint32_t *vals0, uint32_t *keys1,
                                                       uint32_t *vals1, const uint32_t *n_dev, uint64_t n_bound,
                                                       int pass, int passes, int dynamic,
                                                       const uint32_t *__restrict__ hist, uint32_t *lb,
                                                       uint32_t *ctr, uint32_t *st, int cur_word) {
  __shared__ uint32_t dbase[kRadixBins], run[kRadixBins];
  __shared__ uint32_t wcnt[4][kRadixBins];
  __shared__ uint32_t woff[4][kRadixBins];
  __shared__ int s_skip;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint32_t nb = (uint32_t)chunks_of(n);
  // which passes are real
  int parity = pass & 1, final_parity = passes & 1, skip = 0;
  if (dynamic) {
    if (tid == 0) s_skip = 0;
    __syncthreads();
    int np = 0, before = 0;
    for (int p = 0; p < passes; ++p) {
      const int trivial = __syncthreads_or(n > 0 && hist[p * kRadixBins + tid] == n);
      if (!trivial) {
        if (p < pass) ++before;
        ++np;
      } else if (p == pass) {
        skip = 1;
      }
    }
    parity = before & 1;
    final_parity = np & 1;
  }
  const uint32_t vid = virtual_block(ctr);
  if (vid == 0 && tid == 0 && cur_word >= 0) st[cur_word] = (uint32_t)final_parity;
  if (skip || vid >= nb) return;
  const uint32_t *kin = parity ? keys1 : keys0;
  const uint32_t *vin = parity ? vals1 : vals0;
  uint32_t *kout = parity ? keys0 : keys1;
  uint32_t *vout = parity ? vals0 : vals1;
  const int shift = kRadixBits * pass;
  {
    uint32_t tot;
    dbase[tid] = block_exclusive_scan(hist[pass * kRadixBins + tid], &tot);
  }
  run[tid] = 0;
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t blk = (uint64_t)vid * kScanChunk;
  uint32_t kk[kScanItems], vv[kScanItems], rk[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint64_t i = blk + (uint64_t)r * kScanBlock + tid;
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
      const uint32_t b0 = run[tid];
      woff[0][tid] = b0;
      woff[1][tid] = b0 + c0;
      woff[2][tid] = b0 + c0 + c1;
      woff[3][tid] = b0 + c0 + c1 + c2;
      run[tid] = b0 + c0 + c1 + c2 + c3;
      wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
    }
    __syncthreads();
    kk[r] = key;
    vv[r] = valid ? vin[i] : 0u;
    rk[r] = valid ? woff[wave][d] + rank : 0xffffffffu;
  }
  // global position of each digit's run for this chunk
  const uint32_t excl = lookback_digit(lb, vid, tid, run[tid], st + S_ERROR);
  __syncthreads();
  run[tid] = dbase[tid] + excl;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (rk[r] != 0xffffffffu) {
      const uint32_t d = (kk[r] >> shift) & (kRadixBins - 1);
      const uint32_t pos = run[d] + rk[r];
      kout[pos] = kk[r];
      vout[pos] = vv[r];
    }
  }
}

// Sorts (keys, vals) in buffers [0] by `bits` low key bits; with `dynamic`
// the result buffer is published in st[cur_word], otherwise it is buffer
// (passes & 1).
void radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint64_t n_bound, const uint32_t *n_dev, int bits,
                int dynamic, uint32_t *hist, uint32_t *lb, uint32_t *ctr, uint32_t *st, int cur_word,
                hipStream_t s) {
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  const uint32_t nb = (uint32_t)chunks_of(n_bound);
  if (nb == 0 || passes == 0) return;
  unsigned hb = nb < 2048 ? nb : 2048;
  hipLaunchKernelGGL(digit_hist_kernel, dim3(hb), dim3(256), 0, s, keys[0], n_dev, n_bound, passes, hist);
  for (int p = 0; p < passes; ++p)
    hipLaunchKernelGGL(onesweep_kernel, dim3(nb), dim3(256), 0, s, keys[0], vals[0], keys[1], vals[1], n_dev,
                       n_bound, p, passes, dynamic, hist, lb + (uint64_t)p * (nb + 1) * kRadixBins, ctr + p, st,
                       cur_word);
}

// -------------------------------------------------------------- emission

// Exclusive scan of the active-tile counts of the depth-sorted visible
// records -> pair_off[], and the pair total / overflow in the status word.
__global__ void __launch_bounds__(256) pair_scan_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint64_t nvis = st[S_NVIS];
  const uint32_t nb = (uint32_t)chunks_of(nvis);
  const uint32_t vid = virtual_block(st + S_CTR_EMIT);
  if (vid >= nb) return;
  const uint32_t *order = ws_ptr<uint32_t>(ws, h.ws.vis_val[st[S_DEPTH_CUR] ? 1 : 0]);
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  const uint64_t base = (uint64_t)vid * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
  uint32_t cnt[kScanItems];
  uint32_t ts = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    cnt[k] = i < nvis ? nact[order[i]] : 0u;
    ts += cnt[k];
  }
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan(ts, &tot);
  __shared__ uint64_t s_prefix;
  if (threadIdx.x < 64) {
    const uint64_t p = lookback64(ws_ptr<uint64_t>(ws, h.ws.lb_emit), vid, tot, st + S_ERROR);
    if (threadIdx.x == 0) s_prefix = p;
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;
  const uint64_t cap = h.pair_capacity;
  if (vid == nb - 1 && threadIdx.x == 0) {
    const uint64_t need = prefix + tot;
    st[S_PAIRS_LO] = (uint32_t)need;
    st[S_PAIRS_HI] = (uint32_t)(need >> 32);
    st[S_OVERFLOW] = need > cap ? 1u : 0u;
    st[S_NPAIRS] = (uint32_t)(need > cap ? cap : need);
  }
  uint32_t *off = ws_ptr<uint32_t>(ws, h.ws.pair_off);
  uint64_t o = prefix + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    if (i < nvis) off[i] = (uint32_t)(o < cap ? o : cap);
    o += cnt[k];
  }
}

// One thread per depth-sorted visible record: its (global tile, record)
// pairs, active tiles of its rectangle in row-major order, up to capacity.
__global__ void __launch_bounds__(256) emit_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t *st = status_of(ws, h);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st[S_NVIS]) return;
  const uint32_t rec = ws_ptr<uint32_t>(ws, h.ws.vis_val[st[S_DEPTH_CUR] ? 1 : 0])[i];
  uint64_t off = ws_ptr<uint32_t>(ws, h.ws.pair_off)[i];
  const uint64_t cap = h.pair_capacity;
  if (off >= cap) return;
  const int r = upper_index(rec_starts_of(desc), h.n_renders, (uint64_t)rec);
  const DevRender &rd = renders_of(desc)[r];
  const uint2 rr = ws_ptr<uint2>(ws, h.ws.rect)[rec];
  const uint32_t x0 = rr.x & 0xffffu, y0 = rr.x >> 16;
  const uint32_t x1 = min(rr.y & 0xffffu, (uint32_t)rd.tiles_x), y1 = min(rr.y >> 16, (uint32_t)rd.tiles_y);
  const uint32_t *tc = ws_ptr<uint32_t>(ws, h.ws.tile_count);
  uint32_t *key_out = ws_ptr<uint32_t>(ws, h.ws.pair_key[0]);
  uint32_t *val_out = ws_ptr<uint32_t>(ws, h.ws.pair_val[0]);
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

void launch_depth_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)chunks_of(h.n_records)), dim3(256), 0, s, d_desc, ws);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_key[0]), ws_ptr<uint32_t>(ws, h.ws.vis_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_val[0]), ws_ptr<uint32_t>(ws, h.ws.vis_val[1])};
  radix_sort(keys, vals, h.n_records, st + S_NVIS, 32, 1, ws_ptr<uint32_t>(ws, h.ws.dhist),
             ws_ptr<uint32_t>(ws, h.ws.lb_depth), st + S_CTR_DEPTH, st, S_DEPTH_CUR, s);
}

void launch_emit(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  hipLaunchKernelGGL(pair_scan_kernel, dim3((unsigned)chunks_of(h.n_records)), dim3(256), 0, s, d_desc, ws);
  hipLaunchKernelGGL(emit_kernel, dim3(blocks_for(h.n_records)), dim3(256), 0, s, d_desc, ws);
}

void launch_tile_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_key[0]), ws_ptr<uint32_t>(ws, h.ws.pair_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_val[0]), ws_ptr<uint32_t>(ws, h.ws.pair_val[1])};
  radix_sort(keys, vals, h.pair_capacity, st + S_NPAIRS, (int)h.tile_bits, 0, ws_ptr<uint32_t>(ws, h.ws.thist),
             ws_ptr<uint32_t>(ws, h.ws.lb_tile), st + S_CTR_TILE, st, -1, s);
  const uint32_t *sorted_tiles = ws_ptr<uint32_t>(ws, h.ws.sorted_key);
  launch_fill_u32(ws_ptr<uint32_t>(ws, h.ws.ranges), 0u, 2 * h.n_tiles, s);
  hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(h.pair_capacity)), dim3(256), 0, s, d_desc, ws, sorted_tiles);
  if (h.cfg.persistent) {
    hipLaunchKernelGGL(queue_count_kernel, dim3(blocks_for(h.n_tiles)), dim3(256), 0, s, d_desc, ws);
    hipLaunchKernelGGL(queue_offsets_kernel, dim3(1), dim3(64), 0, s, d_desc, ws);
    hipLaunchKernelGGL(queue_fill_kernel, dim3(blocks_for(h.n_tiles)), dim3(256), 0, s, d_desc, ws);
  }
}

}  // namespace pgsag
