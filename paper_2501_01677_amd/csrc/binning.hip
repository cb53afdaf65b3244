// Tile binning (Sec. 3.1: projected Gaussians are assigned to image tiles
// and sorted), restricted to tiles that hold building-mask pixels.
//
// Pipeline (all counts stay on the device; grids are sized from host bounds
// and blocks past the device count exit):
//   tile_mask     masked pixels per tile and, per tile row, the prefix count
//                 of active tiles (one workgroup per tile row), so a support
//                 rectangle's active-tile count is two loads per tile row
//   compact       stable compaction of records with >= 1 active tile into
//                 (depth key, record) lists, with the depth digit histograms
//   depth plan    one wave decides which depth passes are real (a pass whose
//                 digit is the same for every key is skipped) -> plan word
//   radix sort    stable LSD sort of that list by the FP32 depth key
//   chunk pairs   pair totals of every 1024 depth-sorted records
//   emit          per 1024 records: the first pair offset from the earlier
//                 chunks' totals and a workgroup scan of the counts, then
//                 (global tile, record) pairs in depth order, one wave per
//                 64 records emitting 64 pairs at a time
//   radix sort    stable LSD sort of the pairs by tile id -> every tile's list
//                 is in (depth, record) order
//   ranges        per tile [start, end) into the sorted pairs
//   queue         tiles ordered by decreasing list length (LPT) in buckets of
//                 log2(length), tiles without masked pixels last, by a stable
//                 radix pass (tile order kept inside a bucket)
//
// The compaction is single pass: each workgroup takes the next chunk index
// from an atomic counter (so every chunk before it belongs to a workgroup
// that is already running), publishes its chunk total, and looks back 64
// predecessors at a time until it meets an inclusive prefix (decoupled
// look-back).  Waits only ever point backwards, to workgroups that are
// resident and do not wait on later ones, so they end; a bounded spin sets
// an error word instead of waiting forever.  Radix passes use
// reduce-then-scan (chunk digit counts, a per-digit scan, a scatter).  The
// digit histograms the scan needs are accumulated by the compaction (depth
// keys, all passes at once, so the plan can skip passes) or by each pass's
// count kernel (tile ids), in kHistCopies copies (fewer same-word atomics).
#include "internal.h"

namespace pgsag {
namespace {

__device__ inline uint32_t *status_of(void *ws, const Header &h) {
  return ws_ptr<uint32_t>(ws, h.ws.status);
}

// n words of p set to value: 16-byte stores over the 16-byte aligned body,
// single words before and after it.  Nothing is written when `skip` points
// to a non-zero word.
__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, uint64_t n, const uint32_t *skip) {
  if (skip && *skip) return;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t lead = (uint64_t)((16u - ((uintptr_t)p & 15u)) & 15u) / 4u;
  const uint64_t head = lead < n ? lead : n;
  const uint64_t nv = (n - head) / 4;
  if (tid < head) p[tid] = value;
  uint4 *q = reinterpret_cast<uint4 *>(p + head);
  const uint4 v = make_uint4(value, value, value, value);
  for (uint64_t i = tid; i < nv; i += stride) q[i] = v;
  const uint64_t done = head + nv * 4;
  if (tid < n - done) p[done + tid] = value;
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
template <int NW = 4>  // waves in the workgroup
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
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

// Masked pixels of the (tile x, pixel row) spans of one tile row, for masks
// whose rows start on 4-byte boundaries: each thread counts 4 spans per
// round with all their word loads issued together.  WPT = tile / 4 words per
// span; a span ends early at the image edge (W is a multiple of 4 here).
template <int WPT>
__device__ void count_row_spans(const uint8_t *mask, int W, int tx_n, int y0, int rows, uint32_t *cnt) {
  const int items = tx_n * rows;
  for (int it0 = 0; it0 < items; it0 += 4 * (int)blockDim.x) {
    uint32_t cc[4];
    int xx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int it = it0 + u * (int)blockDim.x + (int)threadIdx.x;
      cc[u] = 0;
      xx[u] = 0;
      if (it < items) {
        const int x = it % tx_n, y = y0 + it / tx_n;
        const int a = x * WPT * 4, nw = min(WPT, (W - a) >> 2);
        const uint32_t *m = reinterpret_cast<const uint32_t *>(mask + (uint64_t)y * W + a);
        uint32_t w[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) w[k] = k < nw ? m[k] : 0u;
#pragma unroll
        for (int k = 0; k < WPT; ++k) cc[u] += nonzero_bytes(w[k]);
        xx[u] = x;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (cc[u]) atomicAdd(&cnt[xx[u]], cc[u]);
  }
}

// One workgroup per global tile row: masked (or, without a mask, in-image)
// pixels of every tile of the row, and the row prefix of active flags
// rowsat[ty][x] = number of active tiles among tiles 0..x-1 of row ty.
constexpr int kMaskBlock = 1024;  // threads per tile row: its spans load in one round at 1080p
__global__ void __launch_bounds__(kMaskBlock) tile_mask_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
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
  } else if ((W & 3) == 0 && ((uintptr_t)rd.mask & 3u) == 0) {
    if (tile == 8) count_row_spans<2>(rd.mask, W, tx_n, y0, rows, cnt);
    else if (tile == 16) count_row_spans<4>(rd.mask, W, tx_n, y0, rows, cnt);
    else count_row_spans<8>(rd.mask, W, tx_n, y0, rows, cnt);
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
  {
    const uint32_t wpr = (tx_n + 31) / 32;
    uint32_t *am = ws_ptr<uint32_t>(ws, h.ws.amask) + rd.amask_offset + (uint64_t)ty * wpr;
    for (uint32_t w = threadIdx.x; w < wpr; w += blockDim.x) {
      uint32_t bits = 0;
      for (int b = 0; b < 32; ++b) {
        const uint32_t x = w * 32 + b;
        if (x < (uint32_t)tx_n && cnt[x] > 0) bits |= 1u << b;
      }
      am[w] = bits;
    }
  }
  // empty [0, 0) ranges for every tile of the row (the ranges kernel only
  // writes tiles that receive pairs)
  {
    uint2 *rg = ws_ptr<uint2>(ws, h.ws.ranges) + rd.tile_offset + (uint64_t)ty * tx_n;
    for (int x = threadIdx.x; x < tx_n; x += blockDim.x) rg[x] = make_uint2(0u, 0u);
  }
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
    const uint32_t ex = block_exclusive_scan<kMaskBlock / 64>(v, &tot);
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

// ------------------------------------------------------------ compaction

// Records with at least one active tile, in record order, as (depth key,
// record id) -> vis_key[0], vis_val[0]; the count goes to the status word.
constexpr int kCompactBlock = 1024;                         // threads per 4096-record chunk
constexpr int kCompactItems = kScanChunk / kCompactBlock;  // consecutive records per thread
__global__ void __launch_bounds__(kCompactBlock) compact_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint64_t n = h.n_records;
  const uint32_t nb = (uint32_t)chunks_of(n);
  const uint32_t vid = virtual_block(st + S_CTR_COMPACT);
  if (vid >= nb) return;
  const uint32_t *nact = ws_ptr<uint32_t>(ws, h.ws.nact);
  const uint32_t *dkey = ws_ptr<uint32_t>(ws, h.ws.depth_key);
  const uint64_t base = (uint64_t)vid * kScanChunk + (uint64_t)threadIdx.x * kCompactItems;
  uint32_t f[kCompactItems], dk[kCompactItems];
  uint32_t ts = 0;
  // the depth keys are loaded with the counts, ahead of the scan and the
  // look-back (below, the stores would keep the compiler from hoisting them)
#pragma unroll
  for (int k = 0; k < kCompactItems; ++k) {
    const uint64_t i = base + k;
    f[k] = (i < n && nact[i] > 0) ? 1u : 0u;
    dk[k] = i < n ? dkey[i] : 0u;
    ts += f[k];
  }
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan<kCompactBlock / 64>(ts, &tot);
  __shared__ uint64_t s_prefix;
  if (threadIdx.x < 64) {
    const uint64_t p = lookback64(ws_ptr<uint64_t>(ws, h.ws.lb_compact), vid, tot, st + S_ERROR);
    if (threadIdx.x == 0) s_prefix = p;
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;
  if (vid == nb - 1 && threadIdx.x == 0) st[S_NVIS] = (uint32_t)(prefix + tot);
  uint32_t *ko = ws_ptr<uint32_t>(ws, h.ws.vis_key[0]);
  uint32_t *vo = ws_ptr<uint32_t>(ws, h.ws.vis_val[0]);
  // digit histograms of the depth keys for the radix passes
  __shared__ uint32_t hs[kDepthPasses][kRadixBins];
  if (threadIdx.x < kRadixBins)
    for (int p = 0; p < kDepthPasses; ++p) hs[p][threadIdx.x] = 0;
  __syncthreads();
  uint64_t pos = prefix + ex;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kCompactItems; ++k) {
    const uint64_t i = base + k;
    const uint32_t key = f[k] ? dk[k] : 0u;
    if (f[k]) {
      ko[pos] = key;
      vo[pos] = (uint32_t)i;
      ++pos;
    }
    if (f[k])
      for (int p = 0; p < kDepthPasses - 1; ++p)
        atomicAdd(&hs[p][(key >> (kRadixBits * p)) & (kRadixBins - 1)], 1u);
    // The top digit (sign and high exponent bits) is usually the same for
    // the whole wave: then one lane adds the wave's count instead of every
    // lane hitting the same LDS word.
    const uint32_t top = key >> (kRadixBits * (kDepthPasses - 1));
    const uint64_t act = __ballot(f[k]);
    if (act) {
      const uint32_t ref = __shfl(top, __ffsll((unsigned long long)act) - 1, 64);
      const bool uniform = __ballot(f[k] && top != ref) == 0ull;
      if (uniform) {
        if (lane == __ffsll((unsigned long long)act) - 1) atomicAdd(&hs[kDepthPasses - 1][ref], (uint32_t)__popcll(act));
      } else if (f[k]) {
        atomicAdd(&hs[kDepthPasses - 1][top], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t *dh = ws_ptr<uint32_t>(ws, h.ws.dhist) + (vid % kHistCopies) * kHistStride;
  if (threadIdx.x < kRadixBins)
    for (int p = 0; p < kDepthPasses; ++p)
      if (hs[p][threadIdx.x]) atomicAdd(&dh[p * kRadixBins + threadIdx.x], hs[p][threadIdx.x]);
}

// Which depth passes are real, decided once from the complete histograms
// (a pass whose digit is the same for every key is skipped), for every
// workgroup of the pass kernels: one wave.
__global__ void __launch_bounds__(64) depth_plan_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint32_t *dh = ws_ptr<const uint32_t>(ws, h.ws.dhist);
  const uint32_t n = st[S_NVIS];
  const int lane = threadIdx.x;
  uint32_t skip = 0;
#pragma unroll
  for (int p = 0; p < kDepthPasses; ++p) {
    bool one = false;
#pragma unroll
    for (int q = 0; q < kRadixBins / 64; ++q) {
      uint32_t v = 0;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) v += dh[c * kHistStride + p * kRadixBins + q * 64 + lane];
      one |= v == n;
    }
    if (n > 0 && __ballot(one)) skip |= 1u << p;
  }
  if (lane == 0) st[S_PLAN_DEPTH] = skip;
}

// ------------------------------------------------------- radix sort

// Digit histograms of every pass in one read of the keys.
__global__ void __launch_bounds__(256) digit_hist_kernel(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                         uint64_t n_bound, int passes, int dbits, uint32_t *hist) {
  const uint32_t dmask = (1u << dbits) - 1u;
  __shared__ uint32_t hs[4][kRadixBins];
  for (int p = 0; p < 4; ++p) hs[p][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t k = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&hs[p][(k >> (dbits * p)) & dmask], 1u);
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (hs[p][threadIdx.x])
      atomicAdd(&hist[(blockIdx.x % kHistCopies) * kHistStride + p * kRadixBins + threadIdx.x], hs[p][threadIdx.x]);
}

// Which passes of a sort are real.  With a plan word (bit p set: pass p is
// skipped because its digit is the same for every key), the ping-pong buffer
// of each pass follows the number of real passes before it; without one,
// every pass is real.
struct PassPlan {
  int skip, parity, final_parity;
};

__device__ inline PassPlan plan_pass(const uint32_t *plan_word, int pass, int passes) {
  if (!plan_word) return PassPlan{0, pass & 1, passes & 1};
  const uint32_t plan = *plan_word;
  const uint32_t real = ~plan & ((1u << passes) - 1u);
  return PassPlan{(int)((plan >> pass) & 1u), (int)(__popc(real & ((1u << pass) - 1u)) & 1u), (int)(__popc(real) & 1u)};
}

// Pass part 1: digit counts of every chunk -> table[digit][chunk].  NW
// waves of RI keys per thread: chunks of 64 NW RI keys.  With `hist`, the
// chunk's counts are also added to the pass's digit histogram (copy chunk
// mod kHistCopies), which the digit scan reads next.
template <int RI, int NW>
__global__ void __launch_bounds__(64 * NW) chunk_count_kernel(const uint32_t *keys0, const uint32_t *keys1,
                                                              const uint32_t *n_dev, uint64_t n_bound, int pass,
                                                              int passes, int dbits, const uint32_t *plan_word,
                                                              uint32_t *table, uint32_t nb_bound, uint32_t *hist) {
  constexpr int NT = 64 * NW;
  __shared__ uint32_t hs[kRadixBins];
  const PassPlan pp = plan_pass(plan_word, pass, passes);
  if (pp.skip) return;
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint32_t c = blockIdx.x;
  if ((uint64_t)c * (RI * NT) >= n) return;  // (the scan reads only the chunks that hold keys)
  if (threadIdx.x < kRadixBins) hs[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t *kin = pp.parity ? keys1 : keys0;
  const int shift = dbits * pass;
  const uint32_t dmask = (1u << dbits) - 1u;
  const uint64_t base = (uint64_t)c * (RI * NT);
  // all keys are loaded before the first LDS atomic (one round trip)
  uint32_t kk[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const uint64_t i = base + (uint64_t)r * NT + threadIdx.x;
    kk[r] = i < n ? kin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < RI; ++r)
    if (base + (uint64_t)r * NT + threadIdx.x < n) atomicAdd(&hs[(kk[r] >> shift) & dmask], 1u);
  __syncthreads();
  if (threadIdx.x <= dmask) {
    const uint32_t v = hs[threadIdx.x];
    table[(uint64_t)threadIdx.x * nb_bound + c] = v;
    if (hist && v) atomicAdd(&hist[(c % kHistCopies) * kHistStride + pass * kRadixBins + threadIdx.x], v);
  }
}

// Pass part 2: per digit, exclusive scan of its chunk counts along the
// chunks, offset by the digit's base (exclusive scan of the digit totals):
// table[d][c] becomes the output position of chunk c's first key of digit d.
// One workgroup of 1024 threads per digit; up to 8192 chunks per round are
// loaded at once (coalesced), scanned through LDS as 1024 contiguous
// segments, and stored.
constexpr int kScanRound = 32;      // entries loaded per round: kScanRound x 256
constexpr int kDigitScanBlock = 1024;  // threads per digit (few entries per thread)
__global__ void __launch_bounds__(kDigitScanBlock) chunk_scan_kernel(const uint32_t *n_dev, uint64_t n_bound, int pass,
                                                                     int passes, const uint32_t *plan_word,
                                                                     const uint32_t *hist, uint32_t *table,
                                                                     uint32_t nb_bound, uint32_t chunk) {
  constexpr int NW = kDigitScanBlock / 64;
  __shared__ uint32_t seg[kScanRound * kScanBlock];
  __shared__ uint32_t red[NW];
  const PassPlan pp = plan_pass(plan_word, pass, passes);
  if (pp.skip) return;
  const uint64_t n = bounded_count(n_dev, n_bound);
  const uint32_t nb = (uint32_t)((n + chunk - 1) / chunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int d = blockIdx.x;
  const uint32_t *h = hist + pass * kRadixBins;
  // digit base: sum of the totals of the digits below d (over the copies)
  uint32_t b = 0;
  if (tid < d)
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) b += h[c * kHistStride + tid];
  for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o, 64);
  if (lane == 0) red[wave] = b;
  __syncthreads();
  uint32_t run = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) run += red[w];
  uint32_t *row = table + (uint64_t)d * nb_bound;
  for (uint32_t c0 = 0; c0 < nb; c0 += kScanRound * kScanBlock) {
    const uint32_t m = min((uint32_t)(kScanRound * kScanBlock), nb - c0);
    const uint32_t J = (m + kDigitScanBlock - 1) / kDigitScanBlock;  // entries per thread segment
    for (uint32_t j = 0; j < J; ++j) {
      const uint32_t c = j * kDigitScanBlock + tid;
      seg[c] = c < m ? row[c0 + c] : 0u;
    }
    __syncthreads();
    uint32_t sum = 0;
    for (uint32_t j = 0; j < J; ++j) sum += seg[tid * J + j];
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<NW>(sum, &tot);
    uint32_t acc = run + ex;
    for (uint32_t j = 0; j < J; ++j) {
      const uint32_t v = seg[tid * J + j];
      seg[tid * J + j] = acc;
      acc += v;
    }
    __syncthreads();
    for (uint32_t j = 0; j < J; ++j) {
      const uint32_t c = j * kDigitScanBlock + tid;
      if (c < m) row[c0 + c] = seg[c];
    }
    run += tot;
    __syncthreads();
  }
}

// Pass part 3: stable scatter (chunks of 64 NW RI keys).  Each wave ranks
// its own contiguous 1/NW of the chunk, 64 keys at a time, against
// wave-private running counts (no workgroup barriers); waves are ordered by
// index and chunks by the table.
template <int RI, int NW>
__global__ void __launch_bounds__(64 * NW) chunk_scatter_kernel(uint32_t *keys0, uint32_t *vals0, uint32_t *keys1,
                                                                uint32_t *vals1, const uint32_t *n_dev,
                                                                uint64_t n_bound, int pass, int passes, int dbits,
                                                                const uint32_t *plan_word, const uint32_t *table,
                                                                uint32_t nb_bound, uint32_t *st, int cur_word) {
  __shared__ uint32_t wrun[NW][kRadixBins];  // per-wave running digit counts
  __shared__ uint32_t woff[NW][kRadixBins];  // output position of each wave's first key of a digit
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = bounded_count(n_dev, n_bound);
  const PassPlan pp = plan_pass(plan_word, pass, passes);
  const uint32_t c = blockIdx.x;
  if (c == 0 && tid == 0 && cur_word >= 0) st[cur_word] = (uint32_t)pp.final_parity;
  constexpr int CH = RI * 64 * NW;
  if (pp.skip || (uint64_t)c * CH >= n) return;
  const uint32_t *kin = pp.parity ? keys1 : keys0;
  const uint32_t *vin = pp.parity ? vals1 : vals0;
  uint32_t *kout = pp.parity ? keys0 : keys1;
  uint32_t *vout = pp.parity ? vals0 : vals1;
  const int shift = dbits * pass;
  const uint32_t dmask = (1u << dbits) - 1u;
  // The keys, the values and this chunk's output offset of each digit are
  // all loaded here, so they arrive in one round trip (after the barriers
  // below the compiler could not move the later loads up).
  const uint32_t gb = (tid < kRadixBins && (uint32_t)tid <= dmask) ? table[(uint64_t)tid * nb_bound + c] : 0u;
  const uint64_t qbase = (uint64_t)c * CH + (uint64_t)wave * (CH / NW);
  uint32_t kin_r[RI], vv[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const uint64_t i = qbase + (uint64_t)r * 64 + lane;
    kin_r[r] = i < n ? kin[i] : 0u;
    vv[r] = i < n ? vin[i] : 0u;
  }
  if (tid < kRadixBins)
    for (int w = 0; w < NW; ++w) wrun[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t kk[RI], rk[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const uint64_t i = qbase + (uint64_t)r * 64 + lane;
    const bool valid = i < n;
    const uint32_t key = kin_r[r];
    const uint32_t d = (key >> shift) & dmask;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      if (b >= dbits) break;
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    const uint32_t base = wrun[wave][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wrun[wave][d] = base + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    kk[r] = key;
    rk[r] = valid ? base + rank : 0xffffffffu;
  }
  __syncthreads();
  // chunk-local digit-major order: the chunk's keys are first placed in LDS
  // sorted by digit, then every digit's run is written out contiguously
  __shared__ uint32_t cbase[kRadixBins];   // chunk-local start of each digit
  __shared__ uint32_t gbase[kRadixBins];   // output position of each digit's run
  __shared__ uint32_t skey[CH], sval[CH];
  {
    uint32_t cw[NW], tot_d = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      cw[w] = tid < kRadixBins ? wrun[w][tid] : 0u;
      tot_d += cw[w];
    }
    uint32_t tot;
    const uint32_t cb = block_exclusive_scan<NW>(tot_d, &tot);
    if (tid < kRadixBins) {
      cbase[tid] = cb;
      gbase[tid] = gb;
      uint32_t o = cb;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        woff[w][tid] = o;
        o += cw[w];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    if (rk[r] != 0xffffffffu) {
      const uint32_t d = (kk[r] >> shift) & dmask;
      const uint32_t lp = woff[wave][d] + rk[r];
      skey[lp] = kk[r];
      sval[lp] = vv[r];
    }
  }
  __syncthreads();
  const uint64_t cstart = (uint64_t)c * CH;
  const uint32_t cnt = (uint32_t)min((uint64_t)CH, n - cstart);
  for (uint32_t i = tid; i < cnt; i += 64 * NW) {
    const uint32_t key = skey[i];
    const uint32_t d = (key >> shift) & dmask;
    const uint32_t pos = gbase[d] + (i - cbase[d]);
    kout[pos] = key;
    vout[pos] = sval[i];
  }
}

// Sorts (keys, vals) in buffers [0] by `bits` low key bits, stably.  With a
// plan word (written on the device before the sort) passes it marks are
// skipped and the result buffer is published in st[cur_word]; otherwise it
// is buffer (passes & 1).  The digit histograms (`hist`, zeroed before the
// sort) come from `hist_mode`: kHistByProducer, accumulated by the kernel
// that produced the keys; kHistByCount, by each pass's count kernel;
// kHistByPass, by one extra read of the keys before the first pass.
// `table` holds uint32 [256][chunks].
enum HistMode { kHistByPass = 0, kHistByProducer = 1, kHistByCount = 2 };
template <int RI>
void radix_passes(uint32_t *keys[2], uint32_t *vals[2], uint64_t n_bound, const uint32_t *n_dev, int passes, int dbits,
                  const uint32_t *plan_word, uint32_t *hist, bool count_hist, uint32_t *table, uint32_t *st,
                  int cur_word, hipStream_t s) {
  // eight waves per chunk: each ranks 64 RI keys of the chunk
  constexpr uint32_t chunk = RI * 64 * 8;
  const uint32_t nb = (uint32_t)((n_bound + chunk - 1) / chunk);
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((chunk_count_kernel<RI, 8>), dim3(nb), dim3(512), 0, s, keys[0], keys[1], n_dev, n_bound, p,
                       passes, dbits, plan_word, table, nb, count_hist ? hist : nullptr);
    hipLaunchKernelGGL(chunk_scan_kernel, dim3(1u << dbits), dim3(kDigitScanBlock), 0, s, n_dev, n_bound, p, passes,
                       plan_word, (const uint32_t *)hist, table, nb, chunk);
    hipLaunchKernelGGL((chunk_scatter_kernel<RI, 8>), dim3(nb), dim3(512), 0, s, keys[0], vals[0], keys[1], vals[1],
                       n_dev, n_bound, p, passes, dbits, plan_word, (const uint32_t *)table, nb, st, cur_word);
  }
}

// `big`: chunks of 4096 keys (fewer workgroups, longer per-digit runs,
// better coalesced scatters) rather than 1024 (more workgroups).
void radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint64_t n_bound, const uint32_t *n_dev, int bits,
                const uint32_t *plan_word, int hist_mode, uint32_t *hist, uint32_t *table, uint32_t *st,
                int cur_word, bool big, hipStream_t s) {
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  const int dbits = digit_bits_for((uint32_t)bits);
  if (n_bound == 0 || passes == 0) return;
  if (hist_mode == kHistByPass) {
    const uint64_t hb64 = (n_bound + kRadixChunk - 1) / kRadixChunk;
    const unsigned hb = hb64 < 2048 ? (unsigned)hb64 : 2048u;
    hipLaunchKernelGGL(digit_hist_kernel, dim3(hb), dim3(256), 0, s, keys[0], n_dev, n_bound, passes, dbits, hist);
  }
  const bool count_hist = hist_mode == kHistByCount;
  if (big)
    radix_passes<8>(keys, vals, n_bound, n_dev, passes, dbits, plan_word, hist, count_hist, table, st, cur_word, s);
  else
    radix_passes<2>(keys, vals, n_bound, n_dev, passes, dbits, plan_word, hist, count_hist, table, st, cur_word, s);
}

// -------------------------------------------------------------- emission


// Pairs of every kEmitChunk depth-sorted visible records (the pairs one
// emission workgroup writes): each thread sums the active-tile counts of 4
// consecutive records.
__global__ void __launch_bounds__(kEmitChunk / 4) chunk_pairs_kernel(const void *__restrict__ desc,
                                                                     void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t *st = status_of(ws, h);
  const uint32_t nvis = st[S_NVIS];
  const uint32_t vid = blockIdx.x;
  if ((uint64_t)vid * kEmitChunk >= nvis) return;
  const uint32_t *order = ws_ptr<const uint32_t>(ws, h.ws.vis_val[st[S_DEPTH_CUR] ? 1 : 0]);
  const uint32_t *nact = ws_ptr<const uint32_t>(ws, h.ws.nact);
  const uint32_t i0 = vid * kEmitChunk + threadIdx.x * 4;
  uint32_t rec[4], c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) rec[k] = i0 + k < nvis ? order[i0 + k] : 0xffffffffu;
#pragma unroll
  for (int k = 0; k < 4; ++k) c += rec[k] != 0xffffffffu ? nact[rec[k]] : 0u;
  uint32_t tot;
  block_exclusive_scan<kEmitChunk / 256>(c, &tot);
  if (threadIdx.x == 0) ws_ptr<uint32_t>(ws, h.ws.chunk_pairs)[vid] = tot;
}

// Exclusive prefix (64-bit) of the per-chunk pair totals in one workgroup,
// for batches of more than kEmitDirectChunks emission chunks (below that,
// each emission workgroup adds the earlier chunks' totals itself).
constexpr uint64_t kEmitDirectChunks = 2048;
__global__ void __launch_bounds__(1024) chunk_prefix_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t *st = status_of(ws, h);
  const uint32_t nb = (uint32_t)emit_chunks_of(st[S_NVIS]);
  const uint32_t *cp = ws_ptr<const uint32_t>(ws, h.ws.chunk_pairs);
  uint64_t *co = ws_ptr<uint64_t>(ws, h.ws.chunk_off);
  const uint32_t per = (nb + 1023u) / 1024u;
  const uint32_t a = threadIdx.x * per, b = min(nb, a + per);
  uint64_t sum = 0;
  for (uint32_t j = a; j < b; ++j) sum += cp[j];
  __shared__ uint64_t sc[1024];
  sc[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint64_t v = (int)threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t run = sc[threadIdx.x] - sum;
  for (uint32_t j = a; j < b; ++j) {
    co[j] = run;
    run += cp[j];
  }
}

// Pair emission: one workgroup per kEmitChunk depth-sorted records, one
// wave per 64 of them.  The workgroup's first pair is the sum of the pair
// counts of the earlier chunks (summed by chunk_pairs_kernel), its
// records' offsets the workgroup's exclusive scan of their counts; the last
// workgroup writes the pair total and the overflow flag.  Each lane loads
// one record (id, count, rectangle, render) once; the wave
// then emits the records' pairs 64 at a time, every lane finding the record
// of its pair with a six-step search over the lanes' prefix offsets
// (shuffles) and the k-th active tile of that record's rectangle from the
// per-row active-tile bit masks.  Work per lane is balanced whatever the
// spread of rectangle sizes.
constexpr uint32_t kSegRows = 8;  // rectangle rows staged per record in emission
constexpr uint32_t kRowLaneBits = 12;       // widest row (active tiles) of the row-lane emission
constexpr uint32_t kRowLaneMinPairs = 256;  // fewest pairs of a wave in the row-lane emission
// 16 waves per workgroup (one workgroup per emission chunk).
constexpr int kEmitBlock = kEmitChunk;
__global__ void __launch_bounds__(kEmitBlock) emit_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                          int scanned) {
  const Header &h = *header(desc);
  uint32_t *st = status_of(ws, h);
  const uint32_t nvis = st[S_NVIS];
  const uint32_t nb = (uint32_t)emit_chunks_of(nvis);
  const uint32_t vid = blockIdx.x;
  if (vid >= nb) return;  // (uniform per workgroup)
  __shared__ uint32_t s_seg[kEmitBlock / 64][64][kSegRows];  // per wave, per owner record: row bits of its rectangle
  const int lane = threadIdx.x & 63;
  const uint64_t cap = h.pair_capacity;
  const uint64_t i = (uint64_t)vid * kEmitBlock + threadIdx.x;
  const uint64_t wbase = i - lane;
  const bool own = i < nvis;
  const uint32_t rec = own ? ws_ptr<uint32_t>(ws, h.ws.vis_val[st[S_DEPTH_CUR] ? 1 : 0])[i] : 0u;
  const uint32_t cnt = own ? ws_ptr<uint32_t>(ws, h.ws.nact)[rec] : 0u;
  // pairs of the earlier chunks (scanned: their prefix, written by
  // chunk_prefix_kernel), and the chunk's exclusive scan of counts
  __shared__ uint64_t s_pre[kEmitBlock / 64];
  if (!scanned) {
    const uint32_t *cp = ws_ptr<const uint32_t>(ws, h.ws.chunk_pairs);
    uint64_t pre = 0;
    for (uint32_t j = threadIdx.x; j < vid; j += kEmitBlock) pre += cp[j];
    pre = wave_sum64(pre);
    if (lane == 0) s_pre[threadIdx.x >> 6] = pre;
  }
  uint32_t chunk_total;
  const uint32_t ex = block_exclusive_scan<kEmitBlock / 64>(cnt, &chunk_total);  // (its barriers publish s_pre)
  uint64_t prefix = 0;
  if (scanned) {
    prefix = ws_ptr<const uint64_t>(ws, h.ws.chunk_off)[vid];
  } else {
#pragma unroll
    for (int w = 0; w < kEmitBlock / 64; ++w) prefix += s_pre[w];
  }
  if (vid == nb - 1 && threadIdx.x == 0) {
    const uint64_t need = prefix + chunk_total;
    st[S_PAIRS_LO] = (uint32_t)need;
    st[S_PAIRS_HI] = (uint32_t)(need >> 32);
    st[S_OVERFLOW] = need > cap ? 1u : 0u;
    st[S_NPAIRS] = (uint32_t)(need > cap ? cap : need);
  }
  if (own) {
    const uint64_t o = prefix + ex;
    ws_ptr<uint32_t>(ws, h.ws.pair_off)[i] = (uint32_t)(o < cap ? o : cap);
  }
  if (wbase < nvis) {  // uniform per wave
    const uint32_t ex0 = __shfl(ex, 0, 64);
    const uint64_t off0 = prefix + ex0;  // first pair of the wave
    const uint32_t excl = ex - ex0;      // this lane's first pair in the wave
    const uint32_t total = __shfl(ex + cnt, 63, 64) - ex0;
    // this lane's record geometry
    uint32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0, toff = 0, txn = 1, amoff = 0;
    if (own) {
      const int r = upper_index(rec_starts_of(desc), h.n_renders, (uint64_t)rec);
      const DevRender &rd = renders_of(desc)[r];
      const uint2 rr = ws_ptr<uint2>(ws, h.ws.rect)[rec];
      x0 = rr.x & 0xffffu;
      y0 = rr.x >> 16;
      x1 = min(rr.y & 0xffffu, (uint32_t)rd.tiles_x);
      y1 = min(rr.y >> 16, (uint32_t)rd.tiles_y);
      toff = rd.tile_offset;
      txn = rd.tiles_x;
      amoff = rd.amask_offset;
    }
    const uint32_t *am_all = ws_ptr<uint32_t>(ws, h.ws.amask);
    uint32_t *key_out = ws_ptr<uint32_t>(ws, h.ws.pair_key[0]);
    uint32_t *val_out = ws_ptr<uint32_t>(ws, h.ws.pair_val[0]);
    const bool det = h.cfg.deterministic != 0;
    uint32_t *prec = ws_ptr<uint32_t>(ws, h.ws.pair_rec);
    // Every lane, as owner of its record, stages the active-tile bits of its
    // rectangle's rows (bit 0 = column x0) in LDS once, for rectangles of at
    // most kSegRows rows and 32 columns; the pair lanes below then walk rows
    // in LDS instead of issuing dependent global loads.
    uint32_t *seg = s_seg[threadIdx.x >> 6][lane];
    const bool staged = own && y1 - y0 <= kSegRows && x1 - x0 <= 32;
    uint32_t widest = 0;  // most active tiles in one row of this lane's rectangle
    if (staged) {
      const uint32_t wpr = (txn + 31) / 32;
      const uint32_t wd = x1 - x0;
      const uint32_t sh = x0 & 31;
      const uint32_t nr = y1 - y0;
      // every row's words are loaded before the first is used, so the rows
      // cost one round trip rather than one each
      uint32_t lo[kSegRows], hi[kSegRows];
#pragma unroll
      for (uint32_t r = 0; r < kSegRows; ++r) {
        lo[r] = 0u;
        hi[r] = 0u;
        if (r < nr) {
          const uint32_t *row = am_all + amoff + (y0 + r) * wpr + x0 / 32;
          lo[r] = row[0];
          if (sh + wd > 32) hi[r] = row[1];
        }
      }
#pragma unroll
      for (uint32_t r = 0; r < kSegRows; ++r)
        if (r < nr) {
          const uint64_t two = (uint64_t)lo[r] | ((uint64_t)hi[r] << 32);
          seg[r] = (uint32_t)(two >> sh) & (wd == 32 ? ~0u : ((1u << wd) - 1u));
          widest = max(widest, (uint32_t)__popc(seg[r]));
        }
    }
    const uint64_t staged_mask = __ballot(staged);
    __builtin_amdgcn_wave_barrier();
    if (total >= kRowLaneMinPairs && __ballot(own && cnt > 0 && (!staged || widest > kRowLaneBits)) == 0ull) {
      // The wave emits at least kRowLaneMinPairs pairs, every record with
      // pairs is staged and no row has more than kRowLaneBits active tiles:
      // one lane per (record, row) of 8 records at a time.  The lane takes its row's staged active-tile bits and
      // writes that row's pairs in column order after the pairs of the
      // record's earlier rows, so each record's pairs keep their row-major
      // order; no per-pair search.  (Its eight rounds cost about as much as
      // four rounds of the balanced form, and wider rows would leave most
      // lanes idle while a few walk their bits: such waves take the
      // balanced form.)
      const uint32_t nrows = own && cnt > 0 ? y1 - y0 : 0u;
      const uint32_t tile0 = toff + y0 * txn + x0;  // the rectangle's first tile
      const int gl = lane >> 3, row = lane & 7;
      for (int rb = 0; rb < 64; rb += 8) {
        const int src = rb + gl;
        const uint32_t rn = __shfl(nrows, src, 64);
        if (__ballot(rn > 0u) == 0ull) continue;
        const uint32_t bits0 = (uint32_t)row < rn ? s_seg[threadIdx.x >> 6][src][row] : 0u;
        const uint32_t c = __popc(bits0);
        // the record's pairs in its rows above this one
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
          const uint32_t t = __shfl_up(inc, o, 8);
          if (row >= o) inc += t;
        }
        uint64_t e = off0 + __shfl(excl, src, 64) + (inc - c);
        const uint32_t rowtile = __shfl(tile0, src, 64) + (uint32_t)row * __shfl(txn, src, 64);
        const uint32_t orec = __shfl(rec, src, 64);
        uint32_t bits = bits0;
        while (bits) {
          const uint32_t b = (uint32_t)__ffs(bits) - 1u;
          bits &= bits - 1u;
          if (e < cap) {
            const uint32_t gt = rowtile + b;
            key_out[e] = gt;
            if (det) {
              val_out[e] = (uint32_t)e;
              prec[e] = orec;
            } else {
              val_out[e] = orec;
            }
          }
          ++e;
        }
      }
    } else {
      for (uint32_t j = 0; j < total; j += 64) {
        const uint32_t t = j + lane;
        const bool live = t < total && off0 + t < cap;
        // owner: the last lane whose exclusive prefix is <= t
        int owner = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int cand = owner + step;
          const uint32_t ce = __shfl(excl, cand, 64);
          if (ce <= t) owner = cand;
        }
        uint32_t k = t - __shfl(excl, owner, 64);
        const uint32_t orec = __shfl(rec, owner, 64);
        const uint32_t ox0 = __shfl(x0, owner, 64), oy0 = __shfl(y0, owner, 64);
        const uint32_t ox1 = __shfl(x1, owner, 64), oy1 = __shfl(y1, owner, 64);
        const uint32_t otoff = __shfl(toff, owner, 64), otxn = __shfl(txn, owner, 64);
        const uint32_t oam = __shfl(amoff, owner, 64);
        if (live) {
          uint32_t gt = otoff + oy0 * otxn + ox0;  // (the k-th active tile always exists)
          if ((staged_mask >> owner) & 1ull) {
            const uint32_t *os = s_seg[threadIdx.x >> 6][owner];
            for (uint32_t r = 0; r < oy1 - oy0; ++r) {
              uint32_t bits = os[r];
              const uint32_t c = __popc(bits);
              if (k < c) {
                // position of the k-th set bit: halving search on popcounts
                uint32_t pos = 0;
#pragma unroll
                for (uint32_t wdt = 16; wdt > 0; wdt >>= 1) {
                  const uint32_t lo = __popc(bits & ((1u << wdt) - 1u));
                  if (k >= lo) {
                    k -= lo;
                    bits >>= wdt;
                    pos += wdt;
                  }
                }
                gt = otoff + (oy0 + r) * otxn + ox0 + pos;
                break;
              }
              k -= c;
            }
          } else {
            const uint32_t wpr = (otxn + 31) / 32;
            const uint32_t *am = am_all + oam;
            bool found = false;
            for (uint32_t ty = oy0; ty < oy1 && !found; ++ty) {
              for (uint32_t w = ox0 / 32; w * 32 < ox1; ++w) {
                uint32_t bits = am[ty * wpr + w];
                const uint32_t lo32 = w * 32;
                if (ox0 > lo32) bits &= ~0u << (ox0 - lo32);
                if (ox1 < lo32 + 32) bits &= (1u << (ox1 - lo32)) - 1u;
                const uint32_t c = __popc(bits);
                if (k < c) {
                  for (uint32_t q = 0; q < k; ++q) bits &= bits - 1;
                  gt = otoff + ty * otxn + lo32 + (__ffs(bits) - 1);
                  found = true;
                  break;
                }
                k -= c;
              }
            }
          }
          const uint64_t e = off0 + t;
          key_out[e] = gt;
          if (det) {
            // the tile sort carries the emission index; the record follows
            // it through pair_rec (det_fixup_kernel)
            val_out[e] = (uint32_t)e;
            prec[e] = orec;
          } else {
            val_out[e] = orec;
          }
        }
      }
    }
  }
}

// Deterministic mode: the tile sort has carried every pair's emission index
// (record-major order: a record's pairs are consecutive, its tiles in
// row-major order).  Put the record ids in place for the compositing passes
// and keep the inverse permutation (emission index -> tile-sorted index),
// which the backward's segmented reduction walks record by record.
__global__ void __launch_bounds__(256) det_fixup_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t np = status_of(ws, h)[S_NPAIRS];
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  uint32_t *sv = ws_ptr<uint32_t>(ws, h.ws.sorted_val);
  const uint32_t e = sv[j];
  sv[j] = ws_ptr<const uint32_t>(ws, h.ws.pair_rec)[e];
  ws_ptr<uint32_t>(ws, h.ws.pair_inv)[e] = (uint32_t)j;
}

// ------------------------------------------------------------ ranges

// Tile ranges from the tile-sorted pair keys: every thread takes 4
// consecutive pairs and marks where a tile's run starts and ends.
constexpr int kRangeItems = 4;
__global__ void __launch_bounds__(256) ranges_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                     const uint32_t *__restrict__ tiles) {
  const Header &h = *header(desc);
  const uint32_t np = status_of(ws, h)[S_NPAIRS];
  const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
  if (i0 >= np) return;
  uint2 *ranges = ws_ptr<uint2>(ws, h.ws.ranges);
  uint32_t t[kRangeItems + 2];  // tiles[i0 - 1 .. i0 + kRangeItems]
  t[0] = i0 > 0 ? tiles[i0 - 1] : 0xffffffffu;
#pragma unroll
  for (int k = 0; k <= kRangeItems; ++k) t[k + 1] = i0 + k < np ? tiles[i0 + k] : 0xffffffffu;
#pragma unroll
  for (int k = 0; k < kRangeItems; ++k) {
    const uint64_t i = i0 + k;
    if (i >= np) break;
    const uint32_t tk = t[k + 1];
    if (t[k] != tk) ranges[tk].x = (uint32_t)i;
    if (t[k + 2] != tk) ranges[tk].y = (uint32_t)(i + 1);
  }
}

// ------------------------------------------------------------- queue

__device__ inline uint32_t lpt_bucket(uint32_t masked, uint32_t len) {
  if (masked == 0) return 33;             // nothing to render: last
  if (len == 0) return 32;                // masked pixels but no Gaussian
  return (uint32_t)__clz(len);             // longer lists first (0 = longest)
}

// Sort key of every tile for the LPT queue (value: the tile id).
__global__ void queue_key_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_tiles) return;
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[t];
  const uint32_t m = ws_ptr<uint32_t>(ws, h.ws.tile_count)[t];
  ws_ptr<uint32_t>(ws, h.ws.qkey[0])[t] = lpt_bucket(m, rg.y - rg.x);
  ws_ptr<uint32_t>(ws, h.ws.qval0)[t] = (uint32_t)t;
  // tiles with work (masked pixels and pairs): they lead the LPT queue
  const uint64_t busy = __ballot(m > 0 && rg.y > rg.x);
  if ((threadIdx.x & 63) == 0 && busy) atomicAdd(status_of(ws, h) + S_NQUEUE, (uint32_t)__popcll(busy));
}

inline unsigned blocks_for(uint64_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t s, const uint32_t *skip) {
  if (n == 0) return;
  uint64_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, value, n, skip);
}

void launch_tile_mask(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  hipLaunchKernelGGL(tile_mask_kernel, dim3(h.n_tile_rows), dim3(kMaskBlock), 0, s, d_desc, ws);
}

void launch_recount(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  hipLaunchKernelGGL(recount_kernel, dim3(blocks_for(h.n_records)), dim3(256), 0, s, d_desc, ws);
}

void launch_depth_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)chunks_of(h.n_records)), dim3(kCompactBlock), 0, s, d_desc, ws);
  hipLaunchKernelGGL(depth_plan_kernel, dim3(1), dim3(64), 0, s, d_desc, ws);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_key[0]), ws_ptr<uint32_t>(ws, h.ws.vis_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.vis_val[0]), ws_ptr<uint32_t>(ws, h.ws.vis_val[1])};
  // (below four million records the visible ones rarely fill 4096-key
  // chunks on every workgroup of the chip: the depth sort takes 1024 there)
  radix_sort(keys, vals, h.n_records, st + S_NVIS, 32, st + S_PLAN_DEPTH, kHistByProducer, ws_ptr<uint32_t>(ws, h.ws.dhist),
             ws_ptr<uint32_t>(ws, h.ws.rtable), st, S_DEPTH_CUR, h.n_records >= (1ull << 22), s);
}

void launch_emit(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  const dim3 grid((unsigned)emit_chunks_of(h.n_records));
  hipLaunchKernelGGL(chunk_pairs_kernel, grid, dim3(kEmitChunk / 4), 0, s, d_desc, ws);
  const int scanned = emit_chunks_of(h.n_records) > kEmitDirectChunks ? 1 : 0;
  if (scanned) hipLaunchKernelGGL(chunk_prefix_kernel, dim3(1), dim3(1024), 0, s, d_desc, ws);
  hipLaunchKernelGGL(emit_kernel, grid, dim3(kEmitBlock), 0, s, d_desc, ws, scanned);
}

void launch_tile_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  uint32_t *st = ws_ptr<uint32_t>(ws, h.ws.status);
  uint32_t *keys[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_key[0]), ws_ptr<uint32_t>(ws, h.ws.pair_key[1])};
  uint32_t *vals[2] = {ws_ptr<uint32_t>(ws, h.ws.pair_val[0]), ws_ptr<uint32_t>(ws, h.ws.pair_val[1])};
  radix_sort(keys, vals, h.pair_capacity, st + S_NPAIRS, (int)h.tile_bits, nullptr, kHistByCount,
             ws_ptr<uint32_t>(ws, h.ws.thist), ws_ptr<uint32_t>(ws, h.ws.rtable), st, -1,
             h.pair_capacity >= (1ull << 19), s);
  if (h.cfg.deterministic)
    hipLaunchKernelGGL(det_fixup_kernel, dim3(blocks_for(h.pair_capacity)), dim3(256), 0, s, d_desc, ws);
  const uint32_t *sorted_tiles = ws_ptr<uint32_t>(ws, h.ws.sorted_key);
  hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for((h.pair_capacity + kRangeItems - 1) / kRangeItems)), dim3(256), 0, s,
                     d_desc, ws, sorted_tiles);
  if (h.cfg.persistent) {
    // LPT queue: one stable radix pass on the length bucket, so tiles of a
    // bucket keep their (render, row-major) order and stay spatially close
    hipLaunchKernelGGL(queue_key_kernel, dim3(blocks_for(h.n_tiles)), dim3(256), 0, s, d_desc, ws);
    uint32_t *qk[2] = {ws_ptr<uint32_t>(ws, h.ws.qkey[0]), ws_ptr<uint32_t>(ws, h.ws.qkey[1])};
    uint32_t *qv[2] = {ws_ptr<uint32_t>(ws, h.ws.qval0), ws_ptr<uint32_t>(ws, h.ws.queue)};
    radix_sort(qk, qv, h.n_tiles, nullptr, kRadixBits, nullptr, kHistByPass, ws_ptr<uint32_t>(ws, h.ws.qhist),
               ws_ptr<uint32_t>(ws, h.ws.rtable), st, -1, false, s);
  }
}

}  // namespace pgsag
