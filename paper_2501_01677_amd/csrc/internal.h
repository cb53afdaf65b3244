// Internal definitions shared by the kernels and the host side of libpgsag:
// the packed descriptor (what the device reads), workspace layout, and small
// device helpers.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgsag.h"

namespace pgsag {

constexpr uint32_t kMagic = 0x50475341u;  // "PGSA"
constexpr int kRec = 16;                  // floats per projected record
constexpr int kG2 = 16;                   // floats per 2D-gradient slot
constexpr int kScanItems = 16;            // items per thread in scans / sorts
constexpr int kScanBlock = 256;           // threads per scan / sort block
constexpr int kScanChunk = kScanItems * kScanBlock;  // 4096 elements per block
constexpr int kRadixItems = 4;            // keys per thread in a radix pass
constexpr int kRadixChunk = kRadixItems * kScanBlock;  // 1024 keys per radix chunk
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
// Digit histograms are kept in kHistCopies copies of uint32 [4][256], each
// producing workgroup adding into copy (workgroup & 7): fewer same-word
// atomics per copy; the consumers add the copies.
constexpr int kHistCopies = 8;
constexpr int kHistStride = 4 * kRadixBins;

// Record layout (floats): projected Gaussian for one (render, Gaussian).
enum RecField {
  R_MX = 0, R_MY = 1,              // 2D mean (pixels)
  R_CA = 2, R_CB = 3, R_CC = 4,    // conic: q = a dx^2 + 2 b dx dy + c dy^2
  R_O = 5,                         // opacity
  R_R = 6, R_G = 7, R_B = 8,       // colour
  R_NX = 9, R_NY = 10, R_NZ = 11,  // camera-frame normal
  R_D = 12,                        // plane distance
  R_INV_O = 13,                    // 1 / opacity
  R_RX = 14,                       // support half-width in x (pixels, with margin)
  R_LOG2O = 15                     // log2(opacity)
};

// 2D-gradient slot layout (floats): per record, sums over the blended
// pixels p of dL/dq_p times the offset moments (d = p - mean2d), of
// dL/dalpha_p alpha_p on the unclamped side, and of the feature gradients.
// The record's conic (a, b, c) and 1/o are applied once per record by the
// backward projection:  dL/dmean = -2 [a b; b c] (S_x, S_y),
// dL/d(a, b, c) = (S_xx, 2 S_xy, S_yy),  dL/do = S_o / o.
enum G2Field {
  G_SX = 0, G_SY = 1, G_SXX = 2, G_SXY = 3, G_SYY = 4, G_SO = 5,
  G_R = 6, G_G = 7, G_B = 8, G_NX = 9, G_NY = 10, G_NZ = 11, G_D = 12
};

struct DevCamera {
  int32_t W, H;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float centre[3];  // camera centre in world coordinates, -R^T t
  float limx, limy; // lateral clamp of the projection Jacobian
};

struct DevSet {
  const float *means, *log_scales, *quats, *logits, *sh;
  float *g_means, *g_log_scales, *g_quats, *g_logits, *g_sh;
  int64_t n;
  int32_t sh_degree;
  int32_t n_renders;
  uint64_t gauss_offset;  // prefix of n over sets
  int32_t renders[64];    // render indices drawing this set (n_renders <= 64)
};

struct DevRender {
  DevCamera cam;
  int32_t set, tiles_x, tiles_y, reserved;
  const uint8_t *mask;
  float *o_rgb, *o_normal, *o_dist, *o_depth, *o_alpha;
  int32_t *o_ncontrib;
  const float *g_rgb, *g_normal, *g_dist, *g_depth, *g_alpha, *g_count;
  uint64_t record_offset;  // first record of this render
  uint64_t pixel_offset;   // first per-pixel state slot
  uint32_t tile_offset;    // first global tile id
  uint32_t sat_offset;     // first row-prefix entry (tiles_y rows of tiles_x+1)
  uint32_t row_offset;     // first global tile row
  uint32_t amask_offset;   // first word of the active-tile bit mask (rows of ceil(tiles_x/32) words)
};

struct Layout {
  uint64_t status, tile_count, sat, ranges, queue, rec, depth_key, rect, nact;
  uint64_t vis_key[2], vis_val[2], pair_off;
  uint64_t amask;  // uint32 active-tile bit masks
  uint64_t pair_key[2], pair_val[2];
  uint64_t sorted_key, sorted_val;  // the pair buffers holding the tile-sorted result
  uint64_t pix_T, pix_last, g2;
  // uint32 [n_tiles][waves per tile][3] compositing work per (tile, wave):
  // forward list entries evaluated, backward entries evaluated, backward
  // entries with a contributing lane
  uint64_t work;
  // Deterministic backward only (0 otherwise): the record of every emitted
  // pair (uint32 [capacity], emission order), and one 16-float slot per
  // (tile-sorted pair, wave of the tile) for the backward compositing sums.
  // After the tile sort the spare pair-value buffer holds the inverse
  // permutation (emission index -> tile-sorted index).
  uint64_t pair_rec, part, pair_inv;
  // Region [zero_begin, zero_end) is cleared at the start of every forward:
  // status words, single-pass scan look-back words, digit histograms,
  // radix look-back words and the queue buckets.
  uint64_t zero_begin;
  uint64_t lb_compact;  // uint64 [blocks] look-back words of the compaction scan
  uint64_t dhist, thist;         // uint32 [kHistCopies][4][256] digit histograms (depth, tile)
  uint64_t qhist;                // the same for the queue sort
  uint64_t zero_end;
  uint64_t chunk_pairs;          // uint32 [records / kEmitChunk] pairs of each chunk of depth-sorted records
  uint64_t chunk_off;            // uint64 [records / kEmitChunk] their exclusive prefix (large batches)
  uint64_t rtable;               // uint32 [256][chunks] radix chunk offsets
  uint64_t qkey[2], qval0;       // queue sort buffers (the result lands in `queue`)
  uint64_t stats;
  uint64_t loss;       // double [n_renders][8] loss accumulators
  uint64_t loss_part;  // double [n_renders][64][4] partial sums of the loss terms
  uint64_t end;
};

// Status word layout (uint32 view of ws + layout.status).
enum StatusField {
  S_PAIRS_LO = 0, S_PAIRS_HI = 1, S_OVERFLOW = 2, S_NVIS = 3,
  S_QUEUE_FWD = 4, S_QUEUE_BWD = 5, S_NPAIRS = 6, S_NQUEUE = 7,
  S_DEPTH_CUR = 8,   // which vis buffer holds the depth-sorted records
  S_ERROR = 9,       // non-zero if a look-back wait gave up (results invalid)
  S_PLAN_DEPTH = 10, // bit p set: depth-sort pass p is skipped (one digit for every key)
  S_G2_CLEAN = 11,   // non-zero: the forward compositing has cleared the 2D-gradient slots
  S_CTR_COMPACT = 16,  // chunk tickets of the compaction's look-back scan
  S_WORDS = 64
};

struct Header {
  uint32_t magic, abi;
  int32_t n_sets, n_renders;
  pgsag_config cfg;
  uint64_t n_gauss, n_records, n_tiles, n_pixels, pair_capacity;
  uint32_t sat_total, tile_bits, n_tile_rows, max_sh_degree;
  uint64_t sets_off, renders_off, tile_starts_off, rec_starts_off, row_starts_off;
  uint64_t desc_bytes, ws_bytes;
  int32_t any_grads, reserved;
  // Sets grouped by SH degree for the degree-specialised projection kernels:
  // deg_ids[d] -> int32 [deg_count[d]] set indices, deg_starts[d] -> uint32
  // [deg_count[d] + 1] prefix of 256-thread blocks.
  uint64_t deg_ids_off[4], deg_starts_off[4];
  int32_t deg_count[4];
  uint32_t deg_blocks[4];
  Layout ws;
};

__host__ __device__ inline const Header *header(const void *d) {
  return reinterpret_cast<const Header *>(d);
}
__host__ __device__ inline const DevSet *sets_of(const void *d) {
  return reinterpret_cast<const DevSet *>(static_cast<const char *>(d) + header(d)->sets_off);
}
__host__ __device__ inline const DevRender *renders_of(const void *d) {
  return reinterpret_cast<const DevRender *>(static_cast<const char *>(d) + header(d)->renders_off);
}
// uint32 [n_renders + 1] prefix arrays used for binary searches
__host__ __device__ inline const uint32_t *tile_starts_of(const void *d) {
  return reinterpret_cast<const uint32_t *>(static_cast<const char *>(d) + header(d)->tile_starts_off);
}
__host__ __device__ inline const uint32_t *row_starts_of(const void *d) {
  return reinterpret_cast<const uint32_t *>(static_cast<const char *>(d) + header(d)->row_starts_off);
}
__host__ __device__ inline const uint64_t *rec_starts_of(const void *d) {
  return reinterpret_cast<const uint64_t *>(static_cast<const char *>(d) + header(d)->rec_starts_off);
}

template <typename T>
__host__ __device__ inline T *ws_ptr(void *ws, uint64_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}
template <typename T>
__host__ __device__ inline const T *ws_ptr(const void *ws, uint64_t off) {
  return reinterpret_cast<const T *>(static_cast<const char *>(ws) + off);
}

__host__ __device__ inline const int32_t *deg_ids_of(const void *d, int k) {
  return reinterpret_cast<const int32_t *>(static_cast<const char *>(d) + header(d)->deg_ids_off[k]);
}
__host__ __device__ inline const uint32_t *deg_starts_of(const void *d, int k) {
  return reinterpret_cast<const uint32_t *>(static_cast<const char *>(d) + header(d)->deg_starts_off[k]);
}

// Largest i in [0, n) with a[i] <= x (a ascending, a[0] == 0).
template <typename T>
__device__ inline int upper_index(const T *a, int n, T x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Error reporting of the C ABI (thread-local message read by
// pgsag_last_error): set_error stores the formatted message and returns
// `code`; hip_status turns a pending HIP launch error into PGSAG_HIP_ERROR.
int set_error(int code, const char *fmt, ...);
int hip_status(const char *where);

// ---------------------------------------------------------------- launches
// Host-side launch helpers, defined in the kernel translation units.
// (skip: a device word; when it is non-zero at run time nothing is written)
void launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t s, const uint32_t *skip = nullptr);
void launch_tile_mask(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_preprocess(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_recount(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_depth_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_emit(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_tile_sort(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_composite(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_backward_composite(const void *d_desc, const Header &h, void *ws, hipStream_t s);
// Deterministic backward: clears the per-(pair, wave) slots before the
// compositing pass and adds every record's slots in a fixed order after it.
void launch_det_clear(const void *d_desc, const Header &h, void *ws, hipStream_t s);
void launch_det_reduce(const void *d_desc, const Header &h, void *ws, hipStream_t s);
// Waves (8 x 8 pixel blocks) per tile.
__host__ __device__ inline int waves_per_tile(int tile) { return (tile / 8) * (tile / 8); }
// Adam folded into the backward projection (a disabled instance writes the
// plain gradients).  coef: the step's bias corrections (two floats).
struct AdamArgs {
  float lr, b1, b2, eps;
  const float *coef;
  int64_t m_off, v_off;  // moments at (gradient pointer + offset) floats
  int32_t enabled, write_grads;
};
void launch_backward_preprocess(const void *d_desc, const Header &h, void *ws, const AdamArgs &adam, hipStream_t s);
void launch_adam_coef(int32_t *state, float b1, float b2, hipStream_t s);
void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t step, int32_t *state, hipStream_t s);
void launch_loss(const void *d_desc, const void *h_desc, void *ws, const pgsag_loss_config &lc,
                 const float *const *gt, const float *const *weight, float *out, hipStream_t s);
void launch_luminance_weights(const void *d_desc, const void *h_desc, void *ws, int r, const float *gt,
                              float *weight, hipStream_t s);
void launch_load_stats(const void *d_desc, const Header &h, const void *ws, int r,
                       const float *pixel_weight, float *out, hipStream_t s);

// Blocks of kScanChunk elements covering n.
__host__ __device__ inline uint64_t chunks_of(uint64_t n) { return (n + kScanChunk - 1) / kScanChunk; }
__host__ __device__ inline uint64_t radix_chunks_of(uint64_t n) { return (n + kRadixChunk - 1) / kRadixChunk; }
// Depth-sorted visible records are emitted in chunks of kEmitChunk, one
// workgroup each.
constexpr int kEmitChunk = 1024;
__host__ __device__ inline uint64_t emit_chunks_of(uint64_t n) { return (n + kEmitChunk - 1) / kEmitChunk; }
constexpr int kDepthPasses = 4;
__host__ __device__ inline int tile_passes(uint32_t tile_bits) { return (int)((tile_bits + kRadixBits - 1) / kRadixBits); }
// Digit width of a sort over `bits` key bits: the passes of at most
// kRadixBits each, with the bits spread evenly over them (fewer digits per
// pass give longer runs per digit in a chunk, so better coalesced scatters).
__host__ __device__ inline int digit_bits_for(uint32_t bits) {
  const uint32_t passes = (bits + kRadixBits - 1) / kRadixBits;
  return passes ? (int)((bits + passes - 1) / passes) : kRadixBits;
}

}  // namespace pgsag
