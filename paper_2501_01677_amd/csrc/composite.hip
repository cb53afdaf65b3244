// Per-tile alpha compositing at building-mask pixels (Sec. 3.1, Eq. 1-4)
// and its backward pass.
//
// Shape: one workgroup per tile of T x T pixels, one lane per pixel (each
// pixel is a GPU thread, Sec. 4.3); a wave covers an 8 x 8 pixel block.  The
// tile's depth-ordered list of projected records is staged through LDS in
// batches (one coalesced 64-byte record load per lane), field-major: plane j
// holds 16-byte field j of every slot, so the lanes that stage or scan
// consecutive slots touch consecutive banks.  After each batch load every
// wave builds its own list of the records that can reach the alpha cut-off
// somewhere in its block -- an exact minimum of the record's quadratic form
// over the block's pixel centres -- compacted with ballots.  A list entry
// carries the record's exponent expanded around the block origin, so that a
// lane evaluates
//     e = log2(o) - q/2 * log2(e)  as  F + D lx + E ly + A lx^2 + B lx ly + C ly^2
// with five FMAs from its constant (lx, ly) offsets, and compares e with
// log2(alpha_min).  Forward entries hold all six coefficients and the slot's
// byte offset (no dependent LDS read per entry), and the entry loop is
// unrolled by two so that its prefetch needs no register copies.  Lanes
// whose pixel is unmasked or whose transmittance has stopped idle; the
// workgroup leaves the tile when no lane is alive (__syncthreads_count).
//
// The backward pass walks the same list back to front from the tile's
// largest last-blended index, recovering each pixel's transmittance before a
// fragment as T_i = T_{i+1} / (1 - alpha_i) from the saved final T, keeps the
// suffix sums of the blended features, and forms each contributing record's
// 13 sums over the wave's 64 pixels (7 feature gradients and 6 moments of
// dL/dq) in one of two ways, chosen at launch: either the wave buffers the
// records' two per-pixel weights (alpha T and dL/dq) in LDS and reduces 8
// records at a time as one small matrix product on the matrix cores, or it
// reduces every record at once with lane exchanges.  Each sum is then added
// with one float atomic.  It builds its lists with the same code as the
// forward pass, so it takes the forward's decisions.
//
// In persistent mode a grid of (CUs x occupancy) workgroups pulls chunks of
// tiles from an LPT-ordered queue with an atomic counter; every workgroup
// leaves once the counter passes the end of the queue.
#include <type_traits>

#include "internal.h"

namespace pgsag {
namespace {

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2

// Records staged per LDS batch (64 for 8x8 tiles, else 128: keeps several
// workgroups resident per CU).
template <int T>
constexpr int batch_of() { return T == 8 ? 64 : (T == 16 ? 96 : 64); }
// Backward batches: 96 records with the matrix-core reduction at T = 16 (its
// per-wave buffers leave room for 5 workgroups per CU only then).
template <int T, bool MM>
constexpr int bwd_batch_of() { return MM && T == 16 ? 96 : (T == 8 ? 64 : 128); }

struct Entry {   // one record in one wave's list of the backward pass (16 bytes)
  float F, D, E;
  uint32_t koff; // slot of the record in the batch * 16 (a byte offset into a field plane)
};

// Field plane j of the staged batch at an entry's slot (planes 0..3: the raw
// record, plane 4: the exponent coefficients A, B, C and the record id).
template <int NT>
__device__ __forceinline__ float4 plane_at(const float4 *sb, uint32_t koff, int j) {
  return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(sb) + koff + j * NT * 16);
}

// One record in one wave's list of the forward pass (32 bytes, two 16-byte
// LDS reads): all six exponent coefficients, so evaluating it needs no
// second, dependent LDS read, and the slot as a byte offset into a field
// plane of the staged batch.
struct FwdEntry {
  float F, D, E, A;  // exponent F + D lx + E ly + A lx^2 + B lx ly + C ly^2
  float B, C;
  uint32_t koff;     // slot * 16
  uint32_t pad;
};

// Field j (0..3) of the record of a forward entry in the staged batch
// (field-major, at LDS offset 0 of the forward kernel).
template <int NT>
__device__ __forceinline__ float4 field_of(const float4 *sb, const FwdEntry &e, int j) {
  return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(sb) + e.koff + j * NT * 16);
}

__device__ __forceinline__ void set_entry(Entry &e, const float4 *sb, int NT, int k, float F, float D, float E) {
  e.F = F;
  e.D = D;
  e.E = E;
  e.koff = (uint32_t)k * 16u;
}

__device__ __forceinline__ void set_entry(FwdEntry &e, const float4 *sb, int NT, int k, float F, float D, float E) {
  const float4 r0 = sb[k];
  e.F = F;
  e.D = D;
  e.E = E;
  e.A = -kHalfLog2e * r0.z;
  e.B = -2.f * kHalfLog2e * r0.w;
  e.C = -kHalfLog2e * sb[NT + k].x;
  e.koff = (uint32_t)k * 16u;
  e.pad = 0u;
}

// Minimum of a x^2 + 2 b x y + c y^2 (a, c > 0, ac > b^2) over the box
// [x0, x1] x [y0, y1]: zero when the box holds the origin, otherwise the
// smallest of the four edge minima.
__device__ __forceinline__ float qmin_box(float a, float b, float c, float x0, float x1, float y0, float y1) {
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
  const float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
  float best = 3.0e38f;
  {
    const float y = y0, x = fminf(fmaxf(-b * y * ia, x0), x1);
    best = fminf(best, a * x * x + 2.f * b * x * y + c * y * y);
  }
  {
    const float y = y1, x = fminf(fmaxf(-b * y * ia, x0), x1);
    best = fminf(best, a * x * x + 2.f * b * x * y + c * y * y);
  }
  {
    const float x = x0, y = fminf(fmaxf(-b * x * ic, y0), y1);
    best = fminf(best, a * x * x + 2.f * b * x * y + c * y * y);
  }
  {
    const float x = x1, y = fminf(fmaxf(-b * x * ic, y0), y1);
    best = fminf(best, a * x * x + 2.f * b * x * y + c * y * y);
  }
  return best;
}

// Builds this wave's list for batch slots [0, cnt): records whose exponent
// can reach log2(alpha_min) (with a small margin) at one of the block's
// pixel centres, with their exponent expansion around the block origin
// (ox, oy).  Returns the list length (uniform across the wave).
template <int NT, typename EntryT>
__device__ __forceinline__ int build_list(const float4 *sb, int cnt, float ox, float oy, float l2min,
                                          EntryT *list) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int len = 0;
  for (int base = 0; base < cnt; base += 64) {
    const int k = base + lane;
    bool pass = false;
    float F = 0.f, D = 0.f, E = 0.f;
    if (k < cnt) {
      const float4 r0 = sb[k];
      const float4 r1 = sb[NT + k];
      const float4 r3 = sb[3 * NT + k];
      const float a = r0.z, b = r0.w, c = r1.x, l2o = r3.w;
      const float dx0 = ox - r0.x, dy0 = oy - r0.y;
      const float qm = qmin_box(a, b, c, dx0, dx0 + 7.f, dy0, dy0 + 7.f);
      pass = l2o - kHalfLog2e * qm >= l2min - 1e-3f;
      if (pass) {
        const float q0 = a * dx0 * dx0 + 2.f * b * dx0 * dy0 + c * dy0 * dy0;
        F = l2o - kHalfLog2e * q0;
        D = -2.f * kHalfLog2e * (a * dx0 + b * dy0);
        E = -2.f * kHalfLog2e * (b * dx0 + c * dy0);
      }
    }
    const uint64_t m = __ballot(pass);
    if (pass) {
      EntryT e;
      set_entry(e, sb, NT, k, F, D, E);
      list[len + __popcll(m & lt)] = e;
    }
    len += __popcll(m);
  }
  __builtin_amdgcn_wave_barrier();
  return len;
}

// Exponent of an entry at this lane: F + D lx + E ly + A lx^2 + B lx ly + C ly^2
// with (A, B, C) = -log2(e)/2 (a, 2b, c), in Horner form
//     F + lx (D + A lx + B ly) + ly (E + C ly)
// (five FMAs on the lane's two offsets).  One instruction sequence shared by
// the forward and backward kernels.
struct LaneOffsets {
  float lx, ly;
};

__device__ __forceinline__ float lane_exponent(const FwdEntry &e, const LaneOffsets &L) {
#pragma clang fp contract(off)
  float u = __builtin_fmaf(e.A, L.lx, e.D);
  u = __builtin_fmaf(e.B, L.ly, u);
  const float w = __builtin_fmaf(e.C, L.ly, e.E);
  float v = __builtin_fmaf(L.lx, u, e.F);
  v = __builtin_fmaf(L.ly, w, v);
  return v;
}

__device__ __forceinline__ float lane_exponent(const Entry &e, const float4 &abc, const LaneOffsets &L) {
#pragma clang fp contract(off)
  float u = __builtin_fmaf(abc.x, L.lx, e.D);
  u = __builtin_fmaf(abc.y, L.ly, u);
  const float w = __builtin_fmaf(abc.z, L.ly, e.E);
  float v = __builtin_fmaf(L.lx, u, e.F);
  v = __builtin_fmaf(L.ly, w, v);
  return v;
}

struct TileGeom {
  const DevRender *rd;
  int px, py;   // pixel of this lane
  bool inside;
  float ox, oy; // pixel centre of the wave's block origin
  LaneOffsets L;
};

template <int T>
__device__ __forceinline__ void tile_geom(const void *desc, const Header &h, uint32_t tile, TileGeom &g) {
  const int r = upper_index(tile_starts_of(desc), h.n_renders, tile);
  const DevRender &rd = renders_of(desc)[r];
  g.rd = &rd;
  const uint32_t local = tile - rd.tile_offset;
  const int tx = (int)(local % (uint32_t)rd.tiles_x), ty = (int)(local / (uint32_t)rd.tiles_x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int SB = T / 8;  // 8x8 blocks per tile side
  const int sbx = wave % SB, sby = wave / SB;
  const int bx = tx * T + sbx * 8, by = ty * T + sby * 8;
  const int lx = lane & 7, ly = lane >> 3;
  g.px = bx + lx;
  g.py = by + ly;
  g.inside = g.px < rd.cam.W && g.py < rd.cam.H;
  g.ox = bx + 0.5f;
  g.oy = by + 0.5f;
  g.L.lx = (float)lx;
  g.L.ly = (float)ly;
}

// Stages batch records [j0, j1) into LDS: the raw 64-byte records and (ABC)
// the per-record exponent coefficients (A, B, C) with the record id.
template <int NT, bool ABC>
__device__ __forceinline__ void stage_batch(const float4 *__restrict__ rec4, const uint32_t *__restrict__ vals,
                                            uint32_t j0, uint32_t j1, float4 *sb) {
  const uint32_t j = j0 + threadIdx.x;
  if (threadIdx.x < NT && j < j1) {
    const uint32_t rid = vals[j];
    const float4 *src = rec4 + (uint64_t)rid * 4;
    const float4 r0 = src[0], r1 = src[1];
    const float4 r2 = src[2], r3 = src[3];
    sb[threadIdx.x] = r0;
    sb[NT + threadIdx.x] = r1;
    sb[2 * NT + threadIdx.x] = r2;
    sb[3 * NT + threadIdx.x] = r3;
    if constexpr (ABC)
      sb[4 * NT + threadIdx.x] =
          make_float4(-kHalfLog2e * r0.z, -2.f * kHalfLog2e * r0.w, -kHalfLog2e * r1.x, __uint_as_float(rid));
  }
}

template <int T>
__device__ void forward_tile(const void *__restrict__ desc, const Header &h, void *__restrict__ ws, uint32_t tile,
                             float4 *srec, FwdEntry (*lists)[batch_of<T>()],
                             const uint32_t *__restrict__ vals) {
  constexpr int NT = batch_of<T>();
  TileGeom g;
  tile_geom<T>(desc, h, tile, g);
  const DevRender &rd = *g.rd;
  const int W = rd.cam.W;
  const uint64_t pix = (uint64_t)g.py * W + g.px;
  // a tile without masked pixels only writes its zeros (no mask reads)
  const bool active = ws_ptr<const uint32_t>(ws, h.ws.tile_count)[tile] != 0;
  const bool masked = active && g.inside && (rd.mask == nullptr || rd.mask[pix] != 0);
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[tile];
  const float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  const float amax = h.cfg.alpha_max, tmin = h.cfg.t_min;
  const float l2min = __log2f(h.cfg.alpha_min);
  FwdEntry *list = lists[threadIdx.x >> 6];
  uint32_t nev = 0;  // list entries this wave evaluated (each for all its 64 lanes)
  // The transmittance carries the lane's state in its sign: negative once
  // the lane has stopped (or for an unmasked pixel), so a stopped lane's
  // next candidate transmittance is negative too and it never blends again.
  float Tr = masked ? 1.f : -1.f;
  float F[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int32_t n = 0, last = -1;
  for (uint32_t b = rg.x; b < rg.y; b += NT) {
    if (__syncthreads_count(Tr > 0.f) == 0) break;
    const uint32_t b1 = min(rg.y, b + NT);
    stage_batch<NT, false>(rec4, vals, b, b1, srec);
    __syncthreads();
    if (__ballot(Tr > 0.f) == 0ull) continue;
    const int len = build_list<NT>(srec, (int)(b1 - b), g.ox, g.oy, l2min, list);
    // Branch-free over the lanes (selects, no divergent blocks).  The slot
    // of the last blended record of this batch is kept and turned into the
    // pair index once per batch.
    int lastk = -1;
    const auto eval = [&](const FwdEntry &e) {
      const float ex = lane_exponent(e, g.L);
      const bool pass = ex >= l2min;
      // exp2 >= 0: the median of (x, 0, amax) is min(x, amax) in one instruction
      const float a = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(ex), 0.f, amax);
      const float aT = a * Tr;
      const float Tn = Tr - aT;
      const bool low = Tn < tmin;
      const bool stop = pass && low;
      const bool blend = pass && !low;
      const float4 r1 = field_of<NT>(srec, e, 1), r2 = field_of<NT>(srec, e, 2);
      const float d = field_of<NT>(srec, e, 3).x;
      const float w = blend ? aT : 0.f;
      F[0] = fmaf(w, r1.z, F[0]);
      F[1] = fmaf(w, r1.w, F[1]);
      F[2] = fmaf(w, r2.x, F[2]);
      F[3] = fmaf(w, r2.y, F[3]);
      F[4] = fmaf(w, r2.z, F[4]);
      F[5] = fmaf(w, r2.w, F[5]);
      F[6] = fmaf(w, d, F[6]);
      Tr = blend ? Tn : (stop ? -fabsf(Tr) : Tr);
      n += blend ? 1 : 0;
      lastk = blend ? (int)e.koff : lastk;
    };
    // two entries per iteration: `e` is loop-carried and reloaded after
    // its evaluation, `f` is loaded and used within the iteration
    FwdEntry e = list[0];
    int t = 0;
    while (t < len) {
      const FwdEntry f = list[t + 1 < len ? t + 1 : t];
      eval(e);
      if (t + 1 >= len) {
        t += 1;
        break;
      }
      e = list[t + 2 < len ? t + 2 : t + 1];
      eval(f);
      t += 2;
      if ((t & 7) == 0 && __ballot(Tr > 0.f) == 0ull) break;
    }
    nev += (uint32_t)t;
    if (lastk >= 0) last = (int32_t)(b + ((uint32_t)lastk >> 4));
  }
  // work counter of this (tile, wave): [0] forward entries evaluated
  if ((threadIdx.x & 63) == 0)
    ws_ptr<uint32_t>(ws, h.ws.work)[((uint64_t)tile * ((T / 8) * (T / 8)) + (threadIdx.x >> 6)) * 3] = nev;
  Tr = fabsf(Tr);
  if (!g.inside) return;
  const uint64_t HW = (uint64_t)rd.cam.H * W;
  float rgb0 = 0.f, rgb1 = 0.f, rgb2 = 0.f, alpha = 0.f, depth = 0.f;
  const float fx = g.px + 0.5f, fy = g.py + 0.5f;
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

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), CTRL, 0xf, 0xf, false));
}

// Sum of v[0..15] over the 64 lanes of a wave by recursive halving, using
// only VALU lane exchanges: permlane32/16 swaps for lane distance 32 and 16,
// DPP row rotate by 8, half-row mirror and quad permutations below that.
// Each step keeps half of the values per lane and adds the partner lane's
// copy of them.  Afterwards lane L holds the total of value (L >> 2) & 15.
__device__ __forceinline__ float wave_reduce16(const float v[16]) {
  const int lane = threadIdx.x & 63;
  float w8[8], w4[4], w2[2];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    // lanes 0..31 keep v[s], lanes 32..63 keep v[8 + s]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[s]), __float_as_uint(v[8 + s]), false, false);
    w8[s] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    // lanes with bit 4 clear keep w8[s], the others w8[4 + s]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w8[s]), __float_as_uint(w8[4 + s]), false, false);
    w4[s] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool hi = lane & 8;  // partner: lane ^ 8 (row rotate by 8)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float mine = hi ? w4[2 + s] : w4[s];
      const float send = hi ? w4[s] : w4[2 + s];
      w2[s] = mine + dpp<0x128>(send);
    }
  }
  const bool hi = lane & 4;  // partner: mirrored lane in the same 8-lane half row
  float x = (hi ? w2[1] : w2[0]) + dpp<0x141>(hi ? w2[0] : w2[1]);
  x += dpp<0x4e>(x);  // quad permutation: lane ^ 2
  x += dpp<0xb1>(x);  // quad permutation: lane ^ 1
  return x;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// A wave's per-record sum goes to the record's 2D-gradient slot with a float
// atomic, or (deterministic mode) is stored to the slot of its own (tile
// pair, wave), which nothing else writes.
template <bool DET>
__device__ __forceinline__ void add_or_store(float *p, float v) {
  if constexpr (DET) *p = v;
  else unsafeAtomicAdd(p, v);
}

// Per-wave LDS of the backward pass's per-record reduction.  For up to 8
// contributing records the wave buffers every pixel's colour weight
// w = alpha T (rows 0..7) and alpha times the dL/dalpha gate, i.e.
// -2 dL/dq (rows 8..15); columns are the wave's 64 pixels, stored in 4-float
// granules XOR-swizzled by (row & 7) so that the matrix-layout reads of a
// flush spread over the banks.  info[b] holds buffered record b's id (bits)
// and 2D mean.
struct WaveAcc {
  float a[16][64];
  float4 info[8];
};

// Feature slot n of a pixel in the per-record reduction: the 7 output
// gradients (slots 0..6), then monomials of the pixel's offset (x, y) from
// the block centre: slot 8: 1, 9: x, 10: y, 11: xy, 12: x^2, 13: y^2,
// 14: x, 15: y (slot 7 is zero).
__device__ __forceinline__ float feature_slot(int n, float g, float x, float y) {
  const int ex = (n == 9 || n == 11 || n == 14) ? 1 : (n == 12 ? 2 : 0);
  const int ey = (n == 10 || n == 11 || n == 15) ? 1 : (n == 13 ? 2 : 0);
  const float px = ex == 0 ? 1.f : (ex == 1 ? x : x * x);
  const float py = ey == 0 ? 1.f : (ey == 1 ? y : y * y);
  return n < 7 ? g : (n == 7 ? 0.f : px * py);
}

// Reduces the buffered records over the wave's pixels on the matrix cores:
// C = F^T A^T with A the 16 x 64 buffer and F[p][n] = feature slot n of
// pixel p, in sixteen 16x16x4 FP32 MFMA steps (pixel p of step 4t + j and
// lane group kk being 16t + 4kk + j; bf holds the F operands).  Lane
// (j, kk) receives slots 4kk..4kk+3 of buffered row j: for rows 0..7 (colour
// weights of record j) slots 0..6 are its 7 feature gradients; for rows
// 8..15 (alpha gate = -2 dL/dq of record j - 8) slots 8..13 are the raw
// moments R_1, R_x, R_y, R_xy, R_xx, R_yy about the block centre, which are
// moved to the record's centre with its offset (cx, cy) from the block
// centre:
//   sum u dx = R_x - cx R_1,  sum u dx dy = R_xy - cx R_y - cy R_x + cx cy R_1,
//   sum u dx^2 = R_xx - 2 cx R_x + cx^2 R_1  (lane group 3 takes R_1 from
// group 2), and scaled by -1/2 (exact) to moments of dL/dq, except
// sum(alpha gate) = R_1 itself.  Every valid nonzero value of the first nb
// records is then added to its slot (dst + id * STRIDE), or with DET stored
// there (the slot belongs to this wave and record alone).
template <int STRIDE, bool DET>
__device__ __forceinline__ void flush_records(WaveAcc &acc, int nb, const float (&bf)[16], uint32_t fields,
                                              float bcx, float bcy, float *__restrict__ dst) {
  const int lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
  // two independent accumulation chains (pixel halves), interleaved, so
  // that each MFMA issues while the previous one of the other chain is in
  // flight
  floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const float4 a0 = *reinterpret_cast<const float4 *>(&acc.a[j][((4 * t + kk) ^ (j & 7)) << 2]);
    const float4 a1 = *reinterpret_cast<const float4 *>(&acc.a[j][((4 * (t + 2) + kk) ^ (j & 7)) << 2]);
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * t + 0], a0.x, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * (t + 2) + 0], a1.x, c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * t + 1], a0.y, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * (t + 2) + 1], a1.y, c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * t + 2], a0.z, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * (t + 2) + 2], a1.z, c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * t + 3], a0.w, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[4 * (t + 2) + 3], a1.w, c1, 0, 0, 0);
  }
  const floatx4 c = c0 + c1;
  const int b = j & 7;  // buffered record
  const float4 ib = acc.info[b];
  const float cx = ib.y - bcx, cy = ib.z - bcy;
  // lane group 3 needs R_1 (slot 8, held in c[0] by group 2)
  const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(c[0]), __float_as_uint(c[0]), false, false);
  const float r1 = __uint_as_float(sw[0]);
  // group 2 holds R_1, R_x, R_y, R_xy; group 3 R_xx, R_yy (then R_x, R_y);
  // groups 0 and 1 pass through (branch-free, per-lane 0/1 factors)
  const float s2 = kk == 2 ? 1.f : 0.f, s3 = kk == 3 ? 1.f : 0.f;
  const float cx2 = s2 * cx, cy2 = s2 * cy, cx3 = s3 * cx, cy3 = s3 * cy;
  float o[4];
  o[0] = fmaf(-3.f * s2, c[0], c[0]) + cx3 * fmaf(cx, r1, -2.f * c[2]);
  o[1] = c[1] - cx2 * c[0] + cy3 * fmaf(cy, r1, -2.f * c[3]);
  o[2] = c[2] - cy2 * c[0];
  o[3] = c[3] - cx2 * fmaf(-cy, c[0], c[2]) - cy2 * c[1];
  // (group 2's o[0] is -2 R_1 here: the common factor brings it back)
  const float sc = kk >= 2 ? -0.5f : 1.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] *= sc;
  // The sums go out record-major: staged as 8 rows of 16 fields in the
  // buffer (free once read), then each atomic instruction covers 4 records,
  // so that a record's 13 additions fall in one instruction and cache line.
  // Slots of the other row type go to the unused field 15.
  float *stage = &acc.a[0][0];
  const uint32_t fl = ((kk < 2) == (j < 8)) ? fields : 0x0f0f0f0fu;
#pragma unroll
  for (int r = 0; r < 4; ++r) stage[b * 16 + ((fl >> (8 * r)) & 0xffu)] = o[r];
  __builtin_amdgcn_wave_barrier();
  const int rb = lane >> 4, f = lane & 15;
  const float v0 = stage[rb * 16 + f], v1 = stage[(4 + rb) * 16 + f];
  const uint32_t id0 = __float_as_uint(acc.info[rb].x), id1 = __float_as_uint(acc.info[4 + rb].x);
  if (f < 13) {
    if (rb < nb && v0 != 0.f) add_or_store<DET>(dst + (uint64_t)id0 * STRIDE + f, v0);
    if (4 + rb < nb && v1 != 0.f) add_or_store<DET>(dst + (uint64_t)id1 * STRIDE + f, v1);
  }
}

// G2 fields of this lane's output slots 4kk..4kk+3 in flush_records, one
// byte each (15: no output).
__device__ __forceinline__ uint32_t slot_fields(int kk) {
  return kk == 0 ? (G_R | G_G << 8 | G_B << 16 | (uint32_t)G_NX << 24)
         : kk == 1 ? (G_NY | G_NZ << 8 | G_D << 16 | 15u << 24)
         : kk == 2 ? (G_SO | G_SX << 8 | G_SY << 16 | (uint32_t)G_SXY << 24)
                   : (G_SXX | G_SYY << 8 | 0x0f0fu << 16);
}

// MM: the per-record sums are formed on the matrix cores from LDS-buffered
// weights (flush_records); otherwise every record is reduced across the wave
// at once with lane exchanges (wave_reduce16) and added by one atomic
// instruction.  Same sums, different speed: the matrix-core form spends
// fewer instructions per record, the lane-exchange form less per tile and
// fewer registers and LDS (twice the resident workgroups).
//
// DET (deterministic mode): instead of float atomics into the record's slot,
// each wave stores its sums for a record into the slot of (tile-sorted pair
// index, wave); det_reduce_kernel adds them per record in a fixed order.
template <int T, bool MM, bool DET>
__device__ __forceinline__ void backward_tile(const void *__restrict__ desc, const Header &h, void *__restrict__ ws, uint32_t tile,
                              float4 *sb, Entry (*lists)[bwd_batch_of<T, MM>()],
                              WaveAcc *accs, int *smax, const uint32_t *__restrict__ vals) {
  constexpr int NT = bwd_batch_of<T, MM>();
  constexpr int WPT = (T / 8) * (T / 8);
  constexpr int STRIDE = DET ? WPT * kG2 : kG2;
  // work counters of this (tile, wave): [1] backward entries evaluated, [2]
  // of them with a contributing lane
  uint32_t *work = ws_ptr<uint32_t>(ws, h.ws.work) + ((uint64_t)tile * WPT + (threadIdx.x >> 6)) * 3;
  // nothing to do for a tile without masked pixels (uniform over the workgroup)
  if (ws_ptr<const uint32_t>(ws, h.ws.tile_count)[tile] == 0) {
    if ((threadIdx.x & 63) == 0) work[1] = work[2] = 0u;
    return;
  }
  TileGeom g;
  tile_geom<T>(desc, h, tile, g);
  const DevRender &rd = *g.rd;
  const int W = rd.cam.W;
  const uint64_t pix = (uint64_t)g.py * W + g.px;
  const uint64_t HW = (uint64_t)rd.cam.H * W;
  const bool masked = g.inside && (rd.mask == nullptr || rd.mask[pix] != 0);
  const uint2 rg = ws_ptr<uint2>(ws, h.ws.ranges)[tile];
  const float4 *rec4 = ws_ptr<float4>(ws, h.ws.rec);
  // where the per-record sums go: slot id * STRIDE of dst (id = record, or
  // with DET the tile-sorted pair index; the wave picks its slot of the pair)
  float *dst = DET ? ws_ptr<float>(ws, h.ws.part) + (threadIdx.x >> 6) * kG2 : ws_ptr<float>(ws, h.ws.g2);
  const float amax = h.cfg.alpha_max;
  const float l2min = __log2f(h.cfg.alpha_min);
  const float fx = g.px + 0.5f, fy = g.py + 0.5f;
  Entry *list = lists[threadIdx.x >> 6];

  int32_t last = -1;
  float Tr = 1.f, Tf = 1.f;
  float gch[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float ga = 0.f;
  // dL/d(soft count): every blended fragment's alpha enters the pixel's
  // soft count with weight 1 (the count output's gradient)
  float gcount = 0.f;
  // H = g_alpha T_final - sum_c g_c S_c, S_c the blended features behind the
  // current fragment (plus the background term): dL/dalpha only needs this
  // difference, so it is kept instead of the seven suffix sums.
  float H = 0.f;
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
    if (rd.g_count) gcount = rd.g_count[pix];
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
    H = ga * Tf - Tf * (gch[0] * h.cfg.bg[0] + gch[1] * h.cfg.bg[1] + gch[2] * h.cfg.bg[2]);
  }
  // the tile's largest last-blended index (with MM from a wave maximum by
  // lane exchanges and one LDS atomic per wave; the lane-exchange form keeps
  // per-lane atomics, whose registers it cannot spare)
  int32_t wlast = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
  wlast = __builtin_amdgcn_readfirstlane(wlast);  // uniform: keep it scalar
  if (threadIdx.x == 0) *smax = -1;
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && wlast >= 0) atomicMax(smax, wlast);
  __syncthreads();
  const int maxlast = *smax;
  if (maxlast < (int)rg.x) {  // uniform: no pixel blended anything
    if ((threadIdx.x & 63) == 0) work[1] = work[2] = 0u;
    return;
  }
  uint32_t nev = 0, nact = 0;
  const uint32_t end = (uint32_t)maxlast + 1;
  // With MM, records past the wave's own largest last-blended index
  // contribute to none of its pixels and stay out of its lists.  (The
  // lane-exchange form keeps every record of the tile's range; the limit
  // costs it a wave of occupancy.)
  if constexpr (!MM) wlast = maxlast;
  const int lane = threadIdx.x & 63;
  // the features of the reduction (see flush_records), fixed for the tile:
  // the output gradients of the other pixels come through the wave's buffer
  WaveAcc &acc = accs[threadIdx.x >> 6];
  float bf[16];
  if constexpr (MM) {
#pragma unroll
    for (int c = 0; c < 7; ++c) acc.a[c][lane] = gch[c];
    __builtin_amdgcn_wave_barrier();
    const int n = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int p = ((i >> 2) << 4) + (kk << 2) + (i & 3);
      bf[i] = feature_slot(n, acc.a[n < 7 ? n : 0][p], (float)(p & 7) - 3.5f, (float)(p >> 3) - 3.5f);
    }
    __builtin_amdgcn_wave_barrier();
  }
  const float bcx = g.ox + 3.5f, bcy = g.oy + 3.5f;  // block centre
  const uint32_t fields = slot_fields(lane >> 4);
  int nb = 0;  // buffered records (uniform)
  // Lane b < nb holds the slot (koff) of buffered record b; its id and 2D
  // mean are copied to acc.info by lanes [ninfo, nb) before a flush or the
  // next batch's staging (one masked write per group, not per record).
  uint32_t bkoff = 0u;
  int ninfo = 0;  // (uniform)
  for (int64_t bend = end; bend > (int64_t)rg.x; bend -= NT) {
    const uint32_t bstart = (uint32_t)max((int64_t)rg.x, bend - NT);
    const int cnt = (int)((uint32_t)bend - bstart);
    __syncthreads();
    stage_batch<NT, true>(rec4, vals, bstart, (uint32_t)bend, sb);
    __syncthreads();
    const auto copy_info = [&](int upto) {
      if (lane >= ninfo && lane < upto) {
        const float4 r0 = plane_at<NT>(sb, bkoff, 0);
        const uint32_t id = DET ? bstart + (bkoff >> 4) : __float_as_uint(plane_at<NT>(sb, bkoff, 4).w);
        acc.info[lane] = make_float4(__uint_as_float(id), r0.x, r0.y, 0.f);
      }
      ninfo = upto;
    };
    if (MM ? wlast >= (int32_t)bstart : __ballot(last >= (int32_t)bstart) != 0ull) {
      const int len = build_list<NT>(sb, MM ? min(cnt, wlast - (int32_t)bstart + 1) : cnt, g.ox, g.oy, l2min, list);
      nev += (uint32_t)len;
      if constexpr (!MM) {
        for (int t = len - 1; t >= 0; --t) {
          const Entry cur = list[t];
          const uint32_t ck = cur.koff >> 4;
          const int32_t idx = (int32_t)(bstart + ck);
          const float4 abc = plane_at<NT>(sb, cur.koff, 4);
          // Every lane evaluates the fragment (the wave executes it anyway when
          // any lane contributes); lanes that do not contribute get zero weight.
          const float ex = lane_exponent(cur, abc, g.L);
          const bool contrib = idx <= last && ex >= l2min;
          if (__ballot(contrib) == 0ull) continue;
          ++nact;
          const float raw = __builtin_amdgcn_exp2f(ex);
          const float a = __builtin_amdgcn_fmed3f(raw, 0.f, amax);  // min(raw, amax), raw >= 0
          const float4 r0 = plane_at<NT>(sb, cur.koff, 0), r1 = plane_at<NT>(sb, cur.koff, 1);
          const float4 r2 = plane_at<NT>(sb, cur.koff, 2), r3 = plane_at<NT>(sb, cur.koff, 3);
          const float f[7] = {r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
          const float iom = __builtin_amdgcn_rcpf(1.f - a);  // 1 / (1 - alpha), alpha <= 0.99
          const float Tp = Tr * iom;
          const float w = contrib ? a * Tp : 0.f;
          // dL/dalpha = sum_c g_c (T f_c - S_c / (1 - alpha)) + g_alpha T_final / (1 - alpha)
          //            + g_count
          float Gf = 0.f;
          float v[16];
#pragma unroll
          for (int c = 0; c < 7; ++c) {
            Gf = fmaf(gch[c], f[c], Gf);
            v[6 + c] = w * gch[c];
          }
          const float dLda = fmaf(Tp, Gf, fmaf(H, iom, gcount));
          H = contrib ? fmaf(-w, Gf, H) : H;
          Tr = contrib ? Tp : Tr;
          // alpha = o G with G = exp(-q/2): dalpha/do = G = alpha / o,
          // dalpha/dq = -alpha / 2 (zero on the clamped side of alpha_max)
          const float gate = (contrib && raw <= amax) ? dLda : 0.f;
          const float dx = fx - r0.x, dy = fy - r0.y;
          // moments only: the record's conic and 1/o are applied once per
          // record after the reduction (see G2Field)
          const float ag = a * gate;
          const float dLdq = -0.5f * ag;
          const float qx = dLdq * dx, qy = dLdq * dy;
          v[G_SO] = ag;
          v[G_SX] = qx;
          v[G_SY] = qy;
          v[G_SXX] = qx * dx;
          v[G_SXY] = qx * dy;
          v[G_SYY] = qy * dy;
          v[13] = v[14] = v[15] = 0.f;
          const float tot = wave_reduce16(v);
          const int which = (lane >> 2) & 15;
          if ((lane & 3) == 0 && which < 13 && tot != 0.f)
            add_or_store<DET>(dst + (uint64_t)(DET ? bstart + ck : __float_as_uint(abc.w)) * STRIDE + which, tot);
        }
      } else {
        // Back to front.  A lane that does not blend the fragment takes alpha
        // = 0: its weight w and its dL/dq entry vanish, its transmittance
        // and suffix term are unchanged (T / (1 - 0) = T and H - 0 Gf = H
        // exactly), so the recurrences need no per-value selects.
        // the pixel's last blended index as a byte offset into the batch
        // planes (below 0: none of the batch)
        const int32_t lastoff = min(max(last - (int32_t)bstart, -1), NT) * 16;
        auto step = [&](const Entry &e, const float4 &abc) {
          const float ex = lane_exponent(e, abc, g.L);
          const bool contrib = (int32_t)e.koff <= lastoff && ex >= l2min;
          if (__ballot(contrib) == 0ull) return;
          const float4 r1 = plane_at<NT>(sb, e.koff, 1);
          const float4 r2 = plane_at<NT>(sb, e.koff, 2), r3 = plane_at<NT>(sb, e.koff, 3);
          const float raw = __builtin_amdgcn_exp2f(ex);
          const float a = contrib ? __builtin_amdgcn_fmed3f(raw, 0.f, amax) : 0.f;  // min(raw, amax), raw >= 0
          const float f[7] = {r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
          const float iom = __builtin_amdgcn_rcpf(1.f - a);  // 1 / (1 - alpha), alpha <= 0.99
          const float Tp = Tr * iom;
          const float w = a * Tp;
          // dL/dalpha = sum_c g_c (T f_c - S_c / (1 - alpha)) + g_alpha T_final / (1 - alpha)
          //            + g_count
          float Gf = 0.f;
#pragma unroll
          for (int c = 0; c < 7; ++c) Gf = fmaf(gch[c], f[c], Gf);
          const float dLda = fmaf(Tp, Gf, fmaf(H, iom, gcount));
          H = fmaf(-w, Gf, H);
          Tr = Tp;
          // alpha = o G with G = exp(-q/2): dalpha/do = G = alpha / o,
          // dalpha/dq = -alpha / 2 (zero on the clamped side of alpha_max)
          const float gate = raw <= amax ? dLda : 0.f;
          // buffer w and dL/dq; the record's sums over the wave's pixels
          // are formed on the matrix cores once 8 records are buffered
          // (granule (lane >> 2) of row nb lands at (lane >> 2) ^ nb)
          const int col = lane ^ (nb << 2);
          acc.a[nb][col] = w;
          acc.a[8 + nb][col] = a * gate;
          bkoff = lane == nb ? e.koff : bkoff;
          if (++nb == 8) {
            nact += 8;
            copy_info(8);
            __builtin_amdgcn_wave_barrier();
            flush_records<STRIDE, DET>(acc, 8, bf, fields, bcx, bcy, dst);
            __builtin_amdgcn_wave_barrier();
            nb = 0;
            ninfo = 0;
          }
        };
        // the next entry is read while this one is evaluated (its
        // coefficients, read through the entry's slot, are not: a second
        // prefetched register set would spill)
        Entry e = list[len > 0 ? len - 1 : 0];
        for (int t = len - 1; t >= 0; --t) {
          const Entry en = list[t > 0 ? t - 1 : 0];
          step(e, plane_at<NT>(sb, e.koff, 4));
          e = en;
        }
        copy_info(nb);  // the batch's slots are restaged next
      }
    }
  }
  if (MM && nb > 0) {
    nact += (uint32_t)nb;
    __builtin_amdgcn_wave_barrier();
    flush_records<STRIDE, DET>(acc, nb, bf, fields, bcx, bcy, dst);
  }
  if ((threadIdx.x & 63) == 0) {
    work[1] = nev;
    work[2] = nact;
  }
}

// Tiles per queue pop in persistent mode: the configured chunk, reduced
// when there are fewer than two chunks of tiles with work per workgroup (the
// queue leads with the longest tiles, so large pops would hand the few busy
// tiles to a few workgroups).
__device__ __forceinline__ uint32_t queue_chunk_for(const Header &h, void *ws) {
  const uint32_t busy = ws_ptr<const uint32_t>(ws, h.ws.status)[S_NQUEUE];
  const uint32_t fit = busy / (2u * gridDim.x);
  return max(1u, min((uint32_t)h.cfg.queue_chunk, fit));
}

template <int T>
__global__ void __launch_bounds__(T *T) __attribute__((amdgpu_waves_per_eu(8))) forward_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                        const uint32_t *__restrict__ vals) {
  constexpr int NT = batch_of<T>();
  // one LDS block with the staged batch first, at offset 0 (forward
  // entries hold byte offsets into it); the batch is field-major: plane j
  // (0..3) holds field j of every slot, so a wave reading or writing
  // consecutive slots touches consecutive banks
  struct Smem {
    float4 sb[4 * NT];
    FwdEntry lists[T * T / 64][NT];
    uint32_t item;
  };
  __shared__ Smem sm;
  float4 *sb = sm.sb;
  FwdEntry (*lists)[NT] = sm.lists;
  uint32_t &s_item = sm.item;
  const Header &h = *header(desc);
  if (h.any_grads && !h.cfg.deterministic) {
    // The backward's 2D-gradient slots are cleared here, spread over the
    // grid: this kernel is bound by its arithmetic, so the stores cost
    // little, and the backward then skips its own clearing pass.
    uint4 *g2 = ws_ptr<uint4>(ws, h.ws.g2);
    const uint64_t nv = h.n_records * (uint64_t)kG2 / 4;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (uint64_t)gridDim.x * blockDim.x)
      g2[v] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x == 0) ws_ptr<uint32_t>(ws, h.ws.status)[S_G2_CLEAN] = 1u;
  }
  if (!h.cfg.persistent) {
    forward_tile<T>(desc, h, ws, blockIdx.x, sb, lists, vals);
    return;
  }
  uint32_t *ctr = ws_ptr<uint32_t>(ws, h.ws.status) + S_QUEUE_FWD;
  const uint32_t *queue = ws_ptr<uint32_t>(ws, h.ws.queue);
  const uint32_t chunk = queue_chunk_for(h, ws);
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
      forward_tile<T>(desc, h, ws, queue[it], sb, lists, vals);
    }
  }
}

// Registers sized for the occupancy the LDS allows with MM: 5 workgroups
// per CU at T = 16 (96-record batches, 30.6 KB; 96 VGPRs, the per-tile
// constants spill to scratch outside the record loop), 4 waves per SIMD
// otherwise.
template <int T, bool MM, bool DET>
__global__ void __launch_bounds__(T *T) __attribute__((amdgpu_waves_per_eu(MM ? (T == 16 ? 5 : 4) : 8))) backward_kernel(const void *__restrict__ desc, void *__restrict__ ws,
                                                         const uint32_t *__restrict__ vals) {
  constexpr int NT = bwd_batch_of<T, MM>();
  __shared__ float4 sb[5 * NT];  // field-major staged batch (see forward_kernel)
  __shared__ Entry lists[T * T / 64][NT];
  __shared__ std::conditional_t<MM, WaveAcc, uint32_t> accs_[T * T / 64];
  WaveAcc *accs = reinterpret_cast<WaveAcc *>(accs_);
  __shared__ int smax;
  __shared__ uint32_t s_item;
  const Header &h = *header(desc);
  // the slots this pass accumulates into are no longer clean for the next one
  if (blockIdx.x == 0 && threadIdx.x == 0) ws_ptr<uint32_t>(ws, h.ws.status)[S_G2_CLEAN] = 0u;
  if (!h.cfg.persistent) {
    backward_tile<T, MM, DET>(desc, h, ws, blockIdx.x, sb, lists, accs, &smax, vals);
    return;
  }
  uint32_t *ctr = ws_ptr<uint32_t>(ws, h.ws.status) + S_QUEUE_BWD;
  const uint32_t *queue = ws_ptr<uint32_t>(ws, h.ws.queue);
  const uint32_t chunk = queue_chunk_for(h, ws);
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
      backward_tile<T, MM, DET>(desc, h, ws, queue[it], sb, lists, accs, &smax, vals);
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

template <int T, bool DET>
void launch_bwd_td(const void *d, const Header &h, void *ws, hipStream_t s) {
  const uint32_t *vals = ws_ptr<uint32_t>(ws, h.ws.sorted_val);
  const unsigned grid = h.cfg.persistent ? persistent_grid(h) : (unsigned)h.n_tiles;
  if (h.cfg.bwd_reduce == 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(backward_kernel<T, true, DET>), dim3(grid), dim3(T * T), 0, s, d, ws, vals);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(backward_kernel<T, false, DET>), dim3(grid), dim3(T * T), 0, s, d, ws, vals);
}

template <int T>
void launch_bwd_t(const void *d, const Header &h, void *ws, hipStream_t s) {
  if (h.cfg.deterministic) launch_bwd_td<T, true>(d, h, ws, s);
  else launch_bwd_td<T, false>(d, h, ws, s);
}

// Deterministic mode: zero the (pair, wave) slots of the pairs of this
// forward (a pair/wave slot that no wave writes must read as zero).
__global__ void __launch_bounds__(256) det_clear_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint64_t np = ws_ptr<const uint32_t>(ws, h.ws.status)[S_NPAIRS];
  const uint64_t n4 = np * (uint64_t)waves_per_tile(h.cfg.tile) * (kG2 / 4);
  float4 *p = ws_ptr<float4>(ws, h.ws.part);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Deterministic mode: the segmented reduction.  One thread per visible
// record (depth order): its pairs are emission indices [pair_off, pair_off
// + active tiles) -- its active tiles in row-major order -- and each maps to
// its tile-sorted slot through the inverse permutation.  The record's 13
// sums are added over its pairs in that order and over the waves of each
// tile in index order, then written (not added) to its 2D-gradient slot.
template <int WPT>
__global__ void __launch_bounds__(256) det_reduce_kernel(const void *__restrict__ desc, void *__restrict__ ws) {
  const Header &h = *header(desc);
  const uint32_t *st = ws_ptr<const uint32_t>(ws, h.ws.status);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st[S_NVIS]) return;
  const uint32_t rid = ws_ptr<const uint32_t>(ws, h.ws.vis_val[st[S_DEPTH_CUR] ? 1 : 0])[i];
  const uint64_t e0 = ws_ptr<const uint32_t>(ws, h.ws.pair_off)[i];
  const uint64_t e1 = min(e0 + ws_ptr<const uint32_t>(ws, h.ws.nact)[rid], (uint64_t)st[S_NPAIRS]);
  const uint32_t *inv = ws_ptr<const uint32_t>(ws, h.ws.pair_inv);
  const float4 *part = ws_ptr<const float4>(ws, h.ws.part);
  float s[13];
#pragma unroll
  for (int f = 0; f < 13; ++f) s[f] = 0.f;
  for (uint64_t e = e0; e < e1; ++e) {
    const uint64_t j = inv[e];
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      const float4 *q = part + (j * WPT + w) * (kG2 / 4);
      const float4 a = q[0], b = q[1], c = q[2], d = q[3];
      s[0] += a.x; s[1] += a.y; s[2] += a.z; s[3] += a.w;
      s[4] += b.x; s[5] += b.y; s[6] += b.z; s[7] += b.w;
      s[8] += c.x; s[9] += c.y; s[10] += c.z; s[11] += c.w;
      s[12] += d.x;
    }
  }
  float *g = ws_ptr<float>(ws, h.ws.g2) + (uint64_t)rid * kG2;
#pragma unroll
  for (int f = 0; f < 13; ++f) g[f] = s[f];
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

void launch_det_clear(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.pair_capacity == 0) return;
  uint64_t blocks = (h.pair_capacity * waves_per_tile(h.cfg.tile) * (kG2 / 4) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(det_clear_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_desc, ws);
}

void launch_det_reduce(const void *d_desc, const Header &h, void *ws, hipStream_t s) {
  if (h.n_records == 0) return;
  const dim3 grid((unsigned)((h.n_records + 255) / 256));
  switch (h.cfg.tile) {
    case 8: hipLaunchKernelGGL(det_reduce_kernel<1>, grid, dim3(256), 0, s, d_desc, ws); break;
    case 16: hipLaunchKernelGGL(det_reduce_kernel<4>, grid, dim3(256), 0, s, d_desc, ws); break;
    default: hipLaunchKernelGGL(det_reduce_kernel<16>, grid, dim3(256), 0, s, d_desc, ws); break;
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
