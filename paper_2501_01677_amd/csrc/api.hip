// Host side of the C ABI declared in include/pgsag.h: validation, planning
// of the workspace, packing of the device descriptor and the stage-by-stage
// enqueue of the forward and backward passes.  No device allocation, no
// synchronisation (except pgsag_read_status), no global mutable state except
// the thread-local error string.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace pgsag;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int check_hip(const char *where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PGSAG_HIP_ERROR, "%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
  return PGSAG_OK;
}

}  // namespace

namespace pgsag {

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_status(const char *where) { return check_hip(where); }

}  // namespace pgsag

namespace {

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Sizes {
  uint64_t n_gauss = 0, n_records = 0, n_tiles = 0, n_pixels = 0, sat_total = 0, n_tile_rows = 0;
  uint64_t amask_words = 0;
  uint32_t tile_bits = 0;
  int max_deg = 0;
};

int validate(const pgsag_config *cfg, const pgsag_gaussians *sets, int32_t n_sets, const pgsag_render *renders,
             int32_t n_renders, uint64_t cap, Sizes &z) {
  if (!cfg || !sets || !renders) return fail(PGSAG_INVALID_ARGUMENT, "null config, sets or renders");
  if (cfg->tile != 8 && cfg->tile != 16 && cfg->tile != 32)
    return fail(PGSAG_INVALID_ARGUMENT, "tile must be 8, 16 or 32 (got %d)", cfg->tile);
  if (n_sets < 1 || n_renders < 1) return fail(PGSAG_INVALID_ARGUMENT, "need at least one set and one render");
  if (n_renders > 4096) return fail(PGSAG_UNSUPPORTED, "at most 4096 renders per batch");
  if (cfg->bwd_reduce != 0 && cfg->bwd_reduce != 1)
    return fail(PGSAG_INVALID_ARGUMENT, "bwd_reduce must be 0 or 1 (got %d)", cfg->bwd_reduce);
  if (cfg->deterministic != 0 && cfg->deterministic != 1)
    return fail(PGSAG_INVALID_ARGUMENT, "deterministic must be 0 or 1 (got %d)", cfg->deterministic);
  if (cfg->persistent && (cfg->queue_chunk < 1 || cfg->queue_chunk > 64))
    return fail(PGSAG_INVALID_ARGUMENT, "queue_chunk must be in 1..64");
  if (cfg->persistent && (cfg->workgroups_per_cu < 1 || cfg->workgroups_per_cu > 16))
    return fail(PGSAG_INVALID_ARGUMENT, "workgroups_per_cu must be in 1..16");
  if (!(cfg->alpha_min > 0.f && cfg->alpha_min < cfg->alpha_max && cfg->alpha_max < 1.f))
    return fail(PGSAG_INVALID_ARGUMENT, "need 0 < alpha_min < alpha_max < 1");
  if (!(cfg->t_min > 0.f && cfg->t_min < 1.f)) return fail(PGSAG_INVALID_ARGUMENT, "need 0 < t_min < 1");
  if (!(cfg->z_near > 0.f) || !(cfg->fov_clamp > 0.f) || !(cfg->dilation >= 0.f))
    return fail(PGSAG_INVALID_ARGUMENT, "need z_near > 0, fov_clamp > 0, dilation >= 0");
  if (cap < 1 || cap > 0x3fffffffull) return fail(PGSAG_INVALID_ARGUMENT, "pair_capacity must be in 1..2^30-1");
  std::vector<int> per_set(n_sets, 0);
  for (int s = 0; s < n_sets; ++s) {
    if (sets[s].n < 0) return fail(PGSAG_INVALID_ARGUMENT, "set %d: n < 0", s);
    if (sets[s].sh_degree < 0 || sets[s].sh_degree > 3)
      return fail(PGSAG_INVALID_ARGUMENT, "set %d: sh_degree must be 0..3", s);
    z.n_gauss += (uint64_t)sets[s].n;
    if (sets[s].sh_degree > z.max_deg) z.max_deg = sets[s].sh_degree;
  }
  const int T = cfg->tile;
  for (int r = 0; r < n_renders; ++r) {
    const pgsag_render &rd = renders[r];
    if (rd.set < 0 || rd.set >= n_sets) return fail(PGSAG_INVALID_ARGUMENT, "render %d: set %d out of range", r, rd.set);
    if (++per_set[rd.set] > 64) return fail(PGSAG_UNSUPPORTED, "set %d: more than 64 renders", rd.set);
    const pgsag_camera &c = rd.cam;
    if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
      return fail(PGSAG_INVALID_ARGUMENT, "render %d: image size %dx%d outside 1..65535", r, c.width, c.height);
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(PGSAG_INVALID_ARGUMENT, "render %d: focal lengths must be > 0", r);
    const uint64_t tx = (c.width + T - 1) / T, ty = (c.height + T - 1) / T;
    z.n_tiles += tx * ty;
    z.sat_total += (tx + 1) * (ty + 1);
    z.n_tile_rows += ty;
    z.amask_words += ty * ((tx + 31) / 32);
    z.n_pixels += (uint64_t)c.width * c.height;
    z.n_records += (uint64_t)sets[rd.set].n;
  }
  if (z.n_tiles >= 0xffffffffull || z.n_records >= 0x3fffffffull || z.sat_total >= 0xffffffffull)
    return fail(PGSAG_UNSUPPORTED, "batch too large: records must stay below 2^30, tiles below 2^32");
  uint32_t bits = 0;
  while (bits < 32 && (1ull << bits) < z.n_tiles) ++bits;
  z.tile_bits = bits;
  return PGSAG_OK;
}

Layout make_layout(const pgsag_config &cfg, const Sizes &z, uint64_t cap, int n_renders) {
  Layout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align_up(off + (bytes ? bytes : 4), 256);
    return o;
  };
  L.tile_count = take(z.n_tiles * 4);
  L.sat = take(z.sat_total * 4);
  L.amask = take(z.amask_words * 4);
  L.ranges = take(z.n_tiles * 8);
  L.queue = take(z.n_tiles * 4);
  L.rec = take(z.n_records * kRec * 4);
  L.depth_key = take(z.n_records * 4);
  L.rect = take(z.n_records * 8);
  L.nact = take(z.n_records * 4);
  for (int k = 0; k < 2; ++k) L.vis_key[k] = take(z.n_records * 4);
  for (int k = 0; k < 2; ++k) L.vis_val[k] = take(z.n_records * 4);
  L.pair_off = take(z.n_records * 4);
  for (int k = 0; k < 2; ++k) L.pair_key[k] = take(cap * 4);
  for (int k = 0; k < 2; ++k) L.pair_val[k] = take(cap * 4);
  const int passes = tile_passes(z.tile_bits);
  L.sorted_key = L.pair_key[passes & 1];
  L.sorted_val = L.pair_val[passes & 1];
  L.pix_T = take(z.n_pixels * 4);
  L.pix_last = take(z.n_pixels * 4);
  L.g2 = take(z.n_records * kG2 * 4);
  L.work = take(z.n_tiles * (uint64_t)waves_per_tile(cfg.tile) * 3 * 4);
  if (cfg.deterministic) {
    L.pair_rec = take(cap * 4);
    L.part = take(cap * (uint64_t)waves_per_tile(cfg.tile) * kG2 * 4);
    L.pair_inv = L.pair_val[(passes & 1) ^ 1];
  }
  // contiguous zero-initialised region (status words first)
  L.zero_begin = off;
  const uint64_t status_at = take(S_WORDS * 4);
  L.lb_compact = take((chunks_of(z.n_records) + 1) * 8);
  L.dhist = take(kHistCopies * kHistStride * 4);
  L.thist = take(kHistCopies * kHistStride * 4);
  L.qhist = take(kHistCopies * kHistStride * 4);
  L.zero_end = off;
  L.chunk_pairs = take(emit_chunks_of(z.n_records) * 4);
  L.chunk_off = take(emit_chunks_of(z.n_records) * 8);
  {
    uint64_t big = z.n_records > cap ? z.n_records : cap;
    big = big > z.n_tiles ? big : z.n_tiles;
    L.rtable = take((radix_chunks_of(big) + 1) * 256 * 4);
  }
  for (int k = 0; k < 2; ++k) L.qkey[k] = take(z.n_tiles * 4);
  L.qval0 = take(z.n_tiles * 4);
  L.status = status_at;
  L.stats = take((uint64_t)n_renders * 8 * 8);
  L.loss = take((uint64_t)n_renders * 8 * 8);
  L.loss_part = take((uint64_t)n_renders * 64 * 4 * 8);
  L.end = off;
  return L;
}

struct DescLayout {
  uint64_t sets_off, renders_off, tile_starts_off, row_starts_off, rec_starts_off;
  uint64_t deg_ids_off[4], deg_starts_off[4];
  uint64_t bytes;
};

DescLayout desc_layout(int n_sets, int n_renders) {
  DescLayout d{};
  uint64_t off = align_up(sizeof(Header), 64);
  d.sets_off = off;
  off = align_up(off + sizeof(DevSet) * n_sets, 64);
  d.renders_off = off;
  off = align_up(off + sizeof(DevRender) * n_renders, 64);
  d.tile_starts_off = off;
  off = align_up(off + 4ull * (n_renders + 1), 64);
  d.row_starts_off = off;
  off = align_up(off + 4ull * (n_renders + 1), 64);
  d.rec_starts_off = off;
  off = align_up(off + 8ull * (n_renders + 1), 64);
  for (int k = 0; k < 4; ++k) {
    d.deg_ids_off[k] = off;
    off = align_up(off + 4ull * n_sets, 64);
    d.deg_starts_off[k] = off;
    off = align_up(off + 4ull * (n_sets + 1), 64);
  }
  d.bytes = off;
  return d;
}

const Header *check_desc(const void *host_desc) {
  if (!host_desc) {
    fail(PGSAG_INVALID_ARGUMENT, "null descriptor");
    return nullptr;
  }
  const Header *h = header(host_desc);
  if (h->magic != kMagic || h->abi != PGSAG_ABI_VERSION) {
    fail(PGSAG_INVALID_ARGUMENT, "descriptor was not packed by this library version");
    return nullptr;
  }
  return h;
}

struct StageTimer {
  void **ev;
  hipStream_t s;
  void begin(int k) const {
    if (ev) (void)hipEventRecord(static_cast<hipEvent_t>(ev[2 * k]), s);
  }
  void end(int k) const {
    if (ev) (void)hipEventRecord(static_cast<hipEvent_t>(ev[2 * k + 1]), s);
  }
};

int check_run_args(const Header *h, const void *dev_desc, void *ws, size_t ws_bytes) {
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!dev_desc || !ws) return fail(PGSAG_INVALID_ARGUMENT, "null device descriptor or workspace");
  if (ws_bytes < h->ws_bytes)
    return fail(PGSAG_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %llu", ws_bytes,
                (unsigned long long)h->ws_bytes);
  return PGSAG_OK;
}

}  // namespace

extern "C" {

int pgsag_version(void) { return PGSAG_ABI_VERSION; }

const char *pgsag_last_error(void) { return g_error.c_str(); }

void pgsag_default_config(pgsag_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->tile = 16;
  cfg->persistent = 0;
  cfg->queue_chunk = 1;
  cfg->workgroups_per_cu = 4;
  cfg->alpha_min = 1.0f / 255.0f;
  cfg->t_min = 1e-4f;
  cfg->alpha_max = 0.99f;
  cfg->dilation = 0.3f;
  cfg->z_near = 0.2f;
  cfg->fov_clamp = 1.3f;
  cfg->logit_min = (float)(-std::log(254.0));
  cfg->depth_guard = 1e-6f;
}

int pgsag_plan(const pgsag_config *cfg, const pgsag_gaussians *sets, int32_t n_sets, const pgsag_render *renders,
               int32_t n_renders, uint64_t pair_capacity, pgsag_plan_info *out) {
  if (!out) return fail(PGSAG_INVALID_ARGUMENT, "null output");
  Sizes z;
  int rc = validate(cfg, sets, n_sets, renders, n_renders, pair_capacity, z);
  if (rc) return rc;
  const Layout L = make_layout(*cfg, z, pair_capacity, n_renders);
  const DescLayout d = desc_layout(n_sets, n_renders);
  std::memset(out, 0, sizeof *out);
  out->workspace_bytes = L.end;
  out->desc_bytes = d.bytes;
  out->n_records = z.n_records;
  out->n_tiles = z.n_tiles;
  out->n_pixels = z.n_pixels;
  out->pair_capacity = pair_capacity;
  out->tile_bits = (int32_t)z.tile_bits;
  return PGSAG_OK;
}

int pgsag_pack(const pgsag_config *cfg, const pgsag_gaussians *sets, const pgsag_grads *set_grads, int32_t n_sets,
               const pgsag_render *renders, int32_t n_renders, uint64_t pair_capacity, void *host_desc,
               size_t desc_bytes) {
  Sizes z;
  int rc = validate(cfg, sets, n_sets, renders, n_renders, pair_capacity, z);
  if (rc) return rc;
  const DescLayout d = desc_layout(n_sets, n_renders);
  if (!host_desc) return fail(PGSAG_INVALID_ARGUMENT, "null descriptor buffer");
  if (desc_bytes < d.bytes)
    return fail(PGSAG_WORKSPACE_TOO_SMALL, "descriptor buffer has %zu bytes, needs %llu", desc_bytes,
                (unsigned long long)d.bytes);
  for (int s = 0; s < n_sets; ++s) {
    const pgsag_gaussians &g = sets[s];
    if (g.n > 0 && (!g.means || !g.log_scales || !g.quats || !g.opacity_logits || !g.sh))
      return fail(PGSAG_INVALID_ARGUMENT, "set %d: null parameter pointer", s);
  }
  std::memset(host_desc, 0, d.bytes);
  char *base = static_cast<char *>(host_desc);
  Header *h = reinterpret_cast<Header *>(base);
  h->magic = kMagic;
  h->abi = PGSAG_ABI_VERSION;
  h->n_sets = n_sets;
  h->n_renders = n_renders;
  h->cfg = *cfg;
  h->n_gauss = z.n_gauss;
  h->n_records = z.n_records;
  h->n_tiles = z.n_tiles;
  h->n_pixels = z.n_pixels;
  h->pair_capacity = pair_capacity;
  h->sat_total = (uint32_t)z.sat_total;
  h->tile_bits = z.tile_bits;
  h->n_tile_rows = (uint32_t)z.n_tile_rows;
  h->max_sh_degree = (uint32_t)z.max_deg;
  h->sets_off = d.sets_off;
  h->renders_off = d.renders_off;
  h->tile_starts_off = d.tile_starts_off;
  h->row_starts_off = d.row_starts_off;
  h->rec_starts_off = d.rec_starts_off;
  h->desc_bytes = d.bytes;
  h->ws = make_layout(*cfg, z, pair_capacity, n_renders);
  h->ws_bytes = h->ws.end;
  h->any_grads = set_grads != nullptr;
  for (int k = 0; k < 4; ++k) {
    h->deg_ids_off[k] = d.deg_ids_off[k];
    h->deg_starts_off[k] = d.deg_starts_off[k];
    int32_t *ids = reinterpret_cast<int32_t *>(base + d.deg_ids_off[k]);
    uint32_t *starts = reinterpret_cast<uint32_t *>(base + d.deg_starts_off[k]);
    uint32_t blocks = 0;
    int cnt = 0;
    for (int s2 = 0; s2 < n_sets; ++s2) {
      if (sets[s2].sh_degree != k || sets[s2].n == 0) continue;
      ids[cnt] = s2;
      starts[cnt] = blocks;
      blocks += (uint32_t)((sets[s2].n + 255) / 256);
      ++cnt;
    }
    starts[cnt] = blocks;
    h->deg_count[k] = cnt;
    h->deg_blocks[k] = blocks;
  }

  DevSet *ds = reinterpret_cast<DevSet *>(base + d.sets_off);
  uint64_t goff = 0;
  for (int s = 0; s < n_sets; ++s) {
    const pgsag_gaussians &g = sets[s];
    DevSet &o = ds[s];
    o.means = g.means;
    o.log_scales = g.log_scales;
    o.quats = g.quats;
    o.logits = g.opacity_logits;
    o.sh = g.sh;
    if (set_grads) {
      o.g_means = set_grads[s].means;
      o.g_log_scales = set_grads[s].log_scales;
      o.g_quats = set_grads[s].quats;
      o.g_logits = set_grads[s].opacity_logits;
      o.g_sh = set_grads[s].sh;
    }
    o.n = g.n;
    o.sh_degree = g.sh_degree;
    o.n_renders = 0;
    o.gauss_offset = goff;
    goff += (uint64_t)g.n;
  }
  DevRender *dr = reinterpret_cast<DevRender *>(base + d.renders_off);
  uint32_t *tile_starts = reinterpret_cast<uint32_t *>(base + d.tile_starts_off);
  uint32_t *row_starts = reinterpret_cast<uint32_t *>(base + d.row_starts_off);
  uint64_t *rec_starts = reinterpret_cast<uint64_t *>(base + d.rec_starts_off);
  uint64_t toff = 0, rowoff = 0, satoff = 0, recoff = 0, pixoff = 0, amoff = 0;
  const int T = cfg->tile;
  for (int r = 0; r < n_renders; ++r) {
    const pgsag_render &in = renders[r];
    DevRender &o = dr[r];
    const pgsag_camera &c = in.cam;
    if (in.gout.depth && (!in.out.normal || !in.out.dist))
      return fail(PGSAG_INVALID_ARGUMENT, "render %d: a depth gradient needs the normal and dist outputs", r);
    o.cam.W = c.width;
    o.cam.H = c.height;
    o.cam.fx = c.fx;
    o.cam.fy = c.fy;
    o.cam.cx = c.cx;
    o.cam.cy = c.cy;
    std::memcpy(o.cam.R, c.R, sizeof c.R);
    std::memcpy(o.cam.t, c.t, sizeof c.t);
    for (int k = 0; k < 3; ++k)
      o.cam.centre[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
    o.cam.limx = cfg->fov_clamp * (0.5f * c.width) / c.fx;
    o.cam.limy = cfg->fov_clamp * (0.5f * c.height) / c.fy;
    o.set = in.set;
    o.tiles_x = (c.width + T - 1) / T;
    o.tiles_y = (c.height + T - 1) / T;
    o.mask = in.mask;
    o.o_rgb = in.out.rgb;
    o.o_normal = in.out.normal;
    o.o_dist = in.out.dist;
    o.o_depth = in.out.depth;
    o.o_alpha = in.out.alpha;
    o.o_ncontrib = in.out.n_contrib;
    o.g_rgb = in.gout.rgb;
    o.g_normal = in.gout.normal;
    o.g_dist = in.gout.dist;
    o.g_depth = in.gout.depth;
    o.g_alpha = in.gout.alpha;
    o.g_count = in.gout.count;
    o.record_offset = recoff;
    o.pixel_offset = pixoff;
    o.tile_offset = (uint32_t)toff;
    o.sat_offset = (uint32_t)satoff;
    o.row_offset = (uint32_t)rowoff;
    o.amask_offset = (uint32_t)amoff;
    amoff += (uint64_t)o.tiles_y * ((o.tiles_x + 31) / 32);
    tile_starts[r] = (uint32_t)toff;
    row_starts[r] = (uint32_t)rowoff;
    rec_starts[r] = recoff;
    DevSet &S = ds[in.set];
    S.renders[S.n_renders++] = r;
    toff += (uint64_t)o.tiles_x * o.tiles_y;
    rowoff += (uint64_t)o.tiles_y;
    satoff += (uint64_t)(o.tiles_x + 1) * (o.tiles_y + 1);
    recoff += (uint64_t)sets[in.set].n;
    pixoff += (uint64_t)c.width * c.height;
  }
  tile_starts[n_renders] = (uint32_t)toff;
  row_starts[n_renders] = (uint32_t)rowoff;
  rec_starts[n_renders] = recoff;
  return PGSAG_OK;
}

int pgsag_layout_of(const void *host_desc, pgsag_layout *out) {
  const Header *h = check_desc(host_desc);
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!out) return fail(PGSAG_INVALID_ARGUMENT, "null output");
  const Layout &L = h->ws;
  out->status = L.status;
  out->tile_count = L.tile_count;
  out->sat = L.sat;
  out->ranges = L.ranges;
  out->queue = L.queue;
  out->records = L.rec;
  out->depth_key = L.depth_key;
  out->rect = L.rect;
  out->n_active = L.nact;
  out->pair_tile = L.sorted_key;
  out->pair_record = L.sorted_val;
  out->pixel_T = L.pix_T;
  out->pixel_last = L.pix_last;
  out->grad2d = L.g2;
  out->work = L.work;
  out->end = L.end;
  return PGSAG_OK;
}

int pgsag_forward(const void *host_desc, const void *dev_desc, void *workspace, size_t workspace_bytes, void *stream,
                  void **events) {
  const Header *h = check_desc(host_desc);
  int rc = check_run_args(h, dev_desc, workspace, workspace_bytes);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  StageTimer tm{events, s};
  launch_fill_u32(ws_ptr<uint32_t>(workspace, h->ws.zero_begin), 0u, (h->ws.zero_end - h->ws.zero_begin) / 4, s);
  tm.begin(PGSAG_STAGE_TILE_MASK);
  launch_tile_mask(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_TILE_MASK);
  if ((rc = check_hip("tile mask"))) return rc;
  tm.begin(PGSAG_STAGE_PREPROCESS);
  launch_preprocess(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_PREPROCESS);
  if ((rc = check_hip("preprocess"))) return rc;
  tm.begin(PGSAG_STAGE_DEPTH_SORT);
  launch_depth_sort(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_DEPTH_SORT);
  if ((rc = check_hip("depth sort"))) return rc;
  tm.begin(PGSAG_STAGE_EMIT);
  launch_emit(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_EMIT);
  if ((rc = check_hip("emit"))) return rc;
  tm.begin(PGSAG_STAGE_TILE_SORT);
  launch_tile_sort(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_TILE_SORT);
  if ((rc = check_hip("tile sort"))) return rc;
  tm.begin(PGSAG_STAGE_COMPOSITE);
  launch_composite(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_COMPOSITE);
  return check_hip("composite");
}

namespace {
int run_backward(const Header *h, const void *dev_desc, void *workspace, const AdamArgs &A, void *stream,
                 void **events) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  StageTimer tm{events, s};
  // float atomics add into the 2D-gradient slots; the deterministic
  // reduction stores every slot the backward projection reads
  // the 2D-gradient slots start at zero; the forward compositing has
  // usually cleared them already (then this pass writes nothing)
  if (!h->cfg.deterministic)
    launch_fill_u32(ws_ptr<uint32_t>(workspace, h->ws.g2), 0u, h->n_records * kG2, s,
                    ws_ptr<uint32_t>(workspace, h->ws.status) + S_G2_CLEAN);
  if (h->cfg.persistent) launch_fill_u32(ws_ptr<uint32_t>(workspace, h->ws.status) + S_QUEUE_BWD, 0u, 1, s);
  if (h->cfg.deterministic) launch_det_clear(dev_desc, *h, workspace, s);
  tm.begin(PGSAG_STAGE_BACKWARD_COMPOSITE);
  launch_backward_composite(dev_desc, *h, workspace, s);
  if (h->cfg.deterministic) launch_det_reduce(dev_desc, *h, workspace, s);
  tm.end(PGSAG_STAGE_BACKWARD_COMPOSITE);
  int rc;
  if ((rc = check_hip("backward composite"))) return rc;
  tm.begin(PGSAG_STAGE_BACKWARD_PREPROCESS);
  launch_backward_preprocess(dev_desc, *h, workspace, A, s);
  tm.end(PGSAG_STAGE_BACKWARD_PREPROCESS);
  return check_hip("backward preprocess");
}
}  // namespace

int pgsag_backward(const void *host_desc, const void *dev_desc, void *workspace, size_t workspace_bytes,
                   void *stream, void **events) {
  const Header *h = check_desc(host_desc);
  int rc = check_run_args(h, dev_desc, workspace, workspace_bytes);
  if (rc) return rc;
  if (!h->any_grads) return fail(PGSAG_INVALID_ARGUMENT, "descriptor was packed without gradient buffers");
  AdamArgs A{};
  return run_backward(h, dev_desc, workspace, A, stream, events);
}

int pgsag_backward_adam(const void *host_desc, const void *dev_desc, void *workspace, size_t workspace_bytes,
                        const pgsag_adam_config *adam, void *stream, void **events) {
  const Header *h = check_desc(host_desc);
  int rc = check_run_args(h, dev_desc, workspace, workspace_bytes);
  if (rc) return rc;
  if (!h->any_grads) return fail(PGSAG_INVALID_ARGUMENT, "descriptor was packed without gradient buffers");
  if (!adam || !adam->step_state) return fail(PGSAG_INVALID_ARGUMENT, "null Adam configuration or step state");
  if (!(adam->b1 >= 0.f && adam->b1 < 1.f && adam->b2 >= 0.f && adam->b2 < 1.f))
    return fail(PGSAG_INVALID_ARGUMENT, "betas must be in [0, 1)");
  if ((uintptr_t)adam->step_state & 3u) return fail(PGSAG_INVALID_ARGUMENT, "step state must be 4-byte aligned");
  if (adam->m_offset == 0 || adam->v_offset == 0 || adam->m_offset == adam->v_offset)
    return fail(PGSAG_INVALID_ARGUMENT, "moment offsets must be non-zero and distinct");
  AdamArgs A{};
  A.lr = adam->lr;
  A.b1 = adam->b1;
  A.b2 = adam->b2;
  A.eps = adam->eps;
  A.coef = reinterpret_cast<const float *>(adam->step_state + 1);
  A.m_off = adam->m_offset;
  A.v_off = adam->v_offset;
  A.enabled = 1;
  A.write_grads = adam->write_grads ? 1 : 0;
  launch_adam_coef(adam->step_state, adam->b1, adam->b2, static_cast<hipStream_t>(stream));
  return run_backward(h, dev_desc, workspace, A, stream, events);
}

int pgsag_binning(const void *host_desc, const void *dev_desc, void *workspace, size_t workspace_bytes,
                  void *stream) {
  const Header *h = check_desc(host_desc);
  int rc = check_run_args(h, dev_desc, workspace, workspace_bytes);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_fill_u32(ws_ptr<uint32_t>(workspace, h->ws.zero_begin), 0u, (h->ws.zero_end - h->ws.zero_begin) / 4, s);
  launch_tile_mask(dev_desc, *h, workspace, s);
  launch_recount(dev_desc, *h, workspace, s);
  launch_depth_sort(dev_desc, *h, workspace, s);
  launch_emit(dev_desc, *h, workspace, s);
  launch_tile_sort(dev_desc, *h, workspace, s);
  return check_hip("binning");
}

int pgsag_read_status(const void *host_desc, const void *workspace, pgsag_status *out, void *stream) {
  const Header *h = check_desc(host_desc);
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!workspace || !out) return fail(PGSAG_INVALID_ARGUMENT, "null workspace or output");
  uint32_t w[S_ERROR + 1];
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(w, ws_ptr<uint32_t>(workspace, h->ws.status), sizeof w, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(PGSAG_HIP_ERROR, "read status: %s", hipGetErrorName(e));
  out->pairs_needed = (uint64_t)w[S_PAIRS_LO] | ((uint64_t)w[S_PAIRS_HI] << 32);
  out->overflow = w[S_OVERFLOW];
  out->n_visible = w[S_NVIS];
  out->error = w[S_ERROR];
  out->reserved = 0;
  return PGSAG_OK;
}

int pgsag_adam_step(float *params, const float *grads, float *m, float *v, int64_t n, float lr, float b1, float b2,
                    float eps, int32_t step, void *stream) {
  if (n < 0) return fail(PGSAG_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && (!params || !grads || !m || !v)) return fail(PGSAG_INVALID_ARGUMENT, "null pointer");
  if (step < 1) return fail(PGSAG_INVALID_ARGUMENT, "step must be >= 1");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f)) return fail(PGSAG_INVALID_ARGUMENT, "betas must be in [0, 1)");
  if (((uintptr_t)params | (uintptr_t)grads | (uintptr_t)m | (uintptr_t)v) & 3u)
    return fail(PGSAG_INVALID_ARGUMENT, "pointers must be 4-byte aligned");
  launch_adam(params, grads, m, v, n, lr, b1, b2, eps, step, nullptr, static_cast<hipStream_t>(stream));
  return check_hip("adam");
}

int pgsag_adam_step_device(float *params, const float *grads, float *m, float *v, int64_t n, float lr, float b1,
                           float b2, float eps, int32_t *state, void *stream) {
  if (n < 0) return fail(PGSAG_INVALID_ARGUMENT, "n < 0");
  if (!state) return fail(PGSAG_INVALID_ARGUMENT, "null step state");
  if (n > 0 && (!params || !grads || !m || !v)) return fail(PGSAG_INVALID_ARGUMENT, "null pointer");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f)) return fail(PGSAG_INVALID_ARGUMENT, "betas must be in [0, 1)");
  if (((uintptr_t)params | (uintptr_t)grads | (uintptr_t)m | (uintptr_t)v | (uintptr_t)state) & 3u)
    return fail(PGSAG_INVALID_ARGUMENT, "pointers must be 4-byte aligned");
  launch_adam(params, grads, m, v, n, lr, b1, b2, eps, 0, state, static_cast<hipStream_t>(stream));
  return check_hip("adam (device step)");
}

int pgsag_load_stats(const void *host_desc, const void *dev_desc, const void *workspace,
                     const float *const *pixel_weight, float *out, void *stream) {
  const Header *h = check_desc(host_desc);
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!dev_desc || !workspace || !out) return fail(PGSAG_INVALID_ARGUMENT, "null descriptor, workspace or output");
  const DevRender *rd = renders_of(host_desc);
  for (int r = 0; r < h->n_renders; ++r)
    if (!rd[r].o_ncontrib) return fail(PGSAG_INVALID_ARGUMENT, "render %d: n_contrib output is required", r);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int r = 0; r < h->n_renders; ++r)
    launch_load_stats(dev_desc, *h, workspace, r, pixel_weight ? pixel_weight[r] : nullptr, out, s);
  return check_hip("load stats");
}

void pgsag_default_loss_config(pgsag_loss_config *lc) {
  if (!lc) return;
  std::memset(lc, 0, sizeof *lc);
  lc->lambda_rgb = 1.0f;
  lc->lambda_normal = 0.01f;
  lc->boundary_weight = 0.1f;
  lc->lambda_load = 0.0f;
  lc->normal_norm = 1;
  lc->normal_eps = 1e-6f;
}

int pgsag_loss(const pgsag_loss_config *lc, const void *host_desc, const void *dev_desc, void *workspace,
               uint64_t workspace_bytes, const float *const *gt_rgb, const float *const *pixel_weight, float *loss,
               void *stream) {
  const Header *h = check_desc(host_desc);
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!lc || !dev_desc || !workspace || !gt_rgb || !loss)
    return fail(PGSAG_INVALID_ARGUMENT, "null config, descriptor, workspace, ground truth or loss output");
  if (workspace_bytes < h->ws_bytes) return fail(PGSAG_WORKSPACE_TOO_SMALL, "workspace too small");
  if (lc->normal_norm != 1 && lc->normal_norm != 2) return fail(PGSAG_INVALID_ARGUMENT, "normal_norm must be 1 or 2");
  if (!(lc->lambda_load >= 0.f && lc->lambda_load <= 1.f)) return fail(PGSAG_INVALID_ARGUMENT, "lambda_load must be in [0, 1]");
  if (!(lc->normal_eps >= 0.f)) return fail(PGSAG_INVALID_ARGUMENT, "normal_eps must be >= 0");
  if (lc->load_term != 0 && lc->load_term != 1) return fail(PGSAG_INVALID_ARGUMENT, "load_term must be 0 or 1");
  const DevRender *rd = renders_of(host_desc);
  for (int r = 0; r < h->n_renders; ++r) {
    if (!rd[r].o_rgb || !rd[r].o_normal || !rd[r].o_depth)
      return fail(PGSAG_INVALID_ARGUMENT, "render %d: rgb, normal and depth outputs are required", r);
    if (!rd[r].g_rgb || !rd[r].g_normal || !rd[r].g_depth)
      return fail(PGSAG_INVALID_ARGUMENT, "render %d: rgb, normal and depth grad-output planes are required", r);
    if (!gt_rgb[r]) return fail(PGSAG_INVALID_ARGUMENT, "render %d: null ground truth", r);
    if (lc->load_term == 1 && (!rd[r].o_ncontrib || !rd[r].g_count))
      return fail(PGSAG_INVALID_ARGUMENT, "render %d: the GC-load term needs the n_contrib output and the count "
                  "grad-output plane", r);
  }
  launch_loss(dev_desc, host_desc, workspace, *lc, gt_rgb, pixel_weight, loss, static_cast<hipStream_t>(stream));
  return check_hip("loss");
}

int pgsag_luminance_weights(const void *host_desc, const void *dev_desc, void *workspace, uint64_t workspace_bytes,
                            int32_t render, const float *gt_rgb, float *weight, void *stream) {
  const Header *h = check_desc(host_desc);
  if (!h) return PGSAG_INVALID_ARGUMENT;
  if (!dev_desc || !workspace || !gt_rgb || !weight)
    return fail(PGSAG_INVALID_ARGUMENT, "null descriptor, workspace, ground truth or weight output");
  if (workspace_bytes < h->ws_bytes) return fail(PGSAG_WORKSPACE_TOO_SMALL, "workspace too small");
  if (render < 0 || render >= h->n_renders) return fail(PGSAG_INVALID_ARGUMENT, "render index out of range");
  launch_luminance_weights(dev_desc, host_desc, workspace, render, gt_rgb, weight, static_cast<hipStream_t>(stream));
  return check_hip("luminance weights");
}

}  // extern "C"
