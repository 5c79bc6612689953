// C ABI of the renderer: argument checks, workspace layout, launch order.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/htgs.h"
#include "common.h"

namespace htgs {
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s);
hipError_t launch_opacity_decay(float *x, int64_t n, double lambda, hipStream_t s);
hipError_t launch_preprocess(const GaussPtrs &gp, const KCfg &cfg, const ViewSet &vs, const Ws &w,
                             hipStream_t s);
hipError_t launch_preprocess_bwd(const GaussPtrs &gp, const GradPtrs &gr, const KCfg &cfg,
                                 const ViewSet &vs, const Ws &w, hipStream_t s);
hipError_t launch_sort_passes(const Ws &w, hipStream_t s);
hipError_t launch_depth_sort(const Ws &w, const float *means, int64_t n, const float *w2c,
                             hipStream_t s);
hipError_t launch_ranges(const Ws &w, int total_tiles, hipStream_t s);
hipError_t launch_tile_order(const Ws &w, int total_tiles, hipStream_t s);
hipError_t launch_raster_fwd(const Ws &w, const ViewSet &vs, const KCfg &cfg, float *state,
                             const uint32_t *vals, hipStream_t s);
hipError_t launch_raster_bwd(const Ws &w, const ViewSet &vs, const KCfg &cfg, const float *state,
                             const uint32_t *vals, hipStream_t s);

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kMaxCapacity = (1ll << 30) - 1;

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int64_t status, total, frags, pp_total, hist, ranges, order_hist, dhist, zero_end;
  int64_t sort_cnt, dcnt, records, rects, tslots, refpix, cflags, order, keys0, keys1, vals0, vals1;
  int64_t partials, dkeys0, dkeys1, dvals0, dvals1, bytes;
  int64_t capacity, chunk_stride, dchunk_stride;
  int32_t key_bits, passes, key16, sorted;
};

int bits_for(int64_t tiles) {
  int b = 1;
  while ((1ll << b) < tiles) ++b;
  return b;
}

// partials = false: a forward-only layout (no backward partials); sorted:
// with the depth sort of sorted blending.
Layout make_layout(int64_t n, int n_views, int64_t total_tiles, int64_t capacity,
                   bool partials = true, bool sorted = false) {
  Layout L{};
  L.capacity = capacity;
  L.sorted = sorted;
  // rows of the per-chunk digit-count tables: whole 256-byte lines
  L.dchunk_stride = sorted ? (n + kSortChunk - 1) / kSortChunk : 0;
  L.dchunk_stride = (L.dchunk_stride + 63) / 64 * 64;
  L.key_bits = bits_for(total_tiles);
  L.passes = (L.key_bits + 7) / 8;
  L.key16 = L.key_bits <= 16;
  L.chunk_stride = ((capacity + kSortChunk - 1) / kSortChunk + 63) / 64 * 64;
  const int64_t kb = L.key16 ? 2 : 4;
  int64_t o = 0;
  L.status = o; o = align_up(o + 4 * kStatusWords);
  L.total = o; o = align_up(o + 8);   // instance count
  L.frags = o; o = align_up(o + 2 * 8 * kCounterSpread * kCounterStride);  // fragment counters
  L.pp_total = o; o = align_up(o + 8 * ((n + kPreThreads - 1) / kPreThreads));
  L.hist = o; o = align_up(o + kHistCopies * 4 * 256 * 4);
  L.ranges = o; o = align_up(o + 8 * total_tiles);
  L.order_hist = o; o = align_up(o + 2 * 32 * 4);
  L.dhist = o; o = align_up(o + (sorted ? kHistCopies * 4 * 256 * 4 : 0));
  L.zero_end = o;
  L.sort_cnt = o; o = align_up(o + (int64_t)L.passes * 256 * L.chunk_stride * 4);
  L.dcnt = o; o = align_up(o + 4 * 256 * L.dchunk_stride * 4);
  L.records = o; o = align_up(o + (int64_t)n_views * n * kRecFloats * 4);
  L.rects = o; o = align_up(o + (int64_t)n_views * n * 16);
  L.refpix = o; o = align_up(o + (int64_t)n_views * n * 4);
  L.cflags = o; o = align_up(o + (int64_t)n_views * n);
  L.tslots = o; o = align_up(o + (int64_t)n_views * n * 16);
  L.order = o; o = align_up(o + 4 * total_tiles);
  L.keys0 = o; o = align_up(o + kb * capacity);
  L.keys1 = o; o = align_up(o + kb * capacity);
  L.vals0 = o; o = align_up(o + 4 * capacity);
  L.vals1 = o; o = align_up(o + 4 * capacity);
  L.partials = o; o = align_up(o + (partials ? (int64_t)kPartialFloats * 4 * capacity : 0));
  const int64_t dn = sorted ? 4 * n : 0;
  L.dkeys0 = o; o = align_up(o + dn);
  L.dkeys1 = o; o = align_up(o + dn);
  L.dvals0 = o; o = align_up(o + dn);
  L.dvals1 = o; o = align_up(o + dn);
  L.bytes = o;
  return L;
}

// Largest capacity whose layout fits in ws_bytes, or -1.
int64_t capacity_for(int64_t n, int n_views, int64_t total_tiles, int64_t ws_bytes,
                     bool partials = true, bool sorted = false) {
  if (make_layout(n, n_views, total_tiles, 0, partials, sorted).bytes > ws_bytes) return -1;
  int64_t lo = 0, hi = kMaxCapacity;
  if (make_layout(n, n_views, total_tiles, hi, partials, sorted).bytes <= ws_bytes) return hi;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (make_layout(n, n_views, total_tiles, mid, partials, sorted).bytes <= ws_bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

Ws make_ws(void *base, const Layout &L) {
  char *b = static_cast<char *>(base);
  Ws w{};
  w.status = reinterpret_cast<uint32_t *>(b + L.status);
  w.total = reinterpret_cast<unsigned long long *>(b + L.total);
  w.frags = reinterpret_cast<unsigned long long *>(b + L.frags);
  w.frags_bwd = w.frags + kCounterSpread * kCounterStride;
  w.pp_total = reinterpret_cast<unsigned long long *>(b + L.pp_total);
  w.hist = reinterpret_cast<uint32_t *>(b + L.hist);
  w.sort_cnt = reinterpret_cast<uint32_t *>(b + L.sort_cnt);
  w.ranges = reinterpret_cast<uint2 *>(b + L.ranges);
  w.order_hist = reinterpret_cast<uint32_t *>(b + L.order_hist);
  w.order = reinterpret_cast<uint32_t *>(b + L.order);
  w.records = reinterpret_cast<float *>(b + L.records);
  w.rects = reinterpret_cast<int4 *>(b + L.rects);
  w.tslots = reinterpret_cast<uint4 *>(b + L.tslots);
  w.refpix = reinterpret_cast<uint32_t *>(b + L.refpix);
  w.cflags = reinterpret_cast<uint8_t *>(b + L.cflags);
  w.keys[0] = b + L.keys0;
  w.keys[1] = b + L.keys1;
  w.vals[0] = reinterpret_cast<uint32_t *>(b + L.vals0);
  w.vals[1] = reinterpret_cast<uint32_t *>(b + L.vals1);
  w.partials = reinterpret_cast<float *>(b + L.partials);
  if (L.sorted) {
    w.dkeys[0] = reinterpret_cast<uint32_t *>(b + L.dkeys0);
    w.dkeys[1] = reinterpret_cast<uint32_t *>(b + L.dkeys1);
    w.dvals[0] = reinterpret_cast<uint32_t *>(b + L.dvals0);
    w.dvals[1] = reinterpret_cast<uint32_t *>(b + L.dvals1);
    w.dhist = reinterpret_cast<uint32_t *>(b + L.dhist);
    w.dcnt = reinterpret_cast<uint32_t *>(b + L.dcnt);
    w.perm = w.dvals[0];   // after the four depth-sort passes
    w.dchunk_stride = L.dchunk_stride;
  }
  w.capacity = L.capacity;
  w.chunk_stride = L.chunk_stride;
  w.key_bits = L.key_bits;
  w.passes = L.passes;
  w.key16 = L.key16;
  w.final_buf = L.passes & 1;
  return w;
}

int check_cfg(const htgs_config *cfg) {
  if (!cfg) return HTGS_E_INVAL;
  if (cfg->K < 0 || cfg->K > 32) return HTGS_E_INVAL;
  if (!(cfg->tau_alpha > 0.f && cfg->tau_alpha < 1.f)) return HTGS_E_INVAL;
  if (!(cfg->tau_core >= 0.f && cfg->tau_core <= 1.f)) return HTGS_E_INVAL;
  if (!(cfg->alpha_max > 0.f && cfg->alpha_max < 1.f)) return HTGS_E_INVAL;
  for (int c = 0; c < 3; ++c)
    if (!isfinite(cfg->bg[c])) return HTGS_E_INVAL;
  const bool t8 = cfg->tile_w == 8 && cfg->tile_h == 8;
  const bool t16x8 = cfg->tile_w == 16 && cfg->tile_h == 8;
  const bool t16 = cfg->tile_w == 16 && cfg->tile_h == 16;
  const bool t32x8 = cfg->tile_w == 32 && cfg->tile_h == 8;
  if (!t8 && !t16x8 && !t16 && !t32x8) return HTGS_E_INVAL;
  if ((t16 || t32x8) && cfg->K > 16) return HTGS_E_INVAL;
  const int np = cfg->tile_w * cfg->tile_h;
  if (cfg->lds_batch != 0 && cfg->lds_batch != np && !(t8 && cfg->lds_batch == 2 * np))
    return HTGS_E_INVAL;
  if (cfg->flags &
      ~(uint32_t)(HTGS_FLAG_COST_ORDER | HTGS_FLAG_GRAD_OVERWRITE | HTGS_FLAG_TILE_CULL |
                  HTGS_FLAG_PERSISTENT | HTGS_FLAG_NO_TAIL | HTGS_FLAG_BAKED | HTGS_FLAG_SORTED))
    return HTGS_E_INVAL;
  if ((cfg->flags & HTGS_FLAG_SORTED) && !(cfg->tau_T >= 0.f && cfg->tau_T < 1.f))
    return HTGS_E_INVAL;
  return HTGS_OK;
}

bool sorted_of(const htgs_config *cfg) { return (cfg->flags & HTGS_FLAG_SORTED) != 0; }

// Forward state values per pixel.
int state_vals(const htgs_config *cfg) {
  return sorted_of(cfg) ? kSortedStateValues : state_values(cfg->K);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_gaussians(const htgs_gaussians *g) {
  if (!g) return HTGS_E_INVAL;
  if (g->n < 0 || g->n >= (int64_t)(1 << 27)) return HTGS_E_INVAL;  // segment ids hold 27 bits
  if (g->sh_degree < 0 || g->sh_degree > 3) return HTGS_E_INVAL;
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
    return HTGS_E_INVAL;
  if (!aligned16(g->means) || !aligned16(g->log_scales) || !aligned16(g->quats) ||
      !aligned16(g->opacity_logits) || !aligned16(g->sh))
    return HTGS_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(g->filter_var) & 3u) != 0) return HTGS_E_INVAL;
  return HTGS_OK;
}

int check_cams(const htgs_camera *cams, int32_t n_views, const htgs_config *cfg) {
  if (!cams) return HTGS_E_INVAL;
  if (n_views < 1) return HTGS_E_INVAL;
  if (n_views > HTGS_MAX_VIEWS) return HTGS_E_TOO_MANY_VIEWS;
  for (int v = 0; v < n_views; ++v) {
    const htgs_camera &c = cams[v];
    if (c.width < 1 || c.height < 1) return HTGS_E_INVAL;
    if (!(c.fx > 0.f && c.fy > 0.f) || !isfinite(c.fx) || !isfinite(c.fy)) return HTGS_E_INVAL;
    if (!isfinite(c.cx) || !isfinite(c.cy) || !isfinite(c.z_near)) return HTGS_E_INVAL;
    for (int k = 0; k < 12; ++k)
      if (!isfinite(c.world_to_cam[k])) return HTGS_E_INVAL;
    const int64_t tx = (c.width + cfg->tile_w - 1) / cfg->tile_w;
    const int64_t ty = (c.height + cfg->tile_h - 1) / cfg->tile_h;
    if (tx > 1024 || ty > 1024) return HTGS_E_INVAL;
  }
  return HTGS_OK;
}

int64_t total_tiles_of(const htgs_camera *cams, int32_t n_views, const htgs_config *cfg) {
  int64_t t = 0;
  for (int v = 0; v < n_views; ++v)
    t += (int64_t)((cams[v].width + cfg->tile_w - 1) / cfg->tile_w) *
         ((cams[v].height + cfg->tile_h - 1) / cfg->tile_h);
  return t;
}

// Camera centre: the solution of R x = -t (float64, Cramer's rule).
void camera_centre(const float *m, double out[3]) {
  const double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9],
               i = m[10];
  const double r0 = -(double)m[3], r1 = -(double)m[7], r2 = -(double)m[11];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  out[0] = (r0 * (e * i - f * h) - b * (r1 * i - f * r2) + c * (r1 * h - e * r2)) / det;
  out[1] = (a * (r1 * i - f * r2) - r0 * (d * i - f * g) + c * (d * r2 - r1 * g)) / det;
  out[2] = (a * (e * r2 - r1 * h) - b * (d * r2 - r1 * g) + r0 * (d * h - e * g)) / det;
}

ViewSet make_views(const htgs_camera *cams, int32_t n_views, const htgs_config *cfg,
                   float *const *out_rgb, const float *const *grad_rgb) {
  ViewSet vs;
  memset(&vs, 0, sizeof(vs));
  vs.n = n_views;
  int64_t tiles = 0, state_off = 0;
  for (int v = 0; v < n_views; ++v) {
    const htgs_camera &c = cams[v];
    ViewParams &P = vs.v[v];
    memcpy(P.w2c, c.world_to_cam, sizeof(P.w2c));
    P.fx = c.fx; P.fy = c.fy; P.cx = c.cx; P.cy = c.cy;
    camera_centre(c.world_to_cam, P.cam_pos);
    P.width = c.width; P.height = c.height;
    P.tiles_x = (c.width + cfg->tile_w - 1) / cfg->tile_w;
    P.tiles_y = (c.height + cfg->tile_h - 1) / cfg->tile_h;
    P.tile_base = (int32_t)tiles;
    P.z_near = c.z_near;
    P.state_off = state_off;
    P.out_rgb = out_rgb ? out_rgb[v] : nullptr;
    P.grad_rgb = grad_rgb ? grad_rgb[v] : nullptr;
    tiles += (int64_t)P.tiles_x * P.tiles_y;
    state_off += (int64_t)state_vals(cfg) * P.tiles_x * P.tiles_y * cfg->tile_w * cfg->tile_h;
  }
  vs.total_tiles = (int32_t)tiles;
  return vs;
}

KCfg make_kcfg(const htgs_gaussians *g, const htgs_config *cfg) {
  KCfg k;
  k.n = g->n;
  k.K = cfg->K;
  k.sh_degree = g->sh_degree;
  k.tau_alpha = cfg->tau_alpha;
  k.tau_core = cfg->tau_core;
  k.alpha_max = cfg->alpha_max;
  for (int c = 0; c < 3; ++c) k.bg[c] = cfg->bg[c];
  k.tile_w = cfg->tile_w;
  k.tile_h = cfg->tile_h;
  k.batch_mult = (cfg->lds_batch == 2 * cfg->tile_w * cfg->tile_h) ? 2 : 1;
  k.cost_order = (cfg->flags & HTGS_FLAG_COST_ORDER) ? 1 : 0;
  k.grad_overwrite = (cfg->flags & HTGS_FLAG_GRAD_OVERWRITE) ? 1 : 0;
  k.tile_cull = (cfg->flags & HTGS_FLAG_TILE_CULL) ? 1 : 0;
  k.persistent = (cfg->flags & HTGS_FLAG_PERSISTENT) ? 1 : 0;
  k.no_tail = (cfg->flags & HTGS_FLAG_NO_TAIL) ? 1 : 0;
  k.baked = (cfg->flags & HTGS_FLAG_BAKED) ? 1 : 0;
  k.sorted = sorted_of(cfg) ? 1 : 0;
  k.tau_T = cfg->tau_T;
  return k;
}

GaussPtrs make_gp(const htgs_gaussians *g) {
  return GaussPtrs{g->means, g->log_scales, g->quats, g->opacity_logits, g->sh, g->filter_var};
}

int check_common(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                 const htgs_config *cfg) {
  int e = check_cfg(cfg);
  if (e) return e;
  if ((e = check_gaussians(g))) return e;
  // baked scales and opacities already hold any 3D filter
  if ((cfg->flags & HTGS_FLAG_BAKED) && g->filter_var) return HTGS_E_INVAL;
  if ((e = check_cams(cams, n_views, cfg))) return e;
  if (total_tiles_of(cams, n_views, cfg) >= (1ll << 31)) return HTGS_E_KEYWIDTH;
  // sorted blending: one view (its depth order is per view)
  if (sorted_of(cfg) && n_views != 1) return HTGS_E_INVAL;
  return HTGS_OK;
}

#define HIP_TRY(x)                      \
  do {                                  \
    if ((x) != hipSuccess) return HTGS_E_HIP; \
  } while (0)

// Optional stage timing with HIP events (htgs_profile_enable).
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> free_events;
  struct Rec { int stage; hipEvent_t a, b; int launches; };
  std::vector<Rec> pending;
  hipEvent_t take() {
    if (!free_events.empty()) {
      hipEvent_t e = free_events.back();
      free_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

struct StageTimer {
  Profiler::Rec rec{};
  hipStream_t s;
  bool active = false;
  // timed = false: never records (the no-allocation entry point creates no
  // events)
  StageTimer(int stage, hipStream_t st, int launches = 1, bool timed = true) : s(st) {
    if (!g_prof.on || !timed) return;
    rec.stage = stage;
    rec.launches = launches;
    rec.a = g_prof.take();
    rec.b = g_prof.take();
    active = rec.a && rec.b && hipEventRecord(rec.a, s) == hipSuccess;
  }
  ~StageTimer() {
    if (!active) return;
    if (hipEventRecord(rec.b, s) == hipSuccess) g_prof.pending.push_back(rec);
  }
};

int run_front(const htgs_gaussians *g, const ViewSet &vs, const htgs_config *cfg, const Layout &L,
              void *ws, hipStream_t s, bool sort, bool timed = true) {
  const Ws w = make_ws(ws, L);
  {
    StageTimer t(HTGS_STAGE_FILL, s, 1, timed);
    HIP_TRY(launch_fill_zero(ws, L.zero_end, s));
  }
  if (L.sorted) {
    StageTimer t(HTGS_STAGE_DEPTH_SORT, s, 13, timed);
    HIP_TRY(launch_depth_sort(w, g->means, g->n, vs.v[0].w2c, s));
  }
  {
    StageTimer t(HTGS_STAGE_PREPROCESS, s, 1, timed);
    HIP_TRY(launch_preprocess(make_gp(g), make_kcfg(g, cfg), vs, w, s));
  }
  if (sort && L.capacity > 0) {
    StageTimer t(HTGS_STAGE_SORT, s, 3 * L.passes, timed);
    HIP_TRY(launch_sort_passes(w, s));
  }
  if (sort && L.capacity > 0) {
    StageTimer t(HTGS_STAGE_RANGES, s, 1, timed);
    HIP_TRY(launch_ranges(w, vs.total_tiles, s));
    if (cfg->flags & HTGS_FLAG_COST_ORDER) HIP_TRY(launch_tile_order(w, vs.total_tiles, s));
  }
  return HTGS_OK;
}

// partials = false: forward-only workspace layout, no stage timing (the
// no-allocation entry point).
int forward_impl(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                 const htgs_config *cfg, void *ws, int64_t ws_bytes, void *state,
                 float *const *out_rgb, void *stream, bool partials = true) {
  int e = check_common(g, cams, n_views, cfg);
  if (e) return e;
  if (!ws || !out_rgb) return HTGS_E_INVAL;
  for (int v = 0; v < n_views; ++v)
    if (!out_rgb[v]) return HTGS_E_INVAL;
  const int64_t tiles = total_tiles_of(cams, n_views, cfg);
  const bool srt = sorted_of(cfg);
  const int64_t cap = capacity_for(g->n, n_views, tiles, ws_bytes, partials, srt);
  if (cap < 0) return HTGS_E_WORKSPACE;
  const Layout L = make_layout(g->n, n_views, tiles, cap, partials, srt);
  const ViewSet vs = make_views(cams, n_views, cfg, out_rgb, nullptr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((e = run_front(g, vs, cfg, L, ws, s, true, partials))) return e;
  const Ws w = make_ws(ws, L);
  StageTimer t(HTGS_STAGE_RASTER_FWD, s, 1, partials);
  if (cfg->flags & HTGS_FLAG_PERSISTENT)
    HIP_TRY(launch_fill_zero(static_cast<char *>(ws) + L.status + 4 * kQueueFwd, 16, s));
  HIP_TRY(launch_raster_fwd(w, vs, make_kcfg(g, cfg), static_cast<float *>(state),
                            w.vals[w.final_buf], s));
  return HTGS_OK;
}

int backward_impl(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                  const htgs_config *cfg, void *ws, int64_t ws_bytes, const void *state,
                  const float *const *grad_rgb, const htgs_grads *grads, void *stream) {
  int e = check_common(g, cams, n_views, cfg);
  if (e) return e;
  if (!ws || !state || !grad_rgb || !grads) return HTGS_E_INVAL;
  // inference-only modes have no backward
  if (cfg->flags & (HTGS_FLAG_NO_TAIL | HTGS_FLAG_BAKED)) return HTGS_E_INVAL;
  if (!aligned16(grads->means) || !aligned16(grads->log_scales) || !aligned16(grads->quats) ||
      !aligned16(grads->opacity_logits) || !aligned16(grads->sh))
    return HTGS_E_INVAL;
  if (((reinterpret_cast<uintptr_t>(grads->mean_grad_stat) |
        reinterpret_cast<uintptr_t>(grads->visible_count)) & 3u) != 0)
    return HTGS_E_INVAL;
  for (int v = 0; v < n_views; ++v)
    if (!grad_rgb[v]) return HTGS_E_INVAL;
  const int64_t tiles = total_tiles_of(cams, n_views, cfg);
  const int64_t cap = capacity_for(g->n, n_views, tiles, ws_bytes, true, sorted_of(cfg));
  if (cap < 0) return HTGS_E_WORKSPACE;
  const Layout L = make_layout(g->n, n_views, tiles, cap, true, sorted_of(cfg));
  const ViewSet vs = make_views(cams, n_views, cfg, nullptr, grad_rgb);
  const Ws w = make_ws(ws, L);
  const KCfg k = make_kcfg(g, cfg);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cap > 0) {
    StageTimer t(HTGS_STAGE_RASTER_BWD, s);
    if (cfg->flags & HTGS_FLAG_PERSISTENT)
      HIP_TRY(launch_fill_zero(static_cast<char *>(ws) + L.status + 4 * kQueueBwd, 16, s));
    HIP_TRY(launch_raster_bwd(w, vs, k, static_cast<const float *>(state), w.vals[w.final_buf], s));
  }
  // The preprocess backward sums the instance partials per (Gaussian, view)
  // itself.
  const GradPtrs gr{grads->means, grads->log_scales, grads->quats, grads->opacity_logits,
                    grads->sh, grads->mean_grad_stat, grads->visible_count};
  StageTimer t(HTGS_STAGE_PREPROCESS_BWD, s);
  HIP_TRY(launch_preprocess_bwd(make_gp(g), gr, k, vs, w, s));
  return HTGS_OK;
}

// Sums of the spread fragment counters (forward, backward). Synchronises.
int read_counters(const void *ws, const Layout &L, int64_t *fwd, int64_t *bwd, hipStream_t s) {
  unsigned long long c[2 * kCounterSpread * kCounterStride];
  HIP_TRY(hipMemcpyAsync(c, static_cast<const char *>(ws) + L.frags, sizeof(c),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned long long f = 0, b = 0;
  for (int k = 0; k < kCounterSpread; ++k) {
    f += c[k * kCounterStride];
    b += c[(kCounterSpread + k) * kCounterStride];
  }
  *fwd = (int64_t)f;
  *bwd = (int64_t)b;
  return HTGS_OK;
}

// Workspace of the allocation-free forward: a file-scope device array, one
// copy per GPU (each device that loads the library holds it until the
// process ends). Host code never uses the array's name as an address: the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr int64_t kScratchBytes = (int64_t)HTGS_NOALLOC_WS_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace
__device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on
// the first call on that device), or null if the lookup fails.
void *scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Public status flags of a workspace to a caller's device word.
__global__ void k_copy_status(const uint32_t *__restrict__ status, uint32_t *__restrict__ out) {
  if (threadIdx.x == 0) *out = status[0] & kStatusPublic;
}

}  // namespace
}  // namespace htgs

using namespace htgs;

extern "C" {

int htgs_version(void) { return 4; }

const char *htgs_strerror(int code) {
  switch (code) {
    case HTGS_OK: return "ok";
    case HTGS_E_INVAL: return "invalid argument";
    case HTGS_E_WORKSPACE: return "workspace too small";
    case HTGS_E_KEYWIDTH: return "too many tiles for the key width";
    case HTGS_E_HIP: return "HIP error";
    case HTGS_E_OVERFLOW: return "instance capacity exceeded";
    case HTGS_E_TOO_MANY_VIEWS: return "too many views";
    case HTGS_E_TOO_LARGE:
      return "scene or image too large for the library-owned workspace of the allocation-free "
             "forward";
    default: return "unknown error";
  }
}

int htgs_workspace_bytes(int64_t n, const htgs_camera *cams, int32_t n_views,
                         const htgs_config *cfg, int64_t max_instances, int64_t *bytes_out) {
  int e = check_cfg(cfg);
  if (e) return e;
  if (!bytes_out || n < 0 || max_instances < 0 || max_instances > kMaxCapacity) return HTGS_E_INVAL;
  if ((e = check_cams(cams, n_views, cfg))) return e;
  *bytes_out = make_layout(n, n_views, total_tiles_of(cams, n_views, cfg), max_instances, true,
                           sorted_of(cfg)).bytes;
  return HTGS_OK;
}

int htgs_state_bytes(const htgs_camera *cams, int32_t n_views, const htgs_config *cfg,
                     int64_t *bytes_out) {
  int e = check_cfg(cfg);
  if (e) return e;
  if (!bytes_out) return HTGS_E_INVAL;
  if ((e = check_cams(cams, n_views, cfg))) return e;
  int64_t b = 0;
  for (int v = 0; v < n_views; ++v) {
    const int64_t tx = (cams[v].width + cfg->tile_w - 1) / cfg->tile_w;
    const int64_t ty = (cams[v].height + cfg->tile_h - 1) / cfg->tile_h;
    b += (int64_t)4 * state_vals(cfg) * tx * ty * cfg->tile_w * cfg->tile_h;
  }
  *bytes_out = b;
  return HTGS_OK;
}

int htgs_count_instances(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                         const htgs_config *cfg, void *ws, int64_t ws_bytes,
                         int64_t *instances_out, void *stream) {
  int e = check_common(g, cams, n_views, cfg);
  if (e) return e;
  if (!ws || !instances_out) return HTGS_E_INVAL;
  const int64_t tiles = total_tiles_of(cams, n_views, cfg);
  const int64_t cap = capacity_for(g->n, n_views, tiles, ws_bytes, true, sorted_of(cfg));
  if (cap < 0) return HTGS_E_WORKSPACE;
  // Count with capacity 0: nothing is emitted, the scan still runs.
  const Layout L0 = make_layout(g->n, n_views, tiles, 0, true, sorted_of(cfg));
  const ViewSet vs = make_views(cams, n_views, cfg, nullptr, nullptr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((e = run_front(g, vs, cfg, L0, ws, s, false))) return e;
  unsigned long long total = 0;
  HIP_TRY(hipMemcpyAsync(&total, static_cast<char *>(ws) + L0.total, sizeof(total),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *instances_out = (int64_t)total;
  return HTGS_OK;
}

int htgs_render_forward(const htgs_gaussians *g, const htgs_camera *cam, const htgs_config *cfg,
                        void *ws, int64_t ws_bytes, void *state, float *out_rgb, void *stream) {
  float *outs[1] = {out_rgb};
  return forward_impl(g, cam, 1, cfg, ws, ws_bytes, state, outs, stream);
}

int htgs_render_forward_noalloc(const htgs_gaussians *g, const htgs_camera *cam,
                                const htgs_config *cfg, float *out_rgb, uint32_t *status_out,
                                void *stream) {
  int e = check_common(g, cam, 1, cfg);
  if (e) return e;
  if (!out_rgb) return HTGS_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(status_out) & 3u) != 0) return HTGS_E_INVAL;
  // the forward-only layout with no instance must fit; instances beyond
  // what fits are reported as an overflow in the status word
  if (make_layout(g->n, 1, total_tiles_of(cam, 1, cfg), 0, false, sorted_of(cfg)).bytes >
      kScratchBytes)
    return HTGS_E_TOO_LARGE;
  void *ws = scratch_of_current_device();
  if (!ws) return HTGS_E_HIP;
  float *outs[1] = {out_rgb};
  if ((e = forward_impl(g, cam, 1, cfg, ws, kScratchBytes, nullptr, outs, stream, false)))
    return e;
  if (status_out) {
    const Layout L = make_layout(0, 1, 1, 0);
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const uint32_t *>(static_cast<char *>(ws) + L.status),
                       status_out);
    HIP_TRY(hipGetLastError());
  }
  return HTGS_OK;
}

int htgs_render_backward(const htgs_gaussians *g, const htgs_camera *cam, const htgs_config *cfg,
                         void *ws, int64_t ws_bytes, const void *state, const float *grad_rgb,
                         const htgs_grads *grads, void *stream) {
  const float *gs[1] = {grad_rgb};
  return backward_impl(g, cam, 1, cfg, ws, ws_bytes, state, gs, grads, stream);
}

int htgs_render_forward_batched(const htgs_gaussians *g, const htgs_camera *cams,
                                int32_t n_views, const htgs_config *cfg, void *ws,
                                int64_t ws_bytes, void *state, float *const *out_rgb,
                                void *stream) {
  return forward_impl(g, cams, n_views, cfg, ws, ws_bytes, state, out_rgb, stream);
}

int htgs_render_backward_batched(const htgs_gaussians *g, const htgs_camera *cams,
                                 int32_t n_views, const htgs_config *cfg, void *ws,
                                 int64_t ws_bytes, const void *state,
                                 const float *const *grad_rgb, const htgs_grads *grads,
                                 void *stream) {
  return backward_impl(g, cams, n_views, cfg, ws, ws_bytes, state, grad_rgb, grads, stream);
}

int htgs_read_status(const void *ws, int64_t ws_bytes, uint32_t *flags_out,
                     int64_t *instances_out, int64_t *fragments_out, void *stream) {
  // status and counters sit at fixed offsets at the start of every layout
  const Layout L = make_layout(0, 1, 1, 0);
  if (!ws || !flags_out || ws_bytes < L.pp_total) return HTGS_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t flags = 0;
  unsigned long long total = 0;
  int64_t fwd = 0, bwd = 0;
  HIP_TRY(hipMemcpyAsync(&flags, static_cast<const char *>(ws) + L.status, 4,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&total, static_cast<const char *>(ws) + L.total, 8,
                         hipMemcpyDeviceToHost, s));
  if (fragments_out) {
    int e = read_counters(ws, L, &fwd, &bwd, s);
    if (e) return e;
  }
  HIP_TRY(hipStreamSynchronize(s));
  *flags_out = flags & kStatusPublic;
  if (instances_out) *instances_out = (int64_t)total;
  if (fragments_out) *fragments_out = fwd;
  return HTGS_OK;
}

int htgs_opacity_decay(float *opacity_logits, int64_t n, double lambda, void *stream) {
  if (n < 0 || (n > 0 && !opacity_logits) || !(lambda > 0.0 && lambda <= 1.0)) return HTGS_E_INVAL;
  HIP_TRY(launch_opacity_decay(opacity_logits, n, lambda, static_cast<hipStream_t>(stream)));
  return HTGS_OK;
}

int htgs_debug_fragment_counts(const void *ws, int64_t ws_bytes, int64_t *forward_out,
                               int64_t *backward_out, void *stream) {
  const Layout L = make_layout(0, 1, 1, 0);
  if (!ws || !forward_out || !backward_out || ws_bytes < L.pp_total) return HTGS_E_INVAL;
  return read_counters(ws, L, forward_out, backward_out, static_cast<hipStream_t>(stream));
}

int htgs_profile_enable(int on) {
  g_prof.on = on != 0;
  if (!g_prof.on) {
    for (auto &r : g_prof.pending) {
      g_prof.free_events.push_back(r.a);
      g_prof.free_events.push_back(r.b);
    }
    g_prof.pending.clear();
  }
  return HTGS_OK;
}

int htgs_profile_read(double *ms_out, int64_t *launches_out, int32_t n_stages) {
  if (!ms_out || !launches_out || n_stages < HTGS_NUM_STAGES) return HTGS_E_INVAL;
  for (int i = 0; i < n_stages; ++i) {
    ms_out[i] = 0.0;
    launches_out[i] = 0;
  }
  int rc = HTGS_OK;
  for (auto &r : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      rc = HTGS_E_HIP;
    ms_out[r.stage] += ms;
    launches_out[r.stage] += r.launches;
    g_prof.free_events.push_back(r.a);
    g_prof.free_events.push_back(r.b);
  }
  g_prof.pending.clear();
  return rc;
}

int htgs_debug_export_bins(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                           const htgs_config *cfg, const void *ws, int64_t ws_bytes,
                           uint32_t *keys_out, uint32_t *values_out, int64_t max_out,
                           int32_t *rects_out, int64_t *instances_out, void *stream) {
  int e = check_common(g, cams, n_views, cfg);
  if (e) return e;
  if (!ws || !keys_out || !values_out || !instances_out || max_out < 0) return HTGS_E_INVAL;
  const int64_t tiles = total_tiles_of(cams, n_views, cfg);
  const int64_t cap = capacity_for(g->n, n_views, tiles, ws_bytes, true, sorted_of(cfg));
  if (cap < 0) return HTGS_E_WORKSPACE;
  const Layout L = make_layout(g->n, n_views, tiles, cap, true, sorted_of(cfg));
  const char *b = static_cast<const char *>(ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long total = 0;
  HIP_TRY(hipMemcpyAsync(&total, b + L.total, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t n = (int64_t)total;
  if (n > cap) n = cap;
  *instances_out = (int64_t)total;
  if (n > max_out) n = max_out;
  const int64_t fin = (L.passes & 1) ? L.keys1 : L.keys0;
  const int64_t finv = (L.passes & 1) ? L.vals1 : L.vals0;
  if (n > 0) {
    if (L.key16) {
      uint16_t *tmp = new uint16_t[n];
      HIP_TRY(hipMemcpyAsync(tmp, b + fin, 2 * n, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (int64_t i = 0; i < n; ++i) keys_out[i] = tmp[i];
      delete[] tmp;
    } else {
      HIP_TRY(hipMemcpyAsync(keys_out, b + fin, 4 * n, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(values_out, b + finv, 4 * n, hipMemcpyDeviceToHost, s));
  }
  if (rects_out && g->n > 0)
    HIP_TRY(hipMemcpyAsync(rects_out, b + L.rects, 16 * g->n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HTGS_OK;
}

}  // extern "C"
