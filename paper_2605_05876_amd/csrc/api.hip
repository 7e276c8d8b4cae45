// C ABI of libsurfsplat: context, workspace, and the forward / backward
// pipelines.  See include/surfsplat.h for the contract of every entry point.
//
// Pipeline of ss_render on one stream:
//   envmap levels (per scene, split-sum) -> preprocess + shade (per record)
//   -> per group: depth sort of the records -> scan of their tile counts in
//   that order -> pair emission -> stable sort of the pairs by tile -> tile
//   ranges -> tile order -> raster forward.
// A "group" is a run of views that share one pair list: one group holding
// every view (batched launches) or one group per view (per-view launches).
// ss_render_backward: raster backward (per group) -> preprocess/shade adjoint
// (per surfel) -> environment adjoint (per scene).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.h"
#include "surfsplat.h"

using namespace ss;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};
hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.n >= bytes) return hipSuccess;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.n = bytes;
  return e;
}
void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}
template <class T> T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

struct Group {
  int v0, v1;
  int tile_base, n_tiles;
  long long rec_begin, rec_end;
  long long pair_base, pair_cap;
  int pair_passes;  // radix passes of the pair sort over the bits of the local tile index:
  int pair_first;   // 8-bit digits, the first 9 bits wide when that saves a pass
  long long mask_base, mask_n;  // the group's chunk slots of walk masks (WalkBufs)
  // raster work items when long lists are split: all items, those of split tiles
  long long item_base, item_cap, mitem_base, mitem_cap;
};

struct SceneEnv {
  int He = 0, We = 0;
  DevBuf dirs, lv, Z /* output-texel table (R, 1/Z) of levels 1..6 */, dlv, part /* prefilter partials */;
  DevBuf dlv_fx, adj_part;  // deterministic backward: fixed-point level gradients, adjoint partials
  int lh[7], lw[7];
  long long off[7];   // float offsets of levels 1..6 in lv
  long long doff[7];  // float offsets of levels 0..6 in dlv
  int loc_off[7];     // LDS layout of the privatised level gradients (-1: global atomics)
  int loc_total = 0;
};

int bits_for(long long n) {
  int b = 1;
  while ((1LL << b) < n) ++b;
  return b;
}

}  // namespace

struct ss_context {
  ss_options opt;
  bool reserved = false;
  std::vector<long long> sig;
  std::vector<ViewDev> views_h;
  bool views_uploaded = false;
  int n_views = 0, n_scenes = 0;
  long long N = 0, R = 0, n_pix = 0;
  int n_tiles = 0, max_surf = 0;
  std::vector<Group> groups;
  std::vector<SceneEnv> env;
  DevBuf views_d, recs, counts, offsets, scan_tmp, keys, vals, keys2, vals2, hist, ranges, nl, stats,
      grad, misc, partial, sg, order, stats2, zkey, zkey2, zidx, zidx2, prect, zrect, lpos, qmask,
      pgrad /* deterministic: per-pair gradient partials */, inv /* record -> depth position */,
      detw /* deterministic: per scene fixed-point bound and exponent */,
      items, mitems, segbase /* split lists: work items and their scan scratch */,
      segL, segS, segF, segM, segZ, segZI /* split lists: the segments' local layers and z_max */,
      ovf /* record-major backward: per-pixel table entries of the deeper layers */;
  std::vector<long long> soff;
  long long scan_tmp_n = 0, pair_total = 0, hist_n = 0;
  DevBuf lut;
  int lut_nv = 0, lut_r = 0;
  bool fwd_valid = false;
  bool fwd_cons = false;  // the last forward wrote the per-layer depth statistics
  long long generation = 0;  // number of the last ss_render (its forward state)
  int lds_batch = 128;       // the LDS batch in use (options.lds_batch, or picked by the reserve)
  int seg_len = 0;           // list entries per segment of a split tile list (0: lists are not split)
  bool fwd_split = false;    // the last forward split long lists (the backward walks the same items)
  std::vector<long long> fwd_sig;
  hipStream_t last_stream = nullptr;  // may be the null stream
  bool used = false;                  // a stream call has been made
  // second stream for the environment adjoint, overlapping the geometry adjoint
  // (split-sum; created by the reserve)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // stage timing
  bool prof = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_ev;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

// Device words of a workspace (u32 array `misc`): latched status, the raster
// work queue, per-group pair counts, the tile-order scratch, then 64-bit
// counters (8-byte aligned): non-finite inputs of the forward and of the
// backward, and the raster forward's work counters (E, F, layers, sum of W).
constexpr int kMiscStatus = 0, kMiscQueue = 1, kMiscPairs = 8;
constexpr int kMiscOrder = kMiscPairs + kMaxViews;  // 66 u32: tile-order bucket counts and cursors
constexpr int kMiscNonfinite = kMiscOrder + 66;     // u64 [2]: forward, backward
constexpr int kMiscCounters = kMiscNonfinite + 4;   // u64 [3] + f64: E, F, layers, sum W
constexpr int kMiscSeg = kMiscCounters + 8;         // per group: raster items, items of split tiles
constexpr int kMiscWords = kMiscSeg + 2 * kMaxViews;

#define SS_HIP(x)                                                            \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SS_ERR_NOMEM : SS_ERR_HIP; \
  } while (0)
#define SS_TRY(x)                       \
  do {                                  \
    ss_status s_ = (x);                 \
    if (s_ != SS_OK) return s_;         \
  } while (0)

ss_status check_options(const ss_options* o) {
  if (!o) return SS_ERR_INVALID_ARG;
  if (!(o->r_cut > 0.f) || !(o->gamma > 0.f) || !(o->sigma_f >= 0.f)) return SS_ERR_INVALID_ARG;
  if (o->k_max < 1 || o->k_max > kMaxLayers) return SS_ERR_INVALID_ARG;
  if (o->shade != SS_SHADE_ALBEDO && o->shade != SS_SHADE_SPLITSUM && o->shade != SS_SHADE_NORMAL)
    return SS_ERR_INVALID_ARG;
  const int tk = o->tile_w * 100 + o->tile_h;
  if (tk != 808 && tk != 1608 && tk != 1616 && tk != 3208 && tk != 3216) return SS_ERR_UNSUPPORTED;
  if (o->lds_batch != 0 && o->lds_batch != 32 && o->lds_batch != 64 && o->lds_batch != 128 &&
      o->lds_batch != 256)
    return SS_ERR_UNSUPPORTED;
  if (o->launch != SS_LAUNCH_BATCHED && o->launch != SS_LAUNCH_PER_VIEW) return SS_ERR_INVALID_ARG;
  if (o->depth_stats != 0 && o->depth_stats != 1) return SS_ERR_INVALID_ARG;
  if (o->mip != 0 && o->mip != 1) return SS_ERR_INVALID_ARG;
  if (o->env_lds < -1) return SS_ERR_INVALID_ARG;
  if (!(o->t_min >= 0.f) || !(o->t_min < 1.f)) return SS_ERR_INVALID_ARG;
  if ((o->deterministic | o->validate | o->counters | o->tonemap) & ~1) return SS_ERR_INVALID_ARG;
  if (o->seg_len != 0 && o->seg_len != -1 && (o->seg_len < 256 || o->seg_len > 32768 || o->seg_len % 256 != 0))
    return SS_ERR_INVALID_ARG;
  if (o->bwd_walk < 0 || o->bwd_walk > 2) return SS_ERR_INVALID_ARG;
  return SS_OK;
}

ss_status check_batch(const ss_context* c, const ss_batch* b) {
  if (!b || b->n_scenes < 1 || !b->surfel_offset || b->n_views < 1 || b->n_views > kMaxViews ||
      !b->cameras)
    return SS_ERR_INVALID_ARG;
  if (b->surfel_offset[0] != 0) return SS_ERR_INVALID_ARG;
  for (int s = 0; s < b->n_scenes; ++s) {
    long long n = b->surfel_offset[s + 1] - b->surfel_offset[s];
    if (n < 0 || n > (1LL << 30)) return SS_ERR_INVALID_ARG;
  }
  const long long N = b->surfel_offset[b->n_scenes];
  if (N > 0 && (!b->position || !b->normal || !b->tangent || !b->scale || !b->albedo ||
                !b->roughness || !b->metallic))
    return SS_ERR_INVALID_ARG;
  long long R = 0;
  for (int v = 0; v < b->n_views; ++v) {
    const ss_camera& k = b->cameras[v];
    if (k.scene < 0 || k.scene >= b->n_scenes) return SS_ERR_INVALID_ARG;
    if (k.width < 1 || k.height < 1 || k.width > 16384 || k.height > 16384) return SS_ERR_INVALID_ARG;
    if (!(k.fx > 0.f) || !(k.fy > 0.f) || !(k.znear > 0.f)) return SS_ERR_INVALID_ARG;
    R += b->surfel_offset[k.scene + 1] - b->surfel_offset[k.scene];
  }
  if (R >= (1LL << 32) - 1) return SS_ERR_INVALID_ARG;
  if (c->opt.shade == SS_SHADE_SPLITSUM) {
    if (!b->envmap || !b->env_hw) return SS_ERR_INVALID_ARG;
    for (int s = 0; s < b->n_scenes; ++s) {
      if (!b->envmap[s]) return SS_ERR_INVALID_ARG;
      if (b->env_hw[2 * s] < 4 || b->env_hw[2 * s + 1] < 8 || b->env_hw[2 * s] > 4096 ||
          b->env_hw[2 * s + 1] > 8192)
        return SS_ERR_INVALID_ARG;
    }
  }
  return SS_OK;
}

std::vector<long long> signature(const ss_context* c, const ss_batch* b) {
  std::vector<long long> s;
  s.push_back(b->n_scenes);
  for (int i = 0; i <= b->n_scenes; ++i) s.push_back(b->surfel_offset[i]);
  s.push_back(b->n_views);
  for (int v = 0; v < b->n_views; ++v) {
    s.push_back(b->cameras[v].scene);
    s.push_back(b->cameras[v].width);
    s.push_back(b->cameras[v].height);
  }
  s.push_back(c->opt.shade);
  s.push_back(c->opt.tile_w);
  s.push_back(c->opt.tile_h);
  s.push_back(c->opt.launch);
  if (c->opt.shade == SS_SHADE_SPLITSUM)
    for (int i = 0; i < 2 * b->n_scenes; ++i) s.push_back(b->env_hw[i]);
  return s;
}

// The walk of the raster backward: 1 rows, 2 record-major.  Automatic choice:
// record-major with 256-record batches (where the row walk's per-wave sums
// halve its occupancy), rows otherwise -- the faster of the two on every
// measured workload.
int backward_walk(const ss_context* c) {
  return c->opt.bwd_walk != 0 ? c->opt.bwd_walk : (c->lds_batch >= 256 ? 2 : 1);
}

Params make_params(const ss_context* c) {
  Params p;
  p.r_cut = c->opt.r_cut;
  p.r2 = c->opt.r_cut * c->opt.r_cut;
  p.kappa = c->opt.gamma / (2.f * kPi);
  p.sigma_f = c->opt.sigma_f;
  p.k_max = c->opt.k_max;
  p.shade = c->opt.shade;
  p.tile_w = c->opt.tile_w;
  p.tile_h = c->opt.tile_h;
  p.lut = reinterpret_cast<const float*>(c->lut.p);
  p.lut_nv = c->lut_nv;
  p.lut_r = c->lut_r;
  p.ss_grad = 0;
  p.cons = 0;
  p.mip = c->opt.mip;
  p.t_min = c->opt.t_min;
  p.tonemap = c->opt.tonemap;
  p.counters = c->opt.counters;
  p.bwd_walk = backward_walk(c);
  return p;
}

// Host view descriptors for `b` (layout, cameras and map pointers).
void build_views(ss_context* c, const ss_batch* b, std::vector<ViewDev>& out) {
  out.assign(b->n_views, ViewDev());
  long long pix = 0, rec = 0;
  int tile = 0;
  for (int v = 0; v < b->n_views; ++v) {
    const ss_camera& k = b->cameras[v];
    ViewDev& d = out[v];
    std::memset(&d, 0, sizeof(d));
    d.fx = k.fx; d.fy = k.fy; d.cx = k.cx; d.cy = k.cy;
    for (int i = 0; i < 9; ++i) d.R[i] = k.R[i];
    for (int i = 0; i < 3; ++i) { d.t[i] = k.t[i]; d.bg[i] = k.background[i]; }
    for (int j = 0; j < 3; ++j)
      d.cam_o[j] = -(k.R[j] * k.t[0] + k.R[3 + j] * k.t[1] + k.R[6 + j] * k.t[2]);
    d.znear = k.znear;
    d.W = k.width; d.H = k.height;
    d.tiles_x = (k.width + c->opt.tile_w - 1) / c->opt.tile_w;
    d.tiles_y = (k.height + c->opt.tile_h - 1) / c->opt.tile_h;
    d.tile_base = tile;
    d.scene = k.scene;
    d.surf_off = b->surfel_offset[k.scene];
    d.n_surf = (int)(b->surfel_offset[k.scene + 1] - d.surf_off);
    d.pix_off = pix;
    d.rec_off = rec;
    tile += d.tiles_x * d.tiles_y;
    pix += (long long)k.width * k.height;
    rec += d.n_surf;
    if (c->opt.shade == SS_SHADE_SPLITSUM && k.scene < (int)c->env.size()) {
      SceneEnv& e = c->env[k.scene];
      d.lvl[0] = b->envmap[k.scene];
      d.dlvl[0] = P<float>(e.dlv) + e.doff[0];
      for (int l = 0; l < 7; ++l) d.dlvl_fx[l] = e.dlv_fx.p ? P<long long>(e.dlv_fx) + e.doff[l] : nullptr;
      for (int l = 1; l < 7; ++l) {
        d.lvl[l] = P<float>(e.lv) + e.off[l];
        d.dlvl[l] = P<float>(e.dlv) + e.doff[l];
      }
      for (int l = 0; l < 7; ++l) { d.lh[l] = e.lh[l]; d.lw[l] = e.lw[l]; }
    }
  }
}

ss_status upload_views(ss_context* c, const ss_batch* b, hipStream_t st) {
  std::vector<ViewDev> v;
  build_views(c, b, v);
  const size_t bytes = v.size() * sizeof(ViewDev);
  if (c->views_uploaded && v.size() == c->views_h.size() &&
      std::memcmp(v.data(), c->views_h.data(), bytes) == 0)
    return SS_OK;
  SS_HIP(hipStreamSynchronize(st));
  SS_HIP(hipMemcpy(c->views_d.p, v.data(), bytes, hipMemcpyHostToDevice));
  c->views_h = v;
  c->views_uploaded = true;
  return SS_OK;
}

// Level sizes, float offsets and the LDS layout of the privatised level
// gradients of scene s (no device work).  Returns the float counts of the
// levels 1..6 (lv) and of the gradient levels 0..6 (dlv).
void env_layout(const ss_context* c, const ss_batch* b, int s, SceneEnv& e, long long* lv_n, long long* dlv_n) {
  const int He = b->env_hw[2 * s], We = b->env_hw[2 * s + 1];
  e.lh[0] = He; e.lw[0] = We;
  for (int l = 1; l <= 5; ++l) { e.lh[l] = He >> l > 4 ? He >> l : 4; e.lw[l] = We >> l > 8 ? We >> l : 8; }
  e.lh[6] = 32; e.lw[6] = 64;
  long long o = 0;
  e.off[0] = 0;
  for (int l = 1; l < 7; ++l) { e.off[l] = o; o += 3LL * e.lh[l] * e.lw[l]; }
  *lv_n = o;
  long long d = 0;
  for (int l = 0; l < 7; ++l) { e.doff[l] = d; d += 3LL * e.lh[l] * e.lw[l]; }
  *dlv_n = d;
  // privatise the irradiance level and the specular levels, smallest first,
  // in LDS while they fit
  for (int l = 0; l < 7; ++l) e.loc_off[l] = -1;
  e.loc_total = 0;
  for (int l : {6, 5, 4, 3, 2, 1, 0}) {
    const int n = 3 * e.lh[l] * e.lw[l];
    const int budget = c->opt.deterministic ? 0
                       : (c->opt.env_lds < 0 ? kLocalMapFloats : std::min(c->opt.env_lds, kLocalMapFloats));
    if (e.loc_total + n > budget) break;
    e.loc_off[l] = e.loc_total;
    e.loc_total += n;
  }
}

ss_status prepare_env(ss_context* c, const ss_batch* b, hipStream_t st) {
  if (c->opt.shade != SS_SHADE_SPLITSUM) {
    c->env.clear();
    return SS_OK;
  }
  c->env.resize(b->n_scenes);
  for (int s = 0; s < b->n_scenes; ++s) {
    SceneEnv& e = c->env[s];
    const int He = b->env_hw[2 * s], We = b->env_hw[2 * s + 1];
    long long lv_n = 0, d = 0;
    env_layout(c, b, s, e, &lv_n, &d);
    SS_HIP(ensure(c->partial, (size_t)(kBackwardBlocks + kReduceSplit) * kLocalMapFloats * sizeof(float)));
    SS_HIP(ensure(e.lv, lv_n * sizeof(float)));
    SS_HIP(ensure(e.dlv, d * sizeof(float)));
    SS_HIP(ensure(e.Z, (size_t)(lv_n / 3 + 1) * 4 * sizeof(float)));
    SS_HIP(ensure(e.part, (size_t)envmap_prefilter_chunks(He, We) * (size_t)lv_n * sizeof(float)));
    if (c->opt.deterministic) {
      SS_HIP(ensure(e.dlv_fx, d * sizeof(long long)));
      SS_HIP(ensure(e.adj_part, (size_t)envmap_adjoint_chunks((int)(lv_n / 3)) * He * We * 3 * sizeof(float)));
    }
    if (e.He != He || e.We != We || !e.dirs.p) {
      SS_HIP(ensure(e.dirs, (size_t)He * We * 4 * sizeof(float)));
      SS_HIP(launch_envmap_dirs(P<float>(e.dirs), He, We, st));
      SS_HIP(launch_envmap_out_dirs(He, We, P<float>(e.dirs), e.lh, e.lw, P<float>(e.Z), st));
      e.He = He;
      e.We = We;
    }
  }
  return SS_OK;
}

ss_status run_envmap_prefilter(ss_context* c, const ss_batch* b, hipStream_t st) {
  if (c->opt.shade != SS_SHADE_SPLITSUM) return SS_OK;
  for (int s = 0; s < b->n_scenes; ++s) {
    SceneEnv& e = c->env[s];
    float* out[7];
    out[0] = nullptr;
    for (int l = 1; l < 7; ++l) out[l] = P<float>(e.lv) + e.off[l];
    SS_HIP(launch_envmap_prefilter(b->envmap[s], e.He, e.We, P<float>(e.dirs), P<float>(e.Z), out,
                                   e.lh, e.lw, P<float>(e.part), st));
  }
  return SS_OK;
}

void param_ptrs(const ss_batch* b, const float* p[7]) {
  p[0] = b->position; p[1] = b->normal; p[2] = b->tangent; p[3] = b->scale;
  p[4] = b->albedo; p[5] = b->roughness; p[6] = b->metallic;
}

ss_status run_preprocess(ss_context* c, const ss_batch* b, int v0, int v1, hipStream_t st) {
  const float* pp[7];
  param_ptrs(b, pp);
  int ms = 0;
  for (int v = v0; v < v1; ++v) ms = c->views_h[v].n_surf > ms ? c->views_h[v].n_surf : ms;
  SS_HIP(launch_preprocess(pp, c->N, P<ViewDev>(c->views_d), v0, v1, ms, make_params(c),
                           P<float>(c->recs), P<uint32_t>(c->counts), P<uint32_t>(c->zkey),
                           P<uint2>(c->prect), st));
  return SS_OK;
}

ss_status run_count_scan(ss_context* c, const Group& g, hipStream_t st) {
  uint32_t* misc = P<uint32_t>(c->misc);
  const long long n = g.rec_end - g.rec_begin;
  const int gi = (int)(&g - c->groups.data());
  if (n <= 0) {
    SS_HIP(launch_fill_u32(misc + kMiscPairs + gi, 0u, 1, st));
    return SS_OK;
  }
  SS_HIP(launch_scan_u32(P<uint32_t>(c->counts) + g.rec_begin, P<uint32_t>(c->offsets) + g.rec_begin, n,
                         misc + kMiscPairs + gi, P<uint32_t>(c->scan_tmp), c->scan_tmp_n, st));
  return SS_OK;
}

// Binning of one group (tile binning, Sec. 3.2.1): depth sort of the records,
// slot ranges by a scan of their tile counts in that order, pair emission,
// stable sort of the pairs by tile, tile ranges.  The sorted pairs end in
// (keys, vals).
ss_status run_binning(ss_context* c, const Group& g, int gi, hipStream_t st) {
  uint32_t* misc = P<uint32_t>(c->misc);
  const uint32_t* np = misc + kMiscPairs + gi;
  int* status = reinterpret_cast<int*>(misc + kMiscStatus);
  const long long n = g.rec_end - g.rec_begin;
  if (n <= 0) {
    SS_HIP(launch_fill_u32(misc + kMiscPairs + gi, 0u, 1, st));
    SS_HIP(launch_fill_u32(P<uint32_t>(c->ranges) + 2LL * g.tile_base, 0u, 2LL * g.n_tiles, st));
    return SS_OK;
  }
  uint32_t* zk = P<uint32_t>(c->zkey) + g.rec_begin;
  uint32_t* zi = P<uint32_t>(c->zidx) + g.rec_begin;
  uint2* zr = P<uint2>(c->zrect) + g.rec_begin;
  SS_HIP(launch_radix_sort(zk, zi, P<uint32_t>(c->zkey2) + g.rec_begin, P<uint32_t>(c->zidx2) + g.rec_begin,
                           true, (uint32_t)g.rec_begin, P<uint2>(c->prect), zr,
                           // culled records: depth key 0xffffffff, empty rectangle (1, 0)
                           0xffffffffu, make_uint2(1u, 0u), nullptr, n, n, 4, 8,
                           P<uint32_t>(c->hist), c->hist_n, P<uint32_t>(c->scan_tmp), c->scan_tmp_n, st));
  SS_HIP(launch_scan_rect_tiles(zr, c->opt.tile_w, c->opt.tile_h, P<uint32_t>(c->offsets) + g.rec_begin, n,
                                misc + kMiscPairs + gi, P<uint32_t>(c->scan_tmp), c->scan_tmp_n, st));
  // emit where an odd pass count leaves the sorted pairs in (keys, vals)
  uint32_t* keys = P<uint32_t>(c->keys) + g.pair_base;
  uint32_t* vals = P<uint32_t>(c->vals) + g.pair_base;
  uint32_t* keys2 = P<uint32_t>(c->keys2) + g.pair_base;
  uint32_t* vals2 = P<uint32_t>(c->vals2) + g.pair_base;
  const bool odd = (g.pair_passes & 1) != 0;
  SS_HIP(launch_emit_pairs(zi, zr, P<uint32_t>(c->offsets) + g.rec_begin, P<ViewDev>(c->views_d), g.v0, g.v1, n,
                           c->opt.tile_w, c->opt.tile_h, odd ? keys2 : keys, odd ? vals2 : vals, g.pair_cap, status,
                           st));
  SS_HIP(launch_radix_sort(odd ? keys2 : keys, odd ? vals2 : vals, odd ? keys : keys2, odd ? vals : vals2, false, 0u,
                           nullptr, nullptr, 0u, make_uint2(0u, 0u), np, -1, g.pair_cap, g.pair_passes, g.pair_first,
                           P<uint32_t>(c->hist), c->hist_n,
                           P<uint32_t>(c->scan_tmp), c->scan_tmp_n, st));
  SS_HIP(launch_tile_ranges(keys, np, g.pair_cap, P<uint32_t>(c->ranges), g.tile_base, g.n_tiles, st));
  return SS_OK;
}

// The second stream and its fork/join events of the backward (split-sum);
// created by the reserve, outside any graph capture.
static ss_status ensure_side(ss_context* c) {
  if (c->side || c->opt.shade != SS_SHADE_SPLITSUM) return SS_OK;
  SS_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  SS_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  SS_HIP(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
  return SS_OK;
}

// Host-side plan of a batch: counts, view layout and the groups of views that
// share a pair list (no device work, no allocation).
void plan_batch(ss_context* c, const ss_batch* b, std::vector<ViewDev>& vh) {
  c->n_views = b->n_views;
  c->n_scenes = b->n_scenes;
  c->N = b->surfel_offset[b->n_scenes];
  c->soff.assign(b->surfel_offset, b->surfel_offset + b->n_scenes + 1);
  build_views(c, b, vh);
  c->R = 0;
  c->n_pix = 0;
  c->n_tiles = 0;
  c->max_surf = 0;
  for (const ViewDev& v : vh) {
    c->R += v.n_surf;
    c->n_pix += (long long)v.W * v.H;
    c->n_tiles += v.tiles_x * v.tiles_y;
    c->max_surf = v.n_surf > c->max_surf ? v.n_surf : c->max_surf;
  }
  c->groups.clear();
  const int ng = c->opt.launch == SS_LAUNCH_PER_VIEW ? b->n_views : 1;
  for (int gi = 0; gi < ng; ++gi) {
    Group g;
    g.v0 = ng == 1 ? 0 : gi;
    g.v1 = ng == 1 ? b->n_views : gi + 1;
    g.tile_base = vh[g.v0].tile_base;
    g.n_tiles = 0;
    for (int v = g.v0; v < g.v1; ++v) g.n_tiles += vh[v].tiles_x * vh[v].tiles_y;
    g.rec_begin = vh[g.v0].rec_off;
    g.rec_end = vh[g.v1 - 1].rec_off + vh[g.v1 - 1].n_surf;
    {
      const int bits = g.n_tiles > 1 ? bits_for(g.n_tiles) : 0;
      g.pair_first = bits > 1 && bits % 8 == 1 ? 9 : 8;  // e.g. 17 bits: 9 + 8
      g.pair_passes = bits > 0 ? (bits - (g.pair_first - 8) + 7) / 8 : 0;
    }
    g.pair_base = 0;
    g.pair_cap = 0;
    g.mask_base = 0;
    g.mask_n = 0;
    g.item_base = g.item_cap = g.mitem_base = g.mitem_cap = 0;
    c->groups.push_back(g);
  }
  c->lds_batch = c->opt.lds_batch > 0 ? c->opt.lds_batch : 128;
}

// Chunk slots of the walk masks for every group (after the pair capacities);
// returns the number of 64-bit masks.
long long layout_masks(ss_context* c) {
  long long base = 0;
  for (Group& g : c->groups) {
    g.mask_base = base;
    g.mask_n = mask_slots(g.pair_cap, g.n_tiles);
    base += g.mask_n;
  }
  return base * (long long)(c->opt.tile_w * c->opt.tile_h / 16);
}

// The split-list buffers of a group (items null: lists are not split).
SegBufs seg_bufs(ss_context* c, const Group& g, int gi, bool split) {
  SegBufs sb{};
  if (!split) return sb;
  const size_t np = (size_t)c->opt.tile_w * c->opt.tile_h, m0 = (size_t)g.mitem_base * np;
  uint32_t* misc = P<uint32_t>(c->misc);
  sb.items = P<int4>(c->items) + g.item_base;
  sb.n_items = misc + kMiscSeg + 2 * gi;
  sb.mitems = P<int4>(c->mitems) + g.mitem_base;
  sb.n_mitems = misc + kMiscSeg + 2 * gi + 1;
  sb.seg_len = c->seg_len;
  sb.L = P<float4>(c->segL) + m0 * kSegLayers;
  sb.S = P<uint16_t>(c->segS) + m0 * (kSegLayers + 1);
  sb.F = P<uint16_t>(c->segF) + m0 * kSegLayers;
  sb.M = P<uint32_t>(c->segM) + m0;
  sb.Z = P<float>(c->segZ) + m0;
  sb.ZI = P<float>(c->segZI) + m0;
  return sb;
}

WalkBufs walk_bufs(ss_context* c, const Group& g) {
  WalkBufs w;
  w.pos = P<uint32_t>(c->lpos);
  w.masks = P<uint64_t>(c->qmask);
  w.mask_base = g.mask_base;
  const bool det = c->opt.deterministic && c->pgrad.p;
  w.pgrad = det ? P<float>(c->pgrad) : nullptr;
  w.inv = det ? P<uint32_t>(c->inv) : nullptr;
  w.offs = P<uint32_t>(c->offsets) + g.rec_begin;
  w.pair_base = g.pair_base;
  w.ovf = c->ovf.p ? P<float4>(c->ovf) : nullptr;
  return w;
}

ss_status reserve_impl(ss_context* c, const ss_batch* b, hipStream_t st) {
  c->reserved = false;
  c->fwd_valid = false;
  c->views_uploaded = false;
  c->n_scenes = b->n_scenes;
  SS_TRY(prepare_env(c, b, st));
  std::vector<ViewDev> vh;
  plan_batch(c, b, vh);
  const long long R = c->R > 0 ? c->R : 1;
  SS_HIP(ensure(c->views_d, sizeof(ViewDev) * kMaxViews));
  SS_HIP(ensure(c->recs, (size_t)R * kRecFloats * sizeof(float)));
  SS_HIP(ensure(c->counts, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->offsets, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->zkey, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->zkey2, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->zidx, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->zidx2, (size_t)R * sizeof(uint32_t)));
  SS_HIP(ensure(c->prect, (size_t)R * sizeof(uint2)));
  SS_HIP(ensure(c->zrect, (size_t)R * sizeof(uint2)));
  SS_HIP(ensure(c->misc, kMiscWords * sizeof(uint32_t)));
  c->scan_tmp_n = scan_tmp_size(R > c->n_tiles ? R : c->n_tiles) + 16;
  SS_HIP(ensure(c->scan_tmp, (size_t)c->scan_tmp_n * sizeof(uint32_t)));
  SS_HIP(ensure(c->ranges, (size_t)2 * (c->n_tiles > 0 ? c->n_tiles : 1) * sizeof(uint32_t)));
  SS_HIP(ensure(c->nl, (size_t)(c->n_pix > 0 ? c->n_pix : 1)));
  SS_HIP(ensure(c->order, (size_t)(c->n_tiles > 0 ? c->n_tiles : 1) * sizeof(int)));
  SS_HIP(ensure(c->stats, (size_t)(c->n_pix > 0 ? c->n_pix : 1) * kMaxLayers * sizeof(float4)));
  SS_HIP(ensure(c->lpos, (size_t)(c->n_pix > 0 ? c->n_pix : 1) * kPosStride * sizeof(uint32_t)));
  if (c->opt.depth_stats)
    SS_HIP(ensure(c->stats2, (size_t)(c->n_pix > 0 ? c->n_pix : 1) * kMaxLayers * sizeof(float2)));
  SS_HIP(ensure(c->grad, (size_t)R * kGradStride * sizeof(float)));
  if (c->opt.shade == SS_SHADE_SPLITSUM) SS_HIP(ensure(c->sg, (size_t)R * 12 * sizeof(float)));
  SS_TRY(upload_views(c, b, st));
  // count the pairs once
  SS_TRY(run_envmap_prefilter(c, b, st));
  SS_TRY(run_preprocess(c, b, 0, b->n_views, st));
  for (Group& g : c->groups) SS_TRY(run_count_scan(c, g, st));
  std::vector<uint32_t> np(c->groups.size());
  SS_HIP(hipStreamSynchronize(st));
  SS_HIP(hipMemcpy(np.data(), P<uint32_t>(c->misc) + kMiscPairs, np.size() * sizeof(uint32_t),
                   hipMemcpyDeviceToHost));
  long long base = 0, maxcap = 0;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    Group& g = c->groups[gi];
    const long long p = np[gi];
    g.pair_cap = p + p / 4 + 4096;
    g.pair_base = base;
    base += g.pair_cap;
    maxcap = g.pair_cap > maxcap ? g.pair_cap : maxcap;
  }
  c->pair_total = base;
  if (c->opt.lds_batch == 0) {
    // the largest batch not above the mean tile-list length (at least 32)
    long long np_all = 0;
    for (uint32_t x : np) np_all += x;
    const double mean = c->n_tiles > 0 ? (double)np_all / c->n_tiles : 0.0;
    c->lds_batch = mean >= 256 ? 256 : (mean >= 128 ? 128 : (mean >= 64 ? 64 : 32));
  }
  SS_HIP(ensure(c->qmask, (size_t)layout_masks(c) * sizeof(uint64_t)));
  if (backward_walk(c) == 2) {  // entry float4s per layer: 1, + 1 normal image, + 2 depth statistics
    const int lw4 = 1 + (c->opt.shade == SS_SHADE_NORMAL ? 1 : 0) + (c->opt.depth_stats ? 2 : 0);
    SS_HIP(ensure(c->ovf, (size_t)(c->n_pix > 0 ? c->n_pix : 1) * (kMaxLayers - kBwdTabLayers) * lw4 *
                              sizeof(float4)));
  }
  // split lists (persistent launches): a group's items are its tiles plus one
  // per further segment; a split tile's segments number at most 2 len / seg_len
  c->seg_len = (!c->opt.persistent || c->opt.seg_len < 0) ? 0 : (c->opt.seg_len > 0 ? c->opt.seg_len : 2048);
  if (c->seg_len > 0) {
    long long ib = 0, mb = 0, maxt = 1;
    for (Group& g : c->groups) {
      g.item_base = ib;
      g.item_cap = g.n_tiles + g.pair_cap / c->seg_len + 1;
      g.mitem_base = mb;
      g.mitem_cap = 2 * g.pair_cap / c->seg_len + 2;
      ib += g.item_cap;
      mb += g.mitem_cap;
      maxt = g.n_tiles > maxt ? g.n_tiles : maxt;
    }
    const size_t np = (size_t)mb * c->opt.tile_w * c->opt.tile_h;
    SS_HIP(ensure(c->items, (size_t)ib * sizeof(int4)));
    SS_HIP(ensure(c->mitems, (size_t)mb * sizeof(int4)));
    SS_HIP(ensure(c->segbase, (size_t)2 * maxt * sizeof(uint32_t)));
    SS_HIP(ensure(c->segL, np * kSegLayers * sizeof(float4)));
    SS_HIP(ensure(c->segS, np * (kSegLayers + 1) * sizeof(uint16_t)));
    SS_HIP(ensure(c->segF, np * kSegLayers * sizeof(uint16_t)));
    SS_HIP(ensure(c->segM, np * sizeof(uint32_t)));
    SS_HIP(ensure(c->segZ, np * sizeof(float)));
    SS_HIP(ensure(c->segZI, np * sizeof(float)));
  }
  if (c->opt.deterministic) {
    SS_HIP(ensure(c->pgrad, (size_t)base * sub_tiles(c->opt.tile_w, c->opt.tile_h) * kGradStride * sizeof(float)));
    SS_HIP(ensure(c->inv, (size_t)R * sizeof(uint32_t)));
    SS_HIP(ensure(c->detw, (size_t)2 * (c->n_scenes > 0 ? c->n_scenes : 1) * sizeof(uint32_t)));
  }
  SS_HIP(ensure(c->keys, (size_t)base * sizeof(uint32_t)));
  SS_HIP(ensure(c->keys2, (size_t)base * sizeof(uint32_t)));
  SS_HIP(ensure(c->vals, (size_t)base * sizeof(uint32_t)));
  SS_HIP(ensure(c->vals2, (size_t)base * sizeof(uint32_t)));
  long long maxrec = 0;
  for (const Group& g : c->groups) maxrec = g.rec_end - g.rec_begin > maxrec ? g.rec_end - g.rec_begin : maxrec;
  c->hist_n = radix_hist_size(maxcap) > radix_hist_size(maxrec) ? radix_hist_size(maxcap) : radix_hist_size(maxrec);
  SS_HIP(ensure(c->hist, (size_t)c->hist_n * sizeof(uint32_t)));
  const long long need_scan = scan_tmp_size(c->hist_n > R ? c->hist_n : R) + 16;
  if (need_scan > c->scan_tmp_n) {
    c->scan_tmp_n = need_scan;
    SS_HIP(ensure(c->scan_tmp, (size_t)need_scan * sizeof(uint32_t)));
  }
  c->sig = signature(c, b);
  c->reserved = true;
  SS_TRY(ensure_side(c));
  return SS_OK;
}

// Stage timing: events recorded around a stage when profiling is on; resolved
// (and recycled) by ss_profile_read.
hipEvent_t prof_event(ss_context* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
hipEvent_t prof_begin(ss_context* c, hipStream_t st) {
  if (!c->prof) return nullptr;
  hipEvent_t a = prof_event(c);
  if (a) {
    const hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess && std::getenv("SURFSPLAT_DEBUG"))
      std::fprintf(stderr, "prof_begin: hipEventRecord: %s\n", hipGetErrorString(e));
  }
  return a;
}
void prof_end(ss_context* c, hipEvent_t a, int stage, hipStream_t st) {
  if (!c->prof || !a) return;
  hipEvent_t b = prof_event(c);
  if (!b) return;
  (void)hipEventRecord(b, st);
  c->prof_ev.push_back({stage, {a, b}});
}
enum { ST_ENV = 0, ST_PRE, ST_BIN, ST_RFWD, ST_RBWD, ST_PREBWD, ST_ENVBWD };

size_t workspace_bytes(const ss_context* c) {
  size_t s = c->views_d.n + c->recs.n + c->counts.n + c->offsets.n + c->scan_tmp.n + c->keys.n +
             c->vals.n + c->keys2.n + c->vals2.n + c->hist.n + c->ranges.n + c->nl.n + c->stats.n +
             c->grad.n + c->misc.n + c->lut.n + c->partial.n + c->sg.n + c->order.n + c->stats2.n + c->zkey.n +
             c->zkey2.n + c->zidx.n + c->zidx2.n + c->prect.n + c->zrect.n + c->lpos.n + c->qmask.n +
             c->pgrad.n + c->inv.n + c->detw.n + c->items.n + c->mitems.n + c->segbase.n + c->segL.n + c->segS.n +
             c->segF.n + c->segM.n + c->segZ.n + c->segZI.n + c->ovf.n;
  for (const SceneEnv& e : c->env) s += e.dirs.n + e.lv.n + e.Z.n + e.dlv.n + e.part.n + e.dlv_fx.n + e.adj_part.n;
  return s;
}


// Non-finite surfel parameters (and environment texels) of a batch, counted
// into the 64-bit word `cnt` (options.validate).
ss_status count_nonfinite_inputs(ss_context* c, const ss_batch* b, unsigned long long* cnt, hipStream_t st) {
  const float* pp[7];
  param_ptrs(b, pp);
  const int rows[7] = {3, 3, 3, 2, 3, 1, 1};
  for (int a = 0; a < 7; ++a)
    if (c->N > 0) SS_HIP(launch_count_nonfinite(pp[a], (long long)rows[a] * c->N, cnt, st));
  if (c->opt.shade == SS_SHADE_SPLITSUM)
    for (int s = 0; s < b->n_scenes; ++s)
      SS_HIP(launch_count_nonfinite(b->envmap[s], 3LL * b->env_hw[2 * s] * b->env_hw[2 * s + 1], cnt, st));
  return SS_OK;
}

// The forward pipeline on a planned and sized workspace whose view table is on
// the device: environment levels, then per group preprocess + shading,
// binning, tile order and the raster forward.  Clears the device words it
// relies on first.
ss_status forward_body(ss_context* c, const ss_batch* b, const ss_outputs* out, hipStream_t st) {
  uint32_t* misc = P<uint32_t>(c->misc);
  SS_HIP(launch_fill_u32(misc, 0u, kMiscPairs, st));
  SS_HIP(launch_fill_u32(misc + kMiscNonfinite, 0u, 4, st));  // both non-finite counters
  if (c->opt.counters) SS_HIP(launch_fill_u32(misc + kMiscCounters, 0u, 8, st));
  if (c->opt.validate)
    SS_TRY(count_nonfinite_inputs(c, b, reinterpret_cast<unsigned long long*>(misc + kMiscNonfinite), st));
  hipEvent_t t0 = prof_begin(c, st);
  SS_TRY(run_envmap_prefilter(c, b, st));
  prof_end(c, t0, ST_ENV, st);
  Params prm = make_params(c);
  prm.cons = (out->cons || out->depth) ? 1 : 0;
  int* status = reinterpret_cast<int*>(misc + kMiscStatus);
  // long lists split into segments (persistent launches without depth statistics)
  const bool split = c->seg_len > 0 && c->opt.persistent && !prm.cons;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& g = c->groups[gi];
    t0 = prof_begin(c, st);
    SS_TRY(run_preprocess(c, b, g.v0, g.v1, st));
    prof_end(c, t0, ST_PRE, st);
    t0 = prof_begin(c, st);
    SS_TRY(run_binning(c, g, (int)gi, st));
    uint32_t* vals = P<uint32_t>(c->vals) + g.pair_base;
    int* order = nullptr;
    if (c->opt.persistent) {
      order = P<int>(c->order) + g.tile_base;
      SS_HIP(launch_tile_order(P<uint32_t>(c->ranges), g.tile_base, g.n_tiles, order,
                               misc + kMiscOrder, st));
    }
    const SegBufs sb = seg_bufs(c, g, (int)gi, split);
    if (split)
      SS_HIP(launch_seg_items(P<uint32_t>(c->ranges), order, g.n_tiles, c->seg_len,
                              c->opt.tile_w * c->opt.tile_h, misc + kMiscPairs + gi,
                              P<uint32_t>(c->segbase), misc + kMiscSeg + 2 * gi, P<int4>(c->items) + g.item_base,
                              P<int4>(c->mitems) + g.mitem_base, g.item_cap, g.mitem_cap,
                              P<uint32_t>(c->scan_tmp), c->scan_tmp_n, st));
    prof_end(c, t0, ST_BIN, st);
    SS_HIP(launch_fill_u32(misc + kMiscQueue, 0u, 1, st));
    const WalkBufs wb = walk_bufs(c, g);
    // chunks the forward does not reach keep empty masks
    SS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(wb.masks + g.mask_base * (c->opt.tile_w * c->opt.tile_h / 16)),
                           0u, 2LL * g.mask_n * (c->opt.tile_w * c->opt.tile_h / 16), st));
    t0 = prof_begin(c, st);
    SS_HIP(launch_raster_forward(P<ViewDev>(c->views_d), c->n_views, g.tile_base,
                                 g.tile_base + g.n_tiles, P<uint32_t>(c->ranges), vals,
                                 P<float>(c->recs), prm, c->lds_batch, out->image, out->alpha,
                                 out->n_layers, P<uint8_t>(c->nl), P<float4>(c->stats),
                                 P<float2>(c->stats2), out->cons, out->depth,
                                 reinterpret_cast<int*>(misc + kMiscQueue), order,
                                 c->opt.persistent, status,
                                 reinterpret_cast<unsigned long long*>(misc + kMiscCounters), wb, sb, g.item_cap,
                                 g.mitem_cap, st));
    prof_end(c, t0, ST_RFWD, st);
  }
  c->fwd_split = split;
  return SS_OK;
}

// ---------------------------------------------------------------- fixed workspace
// The workspace of ss_render_static: one file-scope device array per GPU (the
// code object's global segment, held until the process ends).  Host code
// never uses the name `scratch` as an address: it is a host-side stand-in.
// Each device's own address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address reaches kernels.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
long long g_static_cap[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[SS_STATIC_SCRATCH_BYTES];

namespace {

// Address of the current device's copy of `scratch`.
ss_status static_scratch(void** out, int* dev_out) {
  int dev = 0;
  SS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    SS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SS_ERR_HIP;
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  *dev_out = dev;
  return SS_OK;
}

// Buffers cut in order from one region (256-byte aligned); `ok` turns false
// once a request does not fit.
struct Carver {
  char* base;
  size_t cap;
  size_t used = 0;
  bool ok = true;
  void take(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    const size_t off = (used + 255) & ~size_t(255);
    if (!ok || off > cap || bytes > cap - off) {
      ok = false;
      b.p = nullptr;
      b.n = 0;
      return;
    }
    b.p = base + off;
    b.n = bytes;
    used = off + bytes;
  }
};

// View descriptors travel as kernel arguments (no host-to-device copy, so the
// call also works under graph capture), kViewsPerStore at a time.
constexpr int kViewsPerStore = 8;
struct ViewStore {
  ViewDev v[kViewsPerStore];
  int n;
};
static_assert(sizeof(ViewStore) <= 3072, "view store exceeds the kernel-argument budget");
__global__ void store_views_kernel(ViewStore src, ViewDev* dst) {
  const int words = src.n * (int)(sizeof(ViewDev) / sizeof(uint32_t));
  for (int i = threadIdx.x; i < words; i += blockDim.x)
    reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(src.v)[i];
}

// ss_poll's view of the last ss_render_static on the current device: the
// status and pair-count words sit at the start of the array.
ss_status static_poll(ss_diag* out) {
  int dev = 0;
  SS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SS_OK;
  void* p = nullptr;
  long long cap = 0;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    p = g_static_ptr[dev];
    cap = g_static_cap[dev];
  }
  if (!p || cap == 0) return SS_OK;
  SS_HIP(hipDeviceSynchronize());
  uint32_t m[kMiscPairs + 1];
  SS_HIP(hipMemcpy(m, p, sizeof(m), hipMemcpyDeviceToHost));
  out->static_status = (int32_t)m[kMiscStatus];
  out->static_pairs = m[kMiscPairs];
  out->static_pair_capacity = cap;
  return SS_OK;
}
}  // namespace

extern "C" {

ss_status ss_default_options(ss_options* o) {
  if (!o) return SS_ERR_INVALID_ARG;
  o->r_cut = 3.f;
  o->k_max = 16;
  o->gamma = 2.f * kPi;
  o->sigma_f = 0.1f;
  o->shade = SS_SHADE_ALBEDO;
  o->tile_w = 16;
  o->tile_h = 16;
  o->lds_batch = 128;
  o->launch = SS_LAUNCH_BATCHED;
  o->persistent = 1;
  o->depth_stats = 0;
  o->mip = 0;
  o->env_lds = -1;
  o->t_min = 0.f;
  o->deterministic = 0;
  o->validate = 0;
  o->counters = 0;
  o->tonemap = 0;
  o->seg_len = 0;
  o->bwd_walk = 0;
  return SS_OK;
}

ss_status ss_create(const ss_options* opt, ss_context** out) {
  if (!out) return SS_ERR_INVALID_ARG;
  *out = nullptr;
  SS_TRY(check_options(opt));
  ss_context* c = new (std::nothrow) ss_context();
  if (!c) return SS_ERR_NOMEM;
  c->opt = *opt;
  *out = c;
  return SS_OK;
}

ss_status ss_destroy(ss_context* c) {
  if (!c) return SS_ERR_INVALID_ARG;
  if (c->used) (void)hipStreamSynchronize(c->last_stream);
  DevBuf* bufs[] = {&c->views_d, &c->recs, &c->counts, &c->offsets, &c->scan_tmp, &c->keys,
                    &c->vals, &c->keys2, &c->vals2, &c->hist, &c->ranges, &c->nl, &c->stats,
                    &c->grad, &c->misc, &c->lut, &c->partial, &c->sg, &c->order, &c->stats2,
                    &c->zkey, &c->zkey2, &c->zidx, &c->zidx2, &c->prect, &c->zrect, &c->lpos, &c->qmask,
                    &c->pgrad, &c->inv, &c->detw, &c->items, &c->mitems, &c->segbase, &c->segL, &c->segS,
                    &c->segF, &c->segM, &c->segZ, &c->segZI, &c->ovf};
  for (DevBuf* b : bufs) release(*b);
  for (SceneEnv& e : c->env) {
    release(e.dirs); release(e.lv); release(e.Z); release(e.dlv); release(e.part);
    release(e.dlv_fx); release(e.adj_part);
  }
  for (auto& pe : c->prof_ev) { c->ev_pool.push_back(pe.second.first); c->ev_pool.push_back(pe.second.second); }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
    (void)hipEventDestroy(c->fork_ev);
    (void)hipEventDestroy(c->join_ev);
  }
  delete c;
  return SS_OK;
}

ss_status ss_set_options(ss_context* c, const ss_options* opt) {
  if (!c) return SS_ERR_INVALID_ARG;
  SS_TRY(check_options(opt));
  if (c->used) SS_HIP(hipStreamSynchronize(c->last_stream));
  c->opt = *opt;
  c->reserved = false;
  c->fwd_valid = false;
  c->views_uploaded = false;
  return SS_OK;
}

ss_status ss_brdf_lut(float* lut, int32_t n_nv, int32_t n_r, int32_t samples, ss_stream stream) {
  if (!lut || n_nv < 2 || n_r < 2 || n_nv > 1024 || n_r > 1024 || samples < 1 || samples > 65536)
    return SS_ERR_INVALID_ARG;
  SS_HIP(launch_brdf_lut(lut, n_nv, n_r, samples, (hipStream_t)stream));
  return SS_OK;
}

ss_status ss_set_brdf_lut(ss_context* c, const float* lut, int32_t n_nv, int32_t n_r, ss_stream stream) {
  if (!c || !lut || n_nv < 2 || n_r < 2 || n_nv > 1024 || n_r > 1024) return SS_ERR_INVALID_ARG;
  const size_t bytes = (size_t)n_nv * n_r * 2 * sizeof(float);
  if (c->lut.n < bytes && c->used) SS_HIP(hipStreamSynchronize(c->last_stream));
  SS_HIP(ensure(c->lut, bytes));
  SS_HIP(hipMemcpyAsync(c->lut.p, lut, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  c->lut_nv = n_nv;
  c->lut_r = n_r;
  return SS_OK;
}

ss_status ss_reserve(ss_context* c, const ss_batch* b, ss_stream stream, size_t* ws) {
  if (!c) return SS_ERR_INVALID_ARG;
  SS_TRY(check_batch(c, b));
  if (c->opt.shade == SS_SHADE_SPLITSUM && !c->lut.p) return SS_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  c->used = true;
  SS_TRY(reserve_impl(c, b, st));
  if (ws) *ws = workspace_bytes(c);
  return SS_OK;
}

ss_status ss_render(ss_context* c, const ss_batch* b, const ss_outputs* out, ss_stream stream) {
  if (!c || !out || !out->image || !out->alpha) return SS_ERR_INVALID_ARG;
  if ((out->cons || out->depth) && !c->opt.depth_stats) return SS_ERR_INVALID_ARG;
  SS_TRY(check_batch(c, b));
  if (c->opt.shade == SS_SHADE_SPLITSUM && !c->lut.p) return SS_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  c->used = true;
  if (!c->reserved || signature(c, b) != c->sig) SS_TRY(reserve_impl(c, b, st));
  c->fwd_valid = false;
  SS_TRY(upload_views(c, b, st));
  SS_TRY(forward_body(c, b, out, st));
  c->fwd_valid = true;
  c->fwd_cons = out->cons || out->depth;
  c->fwd_sig = c->sig;
  ++c->generation;
  if (out->generation) *out->generation = c->generation;
  return SS_OK;
}

// Environment adjoint of every scene with a requested map gradient, on `st`.
static ss_status envmap_backward(ss_context* c, const ss_grads* gr, const int* status, hipStream_t st) {
  if (c->opt.shade != SS_SHADE_SPLITSUM || !gr->d_envmap) return SS_OK;
  for (int s = 0; s < c->n_scenes; ++s) {
    if (!gr->d_envmap[s]) continue;
    SceneEnv& e = c->env[s];
    const float* dl[7];
    for (int l = 0; l < 7; ++l) dl[l] = P<float>(e.dlv) + e.doff[l];
    SS_HIP(launch_envmap_adjoint(dl, e.lh, e.lw, P<float>(e.Z), e.He, e.We, P<float>(e.dirs),
                                 gr->d_envmap[s], status, c->opt.deterministic ? P<float>(e.adj_part) : nullptr,
                                 st));
  }
  return SS_OK;
}

ss_status ss_render_backward(ss_context* c, const ss_batch* b, const ss_grad_in* gin,
                             const ss_grads* gr, ss_stream stream) {
  if (!c || !gin || !gin->d_image || !gr) return SS_ERR_INVALID_ARG;
  SS_TRY(check_batch(c, b));
  if (!c->fwd_valid || signature(c, b) != c->fwd_sig) return SS_ERR_STATE;
  if (gin->generation != 0 && gin->generation != c->generation) return SS_ERR_STATE;
  if ((gin->d_cons || gin->d_depth) && !c->fwd_cons) return SS_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  c->used = true;
  SS_TRY(upload_views(c, b, st));
  Params prm = make_params(c);
  prm.ss_grad = gr->screen_grad ? 1 : 0;
  prm.cons = (gin->d_cons || gin->d_depth) ? 1 : 0;
  uint32_t* misc = P<uint32_t>(c->misc);
  const int* status = reinterpret_cast<const int*>(misc + kMiscStatus);
  if (c->opt.validate) {
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(misc + kMiscNonfinite) + 1;
    SS_HIP(launch_fill_u32(misc + kMiscNonfinite + 2, 0u, 2, st));
    SS_HIP(launch_count_nonfinite(gin->d_image, 3 * c->n_pix, cnt, st));
    if (gin->d_alpha) SS_HIP(launch_count_nonfinite(gin->d_alpha, c->n_pix, cnt, st));
  }
  const bool det = c->opt.deterministic != 0;
  SS_HIP(launch_fill_f32(P<float>(c->grad), 0.f, (long long)c->R * kGradStride, st));
  if (c->opt.shade == SS_SHADE_SPLITSUM)
    for (SceneEnv& e : c->env) SS_HIP(launch_fill_f32(P<float>(e.dlv), 0.f, (long long)(e.dlv.n / 4), st));
  if (det)
    SS_HIP(launch_fill_f32(P<float>(c->pgrad), 0.f,
                           c->pair_total * sub_tiles(c->opt.tile_w, c->opt.tile_h) * kGradStride, st));
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& g = c->groups[gi];
    if (det)
      SS_HIP(launch_invert_order(P<uint32_t>(c->zidx) + g.rec_begin, g.rec_end - g.rec_begin, P<uint32_t>(c->inv),
                                 st));
    SS_HIP(launch_fill_u32(misc + kMiscQueue, 0u, 1, st));
    hipEvent_t t0 = prof_begin(c, st);
    SS_HIP(launch_raster_backward(P<ViewDev>(c->views_d), c->n_views, g.tile_base,
                                  g.tile_base + g.n_tiles, P<uint32_t>(c->ranges),
                                  P<uint32_t>(c->vals) + g.pair_base, P<float>(c->recs), prm,
                                  c->lds_batch, gin->d_image, gin->d_alpha, P<uint8_t>(c->nl),
                                  P<float4>(c->stats), P<float2>(c->stats2), gin->d_cons, gin->d_depth,
                                  P<float>(c->grad), reinterpret_cast<int*>(misc + kMiscQueue),
                                  c->opt.persistent ? P<int>(c->order) + g.tile_base : nullptr,
                                  c->opt.persistent, walk_bufs(c, g), seg_bufs(c, g, (int)gi, c->fwd_split),
                                  g.item_cap, st));
    if (det)  // each record's gradient: its (record, tile) partials in emission order
      SS_HIP(launch_ordered_record_sums(P<uint32_t>(c->zidx) + g.rec_begin, P<uint2>(c->zrect) + g.rec_begin,
                                        P<uint32_t>(c->offsets) + g.rec_begin, g.rec_end - g.rec_begin,
                                        c->opt.tile_w, c->opt.tile_h, P<float>(c->pgrad), g.pair_base,
                                        g.pair_cap, P<float>(c->grad), st));
    prof_end(c, t0, ST_RBWD, st);
  }
  const float* pp[7];
  param_ptrs(b, pp);
  float* G[7] = {gr->d_position, gr->d_normal, gr->d_tangent, gr->d_scale,
                 gr->d_albedo, gr->d_roughness, gr->d_metallic};
  hipEvent_t t1 = prof_begin(c, st);
  if (c->opt.shade == SS_SHADE_SPLITSUM) {
    for (int s = 0; s < c->n_scenes; ++s) {
      SceneEnv& e = c->env[s];
      float* lg[7];
      for (int l = 0; l < 7; ++l) lg[l] = P<float>(e.dlv) + e.doff[l];
      std::vector<int> sv;
      for (int v = 0; v < c->n_views; ++v)
        if (c->views_h[v].scene == s) sv.push_back(v);
      int* fx_exp = nullptr;
      if (det) {  // fixed-point texel gradients with a scale bounded from this scene's records
        unsigned* bound = P<unsigned>(c->detw) + 2 * s;
        fx_exp = reinterpret_cast<int*>(bound + 1);
        SS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(P<long long>(e.dlv_fx)), 0u,
                               (long long)(e.dlv_fx.n / 4), st));
        SS_HIP(launch_fixed_point_scale(P<float>(c->grad), b->albedo, c->N, P<ViewDev>(c->views_d), sv.data(),
                                        (int)sv.size(), c->soff[s + 1] - c->soff[s], bound, fx_exp, st));
      }
      SS_HIP(launch_shade_backward(pp, c->N, P<ViewDev>(c->views_d), sv.data(), (int)sv.size(), c->soff[s],
                                   (int)(c->soff[s + 1] - c->soff[s]), e.loc_off, e.loc_total,
                                   P<float>(c->partial), lg, prm, P<float>(c->grad), P<float>(c->sg), fx_exp,
                                   st));
      if (det)  // exactly the texels of levels 0..6 (the buffers may be larger)
        SS_HIP(launch_fixed_to_float(P<long long>(e.dlv_fx), e.doff[6] + 3LL * e.lh[6] * e.lw[6], fx_exp,
                                     P<float>(e.dlv), st));
    }
  }
  // The environment adjoint reads only the level gradients that the shading
  // adjoint wrote, as does the geometry adjoint its record gradients: with stage
  // timing off it runs on a second stream beside the geometry adjoint and is
  // joined back into `st` before this call returns.
  const bool fork = c->opt.shade == SS_SHADE_SPLITSUM && gr->d_envmap && !c->prof;
  if (fork) {
    SS_TRY(ensure_side(c));
    SS_HIP(hipEventRecord(c->fork_ev, st));
    SS_HIP(hipStreamWaitEvent(c->side, c->fork_ev, 0));
    SS_TRY(envmap_backward(c, gr, status, c->side));
    SS_HIP(hipEventRecord(c->join_ev, c->side));
  }
  SS_HIP(launch_geometry_backward(pp, c->N, P<ViewDev>(c->views_d), c->n_views, prm, P<float>(c->grad),
                                  P<float>(c->sg), G, P<float>(c->recs), gr->screen_grad,
                                  gr->visible_views, status, st));
  prof_end(c, t1, ST_PREBWD, st);
  if (fork) {
    SS_HIP(hipStreamWaitEvent(st, c->join_ev, 0));
  } else {
    t1 = prof_begin(c, st);
    SS_TRY(envmap_backward(c, gr, status, st));
    prof_end(c, t1, ST_ENVBWD, st);
  }
  return SS_OK;
}

ss_status ss_poll(ss_context* c, ss_diag* out) {
  if (!c || !out) return SS_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  if (c->used) SS_HIP(hipStreamSynchronize(c->last_stream));
  if (c->misc.p) {
    std::vector<uint32_t> m(kMiscWords);
    SS_HIP(hipMemcpy(m.data(), c->misc.p, m.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    out->status = (int32_t)m[kMiscStatus];
    long long np = 0;
    for (size_t g = 0; g < c->groups.size(); ++g) np += m[kMiscPairs + g];
    out->n_pairs = np;
    unsigned long long u[6];
    std::memcpy(u, m.data() + kMiscNonfinite, sizeof(u));
    out->n_nonfinite = (int64_t)(u[0] + u[1]);
    if (c->opt.counters) {
      out->n_evaluated = (int64_t)u[2];
      out->n_fragments = (int64_t)u[3];
      out->n_layers = (int64_t)u[4];
      std::memcpy(&out->sum_layer_weight, &u[5], sizeof(double));
    }
  }
  out->n_records = c->R;
  out->pair_capacity = c->pair_total;
  out->workspace_bytes = (int64_t)workspace_bytes(c);
  out->generation = c->generation;
  SS_TRY(static_poll(out));
  return out->status == 0 ? SS_OK : (ss_status)out->status;
}

ss_status ss_profile_enable(ss_context* c, int32_t enable) {
  if (!c) return SS_ERR_INVALID_ARG;
  c->prof = enable != 0;
  return SS_OK;
}

ss_status ss_profile_read(ss_context* c, double* ms, int64_t* count) {
  if (!c) return SS_ERR_INVALID_ARG;
  if (ms) for (int i = 0; i < SS_NUM_STAGES; ++i) ms[i] = 0.0;
  if (count) for (int i = 0; i < SS_NUM_STAGES; ++i) count[i] = 0;
  if (c->used) SS_HIP(hipStreamSynchronize(c->last_stream));
  int reported = 0;
  for (auto& pe : c->prof_ev) {
    float t = 0.f;
    (void)hipEventSynchronize(pe.second.second);
    const hipError_t e = hipEventElapsedTime(&t, pe.second.first, pe.second.second);
    if (e == hipSuccess) {
      if (ms) ms[pe.first] += t;
      if (count) count[pe.first] += 1;
    } else if (std::getenv("SURFSPLAT_DEBUG") && reported++ < 4) {
      std::fprintf(stderr, "ss_profile_read: stage %d: %s\n", pe.first, hipGetErrorString(e));
    }
    c->ev_pool.push_back(pe.second.first);
    c->ev_pool.push_back(pe.second.second);
  }
  c->prof_ev.clear();
  return SS_OK;
}

}  // extern "C"


// Allocation-free forward: the workspace of one batched group is carved from
// the current device's `scratch` (status words first), the pair capacity is
// whatever is left, and the pipeline is forward_body, as in ss_render.
extern "C" ss_status ss_render_static(ss_context* c, const ss_batch* b, const ss_outputs* out,
                                      ss_stream stream) {
  if (!c || !out || !out->image || !out->alpha) return SS_ERR_INVALID_ARG;
  if ((out->cons || out->depth) && !c->opt.depth_stats) return SS_ERR_INVALID_ARG;
  SS_TRY(check_batch(c, b));
  if (c->opt.shade == SS_SHADE_SPLITSUM && !c->lut.p) return SS_ERR_STATE;
  if (c->opt.launch != SS_LAUNCH_BATCHED) return SS_ERR_UNSUPPORTED;
  void* base = nullptr;
  int dev = 0;
  SS_TRY(static_scratch(&base, &dev));
  hipStream_t st = (hipStream_t)stream;
  // a workspace over the array; nothing below allocates device memory, and
  // none of its buffers is ever released
  ss_context w;
  w.opt = c->opt;
  w.lut = c->lut;
  w.lut_nv = c->lut_nv;
  w.lut_r = c->lut_r;
  Carver cv{static_cast<char*>(base), (size_t)SS_STATIC_SCRATCH_BYTES};
  cv.take(w.misc, kMiscWords * sizeof(uint32_t));
  if (c->opt.shade == SS_SHADE_SPLITSUM) {
    w.env.resize(b->n_scenes);
    for (int s = 0; s < b->n_scenes; ++s) {
      SceneEnv& e = w.env[s];
      const int He = b->env_hw[2 * s], We = b->env_hw[2 * s + 1];
      long long lv_n = 0, dlv_n = 0;
      env_layout(&w, b, s, e, &lv_n, &dlv_n);
      cv.take(e.lv, lv_n * sizeof(float));
      cv.take(e.Z, (size_t)(lv_n / 3 + 1) * 4 * sizeof(float));
      cv.take(e.part, (size_t)envmap_prefilter_chunks(He, We) * (size_t)lv_n * sizeof(float));
      cv.take(e.dirs, (size_t)He * We * 4 * sizeof(float));
      e.He = He;
      e.We = We;
    }
  }
  std::vector<ViewDev> vh;
  plan_batch(&w, b, vh);
  const long long R = w.R > 0 ? w.R : 1;
  const long long npix = w.n_pix > 0 ? w.n_pix : 1, ntiles = w.n_tiles > 0 ? w.n_tiles : 1;
  cv.take(w.views_d, sizeof(ViewDev) * b->n_views);
  cv.take(w.recs, (size_t)R * kRecFloats * sizeof(float));
  for (DevBuf* d : {&w.counts, &w.offsets, &w.zkey, &w.zkey2, &w.zidx, &w.zidx2})
    cv.take(*d, (size_t)R * sizeof(uint32_t));
  cv.take(w.prect, (size_t)R * sizeof(uint2));
  cv.take(w.zrect, (size_t)R * sizeof(uint2));
  cv.take(w.ranges, (size_t)2 * ntiles * sizeof(uint32_t));
  cv.take(w.order, (size_t)ntiles * sizeof(int));
  cv.take(w.nl, (size_t)npix);
  cv.take(w.stats, (size_t)npix * kMaxLayers * sizeof(float4));
  cv.take(w.lpos, (size_t)npix * kPosStride * sizeof(uint32_t));
  if (c->opt.depth_stats) cv.take(w.stats2, (size_t)npix * kMaxLayers * sizeof(float2));
  if (!cv.ok) return SS_ERR_STATIC_LIMIT;
  // pairs (keys and values, double-buffered): what is left after the sort's
  // histogram and scan scratch for that capacity
  Group& g = w.groups[0];
  const long long nrec = g.rec_end - g.rec_begin;
  const size_t left = cv.cap - ((cv.used + 255) & ~size_t(255));
  auto hist_for = [&](long long cp) {
    return radix_hist_size(cp) > radix_hist_size(nrec) ? radix_hist_size(cp) : radix_hist_size(nrec);
  };
  const long long nq = c->opt.tile_w * c->opt.tile_h / 16;
  auto need = [&](long long cp) {
    const long long h = hist_for(cp), sc = scan_tmp_size(h > R ? h : R) + 16;
    return (size_t)(16 * cp + 4 * h + 4 * sc + 8 * nq * mask_slots(cp, g.n_tiles)) + 8 * 256;
  };
  long long cap = (long long)(left / 16);
  while (cap > 0 && need(cap) > left) cap -= cap / 64 > 0 ? cap / 64 : 1;
  if (cap < 4096) return SS_ERR_STATIC_LIMIT;
  g.pair_base = 0;
  g.pair_cap = cap;
  w.pair_total = cap;
  w.hist_n = hist_for(cap);
  w.scan_tmp_n = scan_tmp_size(w.hist_n > R ? w.hist_n : R) + 16;
  for (DevBuf* d : {&w.keys, &w.keys2, &w.vals, &w.vals2}) cv.take(*d, (size_t)cap * sizeof(uint32_t));
  cv.take(w.hist, (size_t)w.hist_n * sizeof(uint32_t));
  cv.take(w.scan_tmp, (size_t)w.scan_tmp_n * sizeof(uint32_t));
  cv.take(w.qmask, (size_t)layout_masks(&w) * sizeof(uint64_t));
  if (!cv.ok) return SS_ERR_STATIC_LIMIT;
  // view table (its map pointers point into the array), direction tables
  for (int v0 = 0; v0 < b->n_views; v0 += kViewsPerStore) {
    ViewStore vs;
    std::memset(&vs, 0, sizeof(vs));
    vs.n = b->n_views - v0 < kViewsPerStore ? b->n_views - v0 : kViewsPerStore;
    for (int i = 0; i < vs.n; ++i) vs.v[i] = vh[v0 + i];
    hipLaunchKernelGGL(store_views_kernel, dim3(1), dim3(256), 0, st, vs, P<ViewDev>(w.views_d) + v0);
    SS_HIP(hipGetLastError());
  }
  w.views_h = vh;
  w.views_uploaded = true;
  for (SceneEnv& e : w.env) {
    SS_HIP(launch_envmap_dirs(P<float>(e.dirs), e.He, e.We, st));
    SS_HIP(launch_envmap_out_dirs(e.He, e.We, P<float>(e.dirs), e.lh, e.lw, P<float>(e.Z), st));
  }
  SS_TRY(forward_body(&w, b, out, st));
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_cap[dev] = cap;
  }
  if (out->generation) *out->generation = 0;
  return SS_OK;
}

// ---------------------------------------------------------------- test access
namespace {
__global__ void extract_records_kernel(const float* recs, long long R, uint32_t* zb, int32_t* rect) {
  long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const float4 q = reinterpret_cast<const float4*>(recs + r * kRecFloats)[3];
  const int rx = __float_as_int(q.x), ry = __float_as_int(q.y);
  if (zb) zb[r] = (uint32_t)__float_as_int(q.z);
  if (rect) {
    rect[4 * r + 0] = rx & 0xffff;
    rect[4 * r + 1] = ry & 0xffff;
    rect[4 * r + 2] = rx >> 16;
    rect[4 * r + 3] = ry >> 16;
  }
}
// Pair keys as (global tile << 32) | bits of the record's z_start.
__global__ void copy_pairs_kernel(const uint32_t* k, const uint32_t* v, long long n, uint64_t tile_base,
                                  const float* recs, uint64_t* ko, uint32_t* vo) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (ko) ko[i] = ((tile_base + k[i]) << 32) | (uint64_t)__float_as_uint(recs[(long long)v[i] * kRecFloats + R_ZS]);
  if (vo) vo[i] = v[i];
}
__global__ void copy_ranges_kernel(const uint32_t* r, int n, uint32_t add, uint32_t* o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t s = r[2 * i], e = r[2 * i + 1];
  o[2 * i] = (e > s) ? s + add : 0u;
  o[2 * i + 1] = (e > s) ? e + add : 0u;
}
}  // namespace

extern "C" ss_status ss_debug_env_levels(ss_context* c, int32_t scene, float* levels, int64_t n, ss_stream stream) {
  if (!c || !c->fwd_valid || c->opt.shade != SS_SHADE_SPLITSUM) return SS_ERR_STATE;
  if (scene < 0 || scene >= (int32_t)c->env.size() || !levels) return SS_ERR_INVALID_ARG;
  const SceneEnv& e = c->env[scene];
  const long long need = e.off[6] + 3LL * e.lh[6] * e.lw[6];
  if (n != need || !e.lv.p) return SS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  SS_HIP(hipMemcpyAsync(levels, e.lv.p, (size_t)need * sizeof(float), hipMemcpyDefault, st));
  SS_HIP(hipStreamSynchronize(st));
  return SS_OK;
}

extern "C" ss_status ss_debug_binning(ss_context* c, uint32_t* rec_zbits, int32_t* rec_rect,
                                      uint64_t* pair_keys, uint32_t* pair_vals, uint32_t* tile_ranges,
                                      int64_t* n_pairs, int64_t* n_tiles, ss_stream stream) {
  if (!c || !c->fwd_valid) return SS_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  SS_HIP(hipStreamSynchronize(st));
  std::vector<uint32_t> np(c->groups.size());
  SS_HIP(hipMemcpy(np.data(), P<uint32_t>(c->misc) + kMiscPairs, np.size() * sizeof(uint32_t),
                   hipMemcpyDeviceToHost));
  if (rec_zbits || rec_rect) {
    hipLaunchKernelGGL(extract_records_kernel, dim3((unsigned)((c->R + 255) / 256)), dim3(256), 0, st,
                       P<float>(c->recs), c->R, rec_zbits, rec_rect);
  }
  long long done = 0;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& g = c->groups[gi];
    const long long n = np[gi];
    if ((pair_keys || pair_vals) && n > 0)
      hipLaunchKernelGGL(copy_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                         P<uint32_t>(c->keys) + g.pair_base, P<uint32_t>(c->vals) + g.pair_base, n,
                         (uint64_t)g.tile_base, P<float>(c->recs), pair_keys ? pair_keys + done : nullptr,
                         pair_vals ? pair_vals + done : nullptr);
    if (tile_ranges && g.n_tiles > 0)
      hipLaunchKernelGGL(copy_ranges_kernel, dim3((g.n_tiles + 255) / 256), dim3(256), 0, st,
                         P<uint32_t>(c->ranges) + 2LL * g.tile_base, g.n_tiles, (uint32_t)done,
                         tile_ranges + 2LL * g.tile_base);
    done += n;
  }
  SS_HIP(hipGetLastError());
  SS_HIP(hipStreamSynchronize(st));
  if (n_pairs) *n_pairs = done;
  if (n_tiles) *n_tiles = c->n_tiles;
  return SS_OK;
}

extern "C" const char* ss_status_str(ss_status s) {
  switch (s) {
    case SS_OK: return "ok";
    case SS_ERR_INVALID_ARG: return "invalid argument";
    case SS_ERR_HIP: return "HIP runtime error";
    case SS_ERR_CAPACITY: return "pair capacity exceeded (call ss_reserve and render again)";
    case SS_ERR_STATE: return "call out of order";
    case SS_ERR_UNSUPPORTED: return "unsupported option";
    case SS_ERR_NOMEM: return "device allocation failed";
    case SS_ERR_STATIC_LIMIT: return "batch exceeds the fixed workspace of ss_render_static";
  }
  return "unknown status";
}
