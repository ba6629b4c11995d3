// lnr_api.hip -- the C ABI of include/lnr.h: argument checks, the context's
// workspace, and the order in which the kernels of one registration or merge
// are enqueued on the caller's stream. No entry point synchronises the device
// (the homographies and match counts stay in device memory between levels).
#include <stdio.h>
#include <string.h>

#include <new>
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "lnr_internal.h"

namespace lnr {
// Event pairs recorded around kernel launches while tracing is on.
struct Tracer {
  struct Rec {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<std::string> names;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;

  int slot_of(const char* n) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) return (int)i;
    names.emplace_back(n);
    return (int)names.size() - 1;
  }
  hipEvent_t take() {
    if (pool_used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[pool_used++];
  }
  void reset() {
    names.clear();
    recs.clear();
    pool_used = 0;
  }
  ~Tracer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

thread_local Tracer* g_tracer = nullptr;


TraceScope::TraceScope(const char* name, hipStream_t st) {
  if (!g_tracer) return;
  Tracer& t = *g_tracer;
  hipEvent_t a = t.take(), b = t.take();
  if (!a || !b) return;
  slot = (int)t.recs.size();
  t.recs.push_back(Tracer::Rec{t.slot_of(name), a, b});
  stream = st;
  if (hipEventRecord(a, st) != hipSuccess) slot = -1;
}

TraceScope::~TraceScope() {
  if (slot < 0 || !g_tracer) return;
  (void)hipEventRecord(g_tracer->recs[slot].b, stream);
}
}  // namespace lnr

struct lnr_ctx {
  int device = 0;
  std::string err;
  void* ws = nullptr;
  size_t ws_size = 0;
  // this device's copy of the fixed scratch of lnr_register_pair_noalloc
  // (null when its address could not be obtained; scratch_err says why)
  void* scratch = nullptr;
  std::string scratch_err;
  bool tracing = false;
  lnr::Tracer tracer;
  // learned proposal: fp32 parameters, AdamW moments, packed bf16 weights
  float* cnn = nullptr;        // [3][nparam]: params, m, v
  uint16_t* cnn_packed = nullptr;
  int cnn_step = 0;
  // domain-transform kernel shapes picked by the autotuner, per (W, H)
  std::map<std::pair<int, int>, lnr::DtShape> dt_shapes;
  // batches: worker streams, fork / join events, cached executable graphs
  std::vector<hipStream_t> workers;
  std::vector<hipEvent_t> events;
  hipStream_t capture = nullptr;
  struct Cached {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    void* tables = nullptr;  // the level-synchronous batch's job tables (device)
  };
  std::vector<Cached> graphs;
  std::map<std::vector<uint64_t>, int> batch_k;  // autotuned concurrency per batch
  std::map<std::vector<uint64_t>, int> batch_kx;  // autotuned search candidates per lane
  void* tables = nullptr;  // job tables of eager level-synchronous batches
  size_t tables_size = 0;
  // search splits picked by the autotuner, per (level width, height, radius)
  std::map<std::tuple<int, int, int>, int> search_split;
};

namespace lnr {
namespace {

// Sets the thread's tracer for the duration of one API call.
struct TraceGuard {
  explicit TraceGuard(lnr_ctx* c) { g_tracer = (c && c->tracing) ? &c->tracer : nullptr; }
  ~TraceGuard() { g_tracer = nullptr; }
};

lnr_status fail(lnr_ctx* ctx, lnr_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

lnr_status hip_fail(lnr_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, LNR_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define LNR_HIP(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);    \
  } while (0)

lnr_status check_params(lnr_ctx* ctx, const lnr_params* p) {
  if (!p) return fail(ctx, LNR_E_ARG, "params is null");
  const int ext = p->corner_half * p->corner_step + (p->quad_r > p->patch_r ? p->quad_r : p->patch_r);
  if (p->tile < 16 || p->tile > 64) return fail(ctx, LNR_E_UNSUPPORTED, "tile must be in [16, 64]");
  if (p->patch_r < 1 || p->patch_r > kMaxPatchR) return fail(ctx, LNR_E_UNSUPPORTED, "patch_r must be in [1, 11]");
  if (p->corner_half < 0 || p->corner_half > 3 || p->corner_step < 1 || p->quad_r < 1)
    return fail(ctx, LNR_E_UNSUPPORTED, "corner candidate grid out of range");
  if (ext > p->tile / 2 - 1)
    return fail(ctx, LNR_E_UNSUPPORTED, "corner candidates and patches must stay inside the tile");
  if (p->corner_t < 0) return fail(ctx, LNR_E_UNSUPPORTED, "corner_t must be >= 0");
  if (p->max_levels < 1 || p->max_levels > kMaxLevels) return fail(ctx, LNR_E_UNSUPPORTED, "max_levels must be in [1, 5]");
  if (p->min_level_dim < p->tile) return fail(ctx, LNR_E_UNSUPPORTED, "min_level_dim must be >= tile");
  if (p->radius0 < 0 || p->radius0 > kMaxRadius || p->radius_coarse < 0 || p->radius_coarse > kMaxRadius)
    return fail(ctx, LNR_E_UNSUPPORTED, "search radii must be in [0, 32]");
  if (p->weed_iters < 1 || p->weed_iters > 65536) return fail(ctx, LNR_E_UNSUPPORTED, "weed_iters must be in [1, 65536]");
  if (p->weed_delta_min < 0 || p->weed_delta_pct < 0 || p->weed_delta_pct > 100)
    return fail(ctx, LNR_E_UNSUPPORTED, "weeding delta out of range");
  if (!(p->weed_eps > 0)) return fail(ctx, LNR_E_UNSUPPORTED, "weed_eps must be > 0");
  if (p->dt_iters < 1 || p->dt_iters > 8) return fail(ctx, LNR_E_UNSUPPORTED, "dt_iters must be in [1, 8]");
  if (!(p->sigma_s > 0) || !(p->sigma_r > 0)) return fail(ctx, LNR_E_UNSUPPORTED, "sigmas must be > 0");
  if (p->ssim_radius < 1 || p->ssim_radius > 8 || !(p->ssim_sigma > 0))
    return fail(ctx, LNR_E_UNSUPPORTED, "SSIM window out of range");
  if (!(p->sigma_e > 0)) return fail(ctx, LNR_E_UNSUPPORTED, "sigma_e must be > 0");
  if (p->learned != 0 && p->learned != 1) return fail(ctx, LNR_E_UNSUPPORTED, "learned must be 0 or 1");
  if (p->search_frame != 0 && p->search_frame != 1)
    return fail(ctx, LNR_E_UNSUPPORTED, "search_frame must be 0 or 1");
  if (p->search_frame == 1 && p->learned)
    return fail(ctx, LNR_E_UNSUPPORTED,
                "the learned proposal is defined on the warped-source search (search_frame 0)");
  if (p->learned) {
    if (p->tile != 32) return fail(ctx, LNR_E_UNSUPPORTED, "the learned proposal needs tile 32");
    if (p->window_r < 0 || p->window_r > p->radius0)
      return fail(ctx, LNR_E_UNSUPPORTED, "window_r must be in [0, radius0]");
    if (!(p->conf_min >= 0.0 && p->conf_min <= 1.0))
      return fail(ctx, LNR_E_UNSUPPORTED, "conf_min must be in [0, 1]");
  }
  return LNR_OK;
}

constexpr int kMaxSide = 6144;  // int64 normal equations and row LDS stay in range

lnr_status check_frame(lnr_ctx* ctx, const lnr_frame* f, const char* name) {
  if (!f) return fail(ctx, LNR_E_ARG, std::string(name) + " is null");
  if (f->format != LNR_Y8 && f->format != LNR_I420 && f->format != LNR_NV12)
    return fail(ctx, LNR_E_UNSUPPORTED, std::string(name) + ": unknown format");
  if (f->width < 1 || f->height < 1 || f->width > kMaxSide || f->height > kMaxSide)
    return fail(ctx, LNR_E_UNSUPPORTED, std::string(name) + ": width/height must be in [1, 6144]");
  if (!f->plane[0] || f->stride[0] < f->width)
    return fail(ctx, LNR_E_ARG, std::string(name) + ": bad Y plane");
  if (f->format == LNR_I420) {
    if (f->width % 2 || f->height % 2)
      return fail(ctx, LNR_E_ARG, std::string(name) + ": I420 needs even width and height");
    if (!f->plane[1] || !f->plane[2] || f->stride[1] < f->width / 2 || f->stride[2] < f->width / 2)
      return fail(ctx, LNR_E_ARG, std::string(name) + ": bad chroma planes");
  }
  if (f->format == LNR_NV12) {
    if (f->width % 2 || f->height % 2)
      return fail(ctx, LNR_E_ARG, std::string(name) + ": NV12 needs even width and height");
    if (!f->plane[1] || f->stride[1] < f->width)
      return fail(ctx, LNR_E_ARG, std::string(name) + ": bad interleaved chroma plane");
  }
  return LNR_OK;
}

// the frame's chroma samples (none for luma-only frames)
Chroma chroma_of(const lnr_frame& f) {
  Chroma c;
  if (f.format == LNR_I420) {
    c.u = f.plane[1]; c.su = f.stride[1];
    c.v = f.plane[2]; c.sv = f.stride[2];
  } else if (f.format == LNR_NV12) {
    c.u = f.plane[1]; c.v = f.plane[1] + 1;
    c.su = c.sv = f.stride[1];
    c.cs = 2;
  }
  return c;
}

Geometry make_geometry(int W, int H, const lnr_params& p) {
  Geometry g;
  g.W = W;
  g.H = H;
  int levels = 1, w = W, h = H;
  while (levels < p.max_levels) {
    const int w2 = w / 2, h2 = h / 2;
    if ((w2 < h2 ? w2 : h2) < p.min_level_dim) break;
    w = w2;
    h = h2;
    ++levels;
  }
  g.levels = levels;
  size_t off = 0;
  int toff = 0;
  w = W;
  h = H;
  for (int l = 0; l < kMaxLevels; ++l) {
    Level& L = g.lv[l];
    if (l >= levels) {
      L = Level{0, 0, 0, 0, toff, off};
      continue;
    }
    if (l) { w /= 2; h /= 2; }
    L.w = w; L.h = h;
    L.ntx = w / p.tile; L.nty = h / p.tile;
    L.tile_off = toff;
    L.pix_off = off;
    toff += L.ntx * L.nty;
    off += (size_t)w * h;
  }
  g.tiles_total = toff;
  g.pyr_bytes = off;
  return g;
}

SearchJob search_job(const uint8_t* ref, const uint8_t* wimg, int w, int h, int ntx,
                     int32_t* cxy, int32_t* disp, uint32_t* ssd, uint8_t* flags,
                     const int32_t* centre = nullptr, unsigned long long* vb = nullptr,
                     const double* Hlit = nullptr, const double* Hwarp = nullptr) {
  SearchJob j;
  j.ref = ref; j.wimg = wimg; j.w = w; j.h = h; j.ntx = ntx;
  j.corner_xy = cxy; j.disp = disp; j.ssd = ssd; j.flags = flags;
  j.centre = centre; j.vb = vb; j.Hlit = Hlit; j.Hwarp = Hwarp;
  return j;
}

int level_words(const Level& L) {
  const int nt = L.ntx * L.nty;
  return nt > 0 ? (nt + 63) / 64 : 1;
}

SearchCfg search_cfg(const lnr_params& p) {
  SearchCfg c;
  c.S = p.tile; c.P = p.patch_r; c.g = p.corner_step; c.K = p.corner_half; c.r = p.quad_r;
  c.thr = p.corner_t * p.quad_r * p.quad_r;
  return c;
}

// the search shape tuned or pinned in this context for levels of w x h
// searched at radius R (0: the automatic shape)
int pinned_search_shape(const lnr_ctx* ctx, int w, int h, int R) {
  auto it = ctx->search_split.find(std::make_tuple(w, h, R));
  return it == ctx->search_split.end() ? 0 : it->second;
}

struct Plan {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

// Grows the workspace; a stream under graph capture cannot allocate, so a
// call that needs more workspace there fails with LNR_E_CAPTURE (size it
// with one call outside the capture first).
lnr_status ensure_ws(lnr_ctx* ctx, size_t bytes, hipStream_t st) {
  if (bytes <= ctx->ws_size) return LNR_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return fail(ctx, LNR_E_CAPTURE,
                "the workspace must grow, which a captured stream cannot do: run the call "
                "once outside the capture first");
  if (ctx->ws) {
    hipError_t e = hipFree(ctx->ws);  // waits for work that may still use it
    ctx->ws = nullptr;
    ctx->ws_size = 0;
    if (e != hipSuccess) return hip_fail(ctx, e, "hipFree(workspace)");
  }
  const size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&ctx->ws, want);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, LNR_E_NOMEM, std::string("workspace hipMalloc failed: ") + hipGetErrorString(e));
  }
  ctx->ws_size = want;
  return LNR_OK;
}

// Fixed scratch of lnr_register_pair_noalloc: one copy on every GPU the
// library runs on, held until the process ends. On the host this name only
// identifies the symbol; its device address comes from hipGetSymbolAddress,
// taken once per device (lnr_create) and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[LNR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Called with `device` current.
void bind_scratch(lnr_ctx* c, int device) {
  if (device >= kMaxDevices) {
    c->scratch_err = "device index beyond the scratch table";
    return;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      c->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return;
    }
    g_scratch_ptr[device] = ptr;
  }
  c->scratch = g_scratch_ptr[device];
}

struct WeedPlan {
  size_t nmatch, G, cnt, bal, vb, sums;
};

WeedPlan plan_weed(Plan& pl, int ntiles, int iters) {
  WeedPlan w;
  const int nt = ntiles > 0 ? ntiles : 1;
  w.nmatch = pl.take(sizeof(int32_t));
  w.G = pl.take(sizeof(double) * 8 * (size_t)iters);
  w.cnt = pl.take(sizeof(int32_t) * (size_t)iters);
  w.bal = pl.take(sizeof(unsigned long long) * (size_t)iters * ((nt + 63) / 64));
  w.vb = pl.take(sizeof(unsigned long long) * (size_t)((nt + 63) / 64));
  w.sums = pl.take(sizeof(long long) * 24);
  return w;
}

WeedBufs weed_bufs(char* base, const WeedPlan& w) {
  WeedBufs b;
  b.nmatch = reinterpret_cast<int32_t*>(base + w.nmatch);
  b.G = reinterpret_cast<double*>(base + w.G);
  b.cnt = reinterpret_cast<int32_t*>(base + w.cnt);
  b.bal = reinterpret_cast<unsigned long long*>(base + w.bal);
  b.vb = reinterpret_cast<unsigned long long*>(base + w.vb);
  b.sums = reinterpret_cast<long long*>(base + w.sums);
  return b;
}

// Workspace layout of one registration (offsets from the pair's base).
struct PairPlan {
  Geometry g;
  size_t bytes, o_hist, o_pref, o_psrc, o_warp, o_maps, o_gt, o_coef, o_cx, o_cc, o_cm, o_cl,
      o_cn;
  WeedPlan wp;
};

lnr_status check_pair(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                      const lnr_params* p, const lnr_registration* out) {
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if ((s = check_frame(ctx, ref, "ref")) != LNR_OK) return s;
  if ((s = check_frame(ctx, src, "src")) != LNR_OK) return s;
  if (!out) return fail(ctx, LNR_E_ARG, "out is null");
  if (ref->width != src->width || ref->height != src->height || ref->format != src->format)
    return fail(ctx, LNR_E_ARG, "ref and src differ in size or format");
  if (ref->width < p->tile || ref->height < p->tile)
    return fail(ctx, LNR_E_TOO_SMALL, "image smaller than one tile");
  if (!out->corner_xy || !out->disp || !out->ssd || !out->flags || !out->counts || !out->H ||
      !out->yeq_ref || !out->flow || !out->image || !out->yeq_warped)
    return fail(ctx, LNR_E_ARG, "a required output pointer is null");
  if (p->learned && !ctx->cnn)
    return fail(ctx, LNR_E_ARG, "learned proposal requested but no network set (lnr_proposal_set)");
  return LNR_OK;
}

PairPlan plan_pair(int W, int H, const lnr_params* p) {
  PairPlan q;
  q.g = make_geometry(W, H, *p);
  const size_t N = (size_t)W * H;
  Plan pl;
  q.o_hist = pl.take(2 * 256 * sizeof(uint32_t));
  q.o_pref = pl.take(q.g.pyr_bytes);
  q.o_psrc = pl.take(q.g.pyr_bytes);
  q.o_warp = pl.take(N);
  q.wp = plan_weed(pl, q.g.lv[0].ntx * q.g.lv[0].nty, p->weed_iters);
  q.o_maps = pl.take(dt_maps_bytes(W, H));
  q.o_gt = pl.take(dt_guide_t_bytes(W, H));
  q.o_coef = pl.take((size_t)p->dt_iters * 256 * sizeof(double));
  const size_t nt0 = (size_t)q.g.lv[0].ntx * q.g.lv[0].nty;
  q.o_cx = p->learned ? pl.take(nt0 * cnn_input_elems() * sizeof(uint16_t)) : 0;
  q.o_cc = p->learned ? pl.take(nt0 * 2 * sizeof(int32_t)) : 0;
  q.o_cm = p->learned ? pl.take(nt0) : 0;
  q.o_cl = p->learned ? pl.take(3 * nt0 * sizeof(int32_t)) : 0;
  q.o_cn = p->learned ? pl.take(3 * sizeof(int32_t)) : 0;
  q.bytes = pl.off;
  return q;
}

__global__ void k_copy_u8(const uint8_t* __restrict__ a, uint8_t* __restrict__ b, size_t n) {
  const size_t i0 = ((size_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (i0 + 16 <= n && ((reinterpret_cast<uintptr_t>(a + i0) | reinterpret_cast<uintptr_t>(b + i0)) & 15) == 0) {
    *reinterpret_cast<uint4*>(b + i0) = *reinterpret_cast<const uint4*>(a + i0);
  } else {
    for (size_t i = i0; i < i0 + 16 && i < n; ++i) b[i] = a[i];
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// The start of one registration: the propagation's coefficient tables, the
// cleared histograms and the identity above the top level (one launch), the
// histograms, and both equalised pyramids (level 0 also written to the
// outputs, no copies).
lnr_status enqueue_pair_setup(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                              const lnr_params* p, lnr_registration* out, const PairPlan& q,
                              char* base, hipStream_t st) {
  const Geometry& g = q.g;
  const int W = ref->width, H = ref->height;
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + q.o_hist);
  uint8_t* pref = reinterpret_cast<uint8_t*>(base + q.o_pref);
  uint8_t* psrc = reinterpret_cast<uint8_t*>(base + q.o_psrc);
  uint8_t* guide_t = reinterpret_cast<uint8_t*>(base + q.o_gt);
  double* coef = reinterpret_cast<double*>(base + q.o_coef);
  // (also cleared: the top level's weeding bits and sums, which its search fills)
  const WeedBufs wb = weed_bufs(base, q.wp);
  LNR_HIP(launch_dt_coef(*p, coef, hist, 512, out->H + 9 * g.levels, st, wb.vb,
                         level_words(g.lv[g.levels - 1]), wb.sums));
  LNR_HIP(launch_hist(ref->plane[0], ref->stride[0], src->plane[0], src->stride[0], W, H, hist, 2, st));
  LNR_HIP(launch_lut_pyr(ref->plane[0], ref->stride[0], src->plane[0], src->stride[0], hist, g,
                         pref, psrc, nullptr, 2, st, out->yeq_ref, out->yeq_src, guide_t));
  return LNR_OK;
}

// The end of one registration: level 0's kept matches propagated to the
// dense flow, and the backward warp of the source.
lnr_status enqueue_pair_finish(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                               const lnr_params* p, lnr_registration* out, const PairPlan& q,
                               char* base, hipStream_t st, char* ref_base = nullptr) {
  const Geometry& g = q.g;
  const int W = ref->width, H = ref->height;
  if (!ref_base) ref_base = base;
  uint8_t* pref = reinterpret_cast<uint8_t*>(ref_base + q.o_pref);
  uint8_t* psrc = reinterpret_cast<uint8_t*>(base + q.o_psrc);
  void* maps = base + q.o_maps;
  uint8_t* guide_t = reinterpret_cast<uint8_t*>(ref_base + q.o_gt);
  double* coef = reinterpret_cast<double*>(base + q.o_coef);
  const DtShape* ds = nullptr;
  auto it = ctx->dt_shapes.find(std::make_pair(W, H));
  if (it != ctx->dt_shapes.end()) ds = &it->second;
  LNR_HIP(launch_flow(out->corner_xy, out->disp, out->flags, g.lv[0].ntx, g.lv[0].nty, p->tile,
                      pref, guide_t, W, H, *p, maps, coef, out->flow, out->ntilde, st, ds, true,
                      true));
  // the paper-literal search's flow is the whole mapping (identity above the top level)
  const double* Hb = p->search_frame == 1 ? out->H + 9 * g.levels : out->H + 9;
  LNR_HIP(launch_backward_warp(src->plane[0], src->stride[0], chroma_of(*src), psrc, W, H, Hb,
                               out->flow, out->image, out->yeq_warped, st));
  return LNR_OK;
}

// The set-up of a source whose reference was prepared with another source
// (register_stack): the tables and clears, the source's histogram and
// pyramid only, and the reference's equalised level 0 copied to this output.
lnr_status enqueue_source_setup(lnr_ctx* ctx, const lnr_frame* src, const lnr_params* p,
                                lnr_registration* out, const uint8_t* yeq_ref_done,
                                const PairPlan& q, char* base, hipStream_t st) {
  const Geometry& g = q.g;
  const int W = src->width, H = src->height;
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + q.o_hist);
  uint8_t* psrc = reinterpret_cast<uint8_t*>(base + q.o_psrc);
  double* coef = reinterpret_cast<double*>(base + q.o_coef);
  const WeedBufs wb = weed_bufs(base, q.wp);
  LNR_HIP(launch_dt_coef(*p, coef, hist, 512, out->H + 9 * g.levels, st, wb.vb,
                         level_words(g.lv[g.levels - 1]), wb.sums));
  LNR_HIP(launch_hist(src->plane[0], src->stride[0], src->plane[0], src->stride[0], W, H, hist, 1,
                      st));
  LNR_HIP(launch_lut_pyr(src->plane[0], src->stride[0], src->plane[0], src->stride[0], hist, g,
                         psrc, psrc, nullptr, 1, st, out->yeq_src, nullptr, nullptr));
  const size_t n = (size_t)W * H;
  LNR_LAUNCH(k_copy_u8, dim3((unsigned)((n + 4095) / 4096)), dim3(256), 0, st, yeq_ref_done,
             out->yeq_ref, n);
  LNR_HIP(hipGetLastError());
  return LNR_OK;
}

// The pyramid levels of one registration (warp, search, weeding, fit per
// level); the reference's pyramid is read at ref_base (default: base).
lnr_status enqueue_pair_levels(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                               const lnr_params* p, lnr_registration* out, const PairPlan& q,
                               char* base, hipStream_t st, char* ref_base = nullptr);

// Enqueue one registration on `st` using the workspace at `base` (checked and
// sized by the caller). Launches only: safe under stream capture.
lnr_status enqueue_pair(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                        const lnr_params* p, lnr_registration* out, const PairPlan& q,
                        char* base, hipStream_t st) {
  lnr_status s0 = enqueue_pair_setup(ctx, ref, src, p, out, q, base, st);
  if (s0 != LNR_OK) return s0;
  if ((s0 = enqueue_pair_levels(ctx, ref, src, p, out, q, base, st)) != LNR_OK) return s0;
  return enqueue_pair_finish(ctx, ref, src, p, out, q, base, st);
}

lnr_status enqueue_pair_levels(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                               const lnr_params* p, lnr_registration* out, const PairPlan& q,
                               char* base, hipStream_t st, char* ref_base) {
  const Geometry& g = q.g;
  const int W = ref->width;
  if (!ref_base) ref_base = base;
  uint8_t* pref = reinterpret_cast<uint8_t*>(ref_base + q.o_pref);
  uint8_t* psrc = reinterpret_cast<uint8_t*>(base + q.o_psrc);
  uint8_t* warped = reinterpret_cast<uint8_t*>(base + q.o_warp);
  const WeedBufs wb = weed_bufs(base, q.wp);
  (void)src;
  const SearchCfg cfg = search_cfg(*p);
  auto tuned = [&](int w, int h, int R) { return pinned_search_shape(ctx, w, h, R); };
  // search_frame 1 (Eq. 3 as printed): no level is warped; each level searches
  // the unwarped source around its prediction, the fits are absolute (composed
  // on the identity above the top level) and so is the propagated flow
  const bool literal = p->search_frame == 1;
  const double* identity = out->H + 9 * g.levels;
  for (int l = g.levels - 1; l >= 0; --l) {
    const Level& L = g.lv[l];
    const int R = l == 0 ? p->radius0 : p->radius_coarse;
    const int nt = L.ntx * L.nty;
    const int words = nt > 0 ? (nt + 63) / 64 : 1;
    if (literal) {
      // the weeding builds the valid-match bits from the flags (k_valid)
      const SearchJob J = search_job(pref + L.pix_off, psrc + L.pix_off, L.w, L.h, L.ntx,
                                     out->corner_xy + 2 * L.tile_off, out->disp + 2 * L.tile_off,
                                     out->ssd + L.tile_off, out->flags + L.tile_off, nullptr,
                                     nullptr, out->H + 9 * (l + 1));
      LNR_HIP(launch_search(J, L.nty, R, cfg, l == 0 ? kRoleLevel0 : kRoleCoarse, st, nullptr, 0,
                            tuned(L.w, L.h, R)));
      LNR_HIP(launch_weed_fit(out->corner_xy + 2 * L.tile_off, out->disp + 2 * L.tile_off,
                              out->flags + L.tile_off, nt, L.w, L.h, l, *p, out->H + 9 * (l + 1),
                              out->H + 9 * l, out->counts + 4 * l, wb, st, false, identity));
      continue;
    }
    // the coarse levels' searches warp their windows on the fly (the set-up or
    // the previous level's solve cleared the weeding bits and sums); level 0
    // is warped in full, straight into the output when it is wanted, and the
    // warp clears the level's weeding buffers and the learned path's counts
    if (l == 0 && out->warped0) warped = out->warped0;
    int32_t* lists = p->learned ? reinterpret_cast<int32_t*>(base + q.o_cl) : nullptr;
    int* counts = p->learned ? reinterpret_cast<int*>(base + q.o_cn) : nullptr;
    if (l == 0)
      LNR_HIP(launch_warp_q8(psrc, L.w, L.h, out->H + 9, warped, st, &wb, words, counts, 3));
    if (l == 0 && p->learned) {
      // corners first (the cornered tiles listed), the network on the
      // cornered tiles (each listed for the window or for the fallback), then
      // the window search of the confident tiles and the exhaustive search
      // (flag 16) of the others, each launch visiting only its list
      uint16_t* x = reinterpret_cast<uint16_t*>(base + q.o_cx);
      int32_t* centre = reinterpret_cast<int32_t*>(base + q.o_cc);
      uint8_t* mode = reinterpret_cast<uint8_t*>(base + q.o_cm);
      // the window is taken where the logit is >= this: conf_min 0 windows
      // every tile, conf_min 1 (a NaN bound, no logit compares >= it) none
      const float logit = p->conf_min <= 0.0 ? -INFINITY
                          : p->conf_min >= 1.0 ? NAN
                          : (float)std::log(p->conf_min / (1.0 - p->conf_min));
      // (the lists are built from the flags and modes by one workgroup each)
      SearchWork wk{};
      wk.njobs = 1;
      wk.ntotal = nt;
      const SearchJob Jc = search_job(pref, warped, L.w, L.h, L.ntx, out->corner_xy, out->disp,
                                      out->ssd, out->flags, nullptr, wb.vb);
      LNR_HIP(launch_search_work(nullptr, wk, R, cfg, kVisitCornersOnly, 0, 0, 8, nt, st, &Jc));
      LNR_HIP(launch_tile_lists(out->flags, nullptr, nt, lists, counts, st));
      LNR_HIP(launch_cnn_input(pref, warped, W, L.h, L.ntx, L.nty, lists, counts, x, st));
      LNR_HIP(launch_cnn_forward(ctx->cnn_packed, ctx->cnn, x, nt, nullptr, nullptr, centre, mode,
                                 p->radius0 - p->window_r, logit, st, lists, counts));
      LNR_HIP(launch_tile_lists(out->flags, mode, nt, lists, counts, st));
      SearchWork ww{};
      ww.njobs = 1;
      ww.list = lists + nt;
      ww.count = counts + 1;
      const SearchJob Jw = search_job(pref, warped, L.w, L.h, L.ntx, out->corner_xy, out->disp,
                                      out->ssd, out->flags, centre, wb.vb);
      LNR_HIP(launch_search_work(nullptr, ww, p->window_r, cfg, kVisitKnownCorner, 0, 0, 8, nt,
                                 st, &Jw));
      SearchWork wf{};
      wf.njobs = 1;
      wf.list = lists + 2 * nt;
      wf.count = counts + 2;
      LNR_HIP(launch_search_work(nullptr, wf, R, cfg, kVisitKnownCorner, 1, tuned(L.w, L.h, R), 8,
                                 nt, st, &Jc));
    } else {
      const SearchJob J = search_job(
          pref + L.pix_off, l == 0 ? warped : psrc + L.pix_off, L.w, L.h, L.ntx,
          out->corner_xy + 2 * L.tile_off, out->disp + 2 * L.tile_off, out->ssd + L.tile_off,
          out->flags + L.tile_off, nullptr, wb.vb, nullptr, l == 0 ? nullptr : out->H + 9 * (l + 1));
      LNR_HIP(launch_search(J, L.nty, R, cfg, l == 0 ? kRoleLevel0 : kRoleCoarse, st, nullptr, 0,
                            tuned(L.w, L.h, R)));
    }
    LNR_HIP(launch_weed_fit(out->corner_xy + 2 * L.tile_off, out->disp + 2 * L.tile_off,
                            out->flags + L.tile_off, nt, L.w, L.h, l, *p, out->H + 9 * (l + 1),
                            out->H + 9 * l, out->counts + 4 * l, wb, st, true, nullptr,
                            l >= 2 ? level_words(g.lv[l - 1]) : 0));
  }
  return LNR_OK;
}

lnr_status register_pair_impl(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                              const lnr_params* p, lnr_registration* out, hipStream_t st) {
  lnr_status s;
  if ((s = check_pair(ctx, ref, src, p, out)) != LNR_OK) return s;
  const PairPlan q = plan_pair(ref->width, ref->height, p);
  if ((s = ensure_ws(ctx, q.bytes, st)) != LNR_OK) return s;
  return enqueue_pair(ctx, ref, src, p, out, q, static_cast<char*>(ctx->ws), st);
}

// rel (host, n values): exposures relative to the reference for the
// irradiance map; null for the exposure fusion
lnr_status merge_impl(lnr_ctx* ctx, int n, int ch, int W, int H, const float* const* imgs,
                      const float* const* yeqs, int ref_index, const lnr_params* p, float* out,
                      hipStream_t st, size_t extra_bytes, size_t* extra_off,
                      const float* rel = nullptr) {
  const int L = merge_levels(W, H);
  const size_t N = (size_t)W * H, tot = merge_pyr_elems(W, H, L);
  Plan pl;
  if (extra_off) *extra_off = pl.take(extra_bytes);
  const size_t o_ssim = pl.take((size_t)n * N * sizeof(float));
  const size_t o_w0 = pl.take((size_t)n * N * sizeof(float));
  const size_t o_pyr = pl.take((size_t)n * (ch + 1) * (tot ? tot : 1) * sizeof(float));
  const size_t o_acc = pl.take((size_t)ch * (tot ? tot : 1) * sizeof(float));
  lnr_status s;
  if ((s = ensure_ws(ctx, pl.off, st)) != LNR_OK) return s;
  char* base = static_cast<char*>(ctx->ws);
  MergeBufs b;
  b.ssim = reinterpret_cast<float*>(base + o_ssim);
  b.w0 = reinterpret_cast<float*>(base + o_w0);
  b.pyr = reinterpret_cast<float*>(base + o_pyr);
  b.acc = reinterpret_cast<float*>(base + o_acc);
  (void)extra_off;
  if (rel)
    LNR_HIP(launch_irradiance(n, ch, W, H, imgs, yeqs, rel, ref_index, *p, b.ssim, out, st));
  else
    LNR_HIP(launch_merge(n, ch, W, H, imgs, yeqs, ref_index, *p, b, out, st));
  return LNR_OK;
}

}  // namespace
}  // namespace lnr

using namespace lnr;

extern "C" {

lnr_status lnr_create(lnr_ctx** ctx, int32_t device) {
  if (!ctx) return LNR_E_ARG;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return LNR_E_ARG;
  lnr_ctx* c = new (std::nothrow) lnr_ctx();
  if (!c) return LNR_E_NOMEM;
  c->device = device;
  int prev = 0;
  const bool have_prev = hipGetDevice(&prev) == hipSuccess;
  if (hipSetDevice(device) == hipSuccess) bind_scratch(c, device);
  else c->scratch_err = "hipSetDevice failed in lnr_create";
  if (have_prev) (void)hipSetDevice(prev);
  *ctx = c;
  return LNR_OK;
}

void lnr_destroy(lnr_ctx* ctx) {
  if (!ctx) return;
  int prev = 0;
  const bool have_prev = hipGetDevice(&prev) == hipSuccess;
  if (hipSetDevice(ctx->device) == hipSuccess) {
    if (ctx->ws && hipFree(ctx->ws) != hipSuccess) ctx->err = "hipFree(workspace) failed";
    if (ctx->cnn && hipFree(ctx->cnn) != hipSuccess) ctx->err = "hipFree(network) failed";
    if (ctx->cnn_packed && hipFree(ctx->cnn_packed) != hipSuccess)
      ctx->err = "hipFree(network) failed";
    for (auto& c : ctx->graphs) {
      (void)hipGraphExecDestroy(c.exec);
      if (c.tables) (void)hipFree(c.tables);
    }
    if (ctx->tables) (void)hipFree(ctx->tables);
    for (hipStream_t w : ctx->workers) (void)hipStreamDestroy(w);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  }
  if (have_prev && hipSetDevice(prev) != hipSuccess) ctx->err = "hipSetDevice(restore) failed";
  delete ctx;
}

const char* lnr_last_error(const lnr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void lnr_default_params(lnr_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->tile = 32;
  p->patch_r = 10;         // 21 x 21 patches (Sec. 2.6)
  p->corner_step = 2;      // grid of 1/16 of the tile (Sec. 2.6)
  p->corner_half = 2;
  p->quad_r = 10;
  p->corner_t = 2;
  p->max_levels = 5;       // Sec. 2.6
  p->min_level_dim = 100;  // Sec. 2.6
  p->radius_coarse = 10;   // Sec. 2.6
  p->radius0 = 16;
  p->weed_iters = 1024;
  p->weed_delta_min = 8;
  p->weed_delta_pct = 2;
  p->dt_iters = 3;
  p->weed_eps = 2.0;
  p->sigma_s = 400.0;      // Sec. 2.6
  p->sigma_r = 1.0;
  p->n_min = 1e-30;
  p->ssim_sigma = 1.5;
  p->ssim_radius = 5;
  p->ssim_c1 = 0.01 * 0.01;
  p->ssim_c2 = 0.03 * 0.03;
  p->sigma_e = 0.2;
  p->seed = 0x1504014410ull;
  p->learned = 0;
  p->window_r = 2;
  p->conf_min = 0.5;
}

lnr_status lnr_query_sizes(int32_t width, int32_t height, int32_t format, const lnr_params* p,
                           lnr_sizes* out) {
  if (!p || !out || width < 1 || height < 1) return LNR_E_ARG;
  if (check_params(nullptr, p) != LNR_OK) return LNR_E_UNSUPPORTED;
  const Geometry g = make_geometry(width, height, *p);
  memset(out, 0, sizeof(*out));
  out->levels = g.levels;
  out->tiles_total = g.tiles_total;
  for (int l = 0; l <= kMaxLevels; ++l) out->tile_off[l] = l < kMaxLevels ? g.lv[l].tile_off : g.tiles_total;
  for (int l = 0; l < g.levels; ++l) {
    out->tile_off[l + 1] = g.lv[l].tile_off + g.lv[l].ntx * g.lv[l].nty;
    out->level_w[l] = g.lv[l].w;
    out->level_h[l] = g.lv[l].h;
  }
  out->channels = format == LNR_I420 || format == LNR_NV12 ? 3 : 1;
  out->blend_levels = merge_levels(width, height);
  return LNR_OK;
}

lnr_status lnr_register_pair(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                             const lnr_params* p, lnr_registration* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  return register_pair_impl(ctx, ref, src, p, out, (hipStream_t)stream);
}

lnr_status lnr_register_pair_noalloc(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                                     const lnr_params* p, lnr_registration* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(nullptr);  // tracing would create events
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  lnr_status s;
  if ((s = check_pair(ctx, ref, src, p, out)) != LNR_OK) return s;
  if (!ctx->scratch) return fail(ctx, LNR_E_HIP, "no scratch on this device: " + ctx->scratch_err);
  const PairPlan q = plan_pair(ref->width, ref->height, p);
  if (q.bytes > (size_t)LNR_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, LNR_E_NOMEM,
                "the registration needs " + std::to_string(q.bytes) +
                    " bytes of scratch; the fixed scratch holds " +
                    std::to_string((size_t)LNR_NOALLOC_SCRATCH_BYTES));
  return enqueue_pair(ctx, ref, src, p, out, q, static_cast<char*>(ctx->scratch),
                      (hipStream_t)stream);
}

}  // extern "C"

namespace {
lnr_status ensure_workers(lnr_ctx* ctx, int K);
size_t round256(size_t b);
}  // namespace

extern "C" {

lnr_status lnr_register_stack(lnr_ctx* ctx, const lnr_frame* frames, int32_t n,
                              const lnr_params* p, lnr_registration* outs, int32_t* ref_index,
                              void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!frames || n < 2 || n > 16 || !outs || !ref_index)
    return fail(ctx, LNR_E_ARG, "register_stack needs 2..16 frames, outputs and ref_index");
  lnr_status s0;
  for (int k = 0; k < n; ++k)
    if ((s0 = check_frame(ctx, &frames[k], "frame")) != LNR_OK) return s0;
  for (int k = 1; k < n; ++k)
    if (frames[k].width != frames[0].width || frames[k].height != frames[0].height)
      return fail(ctx, LNR_E_ARG, "stack frames differ in size");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  // Sec. 2.1: the shortest exposure is the reference (lowest index on ties);
  // without known exposures (not every one positive and finite) the darkest
  // frame, by mean luma (exact integer sums from the frames' histograms;
  // this case waits for the stream once)
  bool known = true;
  for (int k = 0; k < n; ++k)
    if (!(frames[k].exposure > 0.f) || !std::isfinite(frames[k].exposure)) known = false;
  int r = 0;
  if (known) {
    for (int k = 1; k < n; ++k)
      if (frames[k].exposure < frames[r].exposure) r = k;
  } else {
    const hipStream_t st = (hipStream_t)stream;
    if ((s0 = ensure_ws(ctx, (size_t)n * 256 * sizeof(uint32_t), st)) != LNR_OK) return s0;
    uint32_t* hist = static_cast<uint32_t*>(ctx->ws);
    LNR_LAUNCH(k_zero_u32, dim3((n * 256 + 255) / 256), dim3(256), 0, st, hist, n * 256);
    LNR_HIP(hipGetLastError());
    const int W = frames[0].width, H = frames[0].height;
    for (int k = 0; k < n; ++k)
      LNR_HIP(launch_hist(frames[k].plane[0], frames[k].stride[0], frames[k].plane[0],
                          frames[k].stride[0], W, H, hist + 256 * k, 1, st));
    std::vector<uint32_t> hh((size_t)n * 256);
    LNR_HIP(hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           st));
    LNR_HIP(hipStreamSynchronize(st));
    long long best = -1;
    for (int k = 0; k < n; ++k) {
      long long sum = 0;
      for (int v = 0; v < 256; ++v) sum += (long long)v * hh[(size_t)k * 256 + v];
      if (best < 0 || sum < best) { best = sum; r = k; }
    }
  }
  *ref_index = r;
  // n - 1 registrations sharing the reference's equalisation, pyramid and
  // column-major guide (computed once, with the first source), each source
  // in its own workspace slot, the levels and propagation of the sources on
  // the worker streams at once
  const hipStream_t st = (hipStream_t)stream;
  std::vector<int> src_of;
  for (int k = 0; k < n; ++k)
    if (k != r) src_of.push_back(k);
  const int m = (int)src_of.size();
  for (int j = 0; j < m; ++j)
    if ((s0 = check_pair(ctx, &frames[r], &frames[src_of[j]], p, &outs[j])) != LNR_OK) return s0;
  const PairPlan q = plan_pair(frames[r].width, frames[r].height, p);
  const size_t slot = round256(q.bytes);
  if ((s0 = ensure_ws(ctx, (size_t)m * slot, st)) != LNR_OK) return s0;
  if ((s0 = ensure_workers(ctx, m)) != LNR_OK) return s0;
  char* ws = static_cast<char*>(ctx->ws);
  if ((s0 = enqueue_pair_setup(ctx, &frames[r], &frames[src_of[0]], p, &outs[0], q, ws, st)) !=
      LNR_OK)
    return s0;
  for (int j = 1; j < m; ++j)
    if ((s0 = enqueue_source_setup(ctx, &frames[src_of[j]], p, &outs[j], outs[0].yeq_ref, q,
                                   ws + (size_t)j * slot, st)) != LNR_OK)
      return s0;
  LNR_HIP(hipEventRecord(ctx->events[m], st));
  for (int j = 0; j < m; ++j) {
    const hipStream_t w = ctx->workers[j];
    LNR_HIP(hipStreamWaitEvent(w, ctx->events[m], 0));
    char* base = ws + (size_t)j * slot;
    if ((s0 = enqueue_pair_levels(ctx, &frames[r], &frames[src_of[j]], p, &outs[j], q, base, w,
                                  ws)) != LNR_OK)
      return s0;
    if ((s0 = enqueue_pair_finish(ctx, &frames[r], &frames[src_of[j]], p, &outs[j], q, base, w,
                                  ws)) != LNR_OK)
      return s0;
    LNR_HIP(hipEventRecord(ctx->events[j], w));
    LNR_HIP(hipStreamWaitEvent(st, ctx->events[j], 0));
  }
  return LNR_OK;
}

}  // extern "C"

namespace {
// The registered frames' images (the reference converted here, the others
// the registrations' warped images) merged by the fusion, or into the
// irradiance map when `irradiance`.
lnr_status merge_frames(lnr_ctx* ctx, const lnr_frame* frames, int32_t n, int32_t ref_index,
                        const lnr_registration* regs, const lnr_params* p, float* out,
                        void* stream, bool irradiance) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (!frames || n < 1 || n > 16 || ref_index < 0 || ref_index >= n || !out || (n > 1 && !regs))
    return fail(ctx, LNR_E_ARG, "merge needs 1..16 frames, a valid ref_index and outputs");
  for (int k = 0; k < n; ++k)
    if ((s = check_frame(ctx, &frames[k], "frame")) != LNR_OK) return s;
  const lnr_frame& rf = frames[ref_index];
  const int W = rf.width, H = rf.height, ch = rf.format == LNR_Y8 ? 1 : 3;
  for (int k = 0; k < n; ++k)
    if (frames[k].width != W || frames[k].height != H || frames[k].format != rf.format)
      return fail(ctx, LNR_E_ARG, "frames differ in size or format");
  for (int k = 0; k + 1 < n; ++k)
    if (!regs[k].image || !regs[k].yeq_warped || !regs[k].yeq_ref)
      return fail(ctx, LNR_E_ARG, "registration outputs missing");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)W * H;
  // the reference image and its equalised luma live at the head of the
  // workspace; size the whole workspace before anything is enqueued, so the
  // merge below never reallocates it
  const size_t ref_bytes = ((ch * N * sizeof(float) + 255) & ~(size_t)255) + N * sizeof(float);
  {
    const int L = merge_levels(W, H);
    const size_t tot = merge_pyr_elems(W, H, L);
    Plan pl;
    pl.take(ref_bytes);
    pl.take((size_t)n * N * 4);
    pl.take((size_t)n * N * 4);
    pl.take((size_t)n * (ch + 1) * (tot ? tot : 1) * 4);
    pl.take((size_t)ch * (tot ? tot : 1) * 4);
    if ((s = ensure_ws(ctx, pl.off, st)) != LNR_OK) return s;
  }
  char* base = static_cast<char*>(ctx->ws);
  float* ref_img = reinterpret_cast<float*>(base);
  float* ref_yeq = reinterpret_cast<float*>(base + ((ch * N * sizeof(float) + 255) & ~(size_t)255));
  // the reference's RGB and (with registrations) its equalised luma in [0, 1]
  LNR_HIP(launch_frame_rgb_unit(rf.plane[0], rf.stride[0], chroma_of(rf), W, H, ref_img,
                                n > 1 ? regs[0].yeq_ref : nullptr, n > 1 ? ref_yeq : nullptr,
                                st));
  const float* imgs[16];
  const float* yeqs[16];
  if (n == 1) {
    // a fill kernel, not a memset node, so that the call can be graph-captured
    LNR_LAUNCH(k_zero_u32, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
               reinterpret_cast<uint32_t*>(ref_yeq), (int)N);
    LNR_HIP(hipGetLastError());
  }
  int j = 0;
  for (int k = 0; k < n; ++k) {
    if (k == ref_index) {
      imgs[k] = ref_img;
      yeqs[k] = ref_yeq;
    } else {
      imgs[k] = regs[j].image;
      yeqs[k] = regs[j].yeq_warped;
      ++j;
    }
  }
  size_t extra_off = 0;
  if (!irradiance)
    return merge_impl(ctx, n, ch, W, H, imgs, yeqs, ref_index, p, out, st, ref_bytes, &extra_off);
  float rel[16];
  for (int k = 0; k < n; ++k) rel[k] = (float)((double)frames[k].exposure / (double)rf.exposure);
  return merge_impl(ctx, n, ch, W, H, imgs, yeqs, ref_index, p, out, st, ref_bytes, &extra_off,
                    rel);
}
}  // namespace

extern "C" {

lnr_status lnr_merge(lnr_ctx* ctx, const lnr_frame* frames, int32_t n, int32_t ref_index,
                     const lnr_registration* regs, const lnr_params* p, float* out,
                     void* stream) {
  return merge_frames(ctx, frames, n, ref_index, regs, p, out, stream, false);
}

lnr_status lnr_merge_irradiance(lnr_ctx* ctx, const lnr_frame* frames, int32_t n,
                                int32_t ref_index, const lnr_registration* regs,
                                const lnr_params* p, float* out, void* stream) {
  if (ctx && frames && n >= 1 && n <= 16)
    for (int k = 0; k < n; ++k)
      if (!(frames[k].exposure > 0.f) || !std::isfinite(frames[k].exposure))
        return fail(ctx, LNR_E_ARG, "the irradiance map needs positive exposures");
  return merge_frames(ctx, frames, n, ref_index, regs, p, out, stream, true);
}

lnr_status lnr_stage_equalize(lnr_ctx* ctx, const uint8_t* img, int32_t w, int32_t h,
                              int32_t stride, uint8_t* lut, uint8_t* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!img || !out || w < 1 || h < 1 || stride < w || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad equalize arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  lnr_status s;
  if ((s = ensure_ws(ctx, 256 * sizeof(uint32_t), st)) != LNR_OK) return s;
  uint32_t* hist = static_cast<uint32_t*>(ctx->ws);
  Geometry g;
  memset(&g, 0, sizeof(g));
  g.W = w; g.H = h; g.levels = 1;
  g.lv[0].w = w; g.lv[0].h = h; g.lv[0].pix_off = 0;
  LNR_LAUNCH(k_zero_u32, dim3(1), dim3(256), 0, st, hist, 256);
  LNR_HIP(hipGetLastError());
  LNR_HIP(launch_hist(img, stride, img, stride, w, h, hist, 1, st));
  LNR_HIP(launch_lut_pyr(img, stride, img, stride, hist, g, out, out, lut, 1, st));
  return LNR_OK;
}

lnr_status lnr_meter(lnr_ctx* ctx, const uint8_t* y, int32_t w, int32_t h, int32_t stride,
                     int32_t dark, float frac3, float frac4, int32_t* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!y || !out || w < 1 || h < 1 || stride < w || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad metering image");
  if (dark < 0 || dark > 256 || !(frac3 >= 0.f) || !(frac4 >= frac3) || !(frac4 <= 1.f))
    return fail(ctx, LNR_E_ARG, "metering needs 0 <= dark <= 256 and 0 <= frac3 <= frac4 <= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  lnr_status s;
  if ((s = ensure_ws(ctx, 256 * sizeof(uint32_t), st)) != LNR_OK) return s;
  uint32_t* hist = static_cast<uint32_t*>(ctx->ws);
  LNR_LAUNCH(k_zero_u32, dim3(1), dim3(256), 0, st, hist, 256);
  LNR_HIP(hipGetLastError());
  LNR_HIP(launch_hist(y, stride, y, stride, w, h, hist, 1, st));
  LNR_HIP(launch_meter(hist, dark, frac3, frac4, (long long)w * h, out, st));
  return LNR_OK;
}

lnr_status lnr_stage_warp_q8(lnr_ctx* ctx, const uint8_t* src, int32_t w, int32_t h,
                             const double* H, uint8_t* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!src || !H || !out || w < 1 || h < 1 || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad warp arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(launch_warp_q8(src, w, h, H, out, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_stage_search(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped, int32_t w,
                            int32_t h, int32_t R, const lnr_params* p, int32_t* corner_xy,
                            int32_t* disp, uint32_t* ssd, uint8_t* flags, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (!ref || !warped || !corner_xy || !disp || !ssd || !flags || w < 1 || h < 1 ||
      w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad search arguments");
  if (R < 0 || R > kMaxRadius) return fail(ctx, LNR_E_UNSUPPORTED, "radius must be in [0, 32]");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const SearchJob J = search_job(ref, warped, w, h, w / p->tile, corner_xy, disp, ssd, flags);
  LNR_HIP(launch_search(J, h / p->tile, R, search_cfg(*p), kRoleStage, (hipStream_t)stream,
                        nullptr, 0, pinned_search_shape(ctx, w, h, R)));
  return LNR_OK;
}

lnr_status lnr_stage_weed_fit(lnr_ctx* ctx, const int32_t* corner_xy, const int32_t* disp,
                              uint8_t* flags, int32_t ntiles, int32_t w, int32_t h,
                              int32_t level, const lnr_params* p, const double* H_prev,
                              double* H_out, int32_t* counts, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (ntiles < 0 || (ntiles > 0 && (!corner_xy || !disp || !flags)) || !H_prev || !H_out ||
      !counts || w < 1 || h < 1 || w > kMaxSide || h > kMaxSide || level < 0 || level > 255)
    return fail(ctx, LNR_E_ARG, "bad weed/fit arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  Plan pl;
  const WeedPlan wp = plan_weed(pl, ntiles, p->weed_iters);
  if ((s = ensure_ws(ctx, pl.off, (hipStream_t)stream)) != LNR_OK) return s;
  const WeedBufs wb = weed_bufs(static_cast<char*>(ctx->ws), wp);
  LNR_HIP(launch_weed_fit(corner_xy, disp, flags, ntiles, w, h, level, *p, H_prev, H_out, counts,
                          wb, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_stage_flow(lnr_ctx* ctx, const int32_t* corner_xy, const int32_t* disp,
                          const uint8_t* flags, int32_t ntiles, const uint8_t* guide, int32_t w,
                          int32_t h, const lnr_params* p, float* flow, float* ntilde,
                          void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (!guide || !flow || w < 1 || h < 1 || w > kMaxSide || h > kMaxSide ||
      ntiles != (w / p->tile) * (h / p->tile) || (ntiles > 0 && (!corner_xy || !disp || !flags)))
    return fail(ctx, LNR_E_ARG, "bad flow arguments (ntiles must be the level-0 tile count)");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  Plan pl;
  const size_t o_maps = pl.take(dt_maps_bytes(w, h));
  const size_t o_gt = pl.take(dt_guide_t_bytes(w, h));
  const size_t o_coef = pl.take((size_t)p->dt_iters * 256 * sizeof(double));
  if ((s = ensure_ws(ctx, pl.off, (hipStream_t)stream)) != LNR_OK) return s;
  char* base = static_cast<char*>(ctx->ws);
  LNR_HIP(launch_flow(corner_xy, disp, flags, w / p->tile, h / p->tile, p->tile, guide,
                      reinterpret_cast<uint8_t*>(base + o_gt), w, h, *p,
                      base + o_maps, reinterpret_cast<double*>(base + o_coef),
                      flow, ntilde, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_stage_backward_warp(lnr_ctx* ctx, const lnr_frame* src, const uint8_t* yeq,
                                   const double* H, const float* flow, float* image,
                                   float* yeq_warped, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_frame(ctx, src, "src")) != LNR_OK) return s;
  if (!yeq || !H || !flow || !image || !yeq_warped) return fail(ctx, LNR_E_ARG, "bad warp arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(launch_backward_warp(src->plane[0], src->stride[0], chroma_of(*src), yeq, src->width,
                               src->height, H, flow, image, yeq_warped, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_stage_frame_rgb(lnr_ctx* ctx, const lnr_frame* f, const uint8_t* yeq,
                               float* image, float* yeq_out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_frame(ctx, f, "frame")) != LNR_OK) return s;
  if (!image || (yeq && !yeq_out)) return fail(ctx, LNR_E_ARG, "bad frame conversion arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(launch_frame_rgb_unit(f->plane[0], f->stride[0], chroma_of(*f), f->width, f->height,
                                image, yeq, yeq_out, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_stage_merge(lnr_ctx* ctx, int32_t n, int32_t ch, int32_t w, int32_t h,
                           const float* const* imgs, const float* const* yeqs, int32_t ref_index,
                           const lnr_params* p, float* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (n < 1 || n > 16 || (ch != 1 && ch != 3) || w < 1 || h < 1 || w > kMaxSide ||
      h > kMaxSide || !imgs || !yeqs || !out || ref_index < 0 || ref_index >= n)
    return fail(ctx, LNR_E_ARG, "bad merge arguments");
  for (int k = 0; k < n; ++k)
    if (!imgs[k] || !yeqs[k]) return fail(ctx, LNR_E_ARG, "null image or luma pointer");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  return merge_impl(ctx, n, ch, w, h, imgs, yeqs, ref_index, p, out, (hipStream_t)stream, 0,
                    nullptr);
}

lnr_status lnr_stage_irradiance(lnr_ctx* ctx, int32_t n, int32_t ch, int32_t w, int32_t h,
                                const float* const* imgs, const float* const* yeqs,
                                const float* exposures, int32_t ref_index, const lnr_params* p,
                                float* out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (n < 1 || n > 16 || (ch != 1 && ch != 3) || w < 1 || h < 1 || w > kMaxSide ||
      h > kMaxSide || !imgs || !yeqs || !exposures || !out || ref_index < 0 || ref_index >= n)
    return fail(ctx, LNR_E_ARG, "bad irradiance arguments");
  for (int k = 0; k < n; ++k) {
    if (!imgs[k] || !yeqs[k]) return fail(ctx, LNR_E_ARG, "null image or luma pointer");
    if (!(exposures[k] > 0.f) || !std::isfinite(exposures[k]))
      return fail(ctx, LNR_E_ARG, "the irradiance map needs positive exposures");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  float rel[16];
  for (int k = 0; k < n; ++k) rel[k] = (float)((double)exposures[k] / (double)exposures[ref_index]);
  return merge_impl(ctx, n, ch, w, h, imgs, yeqs, ref_index, p, out, (hipStream_t)stream, 0,
                    nullptr, rel);
}

// ---------------------------------------------------------------- batches
}  // extern "C"

namespace {

lnr_status ensure_workers(lnr_ctx* ctx, int K) {
  while ((int)ctx->workers.size() < K) {
    hipStream_t w = nullptr;
    LNR_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
    ctx->workers.push_back(w);
  }
  while ((int)ctx->events.size() < K + 1) {
    hipEvent_t e = nullptr;
    LNR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->events.push_back(e);
  }
  if (!ctx->capture) LNR_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  return LNR_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Longest-processing-time assignment of pairs (by pixel count) to K streams.
std::vector<std::vector<int>> assign_pairs(const lnr_frame* refs, int n, int K) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const long long na = (long long)refs[a].width * refs[a].height;
    const long long nb = (long long)refs[b].width * refs[b].height;
    return na != nb ? na > nb : a < b;
  });
  std::vector<std::vector<int>> lists(K);
  std::vector<long long> load(K, 0);
  for (int i : order) {
    int k = 0;
    for (int j = 1; j < K; ++j)
      if (load[j] < load[k]) k = j;
    lists[k].push_back(i);
    load[k] += (long long)refs[i].width * refs[i].height;
  }
  return lists;
}

// Fork from `origin` to K worker streams, each registering its pairs in its
// own workspace slot, and join back to `origin`.
lnr_status enqueue_batch(lnr_ctx* ctx, const lnr_frame* refs, const lnr_frame* srcs, int n,
                         const lnr_params* p, lnr_registration* outs,
                         const std::vector<PairPlan>& plans, size_t slot, int K,
                         hipStream_t origin) {
  const auto lists = assign_pairs(refs, n, K);
  LNR_HIP(hipEventRecord(ctx->events[K], origin));
  for (int k = 0; k < K; ++k) {
    LNR_HIP(hipStreamWaitEvent(ctx->workers[k], ctx->events[K], 0));
    char* base = static_cast<char*>(ctx->ws) + (size_t)k * slot;
    for (int i : lists[k]) {
      lnr_status s = enqueue_pair(ctx, &refs[i], &srcs[i], p, &outs[i], plans[i], base,
                                  ctx->workers[k]);
      if (s != LNR_OK) return s;
    }
    LNR_HIP(hipEventRecord(ctx->events[k], ctx->workers[k]));
    LNR_HIP(hipStreamWaitEvent(origin, ctx->events[k], 0));
  }
  return LNR_OK;
}

// A level-synchronous batch (plain method, warped-source search): every pair
// has its own workspace; the set-up (equalisation, pyramids) and the end
// (propagation, backward warp) of each pair run on the worker streams, and
// each pyramid level runs for all pairs at once: one warp launch over all
// their rows, one search launch over all their tiles and one launch per
// weeding kernel over all their levels (device job tables).
struct LevelTables {
  size_t o_warp = 0, o_row0 = 0, o_sjob = 0, o_first = 0, o_wjob = 0;  // in the blob
  int njobs = 0, rows = 0, wmax = 0, ntiles = 0, max_tiles = 0;
};
struct BatchLayout {
  std::vector<size_t> off;  // each pair's workspace offset
  size_t ws_bytes = 0;
  int levels = 0;           // the deepest pyramid
  LevelTables lv[kMaxLevels];
  std::vector<uint8_t> blob;  // the job tables (device pointers into the workspace)
};

size_t blob_take(std::vector<uint8_t>& blob, size_t bytes) {
  const size_t o = (blob.size() + 255) & ~(size_t)255;
  blob.resize(o + bytes);
  return o;
}

BatchLayout plan_batch(const lnr_frame* refs, int n, const std::vector<PairPlan>& plans) {
  BatchLayout b;
  b.off.resize((size_t)n);
  for (int i = 0; i < n; ++i) {
    b.off[i] = b.ws_bytes;
    b.ws_bytes += (plans[i].bytes + 255) & ~(size_t)255;
    b.levels = std::max(b.levels, plans[i].g.levels);
  }
  (void)refs;
  return b;
}

// Fills the job tables for the workspace at ws (after it has been sized).
void fill_batch_tables(BatchLayout& b, int n, const lnr_params* p, lnr_registration* outs,
                       const std::vector<PairPlan>& plans, char* ws) {
  b.blob.clear();
  for (int l = 0; l < b.levels; ++l) {
    std::vector<int> jobs;
    for (int i = 0; i < n; ++i)
      if (plans[i].g.levels > l) jobs.push_back(i);
    LevelTables& T = b.lv[l];
    T.njobs = (int)jobs.size();
    T.o_warp = blob_take(b.blob, sizeof(WarpJob) * jobs.size());
    T.o_row0 = blob_take(b.blob, sizeof(int) * (jobs.size() + 1));
    T.o_sjob = blob_take(b.blob, sizeof(SearchJob) * jobs.size());
    T.o_first = blob_take(b.blob, sizeof(int) * (jobs.size() + 1));
    T.o_wjob = blob_take(b.blob, sizeof(WeedJob) * jobs.size());
    int row = 0, tile = 0;
    for (size_t k = 0; k < jobs.size(); ++k) {
      const int i = jobs[k];
      const PairPlan& q = plans[i];
      const Level& L = q.g.lv[l];
      char* base = ws + b.off[i];
      const int nt = L.ntx * L.nty;
      const int words = nt > 0 ? (nt + 63) / 64 : 1;
      const WeedBufs wb = weed_bufs(base, q.wp);
      lnr_registration& o = outs[i];
      uint8_t* warped = reinterpret_cast<uint8_t*>(base + q.o_warp);
      if (l == 0 && o.warped0) warped = o.warped0;
      WarpJob wj;
      wj.src = reinterpret_cast<uint8_t*>(base + q.o_psrc) + L.pix_off;
      wj.w = L.w; wj.h = L.h; wj.nwords = words;
      wj.Hn = o.H + 9 * (l + 1);
      wj.out = warped;
      wj.vb = wb.vb; wj.sums = wb.sums;
      memcpy(b.blob.data() + T.o_warp + k * sizeof(WarpJob), &wj, sizeof(wj));
      memcpy(b.blob.data() + T.o_row0 + k * sizeof(int), &row, sizeof(int));
      // coarse levels warp their windows on the fly, as in a single registration
      const SearchJob sj = search_job(
          reinterpret_cast<uint8_t*>(base + q.o_pref) + L.pix_off,
          l == 0 ? warped : reinterpret_cast<uint8_t*>(base + q.o_psrc) + L.pix_off, L.w, L.h,
          L.ntx, o.corner_xy + 2 * L.tile_off, o.disp + 2 * L.tile_off, o.ssd + L.tile_off,
          o.flags + L.tile_off, nullptr, wb.vb, nullptr, l == 0 ? nullptr : o.H + 9 * (l + 1));
      memcpy(b.blob.data() + T.o_sjob + k * sizeof(SearchJob), &sj, sizeof(sj));
      memcpy(b.blob.data() + T.o_first + k * sizeof(int), &tile, sizeof(int));
      WeedJob ej;
      ej.cxy = o.corner_xy + 2 * L.tile_off; ej.disp = o.disp + 2 * L.tile_off;
      ej.flags = o.flags + L.tile_off;
      ej.ntiles = nt; ej.w = L.w; ej.h = L.h; ej.words = words;
      ej.b = wb;
      ej.Hprev = o.H + 9 * (l + 1); ej.Hbase = ej.Hprev; ej.Hout = o.H + 9 * l;
      ej.counts = o.counts + 4 * l;
      ej.clear_vb = l >= 2 ? wb.vb : nullptr;
      ej.clear_words = l >= 2 ? level_words(q.g.lv[l - 1]) : 0;
      memcpy(b.blob.data() + T.o_wjob + k * sizeof(WeedJob), &ej, sizeof(ej));
      row += L.h;
      tile += nt;
      T.wmax = std::max(T.wmax, L.w);
      T.max_tiles = std::max(T.max_tiles, nt);
    }
    memcpy(b.blob.data() + T.o_row0 + jobs.size() * sizeof(int), &row, sizeof(int));
    memcpy(b.blob.data() + T.o_first + jobs.size() * sizeof(int), &tile, sizeof(int));
    T.rows = row;
    T.ntiles = tile;
  }
  (void)p;
}

lnr_status enqueue_batch_levels(lnr_ctx* ctx, const lnr_frame* refs, const lnr_frame* srcs,
                                int n, const lnr_params* p, lnr_registration* outs,
                                const std::vector<PairPlan>& plans, const BatchLayout& b,
                                const char* tab, int K, int kx, hipStream_t origin) {
  const auto lists = assign_pairs(refs, n, K);
  char* ws = static_cast<char*>(ctx->ws);
  lnr_status s;
  // set-up of every pair on the worker streams
  LNR_HIP(hipEventRecord(ctx->events[K], origin));
  for (int k = 0; k < K; ++k) {
    LNR_HIP(hipStreamWaitEvent(ctx->workers[k], ctx->events[K], 0));
    for (int i : lists[k])
      if ((s = enqueue_pair_setup(ctx, &refs[i], &srcs[i], p, &outs[i], plans[i], ws + b.off[i],
                                  ctx->workers[k])) != LNR_OK)
        return s;
    LNR_HIP(hipEventRecord(ctx->events[k], ctx->workers[k]));
    LNR_HIP(hipStreamWaitEvent(origin, ctx->events[k], 0));
  }
  // the levels, all pairs at once
  const SearchCfg cfg = search_cfg(*p);
  for (int l = b.levels - 1; l >= 0; --l) {
    const LevelTables& T = b.lv[l];
    if (T.njobs == 0) continue;
    const int R = l == 0 ? p->radius0 : p->radius_coarse;
    if (l == 0)  // coarse levels are warped inside their search
      LNR_HIP(launch_warp_jobs(reinterpret_cast<const WarpJob*>(tab + T.o_warp),
                               reinterpret_cast<const int*>(tab + T.o_row0), T.njobs, T.rows,
                               T.wmax, origin));
    SearchWork wk;
    wk.first = reinterpret_cast<const int*>(tab + T.o_first);
    wk.njobs = T.njobs;
    wk.list = nullptr;
    wk.count = nullptr;
    wk.ntotal = T.ntiles;
    wk.out_list = nullptr;
    wk.out_count = nullptr;
    // (coarse levels warp their windows; level 0 reads the warped level)
    LNR_HIP(launch_search_work(reinterpret_cast<const SearchJob*>(tab + T.o_sjob), wk, R, cfg,
                               kVisitSearchAll, 0, 0, kx, T.ntiles, origin, nullptr, l != 0));
    LNR_HIP(launch_weed_jobs(reinterpret_cast<const WeedJob*>(tab + T.o_wjob), T.njobs,
                             T.max_tiles, l, *p, origin));
  }
  // propagation and backward warp of every pair on the worker streams
  LNR_HIP(hipEventRecord(ctx->events[K], origin));
  for (int k = 0; k < K; ++k) {
    LNR_HIP(hipStreamWaitEvent(ctx->workers[k], ctx->events[K], 0));
    for (int i : lists[k])
      if ((s = enqueue_pair_finish(ctx, &refs[i], &srcs[i], p, &outs[i], plans[i], ws + b.off[i],
                                   ctx->workers[k])) != LNR_OK)
        return s;
    LNR_HIP(hipEventRecord(ctx->events[k], ctx->workers[k]));
    LNR_HIP(hipStreamWaitEvent(origin, ctx->events[k], 0));
  }
  return LNR_OK;
}

void push_bytes(std::vector<uint64_t>& key, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; i += 8) {
    uint64_t v = 0;
    memcpy(&v, c + i, n - i < 8 ? n - i : 8);
    key.push_back(v);
  }
}

}  // namespace

extern "C" {

lnr_status lnr_register_batch(lnr_ctx* ctx, const lnr_frame* refs, const lnr_frame* srcs,
                              int32_t n, const lnr_params* p, lnr_registration* outs,
                              int32_t flags, void* stream) {
  if (!ctx) return LNR_E_ARG;
  if (!refs || !srcs || !outs || n < 1 || n > 4096)
    return fail(ctx, LNR_E_ARG, "register_batch needs 1..4096 pairs and their outputs");
  if (flags & ~(LNR_BATCH_GRAPH | LNR_BATCH_AUTOTUNE))
    return fail(ctx, LNR_E_ARG, "unknown batch flags");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  lnr_status s;
  std::vector<PairPlan> plans((size_t)n);
  size_t slot = 0;
  for (int i = 0; i < n; ++i) {
    if ((s = check_pair(ctx, &refs[i], &srcs[i], p, &outs[i])) != LNR_OK) return s;
    plans[i] = plan_pair(refs[i].width, refs[i].height, p);
    slot = std::max(slot, round256(plans[i].bytes));
  }
  const hipStream_t st = (hipStream_t)stream;
  // The plain method runs level-synchronously (every pair's level in one
  // launch per kernel); the learned proposal and the unwarped-source search
  // register each pair on its own over the worker streams.
  const bool levels = !p->learned && p->search_frame == 0;
  BatchLayout lay;
  if (levels) lay = plan_batch(refs, n, plans);
  auto ws_need = [&](int k) { return levels ? lay.ws_bytes : (size_t)k * slot; };
  // the batch's shape: sizes and parameters (concurrency is tuned per shape)
  std::vector<uint64_t> shape;
  push_bytes(shape, p, sizeof(*p));
  for (int i = 0; i < n; ++i)
    shape.push_back(((uint64_t)refs[i].width << 32) | (uint32_t)refs[i].height);
  int K = n < 4 ? n : 4, kx = 8;
  // the level-synchronous batch's job tables (device pointers into the
  // workspace, which must not move after they are written)
  auto upload_eager_tables = [&]() -> lnr_status {
    if ((s = ensure_ws(ctx, ws_need(K), st)) != LNR_OK) return s;
    fill_batch_tables(lay, n, p, outs, plans, static_cast<char*>(ctx->ws));
    LNR_HIP(hipStreamSynchronize(st));  // an earlier eager batch may still read them
    if (ctx->tables_size < lay.blob.size()) {
      if (ctx->tables) LNR_HIP(hipFree(ctx->tables));
      ctx->tables = nullptr;
      ctx->tables_size = 0;
      LNR_HIP(hipMalloc(&ctx->tables, lay.blob.size()));
      ctx->tables_size = lay.blob.size();
    }
    LNR_HIP(hipMemcpy(ctx->tables, lay.blob.data(), lay.blob.size(), hipMemcpyHostToDevice));
    return LNR_OK;
  };
  auto enqueue = [&](int k, int kxx, const char* tab, hipStream_t o) -> lnr_status {
    if (levels)
      return enqueue_batch_levels(ctx, refs, srcs, n, p, outs, plans, lay, tab, k, kxx, o);
    return enqueue_batch(ctx, refs, srcs, n, p, outs, plans, slot, k, o);
  };
  auto kt = ctx->batch_k.find(shape);
  if (kt != ctx->batch_k.end()) {
    K = kt->second;
    auto kk = ctx->batch_kx.find(shape);
    if (kk != ctx->batch_kx.end()) kx = kk->second;
  } else if (flags & LNR_BATCH_AUTOTUNE) {
    if (!levels) {
      // the search's workgroup shape per level, for every size not tuned yet
      for (int i = 0; i < n; ++i) {
        const auto key = std::make_tuple((int)refs[i].width, (int)refs[i].height, (int)p->radius0);
        if (ctx->search_split.count(key)) continue;
        if ((s = lnr_autotune_search(ctx, refs[i].width, refs[i].height, p, nullptr, stream)) !=
            LNR_OK)
          return s;
      }
    }
    // time 1, 2, 4 and 8 concurrent streams on this batch (eager), then (level-
    // synchronous batches) 8 or 12 search candidates per lane or the matrix
    // cores; keep the fastest
    hipEvent_t t0 = nullptr, t1 = nullptr;
    LNR_HIP(hipEventCreate(&t0));
    LNR_HIP(hipEventCreate(&t1));
    auto time_one = [&](int k, int kxx, float* ms) -> lnr_status {
      if ((s = ensure_ws(ctx, ws_need(k), st)) != LNR_OK) return s;
      if ((s = ensure_workers(ctx, k)) != LNR_OK) return s;
      if (levels && (s = upload_eager_tables()) != LNR_OK) return s;
      TraceGuard tg(ctx);
      LNR_HIP(hipEventRecord(t0, st));
      if ((s = enqueue(k, kxx, static_cast<const char*>(ctx->tables), st)) != LNR_OK) return s;
      LNR_HIP(hipEventRecord(t1, st));
      LNR_HIP(hipEventSynchronize(t1));
      LNR_HIP(hipEventElapsedTime(ms, t0, t1));
      return LNR_OK;
    };
    const int cand[4] = {1, 2, 4, 8};
    float best = 0.f;
    for (int c = 0; c < 4; ++c) {
      const int k = cand[c];
      if (k > n) break;
      float ms = 0.f;
      if ((s = time_one(k, 8, &ms)) != LNR_OK) return s;
      if (c == 0 || ms < best) { best = ms; K = k; }
    }
    if (levels)
      for (const int kxx : {12, 0}) {  // 12 candidates per lane, the matrix cores
        float ms = 0.f;
        if ((s = time_one(K, kxx, &ms)) != LNR_OK) return s;
        if (ms < best) { best = ms; kx = kxx; }
      }
    LNR_HIP(hipEventDestroy(t0));
    LNR_HIP(hipEventDestroy(t1));
    ctx->batch_k[shape] = K;
    ctx->batch_kx[shape] = kx;
  }
  if ((s = ensure_ws(ctx, ws_need(K), st)) != LNR_OK) return s;
  if ((s = ensure_workers(ctx, K)) != LNR_OK) return s;
  if (!(flags & LNR_BATCH_GRAPH)) {
    if (levels && (s = upload_eager_tables()) != LNR_OK) return s;
    TraceGuard tg(ctx);
    return enqueue(K, kx, static_cast<const char*>(ctx->tables), st);
  }
  // graph: the whole batch as one executable graph, cached per inputs and
  // outputs (with its own job tables)
  std::vector<uint64_t> key = shape;
  key.push_back((uint64_t)K);
  key.push_back((uint64_t)kx);
  key.push_back((uint64_t)(uintptr_t)ctx->ws);
  for (int i = 0; i < n; ++i) {
    push_bytes(key, &refs[i], sizeof(lnr_frame));
    push_bytes(key, &srcs[i], sizeof(lnr_frame));
    push_bytes(key, &outs[i], sizeof(lnr_registration));
  }
  hipGraphExec_t exec = nullptr;
  for (auto& c : ctx->graphs)
    if (c.key == key) exec = c.exec;
  if (!exec) {
    void* tab = nullptr;
    if (levels) {
      fill_batch_tables(lay, n, p, outs, plans, static_cast<char*>(ctx->ws));
      LNR_HIP(hipMalloc(&tab, lay.blob.size()));
      const hipError_t ec = hipMemcpy(tab, lay.blob.data(), lay.blob.size(),
                                      hipMemcpyHostToDevice);
      if (ec != hipSuccess) {
        (void)hipFree(tab);
        return hip_fail(ctx, ec, "hipMemcpy(batch tables)");
      }
    }
    hipGraph_t graph = nullptr;
    hipError_t eb = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
      if (tab) (void)hipFree(tab);
      return hip_fail(ctx, eb, "hipStreamBeginCapture");
    }
    s = enqueue(K, kx, static_cast<const char*>(tab), ctx->capture);
    const hipError_t ec = hipStreamEndCapture(ctx->capture, &graph);
    hipError_t ei = hipSuccess;
    if (s == LNR_OK && ec == hipSuccess) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (s != LNR_OK || ec != hipSuccess || ei != hipSuccess) {
      if (tab) (void)hipFree(tab);
      if (s != LNR_OK) return s;
      return hip_fail(ctx, ec != hipSuccess ? ec : ei,
                      ec != hipSuccess ? "hipStreamEndCapture" : "hipGraphInstantiate");
    }
    if (ctx->graphs.size() >= 8) {
      LNR_HIP(hipGraphExecDestroy(ctx->graphs.front().exec));
      if (ctx->graphs.front().tables) LNR_HIP(hipFree(ctx->graphs.front().tables));
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(lnr_ctx::Cached{key, exec, tab});
  }
  LNR_HIP(hipGraphLaunch(exec, st));
  return LNR_OK;
}

lnr_status lnr_set_flow_shape(lnr_ctx* ctx, int32_t w, int32_t h, const int32_t* shape) {
  if (!ctx) return LNR_E_ARG;
  if (!shape || w < 1 || h < 1 || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad flow shape arguments");
  DtShape s;
  s.seg = shape[0]; s.nt = shape[1]; s.l = shape[2]; s.ncol = shape[3]; s.nseg = shape[4];
  if (!dt_shape_valid(s, w, h))
    return fail(ctx, LNR_E_UNSUPPORTED, "not an instantiated propagation shape covering w x h");
  ctx->dt_shapes[std::make_pair((int)w, (int)h)] = s;
  return LNR_OK;
}

int32_t lnr_flow_shapes(int32_t w, int32_t h, int32_t* shapes, int32_t max) {
  DtShape c[64];
  const int n = dt_shape_candidates(w, h, c, 64);
  for (int i = 0; i < n && i < max && shapes; ++i) {
    shapes[5 * i] = c[i].seg; shapes[5 * i + 1] = c[i].nt; shapes[5 * i + 2] = c[i].l;
    shapes[5 * i + 3] = c[i].ncol; shapes[5 * i + 4] = c[i].nseg;
  }
  return n;
}

lnr_status lnr_autotune_flow(lnr_ctx* ctx, int32_t w, int32_t h, const lnr_params* p,
                             int32_t* shape_out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (w < p->tile || h < p->tile || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad image size");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)w * h;
  const int ntx = w / p->tile, nty = h / p->tile, nt = ntx * nty;
  Plan pl;
  const size_t o_g = pl.take(N), o_maps = pl.take(dt_maps_bytes(w, h));
  const size_t o_gt = pl.take(dt_guide_t_bytes(w, h));
  const size_t o_flow = pl.take(2 * N * sizeof(float)), o_nt = pl.take(N * sizeof(float));
  const size_t o_coef = pl.take((size_t)p->dt_iters * 256 * sizeof(double));
  const size_t o_cxy = pl.take((size_t)nt * 2 * sizeof(int32_t));
  const size_t o_d = pl.take((size_t)nt * 2 * sizeof(int32_t)), o_f = pl.take((size_t)nt);
  if ((s = ensure_ws(ctx, pl.off, st)) != LNR_OK) return s;
  char* b = static_cast<char*>(ctx->ws);
  // the kernels' work does not depend on the values: a flat guide and no
  // matches time them exactly
  LNR_HIP(hipMemsetAsync(b, 0, pl.off, st));
  DtShape cand[64];
  const int nc = dt_shape_candidates(w, h, cand, 64);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  LNR_HIP(hipEventCreate(&t0));
  LNR_HIP(hipEventCreate(&t1));
  DtShape best = dt_default_shape(w, h);
  float best_ms = 0.f;
  for (int c = 0; c < nc; ++c) {
    float tot = 0.f;
    for (int rep = 0; rep < 4; ++rep) {  // the first run warms up
      LNR_HIP(hipEventRecord(t0, st));
      LNR_HIP(launch_flow(reinterpret_cast<int32_t*>(b + o_cxy), reinterpret_cast<int32_t*>(b + o_d),
                          reinterpret_cast<uint8_t*>(b + o_f), ntx, nty, p->tile,
                          reinterpret_cast<uint8_t*>(b + o_g), reinterpret_cast<uint8_t*>(b + o_gt),
                          w, h, *p,
                          b + o_maps, reinterpret_cast<double*>(b + o_coef),
                          reinterpret_cast<float*>(b + o_flow), reinterpret_cast<float*>(b + o_nt),
                          st, &cand[c]));
      LNR_HIP(hipEventRecord(t1, st));
      LNR_HIP(hipEventSynchronize(t1));
      float ms = 0.f;
      LNR_HIP(hipEventElapsedTime(&ms, t0, t1));
      if (rep) tot += ms;
    }
    if (c == 0 || tot < best_ms) { best_ms = tot; best = cand[c]; }
  }
  LNR_HIP(hipEventDestroy(t0));
  LNR_HIP(hipEventDestroy(t1));
  ctx->dt_shapes[std::make_pair((int)w, (int)h)] = best;
  if (shape_out) {
    shape_out[0] = best.seg; shape_out[1] = best.nt; shape_out[2] = best.l;
    shape_out[3] = best.ncol; shape_out[4] = best.nseg;
  }
  return LNR_OK;
}

lnr_status lnr_set_search_shape(lnr_ctx* ctx, int32_t level_w, int32_t level_h, int32_t radius,
                                int32_t shape) {
  if (!ctx) return LNR_E_ARG;
  const int split = shape & kSearchSplitMask;
  if (level_w < 1 || level_h < 1 || radius < 0 || radius > kMaxRadius || split < 1 ||
      (shape & ~(kSearchKx12 | kSearchMfma | kSearchSplitMask)) ||
      ((shape & kSearchKx12) && (shape & kSearchMfma)))
    return fail(ctx, LNR_E_ARG, "bad search shape");
  lnr_params dp;
  lnr_default_params(&dp);
  if (!search_shape_fits(radius, search_cfg(dp), shape))
    return fail(ctx, LNR_E_ARG, "search shape needs more than 1024 threads or 64 KB");
  ctx->search_split[std::make_tuple((int)level_w, (int)level_h, (int)radius)] = shape;
  return LNR_OK;
}

lnr_status lnr_autotune_search(lnr_ctx* ctx, int32_t w, int32_t h, const lnr_params* p,
                               int32_t* splits_out, void* stream) {
  if (!ctx) return LNR_E_ARG;
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (w < p->tile || h < p->tile || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad image size");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const hipStream_t st = (hipStream_t)stream;
  const Geometry g = make_geometry(w, h, *p);
  const SearchCfg cfg = search_cfg(*p);
  // level 0 is the largest: its buffers serve every level
  const size_t N = (size_t)w * h;
  const int nt = g.lv[0].ntx * g.lv[0].nty;
  Plan pl;
  const size_t o_a = pl.take(N), o_b = pl.take(N);
  const size_t o_cxy = pl.take((size_t)nt * 2 * sizeof(int32_t));
  const size_t o_d = pl.take((size_t)nt * 2 * sizeof(int32_t));
  const size_t o_s = pl.take((size_t)nt * sizeof(uint32_t)), o_f = pl.take((size_t)nt);
  if ((s = ensure_ws(ctx, pl.off, st)) != LNR_OK) return s;
  char* b = static_cast<char*>(ctx->ws);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  LNR_HIP(hipEventCreate(&t0));
  LNR_HIP(hipEventCreate(&t1));
  for (int l = 0; l < g.levels; ++l) {
    const Level& L = g.lv[l];
    const int R = l == 0 ? p->radius0 : p->radius_coarse;
    const int n = L.w * L.h;
    // a textured reference and an identical "warped" source: every tile has
    // corners and every candidate is scored, as on real frames
    LNR_HIP(launch_texture(reinterpret_cast<uint8_t*>(b + o_a), n, 0x5eedu + (uint32_t)l, st));
    LNR_HIP(hipMemcpyAsync(b + o_b, b + o_a, (size_t)n, hipMemcpyDeviceToDevice, st));
    int cand[24];
    const int nc = search_split_candidates(R, cfg, cand, 24);
    int best = cand[0];
    float best_ms = 0.f;
    for (int c = 0; c < nc; ++c) {
      float tot = 0.f;
      for (int rep = 0; rep < 4; ++rep) {  // the first run warms up
        LNR_HIP(hipEventRecord(t0, st));
        const SearchJob J = search_job(
            reinterpret_cast<uint8_t*>(b + o_a), reinterpret_cast<uint8_t*>(b + o_b), L.w, L.h,
            L.ntx, reinterpret_cast<int32_t*>(b + o_cxy), reinterpret_cast<int32_t*>(b + o_d),
            reinterpret_cast<uint32_t*>(b + o_s), reinterpret_cast<uint8_t*>(b + o_f));
        LNR_HIP(launch_search(J, L.nty, R, cfg, kRoleTrial, st, nullptr, 0, cand[c]));
        LNR_HIP(hipEventRecord(t1, st));
        LNR_HIP(hipEventSynchronize(t1));
        float ms = 0.f;
        LNR_HIP(hipEventElapsedTime(&ms, t0, t1));
        if (rep) tot += ms;
      }
      if (c == 0 || tot < best_ms) { best_ms = tot; best = cand[c]; }
    }
    ctx->search_split[std::make_tuple(L.w, L.h, R)] = best;
    if (splits_out) splits_out[l] = best;
  }
  for (int l = g.levels; l < kMaxLevels && splits_out; ++l) splits_out[l] = 0;
  LNR_HIP(hipEventDestroy(t0));
  LNR_HIP(hipEventDestroy(t1));
  return LNR_OK;
}

lnr_status lnr_stage_search_window(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped,
                                   int32_t w, int32_t h, int32_t R, const int32_t* centre,
                                   const lnr_params* p, int32_t* corner_xy, int32_t* disp,
                                   uint32_t* ssd, uint8_t* flags, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  lnr_status s;
  if ((s = check_params(ctx, p)) != LNR_OK) return s;
  if (!ref || !warped || !centre || !corner_xy || !disp || !ssd || !flags || w < 1 || h < 1 ||
      w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad search arguments");
  if (R < 0 || R > kMaxRadius) return fail(ctx, LNR_E_UNSUPPORTED, "radius must be in [0, 32]");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  // the kernel clamps nothing: centres are checked on the host side of the
  // caller's contract (|centre| + R <= 32) by reading them back here
  const int nt = (w / p->tile) * (h / p->tile);
  if (nt > 0) {
    std::vector<int32_t> c((size_t)nt * 2);
    LNR_HIP(hipMemcpyAsync(c.data(), centre, c.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
    LNR_HIP(hipStreamSynchronize((hipStream_t)stream));
    for (int32_t v : c)
      if (v < -kMaxRadius || v > kMaxRadius || std::abs(v) + R > kMaxRadius)
        return fail(ctx, LNR_E_ARG, "window centre out of range (|centre| + R must be <= 32)");
  }
  const SearchJob J = search_job(ref, warped, w, h, w / p->tile, corner_xy, disp, ssd, flags,
                                 centre);
  LNR_HIP(launch_search(J, h / p->tile, R, search_cfg(*p), kRoleStage, (hipStream_t)stream,
                        nullptr, 0, pinned_search_shape(ctx, w, h, R)));
  return LNR_OK;
}

}  // extern "C"

namespace {
// the context's network buffers (parameters, AdamW moments, packed bf16)
lnr_status ensure_cnn(lnr_ctx* ctx) {
  const size_t np = (size_t)cnn_param_count();
  if (!ctx->cnn) {
    hipError_t e = hipMalloc(&ctx->cnn, 3 * np * sizeof(float));
    if (e != hipSuccess) { ctx->cnn = nullptr; return fail(ctx, LNR_E_NOMEM, "network hipMalloc failed"); }
    e = hipMalloc(&ctx->cnn_packed, cnn_packed_elems() * sizeof(uint16_t));
    if (e != hipSuccess) {
      ctx->cnn_packed = nullptr;
      LNR_HIP(hipFree(ctx->cnn));
      ctx->cnn = nullptr;
      return fail(ctx, LNR_E_NOMEM, "network hipMalloc failed");
    }
  }
  return LNR_OK;
}

constexpr uint32_t kNetMagic = 0x50524e4cu;  // "LNRP" little-endian
constexpr uint32_t kNetVersion = 1u;
constexpr uint32_t kCkptMagic = 0x4b524e4cu;  // "LNRK" little-endian
constexpr uint32_t kCkptVersion = 1u;
}  // namespace

extern "C" {

lnr_status lnr_proposal_set(lnr_ctx* ctx, const float* params, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!params) return fail(ctx, LNR_E_ARG, "params is null");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const size_t np = (size_t)cnn_param_count();
  lnr_status s;
  if ((s = ensure_cnn(ctx)) != LNR_OK) return s;
  const hipStream_t st = (hipStream_t)stream;
  LNR_HIP(hipMemcpyAsync(ctx->cnn, params, np * sizeof(float), hipMemcpyDeviceToDevice, st));
  LNR_HIP(hipMemsetAsync(ctx->cnn + np, 0, 2 * np * sizeof(float), st));
  LNR_HIP(launch_cnn_pack(ctx->cnn, ctx->cnn_packed, st));
  ctx->cnn_step = 0;
  return LNR_OK;
}

lnr_status lnr_proposal_get(lnr_ctx* ctx, float* params, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!params) return fail(ctx, LNR_E_ARG, "params is null");
  if (!ctx->cnn) return fail(ctx, LNR_E_ARG, "no network set");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(hipMemcpyAsync(params, ctx->cnn, (size_t)cnn_param_count() * sizeof(float),
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_proposal_save(lnr_ctx* ctx, const char* path, void* stream) {
  if (!ctx) return LNR_E_ARG;
  if (!path) return fail(ctx, LNR_E_ARG, "path is null");
  if (!ctx->cnn) return fail(ctx, LNR_E_ARG, "no network set");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const size_t np = (size_t)cnn_param_count();
  std::vector<float> host(np);
  const hipStream_t st = (hipStream_t)stream;
  LNR_HIP(hipMemcpyAsync(host.data(), ctx->cnn, np * sizeof(float), hipMemcpyDeviceToHost, st));
  LNR_HIP(hipStreamSynchronize(st));
  FILE* f = fopen(path, "wb");
  if (!f) return fail(ctx, LNR_E_WEIGHTS, "cannot open the network file for writing");
  const uint32_t hdr[4] = {kNetMagic, kNetVersion, (uint32_t)np, 0u};
  const bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
                  fwrite(host.data(), sizeof(float), np, f) == np;
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return fail(ctx, LNR_E_WEIGHTS, "writing the network file failed");
  return LNR_OK;
}

lnr_status lnr_proposal_load(lnr_ctx* ctx, const char* path, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!path) return fail(ctx, LNR_E_ARG, "path is null");
  const size_t np = (size_t)cnn_param_count();
  std::vector<float> host(np);
  {
    FILE* f = fopen(path, "rb");
    if (!f) return fail(ctx, LNR_E_WEIGHTS, "cannot open the network file");
    uint32_t hdr[4] = {0u, 0u, 0u, 0u};
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == kNetMagic &&
              hdr[1] == kNetVersion && hdr[2] == (uint32_t)np && hdr[3] == 0u &&
              fread(host.data(), sizeof(float), np, f) == np;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
    fclose(f);
    if (!ok) return fail(ctx, LNR_E_WEIGHTS, "not a network file of this version and size");
  }
  for (size_t i = 0; i < np; ++i)
    if (!std::isfinite(host[i])) return fail(ctx, LNR_E_WEIGHTS, "non-finite network parameter");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  lnr_status s;
  if ((s = ensure_cnn(ctx)) != LNR_OK) return s;
  const hipStream_t st = (hipStream_t)stream;
  LNR_HIP(hipMemcpyAsync(ctx->cnn, host.data(), np * sizeof(float), hipMemcpyHostToDevice, st));
  LNR_HIP(hipMemsetAsync(ctx->cnn + np, 0, 2 * np * sizeof(float), st));
  LNR_HIP(launch_cnn_pack(ctx->cnn, ctx->cnn_packed, st));
  LNR_HIP(hipStreamSynchronize(st));  // the host copy is freed on return
  ctx->cnn_step = 0;
  return LNR_OK;
}

lnr_status lnr_proposal_checkpoint_save(lnr_ctx* ctx, const char* path, uint64_t counter,
                                        void* stream) {
  if (!ctx) return LNR_E_ARG;
  if (!path) return fail(ctx, LNR_E_ARG, "path is null");
  if (!ctx->cnn) return fail(ctx, LNR_E_ARG, "no network set");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const size_t np = (size_t)cnn_param_count();
  std::vector<float> host(3 * np);  // parameters, first and second moments
  const hipStream_t st = (hipStream_t)stream;
  LNR_HIP(hipMemcpyAsync(host.data(), ctx->cnn, 3 * np * sizeof(float), hipMemcpyDeviceToHost,
                         st));
  LNR_HIP(hipStreamSynchronize(st));
  FILE* f = fopen(path, "wb");
  if (!f) return fail(ctx, LNR_E_WEIGHTS, "cannot open the checkpoint file for writing");
  const uint32_t hdr[4] = {kCkptMagic, kCkptVersion, (uint32_t)np, (uint32_t)ctx->cnn_step};
  const bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
                  fwrite(&counter, sizeof(counter), 1, f) == 1 &&
                  fwrite(host.data(), sizeof(float), 3 * np, f) == 3 * np;
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return fail(ctx, LNR_E_WEIGHTS, "writing the checkpoint file failed");
  return LNR_OK;
}

lnr_status lnr_proposal_checkpoint_load(lnr_ctx* ctx, const char* path, uint64_t* counter,
                                        void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!path) return fail(ctx, LNR_E_ARG, "path is null");
  const size_t np = (size_t)cnn_param_count();
  std::vector<float> host(3 * np);
  uint32_t hdr[4] = {0u, 0u, 0u, 0u};
  uint64_t ctr = 0;
  {
    FILE* f = fopen(path, "rb");
    if (!f) return fail(ctx, LNR_E_WEIGHTS, "cannot open the checkpoint file");
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == kCkptMagic &&
              hdr[1] == kCkptVersion && hdr[2] == (uint32_t)np && hdr[3] <= 0x7fffffffu &&
              fread(&ctr, sizeof(ctr), 1, f) == 1 &&
              fread(host.data(), sizeof(float), 3 * np, f) == 3 * np;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the moments
    fclose(f);
    if (!ok) return fail(ctx, LNR_E_WEIGHTS, "not a checkpoint file of this version and size");
  }
  for (size_t i = 0; i < 3 * np; ++i)
    if (!std::isfinite(host[i]) || (i >= 2 * np && host[i] < 0.f))
      return fail(ctx, LNR_E_WEIGHTS, "non-finite checkpoint value or negative second moment");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  lnr_status s;
  if ((s = ensure_cnn(ctx)) != LNR_OK) return s;
  const hipStream_t st = (hipStream_t)stream;
  LNR_HIP(hipMemcpyAsync(ctx->cnn, host.data(), 3 * np * sizeof(float), hipMemcpyHostToDevice,
                         st));
  LNR_HIP(launch_cnn_pack(ctx->cnn, ctx->cnn_packed, st));
  LNR_HIP(hipStreamSynchronize(st));  // the host copy is freed on return
  ctx->cnn_step = (int)hdr[3];
  if (counter) *counter = ctr;
  return LNR_OK;
}

lnr_status lnr_proposal_inputs(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped,
                               int32_t w, int32_t h, uint16_t* x, void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!ref || !warped || !x || w < 32 || h < 32 || w > kMaxSide || h > kMaxSide)
    return fail(ctx, LNR_E_ARG, "bad proposal input arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(launch_cnn_input(ref, warped, w, h, w / 32, h / 32, nullptr, nullptr, x,
                           (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_proposal_forward(lnr_ctx* ctx, const uint16_t* x, int32_t n, float* out,
                                void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!x || !out || n < 0) return fail(ctx, LNR_E_ARG, "bad proposal forward arguments");
  if (!ctx->cnn) return fail(ctx, LNR_E_ARG, "no network set");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  LNR_HIP(launch_cnn_forward(ctx->cnn_packed, ctx->cnn, x, n, out, nullptr, nullptr, nullptr, 0,
                             0.f, (hipStream_t)stream));
  return LNR_OK;
}

lnr_status lnr_proposal_train_step(lnr_ctx* ctx, const uint16_t* x, const int32_t* labels,
                                   int32_t n, float lr, float wd, float* loss, float* grad,
                                   void* stream) {
  if (!ctx) return LNR_E_ARG;
  TraceGuard tg(ctx);
  if (!x || !labels || n < 1) return fail(ctx, LNR_E_ARG, "bad training arguments");
  if (!(lr >= 0.f) || !(wd >= 0.f)) return fail(ctx, LNR_E_ARG, "lr and wd must be >= 0");
  if (!ctx->cnn) return fail(ctx, LNR_E_ARG, "no network set");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  const hipStream_t st = (hipStream_t)stream;
  int pb = 0;
  const int nb = cnn_grad_blocks(n, &pb);
  const size_t np = (size_t)cnn_param_count();
  Plan pl;
  const size_t o_act = pl.take((size_t)n * cnn_act_elems() * sizeof(uint16_t));
  const size_t o_dz = pl.take((size_t)n * cnn_dz_elems() * sizeof(uint16_t));
  const size_t o_out = pl.take((size_t)n * 3 * sizeof(float));
  const size_t o_dO = pl.take((size_t)n * 3 * sizeof(float));
  const size_t o_part = pl.take((size_t)nb * np * sizeof(float));
  lnr_status s;
  if ((s = ensure_ws(ctx, pl.off, st)) != LNR_OK) return s;
  char* base = static_cast<char*>(ctx->ws);
  uint16_t* acts = reinterpret_cast<uint16_t*>(base + o_act);
  uint16_t* dzs = reinterpret_cast<uint16_t*>(base + o_dz);
  float* out = reinterpret_cast<float*>(base + o_out);
  float* dO = reinterpret_cast<float*>(base + o_dO);
  float* part = reinterpret_cast<float*>(base + o_part);
  LNR_HIP(launch_cnn_forward(ctx->cnn_packed, ctx->cnn, x, n, out, acts, nullptr, nullptr, 0,
                             0.f, st));
  LNR_HIP(launch_cnn_backward(ctx->cnn_packed, ctx->cnn, acts, out, labels, n, dO, loss, dzs,
                              part, st));
  const bool update = lr != 0.f || wd != 0.f;
  if (update) ++ctx->cnn_step;
  LNR_HIP(launch_cnn_adamw(part, nb, ctx->cnn, ctx->cnn + np, ctx->cnn + 2 * np, lr, wd,
                           update ? ctx->cnn_step : 1, grad, st));
  if (update) LNR_HIP(launch_cnn_pack(ctx->cnn, ctx->cnn_packed, st));
  return LNR_OK;
}

lnr_status lnr_trace_enable(lnr_ctx* ctx, int32_t on) {
  if (!ctx) return LNR_E_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipSetDevice");
  for (auto& r : ctx->tracer.recs) (void)hipEventSynchronize(r.b);
  ctx->tracer.reset();
  ctx->tracing = on != 0;
  return LNR_OK;
}

int32_t lnr_trace_read(lnr_ctx* ctx, lnr_trace_entry* out, int32_t max) {
  if (!ctx) return LNR_E_ARG;
  Tracer& t = ctx->tracer;
  std::vector<double> ms(t.names.size(), 0.0);
  std::vector<int> cnt(t.names.size(), 0);
  for (auto& r : t.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(ctx, LNR_E_HIP, "hipEventSynchronize");
    float e = 0.f;
    if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess)
      return fail(ctx, LNR_E_HIP, "hipEventElapsedTime");
    ms[r.slot] += e;
    cnt[r.slot] += 1;
  }
  const int n = (int)t.names.size();
  for (int i = 0; i < n && i < max && out; ++i) {
    memset(&out[i], 0, sizeof(out[i]));
    strncpy(out[i].name, t.names[i].c_str(), sizeof(out[i].name) - 1);
    out[i].count = cnt[i];
    out[i].ms_total = ms[i];
  }
  return n;
}

}  // extern "C"
