// C ABI of libclod: host-side validation, workspace carving and launch sequencing.
// Workspaces belong to the caller; only the persistent server allocates (its queue state).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "clod_internal.h"

// Workspace of clod_lod_count_noalloc: a library-owned array, one copy per GPU.  Host code never
// passes this name to a kernel or a copy (on the host it is only a stand-in for the symbol):
// it uses the device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[CLOD_LOD_SCRATCH_BYTES];

namespace clod {

static thread_local char g_err[512] = "";

static clod_status fail(clod_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

static clod_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(CLOD_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return CLOD_OK;
}

#define HIP_TRY(expr, what)                                   \
  do {                                                        \
    clod_status _st = hip_check((expr), (what));              \
    if (_st != CLOD_OK) return _st;                           \
  } while (0)

static_assert(sizeof(clod_view) == 112, "clod_view layout");

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool finite_f(float x) { return isfinite(x) != 0; }

// Radix passes of clod_bin_sort: 4 over the depth keys of the rendered records, then the
// tile-id passes over the pairs.
static int sort_passes(uint32_t tiles_total) { return 4 + tile_passes(tiles_total); }

int sort_blocks(int64_t cap) {
  int64_t g = (cap + kSortTile - 1) / kSortTile;
  if (g < 1) g = 1;
  if (g > kMaxSortBlocks) g = kMaxSortBlocks;
  return (int)g;
}

DupLayout dup_layout(int64_t cap) {
  DupLayout D;
  D.cap = cap;
  size_t o = 0;
  D.keys0 = o; o = align256(o + (size_t)cap * 4);
  D.vals0 = o; o = align256(o + (size_t)cap * 4);
  D.keys1 = o; o = align256(o + (size_t)cap * 4);
  D.vals1 = o; o = align256(o + (size_t)cap * 4);
  D.hist = o; o = align256(o + ((size_t)256 * sort_blocks(cap) + 256) * 4);
  D.owner = o; o = align256(o + ((size_t)(cap + kEmitTile - 1) / kEmitTile + 1) * 4);
  D.total = o;
  return D;
}

static clod_status host_views(int32_t V, const clod_view* vh, HostView* hv, uint32_t& tiles_total,
                              int64_t& pixels_total, uint32_t& loss_blocks) {
  uint64_t tb = 0, pb = 0, lb = 0;
  for (int v = 0; v < V; ++v) {
    const clod_view& c = vh[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
      return fail(CLOD_E_ARG, "view %d: width/height must be in 1..16384", v);
    HostView& h = hv[v];
    h.width = c.width;
    h.height = c.height;
    h.tiles_x = (c.width + kTile - 1) / kTile;
    h.tiles_y = (c.height + kTile - 1) / kTile;
    h.tile_base = (uint32_t)tb;
    h.pix_base = (uint32_t)pb;
    h.loss_block_base = (uint32_t)lb;
    h.loss_blocks = (uint32_t)((3ull * c.width * c.height + kLossChunk - 1) / kLossChunk);
    tb += (uint64_t)h.tiles_x * h.tiles_y;
    pb += (uint64_t)c.width * c.height;
    lb += h.loss_blocks;
    if (tb >= 0xFFFFFFFFull || pb >= 0xFFFFFFFFull) return fail(CLOD_E_ARG, "batch too large (tiles or pixels exceed 2^32)");
  }
  tiles_total = (uint32_t)tb;
  pixels_total = (int64_t)pb;
  loss_blocks = (uint32_t)lb;
  return CLOD_OK;
}

static Layout make_layout(int64_t n, int32_t V, uint32_t tiles_total, int64_t pixels_total, bool any_budget) {
  Layout L;
  L.any_budget = any_budget;
  L.n = n;
  L.V = V;
  L.VN = n * (int64_t)V;
  L.tiles_total = tiles_total;
  L.pixels_total = pixels_total;
  L.scan_blocks = (int32_t)((L.VN + kScanChunk - 1) / kScanChunk);
  size_t o = 0;
  L.hdr = o; o = align256(o + kHdrWords * 8);
  L.vinfo = o; o = align256(o + (size_t)V * sizeof(DevView));
  L.dmax_key = o; o = align256(o + (size_t)V * 8);
  L.counts = o; o = align256(o + (size_t)V * 3 * 8);
  L.gdmax = o; o = align256(o + (size_t)V * 4);
  L.loss_acc = o; o = align256(o + (size_t)V * 4);
  L.ssim_acc = o; o = align256(o + (size_t)V * 4);
  L.loss_part = o; o = align256(o + ((size_t)tiles_total * 3 + (size_t)pixels_total * 3 / kLossChunk + V) * 4);
  L.kpart = o; o = align256(o + (size_t)kMaxProjBlocks * V * 8);
  L.cpart = o; o = align256(o + (size_t)kMaxProjBlocks * V * 4 * 4);
  L.gpart = o; o = align256(o + (size_t)kMaxProjBlocks * V * 4);
  L.sel_state = o; o = align256(o + (size_t)V * sizeof(SelState));
  L.sel_hist = o; o = align256(o + (L.any_budget ? (size_t)V * kSelBlocks * 256 * 4 : 0));
  L.lcount = o; o = align256(o + (size_t)kMaxProjBlocks * 4);   // work-list segment counts
  L.list = o; o = align256(o + (size_t)n * 4);                        // work list of the projection
  L.flags = o; o = align256(o + (size_t)L.VN);
  L.alpha = o; o = align256(o + (size_t)L.VN * 4);
  L.rec = o; o = align256(o + (size_t)L.VN * kRecBytes);
  L.scan_part = o; o = align256(o + ((size_t)L.scan_blocks + 1) * 4 * 2);   // records, emission
  L.ranges = o; o = align256(o + (size_t)tiles_total * 8);
  L.order = o; o = align256(o + (size_t)tiles_total * 4);
  L.tord = o; o = align256(o + (size_t)kTileOrderWords * 4);
  L.pair_part = o; o = align256(o + (size_t)tiles_total * 3 * 8);
  L.gscreen = o; o = align256(o + (size_t)L.VN * kGscreen * 4);
  L.total = o;
  return L;
}

static clod_status check_params(const clod_params& p) {
  if (!(finite_f(p.tau) && p.tau >= 0.f)) return fail(CLOD_E_ARG, "params.tau must be finite and >= 0");
  if (!(finite_f(p.eps) && p.eps > 0.f)) return fail(CLOD_E_ARG, "params.eps must be finite and > 0");
  if (!(finite_f(p.near_z) && p.near_z > 0.f)) return fail(CLOD_E_ARG, "params.near_z must be finite and > 0");
  if (!(finite_f(p.guard) && p.guard > 0.f)) return fail(CLOD_E_ARG, "params.guard must be finite and > 0");
  if (!(finite_f(p.dilation) && p.dilation >= 0.f)) return fail(CLOD_E_ARG, "params.dilation must be finite and >= 0");
  for (int j = 0; j < 3; ++j)
    if (!finite_f(p.bg[j])) return fail(CLOD_E_ARG, "params.bg must be finite");
  return CLOD_OK;
}

static clod_status check_view(const clod_view& c, int v) {
  for (int j = 0; j < 9; ++j)
    if (!finite_f(c.W[j])) return fail(CLOD_E_ARG, "view %d: W not finite", v);
  for (int j = 0; j < 3; ++j)
    if (!finite_f(c.t[j]) || !finite_f(c.c[j])) return fail(CLOD_E_ARG, "view %d: t or c not finite", v);
  if (!(finite_f(c.fx) && c.fx > 0.f && finite_f(c.fy) && c.fy > 0.f && finite_f(c.cx) && finite_f(c.cy)))
    return fail(CLOD_E_ARG, "view %d: intrinsics must be finite with fx, fy > 0", v);
  if (!(finite_f(c.s_v) && c.s_v >= 1.0f)) return fail(CLOD_E_ARG, "view %d: s_v must be finite and >= 1", v);
  if (c.budget < 0) return fail(CLOD_E_ARG, "view %d: budget must be >= 0", v);
  if (c.frame_width != 0 || c.frame_height != 0) {
    if (c.frame_width < 1 || c.frame_height < 1 || c.frame_width > 16384 || c.frame_height > 16384)
      return fail(CLOD_E_ARG, "view %d: frame size must be in 1..16384", v);
    if (c.vx < 0 || c.vy < 0 || (c.vx & 15) || (c.vy & 15))
      return fail(CLOD_E_ARG, "view %d: viewport origin must be non-negative multiples of 16", v);
    if ((int64_t)c.vx + c.width > c.frame_width || (int64_t)c.vy + c.height > c.frame_height)
      return fail(CLOD_E_ARG, "view %d: viewport exceeds the frame", v);
  } else if (c.vx != 0 || c.vy != 0) {
    return fail(CLOD_E_ARG, "view %d: a viewport origin needs a frame size", v);
  }
  double scale = 1.0;
  for (int j = 0; j < 3; ++j) scale = fmax(scale, fabs((double)c.c[j]));
  for (int j = 0; j < 3; ++j) {
    const double cj = -((double)c.W[j] * c.t[0] + (double)c.W[3 + j] * c.t[1] + (double)c.W[6 + j] * c.t[2]);
    if (fabs(cj - (double)c.c[j]) > 1e-4 * scale)
      return fail(CLOD_E_ARG, "view %d: camera centre c differs from -W^T t", v);
  }
  return CLOD_OK;
}

struct Ctx {
  Layout L;
  HostView hv[CLOD_MAX_VIEWS];
  uint32_t loss_blocks = 0;
};

static clod_status prepare(const clod_batch* b, bool need_full_ws, Ctx& cx) {
  if (!b) return fail(CLOD_E_ARG, "batch is NULL");
  if (b->n_views < 1 || b->n_views > CLOD_MAX_VIEWS) return fail(CLOD_E_ARG, "n_views must be in 1..%d", CLOD_MAX_VIEWS);
  if (!b->views_host || !b->views_dev) return fail(CLOD_E_ARG, "views_host and views_dev must be non-NULL");
  if (!b->ws) return fail(CLOD_E_ARG, "ws is NULL");
  if (((uintptr_t)b->ws & 255) != 0) return fail(CLOD_E_ARG, "ws must be 256-byte aligned");
  clod_status st = check_params(b->params);
  if (st != CLOD_OK) return st;
  for (int v = 0; v < b->n_views; ++v) {
    st = check_view(b->views_host[v], v);
    if (st != CLOD_OK) return st;
  }
  uint32_t tiles_total;
  int64_t pixels_total;
  st = host_views(b->n_views, b->views_host, cx.hv, tiles_total, pixels_total, cx.loss_blocks);
  if (st != CLOD_OK) return st;
  const int64_t n = b->n;
  if (n < 0) return fail(CLOD_E_ARG, "batch->n must be >= 0");
  if (n * (int64_t)b->n_views >= 0xFFFFFFFFll) return fail(CLOD_E_ARG, "n * n_views must be < 2^32");
  bool any_budget = false;
  for (int v = 0; v < b->n_views; ++v) any_budget = any_budget || b->views_host[v].budget > 0;
  cx.L = make_layout(n, b->n_views, tiles_total, pixels_total, any_budget);
  for (int v = 0; v < b->n_views; ++v)
    cx.L.ssim_regions += (uint32_t)(((cx.hv[v].tiles_x + 1) / 2) * ((cx.hv[v].tiles_y + 1) / 2));
  // The per-view area and the projection work list precede the per-(view, Gaussian) planes.
  const size_t need = need_full_ws ? cx.L.total : cx.L.flags;
  if (b->ws_bytes < need) return fail(CLOD_E_ARG, "ws_bytes %zu < required %zu", b->ws_bytes, need);
  return CLOD_OK;
}

static clod_status check_scene(const clod_scene* s) {
  if (!s) return fail(CLOD_E_ARG, "scene is NULL");
  if (s->n < 0) return fail(CLOD_E_ARG, "scene.n must be >= 0");
  if (s->sh_degree < 0 || s->sh_degree > 3) return fail(CLOD_E_ARG, "scene.sh_degree must be in 0..3");
  if (s->n > 0 && (!s->mean || !s->log_scale || !s->quat || !s->opacity || !s->decay || !s->sh))
    return fail(CLOD_E_ARG, "scene planes must be non-NULL");
  return CLOD_OK;
}

// Count-only workspace: the sections the LoD counting kernels use, nothing per tile or pixel.
struct CountLayout {
  size_t vinfo, dmax_key, counts, kpart, cpart, sel_state, sel_hist, lcount, list, total;
};

static CountLayout count_layout(int64_t n, int32_t V, bool any_budget) {
  CountLayout C;
  size_t o = 0;
  C.vinfo = o; o = align256(o + (size_t)V * sizeof(DevView));
  C.dmax_key = o; o = align256(o + (size_t)V * 8);
  C.counts = o; o = align256(o + (size_t)V * 3 * 8);
  C.kpart = o; o = align256(o + (size_t)kMaxProjBlocks * V * 8);
  C.cpart = o; o = align256(o + (size_t)kMaxProjBlocks * V * 4 * 4);
  C.sel_state = o; o = align256(o + (size_t)V * sizeof(SelState));
  C.sel_hist = o; o = align256(o + (any_budget ? (size_t)V * kSelBlocks * 256 * 4 : 0));
  C.lcount = o; o = align256(o + (size_t)kMaxProjBlocks * 4);
  C.list = o; o = align256(o + (size_t)n * 4);
  C.total = o;
  return C;
}

// Device address of `scratch` on the device that runs `stream` (the current device for the
// null stream), looked up once per device with that device current and kept.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

static clod_status scratch_address(hipStream_t s, void** out) {
  int dev = 0, cur = 0;
  HIP_TRY(hipGetDevice(&cur), "current device");
  dev = cur;
  if (s) HIP_TRY(hipStreamGetDevice(s, &dev), "stream device");
  if (dev < 0 || dev >= kMaxDevices) return fail(CLOD_E_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    if (dev != cur) HIP_TRY(hipSetDevice(dev), "select the stream's device");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) HIP_TRY(hipSetDevice(cur), "restore the current device");
    HIP_TRY(e, "scratch address");
    if (!p) return fail(CLOD_E_HIP, "scratch address is NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return CLOD_OK;
}

static clod_status dup_check(const clod_batch* b, DupLayout& D) {
  if (!b->dup) return fail(CLOD_E_ARG, "dup is NULL");
  if (((uintptr_t)b->dup & 255) != 0) return fail(CLOD_E_ARG, "dup must be 256-byte aligned");
  const int64_t cap = clod_dup_capacity(b->dup_bytes);
  if (cap < 1) return fail(CLOD_E_ARG, "dup_bytes too small");
  D = dup_layout(cap);
  return CLOD_OK;
}

// The stage sequences of the forward path, shared by the per-stage entry points (a Sink on
// the caller's stream) and the persistent server (a Sink that records a Program).
static hipError_t project_stages(const clod_scene& sc, const clod_view* views_dev, const clod_params& prm,
                                 const Layout& L, void* ws, int64_t* counts_dev, float* eta_dev, const Sink& out) {
  char* w = (char*)ws;
  DevView* vinfo = (DevView*)(w + L.vinfo);
  unsigned long long* dmax_key = (unsigned long long*)(w + L.dmax_key);
  hipError_t e = launch_view_setup(views_dev, L.V, prm, vinfo, (unsigned long long*)(w + L.hdr), out);
  if (e == hipSuccess)
    e = launch_frustum_max(sc, vinfo, L.V, prm.near_z, (unsigned long long*)(w + L.kpart), dmax_key, out);
  if (e == hipSuccess && L.any_budget)
    e = launch_lod_select(sc, vinfo, L.V, prm, dmax_key, (SelState*)(w + L.sel_state), (uint32_t*)(w + L.sel_hist),
                          out);
  if (e == hipSuccess)
    e = launch_project(sc, vinfo, L.V, prm, dmax_key, (uint32_t*)(w + L.cpart), (unsigned long long*)(w + L.counts),
                       counts_dev, eta_dev, (uint8_t*)(w + L.flags), (float*)(w + L.alpha), (float4*)(w + L.rec),
                       (uint32_t*)(w + L.list), (uint32_t*)(w + L.lcount), out);
  return e;
}

static hipError_t bin_stages(const Layout& L, void* ws, const DupLayout& D, void* dup, const Sink& out) {
  hipError_t e = launch_bin_sort(L, ws, D, dup, out);
  if (e == hipSuccess) e = launch_ranges(L, ws, D, dup, sorted_buffer(L.tiles_total), out);
  return e;
}

static const uint32_t* sorted_vals(const clod_batch* b, const Layout& L, const DupLayout& D) {
  return (const uint32_t*)((const char*)b->dup + (sorted_buffer(L.tiles_total) ? D.vals1 : D.vals0));
}

static BlendBufs blend_bufs(const clod_batch* b, const Layout& L, const DupLayout& D) {
  const bool odd = sorted_buffer(L.tiles_total) != 0;
  char* dp = (char*)b->dup;
  const size_t k = odd ? D.keys0 : D.keys1, v = odd ? D.vals0 : D.vals1;   // adjacent: keys, then values
  return BlendBufs{sorted_vals(b, L, D), (unsigned long long*)(dp + k), v + (size_t)D.cap * 4 - k, D.cap};
}

}  // namespace clod

using namespace clod;

extern "C" {

int32_t clod_abi_version(void) { return CLOD_ABI_VERSION; }

const char* clod_last_error(void) { return g_err; }

size_t clod_ws_bytes(int64_t n, int32_t n_views, const clod_view* views_host) {
  if (n < 0 || n_views < 1 || n_views > CLOD_MAX_VIEWS || !views_host) return 0;
  HostView hv[CLOD_MAX_VIEWS];
  uint32_t tiles_total, lb;
  int64_t pixels_total;
  if (host_views(n_views, views_host, hv, tiles_total, pixels_total, lb) != CLOD_OK) return 0;
  bool any_budget = false;
  for (int v = 0; v < n_views; ++v) any_budget = any_budget || views_host[v].budget > 0;
  return make_layout(n, n_views, tiles_total, pixels_total, any_budget).total;
}

size_t clod_dup_bytes(int64_t capacity) {
  if (capacity < 1) capacity = 1;
  return dup_layout(capacity).total;
}

int64_t clod_dup_capacity(size_t dup_bytes) {
  // Largest capacity whose layout fits; the layout grows by 16 bytes per entry.
  int64_t lo = 0, hi = (int64_t)(dup_bytes / 16) + 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (mid >= 0xFFFFFFFFll || dup_layout(mid).total > dup_bytes) hi = mid - 1; else lo = mid;
  }
  return lo;
}

clod_status clod_project(const clod_scene* scene, const clod_batch* batch, int64_t* counts_dev,
                         float* eta_dev, void* stream) {
  g_err[0] = 0;
  clod_status st = check_scene(scene);
  if (st != CLOD_OK) return st;
  Ctx cx;
  st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  if (scene->n != batch->n) return fail(CLOD_E_ARG, "scene->n (%lld) != batch->n (%lld)", (long long)scene->n, (long long)batch->n);
  HIP_TRY(project_stages(*scene, batch->views_dev, batch->params, cx.L, batch->ws, counts_dev, eta_dev,
                         Sink((hipStream_t)stream)),
          "project");
  return CLOD_OK;
}

clod_status clod_bin_sort(const clod_batch* batch, int64_t* n_dup_host, void* stream) {
  g_err[0] = 0;
  Ctx cx;
  clod_status st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  DupLayout D;
  st = dup_check(batch, D);
  if (st != CLOD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const Layout& L = cx.L;
  char* w = (char*)batch->ws;
  HIP_TRY(bin_stages(L, batch->ws, D, batch->dup, Sink(s)), "binning sort");
  if (n_dup_host) {
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, w + L.hdr, sizeof(h), hipMemcpyDeviceToHost, s), "read count");
    HIP_TRY(hipStreamSynchronize(s), "synchronise");
    *n_dup_host = (int64_t)h[0];
    if (h[1]) return fail(CLOD_E_CAPACITY, "%lld tile pairs exceed the duplicate capacity %lld",
                          (long long)h[0], (long long)D.cap);
  }
  return CLOD_OK;
}

clod_status clod_render_fwd(const clod_batch* batch, float* rgb, float* T, uint32_t* last,
                            int64_t* pairs_dev, void* stream) {
  g_err[0] = 0;
  Ctx cx;
  clod_status st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  DupLayout D;
  st = dup_check(batch, D);
  if (st != CLOD_OK) return st;
  if (!rgb || !T || !last) return fail(CLOD_E_ARG, "rgb, T and last must be non-NULL");
  HIP_TRY(launch_blend_fwd(cx.L, batch->ws, blend_bufs(batch, cx.L, D), batch->params, rgb, T, last, pairs_dev,
                           Sink((hipStream_t)stream)),
          "blend forward");
  return CLOD_OK;
}

clod_status clod_render_bwd(const clod_scene* scene, const clod_batch* batch, const float* T,
                            const uint32_t* last, const float* dL_drgb, const float* dL_deta,
                            int32_t accumulate, const clod_scene_grad* grad, int64_t* pairs_dev, void* stream) {
  g_err[0] = 0;
  clod_status st = check_scene(scene);
  if (st != CLOD_OK) return st;
  Ctx cx;
  st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  if (scene->n != batch->n) return fail(CLOD_E_ARG, "scene->n != batch->n");
  DupLayout D;
  st = dup_check(batch, D);
  if (st != CLOD_OK) return st;
  if (!T || !last || !dL_drgb) return fail(CLOD_E_ARG, "T, last and dL_drgb must be non-NULL");
  if (!grad || (scene->n > 0 && (!grad->mean || !grad->log_scale || !grad->quat || !grad->opacity ||
                                 !grad->decay || !grad->sh)))
    return fail(CLOD_E_ARG, "gradient planes must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  const Layout& L = cx.L;
  char* w = (char*)batch->ws;
  HIP_TRY(launch_clear_rendered(L, batch->ws, s), "clear gscreen");
  HIP_TRY(launch_blend_bwd(L, batch->ws, sorted_vals(batch, L, D), batch->params, T, last, dL_drgb, pairs_dev, s),
          "blend backward");
  HIP_TRY(launch_gauss_bwd(*scene, L, batch->ws, batch->params, dL_deta, accumulate, *grad, s),
          "gaussian backward");
  return CLOD_OK;
}

clod_status clod_lod_count(const clod_scene* scene, const clod_batch* batch, int64_t* counts_dev,
                           void* stream) {
  g_err[0] = 0;
  clod_status st = check_scene(scene);
  if (st != CLOD_OK) return st;
  Ctx cx;
  st = prepare(batch, false, cx);
  if (st != CLOD_OK) return st;
  if (!counts_dev) return fail(CLOD_E_ARG, "counts_dev must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  const Layout& L = cx.L;
  char* w = (char*)batch->ws;
  DevView* vinfo = (DevView*)(w + L.vinfo);
  HIP_TRY(launch_view_setup(batch->views_dev, L.V, batch->params, vinfo, nullptr, s), "view setup");
  HIP_TRY(launch_frustum_max(*scene, vinfo, L.V, batch->params.near_z, (unsigned long long*)(w + L.kpart),
                             (unsigned long long*)(w + L.dmax_key), s),
          "frustum max");
  if (L.any_budget)
    HIP_TRY(launch_lod_select(*scene, vinfo, L.V, batch->params, (const unsigned long long*)(w + L.dmax_key),
                              (SelState*)(w + L.sel_state), (uint32_t*)(w + L.sel_hist), s),
            "budget select");
  HIP_TRY(launch_lod_count(*scene, vinfo, L.V, batch->params, (unsigned long long*)(w + L.dmax_key),
                           (uint32_t*)(w + L.cpart), (unsigned long long*)(w + L.counts), counts_dev, nullptr,
                           (uint32_t*)(w + L.list), (uint32_t*)(w + L.lcount), s),
          "lod count");
  return CLOD_OK;
}

clod_status clod_lod_count_noalloc(const clod_scene* scene, int32_t n_views, const clod_view* views_host,
                                   const clod_view* views_dev, const clod_params* params, int64_t* counts_dev,
                                   void* stream) {
  g_err[0] = 0;
  clod_status st = check_scene(scene);
  if (st != CLOD_OK) return st;
  if (n_views < 1 || n_views > CLOD_MAX_VIEWS) return fail(CLOD_E_ARG, "n_views must be in 1..%d", CLOD_MAX_VIEWS);
  if (!views_host || !views_dev || !params || !counts_dev)
    return fail(CLOD_E_ARG, "views_host, views_dev, params and counts_dev must be non-NULL");
  st = check_params(*params);
  if (st != CLOD_OK) return st;
  bool any_budget = false;
  for (int v = 0; v < n_views; ++v) {
    st = check_view(views_host[v], v);
    if (st != CLOD_OK) return st;
    any_budget = any_budget || views_host[v].budget > 0;
  }
  if (scene->n * (int64_t)n_views >= 0xFFFFFFFFll) return fail(CLOD_E_ARG, "n * n_views must be < 2^32");
  const CountLayout Cl = count_layout(scene->n, n_views, any_budget);
  if (Cl.total > (size_t)CLOD_LOD_SCRATCH_BYTES)
    return fail(CLOD_E_ARG, "%lld Gaussians and %d views need %zu bytes of workspace, more than the %u-byte "
                "library scratch of clod_lod_count_noalloc (use clod_lod_count with a workspace)",
                (long long)scene->n, n_views, Cl.total, (unsigned)CLOD_LOD_SCRATCH_BYTES);
  hipStream_t s = (hipStream_t)stream;
  void* base = nullptr;
  st = scratch_address(s, &base);
  if (st != CLOD_OK) return st;
  char* w = (char*)base;
  DevView* vinfo = (DevView*)(w + Cl.vinfo);
  HIP_TRY(launch_view_setup(views_dev, n_views, *params, vinfo, nullptr, s), "view setup");
  HIP_TRY(launch_frustum_max(*scene, vinfo, n_views, params->near_z, (unsigned long long*)(w + Cl.kpart),
                             (unsigned long long*)(w + Cl.dmax_key), s),
          "frustum max");
  if (any_budget)
    HIP_TRY(launch_lod_select(*scene, vinfo, n_views, *params, (const unsigned long long*)(w + Cl.dmax_key),
                              (SelState*)(w + Cl.sel_state), (uint32_t*)(w + Cl.sel_hist), s),
            "budget select");
  HIP_TRY(launch_lod_count(*scene, vinfo, n_views, *params, (unsigned long long*)(w + Cl.dmax_key),
                           (uint32_t*)(w + Cl.cpart), (unsigned long long*)(w + Cl.counts), counts_dev, nullptr,
                           (uint32_t*)(w + Cl.list), (uint32_t*)(w + Cl.lcount), s),
          "lod count");
  return CLOD_OK;
}

// Scene preparation: the workspace of clod_scene_reorder and the call.
struct OrderLayout {
  size_t box, hdr, hist, keys0, keys1, vals1, total;
  int G;
};
static OrderLayout order_layout(int64_t n) {
  OrderLayout O;
  size_t o = 0;
  O.G = sort_blocks(n);
  O.box = o; o = align256(o + 6 * 4);
  O.hdr = o; o = align256(o + (size_t)kHdrWords * 8);
  O.hist = o; o = align256(o + ((size_t)256 * O.G + 256) * 4);
  O.keys0 = o; o = align256(o + (size_t)n * 4);
  O.keys1 = o; o = align256(o + (size_t)n * 4);
  O.vals1 = o; o = align256(o + (size_t)n * 4);
  O.total = o;
  return O;
}

size_t clod_scene_reorder_ws_bytes(int64_t n) {
  if (n < 0 || n > (int64_t)INT32_MAX) return 0;
  return order_layout(n).total;
}

clod_status clod_scene_reorder(const clod_scene* src, const clod_scene_grad* dst, uint32_t* perm, void* ws,
                               size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  clod_status st = check_scene(src);
  if (st != CLOD_OK) return st;
  if (src->n > (int64_t)INT32_MAX) return fail(CLOD_E_ARG, "scene.n must be <= 2^31 - 1");
  if (!dst || !perm) return fail(CLOD_E_ARG, "dst and perm must be non-NULL");
  if (src->n == 0) return CLOD_OK;
  const int64_t n = src->n;
  const int K = (src->sh_degree + 1) * (src->sh_degree + 1);
  const float* sp[6] = {src->mean, src->log_scale, src->quat, src->opacity, src->decay, src->sh};
  float* dp[6] = {dst->mean, dst->log_scale, dst->quat, dst->opacity, dst->decay, dst->sh};
  const int64_t planes[6] = {3, 3, 4, 1, 1, 3 * (int64_t)K};
  for (int i = 0; i < 6; ++i)
    if (!dp[i]) return fail(CLOD_E_ARG, "dst planes must be non-NULL");
  // No destination array may overlap a source array.
  for (int i = 0; i < 6; ++i) {
    const uintptr_t d0 = (uintptr_t)dp[i], d1 = d0 + (uintptr_t)(planes[i] * n * 4);
    for (int j = 0; j < 6; ++j) {
      const uintptr_t s0 = (uintptr_t)sp[j], s1 = s0 + (uintptr_t)(planes[j] * n * 4);
      if (d0 < s1 && s0 < d1) return fail(CLOD_E_ARG, "dst planes must not overlap src planes");
    }
  }
  const OrderLayout O = order_layout(n);
  if (!ws) return fail(CLOD_E_ARG, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(CLOD_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < O.total) return fail(CLOD_E_ARG, "workspace_bytes %zu < required %zu", ws_bytes, O.total);
  char* w = (char*)ws;
  OrderBufs ob{(uint32_t*)(w + O.box), (unsigned long long*)(w + O.hdr), (uint32_t*)(w + O.hist),
               {(uint32_t*)(w + O.keys0), (uint32_t*)(w + O.keys1)}, {perm, (uint32_t*)(w + O.vals1)}, O.G};
  HIP_TRY(launch_scene_reorder(*src, *dst, ob, (hipStream_t)stream), "scene reorder");
  return CLOD_OK;
}

clod_status clod_loss(const clod_batch* batch, const float* rgb, const float* target, float s_max,
                      float lambda_reg, float lambda_dssim, float* ssim_scratch, size_t ssim_scratch_bytes,
                      float* loss_dev, float* dL_drgb, float* dL_deta_dev, void* stream) {
  g_err[0] = 0;
  Ctx cx;
  clod_status st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  if (!rgb || !target || !loss_dev || !dL_drgb) return fail(CLOD_E_ARG, "rgb, target, loss and dL_drgb must be non-NULL");
  if (!(finite_f(s_max) && s_max >= 1.0f)) return fail(CLOD_E_ARG, "s_max must be finite and >= 1");
  if (!(finite_f(lambda_reg) && lambda_reg >= 0.0f)) return fail(CLOD_E_ARG, "lambda_reg must be finite and >= 0");
  if (!(lambda_dssim >= 0.0f && lambda_dssim <= 1.0f)) return fail(CLOD_E_ARG, "lambda_dssim must be in [0, 1]");
  if (lambda_dssim > 0.0f) {
    if (!ssim_scratch) return fail(CLOD_E_ARG, "ssim_scratch must be non-NULL when lambda_dssim > 0");
    if (ssim_scratch_bytes < (size_t)cx.L.pixels_total * 36)
      return fail(CLOD_E_ARG, "ssim_scratch_bytes %zu < 36 * pixels = %zu", ssim_scratch_bytes,
                  (size_t)cx.L.pixels_total * 36);
  }
  for (int v = 0; v < batch->n_views; ++v)
    if (batch->views_host[v].s_v > s_max) return fail(CLOD_E_ARG, "view %d: s_v exceeds s_max", v);
  HIP_TRY(launch_loss(cx.L, batch->ws, batch->n, rgb, target, s_max, lambda_reg, lambda_dssim, ssim_scratch,
                      loss_dev, dL_drgb, dL_deta_dev, cx.loss_blocks, (hipStream_t)stream),
          "loss");
  return CLOD_OK;
}

clod_status clod_adam_step(int64_t n, int32_t sh_degree, const clod_scene_grad* param,
                           const clod_scene_grad* grad, const clod_scene_grad* m,
                           const clod_scene_grad* v, const clod_adam* hp, void* stream) {
  g_err[0] = 0;
  if (n < 0) return fail(CLOD_E_ARG, "n must be >= 0");
  if (sh_degree < 0 || sh_degree > 3) return fail(CLOD_E_ARG, "sh_degree must be in 0..3");
  if (!param || !grad || !m || !v || !hp) return fail(CLOD_E_ARG, "param, grad, m, v and hp must be non-NULL");
  for (int j = 0; j < kAdamGroups; ++j)
    if (!(finite_f(hp->lr[j]) && hp->lr[j] >= 0.f)) return fail(CLOD_E_ARG, "hp->lr[%d] must be finite and >= 0", j);
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f && hp->beta2 >= 0.f && hp->beta2 < 1.f))
    return fail(CLOD_E_ARG, "betas must be in [0, 1)");
  if (!(finite_f(hp->eps) && hp->eps > 0.f)) return fail(CLOD_E_ARG, "eps must be finite and > 0");
  if (hp->step < 1) return fail(CLOD_E_ARG, "hp->step must be >= 1");
  // Bias corrections 1 - beta^t of Adam, in double from the binary32 betas, rounded once.
  const float bias1 = (float)(1.0 - pow((double)hp->beta1, (double)hp->step));
  const float bias2 = (float)(1.0 - pow((double)hp->beta2, (double)hp->step));
  if (!(bias1 > 0.f && bias2 > 0.f)) return fail(CLOD_E_ARG, "bias corrections must be > 0");
  if (n == 0) return CLOD_OK;
  const clod_scene_grad* planes[4] = {param, grad, m, v};
  for (const clod_scene_grad* q : planes)
    if (!q->mean || !q->log_scale || !q->quat || !q->opacity || !q->decay || !q->sh)
      return fail(CLOD_E_ARG, "every parameter plane must be non-NULL");
  const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
  AdamSegs S;
  auto seg = [&](int j, float* (clod_scene_grad::*f), int64_t off, int64_t count) {
    S.s[j].p = param->*f + off;
    S.s[j].g = grad->*f + off;
    S.s[j].m = m->*f + off;
    S.s[j].v = v->*f + off;
    S.s[j].count = count;
    S.s[j].lr = hp->lr[j];
  };
  seg(0, &clod_scene_grad::mean, 0, 3 * n);
  seg(1, &clod_scene_grad::log_scale, 0, 3 * n);
  seg(2, &clod_scene_grad::quat, 0, 4 * n);
  seg(3, &clod_scene_grad::opacity, 0, n);
  seg(4, &clod_scene_grad::decay, 0, n);
  seg(5, &clod_scene_grad::sh, 0, 3 * n);
  seg(6, &clod_scene_grad::sh, 3 * n, 3 * (K - 1) * n);
  HIP_TRY(launch_adam(S, hp->beta1, hp->beta2, hp->eps, bias1, bias2, (hipStream_t)stream), "adam");
  return CLOD_OK;
}

clod_status clod_read_info(const clod_batch* batch, int64_t* info_host, void* stream) {
  g_err[0] = 0;
  Ctx cx;
  clod_status st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  if (!info_host) return fail(CLOD_E_ARG, "info_host is NULL");
  unsigned long long h[2];
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(h, (const char*)batch->ws + cx.L.hdr, sizeof(h), hipMemcpyDeviceToHost, s), "read header");
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  info_host[0] = (int64_t)h[0];
  info_host[1] = (int64_t)h[1];
  info_host[2] = batch->dup ? clod_dup_capacity(batch->dup_bytes) : 0;
  info_host[3] = sort_passes(cx.L.tiles_total);
  return CLOD_OK;
}

clod_status clod_inspect(const clod_batch* batch, int32_t section, const void** dev_ptr,
                         int64_t* count) {
  g_err[0] = 0;
  Ctx cx;
  clod_status st = prepare(batch, true, cx);
  if (st != CLOD_OK) return st;
  if (!dev_ptr || !count) return fail(CLOD_E_ARG, "dev_ptr and count must be non-NULL");
  const Layout& L = cx.L;
  const char* w = (const char*)batch->ws;
  if (section == CLOD_SEC_KEYS || section == CLOD_SEC_VALUES) {
    DupLayout D;
    st = dup_check(batch, D);
    if (st != CLOD_OK) return st;
    const bool odd = sorted_buffer(L.tiles_total) != 0;
    const size_t off = section == CLOD_SEC_KEYS ? (odd ? D.keys1 : D.keys0) : (odd ? D.vals1 : D.vals0);
    *dev_ptr = (const char*)batch->dup + off;
    *count = D.cap;
    return CLOD_OK;
  }
  switch (section) {
    case CLOD_SEC_RANGES: *dev_ptr = w + L.ranges; *count = L.tiles_total; break;
    case CLOD_SEC_REC: *dev_ptr = w + L.rec; *count = L.VN; break;
    case CLOD_SEC_ALPHA: *dev_ptr = w + L.alpha; *count = L.VN; break;
    case CLOD_SEC_FLAGS: *dev_ptr = w + L.flags; *count = L.VN; break;
    case CLOD_SEC_DMAX: *dev_ptr = w + L.dmax_key; *count = L.V; break;
    case CLOD_SEC_GSCREEN: *dev_ptr = w + L.gscreen; *count = L.VN; break;
    case CLOD_SEC_HEADER: *dev_ptr = w + L.hdr; *count = 2; break;
    default: return fail(CLOD_E_ARG, "unknown section %d", section);
  }
  return CLOD_OK;
}

// ---------------------------------------------------------------------------- persistent server
clod_status clod_server_start(int32_t workers, double max_seconds, void* stream, clod_server** server,
                              int32_t* workers_used) {
  g_err[0] = 0;
  if (!server) return fail(CLOD_E_ARG, "server is NULL");
  *server = nullptr;
  if (workers < 0) return fail(CLOD_E_ARG, "workers must be >= 0");
  if (!(max_seconds > 0.0 && max_seconds <= 3600.0)) return fail(CLOD_E_ARG, "max_seconds must be in (0, 3600]");
  Server* S = nullptr;
  HIP_TRY(server_start(workers, max_seconds, (hipStream_t)stream, &S, workers_used), "server start");
  *server = reinterpret_cast<clod_server*>(S);
  return CLOD_OK;
}

clod_status clod_server_submit(clod_server* server, const clod_scene* scene, const clod_batch* batch, float* rgb,
                               float* T, uint32_t* last, int64_t* seq) {
  g_err[0] = 0;
  if (!server || !seq) return fail(CLOD_E_ARG, "server and seq must be non-NULL");
  Server* S = reinterpret_cast<Server*>(server);
  clod_status st = check_scene(scene);
  if (st != CLOD_OK) return st;
  if (scene->n > 0 && !scene->sh_packed)
    return fail(CLOD_E_ARG, "the server reads packed SH coefficients: scene->sh_packed must be set");
  if (!batch) return fail(CLOD_E_ARG, "batch is NULL");
  if (batch->n_views < 1 || batch->n_views > kSrvMaxViews)
    return fail(CLOD_E_ARG, "n_views must be in 1..%d for the server", kSrvMaxViews);
  // The server keeps its own device copy of the views; batch->views_dev is not read.
  clod_batch b = *batch;
  b.views_dev = server_views_dev(S, server_next_seq(S));
  Ctx cx;
  st = prepare(&b, true, cx);
  if (st != CLOD_OK) return st;
  if (scene->n != b.n) return fail(CLOD_E_ARG, "scene->n (%lld) != batch->n (%lld)", (long long)scene->n, (long long)b.n);
  DupLayout D;
  st = dup_check(&b, D);
  if (st != CLOD_OK) return st;
  if (!rgb || !T || !last) return fail(CLOD_E_ARG, "rgb, T and last must be non-NULL");
  if (!server_slot_free(S)) return fail(CLOD_E_BUSY, "all %d server slots hold unfinished jobs", kSrvSlots);
  static thread_local Program P;
  P.n = 0;
  P.full = false;
  const Sink out(&P);
  hipError_t e = project_stages(*scene, b.views_dev, b.params, cx.L, b.ws, nullptr, nullptr, out);
  if (e == hipSuccess) e = bin_stages(cx.L, b.ws, D, b.dup, out);
  if (e == hipSuccess) {
    // Not the very-long-tile path: it reads the block bit planes with scalar loads, and the
    // scalar cache is invalidated only when a launch starts, not between the stages that the
    // resident kernel runs in one launch.
    BlendBufs bb = blend_bufs(&b, cx.L, D);
    bb.spare_bytes = 0;
    e = launch_blend_fwd(cx.L, b.ws, bb, b.params, rgb, T, last, nullptr, out);
  }
  if (P.full) return fail(CLOD_E_UNSUPPORTED, "the job needs more than %d stages", kMaxStages);
  HIP_TRY(e, "job stages");
  HIP_TRY(server_publish(S, P, b.n_views, b.views_host, (const char*)b.ws + cx.L.hdr, seq), "publish");
  return CLOD_OK;
}

clod_status clod_server_poll(clod_server* server, int64_t seq, int32_t* done, int64_t* info) {
  g_err[0] = 0;
  if (!server || !done) return fail(CLOD_E_ARG, "server and done must be non-NULL");
  const int r = server_poll(reinterpret_cast<Server*>(server), seq, info);
  if (r < 0) return fail(CLOD_E_ARG, "job %lld was not published or its slot was reused", (long long)seq);
  *done = r;
  return CLOD_OK;
}

clod_status clod_server_clock(clod_server* server, int64_t* ns) {
  g_err[0] = 0;
  if (!server || !ns) return fail(CLOD_E_ARG, "server and ns must be non-NULL");
  *ns = server_clock_ns(reinterpret_cast<Server*>(server));
  return CLOD_OK;
}

clod_status clod_server_stage_times(clod_server* server, int64_t seq, int64_t* ns, int32_t* kinds, int32_t max,
                                    int32_t* count) {
  g_err[0] = 0;
  if (!server || !ns || !count || max < 1) return fail(CLOD_E_ARG, "server, ns and count must be non-NULL, max >= 1");
  const int k = server_stage_times(reinterpret_cast<Server*>(server), seq, ns, kinds, max);
  if (k < 0) return fail(CLOD_E_ARG, "job %lld is not complete, was not published or its slot was reused", (long long)seq);
  *count = k;
  return CLOD_OK;
}

clod_status clod_server_stop(clod_server* server, int32_t* status) {
  g_err[0] = 0;
  if (!server) return fail(CLOD_E_ARG, "server is NULL");
  int32_t code = 0;
  HIP_TRY(server_stop(reinterpret_cast<Server*>(server), &code), "server stop");
  if (status) *status = code;
  if (code != (int32_t)kSrvStopped)
    return fail(CLOD_E_HIP, "the server ended with status %d (2: deadline reached, 3: protocol error, "
                "4: unsupported stage)", code);
  return CLOD_OK;
}

}  // extern "C"
