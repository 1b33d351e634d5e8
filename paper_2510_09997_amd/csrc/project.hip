// Per-Gaussian stages: view setup, frustum maximum of the camera distance (Sec. 3.2),
// attenuated opacity of Eq. (2) with the LoD mask, EWA projection / cull / tile rectangle /
// SH colour (Sec. 3.1), and the standalone multi-view LoD counter.
//
// Reads are plane-major (structure of arrays): consecutive lanes read consecutive floats of
// a plane, so every wave load is a full 256-byte coalesced transaction.  One thread owns one
// Gaussian and loops over the views of the batch, so parameters are read once per batch.
#include "clod_internal.h"

namespace clod {

// Derives per-view constants on the device (graph-replay safe: reads only views_dev).
// With `hdr` non-NULL the workspace header is cleared as well (a new projection).
__device__ __forceinline__ void view_setup_body(const ViewSetupArgs& a, Blk b) {
  const clod_view* __restrict__ views = a.views;
  const int V = a.V;
  const clod_params& prm = a.prm;
  DevView* __restrict__ out = a.out;
  if (a.hdr && b.id == 0 && threadIdx.x < (unsigned)kHdrWords) a.hdr[threadIdx.x] = 0ull;
  if (threadIdx.x != 0 || b.id != 0) return;
  uint32_t tile_base = 0, pix_base = 0, loss_base = 0, rgn_base = 0;
  // Same camera: every field the positions, projections and colours depend on, bit for bit.
  auto same_camera = [](const clod_view& p, const clod_view& q) {
    for (int j = 0; j < 9; ++j)
      if (__float_as_uint(p.W[j]) != __float_as_uint(q.W[j])) return false;
    for (int j = 0; j < 3; ++j)
      if (__float_as_uint(p.t[j]) != __float_as_uint(q.t[j]) || __float_as_uint(p.c[j]) != __float_as_uint(q.c[j]))
        return false;
    return __float_as_uint(p.fx) == __float_as_uint(q.fx) && __float_as_uint(p.fy) == __float_as_uint(q.fy) &&
           __float_as_uint(p.cx) == __float_as_uint(q.cx) && __float_as_uint(p.cy) == __float_as_uint(q.cy) &&
           p.width == q.width && p.height == q.height && p.frame_width == q.frame_width &&
           p.frame_height == q.frame_height && p.vx == q.vx && p.vy == q.vy;
  };
  int lead = 0;
  for (int v = 0; v < V; ++v) {
    const clod_view& cv = views[v];
    DevView d;
    if (v == 0 || !same_camera(cv, views[v - 1])) lead = v;
    d.cam_lead = lead;
    for (int j = 0; j < 9; ++j) d.W[j] = cv.W[j];
    for (int j = 0; j < 3; ++j) { d.t[j] = cv.t[j]; d.c[j] = cv.c[j]; }
    d.fx = cv.fx; d.fy = cv.fy; d.cx = cv.cx; d.cy = cv.cy;
    d.s_v = cv.s_v;
    // A viewport keeps its frame's frustum: the limits come from the frame size.
    const bool vp = cv.frame_width > 0 || cv.frame_height > 0;
    const int fw = vp ? cv.frame_width : cv.width, fh = vp ? cv.frame_height : cv.height;
    d.limx = prm.guard * ((0.5f * (float)fw) / cv.fx);
    d.limy = prm.guard * ((0.5f * (float)fh) / cv.fy);
    d.ftiles_x = (fw + kTile - 1) / kTile;
    d.ftiles_y = (fh + kTile - 1) / kTile;
    d.vx = vp ? cv.vx : 0;
    d.vy = vp ? cv.vy : 0;
    d.tau_sv = prm.tau * cv.s_v;
    d.width = cv.width;
    d.height = cv.height;
    d.tiles_x = (cv.width + kTile - 1) / kTile;
    d.tiles_y = (cv.height + kTile - 1) / kTile;
    d.tile_base = tile_base;
    d.pix_base = pix_base;
    d.loss_block_base = loss_base;
    d.rgn_base = rgn_base;
    d.budget = cv.budget;
    d.mkey = 0ull;
    tile_base += (uint32_t)(d.tiles_x * d.tiles_y);
    rgn_base += (uint32_t)(((d.tiles_x + 1) / 2) * ((d.tiles_y + 1) / 2));
    pix_base += (uint32_t)(cv.width * cv.height);
    loss_base += (uint32_t)((3u * (uint32_t)(cv.width * cv.height) + kLossChunk - 1) / kLossChunk);
    out[v] = d;
  }
}
__global__ void k_view_setup(ViewSetupArgs a) { view_setup_body(a, grid_blk()); }

__device__ __forceinline__ void fill_body(const FillArgs& a, Blk b) {
  for (int64_t i = (int64_t)b.id * kBlock + threadIdx.x; i < a.count; i += (int64_t)b.n * kBlock) a.p[i] = a.value;
}
__global__ __launch_bounds__(kBlock) void k_fill_u32(FillArgs a) { fill_body(a, grid_blk()); }

// Folds the G per-block partials of view v (every thread of the block takes part).  With kpart: the maximum squared distance, stored as the key
// bits(sqrt(max)) << 32 (0 if the frustum is empty).  With cpart: the counts (sum; also to
// counts_dev when non-NULL), the kept ratio eta = n_mask / n of Eq. (4) (to eta_dev when
// non-NULL; binary32 quotient of the counts converted to binary32) and the lowest index at d_max
// (min), which completes the low half of that key.
__device__ __forceinline__ void fold_view(int v, const unsigned long long* __restrict__ kpart, const uint32_t* __restrict__ cpart,
                          int G, int V, int64_t n, unsigned long long* __restrict__ dmax_key,
                          unsigned long long* __restrict__ counts, int64_t* __restrict__ counts_dev,
                          float* __restrict__ eta_dev) {
  __shared__ unsigned long long sm[4][4];
  __shared__ uint32_t smin[4];
  unsigned long long key = 0ull, c0 = 0, c1 = 0, c2 = 0;
  uint32_t imin = 0xFFFFFFFFu;
  for (int b = threadIdx.x; b < G; b += kBlock) {
    if (kpart) {
      const unsigned long long k = kpart[(int64_t)b * V + v];
      key = k > key ? k : key;
    }
    if (cpart) {
      const uint32_t* c = cpart + ((int64_t)b * V + v) * 4;
      c0 += c[0];
      c1 += c[1];
      c2 += c[2];
      imin = c[3] < imin ? c[3] : imin;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long ok = __shfl_xor(key, o, 64);
    key = ok > key ? ok : key;
    c0 += __shfl_xor(c0, o, 64);
    c1 += __shfl_xor(c1, o, 64);
    c2 += __shfl_xor(c2, o, 64);
    const uint32_t om = __shfl_xor(imin, o, 64);
    imin = om < imin ? om : imin;
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) { sm[w][0] = key; sm[w][1] = c0; sm[w][2] = c1; sm[w][3] = c2; smin[w] = imin; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < 4; ++j) {
      key = sm[j][0] > key ? sm[j][0] : key;
      c0 += sm[j][1]; c1 += sm[j][2]; c2 += sm[j][3];
      imin = smin[j] < imin ? smin[j] : imin;
    }
    if (kpart) {
      const float d2 = __uint_as_float((uint32_t)key);
      dmax_key[v] = key ? (unsigned long long)__float_as_uint(__builtin_sqrtf(d2)) << 32 : 0ull;
    }
    if (cpart) {
      counts[3 * v] = c0; counts[3 * v + 1] = c1; counts[3 * v + 2] = c2;
      if (counts_dev) {
        counts_dev[3 * v] = (int64_t)c0; counts_dev[3 * v + 1] = (int64_t)c1; counts_dev[3 * v + 2] = (int64_t)c2;
      }
      if (eta_dev) eta_dev[v] = n > 0 ? (float)c1 / (float)n : 0.0f;
      const unsigned long long dk = dmax_key[v];
      if (dk) dmax_key[v] = (dk & 0xFFFFFFFF00000000ull) | (unsigned long long)(0xFFFFFFFFu - imin);
    }
  }
  __syncthreads();
}

// Block v folds view v.
__device__ __forceinline__ void fold_body(const FoldArgs& a, Blk b) {
  fold_view((int)b.id, a.kpart, a.cpart, a.G, a.V, a.n, a.dmax_key, a.counts, a.counts_dev, a.eta_dev);
}
__global__ __launch_bounds__(kBlock) void k_reduce_partials(FoldArgs a) { fold_body(a, grid_blk()); }

// Per-block partials instead of global atomics: block b owns the contiguous chunk
// [b*C, (b+1)*C) of Gaussians and writes one partial per view (the frustum-max key, the three
// counts); k_reduce_partials folds them per view (one block per view).  Same-address atomics
// from every wave
// serialise in L2 and would dominate these otherwise bandwidth-bound kernels.

// Frustum maximum of the squared distance per view, as the float bits (order-preserving for
// non-negative values; 0 = no Gaussian in the frustum).  fold_view turns the maximum
// into the key bits(d_max) << 32 (d_max its correctly rounded root, the largest distance),
// and k_classify finds the lowest index at that distance, which completes the key with
// 2^32 - 1 - index (so that ties resolve to the lowest index).
__device__ __forceinline__ void frustum_max_body(const FrustumArgs& a, Blk b) {
  constexpr int kVG = 8;      // views per group (keys held in registers)
  constexpr int kItems = 8;   // Gaussians per thread per round, loaded before any is used
  __shared__ unsigned long long sm[kVG][4];
  const float* __restrict__ mean = a.mean;
  const int64_t n = a.n;
  const DevView* __restrict__ views = a.views;
  const int V = a.V;
  const float near_z = a.near_z;
  unsigned long long* __restrict__ part = a.part;   // [G][V]
  int64_t lo, hi;
  block_chunk(n, b, lo, hi);
  for (int v0 = 0; v0 < V; v0 += kVG) {
    const int vn = V - v0 < kVG ? V - v0 : kVG;
    // A view whose camera run started earlier in this group takes its lead's maximum (same
    // camera, same frustum, same distances) instead of evaluating the Gaussians again.
    uint32_t shared = 0u;   // bit vv: view v0 + vv copies its lead's key
#pragma unroll
    for (int vv = 0; vv < kVG; ++vv)
      if (vv < vn && views[v0 + vv].cam_lead != v0 + vv && views[v0 + vv].cam_lead >= v0) shared |= 1u << vv;
    uint32_t key[kVG];
#pragma unroll
    for (int vv = 0; vv < kVG; ++vv) key[vv] = 0u;
    for (int64_t b0 = lo; b0 < hi; b0 += (int64_t)kItems * kBlock) {
      float px[kItems], py[kItems], pz[kItems];
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const int64_t i = b0 + (int64_t)k * kBlock + threadIdx.x;
        const bool valid = i < hi;
        px[k] = valid ? mean[i] : 0.f;
        py[k] = valid ? mean[n + i] : 0.f;
        pz[k] = valid ? mean[2 * n + i] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const int64_t i = b0 + (int64_t)k * kBlock + threadIdx.x;
        if (i >= hi) continue;
#pragma unroll
        for (int vv = 0; vv < kVG; ++vv) {
          if (vv >= vn) break;
          if ((shared >> vv) & 1u) continue;
          const DevView& Vw = views[v0 + vv];
          float x, y, z, ex, ey, ez;
          to_camera(Vw, px[k], py[k], pz[k], x, y, z);
          if (in_frustum(Vw, x, y, z, near_z)) {
            const uint32_t kk = __float_as_uint(cam_distance2(Vw, px[k], py[k], pz[k], ex, ey, ez));
            key[vv] = kk > key[vv] ? kk : key[vv];
          }
        }
      }
    }
    // (A run's views are consecutive: each shared view copies the one before it.)
#pragma unroll
    for (int vv = 1; vv < kVG; ++vv)
      if ((shared >> vv) & 1u) key[vv] = key[vv - 1];
#pragma unroll
    for (int vv = 0; vv < kVG; ++vv) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint32_t other = __shfl_xor(key[vv], o, 64);
        key[vv] = other > key[vv] ? other : key[vv];
      }
      if (lane_id() == 0) sm[vv][threadIdx.x >> 6] = key[vv];
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)vn) {
      const int vv = threadIdx.x;
      unsigned long long m = sm[vv][0];
      for (int w = 1; w < 4; ++w) m = sm[vv][w] > m ? sm[vv][w] : m;
      part[(int64_t)b.id * V + v0 + vv] = m;
    }
    __syncthreads();
  }
}
__global__ __launch_bounds__(kBlock) void k_frustum_max(FrustumArgs a) { frustum_max_body(a, grid_blk()); }

// Pass 1 over every Gaussian (block b owns the chunk [b*C, (b+1)*C)): per view the frustum
// flag, Eq. (2) and the LoD mask (alpha'' and the F/M flags written for every (view,
// Gaussian)), F and M counts, and the Gaussians that are in some view's
// frustum and kept by its mask appended to the block's segment of the work list (order
// within a segment is arbitrary).  Outside those, nothing else is computed, so the heavy
// pass below runs on full waves instead of the ~40% of lanes a whole-scene pass keeps busy.
// scnt: LDS of 3 V words ([V][3]: F count, M count, lowest index at d_max).
template <bool kWrite>
__device__ __forceinline__ void classify_body(const ClassifyArgs& a, Blk b, uint32_t* scnt) {
  __shared__ uint32_t sbase;
  const clod_scene& sc = a.sc;
  const DevView* __restrict__ views = a.views;
  const int V = a.V;
  const clod_params& prm = a.prm;
  const unsigned long long* __restrict__ dmax_key = a.dmax_key;
  uint32_t* __restrict__ cpart = a.cpart;   // [G][V][4]
  uint8_t* __restrict__ flags_out = a.flags;
  float* __restrict__ alpha_out = a.alpha;
  uint32_t* __restrict__ list = a.list;       // [n]
  uint32_t* __restrict__ lcount = a.lcount;   // [G]
  const int64_t n = sc.n;
  for (int j = threadIdx.x; j < 3 * V; j += kBlock) scnt[j] = j % 3 == 2 ? 0xFFFFFFFFu : 0u;
  if (threadIdx.x == 0) sbase = 0;
  __syncthreads();
  int64_t lo, hi;
  block_chunk(n, b, lo, hi);
  const uint64_t lt = lanemask_lt();
  const int64_t iters = (hi - lo + kBlock - 1) / kBlock;
  // Software pipelined: the next round's parameters are loaded before this round's views are
  // evaluated, so their latency overlaps the arithmetic.
  float nmx = 0.f, nmy = 0.f, nmz = 0.f, nop = 0.f, ndc = 0.f;
  {
    const int64_t i = lo + threadIdx.x;
    if (iters > 0 && i < hi) {
      nmx = sc.mean[i]; nmy = sc.mean[n + i]; nmz = sc.mean[2 * n + i];
      nop = sc.opacity[i]; ndc = sc.decay[i];
    }
  }
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = lo + it * kBlock + threadIdx.x;
    const bool valid = i < hi;
    const float mx = nmx, my = nmy, mz = nmz;
    const float alpha = sigmoid_c(nop), den = decay_den(ndc, prm.eps);   // view independent
    {
      const int64_t i2 = i + kBlock;
      if (it + 1 < iters && i2 < hi) {
        nmx = sc.mean[i2]; nmy = sc.mean[n + i2]; nmz = sc.mean[2 * n + i2];
        nop = sc.opacity[i2]; ndc = sc.decay[i2];
      }
    }
    bool any = false;
    // The camera's part (frustum flag, distance, d / d_max) of the previous view, reused by the
    // views of the same camera run (which have the same frustum maximum).
    int lead = -1;
    bool F = false;
    float d = 0.f, dn = 0.f;
    for (int v = 0; v < V; ++v) {
      const DevView& Vw = views[v];
      bool M = false;
      if (!valid) F = false;
      if (valid) {
        const unsigned long long dk = dmax_key[v];
        if (Vw.cam_lead != lead) {
          float x, y, z, ex, ey, ez;
          to_camera(Vw, mx, my, mz, x, y, z);
          F = in_frustum(Vw, x, y, z, prm.near_z);
          d = cam_distance(Vw, mx, my, mz, ex, ey, ez);
          dn = d / dmax_from_key(dk);
          lead = Vw.cam_lead;
        }
        if (F && dk != 0ull && __float_as_uint(d) == (uint32_t)(dk >> 32)) atomicMin(&scnt[3 * v + 2], (uint32_t)i);
        float q;
        const float a2 = attenuated_dn(dn, Vw.s_v, alpha, den, q);
        M = lod_kept(Vw, a2, i);
        if (kWrite) {
          const int64_t f = (int64_t)v * n + i;
          alpha_out[f] = a2;
          flags_out[f] = (uint8_t)((F ? 1 : 0) | (M ? 2 : 0));
        }
      }
      any = any || (F && M);
      const uint64_t bF = ballot64(F), bM = ballot64(M);
      if (lane_id() == 0) {
        if (bF) atomicAdd(&scnt[3 * v + 0], (uint32_t)__popcll(bF));
        if (bM) atomicAdd(&scnt[3 * v + 1], (uint32_t)__popcll(bM));
      }
    }
    const uint64_t bw = ballot64(any);
    uint32_t wbase = 0;
    if (lane_id() == 0 && bw) wbase = atomicAdd(&sbase, (uint32_t)__popcll(bw));
    wbase = __shfl(wbase, 0, 64);
    if (any) list[lo + wbase + (uint32_t)__popcll(bw & lt)] = (uint32_t)i;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < V; j += kBlock) {
    cpart[((int64_t)b.id * V + j) * 4 + 0] = scnt[3 * j];
    cpart[((int64_t)b.id * V + j) * 4 + 1] = scnt[3 * j + 1];
    cpart[((int64_t)b.id * V + j) * 4 + 3] = scnt[3 * j + 2];
  }
  if (threadIdx.x == 0) lcount[b.id] = sbase;
}
template <bool kWrite>
__global__ __launch_bounds__(kBlock) void k_classify(ClassifyArgs a) {
  extern __shared__ uint32_t scnt_dyn[];
  classify_body<kWrite>(a, grid_blk(), scnt_dyn);
}

// Pass 2 over the work list (entries spread evenly over the blocks): per listed Gaussian the
// geometry of every view again (cheap), then for in-frustum kept views the EWA projection,
// cull and rectangle, remembering which views render it; then the colour of each rendering
// view is evaluated from its SH coefficients.  Records (with depth, rectangle and tiles
// touched in their fourth quad) are written for rendered (view, Gaussian) pairs only.
// sdyn: LDS of G + V words ([G] segment offsets, then [V] rendered counts).
template <int DEG, bool kWriteRecords, bool kPacked>
__device__ __forceinline__ void project_body(const ProjectArgs& a, Blk b, uint32_t* sdyn) {
  __shared__ uint32_t sm[4];
  const clod_scene& sc = a.sc;
  const DevView* __restrict__ views = a.views;
  const int V = a.V;
  const clod_params& prm = a.prm;
  const unsigned long long* __restrict__ dmax_key = a.dmax_key;
  uint32_t* __restrict__ cpart = a.cpart;   // [G][V][4]
  const uint32_t* __restrict__ list = a.list;
  const uint32_t* __restrict__ lcount = a.lcount;
  uint8_t* __restrict__ flags_out = a.flags;
  float4* __restrict__ rec = a.rec;
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t n = sc.n;
  const int G = (int)b.n;
  uint32_t* soff = sdyn;
  uint32_t* scnt = sdyn + G;
  // Exclusive offsets of the G list segments and the list length: every block scans the
  // segment counts itself (G <= 2048: eight per thread, blocked).
  int64_t L;
  {
    constexpr int kPer = kMaxProjBlocks / kBlock;
    static_assert(kPer * kBlock == kMaxProjBlocks, "segment scan layout");
    const int j0 = threadIdx.x * kPer;
    uint32_t c[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      c[k] = j0 + k < G ? lcount[j0 + k] : 0u;
      sum += c[k];
    }
    uint32_t tot;
    uint32_t off = block_exclusive_scan(sum, sm, tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (j0 + k < G) soff[j0 + k] = off;
      off += c[k];
    }
    L = tot;
  }
  for (int j = threadIdx.x; j < V; j += kBlock) scnt[j] = 0;
  __syncthreads();
  const int64_t per = (n + G - 1) / G;   // chunk length of the first pass
  const int64_t stride = (int64_t)G * kBlock;
  // Every lane of the block runs the same number of rounds (ballots stay uniform).
  for (int64_t base = (int64_t)b.id * kBlock; base < L; base += stride) {
    const int64_t e = base + threadIdx.x;
    const bool valid = e < L;
    int64_t i = 0;
    if (valid) {
      int blo = 0, bhi = G - 1;   // last segment whose offset is <= e
      while (blo < bhi) {
        const int mid = (blo + bhi + 1) >> 1;
        if ((int64_t)soff[mid] <= e) blo = mid; else bhi = mid - 1;
      }
      i = (int64_t)list[(int64_t)blo * per + (e - (int64_t)soff[blo])];
    }
    float mx = 0.f, my = 0.f, mz = 0.f, op = 0.f, dc = 0.f;
    if (valid) {
      mx = sc.mean[i]; my = sc.mean[n + i]; mz = sc.mean[2 * n + i];
      op = sc.opacity[i]; dc = sc.decay[i];
    }
    const float alpha = sigmoid_c(op), den = decay_den(dc, prm.eps);   // view independent
    // Rotation and 3D covariance are view independent: computed on first use.
    bool have_cov = false;
    float S[9];
    // The projection (and below the colour) of the last camera run evaluated: views of one run
    // share them (only alpha'' and the mask depend on s_v).
    int geo_lead = -1, col_lead = -1;
    Proj P;
    bool pok = false;
    float col[3] = {0.f, 0.f, 0.f};
    uint8_t cfl = 0;
    for (int v0 = 0; v0 < V; v0 += 32) {
      const int vn = V - v0 < 32 ? V - v0 : 32;
      uint32_t rmask = 0;   // rendered views of the group
      for (int vv = 0; vv < vn; ++vv) {
        const int v = v0 + vv;
        const DevView& Vw = views[v];
        bool R = false;
        if (valid) {
          float x, y, z, ex, ey, ez;
          to_camera(Vw, mx, my, mz, x, y, z);
          const bool F = in_frustum(Vw, x, y, z, prm.near_z);
          const float d = cam_distance(Vw, mx, my, mz, ex, ey, ez);
          float q;
          const float a2 = attenuated_pre(d, dmax_from_key(dmax_key[v]), Vw.s_v, alpha, den, q);
          if (F && lod_kept(Vw, a2, i)) {
            if (!have_cov) {
              const float s0 = cexp(sc.log_scale[i]), s1 = cexp(sc.log_scale[n + i]), s2 = cexp(sc.log_scale[2 * n + i]);
              float Rm[9], w_, x_, y_, z_, rn;
              quat_rot(sc.quat[i], sc.quat[n + i], sc.quat[2 * n + i], sc.quat[3 * n + i], Rm, w_, x_, y_, z_, rn);
              cov3(Rm, s0, s1, s2, S);
              have_cov = true;
            }
            if (Vw.cam_lead != geo_lead) {
              pok = ewa(Vw, x, y, z, S, prm.dilation, P);
              geo_lead = Vw.cam_lead;
            }
            if (pok) {
              R = true;
              if (kWriteRecords) {
                const int64_t f = (int64_t)v * n + i;
                rec[kRecQuads * f] = make_float4(P.u, P.v, a2, P.rad);
                rec[kRecQuads * f + 1] = make_float4(P.A, P.B, P.C, 0.f);
                // Depth, tile rectangle and tiles touched: the fourth quad, so the record is
                // written whole (no partial 64-byte segments, no separate scattered planes).
                rec[kRecQuads * f + 3] =
                    make_float4(z, __uint_as_float((uint32_t)P.x0 | ((uint32_t)P.x1 << 16)),
                                __uint_as_float((uint32_t)P.y0 | ((uint32_t)P.y1 << 16)),
                                __uint_as_float((uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0))));
              }
            }
          }
        }
        rmask |= (R ? 1u : 0u) << vv;
        const uint64_t bR = ballot64(R);
        if (lane_id() == 0 && bR) atomicAdd(&scnt[v], (uint32_t)__popcll(bR));
      }
      if (kWriteRecords && rmask) {
        // Plane-major coefficients are gathered once into registers; a packed per-Gaussian
        // block is instead re-read for every rendering view (cache hits after the first one,
        // float4 chunks when 3K % 4 == 0), which keeps the kernel at half the registers.
        // Either way each channel accumulates in coefficient order.
        float shc[kPacked ? 1 : 3 * K];
        if constexpr (!kPacked) {
#pragma unroll
          for (int k = 0; k < 3 * K; ++k) shc[k] = sc.sh[(int64_t)k * n + i];
        }
        uint32_t m = rmask;
        while (m) {
          const int vv = __builtin_ctz(m);
          m &= m - 1;
          const int v = v0 + vv;
          const DevView& Vw = views[v];
          const int64_t f = (int64_t)v * n + i;
          if (Vw.cam_lead != col_lead) {
          col_lead = Vw.cam_lead;
          float ex, ey, ez;
          const float d = cam_distance(Vw, mx, my, mz, ex, ey, ez);
          const float id = 1.0f / d;
          float Yb[16];
          sh_basis(DEG, ex * id, ey * id, ez * id, Yb);
          float acc[3];
          if constexpr (kPacked) {
            const float* src = sc.sh_packed + (int64_t)i * (3 * K);
            if constexpr ((3 * K) % 4 == 0) {
              const float4* src4 = reinterpret_cast<const float4*>(src);
#pragma unroll
              for (int q = 0; q < (3 * K) / 4; ++q) {
                const float4 c4 = src4[q];
                const float cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int idx = 4 * q + e, k = idx / 3, ch = idx % 3;
                  acc[ch] = k == 0 ? cv[e] * Yb[0] : fmaf_(cv[e], Yb[k], acc[ch]);
                }
              }
            } else {
#pragma unroll
              for (int idx = 0; idx < 3 * K; ++idx) {
                const int k = idx / 3, ch = idx % 3;
                acc[ch] = k == 0 ? src[idx] * Yb[0] : fmaf_(src[idx], Yb[k], acc[ch]);
              }
            }
          } else {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
              float a = shc[ch] * Yb[0];
#pragma unroll
              for (int k = 1; k < K; ++k) a = fmaf_(shc[3 * k + ch], Yb[k], a);
              acc[ch] = a;
            }
          }
          cfl = 1u | 2u | 4u;   // rendered implies in frustum and kept
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const float cv = acc[ch] + 0.5f;
            if (!(cv > 0.0f)) cfl |= (uint8_t)(8 << ch);
            col[ch] = fmaxf(cv, 0.0f);
          }
          }
          rec[kRecQuads * f + 2] = make_float4(col[0], col[1], col[2], 0.f);
          flags_out[f] = cfl;
        }
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < V; j += kBlock) cpart[((int64_t)b.id * V + j) * 4 + 2] = scnt[j];
}

// Plane-major coefficients (or no records).
template <int DEG, bool kWriteRecords>
__global__ __launch_bounds__(kBlock) void k_project(ProjectArgs a) {
  extern __shared__ uint32_t sdyn[];
  project_body<DEG, kWriteRecords, false>(a, grid_blk(), sdyn);
}

// Packed coefficients: fits 128 registers, so four waves per SIMD hide the gather latency.
template <int DEG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_project_packed(ProjectArgs a) {
  extern __shared__ uint32_t sdyn[];
  project_body<DEG, true, true>(a, grid_blk(), sdyn);
}

// Budgeted LoD (a view with budget K, 0 < K < n): the K-th largest selection key, by an MSD
// radix select over the eight bytes of the 64-bit key.  Pass p histograms byte p (from the top)
// of the keys that share the prefix found so far (k_select_hist, one histogram per block and
// view; alpha'' is recomputed from the scene exactly as the projection computes it), then
// k_select_pick finds the byte value holding the wanted rank and narrows the prefix.  After
// eight passes the prefix is the threshold key.  K >= n keeps everything (threshold 0).
// Block b of V * kSelBlocks: chunk b % kSelBlocks of view b / kSelBlocks.
__device__ __forceinline__ void select_hist_body(const SelectArgs& a, Blk b) {
  __shared__ uint32_t h[256];
  const clod_scene& sc = a.sc;
  const DevView* __restrict__ views = a.views;
  const clod_params& prm = a.prm;
  const unsigned long long* __restrict__ dmax_key = a.dmax_key;
  const SelState* __restrict__ state = a.state;
  const int pass = a.pass;
  uint32_t* __restrict__ hist = a.hist;   // [V][kSelBlocks][256]
  const int v = (int)(b.id / kSelBlocks);
  const uint32_t chunk = b.id % kSelBlocks;
  const DevView& Vw = views[v];
  const int64_t n = sc.n;
  if (Vw.budget <= 0 || Vw.budget >= n) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int shift = 56 - 8 * pass;
  const unsigned long long pre = pass == 0 ? 0ull : state[v].prefix >> (shift + 8);
  const float dmax = dmax_from_key(dmax_key[v]);
  int64_t lo, hi;
  block_chunk(n, Blk{chunk, (uint32_t)kSelBlocks}, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    float ex, ey, ez;
    const float d = cam_distance(Vw, sc.mean[i], sc.mean[n + i], sc.mean[2 * n + i], ex, ey, ez);
    float alpha, q;
    const float a2 = attenuated(d, dmax, Vw.s_v, sc.decay[i], sc.opacity[i], prm.eps, alpha, q);
    const unsigned long long key = lod_key(a2, i);
    if (pass == 0 || (key >> (shift + 8)) == pre) atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[((int64_t)v * kSelBlocks + chunk) * 256 + threadIdx.x] = h[threadIdx.x];
}
__global__ __launch_bounds__(kBlock) void k_select_hist(SelectArgs a) { select_hist_body(a, grid_blk()); }

__device__ __forceinline__ void select_pick_body(const SelectArgs& a, Blk b) {
  __shared__ uint32_t sm[4];
  DevView* __restrict__ views = a.views;
  const int64_t n = a.sc.n;
  const int pass = a.pass;
  SelState* __restrict__ state = a.state;
  const uint32_t* __restrict__ hist = a.hist;
  const int v = (int)b.id;
  DevView& Vw = views[v];
  if (Vw.budget <= 0) return;
  if (Vw.budget >= n) {
    if (threadIdx.x == 0) Vw.mkey = 0ull;
    return;
  }
  const unsigned long long rank = pass == 0 ? (unsigned long long)Vw.budget : state[v].rank;
  const unsigned long long prefix = pass == 0 ? 0ull : state[v].prefix;
  // Thread t takes byte value d = 255 - t, so an inclusive scan over t counts the keys whose
  // byte is >= d.
  const uint32_t d = 255u - threadIdx.x;
  uint32_t c = 0;
  for (int b = 0; b < kSelBlocks; ++b) c += hist[((int64_t)v * kSelBlocks + b) * 256 + d];
  uint32_t inc = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(inc, o, 64);
    if (lane_id() >= (uint32_t)o) inc += up;
  }
  if (lane_id() == 63) sm[threadIdx.x >> 6] = inc;
  __syncthreads();
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) inc += sm[w];
  const uint32_t excl = inc - c;
  if (excl < rank && rank <= inc) {
    const int shift = 56 - 8 * pass;
    const unsigned long long np = prefix | ((unsigned long long)d << shift);
    state[v].prefix = np;
    state[v].rank = rank - excl;
    if (pass == 7) Vw.mkey = np;
  }
}
__global__ __launch_bounds__(kBlock) void k_select_pick(SelectArgs a) { select_pick_body(a, grid_blk()); }

hipError_t launch_lod_select(const clod_scene& sc, DevView* vinfo, int V, clod_params prm,
                             const unsigned long long* dmax_key, SelState* state, uint32_t* hist, const Sink& out) {
  if (sc.n == 0) return hipSuccess;
  for (int pass = 0; pass < 8; ++pass) {
    Stage h{};
    h.kind = kStSelectHist;
    h.items = (uint32_t)(kSelBlocks * V);
    h.block = kBlock;
    h.a.select = SelectArgs{sc, vinfo, V, prm, dmax_key, state, hist, pass};
    Stage p = h;
    p.kind = kStSelectPick;
    p.items = (uint32_t)V;
    hipError_t e = out.put(h);
    if (e == hipSuccess) e = out.put(p);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int proj_blocks(int64_t n) {
  int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
  if (g < 1) g = 1;
  if (g > kMaxProjBlocks) g = kMaxProjBlocks;
  return (int)g;
}

hipError_t launch_view_setup(const clod_view* views_dev, int V, clod_params prm, DevView* vinfo,
                             unsigned long long* hdr, const Sink& out) {
  Stage st{};
  st.kind = kStViewSetup;
  st.items = 1;
  st.block = 64;
  st.a.view_setup = ViewSetupArgs{views_dev, V, prm, vinfo, hdr};
  return out.put(st);
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, const Sink& out) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  Stage st{};
  st.kind = kStFill;
  st.items = (uint32_t)g;
  st.block = kBlock;
  st.a.fill = FillArgs{p, value, count};
  return out.put(st);
}

static Stage fold_stage(const unsigned long long* kpart, const uint32_t* cpart, int G, int V,
                        unsigned long long* dmax_key, unsigned long long* counts, int64_t* counts_dev, int64_t n,
                        float* eta_dev) {
  Stage st{};
  st.kind = kStFold;
  st.items = (uint32_t)V;
  st.block = kBlock;
  st.a.fold = FoldArgs{kpart, cpart, G, V, dmax_key, counts, counts_dev, n, eta_dev};
  return st;
}

hipError_t launch_frustum_max(const clod_scene& sc, const DevView* vinfo, int V, float near_z,
                              unsigned long long* kpart, unsigned long long* dmax_key, const Sink& out) {
  if (sc.n == 0) return launch_fill_u32((uint32_t*)dmax_key, 0u, 2 * (int64_t)V, out);
  const int G = proj_blocks(sc.n);
  Stage st{};
  st.kind = kStFrustumMax;
  st.items = (uint32_t)G;
  st.block = kBlock;
  st.a.frustum = FrustumArgs{sc.mean, sc.n, vinfo, V, near_z, kpart};
  hipError_t e = out.put(st);
  if (e == hipSuccess)
    e = out.put(fold_stage(kpart, nullptr, G, V, dmax_key, nullptr, nullptr, sc.n, nullptr));
  return e;
}

template <bool kWrite>
static hipError_t project_impl(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                               unsigned long long* dmax_key, uint32_t* cpart, unsigned long long* counts,
                               int64_t* counts_dev, float* eta_dev, uint8_t* flags, float* alpha, float4* rec,
                               uint32_t* list, uint32_t* lcount, const Sink& out) {
  if (sc.n == 0) {
    hipError_t e = launch_fill_u32((uint32_t*)counts, 0u, 6 * (int64_t)V, out);
    if (e == hipSuccess && counts_dev) e = launch_fill_u32((uint32_t*)counts_dev, 0u, 6 * (int64_t)V, out);
    if (e == hipSuccess && eta_dev) e = launch_fill_u32((uint32_t*)eta_dev, 0u, (int64_t)V, out);
    return e;
  }
  const int G = proj_blocks(sc.n);
  Stage c{};
  c.kind = kStClassify;
  c.items = (uint32_t)G;
  c.block = kBlock;
  c.lds = (uint32_t)(3 * V * sizeof(uint32_t));
  c.a.classify = ClassifyArgs{sc, vinfo, V, kWrite ? 1 : 0, prm, dmax_key, cpart, flags, alpha, list, lcount};
  hipError_t e = out.put(c);
  if (e != hipSuccess) return e;
  // Packed SH is only read when records are written.
  Stage p{};
  p.kind = kStProject;
  p.items = (uint32_t)G;
  p.block = kBlock;
  p.lds = (uint32_t)((G + V) * sizeof(uint32_t));
  p.a.project = ProjectArgs{sc, vinfo, V, prm, dmax_key, cpart, list, lcount, flags, rec, kWrite ? 1 : 0,
                            kWrite && sc.sh_packed != nullptr ? 1 : 0};
  e = out.put(p);
  if (e != hipSuccess) return e;
  // Counts to the workspace and the caller, and the argmax index into the d_max key.
  return out.put(fold_stage(nullptr, cpart, G, V, dmax_key, counts, counts_dev, sc.n, eta_dev));
}

hipError_t launch_project(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                          unsigned long long* dmax_key, uint32_t* cpart, unsigned long long* counts,
                          int64_t* counts_dev, float* eta_dev, uint8_t* flags, float* alpha, float4* rec,
                          uint32_t* list, uint32_t* lcount, const Sink& out) {
  return project_impl<true>(sc, vinfo, V, prm, dmax_key, cpart, counts, counts_dev, eta_dev, flags, alpha, rec, list,
                            lcount, out);
}

hipError_t launch_lod_count(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                            unsigned long long* dmax_key, uint32_t* cpart, unsigned long long* counts,
                            int64_t* counts_dev, float* eta_dev, uint32_t* list, uint32_t* lcount,
                            const Sink& out) {
  return project_impl<false>(sc, vinfo, V, prm, dmax_key, cpart, counts, counts_dev, eta_dev, nullptr, nullptr,
                             nullptr, list, lcount, out);
}

// One kernel per stage kind of this file (the template instance the arguments select).
hipError_t launch_project_stage(const Stage& st, hipStream_t s) {
  const dim3 g(st.items), blk(st.block);
  switch (st.kind) {
    case kStViewSetup: hipLaunchKernelGGL(k_view_setup, g, blk, 0, s, st.a.view_setup); break;
    case kStFill: hipLaunchKernelGGL(k_fill_u32, g, blk, 0, s, st.a.fill); break;
    case kStFrustumMax: hipLaunchKernelGGL(k_frustum_max, g, blk, 0, s, st.a.frustum); break;
    case kStFold: hipLaunchKernelGGL(k_reduce_partials, g, blk, 0, s, st.a.fold); break;
    case kStClassify:
      if (st.a.classify.write) hipLaunchKernelGGL(k_classify<true>, g, blk, st.lds, s, st.a.classify);
      else hipLaunchKernelGGL(k_classify<false>, g, blk, st.lds, s, st.a.classify);
      break;
    case kStProject: {
      const ProjectArgs& a = st.a.project;
      auto kern = a.packed ? k_project_packed<3> : (a.write ? k_project<3, true> : k_project<3, false>);
      switch (a.sc.sh_degree) {
        case 0: kern = a.packed ? k_project_packed<0> : (a.write ? k_project<0, true> : k_project<0, false>); break;
        case 1: kern = a.packed ? k_project_packed<1> : (a.write ? k_project<1, true> : k_project<1, false>); break;
        case 2: kern = a.packed ? k_project_packed<2> : (a.write ? k_project<2, true> : k_project<2, false>); break;
        default: break;
      }
      hipLaunchKernelGGL(kern, g, blk, st.lds, s, a);
      break;
    }
    case kStSelectHist: hipLaunchKernelGGL(k_select_hist, g, blk, 0, s, st.a.select); break;
    case kStSelectPick: hipLaunchKernelGGL(k_select_pick, g, blk, 0, s, st.a.select); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clod
