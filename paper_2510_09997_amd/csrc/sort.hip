// Tile binning (Sec. 3.1, "sorted by depth"): exclusive scan of tiles touched, emission of
// one (tile, depth) key per covered tile, stable LSD radix sort, per-tile ranges.
//
// Everything is device-driven: the pair count D lives in the workspace header and the sort
// kernels read it, so no host synchronisation is needed between the stages (and the whole
// sequence can be captured in a graph).  Counting uses wave64 ballots: a lane's rank among
// lanes with the same digit is popcount(match & lanemask_lt), where match is the AND of
// eight ballots over the digit bits.
#include "clod_internal.h"

namespace clod {

// ---------------------------------------------------------------------------- block scan
// Exclusive scan of one uint32 per thread over the 256-thread block; returns the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* smem /*[4]*/,
                                                          uint32_t& total) {
  const uint32_t lane = lane_id();
  const int wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += up;
  }
  if (lane == 63) smem[wave] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += smem[w];
  total = smem[0] + smem[1] + smem[2] + smem[3];
  __syncthreads();
  return wbase + inc - v;
}

// --------------------------------------------------------------- tiles-touched scan + dup
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ tiles, int64_t count,
                                                        uint32_t* __restrict__ part) {
  __shared__ uint32_t sm[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
    if (j < count) s += tiles[j];
  }
  s = wave_sum(s);
  if (lane_id() == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// Single block: exclusive scan of the block partials; D and the overflow flag to the header.
__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t* __restrict__ part, int nparts,
                                                          unsigned long long* __restrict__ hdr,
                                                          int64_t cap) {
  __shared__ uint32_t sm[4];
  unsigned long long carry = 0;
  for (int base = 0; base < nparts; base += kBlock) {
    const int j = base + threadIdx.x;
    const uint32_t v = j < nparts ? part[j] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, sm, total);
    if (j < nparts) part[j] = (uint32_t)carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    hdr[kHdrDup] = carry;
    hdr[kHdrOverflow] = (long long)carry > cap ? 1ull : 0ull;
  }
}

// Per block: exclusive offsets of its chunk of items (blocked: thread t owns items
// t*16 .. t*16+15), kept in LDS; then the block's output positions are walked in order, 256 at
// a time, so the key and value stores are coalesced whatever the rectangle sizes.  Output o
// of the block belongs to the last item whose offset is <= o (binary search; items with no
// tiles share their successor's offset and are never selected) and is that item's
// (o - offset)-th covered tile in row-major order.
__global__ __launch_bounds__(kBlock) void k_scan_dup(
    const uint32_t* __restrict__ tiles, int64_t count, const uint32_t* __restrict__ part,
    const float* __restrict__ depth, const uint2* __restrict__ rect, const DevView* __restrict__ views,
    int64_t n, const unsigned long long* __restrict__ hdr, int64_t cap,
    unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t sm[4];
  __shared__ uint32_t loff[kScanChunk];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int t = threadIdx.x;
  // Coalesced load of the chunk's counts into LDS, then blocked reads.
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + t;
    loff[k * kBlock + t] = j < count ? tiles[j] : 0u;
  }
  __syncthreads();
  uint32_t loc[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = loff[t * kScanItems + k];
    s += loc[k];
  }
  uint32_t total;
  uint32_t off = block_exclusive_scan(s, sm, total);   // its barriers also end the reads above
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loff[t * kScanItems + k] = off;
    off += loc[k];
  }
  __syncthreads();
  if (hdr[kHdrOverflow] != 0ull) return;
  const int64_t out0 = (int64_t)part[blockIdx.x];
  const uint32_t nn = (uint32_t)n;
  for (uint32_t o = (uint32_t)t; o < total; o += kBlock) {
    int lo = 0, hi = kScanChunk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (loff[mid] <= o) lo = mid; else hi = mid - 1;
    }
    const uint32_t rel = o - loff[lo];
    const uint32_t f = (uint32_t)base + (uint32_t)lo;
    const DevView& Vw = views[f / nn];
    const uint2 rc = rect[f];
    const uint32_t x0 = rc.x & 0xFFFFu, x1 = rc.x >> 16, y0 = rc.y & 0xFFFFu;
    const uint32_t w = x1 - x0;
    const uint32_t ty = y0 + rel / w, tx = x0 + rel % w;
    const uint32_t tile = Vw.tile_base + ty * (uint32_t)Vw.tiles_x + tx;
    const int64_t og = out0 + (int64_t)o;
    if (og < cap) {
      keys[og] = ((unsigned long long)tile << 32) | (unsigned long long)__float_as_uint(depth[f]);
      vals[og] = f;
    }
  }
}

hipError_t launch_scan_dup(const Layout& L, void* ws, const DupLayout& D, void* dup, hipStream_t s) {
  char* w = (char*)ws;
  char* dp = (char*)dup;
  const uint32_t* tiles = (const uint32_t*)(w + L.tiles);
  uint32_t* part = (uint32_t*)(w + L.scan_part);
  unsigned long long* hdr = (unsigned long long*)(w + L.hdr);
  const int nb = L.scan_blocks;
  if (nb == 0) return launch_fill_u32((uint32_t*)hdr, 0u, 4, s);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, tiles, L.VN, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, part, nb, hdr, D.cap);
  hipLaunchKernelGGL(k_scan_dup, dim3(nb), dim3(kBlock), 0, s, tiles, L.VN, part,
                     (const float*)(w + L.depth), (const uint2*)(w + L.rect), (const DevView*)(w + L.vinfo),
                     L.n, hdr, D.cap, (unsigned long long*)(dp + D.keys0), (uint32_t*)(dp + D.vals0));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- radix sort
// Reduce-then-scan LSD radix sort with 8-bit digits.  Block b of G owns the contiguous
// chunk [b*C, (b+1)*C) of the D keys (C a multiple of the 2048-key tile), so the stable
// order across blocks is the block order.

__device__ __forceinline__ void sort_chunk(int64_t D, int G, int b, int64_t& lo, int64_t& hi) {
  const int64_t tiles_total = (D + kSortTile - 1) / kSortTile;
  const int64_t per = (tiles_total + G - 1) / G;
  lo = (int64_t)b * per * kSortTile;
  hi = lo + per * kSortTile;
  if (lo > D) lo = D;
  if (hi > D) hi = D;
}

// Lanes of this wave holding the same 8-bit digit (restricted to `active`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t m = active;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bal = ballot64((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

__global__ __launch_bounds__(kBlock) void k_radix_upsweep(const unsigned long long* __restrict__ keys,
                                                          const unsigned long long* __restrict__ hdr,
                                                          int G, int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[4][256];   // per-wave digit counts
  if (hdr[kHdrOverflow]) return;
  const int64_t D = (int64_t)hdr[kHdrDup];
  const int t = threadIdx.x;
  const int wave = t >> 6;
#pragma unroll
  for (int w = 0; w < 4; ++w) cnt[w][t] = 0;
  __syncthreads();
  int64_t lo, hi;
  sort_chunk(D, G, blockIdx.x, lo, hi);
  // kSortItems keys per thread per step, all loads issued before any is used.
  for (int64_t base = lo; base < hi; base += kSortTile) {
    uint32_t d8[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t idx = base + (int64_t)j * kBlock + t;
      d8[j] = idx < hi ? (uint32_t)(keys[idx] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
      if (d8[j] < 256u) atomicAdd(&cnt[wave][d8[j]], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * G + blockIdx.x] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

// Block d: exclusive scan of digit d's per-block counts hist[d*G .. d*G+G) in place, and
// the digit total in hist[256*G + d].
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t* __restrict__ hist, int G,
                                                             const unsigned long long* __restrict__ hdr) {
  __shared__ uint32_t sm[4];
  if (hdr[kHdrOverflow]) return;
  uint32_t* h = hist + (int64_t)blockIdx.x * G;
  uint32_t carry = 0;
  for (int base = 0; base < G; base += kBlock) {
    const int j = base + threadIdx.x;
    const uint32_t v = j < G ? h[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sm, tot);
    if (j < G) h[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) hist[(int64_t)256 * G + blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBlock) void k_radix_downsweep(
    const unsigned long long* __restrict__ kin, const uint32_t* __restrict__ vin,
    unsigned long long* __restrict__ kout, uint32_t* __restrict__ vout,
    const uint32_t* __restrict__ hist, const unsigned long long* __restrict__ hdr, int G, int shift) {
  __shared__ uint32_t running[256];      // global output position of the next key per digit
  __shared__ uint32_t wcnt[4][256];      // per-wave digit counts within the tile
  __shared__ uint32_t tstart[256];       // tile-local start of each digit
  __shared__ uint32_t sm[4];
  __shared__ unsigned long long skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  if (hdr[kHdrOverflow]) return;
  const int64_t D = (int64_t)hdr[kHdrDup];
  int64_t lo, hi;
  sort_chunk(D, G, blockIdx.x, lo, hi);
  const int t = threadIdx.x;
  const int wave = t >> 6;
  const uint32_t lane = lane_id();
  {
    uint32_t tall;
    const uint32_t digit_base = block_exclusive_scan(hist[(int64_t)256 * G + t], sm, tall);
    running[t] = digit_base + hist[(int64_t)t * G + blockIdx.x];
  }
  const uint64_t lt = lanemask_lt();
  for (int64_t base = lo; base < hi; base += kSortTile) {
    wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
    __syncthreads();
    unsigned long long k8[kSortItems];
    uint32_t v8[kSortItems], d8[kSortItems], r8[kSortItems];
    // Wave w owns keys [base + w*512, base + (w+1)*512), slot j holds base + w*512 + j*64 + lane.
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t idx = base + (int64_t)wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < hi;
      k8[j] = valid ? kin[idx] : 0ull;
      v8[j] = valid ? vin[idx] : 0u;
      const uint32_t d = valid ? (uint32_t)(k8[j] >> shift) & 255u : 256u;
      d8[j] = d;
      const uint64_t active = ballot64(valid);
      const uint64_t m = match_digit(d & 255u, active);
      if (valid) {
        const uint32_t before = wcnt[wave][d];
        r8[j] = before + (uint32_t)__popcll(m & lt);
        if ((m & lt) == 0ull) wcnt[wave][d] = before + (uint32_t)__popcll(m);
      }
    }
    __syncthreads();
    // Per digit t: tile total, cross-wave prefix, tile-local start.
    const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
    const uint32_t ttot = c0 + c1 + c2 + c3;
    uint32_t tall;
    const uint32_t st = block_exclusive_scan(ttot, sm, tall);
    tstart[t] = st;
    wcnt[0][t] = st;
    wcnt[1][t] = st + c0;
    wcnt[2][t] = st + c0 + c1;
    wcnt[3][t] = st + c0 + c1 + c2;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (d8[j] < 256u) {
        const uint32_t pos = wcnt[wave][d8[j]] + r8[j];
        if (pos < (uint32_t)kSortTile) {
          skey[pos] = k8[j];
          sval[pos] = v8[j];
        }
      }
    }
    __syncthreads();
    const int nvalid = (int)((hi - base) < kSortTile ? (hi - base) : kSortTile);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int p = j * kBlock + t;
      if (p < nvalid) {
        const unsigned long long k = skey[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t out = running[d] + (uint32_t)p - tstart[d];
        if ((int64_t)out < D) {
          kout[out] = k;
          vout[out] = sval[p];
        }
      }
    }
    __syncthreads();
    running[t] += ttot;
    __syncthreads();
  }
}

hipError_t launch_radix_sort(const Layout& L, void* ws, const DupLayout& D, void* dup, hipStream_t s) {
  char* w = (char*)ws;
  char* dp = (char*)dup;
  const unsigned long long* hdr = (const unsigned long long*)(w + L.hdr);
  const int G = sort_blocks(D.cap);
  const int passes = sort_passes(L.tiles_total);
  unsigned long long* k[2] = {(unsigned long long*)(dp + D.keys0), (unsigned long long*)(dp + D.keys1)};
  uint32_t* v[2] = {(uint32_t*)(dp + D.vals0), (uint32_t*)(dp + D.vals1)};
  uint32_t* hist = (uint32_t*)(dp + D.hist);
  for (int p = 0; p < passes; ++p) {
    const int src = p & 1, dst = src ^ 1;
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_upsweep, dim3(G), dim3(kBlock), 0, s, k[src], hdr, G, shift, hist);
    hipLaunchKernelGGL(k_radix_digit_scan, dim3(256), dim3(kBlock), 0, s, hist, G, hdr);
    hipLaunchKernelGGL(k_radix_downsweep, dim3(G), dim3(kBlock), 0, s, k[src], v[src], k[dst], v[dst],
                       hist, hdr, G, shift);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- ranges
__global__ __launch_bounds__(kBlock) void k_ranges(const unsigned long long* __restrict__ keys,
                                                   const unsigned long long* __restrict__ hdr,
                                                   uint32_t tiles_total, uint2* __restrict__ ranges) {
  if (hdr[kHdrOverflow]) return;
  const int64_t D = (int64_t)hdr[kHdrDup];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < D; i += (int64_t)gridDim.x * kBlock) {
    const uint32_t t = (uint32_t)(keys[i] >> 32);
    if (t >= tiles_total) continue;
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[t].x = (uint32_t)i;
    if (i == D - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[t].y = (uint32_t)(i + 1);
  }
}

// Longest-list-first order of the tiles (by bit length of the list, ties in any order):
// the blend's running time is dominated by long lists, and starting them first keeps the
// end of the launch from being a few long tiles on an otherwise idle chip.  One block.
__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, uint32_t tiles,
                                                     const unsigned long long* __restrict__ hdr,
                                                     uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[33];
  __shared__ uint32_t off[33];
  if (threadIdx.x < 33) cnt[threadIdx.x] = 0;
  __syncthreads();
  const bool ovf = hdr[kHdrOverflow] != 0ull;
  for (uint32_t t = threadIdx.x; t < tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    const uint32_t len = ovf ? 0u : r.y - r.x;
    atomicAdd(&cnt[len ? 32 - __clz(len) : 0], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 32; b >= 0; --b) { off[b] = run; run += cnt[b]; }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    const uint32_t len = ovf ? 0u : r.y - r.x;
    const uint32_t pos = atomicAdd(&off[len ? 32 - __clz(len) : 0], 1u);
    order[pos] = t;
  }
}

hipError_t launch_ranges(const Layout& L, void* ws, const DupLayout& D, void* dup, int parity,
                         hipStream_t s) {
  char* w = (char*)ws;
  char* dp = (char*)dup;
  hipError_t e = launch_fill_u32((uint32_t*)(w + L.ranges), 0u, 2 * (int64_t)L.tiles_total, s);
  if (e != hipSuccess) return e;
  const unsigned long long* keys = (const unsigned long long*)(dp + (parity ? D.keys1 : D.keys0));
  int64_t g = (D.cap + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)g), dim3(kBlock), 0, s, keys,
                     (const unsigned long long*)(w + L.hdr), L.tiles_total, (uint2*)(w + L.ranges));
  if (L.tiles_total > 0)
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, (const uint2*)(w + L.ranges), L.tiles_total,
                       (const unsigned long long*)(w + L.hdr), (uint32_t*)(w + L.order));
  return hipGetLastError();
}

}  // namespace clod
