// Tile binning (Sec. 3.1, splats sorted by depth per tile).  The order produced is the
// stable order of the keys (tile << 32 | bits(depth)) emitted per rendered (view, Gaussian)
// in index order, i.e. (tile, depth, index); it is built in two sorts that move far fewer
// bytes than one sort of the 64-bit pair keys:
//
//   1. compaction of the rendered records f = v*n + i in index order, keyed by bits(depth);
//   2. stable LSD radix sort of these R records by their 32-bit depth key;
//   3. emission, in that depth order, of one (tile id, f) pair per covered tile (a
//      load-balanced expansion over equal output chunks: every store is coalesced);
//   4. stable LSD radix sort of the D pairs by the tile id only.
//
// Step 4 is stable and its input is in (depth, index) order within every tile, so the result
// is ordered by (tile, depth, index), exactly the order of the single 64-bit sort.  Rendered
// records each cover at least one tile, so R <= D and the record sort runs inside the pair
// buffers.  Everything is device-driven: R and D live in the workspace header and every kernel
// reads them, so no host synchronisation is needed between the stages and the whole sequence
// can be captured in a graph.
#include "clod_internal.h"

namespace clod {

// Loads a chunk of kScanChunk uint32 counts (coalesced) into LDS and replaces them by their
// block-exclusive offsets (blocked: thread t owns items t*16 .. t*16+15).  Returns the total.
__device__ __forceinline__ uint32_t chunk_offsets(uint32_t* loff, uint32_t* sm, uint32_t (&loc)[kScanItems]) {
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = loff[threadIdx.x * kScanItems + k];
    s += loc[k];
  }
  uint32_t total;
  uint32_t off = block_exclusive_scan(s, sm, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loff[threadIdx.x * kScanItems + k] = off;
    off += loc[k];
  }
  __syncthreads();
  return total;
}

// Largest k with loff[k] <= o (loff[0] = 0 <= o); with o below the chunk total this is the
// item that output o belongs to (items with no outputs share their successor's offset).
__device__ __forceinline__ int owner_of(const uint32_t* loff, uint32_t o) {
  int lo = 0, hi = kScanChunk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (loff[mid] <= o) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ step 1: counts and compaction
// The rendered records are the (view, Gaussian) pairs whose flag byte has bit 2 set (the
// projection sets it exactly where it writes a tile rectangle).  Thread t of a block owns the
// 16 records [base + 16t, base + 16t + 16) and reads their flags in one 16-byte load; the
// result is a 16-bit mask, bit k = record base + 16t + k is rendered.
__device__ __forceinline__ uint32_t rendered_mask(const uint8_t* __restrict__ flags, int64_t count, int64_t j0) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if (j0 + 16 <= count) {
    const uint4 q = *reinterpret_cast<const uint4*>(flags + j0);
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else {
    for (int k = 0; k < 16 && j0 + k < count; ++k) w[k >> 2] |= (uint32_t)flags[j0 + k] << (8 * (k & 3));
  }
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t b = (w[q] >> 2) & 0x01010101u;   // bit 2 of each byte, at bits 0, 8, 16, 24
    m |= ((b | (b >> 7) | (b >> 14) | (b >> 21)) & 0xFu) << (4 * q);
  }
  return m;
}

// Single block: exclusive scan of the per-chunk rendered counts; R and the overflow flag (R
// above the capacity) to the header.  D is not known yet: k_emit_partials stores it.  Also
// clears the counters of the tile ordering (tord).
__device__ __forceinline__ void scan_partials_body(const ScanPartialsArgs& a, Blk) {
  __shared__ uint32_t sm[4];
  uint32_t* __restrict__ partR = a.partR;
  const int nparts = a.nparts;
  unsigned long long* __restrict__ hdr = a.hdr;
  const int64_t cap = a.cap;
  uint32_t* __restrict__ tord = a.tord;
  if (threadIdx.x < kTileOrderWords) tord[threadIdx.x] = 0u;
  uint32_t carry = 0;
  // kScanItems consecutive partials per thread per round (one block scan per round).
  for (int base = 0; base < nparts; base += kScanChunk) {
    const int j0 = base + (int)threadIdx.x * kScanItems;
    uint32_t r[kScanItems];
    uint32_t sr = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      r[k] = j0 + k < nparts ? partR[j0 + k] : 0u;
      sr += r[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(sr, sm, tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (j0 + k < nparts) partR[j0 + k] = carry + ex;
      ex += r[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    hdr[kHdrDup] = 0ull;
    hdr[kHdrOverflow] = (int64_t)carry > cap ? 1ull : 0ull;
    hdr[kHdrRend] = carry;
  }
}
__global__ __launch_bounds__(kBlock) void k_scan_partials(ScanPartialsArgs a) { scan_partials_body(a, grid_blk()); }

// Per chunk of kScanChunk records: the number of rendered records.  Also clears the per-tile
// ranges (2 * tiles words) for k_ranges, which writes only the non-empty tiles.
__device__ __forceinline__ void scan_reduce_body(const ScanReduceArgs& a, Blk b) {
  __shared__ uint32_t sm[4];
  for (int64_t q = (int64_t)b.id * kBlock + threadIdx.x; q < a.range_words; q += (int64_t)b.n * kBlock)
    a.ranges[q] = 0u;
  const int64_t j0 = (int64_t)b.id * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  const uint32_t r = wave_sum((uint32_t)__popc(rendered_mask(a.flags, a.count, j0)));
  if (lane_id() == 0) sm[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) a.partR[b.id] = sm[0] + sm[1] + sm[2] + sm[3];
}
__global__ __launch_bounds__(kBlock) void k_scan_reduce(ScanReduceArgs a) { scan_reduce_body(a, grid_blk()); }

// Rendered records of the chunk, in index order, to [partR[b], ...): key bits(depth), value f.
// The depth gathers (one per rendered record, from the record's fourth quad) are issued right
// after the flag load, so their latency overlaps the block scan; keys and indices are then
// placed in LDS so the stores are coalesced.
struct CompactLds {
  uint32_t sk[kScanChunk], sf[kScanChunk];
};
__device__ __forceinline__ void compact_body(const CompactArgs& a, Blk b, CompactLds& S) {
  __shared__ uint32_t sm[4];
  uint32_t* sk = S.sk;
  uint32_t* sf = S.sf;
  const uint8_t* __restrict__ flags = a.flags;
  const int64_t count = a.count;
  const float4* __restrict__ rec = a.rec;
  uint32_t* __restrict__ kout = a.kout;
  uint32_t* __restrict__ vout = a.vout;
  if (a.hdr[kHdrOverflow] != 0ull) return;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)b.id * kScanChunk;
  const int64_t j0 = base + (int64_t)t * kScanItems;
  const uint32_t m = rendered_mask(flags, count, j0);
  uint32_t dk[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    dk[k] = ((m >> k) & 1u) ? __float_as_uint(rec[kRecQuads * (j0 + k) + 3].x) : 0u;   // camera depth
  uint32_t total;
  uint32_t o = block_exclusive_scan((uint32_t)__popc(m), sm, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if ((m >> k) & 1u) {
      sk[o] = dk[k];
      sf[o] = (uint32_t)(j0 + k);
      ++o;
    }
  }
  __syncthreads();
  const int64_t out0 = (int64_t)a.partR[b.id];
  for (uint32_t q = (uint32_t)t; q < total; q += kBlock) {
    kout[out0 + q] = sk[q];
    vout[out0 + q] = sf[q];
  }
}
__global__ __launch_bounds__(kBlock) void k_compact(CompactArgs a) {
  __shared__ CompactLds S;
  compact_body(a, grid_blk(), S);
}

// ---------------------------------------------------------------------------- radix sort
// Reduce-then-scan LSD radix sort of (uint32 key, uint32 value) pairs with 8-bit digits; the
// element count is header word `cw`.  Block b of G owns the contiguous chunk
// [b*C, (b+1)*C) (C a multiple of the 2048-key tile), so the stable order across blocks is the
// block order.

__device__ __forceinline__ void sort_chunk(int64_t N, int G, int b, int64_t& lo, int64_t& hi) {
  const int64_t tiles_total = (N + kSortTile - 1) / kSortTile;
  const int64_t per = (tiles_total + G - 1) / G;
  lo = (int64_t)b * per * kSortTile;
  hi = lo + per * kSortTile;
  if (lo > N) lo = N;
  if (hi > N) hi = N;
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

// Digit counts per 16-lane group of each wave (16 copies, rows padded to 257 words): lanes
// of one atomic instruction that share a digit serialise on its address, and high digits
// take few values, so splitting the wave four ways shortens those chains.
struct UpsweepLds {
  uint32_t cnt[16][257];
};
__device__ __forceinline__ void radix_upsweep_body(const RadixArgs& a, Blk b, UpsweepLds& S) {
  auto& cnt = S.cnt;
  const uint32_t* __restrict__ keys = a.kin;
  const unsigned long long* __restrict__ hdr = a.hdr;
  const int G = a.G, shift = a.shift;
  uint32_t* __restrict__ hist = a.hist;
  if (hdr[kHdrOverflow]) return;
  const int64_t N = (int64_t)hdr[a.cw];
  const int t = threadIdx.x;
  const int copy = t >> 4;
  for (int j = t; j < 16 * 257; j += kBlock) (&cnt[0][0])[j] = 0;
  __syncthreads();
  int64_t lo, hi;
  sort_chunk(N, G, (int)b.id, lo, hi);
  // kSortItems keys per thread per step, all loads issued before any is used.
  for (int64_t base = lo; base < hi; base += kSortTile) {
    uint32_t d8[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t idx = base + (int64_t)j * kBlock + t;
      d8[j] = idx < hi ? (keys[idx] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
      if (d8[j] < 256u) atomicAdd(&cnt[copy][d8[j]], 1u);
  }
  __syncthreads();
  uint32_t total = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) total += cnt[c][t];
  hist[(int64_t)t * G + b.id] = total;
}
__global__ __launch_bounds__(kBlock) void k_radix_upsweep(RadixArgs a) {
  __shared__ UpsweepLds S;
  radix_upsweep_body(a, grid_blk(), S);
}

// Block d: exclusive scan of digit d's per-block counts hist[d*G .. d*G+G) in place, and
// the digit total in hist[256*G + d].
__device__ __forceinline__ void radix_digit_scan_body(const RadixArgs& a, Blk b) {
  __shared__ uint32_t sm[4];
  uint32_t* __restrict__ hist = a.hist;
  const int G = a.G;
  if (a.hdr[kHdrOverflow]) return;
  uint32_t* h = hist + (int64_t)b.id * G;
  uint32_t carry = 0;
  for (int base = 0; base < G; base += kBlock) {
    const int j = base + threadIdx.x;
    const uint32_t v = j < G ? h[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sm, tot);
    if (j < G) h[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) hist[(int64_t)256 * G + b.id] = carry;
}
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(RadixArgs a) { radix_digit_scan_body(a, grid_blk()); }

struct DownsweepLds {
  uint32_t running[256];      // global output position of the next key per digit
  uint32_t wcnt[4][256];      // per-wave digit counts within the tile
  uint32_t tstart[256];       // tile-local start of each digit
  uint32_t skey[kSortTile];
  uint32_t sval[kSortTile];
};
__device__ __forceinline__ void radix_downsweep_body(const RadixArgs& a, Blk b, DownsweepLds& S) {
  __shared__ uint32_t sm[4];
  auto& running = S.running;
  auto& wcnt = S.wcnt;
  auto& tstart = S.tstart;
  auto& skey = S.skey;
  auto& sval = S.sval;
  const uint32_t* __restrict__ kin = a.kin;
  const uint32_t* __restrict__ vin = a.vin;
  uint32_t* __restrict__ kout = a.kout;
  uint32_t* __restrict__ vout = a.vout;
  const uint32_t* __restrict__ hist = a.hist;
  const unsigned long long* __restrict__ hdr = a.hdr;
  const int G = a.G, shift = a.shift;
  if (hdr[kHdrOverflow]) return;
  const int64_t N = (int64_t)hdr[a.cw];
  int64_t lo, hi;
  sort_chunk(N, G, (int)b.id, lo, hi);
  const int t = threadIdx.x;
  const int wave = t >> 6;
  const uint32_t lane = lane_id();
  {
    uint32_t tall;
    const uint32_t digit_base = block_exclusive_scan(hist[(int64_t)256 * G + t], sm, tall);
    running[t] = digit_base + hist[(int64_t)t * G + b.id];
  }
  const uint64_t lt = lanemask_lt();
  for (int64_t base = lo; base < hi; base += kSortTile) {
    wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
    __syncthreads();
    uint32_t k8[kSortItems], v8[kSortItems], d8[kSortItems], r8[kSortItems];
    // Wave w owns keys [base + w*512, base + (w+1)*512), slot j holds base + w*512 + j*64 + lane.
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t idx = base + (int64_t)wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < hi;
      k8[j] = valid ? kin[idx] : 0u;
      v8[j] = valid ? vin[idx] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t idx = base + (int64_t)wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < hi;
      const uint32_t d = valid ? (k8[j] >> shift) & 255u : 256u;
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
        const uint32_t k = skey[p];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t out = running[d] + (uint32_t)p - tstart[d];
        if ((int64_t)out < N) {
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
__global__ __launch_bounds__(kBlock) void k_radix_downsweep(RadixArgs a) {
  __shared__ DownsweepLds S;
  radix_downsweep_body(a, grid_blk(), S);
}

static hipError_t radix_passes(const unsigned long long* hdr, int cw, int G, int first_shift, int passes,
                               uint32_t* const k[2], uint32_t* const v[2], int src0, uint32_t* hist, const Sink& out) {
  for (int p = 0; p < passes; ++p) {
    const int src = (src0 + p) & 1, dst = src ^ 1;
    Stage st{};
    st.block = kBlock;
    st.a.radix = RadixArgs{k[src], v[src], k[dst], v[dst], hist, hdr, cw, G, first_shift + 8 * p};
    st.kind = kStRadixUp;
    st.items = (uint32_t)G;
    hipError_t e = out.put(st);
    st.kind = kStRadixScan;
    st.items = 256;
    if (e == hipSuccess) e = out.put(st);
    st.kind = kStRadixDown;
    st.items = (uint32_t)G;
    if (e == hipSuccess) e = out.put(st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- step 3: ordered emission
// Tiles touched by record f (the last word of its fourth quad).
__device__ __forceinline__ uint32_t rec_tiles(const float4* __restrict__ rec, uint32_t f) {
  return __float_as_uint(rec[kRecQuads * (int64_t)f + 3].w);
}

// Single block: D (summed in 64 bits) and the overflow flag (D above the capacity) to the
// header, and, unless overflowed, the exclusive scan of the chunk totals in place.
__device__ __forceinline__ void emit_partials_body(const EmitPartialsArgs& a, Blk) {
  __shared__ unsigned long long sm[4];
  uint32_t* __restrict__ partE = a.partE;
  unsigned long long* __restrict__ hdr = a.hdr;
  const int nb = a.nb;
  const int64_t cap = a.cap;
  const bool over = hdr[kHdrOverflow] != 0ull;
  const int nparts = over ? nb : (int)(((int64_t)hdr[kHdrRend] + kScanChunk - 1) / kScanChunk);
  const uint32_t lane = lane_id();
  const int wave = threadIdx.x >> 6;
  unsigned long long carry = 0;
  for (int base = 0; base < nparts; base += kBlock) {
    const int j = base + threadIdx.x;
    const unsigned long long v = j < nparts ? partE[j] : 0ull;
    unsigned long long inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long up = __shfl_up(inc, o, 64);
      if (lane >= (uint32_t)o) inc += up;
    }
    if (lane == 63) sm[wave] = inc;
    __syncthreads();
    unsigned long long wb = 0;
    for (int w = 0; w < wave; ++w) wb += sm[w];
    const unsigned long long tot = sm[0] + sm[1] + sm[2] + sm[3];
    __syncthreads();
    if (!over && j < nparts) partE[j] = (uint32_t)(carry + wb + inc - v);
    carry += tot;
  }
  if (threadIdx.x == 0) {
    hdr[kHdrDup] = carry;
    if ((int64_t)carry > cap) hdr[kHdrOverflow] = 1ull;
  }
}
__global__ __launch_bounds__(kBlock) void k_emit_partials(EmitPartialsArgs a) { emit_partials_body(a, grid_blk()); }

// Per chunk of the depth-sorted records: tile pairs of the chunk (saturated at 2^32 - 1,
// which only a total far beyond any capacity reaches); the gathered counts are also stored in
// sorted order (tsorted) for k_emit_offsets.  If R alone exceeded the capacity
// (the only way the overflow flag can be set at this point) the records were never sorted;
// the pair count is then summed over chunk b of all records instead, so that D is still
// reported.
__device__ __forceinline__ void emit_reduce_body(const EmitReduceArgs& a, Blk b) {
  __shared__ unsigned long long sm[4];
  const uint32_t* __restrict__ sorted_f = a.sorted_f;
  const float4* __restrict__ rec = a.rec;
  const uint8_t* __restrict__ flags = a.flags;
  const int64_t count = a.count;
  const unsigned long long* __restrict__ hdr = a.hdr;
  uint32_t* __restrict__ tsorted = a.tsorted;
  const bool over = hdr[kHdrOverflow] != 0ull;
  const int64_t R = (int64_t)hdr[kHdrRend];
  const int64_t base = (int64_t)b.id * kScanChunk;
  if (!over && base >= R) return;
  unsigned long long s = 0;
  if (!over) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
      if (j < R) {
        const uint32_t c = rec_tiles(rec, sorted_f[j]);
        tsorted[j] = c;
        s += c;
      }
    }
  } else {
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
      if (j < count && (flags[j] & 4u)) s += rec_tiles(rec, (uint32_t)j);
    }
  }
  s = wave_sum(s);
  if (lane_id() == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long c = sm[0] + sm[1] + sm[2] + sm[3];
    a.partE[b.id] = c > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)c;
  }
}
__global__ __launch_bounds__(kBlock) void k_emit_reduce(EmitReduceArgs a) { emit_reduce_body(a, grid_blk()); }

// Per chunk of the depth-sorted records: each record's first output position (the global
// exclusive scan of their tile counts, over the R positions of the record keys, which the
// sort no longer needs), and for every output chunk of kEmitTile pairs the record that owns
// its first position.
struct OffsetsLds {
  uint32_t loff[kScanChunk];
};
__device__ __forceinline__ void emit_offsets_body(const EmitOffsetsArgs& a, Blk b, OffsetsLds& S) {
  __shared__ uint32_t sm[4];
  uint32_t* loff = S.loff;
  const uint32_t* __restrict__ tsorted = a.tsorted;
  const unsigned long long* __restrict__ hdr = a.hdr;
  uint32_t* __restrict__ eoff = a.eoff;
  uint32_t* __restrict__ owner = a.owner;
  if (hdr[kHdrOverflow] != 0ull) return;
  const int64_t R = (int64_t)hdr[kHdrRend];
  const int64_t base = (int64_t)b.id * kScanChunk;
  if (base >= R) return;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + t;
    loff[k * kBlock + t] = j < R ? tsorted[j] : 0u;
  }
  uint32_t loc[kScanItems];
  const uint32_t total = chunk_offsets(loff, sm, loc);
  const uint32_t cb = a.partE[b.id];
  for (int i = t; i < kScanChunk; i += kBlock) {
    const int64_t j = base + i;
    if (j >= R) break;
    const uint32_t first = cb + loff[i];
    const uint32_t end = cb + (i + 1 < kScanChunk ? loff[i + 1] : total);
    eoff[j] = first;
    for (uint32_t q = (first + kEmitTile - 1) / kEmitTile; q * (uint64_t)kEmitTile < end; ++q) owner[q] = (uint32_t)j;
  }
}
__global__ __launch_bounds__(kBlock) void k_emit_offsets(EmitOffsetsArgs a) {
  __shared__ OffsetsLds S;
  emit_offsets_body(a, grid_blk(), S);
}

// Output chunk q (pairs [q*M, q*M + M), M = kEmitTile) is produced by the records between
// the owner of its first pair and the owner of the next chunk's first pair (at most M + 1
// of them, since every record has at least one pair).  Each of them is staged in LDS once:
// its first output offset, its index f, the id of the first tile of its rectangle, the
// rectangle width, the view's tile row length and 1/width.  Pair o belongs to the last staged
// record whose offset is <= o, as that record's (o - offset)-th covered tile in row-major
// order.  Chunks are equal-sized whatever the rectangle sizes, and every store is coalesced.
constexpr int kEmitPer = kEmitTile / kBlock;   // consecutive pairs per thread
static_assert(kEmitPer == 8, "the stores below write eight pairs per thread");
struct EmitLds {
  uint32_t se[kEmitTile + 1];
  uint32_t sf[kEmitTile + 1];
  uint32_t sb[kEmitTile + 1];   // tile id of the rectangle's first tile
  uint32_t sw[kEmitTile + 1];   // width | tiles_x << 16
  float sr[kEmitTile + 1];      // 1 / width
};
__device__ __forceinline__ void emit_body(const EmitArgs& a, Blk b, EmitLds& S) {
  auto& se = S.se;
  auto& sf = S.sf;
  auto& sb = S.sb;
  auto& sw = S.sw;
  auto& sr = S.sr;
  const uint32_t* __restrict__ sorted_f = a.sorted_f;
  const uint32_t* __restrict__ eoff = a.eoff;
  const uint32_t* __restrict__ owner = a.owner;
  const float4* __restrict__ rec = a.rec;
  const DevView* __restrict__ views = a.views;
  const int64_t n = a.n;
  const unsigned long long* __restrict__ hdr = a.hdr;
  uint32_t* __restrict__ kout = a.kout;
  uint32_t* __restrict__ vout = a.vout;
  if (hdr[kHdrOverflow] != 0ull) return;
  const int64_t R = (int64_t)hdr[kHdrRend];
  const int64_t D = (int64_t)hdr[kHdrDup];
  const int64_t nch = (D + kEmitTile - 1) / kEmitTile;
  const uint32_t nn = (uint32_t)n;
  for (int64_t q = b.id; q < nch; q += b.n) {
    const int64_t k0 = owner[q];
    const int64_t k1 = q + 1 < nch ? (int64_t)owner[q + 1] : R - 1;
    int cnt = (int)(k1 - k0 + 1);
    if (cnt > kEmitTile + 1) cnt = kEmitTile + 1;   // cannot happen (see above); keeps LDS in bounds
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
      const uint32_t f = sorted_f[k0 + i];
      const DevView& Vw = views[f / nn];
      const float4 q3 = rec[kRecQuads * (int64_t)f + 3];
      const uint32_t rx = __float_as_uint(q3.y), ry = __float_as_uint(q3.z);
      const uint32_t x0 = rx & 0xFFFFu, x1 = rx >> 16, y0 = ry & 0xFFFFu;
      const uint32_t w = x1 - x0, tx = (uint32_t)Vw.tiles_x;
      se[i] = eoff[k0 + i];
      sf[i] = f;
      sb[i] = Vw.tile_base + y0 * tx + x0;
      sw[i] = w | (tx << 16);
      sr[i] = 1.0f / (float)w;
    }
    __syncthreads();
    // Thread t writes the eight consecutive pairs [o0 + 8t, o0 + 8t + 8): one search for the
    // first, then a walk that steps the tile column (and row) and, at a record's end, moves
    // to the next record (each record has at least one pair, so one step never skips one).
    const int64_t o0 = q * kEmitTile;
    const int64_t o1 = o0 + kEmitTile < D ? o0 + kEmitTile : D;
    const int64_t ob = o0 + (int64_t)threadIdx.x * kEmitPer;
    if (ob < o1) {
      const uint32_t o = (uint32_t)ob;
      int lo = 0, hi = cnt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (se[mid] <= o) lo = mid; else hi = mid - 1;
      }
      const uint32_t rel = o - se[lo];
      uint32_t wx = sw[lo];
      uint32_t w = wx & 0xFFFFu;
      // Row of the first pair: rel / w from the rounded reciprocal (off by at most one for
      // quotients below 2^16, as rectangle rows are), then corrected exactly.
      uint32_t ty = (uint32_t)((float)rel * sr[lo]);
      int32_t rem = (int32_t)(rel - ty * w);
      if (rem < 0) { --ty; rem += (int32_t)w; }
      else if (rem >= (int32_t)w) { ++ty; rem -= (int32_t)w; }
      uint32_t tx = (uint32_t)rem;
      uint32_t next = lo + 1 < cnt ? se[lo + 1] : 0xFFFFFFFFu;
      uint32_t key[kEmitPer], val[kEmitPer];
#pragma unroll
      for (int k = 0; k < kEmitPer; ++k) {
        if ((uint32_t)(o + k) == next) {   // the next record starts here
          ++lo;
          wx = sw[lo];
          w = wx & 0xFFFFu;
          tx = 0;
          ty = 0;
          next = lo + 1 < cnt ? se[lo + 1] : 0xFFFFFFFFu;
        }
        key[k] = sb[lo] + ty * (wx >> 16) + tx;
        val[k] = sf[lo];
        if (++tx == w) { tx = 0; ++ty; }
      }
      if (ob + kEmitPer <= o1) {
        uint4* kq = reinterpret_cast<uint4*>(kout + ob);
        uint4* vq = reinterpret_cast<uint4*>(vout + ob);
        kq[0] = make_uint4(key[0], key[1], key[2], key[3]);
        kq[1] = make_uint4(key[4], key[5], key[6], key[7]);
        vq[0] = make_uint4(val[0], val[1], val[2], val[3]);
        vq[1] = make_uint4(val[4], val[5], val[6], val[7]);
      } else {
#pragma unroll
        for (int k = 0; k < kEmitPer; ++k)
          if (ob + k < o1) { kout[ob + k] = key[k]; vout[ob + k] = val[k]; }
      }
    }
    __syncthreads();
  }
}
__global__ __launch_bounds__(kBlock) void k_emit(EmitArgs a) {
  __shared__ EmitLds S;
  emit_body(a, grid_blk(), S);
}

int tile_passes(uint32_t tiles_total) {
  int tb = 0;
  uint32_t m = tiles_total > 0 ? tiles_total - 1 : 0;
  while (m) { ++tb; m >>= 1; }
  return (tb + 7) / 8;
}

int sorted_buffer(uint32_t tiles_total) { return (tile_passes(tiles_total) & 1) ? 0 : 1; }

hipError_t launch_bin_sort(const Layout& L, void* ws, const DupLayout& D, void* dup, const Sink& out) {
  char* w = (char*)ws;
  char* dp = (char*)dup;
  unsigned long long* hdr = (unsigned long long*)(w + L.hdr);
  uint32_t* const k[2] = {(uint32_t*)(dp + D.keys0), (uint32_t*)(dp + D.keys1)};
  uint32_t* const v[2] = {(uint32_t*)(dp + D.vals0), (uint32_t*)(dp + D.vals1)};
  uint32_t* hist = (uint32_t*)(dp + D.hist);
  const int nb = L.scan_blocks;
  uint32_t* ranges = (uint32_t*)(w + L.ranges);
  uint32_t* tord = (uint32_t*)(w + L.tord);
  if (nb == 0) {
    hipError_t e = launch_fill_u32((uint32_t*)hdr, 0u, 2 * kHdrWords, out);
    if (e == hipSuccess) e = launch_fill_u32(ranges, 0u, 2 * (int64_t)L.tiles_total, out);
    if (e == hipSuccess) e = launch_fill_u32(tord, 0u, kTileOrderWords, out);
    return e;
  }
  uint32_t* partR = (uint32_t*)(w + L.scan_part);
  uint32_t* partE = partR + (nb + 1);
  const uint8_t* flags = (const uint8_t*)(w + L.flags);
  const float4* rec = (const float4*)(w + L.rec);
  const int G = sort_blocks(D.cap);
  Stage st{};
  st.block = kBlock;
  hipError_t e = hipSuccess;
  auto put = [&](int32_t kind, int64_t items) {
    st.kind = kind;
    st.items = (uint32_t)items;
    if (e == hipSuccess) e = out.put(st);
  };
  // 1. R and its overflow; compaction of the rendered records into buffer 0.
  st.a.scan_reduce = ScanReduceArgs{flags, L.VN, partR, ranges, 2 * (int64_t)L.tiles_total};
  put(kStScanReduce, nb);
  st.a.scan_partials = ScanPartialsArgs{partR, nb, hdr, D.cap, tord};
  put(kStScanPartials, 1);
  st.a.compact = CompactArgs{flags, L.VN, (const uint32_t*)partR, rec, (const unsigned long long*)hdr, k[0], v[0]};
  put(kStCompact, nb);
  // 2. depth sort of the R records: 4 passes, back in buffer 0.
  if (e == hipSuccess) e = radix_passes(hdr, kHdrRend, G, 0, 4, k, v, 0, hist, out);
  // 3. emission in depth order into buffer 1.
  // The emission output buffer 1 holds the sorted tile counts until k_emit overwrites it.
  st.a.emit_reduce = EmitReduceArgs{(const uint32_t*)v[0], rec, flags, L.VN, (const unsigned long long*)hdr, partE, k[1]};
  put(kStEmitReduce, nb);
  st.a.emit_partials = EmitPartialsArgs{partE, hdr, nb, D.cap};
  put(kStEmitPartials, 1);
  uint32_t* owner = (uint32_t*)(dp + D.owner);
  st.a.emit_offsets = EmitOffsetsArgs{(const uint32_t*)k[1], (const uint32_t*)partE, (const unsigned long long*)hdr,
                                      k[0], owner};
  put(kStEmitOffsets, nb);
  int64_t ge = (D.cap + kEmitTile - 1) / kEmitTile;
  if (ge > 4096) ge = 4096;
  if (ge < 1) ge = 1;
  st.a.emit = EmitArgs{(const uint32_t*)v[0], (const uint32_t*)k[0], (const uint32_t*)owner, rec,
                       (const DevView*)(w + L.vinfo), L.n, (const unsigned long long*)hdr, k[1], v[1]};
  put(kStEmit, ge);
  // 4. stable sort of the D pairs by tile id.
  if (e == hipSuccess) e = radix_passes(hdr, kHdrDup, G, 0, tile_passes(L.tiles_total), k, v, 1, hist, out);
  return e;
}

// ---------------------------------------------------------------------------- ranges
__device__ __forceinline__ void ranges_body(const RangesArgs& a, Blk b) {
  constexpr uint32_t kNone = 0xFFFFFFFFu;   // no neighbour (never a tile id)
  const uint32_t* __restrict__ keys = a.keys;
  const uint32_t tiles_total = a.tiles_total;
  uint2* __restrict__ ranges = a.ranges;
  if (a.hdr[kHdrOverflow]) return;
  const int64_t D = (int64_t)a.hdr[kHdrDup];
  // Four consecutive keys per thread (one 16-byte load), plus the key before and after.
  for (int64_t i0 = 4 * ((int64_t)b.id * kBlock + threadIdx.x); i0 < D; i0 += 4 * (int64_t)b.n * kBlock) {
    uint32_t k[6];
    k[0] = i0 > 0 ? keys[i0 - 1] : kNone;
    if (i0 + 4 <= D) {
      const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
      k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) k[j + 1] = i0 + j < D ? keys[i0 + j] : kNone;
    }
    k[5] = i0 + 4 < D ? keys[i0 + 4] : kNone;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = k[j + 1];
      if (t >= tiles_total) continue;   // also past the end (kNone)
      const int64_t i = i0 + j;
      if (k[j] != t) ranges[t].x = (uint32_t)i;
      if (k[j + 2] != t) ranges[t].y = (uint32_t)(i + 1);
    }
  }
}
__global__ __launch_bounds__(kBlock) void k_ranges(RangesArgs a) { ranges_body(a, grid_blk()); }

// Longest-list-first order of the tiles: a counting sort of the tiles by the bit length of
// their list length, longest first (order within a bucket is arbitrary: tiles are
// independent).  The blend's running time is dominated by long lists, and starting them first
// keeps the end of the launch from being a few long tiles on an otherwise idle chip.
__device__ __forceinline__ uint32_t len_bucket(const uint2 r, bool ovf) {
  const uint32_t len = ovf ? 0u : r.y - r.x;
  return len ? 32u - (uint32_t)__clz(len) : 0u;
}

// Bucket totals: per-block LDS counts, then one global atomic per non-empty bucket.
__device__ __forceinline__ void tile_count_body(const TileOrderArgs& a, Blk b) {
  __shared__ uint32_t cnt[kTileBuckets];
  const uint2* __restrict__ ranges = a.ranges;
  const uint32_t tiles = a.tiles;
  if (threadIdx.x < kTileBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  const bool ovf = a.hdr[kHdrOverflow] != 0ull;
  const uint32_t t0 = b.id * kTileOrderChunk;
  for (uint32_t t = t0 + threadIdx.x; t < tiles && t < t0 + kTileOrderChunk; t += kBlock)
    atomicAdd(&cnt[len_bucket(ranges[t], ovf)], 1u);
  __syncthreads();
  if (threadIdx.x < kTileBuckets && cnt[threadIdx.x]) atomicAdd(&a.tord[threadIdx.x], cnt[threadIdx.x]);
}
__global__ __launch_bounds__(kBlock) void k_tile_count(TileOrderArgs a) { tile_count_body(a, grid_blk()); }

// Scatter: bucket b starts after all longer buckets; each block reserves its slice of every
// bucket with one global atomic (tord[33 + b]) and places its tiles with LDS cursors.
__device__ __forceinline__ void tile_scatter_body(const TileOrderArgs& a, Blk blk) {
  __shared__ uint32_t cnt[kTileBuckets];
  __shared__ uint32_t cur[kTileBuckets];
  const uint2* __restrict__ ranges = a.ranges;
  const uint32_t tiles = a.tiles;
  uint32_t* __restrict__ tord = a.tord;
  uint32_t* __restrict__ order = a.order;
  if (threadIdx.x < kTileBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  const bool ovf = a.hdr[kHdrOverflow] != 0ull;
  const uint32_t t0 = blk.id * kTileOrderChunk;
  for (uint32_t t = t0 + threadIdx.x; t < tiles && t < t0 + kTileOrderChunk; t += kBlock)
    atomicAdd(&cnt[len_bucket(ranges[t], ovf)], 1u);
  __syncthreads();
  if (threadIdx.x < kTileBuckets) {
    const uint32_t b = threadIdx.x;
    uint32_t start = 0;
    for (uint32_t c = b + 1; c < (uint32_t)kTileBuckets; ++c) start += tord[c];
    cur[b] = cnt[b] ? start + atomicAdd(&tord[kTileBuckets + b], cnt[b]) : 0u;
    // The counts of the long and of the very long tiles (the starts of the first buckets below
    // them), for the blend.
    if (b == kLongBucket - 1 && blk.id == 0) tord[kTileLongWord] = start;
    if (b == kVeryLongBucket - 1 && blk.id == 0) tord[kTileVeryLongWord] = start;
  }
  __syncthreads();
  for (uint32_t t = t0 + threadIdx.x; t < tiles && t < t0 + kTileOrderChunk; t += kBlock) {
    const uint32_t pos = atomicAdd(&cur[len_bucket(ranges[t], ovf)], 1u);
    if (pos < tiles) order[pos] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_tile_scatter(TileOrderArgs a) { tile_scatter_body(a, grid_blk()); }

hipError_t launch_ranges(const Layout& L, void* ws, const DupLayout& D, void* dup, int parity, const Sink& out) {
  char* w = (char*)ws;
  char* dp = (char*)dup;
  // The ranges and the ordering counters were cleared by launch_bin_sort.
  const uint32_t* keys = (const uint32_t*)(dp + (parity ? D.keys1 : D.keys0));
  const unsigned long long* hdr = (const unsigned long long*)(w + L.hdr);
  int64_t g = (D.cap + 4 * kBlock - 1) / (4 * kBlock);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  Stage st{};
  st.block = kBlock;
  st.kind = kStRanges;
  st.items = (uint32_t)g;
  st.a.ranges = RangesArgs{keys, hdr, L.tiles_total, (uint2*)(w + L.ranges)};
  hipError_t e = out.put(st);
  if (e == hipSuccess && L.tiles_total > 0) {
    st.items = (L.tiles_total + kTileOrderChunk - 1) / kTileOrderChunk;
    st.a.tile_order = TileOrderArgs{(const uint2*)(w + L.ranges), L.tiles_total, hdr, (uint32_t*)(w + L.tord),
                                    (uint32_t*)(w + L.order)};
    st.kind = kStTileCount;
    e = out.put(st);
    st.kind = kStTileScatter;
    if (e == hipSuccess) e = out.put(st);
  }
  return e;
}

hipError_t launch_sort_stage(const Stage& st, hipStream_t s) {
  const dim3 g(st.items), blk(st.block);
  switch (st.kind) {
    case kStScanReduce: hipLaunchKernelGGL(k_scan_reduce, g, blk, 0, s, st.a.scan_reduce); break;
    case kStScanPartials: hipLaunchKernelGGL(k_scan_partials, g, blk, 0, s, st.a.scan_partials); break;
    case kStCompact: hipLaunchKernelGGL(k_compact, g, blk, 0, s, st.a.compact); break;
    case kStRadixUp: hipLaunchKernelGGL(k_radix_upsweep, g, blk, 0, s, st.a.radix); break;
    case kStRadixScan: hipLaunchKernelGGL(k_radix_digit_scan, g, blk, 0, s, st.a.radix); break;
    case kStRadixDown: hipLaunchKernelGGL(k_radix_downsweep, g, blk, 0, s, st.a.radix); break;
    case kStEmitReduce: hipLaunchKernelGGL(k_emit_reduce, g, blk, 0, s, st.a.emit_reduce); break;
    case kStEmitPartials: hipLaunchKernelGGL(k_emit_partials, g, blk, 0, s, st.a.emit_partials); break;
    case kStEmitOffsets: hipLaunchKernelGGL(k_emit_offsets, g, blk, 0, s, st.a.emit_offsets); break;
    case kStEmit: hipLaunchKernelGGL(k_emit, g, blk, 0, s, st.a.emit); break;
    case kStRanges: hipLaunchKernelGGL(k_ranges, g, blk, 0, s, st.a.ranges); break;
    case kStTileCount: hipLaunchKernelGGL(k_tile_count, g, blk, 0, s, st.a.tile_order); break;
    case kStTileScatter: hipLaunchKernelGGL(k_tile_scatter, g, blk, 0, s, st.a.tile_order); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------- scene preparation: spatial order
// A Morton (Z-order) permutation of a scene's Gaussians by their means, and the gather of every
// plane into that order.  Not a step of the per-frame path: a one-time preparation that puts
// Gaussians that are close in space close in memory, so that the records of neighbouring
// Gaussians (indexed view * n + Gaussian, 64 bytes, gathered by the blend in 128-byte lines)
// tend to serve the same tiles.

// Float bits mapped to an unsigned key of the same order, and back (the bounding box is kept as
// keys so that it can be reduced with integer atomics).
__device__ __forceinline__ uint32_t order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ float order_key_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}
// The 10 low bits of v moved to every third bit (bit b to bit 3b).
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Empty box (min keys all ones, max keys zero) and the sort header: count n, no overflow.
__global__ __launch_bounds__(64) void k_order_init(uint32_t* box, unsigned long long* hdr, int64_t n) {
  const int t = threadIdx.x;
  if (t < 3) box[t] = 0xFFFFFFFFu;
  else if (t < 6) box[t] = 0u;
  else if (t < 6 + kHdrWords) hdr[t - 6] = (t - 6 == kHdrRend) ? (unsigned long long)n : 0ull;
}

// Bounding box of the finite coordinates of the means (per axis, as order keys).
__global__ __launch_bounds__(kBlock) void k_order_box(const float* __restrict__ mean, int64_t n, uint32_t* box) {
  uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float x = mean[a * n + i];
      if (__builtin_isfinite(x)) {
        const uint32_t k = order_key(x);
        mn[a] = k < mn[a] ? k : mn[a];
        mx[a] = k > mx[a] ? k : mx[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t p = __shfl_xor(mn[a], o, 64), q = __shfl_xor(mx[a], o, 64);
      mn[a] = p < mn[a] ? p : mn[a];
      mx[a] = q > mx[a] ? q : mx[a];
    }
  }
  if (lane_id() == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(box + a, mn[a]);
      atomicMax(box + 3 + a, mx[a]);
    }
  }
}

// 30-bit Morton code of each mean (10 bits per axis over the box; x in the lowest bit) and the
// identity values.  Coordinates outside the box or not finite clamp to its faces; an axis with
// no extent contributes zero bits.
__global__ __launch_bounds__(kBlock) void k_order_codes(const float* __restrict__ mean, int64_t n,
                                                        const uint32_t* __restrict__ box, uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t code = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = order_key_inv(box[a]), hi = order_key_inv(box[3 + a]);
    const float ext = hi - lo;
    const float sc = ext > 0.0f ? 1024.0f / ext : 0.0f;
    const float q = fminf(fmaxf((mean[a * n + i] - lo) * sc, 0.0f), 1023.0f);
    code |= spread3((uint32_t)q) << a;
  }
  keys[i] = code;
  vals[i] = (uint32_t)i;
}

// Output position j of every plane takes the Gaussian perm[j].
__global__ __launch_bounds__(kBlock) void k_order_gather(OrderGatherArgs a) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= a.n) return;
  int64_t i = (int64_t)a.perm[j];
  if (i >= a.n) i = j;   // defensive: the sort emits a permutation of 0 .. n-1
  for (int p = 0; p < 6; ++p) {
    const float* __restrict__ src = a.src[p];
    float* __restrict__ dst = a.dst[p];
    for (int q = 0; q < a.planes[p]; ++q) dst[(int64_t)q * a.n + j] = src[(int64_t)q * a.n + i];
  }
}

hipError_t launch_scene_reorder(const clod_scene& src, const clod_scene_grad& dst, const OrderBufs& ob, hipStream_t s) {
  const int64_t n = src.n;
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_order_init, dim3(1), dim3(64), 0, s, ob.box, ob.hdr, n);
  hipLaunchKernelGGL(k_order_box, dim3(nb < 1024u ? nb : 1024u), dim3(kBlock), 0, s, src.mean, n, ob.box);
  hipLaunchKernelGGL(k_order_codes, dim3(nb), dim3(kBlock), 0, s, src.mean, n, (const uint32_t*)ob.box,
                     ob.keys[0], ob.vals[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Stable LSD sort of the 30-bit codes, four 8-bit passes, back in buffer 0 (vals[0] = perm).
  e = radix_passes(ob.hdr, kHdrRend, ob.G, 0, 4, ob.keys, ob.vals, 0, ob.hist, Sink(s));
  if (e != hipSuccess) return e;
  const int K = (src.sh_degree + 1) * (src.sh_degree + 1);
  OrderGatherArgs g{{src.mean, src.log_scale, src.quat, src.opacity, src.decay, src.sh},
                    {dst.mean, dst.log_scale, dst.quat, dst.opacity, dst.decay, dst.sh},
                    {3, 3, 4, 1, 1, 3 * K}, n, ob.vals[0]};
  hipLaunchKernelGGL(k_order_gather, dim3(nb), dim3(kBlock), 0, s, g);
  return hipGetLastError();
}

}  // namespace clod
