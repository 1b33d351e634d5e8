// Per-tile front-to-back blending (Sec. 3.1, Eq. (1)) and its adjoint.
//
// One 256-thread workgroup (4 wave64) per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1) and lane l its pixel (l & 7, l >> 3).  Entries of the tile's sorted list
// are staged in LDS (one per lane or thread, a coalesced gather of the records) and read back
// as LDS broadcasts; entries that provably cannot reach a quadrant are dropped for it (see
// quadrant_mask).  Blocks take tiles longest list first (the order clod_bin_sort computes),
// so the long tiles, not stragglers, start the launch.  Lists of 8,192 entries or more are
// blended with 4x4-pixel blocks per wave (four workgroups per tile); for lists of 65,536 or
// more, a stage before the blend marks per entry the blocks it may reach, and each block's
// wave walks only those entries.
#include "clod_internal.h"

namespace clod {

// XCD-aware launch order.  Consecutive workgroups are dispatched round-robin over the eight
// XCDs, each with its own L2, so tiles next to each other in the launch order (the same list
// length class, neighbours in the frame, sharing many records) would each fetch the shared
// records into a different L2.  Block b instead takes position
// ((b/8/C)*8 + b%8)*C + (b/8)%C of the tile order: runs of C consecutive positions stay on one
// XCD while the launch as a whole still proceeds in order (longest lists first).  The grid is
// rounded up to a multiple of 8C; the map is a bijection on it and blocks past the last tile
// exit at once.
constexpr uint32_t kXcds = 8, kXcdRun = 16;
constexpr uint32_t kLongMaskBlocks = 1024;   // grid of the very-long-tile mask stage

__device__ __forceinline__ uint32_t xcd_tile_pos(uint32_t b) {
  const uint32_t x = b % kXcds, j = b / kXcds, r = j / kXcdRun, i = j % kXcdRun;
  return (r * kXcds + x) * kXcdRun + i;
}

__host__ __device__ inline uint32_t xcd_grid(uint32_t tiles) {
  return (tiles + kXcds * kXcdRun - 1) / (kXcds * kXcdRun) * (kXcds * kXcdRun);
}

// Long tiles are taken by four workgroups each, in runs of eight tiles (one tile per XCD).
__host__ __device__ inline uint32_t long_grid(uint32_t long_tiles) {
  return (4 * long_tiles + 4 * kXcds - 1) / (4 * kXcds) * (4 * kXcds);
}

// The long tiles of this blend: the first tord[kTileLongWord] positions of the tile order
// (written by the tile ordering stage), within the bound the launch was sized for; the very
// long ones (65,536 entries or more) are the first tord[kTileVeryLongWord] of them.
__device__ __forceinline__ uint32_t long_tiles(const BlendArgs& a) {
  const uint32_t nl = a.tord[kTileLongWord];
  return nl < a.long_max ? nl : a.long_max;
}
__device__ __forceinline__ uint32_t very_long_tiles(const uint32_t* tord, uint32_t vl_max) {
  const uint32_t nv = tord[kTileVeryLongWord];
  return nv < vl_max ? nv : vl_max;
}

__device__ __forceinline__ int view_of_tile(const DevView* views, int V, uint32_t tile) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per-entry power cut.  An entry contributes to a pixel only if alpha'' E(power) >= fl(1/255).
// E(p) <= 1 for p <= 0 and E never decreases by more than 2^-23 relative between neighbouring
// inputs, so for power < cut = ln(1 / (255 alpha'')) - 0.01 the product is below
// (1/255) e^-0.01 (1 + 3 2^-23) < 1/255: the contract skips the pair.  The cut is formed as
// (ln(1/255) - 0.01) - ln 2 log2(alpha'') with the hardware log2, whose error here (about
// 1e-6 absolute for alpha'' in [1/255, 1]) the 0.01 margin absorbs.  cut > 0 means the entry
// is skipped at every pixel; alpha'' = 0 (or a flushed subnormal) gives cut = +inf.
__device__ __forceinline__ float entry_cut(float a2) {
  constexpr float kC0 = -5.551263545158426f;   // ln(1/255) - 0.01
  constexpr float kLn2 = 0.6931471805599453f;
  return kC0 - kLn2 * __builtin_amdgcn_logf(a2);
}

// Minimum over the box [X0, X1] x [Y0, Y1] of q(dx, dy) = A dx^2 + 2 B dx dy + C dy^2 (the
// conic's quadratic form, positive definite): 0 if the box holds the origin, else the least of
// the four edge minima (each a clamped 1-D vertex).  The vertices use the hardware reciprocal:
// q along an edge exceeds its minimum by a term quadratic in the vertex offset, so a
// relative offset of a few 2^-24 stays negligible next to the allowance below.
__device__ __forceinline__ float box_qmin(float A, float B, float C, float X0, float X1, float Y0, float Y1) {
  if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return 0.0f;
  const float bc = B * __builtin_amdgcn_rcpf(C), ba = B * __builtin_amdgcn_rcpf(A);
  auto qf = [&](float dx, float dy) { return fmaf(A * dx, dx, fmaf(C * dy, dy, 2.0f * B * dx * dy)); };
  const float yx0 = fminf(fmaxf(-bc * X0, Y0), Y1), yx1 = fminf(fmaxf(-bc * X1, Y0), Y1);
  const float xy0 = fminf(fmaxf(-ba * Y0, X0), X1), xy1 = fminf(fmaxf(-ba * Y1, X0), X1);
  return fminf(fminf(qf(X0, yx0), qf(X1, yx1)), fminf(qf(xy0, Y0), qf(xy1, Y1)));
}

// Second, tighter test for a quadrant: the entry is dropped if the quadratic form stays above
// 2.5 |cut| over the box of the quadrant's pixel centres (widened by 1e-3 px for the rounding
// of the box edges).  With AC / (AC - B^2) <= 5e4 the binary32 evaluation is within 1.2 % of
// the exact form (and the vertex rounding is negligible), so the exact minimum exceeds
// 2.4 |cut| and the same argument as the circle test applies.
// kB x kB pixel block with corner (x0, y0).
template <int kB = 8>
__device__ __forceinline__ bool ellipse_reaches(float u, float v, float A, float B, float C, float cut,
                                                float x0, float y0) {
  constexpr float kHi = (float)kB - 0.499f;
  const float X0 = (x0 + 0.499f) - u, X1 = (x0 + kHi) - u;
  const float Y0 = (y0 + 0.499f) - v, Y1 = (y0 + kHi) - v;
  return box_qmin(A, B, C, X0, X1, Y0, Y1) < 2.5f * -cut;
}

// Conservative per-quadrant cull of a staged entry.  A pixel centre p farther than
// sqrt(2.4 |cut|) rad / 3 + 0.5 from the 2D mean has exact quadratic form
// d^T Q d > 2.4 |cut| (rad >= 3 sqrt(lambda_max)), i.e. exact power < -1.2 |cut|.  The binary32
// power differs from the exact one by a factor common to the conic (the rounding of det,
// <= 2u r) plus independent roundings amplified by at most r = AC / (AC - B^2); with
// r <= 5e4 the total stays below 4%, so the evaluated power is below cut and the pair is
// skipped.  (The radius uses the hardware square root: its relative error of a few 2^-24
// is far inside that slack.)  Culled pairs are therefore exactly pairs the pixel loop would have skipped.
// Entries with a worse conditioned conic are never culled spatially.
__device__ __forceinline__ uint32_t quadrant_mask(float u, float v, float A, float B, float C, float rad,
                                                  float cut, float x0, float y0) {
  if (cut > 0.0f) return 0u;
  const float ac = A * C;
  const float det = ac - B * B;
  if (!(det > 2e-5f * ac) || !(rad < 1e6f)) return 0xFu;
  const float rc = __builtin_amdgcn_sqrtf(2.4f * -cut) * rad * (1.0f / 3.0f) + 0.5f;
  const float rc2 = rc * rc;
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float qx = x0 + (float)((q & 1) * 8), qy = y0 + (float)((q >> 1) * 8);
    const float ddx = fmaxf(0.0f, fmaxf(qx + 0.5f - u, u - (qx + 7.5f)));
    const float ddy = fmaxf(0.0f, fmaxf(qy + 0.5f - v, v - (qy + 7.5f)));
    if (ddx * ddx + ddy * ddy <= rc2 && ellipse_reaches(u, v, A, B, C, cut, qx, qy)) m |= 1u << q;
  }
  return m;
}

// The same test for one kB x kB pixel block with corner (x0, y0): 1 if the entry may touch it.
template <int kB>
__device__ __forceinline__ uint32_t quadrant_mask1(float u, float v, float A, float B, float C, float rad,
                                                   float cut, float x0, float y0) {
  if (!(cut <= 0.0f)) return 0u;   // never live (a NaN cut included: no power reaches it)
  const float ac = A * C;
  const float det = ac - B * B;
  if (!(det > 2e-5f * ac) || !(rad < 1e6f)) return 1u;
  constexpr float kHi = (float)kB - 0.5f;
  const float rc = __builtin_amdgcn_sqrtf(2.4f * -cut) * rad * (1.0f / 3.0f) + 0.5f;
  const float ddx = fmaxf(0.0f, fmaxf(x0 + 0.5f - u, u - (x0 + kHi)));
  const float ddy = fmaxf(0.0f, fmaxf(y0 + 0.5f - v, v - (y0 + kHi)));
  return (ddx * ddx + ddy * ddy <= rc * rc && ellipse_reaches<kB>(u, v, A, B, C, cut, x0, y0)) ? 1u : 0u;
}

// Tiles whose list holds at least 2^(kLongBucket - 1) entries (the dense far views of a large
// scene) are blended with 4x4-pixel blocks per wave: a wave walks only the entries that may
// reach its block, and sixteen waves share the tile instead of four.  The tile order puts them
// first (longest first): they are the first tord[kTileLongWord] positions, taken by the leading
// workgroups of the launch.  Of these, the tiles of at least 2^(kVeryLongBucket - 1) entries
// (the first tord[kTileVeryLongWord]) get their block tests from k_long_mask and their waves
// walk compacted lists.

// Forward blend.  Each wave owns one 8x8 quadrant of a tile (lane l: pixel (l & 7, l >> 3))
// and runs on its own: it takes 64 entries of the tile's sorted list at a time (one entry per
// lane, a coalesced gather), stages the ones that can touch its quadrant in its private LDS
// slice, compacted in list order, and walks them with the next entry's LDS reads issued
// before the current entry's arithmetic.  A wave stops after the batch in which its 64
// pixels saturate, independently of the other quadrants; the only block barrier is the
// final reduction of the optional pair counters.
struct TileLds {
  float4 st[4][3][64];   // per wave: (u, v, hA, nB), (hC, alpha'', r, g), (b, cut, list position, -)
  uint32_t q[4][256];    // per wave: ring of the list positions that reach its 4x4 block (very long tiles)
};

// One tile, at position pos of the batch's tile order, by the 256 threads of the block (four
// independent waves).  Shared by the per-batch launch (k_blend_fwd) and the persistent server.
// kB = 8: the four waves take the tile's four 8x8 quadrants.  kB = 4: the four waves take the
// 4x4 blocks 4 sub .. 4 sub + 3 of the tile (row-major over its 4 x 4 blocks); lane 16 g + p
// takes pixel p of the block, and the lanes of row 0 (g = 0) own the results.
template <bool kCount, int kB = 8>
__device__ __forceinline__ void blend_tile(const BlendArgs& a, uint32_t pos, TileLds& S, uint32_t sub = 0) {
  auto& st = S.st;
  const DevView* __restrict__ views = a.views;
  const int V = a.V;
  const uint32_t tiles_total = a.tiles_total;
  const int64_t VN = a.VN;
  const float4* __restrict__ rec = a.rec;
  const uint2* __restrict__ ranges = a.ranges;
  const uint32_t* __restrict__ svals = a.svals;
  const float bg0 = a.bg0, bg1 = a.bg1, bg2 = a.bg2;
  float* __restrict__ rgb = a.rgb;
  float* __restrict__ Tout = a.T;
  uint32_t* __restrict__ lastout = a.last;
  unsigned long long* __restrict__ pair_part = a.pair_part;
  const uint32_t* __restrict__ order = a.order;
  const uint32_t t = threadIdx.x;
  if (a.hdr[kHdrOverflow]) return;
  if (pos >= tiles_total) return;
  // The long tiles are taken as 4x4 blocks.
  if ((kB == 8) != (pos >= long_tiles(a))) return;
  const int tile_i = (int)order[pos];
  const int v = view_of_tile(views, V, (uint32_t)tile_i);
  const DevView& Vw = views[v];
  const int local = tile_i - (int)Vw.tile_base;
  const int tx = local % Vw.tiles_x, ty = local / Vw.tiles_x;
  const int wave = (int)(t >> 6);
  const uint32_t lane = lane_id();
  const int blk = kB == 8 ? wave : (int)sub * 4 + wave;
  const int qx0 = tx * kTile + (blk % (kTile / kB)) * kB, qy0 = ty * kTile + (blk / (kTile / kB)) * kB;
  const uint32_t pl = kB == 4 ? (lane & 15u) : lane;   // the lane's pixel within the block
  const int px = qx0 + (int)(pl % kB);
  const int py = qy0 + (int)(pl / kB);
  const bool inside = px < Vw.width && py < Vw.height;
  const bool own = inside && (kB == 8 || lane < 16u);
  // Pixel centres and quadrant corners in frame coordinates (the viewport origin added).
  const float pcx = (float)(px + Vw.vx) + 0.5f, pcy = (float)(py + Vw.vy) + 0.5f;
  const float fqx = (float)(qx0 + Vw.vx), fqy = (float)(qy0 + Vw.vy);
  const uint2 rg = ranges[tile_i];
  const float kSkip = 0.0039215688593685627f;   // fl(1/255)
  const float kTmin = 9.99999974737875163e-05f; // fl(1e-4)
  float4* s0 = st[wave][0];
  float4* s1 = st[wave][1];
  float4* s2 = st[wave][2];
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  uint32_t last = 0, term = 0xFFFFFFFFu, nexp = 0, nblend = 0;
  // Lanes whose pixel has terminated (or lies outside the frame), as a wave-uniform mask: the
  // per-entry predicates below are formed as lane masks and turned back into execution masks
  // with inverse ballots, so the termination bookkeeping stays in scalar registers.
  uint64_t dm = ballot64(!own);
  // 4x4 blocks: the n entries of a batch that may reach the block (staged compacted in list
  // order, slots 0 .. n-1), four at a time.  Row g of the wave evaluates entry g of the group
  // for the block's 16 pixels (power, live test, exponential, clamp: the four exponentials are
  // computed side by side, on every lane: lanes outside the live set are masked off after);
  // row 0 then takes the four entries in list order through the contract's termination test
  // and blend, the same operations in the same order as one entry at a time.  Terminated
  // pixels (dm, bits 0..15) drop out of the later entries of a group; their values for those
  // entries are never used.
  auto walk4 = [&](const uint32_t n) {
    const uint32_t row = lane >> 4;
    // One entry of the group for row 0's pixels: alpha (valid on the live lanes lv, bits
    // 0..15), the entry's colour and list position.
    auto step = [&](const float al, const uint64_t lv, const float c0, const float c1, const float c2,
                    const uint32_t pos) {
      const uint64_t lm = lv & ~dm & 0xFFFFull;
      if (lm == 0ull) return;
      const float Tn = T * (1.0f - al);   // used on the live lanes only
      const uint64_t um = ballot64(al >= kSkip) & lm;
      const uint64_t km = ballot64(Tn >= kTmin);
      const uint64_t bm = um & km;
      dm |= um & ~km;
      if (__builtin_amdgcn_inverse_ballot_w64(bm)) {
        const float w = al * T;
        cr = fmaf_(c0, w, cr);
        cg = fmaf_(c1, w, cg);
        cb = fmaf_(c2, w, cb);
        T = Tn;
        last = pos + 1u;
      }
      if (kCount) {
        if (__builtin_amdgcn_inverse_ballot_w64(um & ~km)) term = pos;
        nexp += __builtin_amdgcn_inverse_ballot_w64(lm) ? 1u : 0u;
        nblend += __builtin_amdgcn_inverse_ballot_w64(bm) ? 1u : 0u;
      }
    };
    // Slots k .. k + 3 lie in the wave's 64-entry slice (k is a multiple of 4 below n <= 64);
    // those at or past n hold stale entries, masked off by `slots`.
    for (uint32_t k = 0; k < n; k += 4) {
      const uint32_t fr = k + row;
      const float4 a = s0[fr], c = s1[fr];
      const float4 bc = s2[fr];
      // Colours and list positions of entries 1..3 for row 0 (LDS broadcasts).
      const float4 q1 = s1[k + 1u], q2 = s1[k + 2u], q3 = s1[k + 3u];
      const float4 r1 = s2[k + 1u], r2 = s2[k + 2u], r3 = s2[k + 3u];
      const float dx = a.x - pcx, dy = a.y - pcy;
      const float power = fmaf_(a.z * dx, dx, fmaf_(c.x * dy, dy, (a.w * dx) * dy));
      const uint32_t left = n - k;
      const uint64_t slots = left >= 4u ? ~0ull : (1ull << (16u * left)) - 1ull;
      const uint64_t dm4 = (dm & 0xFFFFull) * 0x0001000100010001ull;
      const uint64_t live = ballot64(power <= 0.0f) & ballot64(power >= bc.y) & ~dm4 & slots;
      if (live == 0ull) continue;
      const float al = fminf(0.99f, c.y * cexp_core<true>(power));
      // Rows 1, 2, 3 of al into row 0 (whole-wave row swaps).
      const auto x16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(al), __float_as_uint(al), false, false);
      const auto x32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(al), __float_as_uint(al), false, false);
      const auto x48 = __builtin_amdgcn_permlane32_swap(x16[1], x16[1], false, false);
      step(al, live, c.z, c.w, bc.x, __float_as_uint(bc.z));
      step(__uint_as_float(x16[1]), live >> 16, q1.z, q1.w, r1.x, __float_as_uint(r1.z));
      step(__uint_as_float(x32[1]), live >> 32, q2.z, q2.w, r2.x, __float_as_uint(r2.z));
      step(__uint_as_float(x48[1]), live >> 48, q3.z, q3.w, r3.x, __float_as_uint(r3.z));
      if (dm == ~0ull) break;
    }
  };
  // One batch of up to 64 entries, its records (g0, g1, g2) already in registers, lane l's
  // at list position j: staged in this wave's LDS slice, culled against the quadrant, then
  // walked.  The entries of a very long tile arrive already compacted to those that may reach
  // the 4x4 block (relc); elsewhere the batch is 64 consecutive entries and is culled here.
  const bool pre = kB == 4 && pos < very_long_tiles(a.tord, a.vl_max);
  auto batch = [&](const uint32_t j, const float4& g0, const float4& g1, const float4& g2,
                   const bool relc) {
    bool rel = false;
    float cut = 0.0f;
    if (kB == 4 && pre) {
      rel = relc;
      if (rel) {
        s0[lane] = make_float4(g0.x, g0.y, -0.5f * g1.x, -g1.y);
        s1[lane] = make_float4(-0.5f * g1.z, g0.z, g2.x, g2.y);
        s2[lane] = make_float4(g2.z, entry_cut(g0.z), __uint_as_float(j - rg.x), 0.f);
      }
    } else if (j < rg.y) {
      cut = entry_cut(g0.z);
      rel = (quadrant_mask1<kB>(g0.x, g0.y, g1.x, g1.y, g1.z, g0.w, cut, fqx, fqy)) != 0u;
    }
    uint64_t mask = ballot64(rel);
    // The entries that may reach the quadrant (block) are staged compacted, in list order
    // (slot = rank of the lane among them), so that the walks below step a counter.  (Those of
    // a very long tile are the leading lanes already.)
    if (!(kB == 4 && pre)) {
      if (rel) {
        const uint32_t slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        s0[slot] = make_float4(g0.x, g0.y, -0.5f * g1.x, -g1.y);
        s1[slot] = make_float4(-0.5f * g1.z, g0.z, g2.x, g2.y);
        s2[slot] = make_float4(g2.z, cut, __uint_as_float(j - rg.x), 0.f);
      }
    }
    const uint32_t n = (uint32_t)__builtin_popcountll(mask);
    if (kB == 8 && (n & 1u) && lane == 63u) {
      s0[n] = make_float4(__builtin_nanf(""), __builtin_nanf(""), 0.0f, 0.0f);
      s2[n] = make_float4(0.0f, __builtin_inff(), 0.0f, 0.0f);
    }
    // The staged entries are read by other lanes of this wave: wait for the LDS writes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (mask == 0ull) return;
    if constexpr (kB == 4) {
      walk4(n);
      return;
    }
    // One entry: the contract's skip, exponential, clamp, termination and blend.  Below the
    // entry's cut (or above 0) the contract skips the pair whatever E returns; live pairs have
    // power in [cut, 0] with cut >= ln(1/255) - 0.01, inside cexp_core's range.  Once some
    // lane is live, every lane evaluates E (an exec-mask region around it would cost scalar
    // instructions and save no vector ones); the skip and termination tests then run on the
    // whole wave and are masked with the live set, so al and Tn of other lanes are never used.
    auto pair = [&](const float4& a, const float4& c, const float4& bc) {
      const float dx = a.x - pcx, dy = a.y - pcy;
      const float power = fmaf_(a.z * dx, dx, fmaf_(c.x * dy, dy, (a.w * dx) * dy));
      // cut <= power <= 0 as one test: a staged entry has cut <= 0 (quadrant_mask1 culls the
      // others), so the median of (power, cut, 0) is power exactly then; a NaN power (the
      // padding entry) compares unequal.
      const uint64_t lm = ballot64(__builtin_amdgcn_fmed3f(power, bc.y, 0.0f) == power) & ~dm;
      if (lm == 0ull) return;
      const float al = fminf(0.99f, c.y * cexp_core<true>(power));
      const float Tn = T * (1.0f - al);
      // al is never NaN (fminf returns 0.99 for a NaN product) and T is in (0, 1], so
      // Tn >= fl(1e-4) is exactly the negation of the contract's termination test.
      const uint64_t um = ballot64(al >= kSkip) & lm;
      const uint64_t km = ballot64(Tn >= kTmin);
      const uint64_t bm = um & km;
      dm |= um & ~km;
      const uint32_t pos = __float_as_uint(bc.z);
      if (__builtin_amdgcn_inverse_ballot_w64(bm)) {
        const float w = al * T;
        cr = fmaf_(c.z, w, cr);
        cg = fmaf_(c.w, w, cg);
        cb = fmaf_(bc.x, w, cb);
        T = Tn;
        last = pos + 1u;
      }
      if (kCount) {   // work counters only when asked for (they cost the per-entry loop)
        if (__builtin_amdgcn_inverse_ballot_w64(um & ~km)) term = pos;
        nexp += __builtin_amdgcn_inverse_ballot_w64(lm) ? 1u : 0u;
        nblend += __builtin_amdgcn_inverse_ballot_w64(bm) ? 1u : 0u;
      }
    };
    // Two register sets in alternation: the LDS reads of the next entry are in flight while
    // the current one is evaluated, with no copies between iterations.  The walk takes the
    // slots two at a time; an odd count is padded with slot n, given a NaN position and a cut
    // of +inf (so no pixel is live for it) before the wave barrier above.  (Slots past that hold stale
    // entries: they may be read ahead, within the slice, but are never walked.)
    // The saturation of all 64 pixels is checked per batch, by the caller: within a batch the
    // loop has no exit test but its count.
    float4 a0 = s0[0], c0 = s1[0], b0 = s2[0];
    for (uint32_t k = 0; k < n; k += 2) {
      const float4 a1 = s0[k + 1u], c1 = s1[k + 1u], b1 = s2[k + 1u];
      pair(a0, c0, b0);
      const uint32_t k2 = k + 2u < 63u ? k + 2u : 63u;
      a0 = s0[k2]; c0 = s1[k2]; b0 = s2[k2];
      pair(a1, c1, b1);
    }
  };
  // Software pipeline over the batches, unrolled by two with a register set each (A, B), so
  // that nothing is copied between batches: while one batch is staged and walked, the records
  // of the next and the sorted indices of the one after are in flight (index -> record is two
  // dependent memory latencies per batch, which few resident waves -- a far frame's handful of
  // long tiles -- cannot hide).  Every load is issued (positions past the list end read its
  // last entry, which is not staged), so the wait counts stay static.
  if (rg.y > rg.x) {
    const uint32_t jmax = rg.y - 1;
    auto index_at = [&](uint32_t q) {
      const uint32_t f = svals[q < jmax ? q : jmax];
      return (int64_t)f < VN ? f : 0u;   // defensive: the sort only emits indices < V*n
    };
    if (kB == 4 && pre) {
      // Very long tile: the wave scans its block's bit plane (one word per 64 entries, read
      // with scalar loads: they do not enter the vector-memory wait count, so the pipeline's
      // gathers stay in flight while it scans), appends the positions of the entries that may
      // reach the block to its LDS ring, and takes them 64 at a time into the same two-set
      // pipeline (indices two batches ahead, records one), so that it gathers, stages and walks
      // only those entries.  (The planes are written by an earlier launch, and the scalar
      // cache is invalidated when a launch starts; the resident serving kernel, which runs a
      // job's stages in one launch, does not take this path.)
      typedef const __attribute__((address_space(4))) unsigned long long* ConstWords;
      // (readfirstlane returns int: each half goes through uint32_t so that the low half is
      // not sign-extended into the high one.)
      const uint64_t pa = (uint64_t)(uintptr_t)(a.lplane + (int64_t)blk * a.pw + (rg.x >> 6) + (uint32_t)tile_i);
      const uint64_t pu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(pa >> 32)) << 32) |
                          (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pa);
      const ConstWords plane = (ConstWords)(uintptr_t)pu;
      const uint32_t nwords = ((rg.y - rg.x) + 63u) >> 6;
      uint32_t* __restrict__ ring = S.q[wave];
      uint32_t head = 0, tail = 0, wi = 0;
      auto fill = [&]() {
        while (tail - head < 192u && wi < nwords) {
          const unsigned long long word = plane[wi];
          const uint32_t lo = (uint32_t)word, hi = (uint32_t)(word >> 32);
          if ((word >> lane) & 1ull)
            ring[(tail + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u))) & 255u] =
                rg.x + 64u * wi + lane;
          tail += (uint32_t)__builtin_popcountll(word);
          ++wi;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      };
      // The next (up to) 64 positions of the ring, one per lane (v: the lane holds one).
      auto take = [&](uint32_t& q, bool& v) {
        fill();
        const uint32_t n = tail - head < 64u ? tail - head : 64u;
        v = lane < n;
        q = v ? ring[(head + lane) & 255u] : rg.x;
        head += n;
      };
      // Ring positions lie in [rg.x, rg.y) (clamped all the same: they come from LDS, so the
      // clamp costs no memory wait); the record indices read there are the sort's own and are
      // not clamped (a clamp of each loaded index would make the wave wait for every gather in
      // flight).
      auto index_of = [&](uint32_t q) { return svals[q < jmax ? q : jmax]; };
      uint32_t qa, qb, ja, jb;
      bool va, vb, ra, rb;
      take(qa, va);
      uint32_t ia = index_of(qa);
      take(qb, vb);
      uint32_t ib = index_of(qb);
      float4 a0 = rec[kRecQuads * (int64_t)ia], a1 = rec[kRecQuads * (int64_t)ia + 1], a2 = rec[kRecQuads * (int64_t)ia + 2];
      float4 b0, b1, b2;
      ja = qa;
      ra = va;
      take(qa, va);
      ia = index_of(qa);
      while (ballot64(ra) != 0ull && dm != ~0ull) {
        b0 = rec[kRecQuads * (int64_t)ib];
        b1 = rec[kRecQuads * (int64_t)ib + 1];
        b2 = rec[kRecQuads * (int64_t)ib + 2];
        jb = qb;
        rb = vb;
        take(qb, vb);
        ib = index_of(qb);
        batch(ja, a0, a1, a2, ra);
        if (ballot64(rb) == 0ull || dm == ~0ull) break;
        a0 = rec[kRecQuads * (int64_t)ia];
        a1 = rec[kRecQuads * (int64_t)ia + 1];
        a2 = rec[kRecQuads * (int64_t)ia + 2];
        ja = qa;
        ra = va;
        take(qa, va);
        ia = index_of(qa);
        batch(jb, b0, b1, b2, rb);
      }
    } else {
    uint32_t ia = index_at(rg.x + lane);
    uint32_t ib = index_at(rg.x + 64 + lane);
    float4 a0 = rec[kRecQuads * (int64_t)ia], a1 = rec[kRecQuads * (int64_t)ia + 1], a2 = rec[kRecQuads * (int64_t)ia + 2];
    float4 b0, b1, b2;
    ia = index_at(rg.x + 128 + lane);
    for (uint32_t base = rg.x; base < rg.y && dm != ~0ull; base += 128) {
      b0 = rec[kRecQuads * (int64_t)ib];
      b1 = rec[kRecQuads * (int64_t)ib + 1];
      b2 = rec[kRecQuads * (int64_t)ib + 2];
      ib = index_at(base + 192 + lane);
      batch(base + lane, a0, a1, a2, false);
      if (base + 64 >= rg.y || dm == ~0ull) break;
      a0 = rec[kRecQuads * (int64_t)ia];
      a1 = rec[kRecQuads * (int64_t)ia + 1];
      a2 = rec[kRecQuads * (int64_t)ia + 2];
      ia = index_at(base + 256 + lane);
      batch(base + 64 + lane, b0, b1, b2, false);
    }
    }
  }
  if (own) {
    const int64_t P = (int64_t)Vw.pix_base;
    const int64_t HW = (int64_t)Vw.width * Vw.height;
    const int64_t p = (int64_t)py * Vw.width + px;
    rgb[3 * P + p] = fmaf_(T, bg0, cr);
    rgb[3 * P + HW + p] = fmaf_(T, bg1, cg);
    rgb[3 * P + 2 * HW + p] = fmaf_(T, bg2, cb);
    Tout[P + p] = T;
    lastout[P + p] = last;
  }
  if (kCount) {
    // Pairs the contract's per-pixel loop evaluates: up to and including the terminating
    // entry, else the whole list.  The four wave totals are added to the tile's (zeroed)
    // partials.
    const unsigned long long ev = !own ? 0ull : (term != 0xFFFFFFFFu ? (unsigned long long)term + 1ull
                                                                         : (unsigned long long)(rg.y - rg.x));
    const unsigned long long es = wave_sum(ev);
    const unsigned long long x = wave_sum((unsigned long long)nexp);
    const unsigned long long bl = wave_sum((unsigned long long)nblend);
    if (lane == 0) {
      atomicAdd(pair_part + 3 * (int64_t)tile_i, es);
      atomicAdd(pair_part + 3 * (int64_t)tile_i + 1, x);
      atomicAdd(pair_part + 3 * (int64_t)tile_i + 2, bl);
    }
  }
}

// Very long tiles, per entry of their lists: the 4x4 blocks of the tile the entry may reach (the
// blend's own block test, run once per entry here instead of once per entry in each of the
// tile's sixteen waves, which all walk these lists to the end in the far views of a large
// scene), as sixteen bit planes: per block, one bit per entry, 64 entries per word.  Wave w of
// the grid takes the 64-entry chunks w, w + W, ... of each very long tile and writes the
// chunk's sixteen words (lane b the word of block b).
__device__ __forceinline__ void long_mask_body(const LongMaskArgs& a, Blk b) {
  if (a.hdr[kHdrOverflow]) return;
  const uint32_t nl = very_long_tiles(a.tord, a.vl_max);
  if (nl == 0u) return;
  const uint32_t lane = lane_id();
  const uint32_t gw = b.id * (kBlock / 64u) + (threadIdx.x >> 6), GW = b.n * (kBlock / 64u);
  for (uint32_t p = 0; p < nl; ++p) {
    const int tile_i = (int)a.order[p];
    const int v = view_of_tile(a.views, a.V, (uint32_t)tile_i);
    const DevView& Vw = a.views[v];
    const int local = tile_i - (int)Vw.tile_base;
    const int tx = local % Vw.tiles_x, ty = local / Vw.tiles_x;
    const uint2 rg = a.ranges[tile_i];
    const uint32_t nchunks = ((rg.y - rg.x) + 63u) >> 6;
    unsigned long long* __restrict__ out = a.lplane + (rg.x >> 6) + (uint32_t)tile_i;
    for (uint32_t c = gw; c < nchunks; c += GW) {
      const uint32_t j = rg.x + 64u * c + lane;
      uint32_t m = 0u;
      if (j < rg.y) {
        uint32_t f = a.svals[j];
        if ((int64_t)f >= a.VN) f = 0u;   // defensive: the sort only emits indices < V*n
        const float4 g0 = a.rec[kRecQuads * (int64_t)f], g1 = a.rec[kRecQuads * (int64_t)f + 1];
        const float cut = entry_cut(g0.z);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const float x0 = (float)(tx * kTile + (q % 4) * 4 + Vw.vx), y0 = (float)(ty * kTile + (q / 4) * 4 + Vw.vy);
          m |= quadrant_mask1<4>(g0.x, g0.y, g1.x, g1.y, g1.z, g0.w, cut, x0, y0) << q;
        }
      }
      unsigned long long mine = 0ull;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const unsigned long long w = ballot64(((m >> q) & 1u) != 0u);
        if (lane == (uint32_t)q) mine = w;
      }
      if (lane < 16u) out[(int64_t)lane * a.pw + c] = mine;
    }
  }
}
__global__ __launch_bounds__(kBlock) void k_long_mask(LongMaskArgs a) { long_mask_body(a, grid_blk()); }

// Long tiles: four workgroups per tile, on one XCD (workgroups b, b + 8, b + 16, b + 24 take
// the same tile: consecutive workgroups go round-robin to the eight XCDs).
__device__ __forceinline__ void long_item(uint32_t b, uint32_t& pos, uint32_t& sub) {
  const uint32_t x = b % kXcds, j = b / kXcds;
  sub = j % 4;
  pos = x + kXcds * (j / 4);
}

// Item b of the blend stage: the leading long_grid(long_tiles) items take the long tiles as
// 4x4 blocks, the next xcd_grid(tiles) items one tile each in the XCD-aware order (both in one
// launch, so that the long tiles run beside the others).  Items past these (the launch is
// sized for the most long tiles the pair capacity allows) map past the last tile and exit.
template <bool kCount>
__device__ __forceinline__ void blend_item(const BlendArgs& a, uint32_t b, TileLds& S) {
  const uint32_t lb = long_grid(long_tiles(a));
  if (b < lb) {
    uint32_t pos, sub;
    long_item(b, pos, sub);
    blend_tile<kCount, 4>(a, pos, S, sub);
  } else {
    blend_tile<kCount>(a, xcd_tile_pos(b - lb), S);
  }
}

// Items a blend stage needs once the tile order is known (the resident kernel sizes its
// claims by it; a per-stage launch covers the bound instead).
__device__ __forceinline__ uint32_t blend_items(const BlendArgs& a) {
  return long_grid(long_tiles(a)) + xcd_grid(a.tiles_total);
}

// Per-batch launch: one workgroup per tile (four per long tile).
template <bool kCount>
__global__ __launch_bounds__(kBlock) void k_blend_fwd(BlendArgs a) {
  __shared__ TileLds S;
  blend_item<kCount>(a, blockIdx.x, S);
}

// Sums the per-tile pair partials into the caller's counters (one block, three atomics).
__device__ __forceinline__ void reduce_pairs_body(const ReducePairsArgs& r, Blk) {
  __shared__ unsigned long long sm[4][3];
  const unsigned long long* __restrict__ part = r.part;
  unsigned long long* __restrict__ out = r.out;
  unsigned long long a = 0, b = 0, c = 0;
  for (uint32_t t = threadIdx.x; t < r.tiles; t += kBlock) {
    a += part[3 * (int64_t)t]; b += part[3 * (int64_t)t + 1]; c += part[3 * (int64_t)t + 2];
  }
  a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
  if (lane_id() == 0) { sm[threadIdx.x >> 6][0] = a; sm[threadIdx.x >> 6][1] = b; sm[threadIdx.x >> 6][2] = c; }
  __syncthreads();
  if (threadIdx.x < 3) atomicAdd(out + threadIdx.x, sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] + sm[3][threadIdx.x]);
}
__global__ __launch_bounds__(kBlock) void k_reduce_pairs(ReducePairsArgs r) { reduce_pairs_body(r, grid_blk()); }

hipError_t launch_blend_fwd(const Layout& L, void* ws, const BlendBufs& bb, clod_params prm, float* rgb, float* T,
                            uint32_t* last, int64_t* pairs, const Sink& out) {
  if (L.tiles_total == 0) return hipSuccess;
  char* w = (char*)ws;
  unsigned long long* part = pairs ? (unsigned long long*)(w + L.pair_part) : nullptr;
  if (part) {
    hipError_t e = launch_fill_u32((uint32_t*)part, 0u, 6 * (int64_t)L.tiles_total, out);
    if (e != hipSuccess) return e;
  }
  // At most cap / 2^(kLongBucket - 1) tiles can be long: the launch covers that many.
  const int64_t cap_long = bb.cap / (1ll << (kLongBucket - 1));
  const uint32_t long_max = (uint32_t)(cap_long < (int64_t)L.tiles_total ? cap_long : (int64_t)L.tiles_total);
  // Very long tiles: at most cap / 2^(kVeryLongBucket - 1); their bit planes (16 planes of
  // pw words) must fit the arrays the tile-id sort left free, else they are blended like the
  // other long tiles.
  const int64_t cap_vl = bb.cap / (1ll << (kVeryLongBucket - 1));
  const uint32_t pw = (uint32_t)((bb.cap + 63) / 64 + (int64_t)L.tiles_total + 1);
  const bool planes_fit = (size_t)16 * pw * sizeof(unsigned long long) <= bb.spare_bytes;
  const uint32_t vl_max =
      planes_fit ? (uint32_t)(cap_vl < (int64_t)L.tiles_total ? cap_vl : (int64_t)L.tiles_total) : 0u;
  if (vl_max > 0) {
    Stage m{};
    m.kind = kStLongMask;
    m.items = kLongMaskBlocks;
    m.block = kBlock;
    m.a.long_mask = LongMaskArgs{(const DevView*)(w + L.vinfo), L.V, (const uint2*)(w + L.ranges),
                                 (const uint32_t*)(w + L.order), (const uint32_t*)(w + L.tord), bb.svals,
                                 (const float4*)(w + L.rec), L.VN, (const unsigned long long*)(w + L.hdr),
                                 bb.spare, pw, vl_max};
    const hipError_t e = out.put(m);
    if (e != hipSuccess) return e;
  }
  Stage st{};
  st.kind = kStBlend;
  st.items = long_grid(long_max) + xcd_grid(L.tiles_total);
  st.block = kBlock;
  st.a.blend = BlendArgs{(const DevView*)(w + L.vinfo), L.V, L.tiles_total, L.VN, (const float4*)(w + L.rec),
                         (const uint2*)(w + L.ranges), bb.svals, (const unsigned long long*)(w + L.hdr), prm.bg[0],
                         prm.bg[1], prm.bg[2], rgb, T, last, part, (const uint32_t*)(w + L.order),
                         (const uint32_t*)(w + L.tord), long_max, part ? 1 : 0, bb.spare, pw, vl_max};
  hipError_t e = out.put(st);
  if (e == hipSuccess && part) {
    Stage r{};
    r.kind = kStReducePairs;
    r.items = 1;
    r.block = kBlock;
    r.a.reduce_pairs = ReducePairsArgs{(const unsigned long long*)part, L.tiles_total, (unsigned long long*)pairs};
    e = out.put(r);
  }
  return e;
}

hipError_t launch_blend_stage(const Stage& st, hipStream_t s) {
  const dim3 g(st.items), blk(st.block);
  switch (st.kind) {
    case kStBlend:
      if (st.a.blend.count) hipLaunchKernelGGL(k_blend_fwd<true>, g, blk, 0, s, st.a.blend);
      else hipLaunchKernelGGL(k_blend_fwd<false>, g, blk, 0, s, st.a.blend);
      break;
    case kStReducePairs: hipLaunchKernelGGL(k_reduce_pairs, g, blk, 0, s, st.a.reduce_pairs); break;
    case kStLongMask: hipLaunchKernelGGL(k_long_mask, g, blk, 0, s, st.a.long_mask); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- adjoint
// Back-to-front over each pixel's blended entries (positions < last), recomputing every
// decision exactly as the forward; transmittance is recovered by division
// (T_k = T_{k+1} / (1 - a_k)); the normalised colour of everything behind entry k obeys
// R_{k-1} = c_k a_k + (1 - a_k) R_k with R = background after the last entry, so
// dC/da_k = T_k (c_k - R_k); only g . R (g = dL/dC of the pixel) is needed, and it obeys the
// same recurrence.  Same quadrant mapping and per-quadrant compaction as the forward (culled
// entries are ones the forward skipped).  Per entry nine sums (five moments of dL/dpower, the
// alpha'' partial and three colour partials) are reduced over the wave, summed over the 4
// waves in LDS, turned into the 9 screen-space partials and added to the global accumulator
// once per tile.  The accumulator holds the nine partials of a record as
// consecutive floats, so the flush sends each entry's nine atomics to one 36-byte span.
// With kCount, each wave adds to the tile's (zeroed) partials the (pixel, entry) lanes its walk
// visits, the pairs whose exponential it evaluates (blended in the forward, power in range) and
// the pairs that contribute to the gradients.
template <bool kCount>
__global__ __launch_bounds__(kBlock) void k_blend_bwd(
    const DevView* __restrict__ views, int V, uint32_t tiles_total, int64_t VN,
    const float4* __restrict__ rec, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ svals, const unsigned long long* __restrict__ hdr,
    float bg0, float bg1, float bg2, const float* __restrict__ Tin,
    const uint32_t* __restrict__ lastin, const float* __restrict__ dL_drgb,
    float* __restrict__ gscreen, const uint32_t* __restrict__ order,
    unsigned long long* __restrict__ pair_part) {
  __shared__ float4 s0[kBlock];   // u, v, A, B
  __shared__ float4 s1[kBlock];   // C, alpha'', r, g
  __shared__ float4 s2[kBlock];   // b, power cut, -A/2, -C/2 (same stride as s0, s1: one address)
  __shared__ float acc[kBlock * kGscreen];   // [entry][9]: odd stride, conflict-free
  __shared__ uint32_t sidx[kBlock];
  __shared__ unsigned long long qmask[4][4];    // [staging wave][quadrant]: entries that may reach it
  __shared__ uint32_t smax[4];
  const uint32_t pos = xcd_tile_pos(blockIdx.x);
  if (pos >= tiles_total) return;
  const int tile_i = (int)order[pos];
  if (hdr[kHdrOverflow]) return;
  const int v = view_of_tile(views, V, (uint32_t)tile_i);
  const DevView& Vw = views[v];
  const int local = tile_i - (int)Vw.tile_base;
  const int tx = local % Vw.tiles_x, ty = local / Vw.tiles_x;
  const int wave = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const int px = tx * kTile + (wave & 1) * 8 + (int)(lane & 7);
  const int py = ty * kTile + (wave >> 1) * 8 + (int)(lane >> 3);
  const bool inside = px < Vw.width && py < Vw.height;
  const float pcx = (float)(px + Vw.vx) + 0.5f, pcy = (float)(py + Vw.vy) + 0.5f;
  const float tx0 = (float)(tx * kTile + Vw.vx), ty0 = (float)(ty * kTile + Vw.vy);
  const uint2 rg = ranges[tile_i];
  const float kSkip = 0.0039215688593685627f;
  const int64_t P = (int64_t)Vw.pix_base;
  const int64_t HW = (int64_t)Vw.width * Vw.height;
  const int64_t p = (int64_t)py * Vw.width + px;
  uint32_t last = 0;
  float T = 1.0f, g0c = 0.f, g1c = 0.f, g2c = 0.f;
  if (inside) {
    last = lastin[P + p];
    T = Tin[P + p];
    g0c = dL_drgb[3 * P + p];
    g1c = dL_drgb[3 * P + HW + p];
    g2c = dL_drgb[3 * P + 2 * HW + p];
  }
  // g . R: the pixel's colour gradient dotted with the normalised colour behind the current
  // entry (R starts as the background), kept as one scalar through the same recurrence.
  float gR = fmaf_(g0c, bg0, fmaf_(g1c, bg1, g2c * bg2));
  // Largest last in the tile bounds the walk.
  uint32_t m = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) { const uint32_t q = __shfl_xor(m, o, 64); m = q > m ? q : m; }
  if (lane == 0) smax[wave] = m;
  __syncthreads();
  const uint32_t tmax = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
  const uint32_t end = rg.x + tmax;   // exclusive
  unsigned long long n_walk = 0, n_live = 0, n_contrib = 0;   // wave-uniform (kCount)
  for (uint32_t hi = end; hi > rg.x;) {
    const uint32_t lo = hi > rg.x + kBlock ? hi - kBlock : rg.x;
    const int cnt = (int)(hi - lo);
    __syncthreads();
    uint32_t qm = 0;
    if ((int)threadIdx.x < cnt) {
      uint32_t f = svals[lo + threadIdx.x];
      if ((int64_t)f >= VN) f = 0;   // defensive: the sort only emits indices < V*n
      const float4 a0 = rec[kRecQuads * (int64_t)f];
      const float4 a1 = rec[kRecQuads * (int64_t)f + 1];
      const float4 a2 = rec[kRecQuads * (int64_t)f + 2];
      const float cut = entry_cut(a0.z);
      s0[threadIdx.x] = make_float4(a0.x, a0.y, a1.x, a1.y);
      s1[threadIdx.x] = make_float4(a1.z, a0.z, a2.x, a2.y);
      s2[threadIdx.x] = make_float4(a2.z, cut, -0.5f * a1.x, -0.5f * a1.z);
      sidx[threadIdx.x] = f;
      qm = quadrant_mask(a0.x, a0.y, a1.x, a1.y, a1.z, a0.w, cut, tx0, ty0);
    }
#pragma unroll
    for (int q = 0; q < kGscreen; ++q) acc[q * kBlock + threadIdx.x] = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t b = ballot64((qm >> q) & 1u);
      if (lane == 0) qmask[wave][q] = b;
    }
    __syncthreads();
    // Walk this quadrant's entries back to front: staging waves 3..0, each mask from its
    // highest bit down.  Masks, entry index and position are wave-uniform (scalar registers).
    for (int c = 3; c >= 0; --c) {
      const unsigned long long mv = qmask[c][wave];
      uint64_t mk = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(mv >> 32)) << 32) |
                    (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mv);
      while (mk != 0ull) {
        const int e = 63 - __builtin_clzll(mk);
        mk &= ~(1ull << e);
        const int k = c * 64 + e;
        const uint32_t pos = lo - rg.x + (uint32_t)k;
        const float4 a = s0[k];
        const float4 c4 = s1[k];
        const float4 bc = s2[k];
        const float dx = a.x - pcx, dy = a.y - pcy;
        const float hA = bc.z, nB = -a.w, hC = bc.w;   // -A/2 and -C/2 staged once per entry
        const float power = fmaf_(hA * dx, dx, fmaf_(hC * dy, dy, (nB * dx) * dy));
        // Live: blended in the forward (position < last) with power in [cut, 0].  Other lanes
        // compute discarded values (finite: their powers are tiny positives or below cut).
        const uint64_t lm = ballot64(pos < last) & ballot64(power <= 0.0f) & ballot64(power >= bc.y);
        if (kCount) {
          n_walk += 64;
          n_live += (unsigned long long)__popcll(lm);
        }
        if (lm == 0ull) continue;
        const float G = cexp_core(power);
        const float prod = c4.y * G;
        const float al = fminf(0.99f, prod);
        const uint64_t cm = ballot64(al >= kSkip) & lm;       // contributing lanes
        if (kCount) n_contrib += (unsigned long long)__popcll(cm);
        if (cm == 0ull) continue;
        const uint64_t gm = ballot64(prod <= 0.99f) & cm;     // ... below the clamp
        const bool contrib = __builtin_amdgcn_inverse_ballot_w64(cm);
        const bool geo = __builtin_amdgcn_inverse_ballot_w64(gm);
        const float oma = 1.0f - al;
        // T before the entry, T / (1 - a): only gradients use it, so a hardware reciprocal with
        // one Newton step (within an ulp) replaces the correctly rounded division.
        const float r0 = __builtin_amdgcn_rcpf(oma);
        const float Tk = T * fmaf(fmaf(-oma, r0, 1.0f), r0, r0);
        const float gc = fmaf_(g0c, c4.z, fmaf_(g1c, c4.w, g2c * bc.x));   // g . c_k
        const float dLda = Tk * (gc - gR);
        // Zeroing the three factors zeroes every partial of the lanes that do not take part
        // (the other factors are finite).
        const float gp = geo ? dLda * prod : 0.f;   // dL/dpower
        const float ga2 = geo ? dLda * G : 0.f;
        const float wgt = contrib ? al * Tk : 0.f;
        const float gr = g0c * wgt, gg = g1c * wgt, gb = g2c * wgt;
        // The partials of u, v and the conic are linear in five moments of dL/dpower over the
        // pixels (sums of gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2); the moments are reduced and
        // the conic coefficients applied once per entry at the flush.
        const float gpx = gp * dx, gpy = gp * dy;
        // Wave totals of the nine sums (eight reduced together: lanes 8q.. hold sum q; the
        // ninth on its own), then one LDS atomic instruction over nine lanes.
        const float g8[8] = {gpx, gpy, gpx * dx, gpx * dy, gpy * dy, ga2, gr, gg};
        const float t8 = wave_sum8(g8);
        const float tb = wave_sum_dpp(gb);
        if ((lane & 7u) == 0u || lane == 1u) {
          const uint32_t q = lane == 1u ? 8u : lane >> 3;
          atomicAdd(&acc[k * kGscreen + q], lane == 1u ? tb : t8);
        }
        if (contrib) {
          gR = fmaf_(al, gc, oma * gR);   // R_{k-1} = c_k a_k + (1 - a_k) R_k, dotted with g
          T = Tk;
        }
      }
    }
    __syncthreads();
    // Flush: consecutive threads take consecutive (entry, partial) items; the first five
    // items of an entry turn its moments into the partials of u, v, A, B and C:
    // du = -(A m0 + B m1), dv = -(C m1 + B m0), dA = -m2 / 2, dB = -m3, dC = -m4 / 2.
    for (int it = threadIdx.x; it < cnt * kGscreen; it += kBlock) {
      const int t = it / kGscreen;
      const int q = it - t * kGscreen;
      float val = acc[it];
      if (q < 5) {
        const float m0 = acc[t * kGscreen], m1 = acc[t * kGscreen + 1];
        const float A = s0[t].z, B = s0[t].w, C = s1[t].x;
        val = q == 0 ? -fmaf_(A, m0, B * m1)
            : q == 1 ? -fmaf_(C, m1, B * m0)
            : q == 3 ? -val : -0.5f * val;
      }
      if (val != 0.0f) atomicAdd(gscreen + (int64_t)sidx[t] * kGscreen + q, val);
    }
    hi = lo;
  }
  if (kCount && lane == 0) {
    atomicAdd(pair_part + 3 * (int64_t)tile_i, n_walk);
    atomicAdd(pair_part + 3 * (int64_t)tile_i + 1, n_live);
    atomicAdd(pair_part + 3 * (int64_t)tile_i + 2, n_contrib);
  }
}

hipError_t launch_blend_bwd(const Layout& L, void* ws, const uint32_t* sorted_vals, clod_params prm,
                            const float* T, const uint32_t* last, const float* dL_drgb, int64_t* pairs,
                            hipStream_t s) {
  if (L.tiles_total == 0) return hipSuccess;
  char* w = (char*)ws;
  const int nb = (int)xcd_grid(L.tiles_total);
  unsigned long long* part = pairs ? (unsigned long long*)(w + L.pair_part) : nullptr;
  if (part) {
    hipError_t e = launch_fill_u32((uint32_t*)part, 0u, 6 * (int64_t)L.tiles_total, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(part ? k_blend_bwd<true> : k_blend_bwd<false>, dim3(nb), dim3(kBlock), 0, s,
                     (const DevView*)(w + L.vinfo), L.V, L.tiles_total, L.VN, (const float4*)(w + L.rec),
                     (const uint2*)(w + L.ranges), sorted_vals, (const unsigned long long*)(w + L.hdr), prm.bg[0],
                     prm.bg[1], prm.bg[2], T, last, dL_drgb, (float*)(w + L.gscreen), (const uint32_t*)(w + L.order),
                     part);
  if (part)
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(kBlock), 0, s,
                       ReducePairsArgs{(const unsigned long long*)part, L.tiles_total, (unsigned long long*)pairs});
  return hipGetLastError();
}

}  // namespace clod
