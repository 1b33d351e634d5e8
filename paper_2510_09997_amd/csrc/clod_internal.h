// Internal declarations of libclod: device view table, workspace layout, binary32 contract
// arithmetic for gfx950, and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/clod.h"

namespace clod {

constexpr int kTile = 16;                  // 16x16-pixel tiles
constexpr int kBlock = 256;                // threads per workgroup (4 wave64)
// One 64-byte record per (view, Gaussian), so the blend's gather of an entry touches one
// aligned 64-byte segment: (u, v, alpha'', radius), (conic A, B, C, 0), (r, g, b, 0), unused.
constexpr int kRecQuads = 4;
constexpr int kRecBytes = kRecQuads * 16;
constexpr int kScanItems = 16;             // items per thread in the tiles-touched scan
constexpr int kScanChunk = kBlock * kScanItems;
// Tile ordering by list length: 33 bucket counts + 33 bucket cursors + the number of long
// tiles (lists of at least 2^(kLongBucket - 1) entries, the leading positions of the order).
constexpr int kEmitTile = 2048;            // tile pairs per output chunk of the emission
constexpr int kTileBuckets = 33;
constexpr int kLongBucket = 14;            // long tiles: 8,192 entries or more
constexpr int kVeryLongBucket = 17;        // very long tiles: 65,536 entries or more
constexpr int kTileLongWord = 2 * kTileBuckets;
constexpr int kTileVeryLongWord = 2 * kTileBuckets + 1;
constexpr int kTileOrderWords = 2 * kTileBuckets + 2;
constexpr int kTileOrderChunk = 1024;       // tiles per block in the ordering kernels
constexpr int kSortItems = 8;              // keys per thread per radix tile
constexpr int kSortTile = kBlock * kSortItems;   // 2048 keys per radix tile
constexpr int kMaxSortBlocks = 1024;
constexpr int kMaxProjBlocks = 2048;      // per-block partial reductions of the per-Gaussian passes
constexpr int kGscreen = 9;                // du, dv, dA, dB, dC, dalpha'', dr, dg, db (interleaved per record)

// Per-view constants derived on the device from clod_view (k_view_setup).
struct DevView {
  float W[9], t[3], c[3];
  float fx, fy, cx, cy;
  float s_v, limx, limy, tau_sv;
  int32_t width, height, tiles_x, tiles_y;
  uint32_t tile_base, pix_base, loss_block_base, rgn_base;   // rgn_base: first 32 x 32 SSIM region
  int32_t ftiles_x, ftiles_y;    // tiles of the frame (the view's own when it is not a viewport)
  int32_t vx, vy;                // viewport origin in the frame, pixels (multiples of 16)
  int32_t cam_lead;              // first view of this view's run of consecutive views with the same
                                 // camera (pose, intrinsics, size, frame): they differ in s_v or
                                 // budget only, so positions, projections and colours are shared
  int64_t budget;                // 0: threshold mask; K > 0: the K largest selection keys
  unsigned long long mkey;       // K > 0: smallest kept selection key (set by the radix select)
};

// Radix select of the budgeted mask: per view, the threshold prefix found so far and the rank
// (1-based, from the largest key) still to find among keys that share it.
struct SelState {
  unsigned long long prefix, rank;
};
constexpr int kSelBlocks = 128;   // blocks per view of the select histograms

// Workspace header words (uint64).
enum : int { kHdrDup = 0, kHdrOverflow = 1, kHdrRend = 2, kHdrWords = 8 };

struct Layout {
  int64_t n = 0;
  int32_t V = 0;
  int64_t VN = 0;
  uint32_t tiles_total = 0;   // sum over views of tiles_x * tiles_y
  uint32_t ssim_regions = 0;  // sum over views of ceil(tiles_x / 2) * ceil(tiles_y / 2)
  int64_t pixels_total = 0;
  int32_t scan_blocks = 0;
  bool any_budget = false;    // some view selects by budget (allocates the select histograms)
  // byte offsets into ws
  size_t hdr, vinfo, dmax_key, counts, gdmax, loss_acc, kpart, cpart, gpart, ssim_acc, loss_part, sel_state, sel_hist, lcount, list, flags, alpha, rec,
      scan_part, ranges, order, tord, pair_part, gscreen, total;
};

// Host-side per-view geometry (must agree with k_view_setup).
struct HostView {
  int32_t width, height, tiles_x, tiles_y;
  uint32_t tile_base, pix_base, loss_blocks, loss_block_base;
};

constexpr int kLossItems = 8;
constexpr int kLossChunk = kBlock * kLossItems;

struct DupLayout {
  int64_t cap = 0;
  size_t keys0, vals0, keys1, vals1, hist, owner, total;
};

DupLayout dup_layout(int64_t cap);
int sort_blocks(int64_t cap);
int tile_passes(uint32_t tiles_total);     // radix passes of the tile-id sort
int sorted_buffer(uint32_t tiles_total);   // ping-pong buffer (0/1) holding the sorted pairs

// ----------------------------------------------------------------------------------------
// Binary32 contract arithmetic (device).  The translation units are compiled with
// -ffp-contract=off, so a*b+c stays two roundings; fused steps use __builtin_fmaf.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ float fmaf_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Float to int32 as the hardware converts (saturating; NaN gives 0).  A C++ conversion of a
// value outside the int32 range is undefined, which matters where lanes outside the live set
// evaluate the exponential on arbitrary arguments (their results are discarded).
__device__ __forceinline__ int cvt_i32_sat(float k) {
  int r;
  asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(k));
  return r;
}

// Contract exponential: Cody-Waite reduction with a 16-bit head of ln 2, degree-7 Taylor
// polynomial (1/j! rounded to binary32) in Horner form, scale by 2^k; zero below -86.
// The contract exponential for x in [-86, 88] (no range or NaN handling): cexp below adds
// those; the blend calls this directly on arguments it has already bounded (kAnyArg: or on any
// argument, for lanes whose result it discards; the result is then unspecified, but no
// operation is undefined, and inside the range it is the same).
template <bool kAnyArg = false>
__device__ __forceinline__ float cexp_core(float x) {
  constexpr float kL2E = 1.44269502162933349609375f;          // fl(1/ln 2)
  constexpr float kLn2Hi = 0.693145751953125f;                // floor(ln2 * 2^16) / 2^16
  constexpr float kLn2Lo = 1.428606765330187045037746429443359375e-06f;  // fl(ln2 - hi)
  constexpr float c7 = 1.98412701138295233249664306640625e-04f;   // fl(1/5040)
  constexpr float c6 = 1.388888922519981861114501953125e-03f;     // fl(1/720)
  constexpr float c5 = 8.3333337679505348205566406250e-03f;       // fl(1/120)
  constexpr float c4 = 4.1666667908430099487304687500e-02f;       // fl(1/24)
  constexpr float c3 = 1.6666667163372039794921875000e-01f;       // fl(1/6)
  float k = __builtin_rintf(x * kL2E);
  float r = fmaf_(-k, kLn2Hi, x);
  r = fmaf_(-k, kLn2Lo, r);
  float p = c7;
  p = fmaf_(p, r, c6);
  p = fmaf_(p, r, c5);
  p = fmaf_(p, r, c4);
  p = fmaf_(p, r, c3);
  p = fmaf_(p, r, 0.5f);
  p = fmaf_(p, r, 1.0f);
  p = fmaf_(p, r, 1.0f);
  // p * 2^k, exact for every k that cexp's clamped range produces (the result stays normal).
  return __builtin_amdgcn_ldexpf(p, kAnyArg ? cvt_i32_sat(k) : (int)k);
}

__device__ __forceinline__ float cexp(float x) {
  if (x != x) return x;
  if (x < -86.0f) return 0.0f;
  if (x > 88.0f) return __builtin_inff();
  return cexp_core(x);
}

// Real spherical harmonics, l <= 3, order l = 0..3, m = -l..l (Cartesian forms on the unit
// sphere).  Constants: closed-form normalisations rounded to binary32.
struct SHK {
  static constexpr float k0 = 0.282094791773878143f;   // 1/(2 sqrt(pi))
  static constexpr float k1 = 0.488602511902919921f;   // sqrt(3/(4 pi))
  static constexpr float k2a = 1.09254843059207907f;   // sqrt(15/pi)/2
  static constexpr float k2b = 0.315391565252520002f;  // sqrt(5/pi)/4
  static constexpr float k2c = 0.546274215296039535f;  // sqrt(15/pi)/4
  static constexpr float k3a = 0.590043589926643520f;  // sqrt(35/(2 pi))/4
  static constexpr float k3b = 2.89061144264055405f;   // sqrt(105/pi)/2
  static constexpr float k3c = 0.457045799464465739f;  // sqrt(21/(2 pi))/4
  static constexpr float k3d = 0.373176332590115391f;  // sqrt(7/pi)/4
  static constexpr float k3e = 1.44530572132027702f;   // sqrt(105/pi)/4
};

__device__ __forceinline__ void sh_basis(int deg, float X, float Y, float Z, float* y) {
  y[0] = SHK::k0;
  if (deg < 1) return;
  y[1] = SHK::k1 * Y;
  y[2] = SHK::k1 * Z;
  y[3] = SHK::k1 * X;
  if (deg < 2) return;
  const float xx = X * X, yy = Y * Y, zz = Z * Z;
  const float xy = X * Y, yz = Y * Z, xz = X * Z;
  y[4] = SHK::k2a * xy;
  y[5] = SHK::k2a * yz;
  y[6] = SHK::k2b * ((2.0f * zz - xx) - yy);
  y[7] = SHK::k2a * xz;
  y[8] = SHK::k2c * (xx - yy);
  if (deg < 3) return;
  const float t4 = (4.0f * zz - xx) - yy;
  y[9] = SHK::k3a * (Y * (3.0f * xx - yy));
  y[10] = SHK::k3b * (xy * Z);
  y[11] = SHK::k3c * (Y * t4);
  y[12] = SHK::k3d * (Z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
  y[13] = SHK::k3c * (X * t4);
  y[14] = SHK::k3e * (Z * (xx - yy));
  y[15] = SHK::k3a * (X * (xx - 3.0f * yy));
}

// Camera-space position (rows of W applied with the fused order of the contract).
__device__ __forceinline__ void to_camera(const DevView& V, float mx, float my, float mz,
                                          float& x, float& y, float& z) {
  x = fmaf_(V.W[0], mx, fmaf_(V.W[1], my, fmaf_(V.W[2], mz, V.t[0])));
  y = fmaf_(V.W[3], mx, fmaf_(V.W[4], my, fmaf_(V.W[5], mz, V.t[1])));
  z = fmaf_(V.W[6], mx, fmaf_(V.W[7], my, fmaf_(V.W[8], mz, V.t[2])));
}

__device__ __forceinline__ bool in_frustum(const DevView& V, float x, float y, float z, float near_z) {
  return (z > near_z) && (fabsf(x) <= V.limx * z) && (fabsf(y) <= V.limy * z);
}

// Squared camera distance; cam_distance is its correctly rounded square root, so the maximum
// distance over a set is the root of the maximum of these.
__device__ __forceinline__ float cam_distance2(const DevView& V, float mx, float my, float mz,
                                               float& ex, float& ey, float& ez) {
  ex = mx - V.c[0];
  ey = my - V.c[1];
  ez = mz - V.c[2];
  return fmaf_(ex, ex, fmaf_(ey, ey, ez * ez));
}

__device__ __forceinline__ float cam_distance(const DevView& V, float mx, float my, float mz,
                                              float& ex, float& ey, float& ez) {
  return __builtin_sqrtf(cam_distance2(V, mx, my, mz, ex, ey, ez));
}

__device__ __forceinline__ float sigmoid_c(float o) { return 1.0f / (1.0f + cexp(-o)); }

// The view-independent denominator of Eq. (2): 2 max(sigma_d, 0)^2 + eps.
__device__ __forceinline__ float decay_den(float decay, float eps) {
  const float r = fmaxf(decay, 0.0f);
  return fmaf_(2.0f * r, r, eps);
}

// Eq. (2) for one view with the per-Gaussian parts (alpha = sigmoid of the opacity logit and
// the decay denominator) computed once and passed in; returns alpha'' and q.
// From the normalised distance dn = d / d_max (the camera's part, shared by views that differ
// only in s_v).
__device__ __forceinline__ float attenuated_dn(float dn, float s_v, float alpha, float den, float& q) {
  const float u = dn * s_v;
  const float num = u * u;
  q = num / den;
  return alpha * cexp(-q);
}
__device__ __forceinline__ float attenuated_pre(float d, float dmax, float s_v, float alpha, float den,
                                                float& q) {
  return attenuated_dn(d / dmax, s_v, alpha, den, q);
}

// Attenuated opacity of Eq. (2) (also returns alpha and q for the adjoint).
__device__ __forceinline__ float attenuated(float d, float dmax, float s_v, float decay, float opac,
                                            float eps, float& alpha, float& q) {
  alpha = sigmoid_c(opac);
  return attenuated_pre(d, dmax, s_v, alpha, decay_den(decay, eps), q);
}

// EWA projection of one Gaussian.  Returns false when culled (det <= 0 or empty rect).
struct Proj {
  float u, v, A, B, C, rad;
  float ca, cb, cc, det;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ void quat_rot(float qw, float qx, float qy, float qz, float* R,
                                         float& w_, float& x_, float& y_, float& z_, float& rn) {
  const float n2 = fmaf_(qw, qw, fmaf_(qx, qx, fmaf_(qy, qy, qz * qz)));
  if (n2 > 0.0f) {
    rn = 1.0f / __builtin_sqrtf(n2);
    w_ = qw * rn; x_ = qx * rn; y_ = qy * rn; z_ = qz * rn;
  } else {
    rn = 0.0f;
    w_ = 1.0f; x_ = y_ = z_ = 0.0f;
  }
  const float xx = x_ * x_, yy = y_ * y_, zz = z_ * z_;
  const float xy = x_ * y_, xz = x_ * z_, yz = y_ * z_;
  const float wx = w_ * x_, wy = w_ * y_, wz = w_ * z_;
  R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
  R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
  R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
}

__device__ __forceinline__ void cov3(const float* R, float s0, float s1, float s2, float* S) {
  float M[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    M[3 * j + 0] = R[3 * j + 0] * s0;
    M[3 * j + 1] = R[3 * j + 1] * s1;
    M[3 * j + 2] = R[3 * j + 2] * s2;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j; k < 3; ++k) {
      const float v = fmaf_(M[3 * j], M[3 * k], fmaf_(M[3 * j + 1], M[3 * k + 1], M[3 * j + 2] * M[3 * k + 2]));
      S[3 * j + k] = v;
      S[3 * k + j] = v;
    }
}

// Projected 2D covariance (with dilation), conic, radius and rectangle.
__device__ __forceinline__ bool ewa(const DevView& V, float x, float y, float z, const float* S,
                                    float dil, Proj& P) {
  const float iz = 1.0f / z;
  const float tx = x * iz, ty = y * iz;
  const float j00 = V.fx * iz, j02 = -(V.fx * tx) * iz;
  const float j11 = V.fy * iz, j12 = -(V.fy * ty) * iz;
  float T[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T[k] = fmaf_(j00, V.W[k], j02 * V.W[6 + k]);
    T[3 + k] = fmaf_(j11, V.W[3 + k], j12 * V.W[6 + k]);
  }
  float U[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      U[3 * r + k] = fmaf_(T[3 * r], S[k], fmaf_(T[3 * r + 1], S[3 + k], T[3 * r + 2] * S[6 + k]));
  const float ca = fmaf_(U[0], T[0], fmaf_(U[1], T[1], U[2] * T[2])) + dil;
  const float cb = fmaf_(U[0], T[3], fmaf_(U[1], T[4], U[2] * T[5]));
  const float cc = fmaf_(U[3], T[3], fmaf_(U[4], T[4], U[5] * T[5])) + dil;
  const float det = fmaf_(ca, cc, -(cb * cb));
  P.ca = ca; P.cb = cb; P.cc = cc; P.det = det;
  if (!(det > 0.0f)) return false;
  const float idet = 1.0f / det;
  P.A = cc * idet;
  P.B = -cb * idet;
  P.C = ca * idet;
  const float mid = 0.5f * (ca + cc);
  const float lam = mid + __builtin_sqrtf(fmaxf(0.0f, fmaf_(mid, mid, -det)));
  const float rad = __builtin_ceilf(3.0f * __builtin_sqrtf(lam));
  P.rad = rad;
  P.u = fmaf_(V.fx, tx, V.cx);
  P.v = fmaf_(V.fy, ty, V.cy);
  // Rectangle in frame tiles, clamped to the frame, then clipped to the viewport (viewport tiles).
  const float TWf = (float)V.ftiles_x, THf = (float)V.ftiles_y;
  float fx0 = __builtin_floorf((P.u - rad) * 0.0625f), fx1 = __builtin_floorf((P.u + rad) * 0.0625f) + 1.0f;
  float fy0 = __builtin_floorf((P.v - rad) * 0.0625f), fy1 = __builtin_floorf((P.v + rad) * 0.0625f) + 1.0f;
  fx0 = fminf(fmaxf(fx0, 0.0f), TWf); fx1 = fminf(fmaxf(fx1, 0.0f), TWf);
  fy0 = fminf(fmaxf(fy0, 0.0f), THf); fy1 = fminf(fmaxf(fy1, 0.0f), THf);
  const int tox = V.vx >> 4, toy = V.vy >> 4;
  P.x0 = max((int)fx0, tox) - tox; P.x1 = min((int)fx1, tox + V.tiles_x) - tox;
  P.y0 = max((int)fy0, toy) - toy; P.y1 = min((int)fy1, toy + V.tiles_y) - toy;
  return P.x0 < P.x1 && P.y0 < P.y1;
}

// Record written by the projection for each rendered (view, Gaussian), kRecQuads float4:
//   (u, v, alpha'', radius), (A, B, C, 0), (r, g, b, 0), (depth, x0 | x1 << 16, y0 | y1 << 16,
//   tiles touched) with the last three as uint32 bits; (u, v) in frame pixels.
// flags: bit0 F, bit1 M, bit2 rendered, bits3..5 colour clamp per channel.

__device__ __forceinline__ float dmax_from_key(unsigned long long key) {
  return key == 0ull ? 1.0f : __uint_as_float((uint32_t)(key >> 32));
}

// Block b of a stage: its index and the stage's block count.  A per-stage launch takes them
// from blockIdx.x and gridDim.x; the persistent server passes the item it claimed.
struct Blk {
  uint32_t id, n;
};
__device__ __forceinline__ Blk grid_blk() { return Blk{blockIdx.x, gridDim.x}; }

// Contiguous chunk [lo, hi) of n items owned by block b (grids capped at kMaxProjBlocks).
__device__ __forceinline__ void block_chunk(int64_t n, Blk b, int64_t& lo, int64_t& hi) {
  const int64_t per = (n + b.n - 1) / b.n;
  lo = (int64_t)b.id * per;
  hi = lo + per;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
}
__device__ __forceinline__ void block_chunk(int64_t n, int64_t& lo, int64_t& hi) { block_chunk(n, grid_blk(), lo, hi); }

// Wave64 helpers.
__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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


template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_read(float x) {
  // Lanes of rows outside kRowMask receive 0.
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, kRowMask, 0xF, false));
}

// Totals over the wave of eight per-lane values at once: lanes 8g .. 8g+7 end with the total of
// v[g].  Each exchange halves the number of live values: permlane32 swaps (halves of the wave),
// permlane16 swaps (rows of a half), a rotation by 8 within rows, then three DPP steps within
// groups of 8 lanes.  18 instructions instead of eight separate reductions.  Every lane of the
// wave must be active.
__device__ __forceinline__ float wave_sum8(const float (&v)[8]) {
  auto swap32 = [](float a, float b) {   // [a_lo + a_hi | b_lo + b_hi]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  };
  auto swap16 = [](float a, float b) {   // rows [a0 + a1 | b0 + b1 | a2 + a3 | b2 + b3]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  };
  const float r0 = swap32(v[0], v[4]), r1 = swap32(v[1], v[5]), r2 = swap32(v[2], v[6]), r3 = swap32(v[3], v[7]);
  const float s0 = swap16(r0, r2), s1 = swap16(r1, r3);   // rows: (v0 v2 v4 v6), (v1 v3 v5 v7)
  const bool hi8 = (__lane_id() & 8u) != 0u;
  const float keep = hi8 ? s1 : s0, send = hi8 ? s0 : s1;
  float u = keep + dpp_read<0x128, 0xF>(send);           // row_ror:8; lanes 8g..8g+7 hold v[g]
  u += dpp_read<0x141, 0xF>(u);                          // row_half_mirror
  u += dpp_read<0x4E, 0xF>(u);                           // quad_perm (2, 3, 0, 1)
  u += dpp_read<0xB1, 0xF>(u);                           // quad_perm (1, 0, 3, 2)
  return u;
}

// Sum over the 64 lanes of a wave with DPP lane moves fused into the adds (no LDS traffic):
// quad swaps give quad sums, the half-row and row mirrors give row (16-lane) sums, and the
// two row broadcasts fold rows 0-2 into row 3.  Returns the total as a wave-uniform value.
// Every lane of the wave must be active.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_read<0xB1, 0xF>(v);    // quad_perm (1, 0, 3, 2)
  v += dpp_read<0x4E, 0xF>(v);    // quad_perm (2, 3, 0, 1)
  v += dpp_read<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_read<0x140, 0xF>(v);   // row_mirror
  v += dpp_read<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_read<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Weight of Eq. (5): w_s = (1 - 0.5 s_v / max(s_v))^2.
__device__ __forceinline__ float w_s_weight(float s_v, float s_max) {
  const float t = 1.0f - 0.5f * s_v / s_max;
  return t * t;
}

// 11-tap normalised Gaussian window (sigma 1.5) of the SSIM term.
struct SsimWindow {
  float g[11];
};

// LoD selection key of a (view, Gaussian): larger alpha'' first, then lower index (alpha'' >= 0,
// so its bit pattern is monotone).  Keys are distinct, so keeping the keys >= the K-th largest
// keeps exactly K Gaussians.
__device__ __forceinline__ unsigned long long lod_key(float a2, int64_t i) {
  return ((unsigned long long)__float_as_uint(a2) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
}

// The LoD mask M of a (view, Gaussian): alpha'' > tau s_v (Sec. 3.2), or membership in the view's
// budget of largest alpha''.
__device__ __forceinline__ bool lod_kept(const DevView& Vw, float a2, int64_t i) {
  return Vw.budget > 0 ? lod_key(a2, i) >= Vw.mkey : a2 > Vw.tau_sv;
}

// ----------------------------------------------------------------------------------------
// Stages of the forward path.  Projection, binning and blending run as a fixed sequence of
// stages; a stage is a grid of independent 256-thread blocks that may start once the previous
// stage has finished.  The launchers below describe each stage (kind, block count, arguments)
// to a Sink, which either launches it at once as its own kernel on a stream or appends it to a
// Program; the persistent server executes such programs from its device queue.  Both
// executors therefore run the same sequence with the same arguments.
// ----------------------------------------------------------------------------------------
enum StageKind : int32_t {
  kStViewSetup = 1, kStFill, kStFrustumMax, kStFold, kStClassify, kStProject, kStSelectHist, kStSelectPick,
  kStScanReduce, kStScanPartials, kStCompact, kStRadixUp, kStRadixScan, kStRadixDown, kStEmitReduce,
  kStEmitPartials, kStEmitOffsets, kStEmit, kStRanges, kStTileCount, kStTileScatter, kStBlend, kStReducePairs,
  kStLongMask
};

struct ViewSetupArgs {
  const clod_view* views; int32_t V; clod_params prm; DevView* out; unsigned long long* hdr;
};
struct FillArgs {
  uint32_t* p; uint32_t value; int64_t count;
};
struct FrustumArgs {
  const float* mean; int64_t n; const DevView* views; int32_t V; float near_z; unsigned long long* part;
};
struct FoldArgs {   // per-view folds of the per-block partials (frustum maximum or counts)
  const unsigned long long* kpart; const uint32_t* cpart; int32_t G, V; unsigned long long* dmax_key;
  unsigned long long* counts; int64_t* counts_dev; int64_t n; float* eta_dev;
};
struct ClassifyArgs {
  clod_scene sc; const DevView* views; int32_t V, write; clod_params prm; const unsigned long long* dmax_key;
  uint32_t* cpart; uint8_t* flags; float* alpha; uint32_t* list; uint32_t* lcount;
};
struct ProjectArgs {
  clod_scene sc; const DevView* views; int32_t V; clod_params prm; const unsigned long long* dmax_key;
  uint32_t* cpart; const uint32_t* list; const uint32_t* lcount; uint8_t* flags; float4* rec;
  int32_t write, packed;   // records written; colours from the packed coefficients
};
struct SelectArgs {
  clod_scene sc; DevView* views; int32_t V; clod_params prm; const unsigned long long* dmax_key;
  SelState* state; uint32_t* hist; int32_t pass;
};
struct ScanReduceArgs {
  const uint8_t* flags; int64_t count; uint32_t* partR; uint32_t* ranges; int64_t range_words;
};
struct ScanPartialsArgs {
  uint32_t* partR; int32_t nparts; unsigned long long* hdr; int64_t cap; uint32_t* tord;
};
struct CompactArgs {
  const uint8_t* flags; int64_t count; const uint32_t* partR; const float4* rec; const unsigned long long* hdr;
  uint32_t* kout; uint32_t* vout;
};
struct RadixArgs {   // one pass: upsweep, digit scan and downsweep share it
  const uint32_t* kin; const uint32_t* vin; uint32_t* kout; uint32_t* vout; uint32_t* hist;
  const unsigned long long* hdr; int32_t cw, G, shift;
};
struct EmitReduceArgs {
  const uint32_t* sorted_f; const float4* rec; const uint8_t* flags; int64_t count; const unsigned long long* hdr;
  uint32_t* partE; uint32_t* tsorted;
};
struct EmitPartialsArgs {
  uint32_t* partE; unsigned long long* hdr; int32_t nb; int64_t cap;
};
struct EmitOffsetsArgs {
  const uint32_t* tsorted; const uint32_t* partE; const unsigned long long* hdr; uint32_t* eoff; uint32_t* owner;
};
struct EmitArgs {
  const uint32_t* sorted_f; const uint32_t* eoff; const uint32_t* owner; const float4* rec; const DevView* views;
  int64_t n; const unsigned long long* hdr; uint32_t* kout; uint32_t* vout;
};
struct RangesArgs {
  const uint32_t* keys; const unsigned long long* hdr; uint32_t tiles_total; uint2* ranges;
};
struct TileOrderArgs {
  const uint2* ranges; uint32_t tiles; const unsigned long long* hdr; uint32_t* tord; uint32_t* order;
};
struct BlendArgs {
  const DevView* views; int32_t V; uint32_t tiles_total; int64_t VN; const float4* rec; const uint2* ranges;
  const uint32_t* svals; const unsigned long long* hdr; float bg0, bg1, bg2; float* rgb; float* T; uint32_t* last;
  unsigned long long* pair_part; const uint32_t* order; const uint32_t* tord;
  uint32_t long_max;      // most long tiles the launch covers (the pair capacity's bound)
  int32_t count;
  // Very long tiles (at most vl_max of them): per 4x4 block b of the tile, one bit per list
  // entry (set if the entry may reach the block), 64 entries per word, the tile's words at
  // lplane[b * pw + rg.x / 64 + tile + w] (from kStLongMask).
  const unsigned long long* lplane; uint32_t pw; uint32_t vl_max;
};
struct LongMaskArgs {
  const DevView* views; int32_t V; const uint2* ranges; const uint32_t* order; const uint32_t* tord;
  const uint32_t* svals; const float4* rec; int64_t VN; const unsigned long long* hdr;
  unsigned long long* lplane; uint32_t pw; uint32_t vl_max;
};
struct ReducePairsArgs {
  const unsigned long long* part; uint32_t tiles; unsigned long long* out;
};

struct Stage {
  int32_t kind;
  uint32_t items;   // blocks
  uint32_t block;   // threads per block of the per-stage launch (the server always runs 256)
  uint32_t lds;     // dynamic LDS bytes of the per-stage launch
  union {
    ViewSetupArgs view_setup; FillArgs fill; FrustumArgs frustum; FoldArgs fold; ClassifyArgs classify;
    ProjectArgs project; SelectArgs select; ScanReduceArgs scan_reduce; ScanPartialsArgs scan_partials;
    CompactArgs compact; RadixArgs radix; EmitReduceArgs emit_reduce; EmitPartialsArgs emit_partials;
    EmitOffsetsArgs emit_offsets; EmitArgs emit; RangesArgs ranges; TileOrderArgs tile_order; BlendArgs blend;
    ReducePairsArgs reduce_pairs; LongMaskArgs long_mask;
  } a;
};

constexpr int kMaxStages = 80;
struct Program {
  int32_t n = 0;
  bool full = false;
  Stage st[kMaxStages];
};

hipError_t launch_stage(const Stage& st, hipStream_t s);
hipError_t launch_project_stage(const Stage& st, hipStream_t s);
hipError_t launch_sort_stage(const Stage& st, hipStream_t s);
hipError_t launch_blend_stage(const Stage& st, hipStream_t s);

// Where the launchers send their stages: launched at once on `stream`, or appended to `prog`.
struct Sink {
  hipStream_t stream = nullptr;
  Program* prog = nullptr;
  Sink(hipStream_t s) : stream(s) {}
  explicit Sink(Program* p) : prog(p) {}
  hipError_t put(const Stage& st) const {
    if (st.items == 0) return hipSuccess;
    if (!prog) return launch_stage(st, stream);
    if (prog->n >= kMaxStages) {
      prog->full = true;
      return hipErrorInvalidValue;
    }
    prog->st[prog->n++] = st;
    return hipSuccess;
  }
};

// Scene preparation (spatial order): device sections of the caller's workspace, and the gather
// of the planes.
struct OrderBufs {
  uint32_t* box;              // 6 order keys: min x, y, z; max x, y, z
  unsigned long long* hdr;    // kHdrWords header words (count in kHdrRend)
  uint32_t* hist;             // (256 G + 256) radix counts
  uint32_t* keys[2];          // codes, ping-pong
  uint32_t* vals[2];          // indices, ping-pong; vals[0] is the caller's permutation
  int G;                      // radix blocks
};
struct OrderGatherArgs {
  const float* src[6]; float* dst[6]; int planes[6]; int64_t n; const uint32_t* perm;
};
hipError_t launch_scene_reorder(const clod_scene& src, const clod_scene_grad& dst, const OrderBufs& ob, hipStream_t s);

// ----------------------------------------------------------------------------------------
// Launchers (each returns the first launch error, or hipSuccess).
// ----------------------------------------------------------------------------------------
hipError_t launch_view_setup(const clod_view* views_dev, int V, clod_params prm, DevView* vinfo,
                             unsigned long long* hdr /* cleared when non-NULL */, const Sink& out);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, const Sink& out);
int proj_blocks(int64_t n);
hipError_t launch_frustum_max(const clod_scene& sc, const DevView* vinfo, int V, float near_z,
                              unsigned long long* kpart, unsigned long long* dmax_key, const Sink& out);
// counts (workspace) and counts_dev (caller's int64 [V][3], nullable) receive the per-view
// {frustum, mask, rendered} counts.
hipError_t launch_project(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                          unsigned long long* dmax_key, uint32_t* cpart, unsigned long long* counts,
                          int64_t* counts_dev, float* eta_dev, uint8_t* flags, float* alpha, float4* rec, uint32_t* list,
                          uint32_t* lcount, const Sink& out);
hipError_t launch_lod_count(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                            unsigned long long* dmax_key, uint32_t* cpart, unsigned long long* counts,
                            int64_t* counts_dev, float* eta_dev, uint32_t* list, uint32_t* lcount, const Sink& out);

// Fused Adam: one segment per learning-rate group.
constexpr int kAdamGroups = 7;
constexpr int kAdamChunk = 8192;   // parameters per block of the Adam launch
struct AdamSeg {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t count;
  float lr;
  int vec;   // all four planes 16-byte aligned: float4 accesses
};
struct AdamSegs {
  AdamSeg s[kAdamGroups];
  int64_t first_block[kAdamGroups + 1];   // blocks of segment j: [first_block[j], first_block[j+1])
};
hipError_t launch_adam(const AdamSegs& segs, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_lod_select(const clod_scene& sc, DevView* vinfo, int V, clod_params prm,
                             const unsigned long long* dmax_key, SelState* state, uint32_t* hist, const Sink& out);

hipError_t launch_bin_sort(const Layout& L, void* ws, const DupLayout& D, void* dup, const Sink& out);
hipError_t launch_ranges(const Layout& L, void* ws, const DupLayout& D, void* dup, int parity,
                         const Sink& out);

// The pair buffers the forward blend reads: the sorted record indices, and the two arrays the
// tile-id sort left free (they hold the very long tiles' block bit planes).
struct BlendBufs {
  const uint32_t* svals; unsigned long long* spare; size_t spare_bytes; int64_t cap;
};
hipError_t launch_blend_fwd(const Layout& L, void* ws, const BlendBufs& bb, clod_params prm, float* rgb, float* T,
                            uint32_t* last, int64_t* pairs, const Sink& out);
hipError_t launch_blend_bwd(const Layout& L, void* ws, const uint32_t* sorted_vals, clod_params prm,
                            const float* T, const uint32_t* last, const float* dL_drgb, int64_t* pairs,
                            hipStream_t s);
hipError_t launch_clear_rendered(const Layout& L, void* ws, hipStream_t s);
hipError_t launch_gauss_bwd(const clod_scene& sc, const Layout& L, void* ws, clod_params prm,
                            const float* dL_deta, int accumulate, const clod_scene_grad& g,
                            hipStream_t s);
hipError_t launch_loss(const Layout& L, void* ws, int64_t n, const float* rgb, const float* target,
                       float s_max, float lambda_reg, float lambda_dssim, float* ssim_scratch, float* loss,
                       float* dL_drgb, float* dL_deta, uint32_t loss_blocks, hipStream_t s);
// Persistent server (server.hip): jobs are forward-render Programs.
constexpr int kSrvSlots = 16;      // jobs in flight
constexpr int kSrvMaxViews = 16;   // views per job
enum SrvStatus : uint32_t { kSrvRunning = 0, kSrvStopped = 1, kSrvDeadline = 2, kSrvProtocol = 3, kSrvUnsupported = 4 };
struct Server;
hipError_t server_start(int32_t workers, double max_seconds, hipStream_t s, Server** out, int32_t* used_workers);
const clod_view* server_views_dev(Server* S, int64_t seq);   // device copy of job seq's views
int64_t server_next_seq(Server* S);
bool server_slot_free(Server* S);                             // the next job's slot is free
hipError_t server_publish(Server* S, const Program& P, int32_t n_views, const clod_view* views_host,
                          const void* hdr_dev, int64_t* seq);
int server_poll(Server* S, int64_t seq, int64_t* info);
int64_t server_clock_ns(Server* S);
int server_stage_times(Server* S, int64_t seq, int64_t* ns, int32_t* kinds, int32_t max);
hipError_t server_stop(Server* S, int32_t* status);

hipError_t launch_ssim(const Layout& L, void* ws, const float* rgb, const float* target, float lambda,
                       float s_max, float* coef, float* ssim_part, float* dL_drgb, hipStream_t s);
constexpr int kSsimRegion = 32;   // output edge of one SSIM block (2 x 2 tiles)

}  // namespace clod
