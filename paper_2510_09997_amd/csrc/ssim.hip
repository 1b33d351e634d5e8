// D-SSIM part of the rendering loss (Sec. 3.3, Eq. (5): L_render is the 3DGS weighted sum of
// L1 and D-SSIM): SSIM per colour channel with an 11 x 11 Gaussian window (sigma 1.5), zero
// padding, C1 = 0.01^2, C2 = 0.03^2, averaged over all pixels and channels of a view.
//
// One 256-thread block per (16 x 16 tile, channel), one thread per output pixel; per-tile
// partial sums of the SSIM map (no same-address atomics), folded per view by the loss.
// The window sums use fused multiply-adds (this term is compared within a tolerance).  Forward:
// the tile and a 5-pixel halo of both images are staged in LDS, the five window moments
// (E[x], E[y], E[x^2], E[y^2], E[xy]) are filtered separably (rows, then columns), and per
// pixel the SSIM value and its derivatives with respect to the three moments that depend on
// the rendered image (E[x], E[x^2], E[xy]) are formed.  The derivatives, already scaled by
// dL/dS = -lambda w_s / (3 H W), go to a per-pixel scratch; the backward filters them back
// (the window is symmetric, so the adjoint of the zero-padded filter is the same filter) and
// adds dL/dx = F*a + 2 x F*b + y F*c to dL/drgb.
#include "clod_internal.h"

namespace clod {

constexpr int kHalo = 5;
constexpr int kWin = 2 * kHalo + 1;
constexpr int kSpan = kTile + 2 * kHalo;   // 26
constexpr float kC1 = 0.0001f;             // 0.01^2
constexpr float kC2 = 0.0009f;             // 0.03^2

__device__ __forceinline__ int view_of_tile_s(const DevView* views, int V, uint32_t tile) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_ssim_fwd(const DevView* __restrict__ views, int V,
                                                     const float* __restrict__ rgb, const float* __restrict__ target,
                                                     SsimWindow win, float lambda, float s_max,
                                                     float* __restrict__ coef, float* __restrict__ ssim_part) {
  __shared__ float sx[kSpan][kSpan + 1], sy[kSpan][kSpan + 1];
  __shared__ float hm[5][kSpan][kTile + 1];
  __shared__ float sred[4];
  const uint32_t tile = blockIdx.x;
  const int ch = blockIdx.y;
  const int v = view_of_tile_s(views, V, tile);
  const DevView& Vw = views[v];
  const int local = (int)(tile - Vw.tile_base);
  const int x0 = (local % Vw.tiles_x) * kTile, y0 = (local / Vw.tiles_x) * kTile;
  const int W = Vw.width, H = Vw.height;
  const int64_t HW = (int64_t)W * H;
  const int64_t img = 3ll * Vw.pix_base + (int64_t)ch * HW;
  for (int idx = threadIdx.x; idx < kSpan * kSpan; idx += kBlock) {
    const int r = idx / kSpan, c = idx % kSpan;
    const int gx = x0 - kHalo + c, gy = y0 - kHalo + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    sx[r][c] = in ? rgb[img + (int64_t)gy * W + gx] : 0.f;
    sy[r][c] = in ? target[img + (int64_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kSpan * kTile; idx += kBlock) {
    const int r = idx / kTile, c = idx % kTile;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const float g = win.g[k], xv = sx[r][c + k], yv = sy[r][c + k];
      a = fmaf(g, xv, a);
      b = fmaf(g, yv, b);
      aa = fmaf(g, xv * xv, aa);
      bb = fmaf(g, yv * yv, bb);
      ab = fmaf(g, xv * yv, ab);
    }
    hm[0][r][c] = a; hm[1][r][c] = b; hm[2][r][c] = aa; hm[3][r][c] = bb; hm[4][r][c] = ab;
  }
  __syncthreads();
  const int r = threadIdx.x / kTile, c = threadIdx.x % kTile;
  float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    const float g = win.g[k];
    mx = fmaf(g, hm[0][r + k][c], mx);
    my = fmaf(g, hm[1][r + k][c], my);
    exx = fmaf(g, hm[2][r + k][c], exx);
    eyy = fmaf(g, hm[3][r + k][c], eyy);
    exy = fmaf(g, hm[4][r + k][c], exy);
  }
  const int px = x0 + c, py = y0 + r;
  float s = 0.f;
  if (px < W && py < H) {
    const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    const float inv = 1.0f / (B1 * B2);
    s = A1 * A2 * inv;
    // dS/d(mu_x), dS/d(sigma_x^2), dS/d(sigma_xy), then the chain to the moments.
    const float d_mu = (2.f * my * A2) * inv - s * (2.f * mx) / B1;
    const float d_var = -s / B2;
    const float d_cov = 2.f * A1 * inv;
    const float up = -lambda * w_s_weight(Vw.s_v, s_max) / (3.0f * (float)HW);
    const int64_t p = (int64_t)py * W + px;
    const int64_t cb = 9ll * Vw.pix_base + (int64_t)(3 * ch) * HW;
    coef[cb + p] = up * (d_mu - 2.f * mx * d_var - my * d_cov);
    coef[cb + HW + p] = up * d_var;
    coef[cb + 2 * HW + p] = up * d_cov;
  }
  s = wave_sum(s);
  if (lane_id() == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) ssim_part[3 * (int64_t)tile + ch] = sred[0] + sred[1] + sred[2] + sred[3];
}

__global__ __launch_bounds__(kBlock) void k_ssim_bwd(const DevView* __restrict__ views, int V,
                                                     const float* __restrict__ rgb, const float* __restrict__ target,
                                                     SsimWindow win, const float* __restrict__ coef,
                                                     float* __restrict__ dL_drgb) {
  __shared__ float sc[3][kSpan][kSpan + 1];
  __shared__ float hm[3][kSpan][kTile + 1];
  const uint32_t tile = blockIdx.x;
  const int ch = blockIdx.y;
  const int v = view_of_tile_s(views, V, tile);
  const DevView& Vw = views[v];
  const int local = (int)(tile - Vw.tile_base);
  const int x0 = (local % Vw.tiles_x) * kTile, y0 = (local / Vw.tiles_x) * kTile;
  const int W = Vw.width, H = Vw.height;
  const int64_t HW = (int64_t)W * H;
  const int64_t cb = 9ll * Vw.pix_base + (int64_t)(3 * ch) * HW;
  for (int idx = threadIdx.x; idx < kSpan * kSpan; idx += kBlock) {
    const int r = idx / kSpan, c = idx % kSpan;
    const int gx = x0 - kHalo + c, gy = y0 - kHalo + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int64_t p = (int64_t)gy * W + gx;
#pragma unroll
    for (int j = 0; j < 3; ++j) sc[j][r][c] = in ? coef[cb + j * HW + p] : 0.f;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kSpan * kTile; idx += kBlock) {
    const int r = idx / kTile, c = idx % kTile;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) a = fmaf(win.g[k], sc[j][r][c + k], a);
      hm[j][r][c] = a;
    }
  }
  __syncthreads();
  const int r = threadIdx.x / kTile, c = threadIdx.x % kTile;
  const int px = x0 + c, py = y0 + r;
  if (px < W && py < H) {
    float fa = 0.f, fb = 0.f, fc = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const float g = win.g[k];
      fa = fmaf(g, hm[0][r + k][c], fa);
      fb = fmaf(g, hm[1][r + k][c], fb);
      fc = fmaf(g, hm[2][r + k][c], fc);
    }
    const int64_t q = 3ll * Vw.pix_base + (int64_t)ch * HW + (int64_t)py * W + px;
    dL_drgb[q] += fa + 2.f * rgb[q] * fb + target[q] * fc;
  }
}

hipError_t launch_ssim(const Layout& L, void* ws, const float* rgb, const float* target, float lambda,
                       float s_max, float* coef, float* ssim_part, float* dL_drgb, hipStream_t s) {
  if (L.tiles_total == 0) return hipSuccess;
  SsimWindow win;
  double g[kWin], sum = 0.0;
  for (int k = 0; k < kWin; ++k) {
    const double d = (double)(k - kHalo);
    g[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < kWin; ++k) win.g[k] = (float)(g[k] / sum);
  const DevView* views = (const DevView*)((char*)ws + L.vinfo);
  hipLaunchKernelGGL(k_ssim_fwd, dim3(L.tiles_total, 3), dim3(kBlock), 0, s, views, L.V, rgb, target, win, lambda,
                     s_max, coef, ssim_part);
  hipLaunchKernelGGL(k_ssim_bwd, dim3(L.tiles_total, 3), dim3(kBlock), 0, s, views, L.V, rgb, target, win,
                     (const float*)coef, dL_drgb);
  return hipGetLastError();
}

}  // namespace clod
