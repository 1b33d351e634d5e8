// D-SSIM part of the rendering loss (Sec. 3.3, Eq. (5): L_render is the 3DGS weighted sum of
// L1 and D-SSIM): SSIM per colour channel with an 11 x 11 Gaussian window (sigma 1.5), zero
// padding, C1 = 0.01^2, C2 = 0.03^2, averaged over all pixels and channels of a view.
//
// One 256-thread block per (32 x 32 region, channel), four outputs per thread in every pass;
// per-region partial sums of the SSIM map (no same-address atomics), folded per view by the
// loss.  The window sums use fused multiply-adds in window order (this term is compared
// within a tolerance).  Forward: the region and a 5-pixel halo of both images are staged in
// LDS, the five window moments (E[x], E[y], E[x^2], E[y^2], E[xy]) are filtered separably --
// each thread filters four consecutive columns of a row from 14 loaded values, then four
// consecutive rows of a column from 14 -- and per pixel the SSIM value and its derivatives
// with respect to the three moments that depend on the rendered image (E[x], E[x^2], E[xy])
// are formed.  The derivatives, already scaled by dL/dS = -lambda w_s / (3 H W), go to a
// per-pixel scratch; the backward filters them back the same way (the window is symmetric,
// so the adjoint of the zero-padded filter is the same filter) and adds
// dL/dx = F*a + 2 x F*b + y F*c to dL/drgb.
#include "clod_internal.h"

namespace clod {

constexpr int kHalo = 5;
constexpr int kWin = 2 * kHalo + 1;
constexpr int kR = kSsimRegion;            // 32 outputs per region edge
constexpr int kS = kR + 2 * kHalo;         // 42 staged rows / columns
constexpr int kQ = 4;                      // outputs per thread per pass
constexpr int kL = kWin + kQ - 1;          // 14 inputs per four outputs
constexpr float kC1 = 0.0001f;             // 0.01^2
constexpr float kC2 = 0.0009f;             // 0.03^2
static_assert(kR * (kR / kQ) == kBlock, "one column task (four rows of one column) per thread");
constexpr int kStage = (kS * kS + kBlock - 1) / kBlock;   // staged elements per thread (7)

struct Region {
  int v, x0, y0;
};

// View and pixel origin of region r (binary search of the views' first regions).
__device__ __forceinline__ Region region_of(const DevView* views, int V, uint32_t r) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].rgn_base <= r) lo = mid; else hi = mid - 1;
  }
  const DevView& Vw = views[lo];
  const int rx = (Vw.tiles_x + 1) / 2;
  const int local = (int)(r - Vw.rgn_base);
  return Region{lo, (local % rx) * kR, (local / rx) * kR};
}

__global__ __launch_bounds__(kBlock) void k_ssim_fwd(const DevView* __restrict__ views, int V,
                                                     const float* __restrict__ rgb, const float* __restrict__ target,
                                                     SsimWindow win, float lambda, float s_max,
                                                     float* __restrict__ coef, float* __restrict__ ssim_part) {
  __shared__ float sx[kS][kS + 1], sy[kS][kS + 1];
  __shared__ float hm[5][kS][kR + 1];
  __shared__ float sred[4];
  const uint32_t region = blockIdx.x;
  const int ch = blockIdx.y;
  const Region R = region_of(views, V, region);
  const DevView& Vw = views[R.v];
  const int x0 = R.x0, y0 = R.y0;
  const int W = Vw.width, H = Vw.height;
  const int64_t HW = (int64_t)W * H;
  const int64_t img = 3ll * Vw.pix_base + (int64_t)ch * HW;
  // Staging: every load of the thread is issued before the first LDS store.
  {
    float lx[kStage], ly[kStage];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int idx = (int)threadIdx.x + q * kBlock;
      const int r = idx / kS, c = idx - r * kS;
      const int gx = x0 - kHalo + c, gy = y0 - kHalo + r;
      const bool in = idx < kS * kS && gx >= 0 && gx < W && gy >= 0 && gy < H;
      lx[q] = in ? rgb[img + (int64_t)gy * W + gx] : 0.f;
      ly[q] = in ? target[img + (int64_t)gy * W + gx] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int idx = (int)threadIdx.x + q * kBlock;
      if (idx < kS * kS) {
        const int r = idx / kS, c = idx - r * kS;
        sx[r][c] = lx[q];
        sy[r][c] = ly[q];
      }
    }
  }
  __syncthreads();
  // Rows: task (r, c0) filters columns c0 .. c0 + 3 of staged row r.
  for (int task = threadIdx.x; task < kS * (kR / kQ); task += kBlock) {
    const int r = task / (kR / kQ), c0 = (task % (kR / kQ)) * kQ;
    float xs[kL], ys[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) { xs[k] = sx[r][c0 + k]; ys[k] = sy[r][c0 + k]; }
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        const float g = win.g[k], xv = xs[j + k], yv = ys[j + k];
        a = fmaf(g, xv, a);
        b = fmaf(g, yv, b);
        aa = fmaf(g, xv * xv, aa);
        bb = fmaf(g, yv * yv, bb);
        ab = fmaf(g, xv * yv, ab);
      }
      hm[0][r][c0 + j] = a; hm[1][r][c0 + j] = b; hm[2][r][c0 + j] = aa; hm[3][r][c0 + j] = bb; hm[4][r][c0 + j] = ab;
    }
  }
  __syncthreads();
  // Columns: thread (c, r0) filters rows r0 .. r0 + 3 of output column c.
  const int c = threadIdx.x % kR, r0 = (threadIdx.x / kR) * kQ;
  float mom[5][kQ];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    float col[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) col[k] = hm[m][r0 + k][c];
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(win.g[k], col[j + k], acc);
      mom[m][j] = acc;
    }
  }
  const float up = -lambda * w_s_weight(Vw.s_v, s_max) / (3.0f * (float)HW);
  const int64_t cb = 9ll * Vw.pix_base + (int64_t)(3 * ch) * HW;
  const int px = x0 + c;
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    const int py = y0 + r0 + j;
    if (px < W && py < H) {
      const float mx = mom[0][j], my = mom[1][j], exx = mom[2][j], eyy = mom[3][j], exy = mom[4][j];
      const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
      const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
      const float inv = 1.0f / (B1 * B2);
      const float sv = A1 * A2 * inv;
      // dS/d(mu_x), dS/d(sigma_x^2), dS/d(sigma_xy), then the chain to the moments.
      const float d_mu = (2.f * my * A2) * inv - sv * (2.f * mx) / B1;
      const float d_var = -sv / B2;
      const float d_cov = 2.f * A1 * inv;
      const int64_t p = (int64_t)py * W + px;
      coef[cb + p] = up * (d_mu - 2.f * mx * d_var - my * d_cov);
      coef[cb + HW + p] = up * d_var;
      coef[cb + 2 * HW + p] = up * d_cov;
      s += sv;
    }
  }
  s = wave_sum(s);
  if (lane_id() == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) ssim_part[3 * (int64_t)region + ch] = sred[0] + sred[1] + sred[2] + sred[3];
}

__global__ __launch_bounds__(kBlock) void k_ssim_bwd(const DevView* __restrict__ views, int V,
                                                     const float* __restrict__ rgb, const float* __restrict__ target,
                                                     SsimWindow win, const float* __restrict__ coef,
                                                     float* __restrict__ dL_drgb) {
  __shared__ float sc[3][kS][kS + 1];
  __shared__ float hm[3][kS][kR + 1];
  const uint32_t region = blockIdx.x;
  const int ch = blockIdx.y;
  const Region R = region_of(views, V, region);
  const DevView& Vw = views[R.v];
  const int x0 = R.x0, y0 = R.y0;
  const int W = Vw.width, H = Vw.height;
  const int64_t HW = (int64_t)W * H;
  const int64_t cb = 9ll * Vw.pix_base + (int64_t)(3 * ch) * HW;
  {
    float lc[3][kStage];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int idx = (int)threadIdx.x + q * kBlock;
      const int r = idx / kS, c = idx - r * kS;
      const int gx = x0 - kHalo + c, gy = y0 - kHalo + r;
      const bool in = idx < kS * kS && gx >= 0 && gx < W && gy >= 0 && gy < H;
      const int64_t p = (int64_t)gy * W + gx;
#pragma unroll
      for (int j = 0; j < 3; ++j) lc[j][q] = in ? coef[cb + j * HW + p] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int idx = (int)threadIdx.x + q * kBlock;
      if (idx < kS * kS) {
        const int r = idx / kS, c = idx - r * kS;
#pragma unroll
        for (int j = 0; j < 3; ++j) sc[j][r][c] = lc[j][q];
      }
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < kS * (kR / kQ); task += kBlock) {
    const int r = task / (kR / kQ), c0 = (task % (kR / kQ)) * kQ;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float xs[kL];
#pragma unroll
      for (int k = 0; k < kL; ++k) xs[k] = sc[j][r][c0 + k];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) a = fmaf(win.g[k], xs[q + k], a);
        hm[j][r][c0 + q] = a;
      }
    }
  }
  __syncthreads();
  const int c = threadIdx.x % kR, r0 = (threadIdx.x / kR) * kQ;
  float f[3][kQ];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    float col[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) col[k] = hm[j][r0 + k][c];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(win.g[k], col[q + k], acc);
      f[j][q] = acc;
    }
  }
  const int px = x0 + c;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int py = y0 + r0 + q;
    if (px < W && py < H) {
      const int64_t i = 3ll * Vw.pix_base + (int64_t)ch * HW + (int64_t)py * W + px;
      dL_drgb[i] += f[0][q] + 2.f * rgb[i] * f[1][q] + target[i] * f[2][q];
    }
  }
}

hipError_t launch_ssim(const Layout& L, void* ws, const float* rgb, const float* target, float lambda,
                       float s_max, float* coef, float* ssim_part, float* dL_drgb, hipStream_t s) {
  if (L.ssim_regions == 0) return hipSuccess;
  SsimWindow win;
  double g[kWin], sum = 0.0;
  for (int k = 0; k < kWin; ++k) {
    const double d = (double)(k - kHalo);
    g[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < kWin; ++k) win.g[k] = (float)(g[k] / sum);
  const DevView* views = (const DevView*)((char*)ws + L.vinfo);
  hipLaunchKernelGGL(k_ssim_fwd, dim3(L.ssim_regions, 3), dim3(kBlock), 0, s, views, L.V, rgb, target, win, lambda,
                     s_max, coef, ssim_part);
  hipLaunchKernelGGL(k_ssim_bwd, dim3(L.ssim_regions, 3), dim3(kBlock), 0, s, views, L.V, rgb, target, win,
                     (const float*)coef, dL_drgb);
  return hipGetLastError();
}

}  // namespace clod
