// Training loss of Sec. 3.3: L_render = (1 - lambda_dssim) L1 + lambda_dssim (1 - SSIM) (the 3DGS
// rendering loss; the SSIM part is in ssim.hip), per view the mean absolute error and its
// gradient (1 - lambda_dssim) w_s sign(rgb - target) / (3 H W), the point-count regulariser of
// Eq. (4) on eta = n_mask / n with target s_v^-1.5 (Eq. 3), and the weighted total of Eq. (5).
#include "clod_internal.h"

namespace clod {

// Blocks are assigned to views by loss_block_base; each block covers kLossChunk values of
// one view's [3][H][W] image.
__global__ __launch_bounds__(kBlock) void k_loss_l1(const DevView* __restrict__ views, int V,
                                                    const float* __restrict__ rgb,
                                                    const float* __restrict__ target, float s_max,
                                                    float l1_weight, float* __restrict__ dL_drgb,
                                                    float* __restrict__ l1_part) {
  __shared__ float sred[4];
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].loss_block_base <= blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const DevView& Vw = views[lo];
  const int64_t cnt = 3ll * Vw.width * Vw.height;
  const int64_t base = 3ll * Vw.pix_base;
  const int64_t j0 = (int64_t)(blockIdx.x - Vw.loss_block_base) * kLossChunk;
  const float ws = w_s_weight(Vw.s_v, s_max);
  const float scale = l1_weight * ws / (float)cnt;
  float s = 0.f;
  auto one = [&](float r, float t, float& g) {
    const float diff = r - t;
    s += fabsf(diff);
    g = diff > 0.f ? scale : (diff < 0.f ? -scale : 0.f);
  };
  const float* rp = rgb + base;
  const float* tp = target + base;
  float* gp = dL_drgb + base;
  const bool vec = (((uintptr_t)rp | (uintptr_t)tp | (uintptr_t)gp) & 15u) == 0u;   // uniform per view
  if (vec) {
    // kLossItems / 4 float4 groups per thread, all loads issued before use.
    static_assert(kLossItems % 4 == 0, "float4 groups");
    constexpr int kV = kLossItems / 4;
    float4 r4[kV], t4[kV];
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int64_t j = j0 + 4 * ((int64_t)k * kBlock + threadIdx.x);
      if (j + 4 <= cnt) { r4[k] = *(const float4*)(rp + j); t4[k] = *(const float4*)(tp + j); }
    }
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int64_t j = j0 + 4 * ((int64_t)k * kBlock + threadIdx.x);
      if (j + 4 <= cnt) {
        float4 g4;
        one(r4[k].x, t4[k].x, g4.x);
        one(r4[k].y, t4[k].y, g4.y);
        one(r4[k].z, t4[k].z, g4.z);
        one(r4[k].w, t4[k].w, g4.w);
        *(float4*)(gp + j) = g4;
      } else {
        for (int64_t q = j; q < cnt && q < j + 4; ++q) one(rp[q], tp[q], gp[q]);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kLossItems; ++k) {
      const int64_t j = j0 + (int64_t)k * kBlock + threadIdx.x;
      if (j < cnt) one(rp[j], tp[j], gp[j]);
    }
  }
  s = wave_sum(s);
  if (lane_id() == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) l1_part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// Block v folds view v's partial sums: its L1 blocks and, with the D-SSIM term, the three
// channel partials of each of its SSIM regions.
__global__ __launch_bounds__(kBlock) void k_loss_reduce(const DevView* __restrict__ views, int V,
                                                        uint32_t loss_blocks, const float* __restrict__ l1_part,
                                                        const float* __restrict__ ssim_part, int with_ssim,
                                                        uint32_t ssim_regions,
                                                        float* __restrict__ l1_acc, float* __restrict__ ssim_acc) {
  __shared__ float sm[2][4];
  const int v = blockIdx.x;
  const DevView& Vw = views[v];
  const uint32_t b0 = Vw.loss_block_base;
  const uint32_t b1 = v + 1 < V ? views[v + 1].loss_block_base : loss_blocks;
  float a = 0.f, s = 0.f;
  for (uint32_t j = b0 + threadIdx.x; j < b1; j += kBlock) a += l1_part[j];
  if (with_ssim) {
    const int64_t t0 = 3ll * Vw.rgn_base, t1 = 3ll * (v + 1 < V ? views[v + 1].rgn_base : ssim_regions);
    for (int64_t j = t0 + threadIdx.x; j < t1; j += kBlock) s += ssim_part[j];
  }
  a = wave_sum(a);
  s = wave_sum(s);
  if (lane_id() == 0) { sm[0][threadIdx.x >> 6] = a; sm[1][threadIdx.x >> 6] = s; }
  __syncthreads();
  if (threadIdx.x == 0) {
    l1_acc[v] = sm[0][0] + sm[0][1] + sm[0][2] + sm[0][3];
    ssim_acc[v] = sm[1][0] + sm[1][1] + sm[1][2] + sm[1][3];
  }
}

__global__ void k_loss_scalars(const DevView* __restrict__ views, int V, int64_t n,
                               const unsigned long long* __restrict__ counts,
                               const float* __restrict__ l1_acc, const float* __restrict__ ssim_acc,
                               float s_max, float lambda_reg, float lambda_dssim,
                               float* __restrict__ loss, float* __restrict__ dL_deta) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const DevView& Vw = views[v];
  const float sv = Vw.s_v;
  const float cnt = 3.0f * (float)Vw.width * (float)Vw.height;
  const float l1 = l1_acc[v] / cnt;
  const float lr = lambda_dssim > 0.f ? (1.0f - lambda_dssim) * l1 + lambda_dssim * (1.0f - ssim_acc[v] / cnt) : l1;
  const float eta = n > 0 ? (float)counts[3 * v + 1] / (float)n : 0.f;
  const float eta_t = 1.0f / (sv * sqrtf(sv));
  const float ex = fmaxf(eta - eta_t, 0.f);
  const float w = (sv - 1.0f) * (sv - 1.0f);
  const float lreg = w * ex * ex;
  const float ws = w_s_weight(sv, s_max);
  loss[v] = ws * (lr + lambda_reg * lreg);
  if (dL_deta) dL_deta[v] = ws * lambda_reg * 2.0f * w * ex;
}

hipError_t launch_loss(const Layout& L, void* ws, int64_t n, const float* rgb, const float* target,
                       float s_max, float lambda_reg, float lambda_dssim, float* ssim_scratch, float* loss,
                       float* dL_drgb, float* dL_deta, uint32_t loss_blocks, hipStream_t s) {
  char* w = (char*)ws;
  float* acc = (float*)(w + L.loss_acc);
  float* sacc = (float*)(w + L.ssim_acc);
  float* spart = (float*)(w + L.loss_part);                   // [regions][3] SSIM partials
  float* lpart = spart + 3 * (int64_t)L.tiles_total;          // [loss blocks] L1 partials
  const DevView* views = (const DevView*)(w + L.vinfo);
  if (loss_blocks > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3(loss_blocks), dim3(kBlock), 0, s, views, L.V, rgb, target, s_max,
                       1.0f - lambda_dssim, dL_drgb, lpart);
  if (lambda_dssim > 0.f) {
    hipError_t e = launch_ssim(L, ws, rgb, target, lambda_dssim, s_max, ssim_scratch, spart, dL_drgb, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_loss_reduce, dim3(L.V), dim3(kBlock), 0, s, views, L.V, loss_blocks, (const float*)lpart,
                     (const float*)spart, lambda_dssim > 0.f ? 1 : 0, L.ssim_regions, acc, sacc);
  hipLaunchKernelGGL(k_loss_scalars, dim3((L.V + 63) / 64), dim3(64), 0, s, views, L.V, n,
                     (const unsigned long long*)(w + L.counts), (const float*)acc, (const float*)sacc, s_max,
                     lambda_reg, lambda_dssim, loss, dL_deta);
  return hipGetLastError();
}

}  // namespace clod
