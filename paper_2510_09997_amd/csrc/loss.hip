// Training loss of Sec. 3.3 with L_render = L1: per view the mean absolute error, its
// gradient w_s sign(rgb - target) / (3 H W), the point-count regulariser of Eq. (4) on
// eta = n_mask / n with target s_v^-1.5 (Eq. 3), and the weighted total of Eq. (5).
#include "clod_internal.h"

namespace clod {

__device__ __forceinline__ float w_s(float s_v, float s_max) {
  const float t = 1.0f - 0.5f * s_v / s_max;
  return t * t;
}

// Blocks are assigned to views by loss_block_base; each block covers kLossChunk values of
// one view's [3][H][W] image.
__global__ __launch_bounds__(kBlock) void k_loss_l1(const DevView* __restrict__ views, int V,
                                                    const float* __restrict__ rgb,
                                                    const float* __restrict__ target, float s_max,
                                                    float* __restrict__ dL_drgb,
                                                    float* __restrict__ l1_acc) {
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
  const float ws = w_s(Vw.s_v, s_max);
  const float scale = ws / (float)cnt;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kLossItems; ++k) {
    const int64_t j = j0 + (int64_t)k * kBlock + threadIdx.x;
    if (j < cnt) {
      const float diff = rgb[base + j] - target[base + j];
      s += fabsf(diff);
      dL_drgb[base + j] = diff > 0.f ? scale : (diff < 0.f ? -scale : 0.f);
    }
  }
  s = wave_sum(s);
  if (lane_id() == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(l1_acc + lo, sred[0] + sred[1] + sred[2] + sred[3]);
}

__global__ void k_loss_scalars(const DevView* __restrict__ views, int V, int64_t n,
                               const unsigned long long* __restrict__ counts,
                               const float* __restrict__ l1_acc, float s_max, float lambda_reg,
                               float* __restrict__ loss, float* __restrict__ dL_deta) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const DevView& Vw = views[v];
  const float sv = Vw.s_v;
  const float l1 = l1_acc[v] / (3.0f * (float)Vw.width * (float)Vw.height);
  const float eta = n > 0 ? (float)counts[3 * v + 1] / (float)n : 0.f;
  const float eta_t = 1.0f / (sv * sqrtf(sv));
  const float ex = fmaxf(eta - eta_t, 0.f);
  const float w = (sv - 1.0f) * (sv - 1.0f);
  const float lreg = w * ex * ex;
  const float ws = w_s(sv, s_max);
  loss[v] = ws * (l1 + lambda_reg * lreg);
  if (dL_deta) dL_deta[v] = ws * lambda_reg * 2.0f * w * ex;
}

hipError_t launch_loss(const Layout& L, void* ws, int64_t n, const float* rgb, const float* target,
                       float s_max, float lambda_reg, float* loss, float* dL_drgb, float* dL_deta,
                       uint32_t loss_blocks, hipStream_t s) {
  char* w = (char*)ws;
  float* acc = (float*)(w + L.loss_acc);
  hipError_t e = launch_fill_u32((uint32_t*)acc, 0u, L.V, s);
  if (e != hipSuccess) return e;
  const DevView* views = (const DevView*)(w + L.vinfo);
  if (loss_blocks > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3(loss_blocks), dim3(kBlock), 0, s, views, L.V, rgb, target, s_max,
                       dL_drgb, acc);
  hipLaunchKernelGGL(k_loss_scalars, dim3((L.V + 63) / 64), dim3(64), 0, s, views, L.V, n,
                     (const unsigned long long*)(w + L.counts), (const float*)acc, s_max, lambda_reg,
                     loss, dL_deta);
  return hipGetLastError();
}

}  // namespace clod
