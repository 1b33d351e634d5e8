// Fused Adam step over every per-Gaussian parameter plane (Sec. 4.1: the 3DGS optimiser
// recipe with the decay factor sigma_d of Eq. (2) as one more parameter, with its own learning
// rate).  One launch covers the seven learning-rate groups (blockIdx.y = group); each element
// is read once (parameter, gradient, two moments) and written once (parameter, moments).
//
// Binary32 operation order, no fused multiply-add (compiled with -ffp-contract=off):
//   m' = b1*m + c1*g;  v' = b2*v + c2*(g*g);  p' = p - lr*((m'/bc1) / (sqrt(v'/bc2) + eps))
// with c = 1 - b in binary32 and bc = 1 - b^t supplied by the caller.
#include "clod_internal.h"

namespace clod {

__global__ __launch_bounds__(kBlock) void k_adam(AdamSegs segs, float b1, float b2, float eps, float bc1,
                                                 float bc2) {
  const AdamSeg sg = segs.s[blockIdx.y];
  const float c1 = 1.0f - b1, c2 = 1.0f - b2;
  constexpr int kItems = 4;
  const int64_t stride = (int64_t)gridDim.x * kBlock * kItems;
  for (int64_t base = (int64_t)blockIdx.x * kBlock * kItems + threadIdx.x; base < sg.count; base += stride) {
    float p[kItems], g[kItems], m[kItems], v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock;
      const bool ok = j < sg.count;
      p[k] = ok ? sg.p[j] : 0.f;
      g[k] = ok ? sg.g[j] : 0.f;
      m[k] = ok ? sg.m[j] : 0.f;
      v[k] = ok ? sg.v[j] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock;
      if (j < sg.count) {
        const float m2 = b1 * m[k] + c1 * g[k];
        const float v2 = b2 * v[k] + c2 * (g[k] * g[k]);
        const float mh = m2 / bc1;
        const float vh = v2 / bc2;
        sg.p[j] = p[k] - sg.lr * (mh / (__builtin_sqrtf(vh) + eps));
        sg.m[j] = m2;
        sg.v[j] = v2;
      }
    }
  }
}

hipError_t launch_adam(const AdamSegs& segs, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  int64_t mx = 0;
  for (int j = 0; j < kAdamGroups; ++j) mx = segs.s[j].count > mx ? segs.s[j].count : mx;
  if (mx == 0) return hipSuccess;
  int64_t gx = (mx + kBlock * 4 - 1) / (kBlock * 4);
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)gx, kAdamGroups), dim3(kBlock), 0, s, segs, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace clod
