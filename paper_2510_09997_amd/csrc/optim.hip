// Fused Adam step over every per-Gaussian parameter plane (Sec. 4.1: the 3DGS optimiser
// recipe with the decay factor sigma_d of Eq. (2) as one more parameter, with its own learning
// rate).  One launch covers the seven learning-rate groups; each element
// is read once (parameter, gradient, two moments) and written once (parameter, moments).
//
// Binary32 operation order, no fused multiply-add (compiled with -ffp-contract=off):
//   m' = b1*m + c1*g;  v' = b2*v + c2*(g*g);  p' = p - lr*((m'/bc1) / (sqrt(v'/bc2) + eps))
// with c = 1 - b in binary32 and bc = 1 - b^t supplied by the caller.
#include "clod_internal.h"

namespace clod {

// Each segment (learning-rate group) gets blocks in proportion to its size, kAdamChunk
// parameters per block, so the large SH segment is not held to a fixed share of the grid.
// Aligned segments move float4s (two per thread in flight), others single floats; the
// arithmetic of a parameter is the same either way.
__global__ __launch_bounds__(kBlock) void k_adam(AdamSegs segs, float b1, float b2, float eps, float bc1,
                                                 float bc2) {
  int j = 0;
  while (j + 1 < kAdamGroups && (int64_t)blockIdx.x >= segs.first_block[j + 1]) ++j;
  const AdamSeg sg = segs.s[j];
  const float c1 = 1.0f - b1, c2 = 1.0f - b2;
  const int64_t e0 = ((int64_t)blockIdx.x - segs.first_block[j]) * kAdamChunk;
  const int64_t e1 = e0 + kAdamChunk < sg.count ? e0 + kAdamChunk : sg.count;
  auto upd = [&](float p, float g, float m, float v, float& po, float& mo, float& vo) {
    const float m2 = b1 * m + c1 * g;
    const float v2 = b2 * v + c2 * (g * g);
    const float mh = m2 / bc1;
    const float vh = v2 / bc2;
    po = p - sg.lr * (mh / (__builtin_sqrtf(vh) + eps));
    mo = m2;
    vo = v2;
  };
  auto scalar = [&](int64_t k) { upd(sg.p[k], sg.g[k], sg.m[k], sg.v[k], sg.p[k], sg.m[k], sg.v[k]); };
  if (!sg.vec) {
    for (int64_t k = e0 + threadIdx.x; k < e1; k += kBlock) scalar(k);
    return;
  }
  // Two float4 groups per thread per round: [q, q+4) and [q + 4*kBlock, q + 4*kBlock + 4).
  for (int64_t q = e0 + 4 * (int64_t)threadIdx.x; q < e1; q += 8 * (int64_t)kBlock) {
    const int64_t q2 = q + 4 * (int64_t)kBlock;
    const bool f1 = q + 4 <= e1, f2 = q2 + 4 <= e1;
    float4 p4[2], g4[2], m4[2], v4[2];
    if (f1) {
      p4[0] = *(const float4*)(sg.p + q); g4[0] = *(const float4*)(sg.g + q);
      m4[0] = *(const float4*)(sg.m + q); v4[0] = *(const float4*)(sg.v + q);
    }
    if (f2) {
      p4[1] = *(const float4*)(sg.p + q2); g4[1] = *(const float4*)(sg.g + q2);
      m4[1] = *(const float4*)(sg.m + q2); v4[1] = *(const float4*)(sg.v + q2);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t base = h ? q2 : q;
      if (h ? f2 : f1) {
        float4 po, mo, vo;
        upd(p4[h].x, g4[h].x, m4[h].x, v4[h].x, po.x, mo.x, vo.x);
        upd(p4[h].y, g4[h].y, m4[h].y, v4[h].y, po.y, mo.y, vo.y);
        upd(p4[h].z, g4[h].z, m4[h].z, v4[h].z, po.z, mo.z, vo.z);
        upd(p4[h].w, g4[h].w, m4[h].w, v4[h].w, po.w, mo.w, vo.w);
        *(float4*)(sg.p + base) = po;
        *(float4*)(sg.m + base) = mo;
        *(float4*)(sg.v + base) = vo;
      } else {
        for (int64_t k = base; k < e1; ++k) scalar(k);   // the segment's last, partial group
      }
    }
  }
}

hipError_t launch_adam(const AdamSegs& segs_in, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  AdamSegs segs = segs_in;
  int64_t blocks = 0;
  for (int j = 0; j < kAdamGroups; ++j) {
    segs.first_block[j] = blocks;
    blocks += (segs.s[j].count + kAdamChunk - 1) / kAdamChunk;
    const AdamSeg& sg = segs.s[j];
    segs.s[j].vec = ((uintptr_t)sg.p % 16 == 0 && (uintptr_t)sg.g % 16 == 0 && (uintptr_t)sg.m % 16 == 0 &&
                     (uintptr_t)sg.v % 16 == 0) ? 1 : 0;
  }
  segs.first_block[kAdamGroups] = blocks;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kBlock), 0, s, segs, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace clod
