// Per-Gaussian stages: view setup, frustum maximum of the camera distance (Sec. 3.2),
// attenuated opacity of Eq. (2) with the LoD mask, EWA projection / cull / tile rectangle /
// SH colour (Sec. 3.1), and the standalone multi-view LoD counter.
//
// Reads are plane-major (structure of arrays): consecutive lanes read consecutive floats of
// a plane, so every wave load is a full 256-byte coalesced transaction.  One thread owns one
// Gaussian and loops over the views of the batch, so parameters are read once per batch.
#include "clod_internal.h"

namespace clod {

// Derives per-view constants on the device (graph-replay safe: reads only views_dev).
__global__ void k_view_setup(const clod_view* __restrict__ views, int V, clod_params prm,
                             DevView* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t tile_base = 0, pix_base = 0, loss_base = 0;
  for (int v = 0; v < V; ++v) {
    const clod_view& cv = views[v];
    DevView d;
    for (int j = 0; j < 9; ++j) d.W[j] = cv.W[j];
    for (int j = 0; j < 3; ++j) { d.t[j] = cv.t[j]; d.c[j] = cv.c[j]; }
    d.fx = cv.fx; d.fy = cv.fy; d.cx = cv.cx; d.cy = cv.cy;
    d.s_v = cv.s_v;
    d.limx = prm.guard * ((0.5f * (float)cv.width) / cv.fx);
    d.limy = prm.guard * ((0.5f * (float)cv.height) / cv.fy);
    d.tau_sv = prm.tau * cv.s_v;
    d.width = cv.width;
    d.height = cv.height;
    d.tiles_x = (cv.width + kTile - 1) / kTile;
    d.tiles_y = (cv.height + kTile - 1) / kTile;
    d.tile_base = tile_base;
    d.pix_base = pix_base;
    d.loss_block_base = loss_base;
    d.pad0 = 0;
    tile_base += (uint32_t)(d.tiles_x * d.tiles_y);
    pix_base += (uint32_t)(cv.width * cv.height);
    loss_base += (uint32_t)((3u * (uint32_t)(cv.width * cv.height) + kLossChunk - 1) / kLossChunk);
    out[v] = d;
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Frustum maximum of d per view: key = bits(d) << 32 | (2^32 - 1 - i), so the 64-bit
// maximum is the largest distance and, among equal distances, the lowest index.
__global__ __launch_bounds__(kBlock) void k_frustum_max(
    const float* __restrict__ mean, int64_t n, const DevView* __restrict__ views, int V,
    float near_z, unsigned long long* __restrict__ dmax_key) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  float mx = 0.f, my = 0.f, mz = 0.f;
  if (valid) { mx = mean[i]; my = mean[n + i]; mz = mean[2 * n + i]; }
  for (int v = 0; v < V; ++v) {
    const DevView& Vw = views[v];
    unsigned long long key = 0ull;
    if (valid) {
      float x, y, z, ex, ey, ez;
      to_camera(Vw, mx, my, mz, x, y, z);
      if (in_frustum(Vw, x, y, z, near_z)) {
        const float d = cam_distance(Vw, mx, my, mz, ex, ey, ez);
        key = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
      }
    }
    // Wave maximum, then one atomic per wave.
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long other = __shfl_xor(key, o, 64);
      key = other > key ? other : key;
    }
    if (lane_id() == 0 && key != 0ull) atomicMax(dmax_key + v, key);
  }
}

__device__ __forceinline__ void wave_count_add(unsigned long long* dst, bool pred) {
  const uint64_t b = ballot64(pred);
  if (lane_id() == 0 && b) atomicAdd(dst, (unsigned long long)__popcll(b));
}

template <bool kWriteRecords>
__global__ __launch_bounds__(kBlock) void k_project(
    clod_scene sc, const DevView* __restrict__ views, int V, clod_params prm,
    const unsigned long long* __restrict__ dmax_key, unsigned long long* __restrict__ counts,
    uint8_t* __restrict__ flags_out, float4* __restrict__ rec, uint2* __restrict__ rect_out,
    uint32_t* __restrict__ tiles_out) {
  const int64_t n = sc.n;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const int deg = sc.sh_degree;
  const int K = (deg + 1) * (deg + 1);
  float mx = 0.f, my = 0.f, mz = 0.f, op = 0.f, dc = 0.f;
  if (valid) {
    mx = sc.mean[i]; my = sc.mean[n + i]; mz = sc.mean[2 * n + i];
    op = sc.opacity[i]; dc = sc.decay[i];
  }
  // Rotation and 3D covariance are view independent: computed on first use.
  bool have_cov = false;
  float S[9];
  for (int v = 0; v < V; ++v) {
    const DevView& Vw = views[v];
    const int64_t f = (int64_t)v * n + i;
    bool F = false, M = false, R = false;
    uint8_t fl = 0;
    if (valid) {
      float x, y, z, ex, ey, ez;
      to_camera(Vw, mx, my, mz, x, y, z);
      F = in_frustum(Vw, x, y, z, prm.near_z);
      const float d = cam_distance(Vw, mx, my, mz, ex, ey, ez);
      const float dmax = dmax_from_key(dmax_key[v]);
      float alpha, q;
      const float a2 = attenuated(d, dmax, Vw.s_v, dc, op, prm.eps, alpha, q);
      M = a2 > Vw.tau_sv;
      fl = (uint8_t)((F ? 1 : 0) | (M ? 2 : 0));
      float4 g0 = make_float4(0.f, 0.f, a2, 0.f);
      if (F && M) {
        if (!have_cov) {
          const float s0 = cexp(sc.log_scale[i]), s1 = cexp(sc.log_scale[n + i]), s2 = cexp(sc.log_scale[2 * n + i]);
          float Rm[9], w_, x_, y_, z_, rn;
          quat_rot(sc.quat[i], sc.quat[n + i], sc.quat[2 * n + i], sc.quat[3 * n + i], Rm, w_, x_, y_, z_, rn);
          cov3(Rm, s0, s1, s2, S);
          have_cov = true;
        }
        Proj P;
        if (ewa(Vw, x, y, z, S, prm.dilation, P)) {
          R = true;
          if (kWriteRecords) {
            const float id = 1.0f / d;
            float Yb[16];
            sh_basis(deg, ex * id, ey * id, ez * id, Yb);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
              float acc = sc.sh[(int64_t)ch * n + i] * Yb[0];
              for (int k = 1; k < K; ++k) acc = fmaf_(sc.sh[((int64_t)k * 3 + ch) * n + i], Yb[k], acc);
              const float cv = acc + 0.5f;
              if (!(cv > 0.0f)) fl |= (uint8_t)(8 << ch);
              col[ch] = fmaxf(cv, 0.0f);
            }
            g0 = make_float4(P.u, P.v, a2, z);
            rec[(int64_t)V * n + f] = make_float4(P.A, P.B, P.C, P.rad);
            rec[2 * (int64_t)V * n + f] = make_float4(col[0], col[1], col[2], 0.f);
            rect_out[f] = make_uint2((uint32_t)P.x0 | ((uint32_t)P.x1 << 16), (uint32_t)P.y0 | ((uint32_t)P.y1 << 16));
            tiles_out[f] = (uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0));
          }
          fl |= 4;
        }
      }
      if (kWriteRecords) {
        rec[f] = g0;
        if (!R) tiles_out[f] = 0u;
        flags_out[f] = fl;
      }
    }
    wave_count_add(counts + 3 * v + 0, F);
    wave_count_add(counts + 3 * v + 1, M);
    wave_count_add(counts + 3 * v + 2, R);
  }
}

__global__ void k_counts_out(const unsigned long long* __restrict__ c, int V, int64_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 3 * V) out[j] = (int64_t)c[j];
}

static int grid_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

hipError_t launch_view_setup(const clod_view* views_dev, int V, clod_params prm, DevView* vinfo,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_view_setup, dim3(1), dim3(64), 0, s, views_dev, V, prm, vinfo);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_frustum_max(const clod_scene& sc, const DevView* vinfo, int V, float near_z,
                              unsigned long long* dmax_key, hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_frustum_max, dim3(grid_for(sc.n)), dim3(kBlock), 0, s, sc.mean, sc.n, vinfo,
                     V, near_z, dmax_key);
  return hipGetLastError();
}

hipError_t launch_project(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                          const unsigned long long* dmax_key, unsigned long long* counts,
                          uint8_t* flags, float4* rec, uint2* rect, uint32_t* tiles, hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project<true>, dim3(grid_for(sc.n)), dim3(kBlock), 0, s, sc, vinfo, V, prm,
                     dmax_key, counts, flags, rec, rect, tiles);
  return hipGetLastError();
}

hipError_t launch_lod_count(const clod_scene& sc, const DevView* vinfo, int V, clod_params prm,
                            const unsigned long long* dmax_key, unsigned long long* counts,
                            hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project<false>, dim3(grid_for(sc.n)), dim3(kBlock), 0, s, sc, vinfo, V, prm,
                     dmax_key, counts, nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_counts_out(const unsigned long long* counts, int V, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_counts_out, dim3((3 * V + 255) / 256), dim3(256), 0, s, counts, V, out);
  return hipGetLastError();
}

}  // namespace clod
