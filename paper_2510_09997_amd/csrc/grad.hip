// Per-Gaussian adjoint: screen-space partials (u, v, conic, alpha'', colour) are chained back
// to the scene parameters through the EWA projection, the SH colour, the attenuated opacity
// of Eq. (2) (opacity logit, decay factor, normalised distance and so the mean) and the
// point-count regulariser's straight-through term (d eta / d alpha''_i = 1/n, Sec. 3.3).
// The normalised distance also depends on the frustum maximum (Sec. 3.2); its partial is
// reduced per view here and applied to the argmax Gaussian by k_dmax_fix.
//
// One thread per Gaussian loops over the batch's views and writes each gradient plane once
// (coalesced, no atomics): k_gauss_bwd everything but the SH colour, k_sh_bwd the SH
// coefficients and the view-direction part of the mean's gradient.  Forward intermediates of rendered (view, Gaussian) pairs are
// recomputed with the contract arithmetic of the projection.  The Eq. (2) adjoint, which the
// point-count term needs for every (view, Gaussian), uses the hardware reciprocal, square root
// and exp2 instead (relative errors of a few 1e-7, far inside the gradients' 1e-4 tolerance),
// with the per-Gaussian and per-view factors hoisted out of the view loop.

#include "clod_internal.h"

namespace clod {
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

__global__ __launch_bounds__(kBlock) void k_gauss_bwd(
    clod_scene sc, const DevView* __restrict__ views, int V, clod_params prm,
    const unsigned long long* __restrict__ dmax_key, const uint8_t* __restrict__ flags,
    const float* __restrict__ gscreen, int64_t VN, const float* __restrict__ dL_deta,
    float* __restrict__ gpart /* [G][V] */, int accumulate, clod_scene_grad g) {
  // Dynamic LDS: [V] per-block sums of the frustum-maximum partial.  The SH coefficients'
  // gradients and the view-direction term of the mean's are left to k_sh_bwd.
  extern __shared__ float lds[];
  float* gsum = lds;
  const int64_t n = sc.n;
  const float inv_n = 1.0f / (float)n;
  for (int v = threadIdx.x; v < V; v += kBlock) gsum[v] = 0.f;
  __syncthreads();
  int64_t lo, hi;
  block_chunk(n, lo, hi);
  const int64_t iters = (hi - lo + kBlock - 1) / kBlock;
  for (int64_t it = 0; it < iters; ++it) {
  const int64_t i = lo + it * kBlock + threadIdx.x;
  const bool valid = i < hi;
  float mx = 0.f, my = 0.f, mz = 0.f, op = 0.f, dc = 0.f;
  if (valid) {
    mx = sc.mean[i]; my = sc.mean[n + i]; mz = sc.mean[2 * n + i];
    op = sc.opacity[i]; dc = sc.decay[i];
  }
  float gmx = 0.f, gmy = 0.f, gmz = 0.f, gop = 0.f, gdc = 0.f;
  float gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  // View-independent factors of Eq. (2): alpha = sigmoid(o), 1 / (2 relu(sigma)^2 + eps).
  const float alpha = frcp(1.0f + fexp(-op));
  const float r = fmaxf(dc, 0.0f);
  const float iden = frcp(2.f * r * r + prm.eps);
  bool have_cov = false;
  float s[3], Rm[9], S[9], qn[4], rn = 0.f;
  // dL/dSigma summed over the rendering views (Sigma is view independent, so the chain
  // Sigma -> M -> (scale, rotation) -> quaternion runs once, after the view loop).
  float gSig[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
  for (int v = 0; v < V; ++v) {
    const DevView& Vw = views[v];
    float gdm = 0.f;
    if (valid) {
      const int64_t f = (int64_t)v * n + i;
      const uint8_t fl = flags[f];
      float ex, ey, ez;
      const float d = __builtin_amdgcn_sqrtf(cam_distance2(Vw, mx, my, mz, ex, ey, ez));
      const float idmax = frcp(dmax_from_key(dmax_key[v]));
      const float uu = d * idmax * Vw.s_v;   // s_v-scaled normalised distance
      const float q = uu * uu * iden;
      const float a2 = alpha * fexp(-q);
      float ga2 = dL_deta ? dL_deta[v] * inv_n : 0.f;
      float gx = 0.f, gy = 0.f, gz = 0.f;     // camera-space position
      float gex = 0.f, gey = 0.f, gez = 0.f;  // world offset mu - c
      if (fl & 4) {
        const float* gs = gscreen + f * kGscreen;
        const float gu = gs[0], gv = gs[1];
        const float gA = gs[2], gB = gs[3], gC = gs[4];
        ga2 += gs[5];
        float x, y, z;
        to_camera(Vw, mx, my, mz, x, y, z);
        if (!have_cov) {
          s[0] = cexp(sc.log_scale[i]); s[1] = cexp(sc.log_scale[n + i]); s[2] = cexp(sc.log_scale[2 * n + i]);
          quat_rot(sc.quat[i], sc.quat[n + i], sc.quat[2 * n + i], sc.quat[3 * n + i], Rm, qn[0], qn[1], qn[2], qn[3], rn);
          cov3(Rm, s[0], s[1], s[2], S);
          have_cov = true;
        }
        // Mean in screen space.
        const float iz = 1.0f / z;
        gx += gu * Vw.fx * iz;
        gy += gv * Vw.fy * iz;
        gz += -(gu * Vw.fx * x + gv * Vw.fy * y) * iz * iz;
        // Conic -> 2D covariance (a, b, c include the dilation).
        Proj P;
        ewa(Vw, x, y, z, S, prm.dilation, P);
        const float a = P.ca, b = P.cb, c = P.cc;
        const float id2 = 1.0f / (P.det * P.det);
        const float ga = (-c * c * gA + b * c * gB - b * b * gC) * id2;
        const float gb = (2.f * b * c * gA - (a * c + b * b) * gB + 2.f * a * b * gC) * id2;
        const float gcc = (-b * b * gA + a * b * gB - a * a * gC) * id2;
        // Sigma' = T Sigma T^T with T = J W; symmetric gradient G' = [[ga, gb/2], [gb/2, gcc]].
        const float j00 = Vw.fx * iz, j02 = -Vw.fx * x * iz * iz;
        const float j11 = Vw.fy * iz, j12 = -Vw.fy * y * iz * iz;
        float T[6];
        for (int k = 0; k < 3; ++k) {
          T[k] = j00 * Vw.W[k] + j02 * Vw.W[6 + k];
          T[3 + k] = j11 * Vw.W[3 + k] + j12 * Vw.W[6 + k];
        }
        const float Gp00 = ga, Gp01 = 0.5f * gb, Gp11 = gcc;
        // TS = T Sigma (2x3)
        float TS[6];
        for (int r = 0; r < 2; ++r)
          for (int k = 0; k < 3; ++k)
            TS[3 * r + k] = T[3 * r] * S[k] + T[3 * r + 1] * S[3 + k] + T[3 * r + 2] * S[6 + k];
        // dL/dT = 2 G' T Sigma
        float gT[6];
        for (int k = 0; k < 3; ++k) {
          gT[k] = 2.f * (Gp00 * TS[k] + Gp01 * TS[3 + k]);
          gT[3 + k] = 2.f * (Gp01 * TS[k] + Gp11 * TS[3 + k]);
        }
        // dL/dSigma = T^T G' T (symmetric 3x3), accumulated over the views.
        {
          const float u0 = Gp00 * T[0] + Gp01 * T[3], u1 = Gp00 * T[1] + Gp01 * T[4], u2 = Gp00 * T[2] + Gp01 * T[5];
          const float w0 = Gp01 * T[0] + Gp11 * T[3], w1 = Gp01 * T[1] + Gp11 * T[4], w2 = Gp01 * T[2] + Gp11 * T[5];
          gSig[0] += T[0] * u0 + T[3] * w0;
          gSig[1] += T[0] * u1 + T[3] * w1;
          gSig[2] += T[0] * u2 + T[3] * w2;
          gSig[3] += T[1] * u1 + T[4] * w1;
          gSig[4] += T[1] * u2 + T[4] * w2;
          gSig[5] += T[2] * u2 + T[5] * w2;
        }
        // dL/dJ = dL/dT W^T; J depends on (x, y, z).
        float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
        for (int k = 0; k < 3; ++k) {
          gJ00 += gT[k] * Vw.W[k];
          gJ02 += gT[k] * Vw.W[6 + k];
          gJ11 += gT[3 + k] * Vw.W[3 + k];
          gJ12 += gT[3 + k] * Vw.W[6 + k];
        }
        const float iz2 = iz * iz, iz3 = iz2 * iz;
        gz += -Vw.fx * iz2 * gJ00 + 2.f * Vw.fx * x * iz3 * gJ02 - Vw.fy * iz2 * gJ11 + 2.f * Vw.fy * y * iz3 * gJ12;
        gx += -Vw.fx * iz2 * gJ02;
        gy += -Vw.fy * iz2 * gJ12;
      }
      // Eq. (2): alpha'' = sigmoid(o) exp(-q), q = (d' s_v)^2 / (2 relu(sigma)^2 + eps).
      gop += ga2 * a2 * (1.0f - alpha);
      const float gqv = -ga2 * a2;
      const float gnum = gqv * iden;
      const float gden = -gqv * q * iden;
      if (dc > 0.0f) gdc += gden * 4.f * r;
      const float gdn = gnum * 2.f * uu * Vw.s_v;
      const float gd = gdn * idmax;
      gdm = -gdn * d * idmax * idmax;
      const float gdd = gd * frcp(d);
      gex += gdd * ex;
      gey += gdd * ey;
      gez += gdd * ez;
      // Camera-space gradient back to the world mean (p = W mu + t).
      gmx += Vw.W[0] * gx + Vw.W[3] * gy + Vw.W[6] * gz + gex;
      gmy += Vw.W[1] * gx + Vw.W[4] * gy + Vw.W[7] * gz + gey;
      gmz += Vw.W[2] * gx + Vw.W[5] * gy + Vw.W[8] * gz + gez;
    }
    // Per-view, per-block sum of the frustum-maximum partial (LDS, one add per wave).
    gdm = wave_sum(gdm);
    if (lane_id() == 0 && gdm != 0.f) atomicAdd(&gsum[v], gdm);
  }
  if (have_cov) {
    // Sigma = M M^T, M = R diag(s): dL/dM = 2 (dL/dSigma) M.
    const float gS[9] = {gSig[0], gSig[1], gSig[2], gSig[1], gSig[3], gSig[4], gSig[2], gSig[4], gSig[5]};
    float Mm[9];
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l < 3; ++l) Mm[3 * j + l] = Rm[3 * j + l] * s[l];
    float gM[9];
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l < 3; ++l)
        gM[3 * j + l] = 2.f * (gS[3 * j] * Mm[l] + gS[3 * j + 1] * Mm[3 + l] + gS[3 * j + 2] * Mm[6 + l]);
    float gR[9];
    for (int l = 0; l < 3; ++l) {
      float gs_l = 0.f;
      for (int j = 0; j < 3; ++j) {
        gs_l += gM[3 * j + l] * Rm[3 * j + l];
        gR[3 * j + l] = gM[3 * j + l] * s[l];
      }
      gls[l] += gs_l * s[l];
    }
    // Rotation matrix of the unit quaternion (w, x, y, z).
    const float w_ = qn[0], x_ = qn[1], y_ = qn[2], z_ = qn[3];
    const float gw = 2.f * (-z_ * gR[1] + y_ * gR[2] + z_ * gR[3] - x_ * gR[5] - y_ * gR[6] + x_ * gR[7]);
    const float gxq = 2.f * (-2.f * x_ * gR[4] - 2.f * x_ * gR[8] + y_ * gR[1] + z_ * gR[2] + y_ * gR[3] - w_ * gR[5] + z_ * gR[6] + w_ * gR[7]);
    const float gyq = 2.f * (-2.f * y_ * gR[0] - 2.f * y_ * gR[8] + x_ * gR[1] + w_ * gR[2] + x_ * gR[3] + z_ * gR[5] - w_ * gR[6] + z_ * gR[7]);
    const float gzq = 2.f * (-2.f * z_ * gR[0] - 2.f * z_ * gR[4] - w_ * gR[1] + x_ * gR[2] + w_ * gR[3] + y_ * gR[5] + x_ * gR[6] + y_ * gR[7]);
    const float qdot = w_ * gw + x_ * gxq + y_ * gyq + z_ * gzq;
    gq[0] += (gw - w_ * qdot) * rn;
    gq[1] += (gxq - x_ * qdot) * rn;
    gq[2] += (gyq - y_ * qdot) * rn;
    gq[3] += (gzq - z_ * qdot) * rn;
  }
  if (valid) {
    auto put = [&](float* p, int64_t idx, float val) { p[idx] = accumulate ? p[idx] + val : val; };
    put(g.mean, i, gmx); put(g.mean, n + i, gmy); put(g.mean, 2 * n + i, gmz);
#pragma unroll
    for (int l = 0; l < 3; ++l) put(g.log_scale, l * n + i, gls[l]);
#pragma unroll
    for (int l = 0; l < 4; ++l) put(g.quat, l * n + i, gq[l]);
    put(g.opacity, i, gop);
    put(g.decay, i, gdc);
  }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < V; v += kBlock) gpart[(int64_t)blockIdx.x * V + v] = gsum[v];
}

// The SH colour's adjoint for one rendering view, in double precision: the basis values Y_k of
// the exact unit direction (dL/dc_k = dL/dcolour * Y_k) and the direction gradient
// sum_k gY_k dY_k/d(X, Y, Z).  Several basis polynomials cancel near their zero sets (for
// example X (X^2 - 3 Y^2)), where a binary32 evaluation loses relative accuracy in proportion to
// 1 / |polynomial|; evaluated in double from the double direction and then rounded once, each
// basis value and partial is within an ulp of the exact one.  The sums over k and channels stay
// in binary32 (their rounding is relative to the magnitude of their terms).  The forward
// colour keeps the binary32 contract; the adjoint is that of the exact basis.  Cartesian
// forms and closed-form normalisations as in the forward (sh_basis).
template <int DEG>
__device__ __forceinline__ void sh_adjoint_d(double X, double Y, double Z, float gc0, float gc1, float gc2,
                                             const float* c, float* acc, float& gX, float& gY, float& gZ) {
  constexpr double k0 = 0.28209479177387814, k1 = 0.4886025119029199, k2a = 1.0925484305920792,
                   k2b = 0.31539156525252005, k2c = 0.5462742152960396, k3a = 0.5900435899266435,
                   k3b = 2.890611442640554, k3c = 0.4570457994644658, k3d = 0.3731763325901154,
                   k3e = 1.445305721320277;
  gX = 0.f; gY = 0.f; gZ = 0.f;
  // One basis function: its value feeds the coefficient gradients, its partials the direction.
  auto term = [&](int k, double y, double dx, double dy, double dz) {
    const float yf = (float)y;
    acc[3 * k + 0] += gc0 * yf;
    acc[3 * k + 1] += gc1 * yf;
    acc[3 * k + 2] += gc2 * yf;
    const float gk = gc0 * c[3 * k + 0] + gc1 * c[3 * k + 1] + gc2 * c[3 * k + 2];
    gX += gk * (float)dx;
    gY += gk * (float)dy;
    gZ += gk * (float)dz;
  };
  term(0, k0, 0.0, 0.0, 0.0);
  if (DEG < 1) return;
  term(1, k1 * Y, 0.0, k1, 0.0);
  term(2, k1 * Z, 0.0, 0.0, k1);
  term(3, k1 * X, k1, 0.0, 0.0);
  if (DEG < 2) return;
  const double xx = X * X, yy = Y * Y, zz = Z * Z;
  term(4, k2a * X * Y, k2a * Y, k2a * X, 0.0);
  term(5, k2a * Y * Z, 0.0, k2a * Z, k2a * Y);
  term(6, k2b * (2.0 * zz - xx - yy), -2.0 * k2b * X, -2.0 * k2b * Y, 4.0 * k2b * Z);
  term(7, k2a * X * Z, k2a * Z, 0.0, k2a * X);
  term(8, k2c * (xx - yy), 2.0 * k2c * X, -2.0 * k2c * Y, 0.0);
  if (DEG < 3) return;
  const double t4 = 4.0 * zz - xx - yy;
  term(9, k3a * Y * (3.0 * xx - yy), 6.0 * k3a * X * Y, k3a * (3.0 * xx - 3.0 * yy), 0.0);
  term(10, k3b * X * Y * Z, k3b * Y * Z, k3b * X * Z, k3b * X * Y);
  term(11, k3c * Y * t4, -2.0 * k3c * X * Y, k3c * (4.0 * zz - xx - 3.0 * yy), 8.0 * k3c * Y * Z);
  term(12, k3d * Z * (2.0 * zz - 3.0 * xx - 3.0 * yy), -6.0 * k3d * X * Z, -6.0 * k3d * Y * Z,
       k3d * (6.0 * zz - 3.0 * xx - 3.0 * yy));
  term(13, k3c * X * t4, k3c * (4.0 * zz - 3.0 * xx - yy), -2.0 * k3c * X * Y, 8.0 * k3c * X * Z);
  term(14, k3e * Z * (xx - yy), 2.0 * k3e * X * Z, -2.0 * k3e * Y * Z, k3e * (xx - yy));
  term(15, k3a * X * (xx - 3.0 * yy), k3a * (3.0 * xx - 3.0 * yy), -6.0 * k3a * X * Y, 0.0);
}


// SH colour adjoint per Gaussian: the coefficients are loaded once and their gradients
// accumulated in registers over the rendering views (dL/dc_k = sum over views of the colour
// gradient times the basis value; clamped channels pass no gradient); the view-direction term
// dL/dmu = (dL/dd_hat - d_hat (d_hat . dL/dd_hat)) / |mu - c| is added to the mean's gradient
// written by k_gauss_bwd.  Direction, basis and its partials in double (sh_adjoint_d).
template <int DEG>
__global__ __launch_bounds__(kBlock) void k_sh_bwd(clod_scene sc, const DevView* __restrict__ views, int V,
                                                   const uint8_t* __restrict__ flags,
                                                   const float* __restrict__ gscreen, int64_t VN, int accumulate,
                                                   clod_scene_grad g) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t n = sc.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const float mx = sc.mean[i], my = sc.mean[n + i], mz = sc.mean[2 * n + i];
    float c[3 * K], acc[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
      c[k] = sc.sh[(int64_t)k * n + i];
      acc[k] = 0.f;
    }
    float gmx = 0.f, gmy = 0.f, gmz = 0.f;
    // Rendering views, 32 at a time: the flag loads of a group are independent (issued
    // together), and only the set bits are walked; most (view, Gaussian) pairs of a batch
    // are not rendered.
    for (int v0 = 0; v0 < V; v0 += 32) {
      const int vn = V - v0 < 32 ? V - v0 : 32;
      uint32_t rmask = 0;
#pragma unroll 8
      for (int j = 0; j < vn; ++j) rmask |= (uint32_t)((flags[(int64_t)(v0 + j) * n + i] >> 2) & 1u) << j;
      while (rmask) {
        const int v = v0 + __builtin_ctz(rmask);
        rmask &= rmask - 1;
        const int64_t f = (int64_t)v * n + i;
        const uint8_t fl = flags[f];
        const DevView& Vw = views[v];
        const float gc0 = (fl & 8) ? 0.f : gscreen[f * kGscreen + 6];
        const float gc1 = (fl & 16) ? 0.f : gscreen[f * kGscreen + 7];
        const float gc2 = (fl & 32) ? 0.f : gscreen[f * kGscreen + 8];
        // Exact offset and unit direction (binary32 inputs, double arithmetic).
        const double ex = (double)mx - (double)Vw.c[0], ey = (double)my - (double)Vw.c[1],
                     ez = (double)mz - (double)Vw.c[2];
        const double id = 1.0 / sqrt(ex * ex + ey * ey + ez * ez);
        const double X = ex * id, Y = ey * id, Z = ez * id;
        float gX, gYd, gZ;
        sh_adjoint_d<DEG>(X, Y, Z, gc0, gc1, gc2, c, acc, gX, gYd, gZ);
        const float Xf = (float)X, Yf = (float)Y, Zf = (float)Z, idf = (float)id;
        const float dot = Xf * gX + Yf * gYd + Zf * gZ;
        gmx += (gX - Xf * dot) * idf;
        gmy += (gYd - Yf * dot) * idf;
        gmz += (gZ - Zf * dot) * idf;
      }
    }
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
      float* p = g.sh + (int64_t)k * n + i;
      *p = accumulate ? *p + acc[k] : acc[k];
    }
    g.mean[i] += gmx;
    g.mean[n + i] += gmy;
    g.mean[2 * n + i] += gmz;
  }
}

// Frustum-maximum path: d_max = d_k for the argmax k, so dL/dmu_k += dL/ddmax (mu_k - c) / d_k.
// One block.  The per-block partials gpart[b][v] are summed with coalesced reads: thread
// (p, v) of P phases (P the largest power of two with P*V <= 256) sums rows b = p, p + P, ...,
// then a fixed tree over the phases; views above 256 are summed one thread each.  The
// contribution of every view is formed in parallel and each distinct argmax Gaussian gets the
// sum of its views' contributions in view order (deterministic).
__global__ __launch_bounds__(kBlock) void k_dmax_fix(clod_scene sc, const DevView* __restrict__ views, int V,
                           const unsigned long long* __restrict__ dmax_key,
                           const float* __restrict__ gpart, int G, float* __restrict__ gdmax,
                           clod_scene_grad g) {
  __shared__ float red[kBlock];
  __shared__ uint32_t sk[CLOD_MAX_VIEWS];
  __shared__ float sx[CLOD_MAX_VIEWS], sy[CLOD_MAX_VIEWS], sz[CLOD_MAX_VIEWS];
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const int t = threadIdx.x;
  const int64_t n = sc.n;
  for (int v0 = 0; v0 < V; v0 += kBlock) {
    const int vn = V - v0 < kBlock ? V - v0 : kBlock;
    int P = 1;
    while (2 * P * vn <= kBlock) P *= 2;
    const int p = t / vn, v = v0 + t % vn;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (p < P) {
      const float* gp = gpart + v;
      int b = p;
      for (; b + 3 * P < G; b += 4 * P) {   // four independent loads in flight
        a0 += gp[(int64_t)b * V];
        a1 += gp[(int64_t)(b + P) * V];
        a2 += gp[(int64_t)(b + 2 * P) * V];
        a3 += gp[(int64_t)(b + 3 * P) * V];
      }
      for (; b < G; b += P) a0 += gp[(int64_t)b * V];
    }
    red[t] = p < P ? (a0 + a1) + (a2 + a3) : 0.f;
    if (vn == 1) {
      // One view: a wave sum and the four wave totals instead of eight tree levels.
      const float ws = wave_sum(red[t]);
      __syncthreads();
      if (lane_id() == 0) red[t] = ws;
      __syncthreads();
      if (t == 0) red[0] = (red[0] + red[64]) + (red[128] + red[192]);
      __syncthreads();
    } else {
      __syncthreads();
      for (int h = P / 2; h > 0; h /= 2) {
        if (p < h) red[t] += red[t + h * vn];
        __syncthreads();
      }
    }
    if (t < vn) gdmax[v0 + t] = red[t];
    __syncthreads();
    if (t < vn) {
      const int vv = v0 + t;
      const unsigned long long key = dmax_key[vv];
      const int64_t kk = key == 0ull ? n : (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
      sk[vv] = kk < n ? (uint32_t)kk : kNone;
      if (kk < n) {
        float ex, ey, ez;
        const float d = cam_distance(views[vv], sc.mean[kk], sc.mean[n + kk], sc.mean[2 * n + kk], ex, ey, ez);
        const float gd = red[t] / d;
        sx[vv] = gd * ex; sy[vv] = gd * ey; sz[vv] = gd * ez;
      }
    }
    __syncthreads();
  }
  for (int v = t; v < V; v += kBlock) {
    const uint32_t k = sk[v];
    if (k == kNone) continue;
    bool first = true;
    for (int u = 0; u < v && first; ++u) first = sk[u] != k;
    if (!first) continue;
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int w = v; w < V; ++w)
      if (sk[w] == k) { ax += sx[w]; ay += sy[w]; az += sz[w]; }
    g.mean[k] += ax;
    g.mean[n + k] += ay;
    g.mean[2 * n + k] += az;
  }
}

// Zeroes the nine screen-space partials of every rendered (view, Gaussian) record, the only
// ones the blend adjoint accumulates into and the per-Gaussian adjoints read (a few percent of
// V*n in a multi-view batch, so clearing the whole accumulator would mostly write unused
// memory).  Sixteen flags per thread, one 16-byte load where all sixteen lie inside V*n.
__global__ __launch_bounds__(kBlock) void k_clear_rendered(const uint8_t* __restrict__ flags, int64_t VN,
                                                           float* __restrict__ gscreen) {
  const int64_t chunks = (VN + 15) / 16;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < chunks; c += (int64_t)gridDim.x * kBlock) {
    const int64_t f0 = c * 16;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (f0 + 16 <= VN) {
      const uint4 q = *(const uint4*)(flags + f0);
      w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
    } else {
      for (int j = 0; f0 + j < VN; ++j) w[j >> 2] |= (uint32_t)flags[f0 + j] << (8 * (j & 3));
    }
    // Bit 2 of each flag byte: rendered.
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) m |= ((w[j >> 2] >> (8 * (j & 3) + 2)) & 1u) << j;
    while (m) {
      const int j = __builtin_ctz(m);
      m &= m - 1;
      float* g = gscreen + (f0 + j) * kGscreen;
#pragma unroll
      for (int q = 0; q < kGscreen; ++q) g[q] = 0.0f;
    }
  }
}

hipError_t launch_clear_rendered(const Layout& L, void* ws, hipStream_t s) {
  if (L.VN == 0) return hipSuccess;
  char* w = (char*)ws;
  int64_t g = ((L.VN + 15) / 16 + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_clear_rendered, dim3((unsigned)g), dim3(kBlock), 0, s, (const uint8_t*)(w + L.flags), L.VN,
                     (float*)(w + L.gscreen));
  return hipGetLastError();
}

hipError_t launch_gauss_bwd(const clod_scene& sc, const Layout& L, void* ws, clod_params prm,
                            const float* dL_deta, int accumulate, const clod_scene_grad& g,
                            hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  char* w = (char*)ws;
  float* gdmax = (float*)(w + L.gdmax);
  float* gpart = (float*)(w + L.gpart);
  // One partial per block and view: the grid is capped and each block walks a chunk.
  const int grid = proj_blocks(sc.n);
  hipLaunchKernelGGL(k_gauss_bwd, dim3(grid), dim3(kBlock), (size_t)L.V * sizeof(float), s, sc,
                     (const DevView*)(w + L.vinfo), L.V, prm, (const unsigned long long*)(w + L.dmax_key),
                     (const uint8_t*)(w + L.flags), (const float*)(w + L.gscreen), L.VN, dL_deta, gpart,
                     accumulate, g);
  auto sh_kern = k_sh_bwd<3>;
  switch (sc.sh_degree) {
    case 0: sh_kern = k_sh_bwd<0>; break;
    case 1: sh_kern = k_sh_bwd<1>; break;
    case 2: sh_kern = k_sh_bwd<2>; break;
    default: break;
  }
  int64_t gs = (sc.n + kBlock - 1) / kBlock;
  if (gs > 8192) gs = 8192;
  hipLaunchKernelGGL(sh_kern, dim3((unsigned)gs), dim3(kBlock), 0, s, sc, (const DevView*)(w + L.vinfo), L.V,
                     (const uint8_t*)(w + L.flags), (const float*)(w + L.gscreen), L.VN, accumulate, g);
  hipLaunchKernelGGL(k_dmax_fix, dim3(1), dim3(kBlock), 0, s, sc, (const DevView*)(w + L.vinfo), L.V,
                     (const unsigned long long*)(w + L.dmax_key), (const float*)gpart, grid, gdmax, g);
  return hipGetLastError();
}

}  // namespace clod
