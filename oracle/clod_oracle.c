/*
 * clod_oracle.c -- CPU oracle for the CLoD-GS render path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load this library.
 * The product path (the HIP library) never calls it, links it or shares code with it.
 *
 * What it computes (CLoD-GS, arXiv 2510.09997):
 *   - Sec. 3.1, Eq. (1): front-to-back alpha blending of depth-sorted projected Gaussians,
 *     with alpha'_i = alpha''_i * G2D_i(pixel centre).
 *   - Sec. 3.2: camera distance d_i = |mu_i - c|, normalised by the maximum distance over the
 *     Gaussians inside the view frustum; Eq. (2) attenuated opacity
 *     alpha''_i = alpha_i * exp(-(d'_i s_v)^2 / (2 ReLU(sigma_d,i)^2 + eps));
 *     LoD mask M_i = alpha''_i > tau * s_v; only masked-in Gaussians are rendered.  For the
 *     primitive-budget selection of the Sec. 4 comparisons (the Gaussians of highest
 *     attenuated opacity) the caller passes the mask instead (oracle.py forms it).
 *   - The 3DGS projection the paper builds on (Sec. 3.1 "projected onto the 2D image
 *     plane"; Sec. 4.1 "built on the official 3DGS implementation"): EWA splatting with a
 *     0.3 px^2 dilation, 3-sigma screen radius, 16x16 tiles.
 *
 * Precision.  The paper fixes no precision.  Every quantity that decides an integer (the
 * frustum flag, the LoD mask, the tile rectangle, the depth key, the per-pixel skip and
 * termination, hence the last-contributor index) is computed here in IEEE binary32 under a
 * written arithmetic contract: the operation order below, round-to-nearest-even, correctly
 * rounded division and square root, fused multiply-add only where fmaf() is written, and the
 * contract exponential cexp32().  The file must be compiled with -ffp-contract=off and
 * without -ffast-math.  Floating-point colour and gradients are compared against a separate
 * FP64 path (oracle/oracle.py) that replays these decisions.
 *
 * Layouts (all planes contiguous, plane-major "structure of arrays"):
 *   mean [3][n], log_scale [3][n], quat [4][n] as (w,x,y,z), opacity logit [n], decay [n],
 *   sh [(deg+1)^2][3][n].
 *   view: 28 floats = W[9] (row-major world->camera rotation), t[3], c[3] (camera centre),
 *         fx, fy, cx, cy, width, height, s_v, frame width, frame height, viewport x, viewport y,
 *         (unused x2).  A view may render a viewport (a width x height window at (x, y), both
 *         multiples of 16) of a larger frame: the frustum and the frustum maximum of Sec. 3.2
 *         are the frame's, pixel coordinates are the frame's, and the tile rectangles are the
 *         frame's clipped to the viewport.  Frame size 0 means the frame is the view.
 *   params: 8 floats = tau, eps, near_z, guard, dilation, bg[3].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------ */
/* Contract exponential.                                                                 */
/* Cody-Waite range reduction x = k ln2 + r, |r| <= ln2/2, with ln2 split into a 16-bit   */
/* head (so k*head is exact for |k| <= 256) and a binary32 tail; e^r by its Taylor        */
/* polynomial of degree 7 (coefficients 1/j! rounded to binary32) in Horner form with      */
/* fused multiply-adds; the result scaled by 2^k built from the exponent field.           */
/* Results below 2^-124 are flushed to zero (x < -86), x > 88 gives +inf.                  */
/* ------------------------------------------------------------------------------------ */
static float f_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t bits_of(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

static float g_ln2_hi, g_ln2_lo, g_log2e, g_c[8];
static int g_init = 0;
static void contract_init(void) {
    if (g_init) return;
    /* ln2 = 0.693147...; head = ln2 truncated to 16 fractional bits (ln2 < 1). */
    double ln2 = log(2.0);
    double head = floor(ln2 * 65536.0) / 65536.0;
    g_ln2_hi = (float)head;
    g_ln2_lo = (float)(ln2 - head);
    g_log2e = (float)(1.0 / ln2);
    double fact = 1.0;
    for (int j = 0; j < 8; ++j) { if (j > 0) fact *= (double)j; g_c[j] = (float)(1.0 / fact); }
    g_init = 1;
}

static float cexp32(float x) {
    if (x != x) return x;
    if (x < -86.0f) return 0.0f;
    if (x > 88.0f) return INFINITY;
    float k = rintf(x * g_log2e);
    float r = fmaf(-k, g_ln2_hi, x);
    r = fmaf(-k, g_ln2_lo, r);
    float p = g_c[7];
    for (int j = 6; j >= 0; --j) p = fmaf(p, r, g_c[j]);
    int ki = (int)k;
    return p * f_from_bits((uint32_t)(ki + 127) << 23);
}

/* ------------------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3 (Cartesian form on the unit sphere), in the   */
/* order l = 0..3, m = -l..l.  Normalisation constants from their closed forms.          */
/* ------------------------------------------------------------------------------------ */
static float g_k0, g_k1, g_k2a, g_k2b, g_k2c, g_k3a, g_k3b, g_k3c, g_k3d, g_k3e;
static void sh_init(void) {
    const double pi = 3.14159265358979323846;
    g_k0 = (float)(0.5 * sqrt(1.0 / pi));
    g_k1 = (float)sqrt(3.0 / (4.0 * pi));
    g_k2a = (float)(0.5 * sqrt(15.0 / pi));
    g_k2b = (float)(0.25 * sqrt(5.0 / pi));
    g_k2c = (float)(0.25 * sqrt(15.0 / pi));
    g_k3a = (float)(0.25 * sqrt(35.0 / (2.0 * pi)));
    g_k3b = (float)(0.5 * sqrt(105.0 / pi));
    g_k3c = (float)(0.25 * sqrt(21.0 / (2.0 * pi)));
    g_k3d = (float)(0.25 * sqrt(7.0 / pi));
    g_k3e = (float)(0.25 * sqrt(105.0 / pi));
}

/* Fills y[0..(deg+1)^2) for the unit direction (X,Y,Z). */
static void sh_basis32(int deg, float X, float Y, float Z, float *y) {
    y[0] = g_k0;
    if (deg < 1) return;
    y[1] = g_k1 * Y;
    y[2] = g_k1 * Z;
    y[3] = g_k1 * X;
    if (deg < 2) return;
    float xx = X * X, yy = Y * Y, zz = Z * Z;
    float xy = X * Y, yz = Y * Z, xz = X * Z;
    y[4] = g_k2a * xy;
    y[5] = g_k2a * yz;
    y[6] = g_k2b * ((2.0f * zz - xx) - yy);
    y[7] = g_k2a * xz;
    y[8] = g_k2c * (xx - yy);
    if (deg < 3) return;
    float t4z = (4.0f * zz - xx) - yy;
    y[9] = g_k3a * (Y * (3.0f * xx - yy));
    y[10] = g_k3b * (xy * Z);
    y[11] = g_k3c * (Y * t4z);
    y[12] = g_k3d * (Z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
    y[13] = g_k3c * (X * t4z);
    y[14] = g_k3e * (Z * (xx - yy));
    y[15] = g_k3a * (X * (xx - 3.0f * yy));
}

/* ------------------------------------------------------------------------------------ */
typedef struct {
    float W[9], t[3], c[3];
    float fx, fy, cx, cy;
    int w, h;
    float sv;
    int fw, fh, vx, vy;   /* frame size and viewport origin (pixels) */
} oview;

static void unpack_view(const float *v, oview *o) {
    memcpy(o->W, v, 9 * sizeof(float));
    memcpy(o->t, v + 9, 3 * sizeof(float));
    memcpy(o->c, v + 12, 3 * sizeof(float));
    o->fx = v[15]; o->fy = v[16]; o->cx = v[17]; o->cy = v[18];
    o->w = (int)v[19]; o->h = (int)v[20]; o->sv = v[21];
    o->fw = (int)v[22]; o->fh = (int)v[23]; o->vx = (int)v[24]; o->vy = (int)v[25];
    if (o->fw == 0 && o->fh == 0) { o->fw = o->w; o->fh = o->h; o->vx = 0; o->vy = 0; }
}

void oracle_init(void) { contract_init(); sh_init(); }

/* Elementwise contract exponential (for tests). */
void oracle_exp(const float *x, float *y, int64_t n) {
    oracle_init();
    for (int64_t i = 0; i < n; ++i) y[i] = cexp32(x[i]);
}

/* Walks every binary32 value in [lo, hi] in increasing order (in parallel chunks) and
   reports: out[0] = number of decreasing steps of cexp32, out[1] = max error in ulps against
   the double-precision exp (normal results only), out[2] = number of values visited,
   out[3] = largest relative drop (y_prev - y) / y_prev over decreasing steps. */
static int32_t ordered_of(float f) { int32_t b; memcpy(&b, &f, 4); return b < 0 ? (int32_t)0x80000000 - b : b; }
static float float_of_ordered(int32_t o) { int32_t b = o < 0 ? (int32_t)0x80000000 - o : o; float f; memcpy(&f, &b, 4); return f; }

void oracle_exp_scan(float lo, float hi, double *out) {
    oracle_init();
    int64_t olo = ordered_of(lo), ohi = ordered_of(hi);
    int64_t total = ohi - olo + 1;
    int64_t nonmono = 0;
    double maxulp = 0.0, maxdrop = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : nonmono) reduction(max : maxulp, maxdrop)
    for (int64_t ch = 0; ch < 256; ++ch) {
        int64_t a = olo + total * ch / 256, b = olo + total * (ch + 1) / 256;
        float prev = a > olo ? cexp32(float_of_ordered((int32_t)(a - 1))) : -1.0f;
        for (int64_t o = a; o < b; ++o) {
            float x = float_of_ordered((int32_t)o);
            float y = cexp32(x);
            if (prev >= 0.0f && y < prev) {
                ++nonmono;
                double dr = ((double)prev - (double)y) / (double)prev;
                if (dr > maxdrop) maxdrop = dr;
            }
            prev = y;
            double ref = exp((double)x);
            if (ref >= 1.1754943508222875e-38 * 8.0 && ref < 3.0e38) {
                float rf = (float)ref;
                double ulp = (double)nextafterf(rf, INFINITY) - (double)rf;
                double e = fabs((double)y - ref) / ulp;
                if (e > maxulp) maxulp = e;
            }
        }
    }
    out[0] = (double)nonmono;
    out[1] = maxulp;
    out[2] = (double)total;
    out[3] = maxdrop;
}

void oracle_sh_basis(const float *dirs, int64_t n, int deg, float *out) {
    oracle_init();
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) sh_basis32(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], out + K * i);
}

/* ------------------------------------------------------------------------------------ */
/* Per-view pass over all Gaussians: view transform, frustum, distance, frustum maximum, */
/* Eq. (2), mask, EWA projection, cull, tile rectangle, SH colour.                        */
/*                                                                                        */
/* Outputs (length n unless noted):                                                      */
/*   flags[i]: bit0 F (in frustum), bit1 M (LoD mask), bit2 rendered                     */
/*             (= F and M and det > 0 and a non-empty tile rectangle),                    */
/*             bits3..5 colour channel r/g/b clamped at zero (gradient blocked).          */
/*   rec[i][10]: u, v, depth z, conic A, B, C, alpha'', r, g, b    (rendered only)        */
/*   rect[i][4]: tile x0, x1, y0, y1 (half-open)                   (rendered only)        */
/*   aux[i][6]: d, alpha, cov a, b, c, radius  (d, alpha for all; rest when F and M)      */
/*   *dmax, *argmax: frustum maximum of d (1 and -1 if the frustum is empty).             */
/*   counts[3]: n_F, n_M, n_rendered.                                                     */
/* ------------------------------------------------------------------------------------ */
void oracle_view_pass(int64_t n, int deg, const float *mean, const float *lsc, const float *quat,
                      const float *opac, const float *decay, const float *sh,
                      const float *view24, const float *par8, const uint8_t *mask_in,
                      uint8_t *flags, float *rec, int32_t *rect, float *aux,
                      float *dmax_out, int64_t *argmax_out, int64_t *counts) {
    oracle_init();
    oview V;
    unpack_view(view24, &V);
    const float tau = par8[0], eps = par8[1], nearz = par8[2], guard = par8[3], dil = par8[4];
    const int K = (deg + 1) * (deg + 1);
    const int TW = (V.w + 15) / 16, TH = (V.h + 15) / 16;          /* viewport tiles */
    const int FTW = (V.fw + 15) / 16, FTH = (V.fh + 15) / 16;      /* frame tiles */
    const int TOX = V.vx / 16, TOY = V.vy / 16;                     /* viewport origin, tiles */
    const float limx = guard * ((0.5f * (float)V.fw) / V.fx);
    const float limy = guard * ((0.5f * (float)V.fh) / V.fy);

    /* Pass 1: frustum and distance; maximum over the frustum, lowest index on ties. */
    float dmax = 0.0f;
    int64_t arg = -1;
    for (int64_t i = 0; i < n; ++i) {
        float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
        float z = fmaf(V.W[6], mx, fmaf(V.W[7], my, fmaf(V.W[8], mz, V.t[2])));
        float x = fmaf(V.W[0], mx, fmaf(V.W[1], my, fmaf(V.W[2], mz, V.t[0])));
        float y = fmaf(V.W[3], mx, fmaf(V.W[4], my, fmaf(V.W[5], mz, V.t[1])));
        int F = (z > nearz) && (fabsf(x) <= limx * z) && (fabsf(y) <= limy * z);
        float ex = mx - V.c[0], ey = my - V.c[1], ez = mz - V.c[2];
        float d = sqrtf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
        if (F && (arg < 0 || d > dmax)) { dmax = d; arg = i; }
    }
    if (arg < 0) dmax = 1.0f;
    *dmax_out = dmax;
    *argmax_out = arg;

    int64_t nF = 0, nM = 0, nR = 0;
    float ybas[16];
    for (int64_t i = 0; i < n; ++i) {
        float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
        float z = fmaf(V.W[6], mx, fmaf(V.W[7], my, fmaf(V.W[8], mz, V.t[2])));
        float x = fmaf(V.W[0], mx, fmaf(V.W[1], my, fmaf(V.W[2], mz, V.t[0])));
        float y = fmaf(V.W[3], mx, fmaf(V.W[4], my, fmaf(V.W[5], mz, V.t[1])));
        int F = (z > nearz) && (fabsf(x) <= limx * z) && (fabsf(y) <= limy * z);
        float ex = mx - V.c[0], ey = my - V.c[1], ez = mz - V.c[2];
        float d = sqrtf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));

        /* Eq. (2) and the mask. */
        float dn = d / dmax;
        float sdn = dn * V.sv;
        float num = sdn * sdn;
        float rr = fmaxf(decay[i], 0.0f);
        float den = fmaf(2.0f * rr, rr, eps);
        float q = num / den;
        float alpha = 1.0f / (1.0f + cexp32(-opac[i]));
        float a2 = alpha * cexp32(-q);
        /* The mask: the threshold of Sec. 3.2, or a given selection (budgeted LoD). */
        int M = mask_in ? (mask_in[i] != 0) : (a2 > tau * V.sv);

        uint8_t fl = (uint8_t)((F ? 1 : 0) | (M ? 2 : 0));
        nF += F;
        nM += M;
        float *ax = aux + 6 * i;
        ax[0] = d; ax[1] = alpha; ax[2] = ax[3] = ax[4] = ax[5] = 0.0f;
        float *rc = rec + 10 * i;
        for (int j = 0; j < 10; ++j) rc[j] = 0.0f;
        int32_t *rt = rect + 4 * i;
        rt[0] = rt[1] = rt[2] = rt[3] = 0;

        if (F && M) {
            /* Covariance from scale and rotation. */
            float s0 = cexp32(lsc[i]), s1 = cexp32(lsc[n + i]), s2 = cexp32(lsc[2 * n + i]);
            float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
            float n2 = fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
            float w_, x_, y_, z_;
            if (n2 > 0.0f) {
                float rn = 1.0f / sqrtf(n2);
                w_ = qw * rn; x_ = qx * rn; y_ = qy * rn; z_ = qz * rn;
            } else {
                w_ = 1.0f; x_ = y_ = z_ = 0.0f;
            }
            float xx = x_ * x_, yy = y_ * y_, zz = z_ * z_;
            float xy = x_ * y_, xz = x_ * z_, yz = y_ * z_;
            float wx = w_ * x_, wy = w_ * y_, wz = w_ * z_;
            float R[9];
            R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
            R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
            R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
            float Mm[9];
            for (int j = 0; j < 3; ++j) {
                Mm[3 * j + 0] = R[3 * j + 0] * s0;
                Mm[3 * j + 1] = R[3 * j + 1] * s1;
                Mm[3 * j + 2] = R[3 * j + 2] * s2;
            }
            float S[9];
            for (int j = 0; j < 3; ++j)
                for (int k = j; k < 3; ++k) {
                    float v = fmaf(Mm[3 * j], Mm[3 * k], fmaf(Mm[3 * j + 1], Mm[3 * k + 1], Mm[3 * j + 2] * Mm[3 * k + 2]));
                    S[3 * j + k] = v;
                    S[3 * k + j] = v;
                }
            /* Perspective Jacobian at the camera-space mean, composed with the rotation. */
            float iz = 1.0f / z;
            float tx = x * iz, ty = y * iz;
            float j00 = V.fx * iz, j02 = -(V.fx * tx) * iz;
            float j11 = V.fy * iz, j12 = -(V.fy * ty) * iz;
            float T[6];
            for (int k = 0; k < 3; ++k) {
                T[k] = fmaf(j00, V.W[k], j02 * V.W[6 + k]);
                T[3 + k] = fmaf(j11, V.W[3 + k], j12 * V.W[6 + k]);
            }
            float U[6];
            for (int r = 0; r < 2; ++r)
                for (int k = 0; k < 3; ++k)
                    U[3 * r + k] = fmaf(T[3 * r], S[k], fmaf(T[3 * r + 1], S[3 + k], T[3 * r + 2] * S[6 + k]));
            float ca = fmaf(U[0], T[0], fmaf(U[1], T[1], U[2] * T[2])) + dil;
            float cb = fmaf(U[0], T[3], fmaf(U[1], T[4], U[2] * T[5]));
            float cc = fmaf(U[3], T[3], fmaf(U[4], T[4], U[5] * T[5])) + dil;
            float det = fmaf(ca, cc, -(cb * cb));
            ax[2] = ca; ax[3] = cb; ax[4] = cc;
            if (det > 0.0f) {
                float idet = 1.0f / det;
                float A = cc * idet, B = -cb * idet, C = ca * idet;
                float mid = 0.5f * (ca + cc);
                float lam = mid + sqrtf(fmaxf(0.0f, fmaf(mid, mid, -det)));
                float rad = ceilf(3.0f * sqrtf(lam));
                ax[5] = rad;
                float u = fmaf(V.fx, tx, V.cx), v = fmaf(V.fy, ty, V.cy);
                float fx0 = floorf((u - rad) * 0.0625f), fx1 = floorf((u + rad) * 0.0625f) + 1.0f;
                float fy0 = floorf((v - rad) * 0.0625f), fy1 = floorf((v + rad) * 0.0625f) + 1.0f;
                fx0 = fminf(fmaxf(fx0, 0.0f), (float)FTW); fx1 = fminf(fmaxf(fx1, 0.0f), (float)FTW);
                fy0 = fminf(fmaxf(fy0, 0.0f), (float)FTH); fy1 = fminf(fmaxf(fy1, 0.0f), (float)FTH);
                /* The frame's rectangle clipped to the viewport, in viewport tiles. */
                int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
                x0 = (x0 > TOX ? x0 : TOX) - TOX; x1 = (x1 < TOX + TW ? x1 : TOX + TW) - TOX;
                y0 = (y0 > TOY ? y0 : TOY) - TOY; y1 = (y1 < TOY + TH ? y1 : TOY + TH) - TOY;
                if (x0 < x1 && y0 < y1) {
                    /* View-dependent colour. */
                    float id = 1.0f / d;
                    sh_basis32(deg, ex * id, ey * id, ez * id, ybas);
                    float col[3];
                    for (int ch = 0; ch < 3; ++ch) {
                        float acc = sh[(0 * 3 + ch) * n + i] * ybas[0];
                        for (int k = 1; k < K; ++k) acc = fmaf(sh[(k * 3 + ch) * n + i], ybas[k], acc);
                        float cv = acc + 0.5f;
                        if (!(cv > 0.0f)) fl |= (uint8_t)(8 << ch);
                        col[ch] = fmaxf(cv, 0.0f);
                    }
                    rc[0] = u; rc[1] = v; rc[2] = z;
                    rc[3] = A; rc[4] = B; rc[5] = C; rc[6] = a2;
                    rc[7] = col[0]; rc[8] = col[1]; rc[9] = col[2];
                    rt[0] = x0; rt[1] = x1; rt[2] = y0; rt[3] = y1;
                    fl |= 4;
                    ++nR;
                }
            }
        }
        if (!(fl & 4)) rc[6] = a2; /* alpha'' is reported for every Gaussian */
        flags[i] = fl;
    }
    counts[0] = nF; counts[1] = nM; counts[2] = nR;
}

/* ------------------------------------------------------------------------------------ */
/* Per-tile lists: for every tile, the rendered Gaussians whose tile rectangle contains  */
/* it, ordered by (depth, index).  Depth comparison is on the binary32 value (z > 0).     */
/* tile_off has T+1 entries; entries (capacity cap) receives the Gaussian indices.       */
/* Returns the total number of (tile, Gaussian) pairs.                                   */
/* ------------------------------------------------------------------------------------ */
typedef struct { uint32_t depth; int32_t idx; } dkey;
static int cmp_dkey(const void *a, const void *b) {
    const dkey *x = (const dkey *)a, *y = (const dkey *)b;
    if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

int64_t oracle_tile_lists(int64_t n, const uint8_t *flags, const float *rec, const int32_t *rect,
                          int w, int h, int64_t *tile_off, int32_t *entries, int64_t cap) {
    const int TW = (w + 15) / 16, TH = (h + 15) / 16;
    const int64_t T = (int64_t)TW * TH;
    for (int64_t t = 0; t <= T; ++t) tile_off[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(flags[i] & 4)) continue;
        const int32_t *r = rect + 4 * i;
        for (int ty = r[2]; ty < r[3]; ++ty)
            for (int tx = r[0]; tx < r[1]; ++tx) tile_off[(int64_t)ty * TW + tx + 1] += 1;
    }
    for (int64_t t = 0; t < T; ++t) tile_off[t + 1] += tile_off[t];
    int64_t D = tile_off[T];
    if (!entries || cap < D) return D;
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    for (int64_t t = 0; t < T; ++t) fill[t] = tile_off[t];
    for (int64_t i = 0; i < n; ++i) {
        if (!(flags[i] & 4)) continue;
        const int32_t *r = rect + 4 * i;
        for (int ty = r[2]; ty < r[3]; ++ty)
            for (int tx = r[0]; tx < r[1]; ++tx) entries[fill[(int64_t)ty * TW + tx]++] = (int32_t)i;
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < T; ++t) {
        int64_t a = tile_off[t], b = tile_off[t + 1];
        if (b - a < 2) continue;
        dkey *tmp = (dkey *)malloc(sizeof(dkey) * (size_t)(b - a));
        for (int64_t j = a; j < b; ++j) {
            tmp[j - a].idx = entries[j];
            tmp[j - a].depth = bits_of(rec[10 * (int64_t)entries[j] + 2]);
        }
        qsort(tmp, (size_t)(b - a), sizeof(dkey), cmp_dkey);
        for (int64_t j = a; j < b; ++j) entries[j] = tmp[j - a].idx;
        free(tmp);
    }
    return D;
}

/* ------------------------------------------------------------------------------------ */
/* Blend of one pixel (Eq. (1)), shared by the image loop and the per-tile status dump.  */
/* Returns the number of list entries evaluated (including the one that terminated).      */
/* status (nullable) receives per list position: 0 skipped / not reached, 1 blended,      */
/* 2 blended with the 0.99 clamp active.                                                  */
/* ------------------------------------------------------------------------------------ */
static int64_t blend_pixel_counts(int px, int py, const float *rec, const int32_t *list, int64_t len,
                                  float *out_rgb, float *out_T, int32_t *out_last, uint8_t *status,
                                  int64_t *nexp_out, int64_t *nblend_out);
static int64_t blend_pixel(int px, int py, const float *rec, const int32_t *list, int64_t len,
                           float *out_rgb, float *out_T, int32_t *out_last, uint8_t *status) {
    int64_t a, b;
    return blend_pixel_counts(px, py, rec, list, len, out_rgb, out_T, out_last, status, &a, &b);
}

/* Also counts the pairs whose exponential is needed (power in [-5.6, 0]; below -5.6 the
   product with alpha'' <= 1 is under 1/255 whatever the exponential returns) and the pairs
   blended. */
static int64_t blend_pixel_counts(int px, int py, const float *rec, const int32_t *list, int64_t len,
                                  float *out_rgb, float *out_T, int32_t *out_last, uint8_t *status,
                                  int64_t *nexp_out, int64_t *nblend_out) {
    int64_t nexp = 0, nblend = 0;
    const float skip = (float)(1.0 / 255.0);
    const float tmin = 1e-4f;
    float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    int32_t last = 0;
    int64_t evaluated = 0;
    for (int64_t k = 0; k < len; ++k) {
        const float *g = rec + 10 * (int64_t)list[k];
        ++evaluated;
        float dx = g[0] - pcx, dy = g[1] - pcy;
        float hA = -0.5f * g[3], hC = -0.5f * g[5], nB = -g[4];
        float power = fmaf(hA * dx, dx, fmaf(hC * dy, dy, (nB * dx) * dy));
        if (power > 0.0f) continue;
        if (power >= -5.6f) ++nexp;
        float prod = g[6] * cexp32(power);
        float a = fminf(0.99f, prod);
        if (a < skip) continue;
        float Tn = T * (1.0f - a);
        if (Tn < tmin) break;
        ++nblend;
        float wgt = a * T;
        cr = fmaf(g[7], wgt, cr);
        cg = fmaf(g[8], wgt, cg);
        cb = fmaf(g[9], wgt, cb);
        T = Tn;
        last = (int32_t)(k + 1);
        if (status) status[k] = (uint8_t)(prod > 0.99f ? 2 : 1);
    }
    out_rgb[0] = cr; out_rgb[1] = cg; out_rgb[2] = cb;
    *out_T = T;
    *out_last = last;
    *nexp_out = nexp;
    *nblend_out = nblend;
    return evaluated;
}

/* Full image: rgb [3][h][w] (colour plus T * bg), T [h][w], last [h][w].
   Returns the number of (pixel, entry) pairs evaluated. */
int64_t oracle_blend(int w, int h, int vx, int vy, const float *rec, const int64_t *tile_off,
                     const int32_t *entries, const float *bg3, float *rgb, float *Tout, int32_t *last,
                     int64_t *classes) {
    const int TW = (w + 15) / 16, TH = (h + 15) / 16;
    int64_t pairs = 0, nx = 0, nb = 0;
    const int64_t HW = (int64_t)w * h;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : pairs, nx, nb)
    for (int64_t t = 0; t < (int64_t)TW * TH; ++t) {
        int tx = (int)(t % TW), ty = (int)(t / TW);
        for (int ly = 0; ly < 16; ++ly)
            for (int lx = 0; lx < 16; ++lx) {
                int px = tx * 16 + lx, py = ty * 16 + ly;
                if (px >= w || py >= h) continue;
                float c[3], T;
                int32_t l;
                int64_t ex, bl;
                /* Pixel centres in frame coordinates (viewport origin added). */
                pairs += blend_pixel_counts(vx + px, vy + py, rec, entries + tile_off[t], tile_off[t + 1] - tile_off[t],
                                            c, &T, &l, NULL, &ex, &bl);
                nx += ex;
                nb += bl;
                int64_t p = (int64_t)py * w + px;
                rgb[p] = fmaf(T, bg3[0], c[0]);
                rgb[HW + p] = fmaf(T, bg3[1], c[1]);
                rgb[2 * HW + p] = fmaf(T, bg3[2], c[2]);
                Tout[p] = T;
                last[p] = l;
            }
    }
    if (classes) { classes[0] = pairs; classes[1] = nx; classes[2] = nb; }
    return pairs;
}

/* Blend decisions of one tile for the FP64 replay: status[256][lmax] (row = ly*16+lx). */
void oracle_tile_status(int w, int h, int vx, int vy, int64_t tile, const float *rec, const int64_t *tile_off,
                        const int32_t *entries, int64_t lmax, uint8_t *status) {
    const int TW = (w + 15) / 16;
    int tx = (int)(tile % TW), ty = (int)(tile / TW);
    int64_t len = tile_off[tile + 1] - tile_off[tile];
    if (len > lmax) len = lmax;
    memset(status, 0, (size_t)(256 * lmax));
    for (int ly = 0; ly < 16; ++ly)
        for (int lx = 0; lx < 16; ++lx) {
            int px = tx * 16 + lx, py = ty * 16 + ly;
            if (px >= w || py >= h) continue;
            float c[3], T;
            int32_t l;
            blend_pixel(vx + px, vy + py, rec, entries + tile_off[tile], len, c, &T, &l,
                        status + (int64_t)(ly * 16 + lx) * lmax);
        }
}

/* One pixel, for sampled checks at full size: the caller passes that pixel's tile list. */
void oracle_blend_one(int px, int py, const float *rec, const int32_t *list, int64_t len,
                      float *rgb3, float *T, int32_t *last) {
    oracle_init();
    blend_pixel(px, py, rec, list, len, rgb3, T, last, NULL);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
