// Kalman-filter primitives of the gfx950 tracker (GPU library internal),
// shared by the sector tracker's kernels and the second phase.
//
// Track model of Sec. 2 (Rohr, LHCP 2017): state (y, z, sin phi,
// tan lambda, q/pT) at a pad-row plane x of a sector frame, propagated with
// Bz only.  Compiled with -ffp-contract=off and correctly rounded FP32
// division and square root: fused multiply-adds appear only where written.
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca_internal.h"

namespace tpcca {

// Track state at plane x: p = (y, z, sin phi, tan lambda, q/pT), C lower
// triangle (00,10,11,20,21,22,30,31,32,33,40,41,42,43,44).
struct KState {
  float p[5];
  float C[15];
  float x;
};

// Propagation x -> x1 with Bz only (Sec. 2).  sin(phi) is linear in x
// along a circle of curvature kB q/pT; dy = dx (s0 + s1) / (c0 + c1); the
// arc length (signed like dx) is the chord times the Maclaurin series of
// asin(u)/u to u^8, u = chord |k| / 2.  The Jacobian is the simplified one
// that drops the curvature term of the arc length.  C <- F C F^T.
__device__ __forceinline__ bool kf_propagate(const ParamsDev &P, KState &s, float x1) {
  const float dx = x1 - s.x;
  const float kk = P.kB * s.p[4];
  const float s0 = s.p[2];
  const float s1 = __builtin_fmaf(kk, dx, s0);
  if (!(fabsf(s1) <= P.max_sin)) return false;
  const float c0 = sqrtf(__builtin_fmaf(-s0, s0, 1.0f));
  const float c1 = sqrtf(__builtin_fmaf(-s1, s1, 1.0f));
  const float cc = c0 + c1;
  const float tt = (s0 + s1) / cc;
  const float dy = dx * tt;
  const float ch2 = __builtin_fmaf(dy, dy, dx * dx);
  const float ch = sqrtf(ch2);
  const float chs = dx < 0.0f ? -ch : ch;
  const float u2 = ch2 * kk * kk * 0.25f;
  float h = (float)(35.0 / 1152.0);
  h = __builtin_fmaf(u2, h, (float)(5.0 / 112.0));
  h = __builtin_fmaf(u2, h, (float)(3.0 / 40.0));
  h = __builtin_fmaf(u2, h, (float)(1.0 / 6.0));
  h = __builtin_fmaf(u2, h, 1.0f);
  const float dS = chs * h;
  const float t = s.p[3];

  const float a = dx * (2.0f + tt * (s0 / c0 + s1 / c1)) / cc;
  const float b = dx * P.kB * dx * (1.0f + tt * s1 / c1) / cc;
  const float g = ch > 0.0f ? t * (dy / chs) : 0.0f;
  const float cz = g * a;
  const float dzq = g * b;
  const float e = dS;
  const float f = P.kB * dx;

  s.p[0] = s.p[0] + dy;
  s.p[1] = s.p[1] + t * dS;
  s.p[2] = s1;
  s.x = x1;

  float *C = s.C;
  const float c00 = C[0], c10 = C[1], c11 = C[2], c20 = C[3], c21 = C[4], c22 = C[5];
  const float c30 = C[6], c31 = C[7], c32 = C[8], c33 = C[9];
  const float c40 = C[10], c41 = C[11], c42 = C[12], c43 = C[13], c44 = C[14];
  const float fc00 = c00 + a * c20 + b * c40;
  const float fc02 = c20 + a * c22 + b * c42;
  const float fc04 = c40 + a * c42 + b * c44;
  const float fc10 = c10 + cz * c20 + e * c30 + dzq * c40;
  const float fc11 = c11 + cz * c21 + e * c31 + dzq * c41;
  const float fc12 = c21 + cz * c22 + e * c32 + dzq * c42;
  const float fc13 = c31 + cz * c32 + e * c33 + dzq * c43;
  const float fc14 = c41 + cz * c42 + e * c43 + dzq * c44;
  const float fc20 = c20 + f * c40;
  const float fc21 = c21 + f * c41;
  const float fc22 = c22 + f * c42;
  const float fc23 = c32 + f * c43;
  const float fc24 = c42 + f * c44;
  C[0] = fc00 + a * fc02 + b * fc04;
  C[1] = fc10 + a * fc12 + b * fc14;
  C[2] = fc11 + cz * fc12 + e * fc13 + dzq * fc14;
  C[3] = fc20 + a * fc22 + b * fc24;
  C[4] = fc21 + cz * fc22 + e * fc23 + dzq * fc24;
  C[5] = fc22 + f * fc24;
  C[6] = c30 + a * c32 + b * c43;
  C[7] = c31 + cz * c32 + e * c33 + dzq * c43;
  C[8] = c32 + f * c43;
  C[9] = c33;
  C[10] = c40 + a * c42 + b * c44;
  C[11] = c41 + cz * c42 + e * c43 + dzq * c44;
  C[12] = c42 + f * c44;
  C[13] = c43;
  C[14] = c44;
  return true;
}

// chi2 of a 2-D measurement against the state (S = C_yz + R).
__device__ __forceinline__ bool kf_chi2(const ParamsDev &P, const KState &s, float ym, float zm,
                                        float &chi2) {
  const float r0 = ym - s.p[0];
  const float r1 = zm - s.p[1];
  const float s00 = s.C[0] + P.ery;
  const float s10 = s.C[1];
  const float s11 = s.C[2] + P.erz;
  const float det = s00 * s11 - s10 * s10;
  if (!(det > 0.0f)) return false;
  const float inv = 1.0f / det;
  const float i00 = s11 * inv, i10 = -s10 * inv, i11 = s00 * inv;
  const float v0 = i00 * r0 + i10 * r1;
  const float v1 = i10 * r0 + i11 * r1;
  chi2 = r0 * v0 + r1 * v1;
  return true;
}

// Kalman update with (ym, zm): K = C H^T S^-1, p += K r, C -= K H C.
__device__ __forceinline__ bool kf_update(const ParamsDev &P, KState &s, float ym, float zm,
                                          float &chi2) {
  const float r0 = ym - s.p[0];
  const float r1 = zm - s.p[1];
  const float s00 = s.C[0] + P.ery;
  const float s10 = s.C[1];
  const float s11 = s.C[2] + P.erz;
  const float det = s00 * s11 - s10 * s10;
  if (!(det > 0.0f)) return false;
  const float inv = 1.0f / det;
  const float i00 = s11 * inv, i10 = -s10 * inv, i11 = s00 * inv;
  const float v0 = i00 * r0 + i10 * r1;
  const float v1 = i10 * r0 + i11 * r1;
  chi2 = r0 * v0 + r1 * v1;
  // first two columns of C (old values), row k = (C_k0, C_k1)
  const float cj0[5] = {s.C[0], s.C[1], s.C[3], s.C[6], s.C[10]};
  const float cj1[5] = {s.C[1], s.C[2], s.C[4], s.C[7], s.C[11]};
  float k0[5], k1[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    k0[k] = cj0[k] * i00 + cj1[k] * i10;
    k1[k] = cj0[k] * i10 + cj1[k] * i11;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) s.p[k] = s.p[k] + k0[k] * r0 + k1[k] * r1;
  int idx = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      s.C[idx] = s.C[idx] - (k0[i] * cj0[j] + k1[i] * cj1[j]);
      ++idx;
    }
  return true;
}

}  // namespace tpcca
