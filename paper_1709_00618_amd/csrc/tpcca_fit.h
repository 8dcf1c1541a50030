// Device helpers of the sector tracker's fit kernels (GPU library internal):
// grid lookups, the hit-slot encoding, the claim key of the selection and
// the tracklet record of a failed fit.
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca_internal.h"
#include "tpcca_kf.h"

namespace tpcca {

// Floats as ints that order like the floats (atomic min / max of floats).
__device__ __forceinline__ int ordered_int(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : (i ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float from_ordered(int i) {
  return __int_as_float(i >= 0 ? i : (i ^ 0x7FFFFFFF));
}

// z bin of a row (RowTab): clamp(floor((z - z0) * inv), 0, nb - 1).
__device__ __forceinline__ int zbin(const RowTab &t, float z) {
  float v = (z - t.z0) * t.inv;
  v = fminf(fmaxf(v, 0.0f), (float)(t.nb - 1));  // NaN -> 0
  return (int)v;
}

// sorted-index range of the bins covering [z - lim, z + lim] (a superset
// of the hits inside the window; the exact window test follows)
__device__ __forceinline__ void bin_range(const RowTab &t, const int32_t *binbeg, float z,
                                          float lim, int &b, int &e) {
  const float pad = 1e-3f + 1e-6f * fabsf(z);
  const int lo = zbin(t, z - lim - pad);
  const int hi = zbin(t, z + lim + pad);
  b = binbeg[t.bin0 + lo];
  e = binbeg[t.bin0 + hi + 1];
}

// A tracklet's hit slot holds the hit's unit-local sorted index (24 bits:
// units hold fewer than 2^24 clusters) and its pad row (top 8 bits), so the
// refit needs no row lookup.
__device__ __forceinline__ int32_t slot_enc(int g, int ucl, int row) {
  return (int32_t)(((uint32_t)row << 24) | (uint32_t)(g - ucl));
}
__device__ __forceinline__ int slot_hit(int32_t v, int ucl) { return ucl + (int)((uint32_t)v & 0xFFFFFFu); }
__device__ __forceinline__ int slot_row(int32_t v) { return (int)((uint32_t)v >> 24); }

// Phases of a tracklet's fit (Fig. 1c): chain updates and outward following
// (pass 1), inward refit and extension below the chain (pass 2).
enum : int { kIdle = 0, kChain = 1, kFollow = 2, kRefit = 3, kExtend = 4 };

// Claim key of the selection: more hits, then smaller chi2 (FP32 bits of
// a non-negative float order like its value), then smaller start ID.
__device__ __forceinline__ unsigned long long claim_key(int n_hits, float chi2, int start_id) {
  const float c = chi2 > 0.0f ? chi2 : 0.0f;
  const unsigned int bits = __float_as_uint(c);
  return ((unsigned long long)(unsigned int)n_hits << 56) |
         ((unsigned long long)(0xFFFFFFFFu - bits) << 24) |
         (unsigned long long)(0xFFFFFFu - (unsigned int)start_id);
}

__device__ __forceinline__ void kf_fail(const Bufs &B, int t, int start_id, int n_chain) {
  tpcca_tracklet_t o;
  for (int k = 0; k < 15; ++k) {
    o.cov[k] = 0.0f;
    o.cov_out[k] = 0.0f;
  }
  for (int k = 0; k < 5; ++k) {
    o.p[k] = 0.0f;
    o.p_out[k] = 0.0f;
  }
  o.start_id = start_id;
  o.n_chain = n_chain;
  o.status = 2;
  o.n_hits = 0;
  o.n_pass1 = 0;
  o.ndf = 0;
  o.row_ref = 0;
  o.row_out = 0;
  o.x_ref = 0.0f;
  o.x_out = 0.0f;
  o.chi2 = 0.0f;
  B.trk[t] = o;
}

__device__ __forceinline__ void kf_restart(const ParamsDev &P, KState &st) {
  if (P.inflate > 0.0f) {
#pragma unroll
    for (int k = 0; k < 15; ++k) st.C[k] = st.C[k] * P.inflate;
  } else {
#pragma unroll
    for (int k = 0; k < 15; ++k) st.C[k] = 0.0f;
    st.C[0] = P.r00;
    st.C[2] = P.r11;
    st.C[5] = P.c22;
    st.C[9] = P.c33;
    st.C[14] = P.c44;
  }
}

}  // namespace tpcca
