// gfx950 kernels of the second phase (Rohr, LHCP 2017):
//   merge     Sec. 2: segments of neighbouring sectors that continue each
//             other pair up (mutual best chi^2) and chain into final tracks
//   refit     Sec. 2: Kalman refit of every final track through the won hits
//             of its segments, rotating between sector frames
//   vertices  Sec. 5: z of each track at the beam axis -> time estimate;
//             sorted estimates chain into vertices; tracks join the nearest
//   flags     Sec. 3: clusters of tracks below 50 MeV, of later looper legs
//             and of highly inclined segments
//   compress  Sec. 3: track-model residuals of the quantised clusters, and
//             the inverse
//
// One thread per segment (pairing, compression) or per final track (refit,
// flags); the per-unit z-binned segment index keeps the pair search to the
// facing ends within merge_dz_ends.  Every result is defined by comparisons
// of (chi^2, key) or by sorted order, so the order threads run in never
// matters.  Floating point as in the sector tracker: no contraction, fused
// multiply-adds only where written, correctly rounded / and sqrt.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "tpcca_dev.h"
#include "tpcca_internal.h"
#include "tpcca_kf.h"
#include "tpcca_phase2.h"

namespace tpcca {
namespace {

__device__ __forceinline__ int p2_side(int s) { return s < 18 ? 0 : 1; }
__device__ __forceinline__ int p2_next_sector(int s) { return p2_side(s) * 18 + ((s % 18) + 1) % 18; }

__device__ __forceinline__ int ord_i(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : (i ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float from_ord(int i) { return __int_as_float(i >= 0 ? i : (i ^ 0x7FFFFFFF)); }

// unit of global segment g (seg_begin ascending, n_units + 1 entries)
__device__ __forceinline__ int p2_unit_of(const P2Bufs &Q, int g) {
  int lo = 0, hi = Q.n_units;  // seg_begin[lo] <= g < seg_begin[hi]
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (Q.seg_begin[m] <= g) lo = m;
    else hi = m;
  }
  return lo;
}

__device__ __forceinline__ const tpcca_track_t &p2_track(const Bufs &B, const P2Bufs &Q, int g, int u) {
  return B.tracks[B.unit_res[u].track_begin + (g - Q.seg_begin[u])];
}
__device__ __forceinline__ int64_t p2_hit0(const Bufs &B, const tpcca_track_t &t, int u) {
  return B.unit_res[u].hit_begin + t.hit_offset;
}

// Rotation of a state from the frame of the sector at angle alpha' into the
// frame at alpha' - delta (cs = cos delta, sn = sin delta): the point keeps
// its place, the direction turns by delta, z, tan lambda and q/pT stay; the
// covariance moves with the Jacobian at a fixed plane (dy = c'/c dy',
// dz = t sn / c dy', d sin phi = c / c' d sin phi'), without the curvature
// term of the turn along the shift.  Fails unless the track crosses the new
// plane towards larger x with |sin phi| <= max_sin.
__device__ __forceinline__ bool p2_rotate(float max_sin, float cs, float sn, KState &st) {
  const float x0 = st.x, y0 = st.p[0], s0 = st.p[2], t = st.p[3];
  const float c0 = sqrtf(__builtin_fmaf(-s0, s0, 1.0f));
  const float s1 = s0 * cs + c0 * sn;
  const float c1 = c0 * cs - s0 * sn;
  if (!(c1 > 0.0f) || !(fabsf(s1) <= max_sin)) return false;
  const float j00 = c0 / c1;
  const float j10 = t * sn / c1;
  const float j22 = c1 / c0;
  st.x = x0 * cs - y0 * sn;
  st.p[0] = x0 * sn + y0 * cs;
  st.p[2] = s1;
  float *C = st.C;
  const float c00 = C[0], c10 = C[1], c11 = C[2], c20 = C[3], c21 = C[4], c22 = C[5];
  const float c30 = C[6], c31 = C[7], c32 = C[8];
  const float c40 = C[10], c41 = C[11], c42 = C[12];
  C[0] = j00 * j00 * c00;
  C[1] = j00 * (c10 + j10 * c00);
  C[2] = c11 + 2.0f * j10 * c10 + j10 * j10 * c00;
  C[3] = j22 * j00 * c20;
  C[4] = j22 * (c21 + j10 * c20);
  C[5] = j22 * j22 * c22;
  C[6] = j00 * c30;
  C[7] = c31 + j10 * c30;
  C[8] = j22 * c32;
  C[10] = j00 * c40;
  C[11] = c41 + j10 * c40;
  C[12] = j22 * c42;
  return true;
}

__device__ __forceinline__ int p2_ci(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// d^T (C1 + C2)^-1 d: Cholesky row by row, forward substitution, sum of
// squares in index order.
__device__ __forceinline__ bool p2_chi2_5(const float *d, const float *C1, const float *C2, float &chi2) {
  float L[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float sum = C1[p2_ci(i, j)] + C2[p2_ci(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) sum = sum - L[i][k] * L[j][k];
      if (i == j) {
        if (!(sum > 0.0f)) return false;
        L[i][i] = sqrtf(sum);
      } else {
        L[i][j] = sum / L[j][j];
      }
    }
  float w[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float sum = d[i];
#pragma unroll
    for (int k = 0; k < i; ++k) sum = sum - L[i][k] * w[k];
    w[i] = sum / L[i][i];
  }
  float c = w[0] * w[0];
#pragma unroll
  for (int i = 1; i < 5; ++i) c = c + w[i] * w[i];
  chi2 = c;
  return true;
}

__device__ __forceinline__ KState p2_inner(const tpcca_track_t &t) {
  KState s;
#pragma unroll
  for (int k = 0; k < 5; ++k) s.p[k] = t.p[k];
  s.p[1] = 0.0f;
#pragma unroll
  for (int k = 0; k < 15; ++k) s.C[k] = t.cov[k];
  s.x = t.x_ref;
  return s;
}

// z bin of the pairing grid of a unit with nz bins per row over its z range
__device__ __forceinline__ int p2_zbin(const int2 &zm, int nz, float z) {
  const float z0 = from_ord(zm.x), z1 = from_ord(zm.y);
  const float inv = (float)nz / fmaxf(z1 - z0, 1e-3f);
  float v = (z - z0) * inv;
  v = fminf(fmaxf(v, 0.0f), (float)(nz - 1));
  return (int)v;
}

// ---------------------------------------------------------- segments ---
// Segment index of every unit (one block): seg_begin = exclusive scan of the
// units' accepted track counts.
// The unit's pairing grid: R rows x nz z bins, nz from the unit's segment
// count (about two segments per row and bin), so that a segment's candidates
// are read from the few bins its row gap and z window cover.
__device__ __forceinline__ int p2_grid_nz(int n_seg, int R) { return max(1, min(1024, (2 * n_seg) / R)); }

__global__ __launch_bounds__(1024) void k_p2_seg_index(Bufs B, P2Bufs Q, int R) {
  __shared__ int64_t lds[1024 / 64 + 1];
  int64_t carry = 0, bcarry = 0;
  for (int u0 = 0; u0 < Q.n_units; u0 += 1024) {
    const int u = u0 + (int)threadIdx.x;
    const int ns = u < Q.n_units ? B.unit_res[u].n_tracks : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<int64_t>(ns, lds, &tot);
    const int nz = p2_grid_nz(ns, R);
    int64_t btot;
    const int64_t bex = block_exclusive_scan<int64_t>(u < Q.n_units ? (int64_t)R * nz : 0, lds, &btot);
    if (u < Q.n_units) {
      Q.seg_begin[u] = (int32_t)(carry + ex);
      Q.unit_nz[u] = nz;
      Q.unit_bbase[u] = bcarry + bex;
    }
    carry += tot;
    bcarry += btot;
  }
  if (threadIdx.x == 0) {
    Q.seg_begin[Q.n_units] = (int32_t)carry;
    Q.cnt->n_seg = (int32_t)carry;
    Q.cnt->seg_next = 0;
    Q.cnt->fin_next = 0;
  }
}

// ---------------------------------------------------------- compression ---
__device__ __forceinline__ int32_t p2_quant(float v, float q) {
  const float r = __builtin_rintf(v / q);
  return fabsf(r) < 1073741824.0f ? (int32_t)r : 0;
}

struct CmpFit {
  KState st;
  float zr;
  __device__ void start(const ParamsDev &P, const P2Params &q, const float *row_x, int row0, int32_t yq0,
                        int32_t zq0, float s, float t, float qpt) {
    st.x = row_x[row0];
    st.p[0] = (float)yq0 * q.qy;
    zr = (float)zq0 * q.qz;
    st.p[1] = 0.0f;
    st.p[2] = s;
    st.p[3] = t;
    st.p[4] = qpt;
#pragma unroll
    for (int k = 0; k < 15; ++k) st.C[k] = 0.0f;
    st.C[0] = P.ery;
    st.C[2] = P.erz;
    st.C[5] = q.c22;
    st.C[9] = q.c33;
    st.C[14] = q.c44;
  }
  __device__ bool predict(const ParamsDev &P, const P2Params &q, const float *row_x, int r, int32_t &py,
                          int32_t &pz) {
    const bool ok = kf_propagate(P, st, row_x[r]);
    py = p2_quant(st.p[0], q.qy);
    pz = p2_quant(st.p[1] + zr, q.qz);
    return ok;
  }
  __device__ void take(const ParamsDev &P, const P2Params &q, bool ok, int32_t yq, int32_t zq) {
    if (!ok) return;
    float c2;
    (void)kf_update(P, st, (float)yq * q.qy, (float)zq * q.qz - zr, c2);
  }
};

// Per hit position of the track hit array: the hit's y, z, pad row and
// cluster ID gathered once (one coalesced pass), so that the per-track
// kernels below read their hits contiguously instead of chasing cluster IDs.
__global__ __launch_bounds__(256) void k_p2_hits(Bufs B, P2Bufs Q, int R) {
  // the pad-row positions: the row of an assigned cluster is the one its x
  // lies on (it passed that test when it was loaded; rows lie more than
  // 2e-3 cm apart), found in LDS instead of a random read of its row byte
  __shared__ float s_rx[kMaxRows + 1];
  __shared__ int s_unit;
  for (int i = threadIdx.x; i < R; i += blockDim.x) s_rx[i] = B.row_x[i];
  const int U = Q.n_units;
  const int64_t h_lo = B.unit_res[0].hit_begin;
  const int64_t h_hi = B.unit_res[U - 1].hit_begin + B.unit_res[U - 1].n_track_hits;
  const int2 pc = order_piece((int)((h_hi - h_lo + blockDim.x - 1) / blockDim.x));
  for (int ck = pc.x; ck < pc.y; ++ck) {
    const int64_t hb = h_lo + (int64_t)ck * blockDim.x;
    const int64_t h = hb + threadIdx.x;
    // unit whose hit range holds the block's first hit (ranges ascend with
    // the unit; runs leave gaps), found once per block
    __syncthreads();
    if (threadIdx.x == 0) {
      int lo = 0, hi = U;
      while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (B.unit_res[m].hit_begin <= hb) lo = m;
        else hi = m;
      }
      s_unit = lo;
    }
    __syncthreads();
    if (h >= h_hi) continue;
    int u = s_unit;
    while (u + 1 < U && B.unit_res[u + 1].hit_begin <= h) ++u;  // the block's range crosses a unit
    const tpcca_unit_result_t &r = B.unit_res[u];
    if (h >= r.hit_begin + r.n_track_hits) continue;
    const UnitDev U_ = B.units[u];
    const int id = B.hits_out[h];
    const float4 c = U_.cl[id];
    int lo = 0, n = R;  // first row with x >= c.x - 1e-3
    while (n > 0) {
      const int half = n >> 1;
      if (s_rx[lo + half] < c.x - 1e-3f) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    const int row = (lo < R && fabsf(c.x - s_rx[lo]) <= 1e-3f) ? lo : (int)U_.row[id];
    Q.hrec[h] = make_float4(c.y, c.z, __int_as_float(row), __int_as_float(id));
  }
}

// Per segment: rows of its first and last won hit, inner and outer z, the
// outer end (the fitted inner state propagated to each won hit's row in
// ascending order) and the segment's compressed form (record and residuals);
// clears the pairing words.
__global__ __launch_bounds__(256) void k_p2_seg_prep(Bufs B, P2Bufs Q, ParamsDev P, P2Params q) {
  __shared__ float s_rx[kMaxRows + 1];  // pad-row positions (off the dependent chain)
  for (int i = threadIdx.x; i < P.n_rows; i += blockDim.x) s_rx[i] = B.row_x[i];
  __syncthreads();
  const int n = Q.cnt->n_seg;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1;
  // Persistent, one segment per lane at a time: every iteration takes one
  // hit step of each lane's segment, and a lane whose segment is done writes
  // its outputs and takes the next one from its wave's pool (64 consecutive
  // segments claimed with one atomic), so lanes do not wait for the longest
  // segment of their wave.  Each segment sees the same operation sequence.
  int g = -1, u = 0, k = 0, nh = 0, r_first = 0, r_last = 0;
  int64_t h0 = 0;
  bool ok = false;
  float zin = 0.0f;
  KState st;
  CmpFit fit;
  float4 nxt = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int pnext = 0, pend = 0;
  bool exhausted = false;
  for (;;) {
    if (g >= 0 && k >= nh) {
      // the segment is done: its outer end and pairing words
      P2Out o;
      o.x = st.x;
#pragma unroll
      for (int j = 0; j < 5; ++j) o.p[j] = st.p[j];
#pragma unroll
      for (int j = 0; j < 15; ++j) o.C[j] = st.C[j];
      o.ok = ok ? 1 : 0;
      Q.seg_out[g] = o;
      Q.seg_unit[g] = u;
      Q.seg_nh[g] = nh;
      Q.seg_hb[g] = h0;
      Q.seg_rows[g] = make_int2(r_first, r_last);
      Q.seg_zin[g] = zin;
      Q.seg_zout[g] = st.p[1] + zin;
      Q.best_a[g] = ~0ull;
      Q.best_b[g] = ~0ull;
      Q.next[g] = -1;
      Q.prev[g] = -1;
      g = -1;
    }
    const unsigned long long idle = __ballot(g < 0);
    if (idle) {
      if (pnext == pend && !exhausted) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&Q.cnt->seg_next, 64);
        base = __shfl(base, 0, 64);
        if (base >= n) {
          exhausted = true;
        } else {
          pnext = base;
          pend = min(base + 64, n);
        }
      }
      if (pnext < pend) {
        const int take = min(__popcll(idle), pend - pnext);
        const int rank = __popcll(idle & below);
        if (g < 0 && rank < take) {
          g = Q.order[pnext + rank];
          u = p2_unit_of(Q, g);
          const tpcca_track_t &t = p2_track(B, Q, g, u);
          h0 = p2_hit0(B, t, u);
          nh = t.n_hits;
          zin = t.p[1];
          st = p2_inner(t);
          const float4 *hr = Q.hrec + h0;
          const float4 c0 = hr[0];
          r_first = __float_as_int(c0.z);
          r_last = r_first;
          ok = kf_propagate(P, st, s_rx[r_first]);
          // Sec. 3 compression of the segment in the same pass over its hits
          // (the two fits are independent chains of operations)
          const int32_t yq0 = p2_quant(c0.x, q.qy), zq0 = p2_quant(c0.y, q.qz);
          int32_t *rc = Q.rec + 6 * (int64_t)g;
          rc[0] = r_first;
          rc[1] = yq0;
          rc[2] = zq0;
          rc[3] = (int32_t)__float_as_uint(t.p[2]);
          rc[4] = (int32_t)__float_as_uint(t.p[3]);
          rc[5] = (int32_t)__float_as_uint(t.p[4]);
          fit.start(P, q, s_rx, r_first, yq0, zq0, t.p[2], t.p[3], t.p[4]);
          // residuals: one aligned 16-B record per hit (row step, y, z, 0)
          reinterpret_cast<int4 *>(Q.res)[h0] = make_int4(0, 0, 0, 0);
          nxt = nh > 1 ? hr[1] : c0;
          k = 1;
        }
        pnext += take;
      }
    }
    if (!__any(g >= 0)) break;
    if (g >= 0 && k < nh) {
      const float4 c = nxt;
      if (k + 1 < nh) nxt = Q.hrec[h0 + k + 1];  // the next record's load overlaps this step
      const int r = __float_as_int(c.z);
      if (ok && !kf_propagate(P, st, s_rx[r])) ok = false;
      int32_t py, pz;
      const bool pok = fit.predict(P, q, s_rx, r, py, pz);
      const int32_t yq = p2_quant(c.x, q.qy), zq = p2_quant(c.y, q.qz);
      reinterpret_cast<int4 *>(Q.res)[h0 + k] = make_int4(r - r_last, yq - py, zq - pz, 0);
      fit.take(P, q, pok, yq, zq);
      r_last = r;
      ++k;
    }
  }
}

// z range of each unit's inner z values (one block per unit, no atomics)
__global__ __launch_bounds__(256) void k_p2_zrange(P2Bufs Q) {
  __shared__ int lmin[4], lmax[4];
  for (int u = blockIdx.x; u < Q.n_units; u += gridDim.x) {
    int mn = 0x7FFFFFFF, mx = (int)0x80000000;
    for (int g = Q.seg_begin[u] + (int)threadIdx.x; g < Q.seg_begin[u + 1]; g += blockDim.x) {
      const int o = ord_i(Q.seg_zin[g]);
      mn = min(mn, o);
      mx = max(mx, o);
    }
    for (int d = 32; d > 0; d >>= 1) {
      mn = min(mn, __shfl_xor(mn, d, 64));
      mx = max(mx, __shfl_xor(mx, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      lmin[threadIdx.x >> 6] = mn;
      lmax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      Q.zmm[u] = make_int2(min(min(lmin[0], lmin[1]), min(lmin[2], lmin[3])),
                           max(max(lmax[0], lmax[1]), max(lmax[2], lmax[3])));
    __syncthreads();
  }
}

// grid cell of segment g in its unit: (first won row, z bin)
__device__ __forceinline__ int64_t p2_cell(const P2Bufs &Q, int g, int u) {
  const int nz = Q.unit_nz[u];
  return Q.unit_bbase[u] + (int64_t)Q.seg_rows[g].x * nz + p2_zbin(Q.zmm[u], nz, Q.seg_zin[g]);
}

__global__ __launch_bounds__(256) void k_p2_bin_count(P2Bufs Q) {
  const int n = Q.cnt->n_seg;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x)
    atomicAdd(&Q.bin_cnt[p2_cell(Q, g, Q.seg_unit[g])], 1);
}

// per unit: exclusive scan of its cell counts (one block per unit, in
// passes of 1024 cells); the counts become the scatter cursors; the cell
// starts of unit u sit at bin_beg[unit_bbase[u] + u ..] (one extra entry)
__global__ __launch_bounds__(1024) void k_p2_bin_scan(P2Bufs Q, int R) {
  __shared__ int32_t lds[1024 / 64 + 1];
  for (int u = blockIdx.x; u < Q.n_units; u += gridDim.x) {
    const int nb = R * Q.unit_nz[u];
    int32_t *cnt = Q.bin_cnt + Q.unit_bbase[u];
    int32_t *beg = Q.bin_beg + Q.unit_bbase[u] + u;
    int32_t carry = 0;
    for (int i0 = 0; i0 < nb; i0 += 1024) {
      const int i = i0 + (int)threadIdx.x;
      const int32_t v = i < nb ? cnt[i] : 0;
      int32_t tot;
      const int32_t ex = block_exclusive_scan<int32_t>(v, lds, &tot) + carry;
      if (i < nb) {
        beg[i] = ex;
        cnt[i] = ex;
      }
      carry += tot;
    }
    if (threadIdx.x == 0) beg[nb] = carry;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_p2_bin_scatter(P2Bufs Q) {
  const int n = Q.cnt->n_seg;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    const int u = Q.seg_unit[g];
    const int pos = atomicAdd(&Q.bin_cnt[p2_cell(Q, g, u)], 1);
    Q.bin_seg[Q.seg_begin[u] + pos] = g;
    Q.bin_rz[Q.seg_begin[u] + pos] = make_int2(Q.seg_rows[g].x, __float_as_int(Q.seg_zin[g]));
  }
}

// key of a segment for the tie-breaks: (sector << 24) | index among its
// unit's tracks (ascending start ID, so the order is that of (sector,
// start ID))
__device__ __forceinline__ uint32_t p2_key(const P2Bufs &Q, int g, int u, int sector) {
  return ((uint32_t)sector << 24) | (uint32_t)(g - Q.seg_begin[u]);
}

// ------------------------------------------------------------- pairing ---
// Candidate pairs are enumerated per segment A with an outer end: every B of
// the two neighbouring units whose inner z lies within merge_dz_ends of A's
// outer z (the z-binned index, read as compact (row, z) records) and whose
// first won row follows A's last by 1 to merge_max_gap.  The enumeration
// runs twice, first counting each A's candidates, then (after a scan gives
// the offsets) writing the pairs, which a third kernel tests one per thread:
// the expensive test then never leaves lanes of a wave waiting for the few
// lanes whose A has a candidate.
template <typename Fn>
__device__ __forceinline__ void p2_candidates(const P2Bufs &Q, const P2Params &q, int R, int a, Fn &&fn) {
  const P2Out &oa = Q.seg_out[a];
  if (!oa.ok) return;
  const int ua = Q.seg_unit[a];
  const P2Unit UA = Q.units[ua];
  const float zA = Q.seg_zout[a];
  const int rowA = Q.seg_rows[a].y;
  for (int side = 0; side < 2; ++side) {
    const int ub = side == 0 ? UA.prev : UA.next;
    if (ub < 0) continue;
    if (Q.seg_begin[ub + 1] == Q.seg_begin[ub]) continue;
    const int2 zm = Q.zmm[ub];
    const int nz = Q.unit_nz[ub];
    const float pad = 1e-3f + 1e-6f * fabsf(zA);
    const int b0 = p2_zbin(zm, nz, zA - q.dz_ends - pad), b1 = p2_zbin(zm, nz, zA + q.dz_ends + pad);
    const int32_t *beg = Q.bin_beg + Q.unit_bbase[ub] + ub;
    const int sb = Q.seg_begin[ub];
    const int r1 = min(rowA + q.max_gap, R - 1);
    for (int r = rowA + 1; r <= r1; ++r) {
      const int i0 = sb + beg[r * nz + b0], i1 = sb + beg[r * nz + b1 + 1];
      for (int i = i0; i < i1; ++i) {
        const int2 rz = Q.bin_rz[i];
        const int gap = rz.x - rowA;
        if (gap < 1 || gap > q.max_gap) continue;
        if (!(fabsf(__int_as_float(rz.y) - zA) <= q.dz_ends)) continue;
        fn(i);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_p2_pair_count(P2Bufs Q, P2Params q, int R, int32_t *count) {
  const int n = Q.cnt->n_seg;
  const int2 pc = order_piece(n);
  for (int a = pc.x + (int)threadIdx.x; a < pc.y; a += (int)blockDim.x) {
    int c = 0;
    p2_candidates(Q, q, R, a, [&](int) { ++c; });
    count[a] = c;
  }
}

__global__ __launch_bounds__(256) void k_p2_pair_fill(P2Bufs Q, P2Params q, int R, const int64_t *begin, int2 *pairs) {
  const int n = Q.cnt->n_seg;
  const int2 pc = order_piece(n);
  for (int a = pc.x + (int)threadIdx.x; a < pc.y; a += (int)blockDim.x) {
    int64_t w = begin[a];
    p2_candidates(Q, q, R, a, [&](int i) { pairs[w++] = make_int2(a, Q.bin_seg[i]); });
  }
}

// One pair per thread: B's inner state rotated into A's frame, A's outer end
// propagated to that plane, windows and the chi^2 of the difference; A keeps
// its best B and B its best A through 64-bit atomic minima of (chi^2 bits,
// key).
__global__ __launch_bounds__(256) void k_p2_pair_eval(Bufs B, P2Bufs Q, ParamsDev P, P2Params q, const int2 *pairs,
                                                      int64_t n_pairs) {
  int64_t k0, k1;
  order_range(n_pairs, k0, k1);
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int2 pr = pairs[k];
    const int a = pr.x, b = pr.y;
    const int ua = Q.seg_unit[a], ub = Q.seg_unit[b];
    const int sa_sec = Q.units[ua].sector, sb_sec = Q.units[ub].sector;
    const float zrA = Q.seg_zin[a], zrB = Q.seg_zin[b];
    const tpcca_track_t &tb = B.tracks[B.unit_res[ub].track_begin + (b - Q.seg_begin[ub])];
    KState sb = p2_inner(tb);
    const float sn = p2_next_sector(sa_sec) == sb_sec ? q.sn : -q.sn;
    if (!p2_rotate(q.max_sin, q.cs, sn, sb)) continue;
    const P2Out &oa = Q.seg_out[a];
    KState sa;
    sa.x = oa.x;
#pragma unroll
    for (int j = 0; j < 5; ++j) sa.p[j] = oa.p[j];
#pragma unroll
    for (int j = 0; j < 15; ++j) sa.C[j] = oa.C[j];
    if (!kf_propagate(P, sa, sb.x)) continue;
    float d[5];
    d[0] = sb.p[0] - sa.p[0];
    d[1] = (zrB - zrA) - sa.p[1];
    d[2] = sb.p[2] - sa.p[2];
    d[3] = sb.p[3] - sa.p[3];
    d[4] = sb.p[4] - sa.p[4];
    if (!(fabsf(d[0]) <= q.wy) || !(fabsf(d[1]) <= q.wz)) continue;
    float c;
    if (!p2_chi2_5(d, sa.C, sb.C, c)) continue;
    if (!(c <= q.chi2)) continue;
    const unsigned long long hi = (unsigned long long)__float_as_uint(c) << 32;
    atomicMin(&Q.best_b[a], hi | p2_key(Q, b, ub, sb_sec));
    atomicMin(&Q.best_a[b], hi | p2_key(Q, a, ua, sa_sec));
  }
}

// segment of a key found among the neighbours of unit u
__device__ __forceinline__ int p2_seg_of_key(const P2Bufs &Q, int u, uint32_t key) {
  const P2Unit U = Q.units[u];
  const int sector = (int)(key >> 24);
  const int v = (U.prev >= 0 && Q.units[U.prev].sector == sector) ? U.prev : U.next;
  return Q.seg_begin[v] + (int)(key & 0xFFFFFFu);
}

// mutual best partners merge
__global__ __launch_bounds__(256) void k_p2_links(P2Bufs Q) {
  const int n = Q.cnt->n_seg;
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
    const unsigned long long kb = Q.best_b[a];
    if (kb == ~0ull) continue;
    const int ua = Q.seg_unit[a];
    const int b = p2_seg_of_key(Q, ua, (uint32_t)kb);
    const unsigned long long ka = Q.best_a[b];
    if ((uint32_t)ka == p2_key(Q, a, ua, Q.units[ua].sector)) {
      Q.next[a] = b;
      Q.prev[b] = a;
    }
  }
}

// --------------------------------------------------------------- scans ---
// Tile sums of a per-element count over [0, n) (n on the device; tiles
// beyond it sum to 0); one block per tile.
template <typename Get>
__global__ __launch_bounds__(256) void k_p2_tile_sums(Get get, const int32_t *n_ptr, int64_t *sums, int ntiles) {
  __shared__ int64_t part[256 / 64];
  const int n = *n_ptr;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int64_t v = 0;
    for (int i = t * kP2Tile + (int)threadIdx.x; i < (t + 1) * kP2Tile && i < n; i += 256) v += get(i);
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) sums[t] = part[0] + part[1] + part[2] + part[3];
    __syncthreads();
  }
}

// exclusive scan of ntiles sums in place (one block); sums[ntiles] = total,
// also stored to *total_out when given
__global__ __launch_bounds__(1024) void k_p2_scan_sums(int64_t *sums, int ntiles, int32_t *total32,
                                                      int64_t *total64) {
  __shared__ int64_t lds[1024 / 64 + 1];
  int64_t carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += 1024) {
    const int t = t0 + (int)threadIdx.x;
    const int64_t v = t < ntiles ? sums[t] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<int64_t>(v, lds, &tot);
    if (t < ntiles) sums[t] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    sums[ntiles] = carry;
    if (total32) *total32 = (int32_t)carry;
    if (total64) *total64 = carry;
  }
}

// Per tile: exclusive prefix of each element, handed to put(i, prefix, value).
template <typename Get, typename Put>
__global__ __launch_bounds__(256) void k_p2_tile_apply(Get get, Put put, const int32_t *n_ptr,
                                                       const int64_t *sums, int ntiles) {
  __shared__ int64_t lds[256 / 64 + 1];
  constexpr int per = kP2Tile / 256;
  const int n = *n_ptr;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int base = t * kP2Tile + (int)threadIdx.x * per;
    int64_t v[per];
    int64_t loc = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      v[k] = base + k < n ? get(base + k) : 0;
      loc += v[k];
    }
    int64_t ex = block_exclusive_scan<int64_t>(loc, lds, nullptr) + sums[t];
#pragma unroll
    for (int k = 0; k < per; ++k) {
      if (base + k < n) put(base + k, ex, v[k]);
      ex += v[k];
    }
  }
}

struct GetStart {
  const int32_t *prev;
  __device__ int64_t operator()(int i) const { return prev[i] < 0 ? 1 : 0; }
};
struct PutStart {
  int32_t *final_start;
  __device__ void operator()(int i, int64_t ex, int64_t v) const {
    if (v) final_start[ex] = i;
  }
};
struct GetCount {
  const int32_t *c;
  __device__ int64_t operator()(int i) const { return c[i]; }
};
struct PutOffset {
  int64_t *off;
  __device__ void operator()(int i, int64_t ex, int64_t) const { off[i] = ex; }
};
struct GetFinalHits {
  const int32_t *nh;
  __device__ int64_t operator()(int i) const { return nh[i]; }
};
struct PutFinalHits {
  int64_t *hbeg;
  __device__ void operator()(int i, int64_t ex, int64_t) const { hbeg[i] = ex; }
};

template <typename Get, typename Put>
hipError_t p2_scan(Get get, Put put, const int32_t *n_ptr, int64_t cap, int64_t *tmp, int32_t *total32,
                   int64_t *total64, hipStream_t s) {
  const int ntiles = (int)(cap / kP2Tile + 1);
  const int grid = std::min(ntiles, 4096);
  k_p2_tile_sums<<<grid, 256, 0, s>>>(get, n_ptr, tmp, ntiles);
  k_p2_scan_sums<<<1, 1024, 0, s>>>(tmp, ntiles, total32, total64);
  k_p2_tile_apply<<<grid, 256, 0, s>>>(get, put, n_ptr, tmp, ntiles);
  return hipGetLastError();
}

// ------------------------------------------------------------- finals ---
// Per final track (from its innermost segment): segments and won hits.
__global__ __launch_bounds__(256) void k_p2_final_count(Bufs B, P2Bufs Q) {
  const int n = Q.cnt->n_final;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n; f += gridDim.x * blockDim.x) {
    int nh = 0, m = 0;
    // a chain holds at most 18 segments (rows grow along it, one sector
    // boundary per link); the bound also guards the loop
    for (int g = Q.final_start[f]; g >= 0 && m < 18; g = Q.next[g], ++m) {
      const int u = Q.seg_unit[g];
      Q.seg_fpos[g] = nh;
      nh += p2_track(B, Q, g, u).n_hits;
      Q.final_of[g] = f;
    }
    Q.final_nhits[f] = nh;
  }
}

// Hit lists of the final tracks, inner segment first: sixteen lanes per
// segment copy its won hits (sector << 24 | cluster ID) to its place in its
// final's list, contiguous reads and writes.
__global__ __launch_bounds__(256) void k_p2_final_hits(Bufs B, P2Bufs Q) {
  const int n = Q.cnt->n_seg;
  const int gl = threadIdx.x & 15;
  const int ng = (gridDim.x * blockDim.x) >> 4;
  for (int g = (blockIdx.x * blockDim.x + threadIdx.x) >> 4; g < n; g += ng) {
    const int f = Q.final_of[g];
    const int64_t dst = Q.final_hbeg[f] + Q.seg_fpos[g];
    const int64_t src = Q.seg_hb[g];
    const int nh = Q.seg_nh[g];
    const int32_t sec = Q.units[Q.seg_unit[g]].sector << 24;
    for (int j = gl; j < nh; j += 16) Q.final_hits[dst + j] = sec | B.hits_out[src + j];
  }
}

// Refit of each final track and its extrapolation to the axis.  The refit
// starts from the outermost segment's outer end with the covariance times
// refit_inflate, updates with every won hit from the outside in
// (propagating hit to hit), rotates the state into the next inner segment's
// frame between segments, and keeps z relative to the outermost segment's
// inner z; then z at the plane x = 0 in dca_steps equal steps (Sec. 5).
//
// Persistent, one final track per lane at a time: every iteration takes one
// step (a hit, a rotation into the next segment's frame, or a step to the
// axis) of each lane's track, and a lane whose track is done takes the next
// one from its wave's pool (64 consecutive tracks claimed with one atomic),
// so tracks of 1 and of 18 segments do not hold each other up.  Each track
// sees the same operation sequence.
__device__ __forceinline__ void p2_final_failed(const P2Bufs &Q, int f) {
  tpcca_final_t &o = Q.finals[f];
  o.status = 2;
  o.n_hits = Q.final_nhits[f];
  o.ndf = 0;
  o.row_ref = 0;
  o.x_ref = 0.0f;
  o.chi2 = 0.0f;
#pragma unroll
  for (int k = 0; k < 5; ++k) o.p[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 15; ++k) o.cov[k] = 0.0f;
  o.z0_ok = 0;
  o.z0 = 0.0f;
  o.t0 = 0.0f;
  o.z_conv = 0.0f;
}

__global__ __launch_bounds__(256) void k_p2_refit(Bufs B, P2Bufs Q, ParamsDev P, P2Params q) {
  // the pad-row positions in LDS: a row step reads its plane without a
  // global load on the dependent chain
  __shared__ float s_rx[kMaxRows + 1];
  for (int i = threadIdx.x; i < P.n_rows; i += blockDim.x) s_rx[i] = B.row_x[i];
  __syncthreads();
  const int n = Q.cnt->n_final;
  const int N = q.dca_steps;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1;
  enum : int { kFree = 0, kHits = 1, kAxis = 2 };
  int phase = kFree;
  int f = 0, gc = 0, sec_c = 0, sector0 = 0, j = 0, nh = 0, row_ref = 0, kd = 0;
  int64_t hb = 0;
  float zr = 0.0f, chi2 = 0.0f, x0 = 0.0f;
  KState st;
  float4 nxt = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int pnext = 0, pend = 0;
  bool exhausted = false;
  for (;;) {
    // ---- transitions of lanes whose current segment, hits or axis steps
    // are done
    if (phase == kHits && j < 0) {
      const int gp = Q.prev[gc];  // the next inner segment of the chain
      if (gp < 0) {
        // every hit taken: the fit at the innermost hit
        tpcca_final_t &o = Q.finals[f];
        o.status = 0;
        o.n_hits = nh;
        o.ndf = 2 * nh - 5;
        o.row_ref = row_ref;
        o.x_ref = st.x;
        o.chi2 = chi2;
#pragma unroll
        for (int k = 0; k < 5; ++k) o.p[k] = st.p[k];
        o.p[1] = st.p[1] + zr;
#pragma unroll
        for (int k = 0; k < 15; ++k) o.cov[k] = st.C[k];
        o.z_conv = st.p[1] + zr;
        x0 = st.x;
        kd = 1;
        phase = kAxis;
      } else {
        const int sec_p = Q.units[Q.seg_unit[gp]].sector;
        const float sn = p2_next_sector(sec_p) == sec_c ? q.sn : -q.sn;
        if (!p2_rotate(q.max_sin, q.cs, sn, st)) {
          p2_final_failed(Q, f);
          phase = kFree;
        } else {
          gc = gp;
          sec_c = sec_p;
          hb = Q.seg_hb[gc];
          j = Q.seg_nh[gc] - 1;
          nxt = Q.hrec[hb + j];
        }
      }
    }
    if (phase == kAxis && kd > N) {
      tpcca_final_t &o = Q.finals[f];
      const float z0 = st.p[1] + zr;
      o.z0_ok = 1;
      o.z0 = z0;
      o.t0 = p2_side(sector0) == 0 ? -z0 / q.vdrift : z0 / q.vdrift;
      phase = kFree;
    }
    // ---- idle lanes take the next tracks of their wave's pool
    const unsigned long long idle = __ballot(phase == kFree);
    if (idle) {
      if (pnext == pend && !exhausted) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&Q.cnt->fin_next, 64);
        base = __shfl(base, 0, 64);
        if (base >= n) {
          exhausted = true;
        } else {
          pnext = base;
          pend = min(base + 64, n);
        }
      }
      if (pnext < pend) {
        const int take = min(__popcll(idle), pend - pnext);
        const int rank = __popcll(idle & below);
        if (phase == kFree && rank < take) {
          f = Q.order[pnext + rank];
          const int g0 = Q.final_start[f];
          // rows grow along a chain and each link crosses a sector boundary
          // of one side: at most 18 segments
          int last = g0, m = 1;
          for (int g = Q.next[g0]; g >= 0 && m < 18; g = Q.next[g]) {
            last = g;
            ++m;
          }
          const int u0 = Q.seg_unit[g0];
          sector0 = Q.units[u0].sector;
          tpcca_final_t &o = Q.finals[f];
          o.slot = Q.units[u0].slot;
          o.sector = sector0;
          o.n_seg = m;
          o.vertex = -1;
          o.z0_ok = 0;
          o.first_seg = (int32_t)p2_key(Q, g0, u0, sector0);
          o.hit_begin = Q.final_hbeg[f];
          o.pad_ = 0;
          const P2Out &oe = Q.seg_out[last];
          if (oe.ok == 0) {
            p2_final_failed(Q, f);
          } else {
            st.x = oe.x;
#pragma unroll
            for (int k = 0; k < 5; ++k) st.p[k] = oe.p[k];
#pragma unroll
            for (int k = 0; k < 15; ++k) st.C[k] = oe.C[k] * q.inflate;
            zr = Q.seg_zin[last];
            chi2 = 0.0f;
            nh = 0;
            row_ref = 0;
            gc = last;
            sec_c = Q.units[Q.seg_unit[last]].sector;
            hb = Q.seg_hb[gc];
            j = Q.seg_nh[gc] - 1;
            nxt = Q.hrec[hb + j];
            phase = kHits;
          }
        }
        pnext += take;
      }
    }
    if (!__any(phase != kFree)) {
      if (exhausted) break;
      continue;
    }
    // ---- one step
    if (phase == kHits && j >= 0) {
      const float4 c = nxt;
      if (j > 0) nxt = Q.hrec[hb + j - 1];  // the next record's load overlaps this step
      const int r = __float_as_int(c.z);
      float c2;
      if ((nh > 0 && !kf_propagate(P, st, s_rx[r])) || !kf_update(P, st, c.x, c.y - zr, c2)) {
        p2_final_failed(Q, f);
        phase = kFree;
      } else {
        chi2 = chi2 + c2;
        ++nh;
        row_ref = r;
        --j;
      }
    } else if (phase == kAxis) {
      const float xk = (x0 * (float)(N - kd)) / (float)N;
      if (!kf_propagate(P, st, xk)) {
        tpcca_final_t &o = Q.finals[f];
        o.z0 = 0.0f;
        o.t0 = 0.0f;
        phase = kFree;
      } else {
        ++kd;
      }
    }
  }
}

// ----------------------------------------------------------- vertices ---
struct GetCand {
  const tpcca_final_t *finals;
  P2Params q;
  __device__ int64_t operator()(int i) const {
    const tpcca_final_t &o = finals[i];
    return (o.status == 0 && o.z0_ok && o.n_hits >= q.vtx_min_hits && fabsf(o.p[4]) <= q.rej_looper) ? 1 : 0;
  }
};
struct PutCand {
  const tpcca_final_t *finals;
  unsigned long long *key;
  int32_t *val;
  __device__ void operator()(int i, int64_t ex, int64_t v) const {
    if (!v) return;
    // ascending (slot, t0): the t0 bits made order-preserving as unsigned
    const uint32_t b = __float_as_uint(finals[i].t0);
    const uint32_t ob = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    key[ex] = ((unsigned long long)(uint32_t)finals[i].slot << 32) | ob;
    val[ex] = i;
  }
};

// group starts among the sorted estimates: a new slot, or a step > gap
__global__ __launch_bounds__(256) void k_p2_group_marks(P2Bufs Q, const unsigned long long *key, const int32_t *val,
                                                       P2Params q) {
  const int n = Q.cnt->n_cand;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int slot = (int)(key[i] >> 32);
    int start = 1;
    if (i > 0 && (int)(key[i - 1] >> 32) == slot) {
      const float d = Q.finals[val[i]].t0 - Q.finals[val[i - 1]].t0;
      start = (d <= q.gap_us) ? 0 : 1;
    }
    if (i == 0 || (int)(key[i - 1] >> 32) != slot) Q.slot_first[slot] = i;
    Q.gstart[i] = start;
  }
}

struct GetFlag {
  const int32_t *flag;
  __device__ int64_t operator()(int i) const { return flag[i]; }
};
struct PutGroup {
  int32_t *group_pos;
  __device__ void operator()(int i, int64_t ex, int64_t v) const {
    if (v) group_pos[ex] = i;
  }
};

// per group: vertex if it has at least vtx_min_tracks members (flag for
// the compaction scan)
__global__ __launch_bounds__(256) void k_p2_group_size(P2Bufs Q, int32_t *is_vtx, P2Params q) {
  const int n = Q.cnt->n_group;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int e = k + 1 < n ? Q.group_pos[k + 1] : Q.cnt->n_cand;
    is_vtx[k] = (e - Q.group_pos[k]) >= q.vtx_min_tracks ? 1 : 0;
  }
}

struct PutVertex {
  P2Bufs Q;
  const unsigned long long *key;
  const int32_t *val;
  __device__ void operator()(int k, int64_t ex, int64_t v) const {
    if (!v) return;
    const int n = Q.cnt->n_group;
    const int b = Q.group_pos[k];
    const int e = k + 1 < n ? Q.group_pos[k + 1] : Q.cnt->n_cand;
    const int slot = (int)(key[b] >> 32);
    tpcca_vertex_t vt;
    vt.slot = slot;
    vt.n_tracks = e - b;
    vt.first = b - Q.slot_first[slot];
    vt.t0 = Q.finals[val[b + (e - b - 1) / 2]].t0;
    Q.vertices[ex] = vt;
  }
};

__global__ __launch_bounds__(256) void k_p2_vranges(P2Bufs Q) {
  const int n = Q.cnt->n_vtx;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int s = Q.vertices[v].slot;
    if (v == 0 || Q.vertices[v - 1].slot != s) Q.slot_vbeg[s] = v;
    if (v == n - 1 || Q.vertices[v + 1].slot != s) Q.slot_vend[s] = v + 1;
  }
}

// every track with a time estimate joins the nearest vertex of its slot
// (the earlier one on a tie) within vtx_attach_us; its z follows
__global__ __launch_bounds__(256) void k_p2_attach(P2Bufs Q, P2Params q) {
  const int n = Q.cnt->n_final;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n; f += gridDim.x * blockDim.x) {
    tpcca_final_t &o = Q.finals[f];
    if (!o.z0_ok) continue;
    const int vb = Q.slot_vbeg[o.slot], ve = Q.slot_vend[o.slot];
    if (ve <= vb) continue;
    const float t = o.t0;
    // first vertex with t0 >= t (vertex times strictly ascend in a slot)
    int lo = vb, hi = ve;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Q.vertices[mid].t0 < t) lo = mid + 1;
      else hi = mid;
    }
    int best = -1;
    float bd = 0.0f;
    for (int v = lo - 1; v <= lo; ++v) {
      if (v < vb || v >= ve) continue;
      const float d = fabsf(t - Q.vertices[v].t0);
      if (best < 0 || d < bd) {
        best = v;
        bd = d;
      }
    }
    if (!(bd <= q.attach_us)) continue;
    o.vertex = best - vb;
    const float shift = q.vdrift * Q.vertices[best].t0;
    const float zp = o.p[1];
    o.z_conv = p2_side(o.sector) == 0 ? zp + shift : zp - shift;
  }
}

// ---------------------------------------------------------------- flags ---
// Per segment, what its clusters' rejection flags need: the flags of its
// final track (q/pT of the refit, or the segment's own where the refit
// failed; the vertex) and the segment's state for the inclination test.
__global__ __launch_bounds__(256) void k_p2_seg_flags(Bufs B, P2Bufs Q, ParamsDev P, P2Params q) {
  const int n = Q.cnt->n_seg;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    const int u = Q.seg_unit[g];
    const tpcca_track_t &t = p2_track(B, Q, g, u);
    const tpcca_final_t &o = Q.finals[Q.final_of[g]];
    const float qpt = o.status == 0 ? o.p[4] : t.p[4];
    int fl = 0;
    if (fabsf(qpt) > q.rej_qpt) fl |= 1;
    if (fabsf(qpt) > q.rej_looper && o.vertex < 0) fl |= 2;
    Q.seg_flag[g] = make_float4(P.kB * t.p[4], t.x_ref, t.p[2], __int_as_float(fl));
  }
}

// Rejection flags, one thread per cluster (coalesced over the batch's
// clusters): an assigned cluster takes its segment's flags and the
// inclination of the segment's state at the cluster's row,
// fma(kB q/pT, x_row - x_ref, sin phi).
__global__ __launch_bounds__(256) void k_p2_flags(Bufs B, P2Bufs Q, P2Params q, int64_t n_cl) {
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < n_cl;
       gi += (int64_t)gridDim.x * blockDim.x) {
    const int a = B.assign[gi];
    uint8_t fl = 0;
    if (a >= 0) {
      // unit of cluster gi (cl_begin ascends with the unit)
      int lo = 0, hi = Q.n_units;
      while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (B.units[m].cl_begin <= gi) lo = m;
        else hi = m;
      }
      const UnitDev &U = B.units[lo];
      const float4 sf = Q.seg_flag[Q.seg_begin[lo] + a];
      const float dx = B.row_x[U.row[gi - U.cl_begin]] - sf.y;
      const float s = __builtin_fmaf(sf.x, dx, sf.z);
      fl = (uint8_t)(__float_as_int(sf.w) | (fabsf(s) > q.rej_sin ? 4 : 0));
    }
    Q.flags[gi] = fl;
  }
}

__global__ __launch_bounds__(256) void k_p2_decompress(ParamsDev P, P2Params q, const float *row_x, int n_seg,
                                                      int R, const int32_t *n_hits, const int64_t *hit_begin,
                                                      const int32_t *rec, const int32_t *res, int32_t *yq,
                                                      int32_t *zq, uint8_t *rows) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_seg; g += gridDim.x * blockDim.x) {
    const int32_t *rc = rec + 6 * (int64_t)g;
    const int64_t h0 = hit_begin[g];
    int r = rc[0];
    if (r < 0 || r >= R) continue;
    CmpFit fit;
    fit.start(P, q, row_x, r, rc[1], rc[2], __uint_as_float((uint32_t)rc[3]), __uint_as_float((uint32_t)rc[4]),
              __uint_as_float((uint32_t)rc[5]));
    yq[h0] = rc[1];
    zq[h0] = rc[2];
    rows[h0] = (uint8_t)r;
    for (int j = 1; j < n_hits[g]; ++j) {
      const int4 rs = reinterpret_cast<const int4 *>(res)[h0 + j];
      r += rs.x;
      if (r < 0 || r >= R) break;  // corrupt input: leave the rest untouched
      int32_t py, pz;
      const bool ok = fit.predict(P, q, row_x, r, py, pz);
      const int32_t y = rs.y + py, z = rs.z + pz;
      yq[h0 + j] = y;
      zq[h0 + j] = z;
      rows[h0 + j] = (uint8_t)r;
      fit.take(P, q, ok, y, z);
    }
  }
}

__global__ void k_p2_fill_u8(uint8_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
// ---------------------------------------------------------------- order ---
// Processing order of the persistent per-lane kernels (segment preparation
// with compression, final refit): items by descending length, a counting
// sort over kLenBins length classes.  A wave claims 64 consecutive items of
// the order, so its lanes get about equally long work and finish together
// instead of each wave waiting for the longest of 64 items in input order.
// The order changes no result: each item's outputs depend on that item
// alone.  Items of one length keep no particular order among themselves
// (ranks inside a block from LDS atomics, block bases from global ones).
constexpr int kLenBins = 512;
constexpr int kLenPer = 4;  // items per thread and pass of the scatter

struct SegLen {  // a segment: its won hits
  __device__ int count(const P2Bufs &Q) const { return Q.cnt->n_seg; }
  __device__ int len(const Bufs &B, const P2Bufs &Q, int g) const {
    return p2_track(B, Q, g, p2_unit_of(Q, g)).n_hits;
  }
};
struct FinLen {  // a final track: its hits
  __device__ int count(const P2Bufs &Q) const { return Q.cnt->n_final; }
  __device__ int len(const Bufs &, const P2Bufs &Q, int f) const { return Q.final_nhits[f]; }
};
__device__ __forceinline__ int len_bin(int len) { return kLenBins - 1 - min(max(len, 0), kLenBins - 1); }

template <class L>
__global__ __launch_bounds__(256) void k_p2_len_hist(Bufs B, P2Bufs Q, L l) {
  __shared__ int32_t h[kLenBins];
  for (int i = threadIdx.x; i < kLenBins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int n = l.count(Q);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&h[len_bin(l.len(B, Q, i))], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < kLenBins; i += blockDim.x)
    if (h[i]) atomicAdd(&Q.len_hist[i], h[i]);
}

// the classes' first positions (exclusive scan of their counts)
__global__ __launch_bounds__(kLenBins) void k_p2_len_scan(P2Bufs Q) {
  __shared__ int32_t lds[kLenBins / 64 + 1];
  int32_t tot;
  Q.len_cursor[threadIdx.x] = block_exclusive_scan<int32_t>(Q.len_hist[threadIdx.x], lds, &tot);
}

template <class L>
__global__ __launch_bounds__(256) void k_p2_len_scatter(Bufs B, P2Bufs Q, L l) {
  __shared__ int32_t h[kLenBins], base[kLenBins];
  const int n = l.count(Q);
  constexpr int span = 256 * kLenPer;
  for (int c0 = blockIdx.x * span; c0 < n; c0 += gridDim.x * span) {  // uniform per block
    for (int i = threadIdx.x; i < kLenBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int bin[kLenPer], rank[kLenPer];
#pragma unroll
    for (int k = 0; k < kLenPer; ++k) {
      const int i = c0 + k * 256 + (int)threadIdx.x;
      bin[k] = -1;
      rank[k] = 0;
      if (i < n) {
        bin[k] = len_bin(l.len(B, Q, i));
        rank[k] = atomicAdd(&h[bin[k]], 1);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLenBins; i += blockDim.x)
      if (h[i]) base[i] = atomicAdd(&Q.len_cursor[i], h[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kLenPer; ++k)
      if (bin[k] >= 0) Q.order[base[bin[k]] + rank[k]] = c0 + k * 256 + (int)threadIdx.x;
    __syncthreads();  // h and base are refilled by the next pass
  }
}

__global__ void k_p2_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline int p2_grid(int64_t n, int block, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

// Q.order = items 0..count-1 by descending length (count read on the device;
// cap bounds it)
template <class L>
void p2_len_order(const Bufs &B, const P2Bufs &Q, L l, int64_t cap, hipStream_t s) {
  k_p2_fill_i32<<<1, kLenBins, 0, s>>>(Q.len_hist, kLenBins, 0);
  k_p2_len_hist<L><<<p2_grid(cap, 256, 256), 256, 0, s>>>(B, Q, l);
  k_p2_len_scan<<<1, kLenBins, 0, s>>>(Q);
  k_p2_len_scatter<L><<<p2_grid(cap, 256 * kLenPer, 2048), 256, 0, s>>>(B, Q, l);
}

}  // namespace

// cells of the units' pairing grids: R x nz per unit, nz <= max(1, 2 n / R)
int64_t p2_grid_cells(int64_t seg_cap, int64_t n_units, int R) { return 2 * seg_cap + (int64_t)R * n_units; }

hipError_t p2_launch_merge(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q, int n_units,
                           int64_t seg_cap, int64_t hit_span, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  const int gs = p2_grid(seg_cap, 256, 8192);
  const int R = P.n_rows;
  const int64_t cells = p2_grid_cells(seg_cap, n_units, R);
  k_p2_fill_i32<<<p2_grid(cells, 256, 8192), 256, 0, s>>>(Q.bin_cnt, cells, 0);
  k_p2_seg_index<<<1, 1024, 0, s>>>(B, Q, R);
  k_p2_hits<<<p2_grid(hit_span, 256, 16384), 256, 0, s>>>(B, Q, R);
  p2_len_order(B, Q, SegLen{}, seg_cap, s);
  k_p2_seg_prep<<<p2_grid(seg_cap, 256, 2048), 256, 0, s>>>(B, Q, P, q);  // persistent
  k_p2_zrange<<<std::min(n_units, 4096), 256, 0, s>>>(Q);
  k_p2_bin_count<<<gs, 256, 0, s>>>(Q);
  k_p2_bin_scan<<<std::min(n_units, 4096), 1024, 0, s>>>(Q, R);
  k_p2_bin_scatter<<<gs, 256, 0, s>>>(Q);
  // candidate pairs: counts and their offsets (the total goes to the host)
  k_p2_pair_count<<<gs, 256, 0, s>>>(Q, q, R, Q.final_nhits);
  return p2_scan(GetCount{Q.final_nhits}, PutOffset{Q.final_hbeg}, &Q.cnt->n_seg, seg_cap, Q.scan_tmp, nullptr,
                 &Q.cnt->n_pairs, s);
}

hipError_t p2_launch_pairs(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q, int64_t seg_cap,
                           int2 *pairs, int64_t n_pairs, hipStream_t s) {
  const int gs = p2_grid(seg_cap, 256, 8192);
  // the count and offset arrays are borrowed from the final tracks' arrays,
  // which the steps below fill afresh
  if (n_pairs > 0) {
    k_p2_pair_fill<<<gs, 256, 0, s>>>(Q, q, P.n_rows, Q.final_hbeg, pairs);
    k_p2_pair_eval<<<p2_grid(n_pairs, 256, 16384), 256, 0, s>>>(B, Q, P, q, pairs, n_pairs);
  }
  k_p2_links<<<gs, 256, 0, s>>>(Q);
  // final tracks: chain starts, their hit counts, hit offsets, refit
  hipError_t e = p2_scan(GetStart{Q.prev}, PutStart{Q.final_start}, &Q.cnt->n_seg, seg_cap, Q.scan_tmp,
                         &Q.cnt->n_final, nullptr, s);
  if (e != hipSuccess) return e;
  k_p2_final_count<<<gs, 256, 0, s>>>(B, Q);
  e = p2_scan(GetFinalHits{Q.final_nhits}, PutFinalHits{Q.final_hbeg}, &Q.cnt->n_final, seg_cap, Q.scan_tmp,
              nullptr, &Q.cnt->n_final_hits, s);
  if (e != hipSuccess) return e;
  k_p2_final_hits<<<p2_grid((int64_t)seg_cap * 16, 256, 16384), 256, 0, s>>>(B, Q);
  p2_len_order(B, Q, FinLen{}, seg_cap, s);
  k_p2_refit<<<p2_grid(seg_cap, 256, 2048), 256, 0, s>>>(B, Q, P, q);  // persistent
  // vertex candidates, compacted with their sort keys
  e = p2_scan(GetCand{Q.finals, q}, PutCand{Q.finals, Q.vkey[0], Q.vval[0]}, &Q.cnt->n_final, seg_cap,
              Q.scan_tmp, &Q.cnt->n_cand, nullptr, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

size_t p2_sort_tmp_bytes(int32_t n) {
  size_t bytes = 0;
  hipcub::DoubleBuffer<unsigned long long> k(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> v(nullptr, nullptr);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k, v, std::max(n, 1));
  return bytes;
}

hipError_t p2_launch_vertices(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q,
                              int32_t n_final, int32_t n_cand, int32_t n_slots, void *sort_tmp,
                              size_t sort_tmp_bytes, hipStream_t s) {
  (void)B;
  (void)P;
  const unsigned long long *key = Q.vkey[0];
  const int32_t *val = Q.vval[0];
  if (n_cand > 0) {
    hipcub::DoubleBuffer<unsigned long long> k(Q.vkey[0], Q.vkey[1]);
    hipcub::DoubleBuffer<int32_t> v(Q.vval[0], Q.vval[1]);
    size_t bytes = sort_tmp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(sort_tmp, bytes, k, v, n_cand, 0, 64, s);
    if (e != hipSuccess) return e;
    key = k.Current();
    val = v.Current();
  }
  k_p2_fill_i32<<<p2_grid(n_slots, 256, 256), 256, 0, s>>>(Q.slot_vbeg, n_slots, 0);
  k_p2_fill_i32<<<p2_grid(n_slots, 256, 256), 256, 0, s>>>(Q.slot_vend, n_slots, 0);
  if (n_cand > 0) {
    const int gc = p2_grid(n_cand, 256, 8192);
    k_p2_group_marks<<<gc, 256, 0, s>>>(Q, key, val, q);
    hipError_t e = p2_scan(GetFlag{Q.gstart}, PutGroup{Q.group_pos}, &Q.cnt->n_cand, n_cand, Q.scan_tmp,
                           &Q.cnt->n_group, nullptr, s);
    if (e != hipSuccess) return e;
    // gstart is free again: it holds the vertex flags of the groups
    k_p2_group_size<<<gc, 256, 0, s>>>(Q, Q.gstart, q);
    e = p2_scan(GetFlag{Q.gstart}, PutVertex{Q, key, val}, &Q.cnt->n_group, n_cand, Q.scan_tmp, &Q.cnt->n_vtx,
                nullptr, s);
    if (e != hipSuccess) return e;
    k_p2_vranges<<<gc, 256, 0, s>>>(Q);
  } else {
    k_p2_fill_i32<<<1, 64, 0, s>>>(&Q.cnt->n_vtx, 1, 0);
  }
  if (n_final > 0) k_p2_attach<<<p2_grid(n_final, 256, 8192), 256, 0, s>>>(Q, q);
  return hipGetLastError();
}

hipError_t p2_launch_finish(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q,
                            int32_t n_seg, int32_t n_final, int64_t n_clusters, hipStream_t s) {
  if (n_seg > 0) k_p2_seg_flags<<<p2_grid(n_seg, 256, 8192), 256, 0, s>>>(B, Q, P, q);
  if (n_clusters > 0) k_p2_flags<<<p2_grid(n_clusters, 256, 16384), 256, 0, s>>>(B, Q, q, n_clusters);
  return hipGetLastError();
}

hipError_t p2_launch_decompress(const ParamsDev &P, const P2Params &q, const float *row_x, int32_t n_seg,
                                const int32_t *n_hits, const int64_t *hit_begin, const int32_t *rec,
                                const int32_t *res, int32_t *yq, int32_t *zq, uint8_t *rows, hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  k_p2_decompress<<<p2_grid(n_seg, 256, 8192), 256, 0, s>>>(P, q, row_x, n_seg, P.n_rows, n_hits, hit_begin, rec,
                                                           res, yq, zq, rows);
  return hipGetLastError();
}

}  // namespace tpcca
