// Row-synchronous variant of the tracklet fit and track following (Rohr,
// LHCP 2017, Sec. 2, Fig. 1c) for gfx950: the lanes of a wave step through
// the pad rows together, so that the part of each row their windows cover
// is read once, coalesced, into LDS and searched there.
//
// Every tracklet sees exactly the operation sequence of the per-lane fit
// (k_kf): seed on the chain's first hit, pass 1 through the chain and
// outward, pass 2 restarted at the outermost pass-1 hit, inward through the
// pass-1 hits and below the chain.  Only where the hits are read from and
// which lane runs a tracklet change, so the results are bit-identical.
//
// Work division.  Tracklets of a unit are ordered by the z their seed line
// (first and last chain hit) reaches at the middle pad row and cut into
// chunks; a wave takes one chunk at a time.  Pass 1 sweeps the rows upward:
// at row r the idle lanes take the chunk's tracklets that start at row
// r - 1, so a lane runs several tracklets one after another in a sweep, and
// further sweeps pick up those that found no free lane.  Pass 2 sweeps
// downward the same way, a tracklet entering at the row of its outermost
// pass-1 hit.  Between the two passes a tracklet's state waits in its
// record (relative z in p_out[1] until pass 2 takes it up).
//
// Staging.  At each row the wave takes the union of the bins its lanes'
// windows cover (the search windows of following lanes; the same window
// around the prediction for lanes with a given hit), loads those bins' start
// entries and then their hits (and, while chains run, the hits' links) into
// LDS, and every lane searches or reads its given hit there.  A row whose
// union is wider than the staging area is read from global memory as in
// k_kf.
#include <hip/hip_runtime.h>

#include "tpcca_dev.h"
#include "tpcca_fit.h"
#include "tpcca_internal.h"
#include "tpcca_kernels.h"
#include "tpcca_kf.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace tpcca {

constexpr int kZoPer = 16;        // tracklets per z bucket of the order (on average)
constexpr int kStageBins = 256;   // bin-begin entries staged per wave and row
constexpr int kStageHits = 256;   // hits staged per wave and row

// ---------------------------------------------------------------- order ---
// Tracklet count of unit u of the run and its first tracklet.
__device__ __forceinline__ int unit_tracklets(const Bufs &B, const RunDev &rd, int u, int &T0) {
  T0 = B.unit_tbegin[u];
  const int T1 = u + 1 < rd.u1 ? B.unit_tbegin[u + 1] : rd.trk0 + rd.n_trk;
  return T1 - T0;
}

// Counting sort of each unit's tracklets by the z of their seed line at the
// middle row: bucket counts (the rank inside a bucket comes from the atomic).
// Unit u's n / kZoPer + 1 buckets start at T0 / kZoPer + 2 u (T0 its first
// tracklet): disjoint for all units and runs, with a spare entry after each
// unit, and no scan over units needed.
__global__ void k_zo_count(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  const float xm = B.row_x[R / 2];
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(B.zo_cnt);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rd.n_trk; i += gridDim.x * blockDim.x) {
    const int t = rd.trk0 + i;
    const int u = B.trk_unit[t];
    int T0;
    const int n = unit_tracklets(B, rd, u, T0);
    const int nb = n / kZoPer + 1;
    const int64_t base = (int64_t)(T0 / kZoPer) + 2 * (int64_t)u;
    const int g0 = B.trk_start[t];
    const int2 ci = B.cinfo[g0];
    const int r0 = B.srow[g0];
    const float2 h0 = B.yz[g0], hL = B.yz[ci.x];
    const float x0 = B.row_x[r0], xL = B.row_x[r0 + ci.y - 1];
    const float zm = h0.y + (hL.y - h0.y) / (xL - x0) * (xm - x0);
    const float zlo = from_ordered(B.zmm[2 * u]), zhi = from_ordered(B.zmm[2 * u + 1]);
    float f = (zm - zlo) / fmaxf(zhi - zlo, 1e-3f) * (float)nb;
    f = fminf(fmaxf(f, 0.0f), (float)(nb - 1));  // NaN -> 0
    const int64_t key = base + (int)f;
    const unsigned long long rank = atomicAdd(cnt + key, 1ull);
    B.zo_tmp[t] = make_int2((int)key, (int)rank);
  }
}

// Positions from the bucket counts, scanned over the run's keys: the fit
// order, unit by unit.
__global__ void k_zo_apply(Bufs B, int run) {
  RunDev &rd = B.runs[run];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rd.n_trk; i += gridDim.x * blockDim.x) {
    const int2 kr = B.zo_tmp[rd.trk0 + i];
    const int64_t pos = B.zo_cnt[kr.x] + kr.y;
    if (pos < 0 || pos >= rd.n_trk) {  // never write outside the run's slots
      atomicOr(&rd.err, 2);
      continue;
    }
    B.kf_order[rd.trk0 + pos] = rd.trk0 + i;
  }
}

// Chunks of the order: unit u gets n / gc + 1 chunks of equal size (at most
// gc tracklets) from chunk slot T0 / gc + u; the slots in between hold empty
// chunks (cleared before).
__global__ void k_chunk_table(Bufs B, int run, int gc) {
  const RunDev &rd = B.runs[run];
  for (int u = rd.u0 + blockIdx.x * blockDim.x + threadIdx.x; u < rd.u1; u += gridDim.x * blockDim.x) {
    int T0;
    const int n = unit_tracklets(B, rd, u, T0);
    const int nck = n / gc + 1;
    const int sz = (n + nck - 1) / nck;
    const int64_t cb = (int64_t)(T0 / gc) + u;
    for (int j = 0; j < nck; ++j) {
      const int beg = j * sz;
      B.kf_chunks[cb + j] = make_int4(u, T0 - rd.trk0 + beg, max(0, min(sz, n - beg)), 0);
    }
  }
}

// ----------------------------------------------------------------- wave ---
__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
// Lanes of one wave exchange data through LDS and global memory: complete
// this wave's accesses before any lane reads what another wrote.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// The same for data exchanged through LDS only (waits for LDS accesses,
// not for the wave's global loads and stores in flight).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


// ------------------------------------------------------------------ fit ---
template <int kMinWaves>
__global__ __launch_bounds__(kKfBlock, kMinWaves) void k_kf_rows(Bufs B, ParamsDev P, int run, int64_t c0, int n_chunks) {
  RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
  const unsigned long long below = (1ull << lane) - 1;
  __shared__ float s_rx[kMaxRows + 1];
  for (int i = threadIdx.x; i < R; i += blockDim.x) s_rx[i] = B.row_x[i];
  __syncthreads();
  constexpr int NW = kKfBlock / 64;
  __shared__ float2 s_yz[NW][kStageHits];
  __shared__ int32_t s_up[NW][kStageHits];
  __shared__ int32_t s_bin[NW][kStageBins];
  __shared__ uint16_t s_off[NW][kMaxRows + 2]; // list of the pass: first entry of each entry row
  __shared__ int32_t s_cur[NW][kMaxRows + 2];  // next entry of each entry row
  float2 *const yzs = s_yz[wv];
  int32_t *const ups = s_up[wv];
  int32_t *const bins = s_bin[wv];
  uint16_t *const off = s_off[wv];
  int32_t *const cur = s_cur[wv];
  // hit slots go to memory eight at a time (one aligned 32-B group), as in k_kf
  constexpr int G = kSlotGrp, GM = kSlotGrp - 1;
  __shared__ int32_t s_slot[G][kKfBlock];
  const int Rs = slot_stride(R);
  int t = 0;
  auto slot_flush = [&](int j) {
    int4 *dst = reinterpret_cast<int4 *>(B.trk_hits + (int64_t)t * Rs + (j & ~GM));
    dst[0] = make_int4(s_slot[0][tid], s_slot[1][tid], s_slot[2][tid], s_slot[3][tid]);
    dst[1] = make_int4(s_slot[4][tid], s_slot[5][tid], s_slot[6][tid], s_slot[7][tid]);
  };
  auto slot_put = [&](int j, int32_t v) {
    s_slot[j & GM][tid] = v;
    if ((j & GM) == GM) slot_flush(j);
  };
  auto slot_load = [&](int j) {  // the group holding slot j
    const int4 *src = reinterpret_cast<const int4 *>(B.trk_hits + (int64_t)t * Rs + (j & ~GM));
    const int4 q0 = src[0], q1 = src[1];
    s_slot[0][tid] = q0.x;
    s_slot[1][tid] = q0.y;
    s_slot[2][tid] = q0.z;
    s_slot[3][tid] = q0.w;
    s_slot[4][tid] = q1.x;
    s_slot[5][tid] = q1.y;
    s_slot[6][tid] = q1.z;
    s_slot[7][tid] = q1.w;
  };

  int phase = kIdle;
  int start_id = 0, n_chain = 0, r0 = 0, k = 0, miss = 0, n1 = 0, ne = 0, rlast = 0;
  int gnext = 0;   // the chain's next hit (pass 1)
  float zr = 0.0f; // z of the chain's first hit: the origin of the state's z
  float chi2 = 0.0f;
  KState st;
  // the state at the last hit taken (pass 1: outermost, pass 2: innermost),
  // in LDS to leave registers for occupancy
  __shared__ float s_aux[21][kKfBlock];
  auto save_aux = [&]() {
#pragma unroll
    for (int q = 0; q < 5; ++q) s_aux[q][tid] = st.p[q];
#pragma unroll
    for (int q = 0; q < 15; ++q) s_aux[5 + q][tid] = st.C[q];
    s_aux[20][tid] = st.x;
  };
  unsigned int cands = 0;
  unsigned int steps = 0, tests = 0, updates = 0, iters = 0;
  const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();

  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(&rd.kf_next[0], 1);
    c = __shfl(c, 0, 64);
    if (c >= n_chunks) {
      if (lane == 0) atomicMin(&rd.kf_t_drain, (unsigned long long)__builtin_amdgcn_s_memrealtime());
      break;
    }
    const int4 chk = B.kf_chunks[c0 + c];
    const int n = chk.z;
    if (n <= 0) continue;
    const int u = chk.x;
    const int ucl = B.units[u].cl_begin;
    const int lbase = rd.trk0 + chk.y;  // the chunk's positions in kf_order and kf_tmp
    const RowTab *const rtab = B.rowtab + (int64_t)u * (R + 1);

    for (int pass = 1; pass <= 2; ++pass) {
      // ---- the pass's list: the chunk's tracklets grouped by entry row
      // (pass 1: start row; pass 2: row of the outermost pass-1 hit, for the
      // tracklets whose pass 1 ended normally), written to kf_tmp
      for (int r = lane; r <= R + 1; r += 64) cur[r] = 0;
      wave_lds_sync();
      for (int i = lane; i < n; i += 64) {
        const int tt = B.kf_order[lbase + i];
        int key;
        if (pass == 1) {
          key = B.srow[B.trk_start[tt]];
        } else {
          const tpcca_tracklet_t &o = B.trk[tt];
          key = o.status == 3 ? o.row_out : -1;
        }
        if (key >= 0 && key < R) atomicAdd(&cur[key], 1);
      }
      wave_lds_sync();
      {
        int v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 4 * lane + q;
          v[q] = r < R ? cur[r] : 0;
          s += v[q];
        }
        int incl = s;
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        int ex = incl - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 4 * lane + q;
          if (r <= R) {
            off[r] = (uint16_t)ex;
            cur[r] = ex;
          }
          ex += v[q];
        }
      }
      wave_lds_sync();
      for (int i = lane; i < n; i += 64) {
        const int tt = B.kf_order[lbase + i];
        if (pass == 1) {
          // the seed record in list order (32 B, in the selection's won-mask
          // words, unused until the selection): tracklet, slot of the first
          // hit (holding the start row), chain length << 24 | start ID, the
          // chain's second hit; the seed's y, z, sin phi, tan lambda (the
          // per-lane fit's operations)
          const int g0 = B.trk_start[tt];
          const int2 ci = B.cinfo[g0];
          const int key = B.srow[g0];
          const int sid0 = B.sid[g0];
          const int nx = B.upc[g0];
          const float2 h0 = B.yz[g0], hL = B.yz[ci.x];
          const float x0 = s_rx[key], xL = s_rx[key + ci.y - 1];
          const float dxs = xL - x0;
          const float ty = (hL.x - h0.x) / dxs;
          const float sn = ty / sqrtf(__builtin_fmaf(ty, ty, 1.0f));
          const float tz = (hL.y - h0.y) / dxs;
          const float tl2 = tz * sqrtf(__builtin_fmaf(-sn, sn, 1.0f));
          if (key >= 0 && key < R) {
            int4 *dst = reinterpret_cast<int4 *>(B.wonmask) + 2 * (int64_t)(lbase + atomicAdd(&cur[key], 1));
            dst[0] = make_int4(tt, slot_enc(g0, ucl, key), (ci.y << 24) | sid0, nx);
            dst[1] = make_int4(__float_as_int(h0.x), __float_as_int(h0.y), __float_as_int(sn), __float_as_int(tl2));
          }
        } else {
          const tpcca_tracklet_t &o = B.trk[tt];
          const int key = o.status == 3 ? o.row_out : -1;
          if (key >= 0 && key < R) B.kf_tmp[lbase + atomicAdd(&cur[key], 1)] = tt;
        }
      }
      // the list in global memory is read by other lanes of this wave
      wave_sync();
      for (int r = lane; r < R; r += 64) cur[r] = off[r];
      wave_lds_sync();
      int pending = off[R];

      // ---- sweeps
      int rs = 0;
      for (;;) {
        if (pass == 1 ? rs > R : rs < -1) {
          // every tracklet ends by the row past the last (pass 1) or first
          // (pass 2); one still running means inconsistent slots: fail it
          if (phase != kIdle) {
            kf_fail(B, t, start_id, n_chain);
            phase = kIdle;
            atomicOr(&rd.err, 2);
          }
        }
        if (!__any(phase != kIdle)) {
          if (pending == 0) break;
          // a new sweep from the first row (in the pass's direction) that
          // still has tracklets to enter
          int found = -1;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = 64 * q + lane;
            const unsigned long long m = __ballot(r < R && off[r + 1] > cur[r]);
            if (m) {
              if (pass == 1) {
                if (found < 0) found = 64 * q + __builtin_ctzll(m);
              } else {
                found = 64 * q + 63 - __builtin_clzll(m);
              }
            }
          }
          if (found < 0) {  // the counts disagree with the list (cannot happen)
            if (lane == 0) atomicOr(&rd.err, 2);
            break;
          }
          rs = pass == 1 ? found + 1 : found;
        }
        // refill: idle lanes take the tracklets entering at this row
        {
          const int rr = pass == 1 ? rs - 1 : rs;
          if (rr >= 0 && rr < R) {
            const unsigned long long idle = __ballot(phase == kIdle);
            const int e0 = cur[rr];
            const int avail = off[rr + 1] - e0;
            if (idle && avail > 0) {
              const int take = min(__popcll(idle), avail);
              const int rank = __popcll(idle & below);
              if (phase == kIdle && rank < take) {
                if (pass == 1) {
                  const int4 *src = reinterpret_cast<const int4 *>(B.wonmask) + 2 * (int64_t)(lbase + e0 + rank);
                  const int4 a = src[0], b = src[1];
                  t = a.x;
                  r0 = slot_row(a.y);
                  n_chain = (int)((uint32_t)a.z >> 24);
                  start_id = a.z & 0xFFFFFF;
                  const float h0y = __int_as_float(b.y);
                  zr = h0y;
                  st.p[0] = __int_as_float(b.x);
                  st.p[1] = h0y - zr;
                  st.p[2] = __int_as_float(b.z);
                  st.p[3] = __int_as_float(b.w);
                  st.p[4] = 0.0f;
#pragma unroll
                  for (int q = 0; q < 15; ++q) st.C[q] = 0.0f;
                  st.C[0] = P.ery;
                  st.C[2] = P.erz;
                  st.C[5] = P.c22;
                  st.C[9] = P.c33;
                  st.C[14] = P.c44;
                  st.x = s_rx[r0];
                  s_slot[0][tid] = a.y;
                  gnext = a.w;
                  rlast = r0;
                  k = 1;
                  chi2 = 0.0f;
                  phase = kChain;
                } else {
                  t = B.kf_tmp[lbase + e0 + rank];
                  tpcca_tracklet_t &o = B.trk[t];
                  // start ID, chain length, start row and the z origin were
                  // left in the record by pass 1
                  start_id = o.start_id;
                  n_chain = o.n_chain;
                  r0 = o.row_ref;
                  zr = o.x_ref;
#pragma unroll
                  for (int q = 0; q < 5; ++q) st.p[q] = o.p_out[q];
#pragma unroll
                  for (int q = 0; q < 15; ++q) st.C[q] = o.cov_out[q];
                  st.x = o.x_out;
                  n1 = o.n_pass1;
                  o.p_out[1] = st.p[1] + zr;  // the record holds the absolute z
                  kf_restart(P, st);
                  chi2 = 0.0f;
                  ne = 0;
                  k = n1 - 1;
                  slot_load(k);
                  phase = kRefit;
                }
              }
              if (lane == 0) cur[rr] = e0 + take;
              pending -= take;
            }
          }
        }
        // ---- the row step at rs: one propagation, the staged row, one
        // search or given hit, one test, one update
        bool act = false, prop = false, end = false;
        int given = -1;
        if (phase == kChain) {
          act = prop = true;
          given = gnext;
        } else if (phase == kFollow) {
          end = rs >= R;
          act = prop = !end;
        } else if (phase == kRefit) {
          const int32_t v = s_slot[k & GM][tid];
          act = slot_row(v) == rs;
          prop = act && k < n1 - 1;
          given = act ? slot_hit(v, ucl) : -1;
        } else if (phase == kExtend) {
          end = rs < 0;
          act = prop = !end;
        }
        steps += __popcll(__ballot(prop));
        ++iters;
        bool ok = true;
        if (prop) ok = kf_propagate(P, st, s_rx[rs]);
        const bool need = act && ok;
        // windows and their bins (as kf_search computes them)
        RowTab trow;
        const bool row_ok = rs >= 0 && rs < R;
        if (row_ok) trow = rtab[rs];
        float wy = 0.0f, wz = 0.0f;
        int lo = 0x7FFFFFFF, hi = -1;
        if (need) {
          wy = P.nsig * sqrtf(st.C[0] + P.ery);
          wz = P.nsig * sqrtf(st.C[2] + P.erz);
          if (wy > P.wmax) wy = P.wmax;
          if (wz > P.wmax) wz = P.wmax;
          const float zc = zr + st.p[1];
          const float pad = 1e-3f + 1e-6f * fabsf(zc);
          lo = zbin(trow, zc - wz - pad);
          hi = zbin(trow, zc + wz + pad);
        }
        const int blo = wave_min_i(lo), bhi = wave_max_i(hi);
        bool bins_ok = false, hits_ok = false;
        int Hb = 0, He = 0;
        if (bhi >= 0 && bhi - blo + 2 <= kStageBins) {
          const int nbn = bhi - blo + 2;
          for (int j = lane; j < nbn; j += 64) bins[j] = B.binbeg[trow.bin0 + blo + j];
          wave_lds_sync();
          bins_ok = true;
          Hb = bins[0];
          He = bins[nbn - 1];
          if (He - Hb <= kStageHits) {
            const bool links = pass == 1 && __any(need && phase == kChain);
            for (int j = lane; j < He - Hb; j += 64) {
              yzs[j] = B.yz[Hb + j];
              if (links) ups[j] = B.upc[Hb + j];
            }
            wave_lds_sync();
            hits_ok = true;
          }
        }
        int h = given;
        float2 cc = make_float2(0.0f, 0.0f);
        const bool search = need && given < 0;
        if (need && given >= 0) cc = (hits_ok && given >= Hb && given < He) ? yzs[given - Hb] : B.yz[given];
        if (search) {
          int b, e;
          if (bins_ok) {
            b = bins[lo - blo];
            e = bins[hi + 1 - blo];
          } else {
            b = B.binbeg[trow.bin0 + lo];
            e = B.binbeg[trow.bin0 + hi + 1];
          }
          cands += (unsigned int)(e - b);
          int best = -1;
          float bd2 = __builtin_inff();
          for (int i = b; i < e; ++i) {
            const float2 q = hits_ok ? yzs[i - Hb] : B.yz[i];
            if (!(fabsf(q.x - st.p[0]) <= wy && fabsf((q.y - zr) - st.p[1]) <= wz)) continue;
            const float dy = q.x - st.p[0];
            const float dz = (q.y - zr) - st.p[1];
            const float d2 = __builtin_fmaf(dy, dy, dz * dz);
            // equal distances (rare) are decided by the lower cluster ID
            if (d2 < bd2 || (d2 == bd2 && B.sid[i] < B.sid[best])) {
              bd2 = d2;
              best = i;
              cc = q;
            }
          }
          h = best;
        }
        const float zm = cc.y - zr;
        bool acc = need && h >= 0;
        tests += __popcll(__ballot(acc && search));
        if (acc && search) {
          float cc2;
          acc = kf_chi2(P, st, cc.x, zm, cc2) && cc2 <= P.pick_chi2;
        }
        float c2 = 0.0f;
        updates += __popcll(__ballot(acc));
        const bool upd = acc && kf_update(P, st, cc.x, zm, c2);
        bool fin = false;  // a tracklet fit ended with enough hits: claim them
        // ---- bookkeeping
        if (phase == kChain) {
          if (!upd) {
            kf_fail(B, t, start_id, n_chain);
            phase = kIdle;
          } else {
            slot_put(k, slot_enc(h, ucl, rs));
            rlast = rs;
            if (++k == n_chain) {
              save_aux();
              miss = 0;
              n1 = n_chain;
              phase = kFollow;
            } else {
              // the chain's next hit: the link of this one, from LDS when staged
              gnext = (hits_ok && h >= Hb && h < He) ? ups[h - Hb] : B.upc[h];
            }
          }
        } else if (phase == kFollow) {
          if (!end) {
            if (!ok) {
              end = true;
            } else if (upd) {
              slot_put(n1, slot_enc(h, ucl, rs));
              ++n1;
              rlast = rs;
              save_aux();
              miss = 0;
            } else if (++miss >= P.max_miss) {
              end = true;
            }
          }
          if (end) {
            // end of pass 1: the last (partial) slot group to memory, the
            // state at the outermost hit into the record for pass 2
            if (n1 & GM) slot_flush(n1 - 1);
            tpcca_tracklet_t &o = B.trk[t];
#pragma unroll
            for (int q = 0; q < 5; ++q) o.p_out[q] = s_aux[q][tid];  // z relative to zr until pass 2
#pragma unroll
            for (int q = 0; q < 15; ++q) o.cov_out[q] = s_aux[5 + q][tid];
            o.x_out = s_aux[20][tid];
            o.n_pass1 = n1;
            o.row_out = rlast;
            o.start_id = start_id;
            o.n_chain = n_chain;
            o.row_ref = r0;   // until pass 2 ends: the start row
            o.x_ref = zr;     // until pass 2 ends: the z origin
            o.status = 3;     // pass 2 pending
            phase = kIdle;
          }
        } else if (phase == kRefit) {
          if (act) {
            if (!upd) {
              kf_fail(B, t, start_id, n_chain);
              phase = kIdle;
            } else {
              chi2 = chi2 + c2;
              if (--k < 0) {
                save_aux();
                ne = 0;
                miss = 0;
                phase = kExtend;
              } else if ((k & GM) == GM) {
                slot_load(k);
              }
            }
          }
        } else if (phase == kExtend) {
          if (!end) {
            if (!ok) {
              end = true;
            } else if (upd) {
              chi2 = chi2 + c2;
              const int j = n1 + ne;
              if ((j & ~GM) < n1)  // a group shared with pass-1 slots: this slot alone
                B.trk_hits[(int64_t)t * Rs + j] = slot_enc(h, ucl, rs);
              else
                slot_put(j, slot_enc(h, ucl, rs));
              ++ne;
              save_aux();
              miss = 0;
            } else if (++miss >= P.max_miss) {
              end = true;
            }
          }
          if (end) {
            tpcca_tracklet_t &o = B.trk[t];
            o.start_id = start_id;
            o.n_chain = n_chain;
            o.n_hits = n1 + ne;
            o.n_pass1 = n1;
            o.ndf = 2 * (n1 + ne) - 5;
            const int jl = n1 + ne - 1;
            if (ne > 0 && (jl & GM) != GM && (jl & ~GM) >= n1) slot_flush(jl);
            const int32_t *hl = B.trk_hits + (int64_t)t * Rs;
            o.row_out = slot_row(hl[n1 - 1]);
            o.row_ref = ne > 0 ? slot_row(hl[n1 + ne - 1]) : r0;
            o.x_ref = s_aux[20][tid];
            o.chi2 = chi2;
#pragma unroll
            for (int q = 0; q < 5; ++q) o.p[q] = s_aux[q][tid];
            o.p[1] = s_aux[1][tid] + zr;
#pragma unroll
            for (int q = 0; q < 15; ++q) o.cov[q] = s_aux[5 + q][tid];
            o.status = (n1 + ne) < P.min_hits ? 1 : 0;
            fin = o.status == 0;
            phase = kIdle;
          }
        }
        // ---- the selection's claims of the tracklets that ended in this step
        unsigned long long fm = P.kf_claims ? __ballot(fin) : 0ull;
        if (fm) {
          wave_sync();  // hit slots written by other lanes of this wave
          while (fm) {
            const int src = __builtin_ctzll(fm);
            fm &= fm - 1;
            const int tt = __builtin_amdgcn_readlane(t, src);
            const int nn = __builtin_amdgcn_readlane(n1 + ne, src);
            const unsigned long long kk = claim_key(
                nn, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(chi2), src)),
                __builtin_amdgcn_readlane(start_id, src));
            const int32_t *hh = B.trk_hits + (int64_t)tt * Rs;
            for (int j = lane; j < nn; j += 64) atomicMax(&B.owner[slot_hit(hh[j], ucl)], kk);
          }
        }
        // the bins and hits of this row are read by the next row's staging
        // only after every lane is done with them
        if (bins_ok) wave_lds_sync();
        rs += pass == 1 ? 1 : -1;
      }
      // the records and slots this pass wrote are read by other lanes next
      wave_sync();
    }
  }
  unsigned long long c64 = wave_sum((unsigned long long)cands);
  if (lane == 0) {
    atomicAdd(&rd.kf_steps, (unsigned long long)steps);
    atomicAdd(&rd.kf_cands, c64);
    atomicAdd(&rd.kf_tests, (unsigned long long)tests);
    atomicAdd(&rd.kf_updates, (unsigned long long)updates);
    atomicAdd(&rd.kf_iters, (unsigned long long)iters);
    atomicMin(&rd.kf_t_start, t_start);
    atomicMax(&rd.kf_t_end, (unsigned long long)__builtin_amdgcn_s_memrealtime());
  }
}

// ------------------------------------------------------------ launchers ---
static inline int grid_of(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

// Key and chunk-slot ranges of a run: [k0, k1) and [c0, c1).
static inline void rows_ranges(const RunHost &h, int gc, int64_t &k0, int64_t &k1, int64_t &c0, int64_t &c1) {
  k0 = h.trk0 / kZoPer + 2 * (int64_t)h.u0;
  k1 = (int64_t)(h.trk0 + h.trk_cap) / kZoPer + 2 * (int64_t)h.u1 - 1;
  c0 = h.trk0 / gc + (int64_t)h.u0;
  c1 = (int64_t)(h.trk0 + h.trk_cap) / gc + h.u1;
}

hipError_t launch_kf_order_rows(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s) {
  const int nu = h.u1 - h.u0;
  if (h.trk_cap <= 0 || nu <= 0) return hipSuccess;
  int64_t k0, k1, c0, c1;
  rows_ranges(h, P.kf_rows, k0, k1, c0, c1);
  hipError_t e = launch_fill_u64(reinterpret_cast<unsigned long long *>(B.zo_cnt + k0), k1 - k0, 0ull, s);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t *>(B.kf_chunks + c0), 4 * (c1 - c0), 0, s);
  if (e != hipSuccess) return e;
  k_zo_count<<<grid_of(h.trk_cap, 256, 4096), 256, 0, s>>>(B, P, run);
  e = launch_scan_tiles(B.zo_cnt + k0, k1 - k0, s);
  if (e != hipSuccess) return e;
  k_zo_apply<<<grid_of(h.trk_cap, 256, 4096), 256, 0, s>>>(B, run);
  k_chunk_table<<<grid_of(nu, 64, 1024), 64, 0, s>>>(B, run, P.kf_rows);
  return hipGetLastError();
}

struct RowsOccupancy {
  int cus = 1;
  int per = 1;
};

static const RowsOccupancy &rows_occupancy() {
  static std::mutex mu;
  static std::map<int, RowsOccupancy> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  RowsOccupancy o;
  int cus = 0, per = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_kf_rows<3>, kKfBlock, 0);
  o.cus = std::max(1, cus);
  o.per = std::max(1, per);
  return cache.emplace(dev, o).first->second;
}

hipError_t launch_kf_rows(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s) {
  const RowsOccupancy &o = rows_occupancy();
  const int bpc = P.kf_blocks_per_cu > 0 ? std::min(P.kf_blocks_per_cu, o.per) : o.per;
  if (h.trk_cap <= 0 || h.u1 <= h.u0) return hipSuccess;
  int64_t k0, k1, c0, c1;
  rows_ranges(h, P.kf_rows, k0, k1, c0, c1);
  const int g = grid_of(c1 - c0, 2, o.cus * bpc);  // two waves per block
  k_kf_rows<3><<<g, kKfBlock, 0, s>>>(B, P, run, c0, (int)(c1 - c0));
  return hipGetLastError();
}

}  // namespace tpcca
