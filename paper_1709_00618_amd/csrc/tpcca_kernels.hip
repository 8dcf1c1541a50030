// gfx950 kernels of the TPC sector tracker.
//
// Stages (Rohr, LHCP 2017, Sec. 2 and Fig. 1):
//   grid      counting sort of clusters by (unit, pad row, z bin)
//   links     CA neighbour finding: best straight-line (down, up) pair (Fig. 1a)
//   clean     keep reciprocal links; chains start at up-only hits (Fig. 1b)
//   tracklets chain compaction, then a per-thread two-pass Kalman fit with
//             track following (Fig. 1c)
//   select    one-round claim of clusters by (hits, chi2, id) keys, acceptance,
//             compaction of tracks, hits and the cluster assignment
//
// Every kernel is a grid-stride loop over work whose extent it reads from a
// device-side run descriptor, so the same launches serve one sector, one
// event, or a whole batch replayed from a captured graph.
//
// Floating point: compiled with -ffp-contract=off and correctly rounded FP32
// division and square root; fused multiply-adds appear only where written as
// __builtin_fmaf.  Decisions therefore reproduce, bit for bit, any other
// IEEE-754 implementation of the same operation sequence.
#include <hip/hip_runtime.h>

#include "tpcca_internal.h"
#include "tpcca_kernels.h"
#include "tpcca_dev.h"
#include "tpcca_kf.h"
#include "tpcca_fit.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace tpcca {

// ------------------------------------------------------------- helpers ---

// pad row of a cluster after validation; invalid clusters go to row R
__device__ __forceinline__ int valid_row(float4 c, int r, const float *row_x, int R) {
  if (r >= R) return R;
  if (!(isfinite(c.x) && isfinite(c.y) && isfinite(c.z))) return R;
  if (!(fabsf(c.x - row_x[r]) <= 1e-3f)) return R;
  return r;
}


// ----------------------------------------------------------- utilities ---
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Reset of a run's per-unit tables and device counters.
__global__ void k_run_reset(Bufs B, int run, int R) {
  RunDev &rd = B.runs[run];
  const int units = rd.u1 - rd.u0;
  const int nrow = units * (R + 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nrow; i += gridDim.x * blockDim.x) {
    B.row_cnt[(int64_t)rd.u0 * (R + 1) + i] = 0;
    B.row_fill[(int64_t)rd.u0 * (R + 1) + i] = 0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < units; i += gridDim.x * blockDim.x) {
    B.zmm[2 * (rd.u0 + i)] = 0x7FFFFFFF;
    B.zmm[2 * (rd.u0 + i) + 1] = (int)0x80000000;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rd.n_trk = 0;
    rd.n_acc = 0;
    rd.n_acc_hits = 0;
    rd.err = 0;
    for (int q = 0; q < kXcds; ++q) rd.kf_next[q] = 0;
    rd.n_starts = 0;
    rd.kf_steps = 0;
    rd.kf_cands = 0;
    rd.kf_tests = 0;
    rd.kf_updates = 0;
    rd.kf_iters = 0;
    rd.kf_t_start = rd.kf_t_drain = ~0ull;
    rd.kf_t_end = 0;
  }
}

// ---------------------------------------------------------------- grid ---
// Pass 1: clusters per (unit, row) and the z range of each unit.
// The kChunk / kBlock clusters of a thread in a chunk, loaded before any of
// them is used (independent loads in flight); the row positions come from LDS.
constexpr int kPer = kChunk / kBlock;

__device__ __forceinline__ void load_chunk(const UnitDev &U, const Chunk &ch, const float *s_rx, int R,
                                           float4 (&c4)[kPer], int (&r)[kPer]) {
  int raw[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = threadIdx.x + q * kBlock;
    const int li = ch.begin + (i < ch.count ? i : 0);
    c4[q] = U.cl[li];
    raw[q] = U.row[li];
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) r[q] = valid_row(c4[q], raw[q], s_rx, R);
}

// Each block counts a contiguous range of chunks: per chunk the row
// histogram (chunk_hist, read by the scatter pass), and per unit the row
// counts and z range, accumulated in LDS over the range's chunks of that
// unit and added to the unit's totals once per unit (atomics on the same
// few words from every chunk would serialise).
__global__ __launch_bounds__(kBlock) void k_count(Bufs B, int run, int R) {
  __shared__ int hist[kMaxRows + 1];
  __shared__ int acc[kMaxRows + 1];
  __shared__ int smin[kBlock / 64], smax[kBlock / 64], serr;
  __shared__ float s_rx[kMaxRows + 1];
  const RunDev &rd = B.runs[run];
  for (int r = threadIdx.x; r < R; r += blockDim.x) s_rx[r] = B.row_x[r];
  for (int r = threadIdx.x; r <= R; r += blockDim.x) acc[r] = 0;
  const int nch = rd.c1 - rd.c0;
  const int per = (nch + (int)gridDim.x - 1) / (int)gridDim.x;
  const int cb = rd.c0 + (int)blockIdx.x * per, ce = min(rd.c1, cb + per);
  int acc_unit = -1, acc_zmin = 0x7FFFFFFF, acc_zmax = (int)0x80000000;  // block-uniform
  // adds the accumulated counts and z range of unit acc_unit to its totals
  auto flush = [&]() {
    for (int r = threadIdx.x; r <= R; r += blockDim.x) {
      if (acc[r]) atomicAdd(&B.row_cnt[(int64_t)acc_unit * (R + 1) + r], acc[r]);
      acc[r] = 0;
    }
    if (threadIdx.x == 0 && acc_zmin != 0x7FFFFFFF) {
      atomicMin(&B.zmm[2 * acc_unit], acc_zmin);
      atomicMax(&B.zmm[2 * acc_unit + 1], acc_zmax);
    }
    acc_zmin = 0x7FFFFFFF;
    acc_zmax = (int)0x80000000;
  };
  for (int c = cb; c < ce; ++c) {
    const Chunk ch = B.chunks[c];
    const UnitDev U = B.units[ch.unit];
    if (ch.unit != acc_unit) {
      if (acc_unit >= 0) flush();
      acc_unit = ch.unit;
    }
    for (int r = threadIdx.x; r <= R; r += blockDim.x) hist[r] = 0;
    if (threadIdx.x == 0) serr = 0;
    __syncthreads();
    int zmin = 0x7FFFFFFF, zmax = (int)0x80000000, bad = 0;
    float4 cq[kPer];
    int rq[kPer];
    load_chunk(U, ch, s_rx, R, cq, rq);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (threadIdx.x + q * kBlock >= ch.count) break;
      const float4 c4 = cq[q];
      const int r = rq[q];
      atomicAdd(&hist[r], 1);
      if (r < R) {
        const int oz = ordered_int(c4.z);
        zmin = min(zmin, oz);
        zmax = max(zmax, oz);
      } else {
        bad = 1;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      zmin = min(zmin, __shfl_xor(zmin, o, 64));
      zmax = max(zmax, __shfl_xor(zmax, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      smin[threadIdx.x >> 6] = zmin;
      smax[threadIdx.x >> 6] = zmax;
    }
    if (bad) serr = 1;
    __syncthreads();
    for (int w = 0; w < kBlock / 64; ++w) {  // every thread: the block's z range
      acc_zmin = min(acc_zmin, smin[w]);
      acc_zmax = max(acc_zmax, smax[w]);
    }
    if (threadIdx.x == 0 && serr) B.runs[run].err = 1;
    for (int r = threadIdx.x; r <= R; r += blockDim.x) {
      B.chunk_hist[(int64_t)c * (R + 1) + r] = hist[r];
      acc[r] += hist[r];
    }
    __syncthreads();
  }
  if (acc_unit >= 0) flush();
}

// Pass 2 (one block per unit): row offsets and z-bin layout of every row.
__global__ __launch_bounds__(kBlock) void k_plan(Bufs B, int run, int R, int hits_per_bin, int tile) {
  __shared__ int64_t lds64[kBlock / 64 + 1];
  __shared__ int32_t lds32[kBlock / 64 + 1];
  const RunDev &rd = B.runs[run];
  for (int u = rd.u0 + blockIdx.x; u < rd.u1; u += gridDim.x) {
    const UnitDev U = B.units[u];
    const int r = threadIdx.x;
    const int cnt = r <= R ? B.row_cnt[(int64_t)u * (R + 1) + r] : 0;
    int32_t tot;
    const int32_t begin = block_exclusive_scan<int32_t>(cnt, lds32, &tot);
    int nb = 0;
    if (r < R) nb = max(1, min(cnt / hits_per_bin, kMaxBinsRow));
    else if (r == R) nb = 1;
    const int64_t width = r <= R ? (int64_t)nb + 1 : 0;
    int64_t wtot;
    const int64_t boff = block_exclusive_scan<int64_t>(width, lds64, &wtot);
    float z0 = 0.0f, z1 = 1.0f;
    const int a = B.zmm[2 * u], b = B.zmm[2 * u + 1];
    if (a != 0x7FFFFFFF) {
      z0 = from_ordered(a);
      z1 = from_ordered(b);
    }
    float span = z1 - z0;
    if (!(span > 1e-3f)) span = 1e-3f;
    if (r <= R) {
      RowTab t;
      t.begin = U.cl_begin + begin;
      t.count = cnt;
      t.nb = nb;
      t.bin0 = (int32_t)(U.bin_base + boff);
      t.pad_[0] = t.pad_[1] = 0;
      t.z0 = z0;
      t.inv = (float)nb / span;
      B.rowtab[(int64_t)u * (R + 1) + r] = t;
    }
    // row tiles of at most `tile` hits for the neighbour search; the unused
    // slots of the unit's reservation are marked empty
    const int nt = r <= R ? (cnt + tile - 1) / tile : 0;
    int32_t ttot;
    const int32_t toff = block_exclusive_scan<int32_t>(nt, lds32, &ttot);
    for (int i = 0; i < nt; ++i)
      B.tiles[U.tile_base + toff + i] =
          make_int4(u, r, U.cl_begin + begin + i * tile, min(tile, cnt - i * tile));
    const int cap = U.n / tile + R + 2;
    for (int i = ttot + r; i < cap; i += blockDim.x) B.tiles[U.tile_base + i] = make_int4(u, 0, 0, 0);
    __syncthreads();
  }
}

// Pass 3: group the clusters by (unit, row) into the staging buffer.  A
// block takes up to four consecutive chunks (kGroup), adds up their row
// histograms from the count pass, reserves one contiguous range per
// (unit, row) in the row's segment, and writes the records there through
// LDS cursors.  The order inside a row is arbitrary (every later decision
// compares cluster IDs, never positions).
constexpr int kGroup = 4;

__global__ __launch_bounds__(kBlock) void k_rowscatter(Bufs B, int run, int R) {
  __shared__ int hist[kGroup * (kMaxRows + 1)];
  __shared__ int cursor[kGroup * (kMaxRows + 1)];
  __shared__ int slot_unit[kGroup];
  __shared__ float s_rx[kMaxRows + 1];
  const RunDev &rd = B.runs[run];
  for (int r = threadIdx.x; r < R; r += blockDim.x) s_rx[r] = B.row_x[r];
  const int nslots = kGroup * (R + 1);
  const int ngroups = (rd.c1 - rd.c0 + kGroup - 1) / kGroup;
  for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    const int c0 = rd.c0 + gi * kGroup;
    const int c1 = min(rd.c1, c0 + kGroup);
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) hist[k] = 0;
    if (threadIdx.x == 0) {
      // distinct units of the group get consecutive slots
      int us = -1, prev = -1;
      for (int c = c0; c < c1; ++c) {
        const int u = B.chunks[c].unit;
        if (u != prev) {
          ++us;
          prev = u;
        }
        slot_unit[c - c0] = us;
      }
    }
    __syncthreads();
    // histogram of (unit slot, row): the count pass's per-chunk histograms
    for (int c = c0; c < c1; ++c) {
      const int so = slot_unit[c - c0] * (R + 1);
      for (int r = threadIdx.x; r <= R; r += blockDim.x) hist[so + r] += B.chunk_hist[(int64_t)c * (R + 1) + r];
      __syncthreads();  // chunks of one unit add into the same slots
    }
    // reserve one range per non-empty (unit, row)
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) {
      const int cnt = hist[k];
      cursor[k] = 0;
      if (cnt) {
        const int us = k / (R + 1), r = k - us * (R + 1);
        int u = -1;
        for (int c = c0; c < c1; ++c)
          if (slot_unit[c - c0] == us) {
            u = B.chunks[c].unit;
            break;
          }
        const int64_t rr = (int64_t)u * (R + 1) + r;
        cursor[k] = B.rowtab[rr].begin + atomicAdd(&B.row_fill[rr], cnt);
      }
    }
    __syncthreads();
    // write the records into the reserved runs
    for (int c = c0; c < c1; ++c) {
      const Chunk ch = B.chunks[c];
      const UnitDev U = B.units[ch.unit];
      const int so = slot_unit[c - c0] * (R + 1);
      float4 cq[kPer];
      int rq[kPer];
      load_chunk(U, ch, s_rx, R, cq, rq);
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kBlock;
        if (i >= ch.count) break;
        const int pos = atomicAdd(&cursor[so + rq[q]], 1);
        B.rtmp[pos] = make_int4(__float_as_int(cq[q].y), __float_as_int(cq[q].z), ch.begin + i, rq[q]);
      }
    }
    __syncthreads();
  }
}

// LDS index of bin k in the row sort's histogram: one padding word per 32
// bins, so that the scan's per-thread runs of 32 consecutive bins start in
// different banks.
__device__ __forceinline__ int hpad(int k) { return k + (k >> 5); }

// Pass 4, one block per (unit, row): counting sort of the row's records by
// z bin in LDS; writes the row's bin offsets and its sorted hits.
//   kStage false (sparse rows, kT = 256): the records are read twice (count,
//     then scatter) and scattered straight into the row's own segment.
//   kStage true (dense rows, kT = 1024, one block per CU by its LDS): a row
//     of up to kT * 8 records is read once into registers, sorted into LDS
//     and written out in order, so that no partially written line leaves
//     L2; a longer row takes the scatter path.
template <int kT, bool kStage>
__global__ __launch_bounds__(kT) void k_rowsort(Bufs B, int run, int R) {
  constexpr int kPer = 8, kCap = kStage ? kT * kPer : 1;
  __shared__ int hist[kMaxBinsRow + kMaxBinsRow / 32];
  __shared__ int lds[kT / 64 + 1];
  __shared__ float2 s_yz[kCap];
  __shared__ int32_t s_sid[kCap];
  __shared__ uint8_t s_row[kCap];
  const RunDev &rd = B.runs[run];
  const int nrows = (rd.u1 - rd.u0) * (R + 1);
  constexpr int per = kMaxBinsRow / kT;
  for (int w = blockIdx.x; w < nrows; w += gridDim.x) {
    const int64_t rr = (int64_t)rd.u0 * (R + 1) + w;
    const RowTab t = B.rowtab[rr];
    for (int k = threadIdx.x; k < t.nb; k += blockDim.x) hist[hpad(k)] = 0;
    __syncthreads();
    const bool staged = kStage && t.count <= kCap;  // uniform over the block
    int4 rec[kStage ? kPer : 1];
    int bin[kStage ? kPer : 1];
    if (staged) {
#pragma unroll
      for (int q = 0; q < (kStage ? kPer : 1); ++q) {
        const int i = threadIdx.x + q * kT;
        if (i < t.count) rec[q] = B.rtmp[t.begin + i];
      }
#pragma unroll
      for (int q = 0; q < (kStage ? kPer : 1); ++q) {
        const int i = threadIdx.x + q * kT;
        if (i < t.count) {
          bin[q] = zbin(t, __int_as_float(rec[q].y));
          atomicAdd(&hist[hpad(bin[q])], 1);
        }
      }
    } else {
#pragma unroll 4
      for (int i = threadIdx.x; i < t.count; i += blockDim.x) {
        const int4 r4 = B.rtmp[t.begin + i];
        atomicAdd(&hist[hpad(zbin(t, __int_as_float(r4.y)))], 1);
      }
    }
    __syncthreads();
    // exclusive scan of the nb bin counts (per consecutive entries per thread)
    int v[per];
    int loc = 0;
    for (int q = 0; q < per; ++q) {
      const int k = threadIdx.x * per + q;
      v[q] = k < t.nb ? hist[hpad(k)] : 0;
      loc += v[q];
    }
    int tot;
    int ex = block_exclusive_scan<int>(loc, lds, &tot);
    for (int q = 0; q < per; ++q) {
      const int k = threadIdx.x * per + q;
      if (k < t.nb) hist[hpad(k)] = ex;
      ex += v[q];
    }
    __syncthreads();
    // bin begins, written in coalesced order
    for (int k = threadIdx.x; k < t.nb; k += blockDim.x) B.binbeg[t.bin0 + k] = t.begin + hist[hpad(k)];
    if (threadIdx.x == 0) B.binbeg[t.bin0 + t.nb] = t.begin + t.count;
    __syncthreads();  // every begin is read before the scatter moves the cursors
    if (staged) {
#pragma unroll
      for (int q = 0; q < (kStage ? kPer : 1); ++q) {
        const int i = threadIdx.x + q * kT;
        if (i < t.count) {
          const int pos = atomicAdd(&hist[hpad(bin[q])], 1);
          s_yz[pos] = make_float2(__int_as_float(rec[q].x), __int_as_float(rec[q].y));
          s_sid[pos] = rec[q].z;
          s_row[pos] = (uint8_t)rec[q].w;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < t.count; i += blockDim.x) {
        B.yz[t.begin + i] = s_yz[i];
        B.sid[t.begin + i] = s_sid[i];
        B.srow[t.begin + i] = s_row[i];
      }
    } else {
#pragma unroll 4
      for (int i = threadIdx.x; i < t.count; i += blockDim.x) {
        const int4 r4 = B.rtmp[t.begin + i];
        const float z = __int_as_float(r4.y);
        const int pos = t.begin + atomicAdd(&hist[hpad(zbin(t, z))], 1);
        B.yz[pos] = make_float2(__int_as_float(r4.x), z);
        B.sid[pos] = r4.z;
        B.srow[pos] = (uint8_t)r4.w;
      }
    }
    __syncthreads();
  }
}

// Row of sorted hit g from the unit's row table held in LDS.
__device__ __forceinline__ int row_of(const RowTab *t, int R, int g) {
  int lo = 0, hi = R;  // rows 0..R; find last row with begin <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].begin <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- links ---
// Fig. 1a: for every hit of rows 1..R-2 the pair (u in row+1, d in row-1)
// inside |dy|, |dz| <= W dx that minimises (chi2, id_u, id_d), where chi2 is
// the squared deviation of the hit from the line d -> u at the hit's row.
//
// One block per row tile (<= kT hits of one row, contiguous in z-bin
// order; the tile size is a schedule knob: 128, 256 or 512).  The z bins of rows r-1 and r+1 that any hit of the tile can reach
// are a contiguous range of sorted hits; they are staged in LDS with their
// bin offsets, so every candidate test reads LDS.  Tiles whose neighbour
// ranges exceed the LDS capacity read the candidates from global memory.
// Tiles are walked XCD by XCD so that neighbouring rows of a unit share an
// L2.
// Staging capacities come in variants (tuning knob link_stage): larger ones
// fall back to global memory less often, smaller ones let more blocks share
// a CU's LDS.  Variant 0 takes 19.5 KB of LDS; the kernel is held to 72
// VGPRs (seven waves per SIMD), so 7 blocks of 256 threads share a CU.
template <int kV> struct LinkCaps;
template <> struct LinkCaps<0> { static constexpr int nbr = 1024, bins = 768; };
template <> struct LinkCaps<1> { static constexpr int nbr = 1536, bins = 1024; };
template <> struct LinkCaps<2> { static constexpr int nbr = 768, bins = 512; };

template <bool kLds>
__device__ __forceinline__ float2 cand(const Bufs &B, const float2 *src, int i, int off) {
  return kLds ? src[i - off] : B.yz[i];
}

// Best pair so far (chi2, sorted indices of the up and down hits).
struct LinkBest {
  float c2;
  int u, d;
};

// The straight-line deviation of a (u, d) pair: the deviation is formed
// from coordinate differences, (h - d) - w (u - d), rounded once:
// differences of nearby hits are exact, so it keeps its precision at the
// large z' of a time frame.
__device__ __forceinline__ float link_c2(float2 h, float w, float2 cu, float2 cd) {
  const float ey = __builtin_fmaf(-(cu.x - cd.x), w, h.x - cd.x);
  const float ez = __builtin_fmaf(-(cu.y - cd.y), w, h.y - cd.y);
  return __builtin_fmaf(ey, ey, ez * ez);
}

// One (u, d) pair against the best so far: smaller chi2, ties by cluster IDs.
__device__ __forceinline__ void link_pair(const Bufs &B, float2 h, float w, float2 cu, float2 cd, int u, int d,
                                          LinkBest &b) {
  const float c2 = link_c2(h, w, cu, cd);
  bool take = c2 < b.c2;
  if (!take && c2 == b.c2 && b.u >= 0) {
    const int iu = B.sid[u], id = B.sid[d], ibu = B.sid[b.u], ibd = B.sid[b.d];
    take = iu < ibu || (iu == ibu && id < ibd);
  }
  if (take) {
    b.c2 = c2;
    b.u = u;
    b.d = d;
  }
}

// Every pair of the two windows: used when a side holds more window hits
// than the lists, or when the tile's neighbours are not staged.  Rare, and
// kept out of line so that the common path compiles to short loops.
template <bool kLds>
__device__ __noinline__ LinkBest link_all_pairs(const Bufs &B, float2 h, float luy, float luz, float ldy,
                                                float ldz, float w, int ub, int ue, int db, int de,
                                                const float2 *cu_src, const float2 *cd_src, int u_off,
                                                int d_off) {
  LinkBest b{__builtin_inff(), -1, -1};
  for (int u = ub; u < ue; ++u) {
    const float2 cu = cand<kLds>(B, cu_src, u, u_off);
    if (!(fabsf(cu.x - h.x) <= luy && fabsf(cu.y - h.y) <= luz)) continue;
    for (int d = db; d < de; ++d) {
      const float2 cd = cand<kLds>(B, cd_src, d, d_off);
      if (!(fabsf(cd.x - h.x) <= ldy && fabsf(cd.y - h.y) <= ldz)) continue;
      link_pair(B, h, w, cu, cd, u, d, b);
    }
  }
  return b;
}

// Marks the staged hits in [b, e) (at most kMaxScan of them) that lie inside
// the window around h: bit k stands for hit b + k.  The loop has no
// branches: lanes of a wave scan in step, two candidates per step (one
// paired LDS read), and the bit positions of each step are the same for
// every lane (the step count is uniform; candidates 32.. go to the high
// word in a second loop, so no 64-bit shift is needed).  The second read of
// the last step may touch the entry after the range (the staging arrays
// hold one spare entry); bits past the range are cleared after the loops.
__device__ __forceinline__ bool in_window(float2 c, float2 h, float ly, float lz) {
  // bitwise &: both tests are evaluated (no short-circuit branches)
  return (fabsf(c.x - h.x) <= ly) & (fabsf(c.y - h.y) <= lz);
}

__device__ __forceinline__ unsigned long long window_mask(const float2 *src, int off, int b, int e, float2 h,
                                                          float ly, float lz) {
  unsigned int lo = 0u, hi = 0u;
  for (int k = 0; k < 32 && b + k < e; k += 2) {
    const float2 c0 = src[b + k - off], c1 = src[b + k + 1 - off];
    lo |= (in_window(c0, h, ly, lz) ? 1u << k : 0u) | (in_window(c1, h, ly, lz) ? 2u << k : 0u);
  }
  for (int k = 32; b + k < e; k += 2) {
    const float2 c0 = src[b + k - off], c1 = src[b + k + 1 - off];
    hi |= (in_window(c0, h, ly, lz) ? 1u << (k - 32) : 0u) | (in_window(c1, h, ly, lz) ? 2u << (k - 32) : 0u);
  }
  const int n = e - b;
  const unsigned long long m = ((unsigned long long)hi << 32) | lo;
  return n >= 64 ? m : m & ((1ull << n) - 1ull);
}

// Candidate ranges up to this long take the mask path (one 64-bit mask).
constexpr int kMaxScan = 64;

// The common path, neighbours staged in LDS: the window hits of each side
// are marked in a bit mask, then the marked hits are paired (the pair loop
// runs over the few marked hits only, so lanes with different candidate
// counts do not multiply their trip counts).  Longer ranges take the full
// double loop.  The best pair is the smallest (chi2, up ID, down ID): the
// pair loop compares chi2 alone and notes whether another pair equals the
// best one's chi2; only then (rare: exact float ties) are the pairs visited
// again with the cluster IDs read, so that the ID reads stay out of the
// common loop.  The order of the visits does not change the result.
__device__ __forceinline__ LinkBest link_hit_lds(const Bufs &B, float2 h, float luy, float luz, float ldy,
                                                 float ldz, float w, int ub, int ue, int db, int de,
                                                 const float2 *s_up, const float2 *s_dn, int u_off, int d_off) {
  if (ue - ub > kMaxScan || de - db > kMaxScan)
    return link_all_pairs<true>(B, h, luy, luz, ldy, ldz, w, ub, ue, db, de, s_up, s_dn, u_off, d_off);
  LinkBest b{__builtin_inff(), -1, -1};
  const unsigned long long mu = window_mask(s_up, u_off, ub, ue, h, luy, luz);
  if (mu == 0ull) return b;
  const unsigned long long md = window_mask(s_dn, d_off, db, de, h, ldy, ldz);
  if (md == 0ull) return b;
  // the best pair is kept as bit positions in the two masks until the end
  const float2 *const su = s_up + (ub - u_off), *const sd = s_dn + (db - d_off);
  bool tie = false;
  auto visit = [&](int pu, float2 cu, int pd) {
    const float c2 = link_c2(h, w, cu, sd[pd]);
    const bool better = c2 < b.c2;
    tie = !better && (tie || c2 == b.c2);
    b.c2 = better ? c2 : b.c2;
    b.u = better ? pu : b.u;
    b.d = better ? pd : b.d;
  };
  if (__ballot(((mu | md) >> 32) != 0ull) == 0ull) {
    // every lane's marks fit the low word (the common case): 32-bit loops
    for (unsigned int a = (unsigned int)mu; a != 0u; a &= a - 1u) {
      const int pu = __builtin_ctz(a);
      const float2 cu = su[pu];
      for (unsigned int q = (unsigned int)md; q != 0u; q &= q - 1u) visit(pu, cu, __builtin_ctz(q));
    }
  } else {
    for (unsigned long long a = mu; a != 0ull; a &= a - 1ull) {
      const int pu = __builtin_ctzll(a);
      const float2 cu = su[pu];
      for (unsigned long long q = md; q != 0ull; q &= q - 1ull) visit(pu, cu, __builtin_ctzll(q));
    }
  }
  if (b.u >= 0) {
    b.u += ub;
    b.d += db;
  }
  if (tie) {
    b = LinkBest{__builtin_inff(), -1, -1};
    for (unsigned long long a = mu; a != 0ull; a &= a - 1ull) {
      const int u = ub + __builtin_ctzll(a);
      const float2 cu = s_up[u - u_off];
      for (unsigned long long q = md; q != 0ull; q &= q - 1ull) {
        const int d = db + __builtin_ctzll(q);
        link_pair(B, h, w, cu, s_dn[d - d_off], u, d, b);
      }
    }
  }
  return b;
}

template <int kV, int kT>
__global__ __launch_bounds__(kT, 7) void k_links(Bufs B, ParamsDev P, int run) {
  constexpr int kNbrCap = LinkCaps<kV>::nbr, kBinCap = LinkCaps<kV>::bins;
  static_assert(kNbrCap < 65536, "bin offsets are 16-bit");
  __shared__ float2 s_up[kNbrCap + 1], s_dn[kNbrCap + 1];  // + the spare entry of window_mask
  __shared__ uint16_t s_bup[kBinCap + 1], s_bdn[kBinCap + 1];  // bin starts - ua / - da
  __shared__ int s_red[2 * (kT / 64)];
  // defined contents for the entries after a tile's staged range (read by
  // window_mask's last step, never used); the tile loop's first barrier
  // orders this before any read
  for (int q = threadIdx.x; q <= kNbrCap; q += blockDim.x) s_up[q] = s_dn[q] = make_float2(0.0f, 0.0f);
  const int R = P.n_rows;
  // the interpolation weight of each inner row, w = dx_down / (dx_down +
  // dx_up), computed once per block (the same operations as per tile)
  __shared__ float s_w[kMaxRows + 1];
  for (int q = 1 + threadIdx.x; q < R - 1; q += blockDim.x) {
    const float xr = B.row_x[q];
    const float dxu = B.row_x[q + 1] - xr, dxd = xr - B.row_x[q - 1];
    s_w[q] = dxd / (dxd + dxu);
  }
  const RunDev &rd = B.runs[run];
  const int ntile = rd.tile1 - rd.tile0;
  // XCD-aware walk: blocks b with b % 8 == x take the x-th eighth of tiles
  const int nx = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int per = (ntile + 7) >> 3;
  const int lo = xcd * per, hi = min(ntile, lo + per);
  for (int it = lo + (int)(blockIdx.x >> 3); it < hi; it += nx) {
    const int4 tile = B.tiles[rd.tile0 + it];
    const int cnt = tile.w;
    if (cnt == 0) continue;
    const int u = tile.x, r = tile.y, g0 = tile.z;
    const int i = threadIdx.x;
    const int g = g0 + i;
    if (r < 1 || r > R - 2) {
      if (i < cnt) {
        B.up[g] = -1;
        B.dn[g] = -1;
      }
      continue;
    }
    const RowTab *rtu = B.rowtab + (int64_t)u * (R + 1);
    const RowTab tu = rtu[r + 1], td = rtu[r - 1];
    const float xr = B.row_x[r];
    const float dxu = B.row_x[r + 1] - xr;
    const float dxd = xr - B.row_x[r - 1];
    const float luy = P.wy * dxu, luz = P.wz * dxu, ldy = P.wy * dxd, ldz = P.wz * dxd;
    float2 h = make_float2(0.0f, 0.0f);
    int zmin = 0x7FFFFFFF, zmax = (int)0x80000000;
    if (i < cnt) {
      h = B.yz[g];
      zmin = zmax = ordered_int(h.y);
    }
    zmin = wave_min_dpp(zmin);
    zmax = wave_max_dpp(zmax);
    if ((i & 63) == 0) {
      s_red[i >> 6] = zmin;
      s_red[(kT / 64) + (i >> 6)] = zmax;
    }
    __syncthreads();  // also orders the row weights before their first read
    const float w = s_w[r];
    // the tile's z range: the waves' ordered-int extremes combined as
    // integers and converted once, in scalar registers (the tile-wide bin
    // indices below are made wave-uniform the same way)
    int zlo_o = s_red[0], zhi_o = s_red[kT / 64];
    for (int q = 1; q < kT / 64; ++q) {
      zlo_o = min(zlo_o, s_red[q]);
      zhi_o = max(zhi_o, s_red[(kT / 64) + q]);
    }
    const float zlo = from_ordered(__builtin_amdgcn_readfirstlane(zlo_o));
    const float zhi = from_ordered(__builtin_amdgcn_readfirstlane(zhi_o));
    // tile-wide bin ranges of the neighbour rows (a superset of every hit's)
    const float tpad = 1e-3f + 1e-6f * fmaxf(fabsf(zlo), fabsf(zhi));
    const int ublo = __builtin_amdgcn_readfirstlane(zbin(tu, zlo - luz - tpad));
    const int ubhi = __builtin_amdgcn_readfirstlane(zbin(tu, zhi + luz + tpad));
    const int dblo = __builtin_amdgcn_readfirstlane(zbin(td, zlo - ldz - tpad));
    const int dbhi = __builtin_amdgcn_readfirstlane(zbin(td, zhi + ldz + tpad));
    const int ua = B.binbeg[tu.bin0 + ublo], ue_ = B.binbeg[tu.bin0 + ubhi + 1];
    const int da = B.binbeg[td.bin0 + dblo], de_ = B.binbeg[td.bin0 + dbhi + 1];
    const bool lds = (ue_ - ua) <= kNbrCap && (de_ - da) <= kNbrCap && (ubhi - ublo + 2) <= kBinCap &&
                     (dbhi - dblo + 2) <= kBinCap;
    if (lds) {
      for (int q = i; q < ue_ - ua; q += blockDim.x) s_up[q] = B.yz[ua + q];
      for (int q = i; q < de_ - da; q += blockDim.x) s_dn[q] = B.yz[da + q];
      for (int q = i; q <= ubhi - ublo + 1; q += blockDim.x)
        s_bup[q] = (uint16_t)(B.binbeg[tu.bin0 + ublo + q] - ua);
      for (int q = i; q <= dbhi - dblo + 1; q += blockDim.x)
        s_bdn[q] = (uint16_t)(B.binbeg[td.bin0 + dblo + q] - da);
    }
    __syncthreads();
    if (i < cnt) {
      const float pad = 1e-3f + 1e-6f * fabsf(h.y);
      const int bu0 = zbin(tu, h.y - luz - pad), bu1 = zbin(tu, h.y + luz + pad);
      const int bd0 = zbin(td, h.y - ldz - pad), bd1 = zbin(td, h.y + ldz + pad);
      LinkBest b;
      if (lds) {
        const int ub = ua + s_bup[bu0 - ublo], ue = ua + s_bup[bu1 + 1 - ublo];
        const int db = da + s_bdn[bd0 - dblo], de = da + s_bdn[bd1 + 1 - dblo];
        b = link_hit_lds(B, h, luy, luz, ldy, ldz, w, ub, ue, db, de, s_up, s_dn, ua, da);
      } else {
        const int ub = B.binbeg[tu.bin0 + bu0], ue = B.binbeg[tu.bin0 + bu1 + 1];
        const int db = B.binbeg[td.bin0 + bd0], de = B.binbeg[td.bin0 + bd1 + 1];
        b = link_all_pairs<false>(B, h, luy, luz, ldy, ldz, w, ub, ue, db, de, nullptr, nullptr, 0, 0);
      }
      const bool ok = b.u >= 0 && b.c2 <= P.link_chi2;
      B.up[g] = ok ? b.u : -1;
      B.dn[g] = ok ? b.d : -1;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- clean ---
// Fig. 1b: keep a link only if its partner links back; a hit with an up
// link and no down link starts a chain.  Each chunk lists its start hits in
// its own region of a staging array (an LDS counter, no global atomics) and
// stores their count for the scan that compacts the lists.
__global__ __launch_bounds__(kBlock) void k_clean(Bufs B, int run) {
  __shared__ int cnt;
  const RunDev &rd = B.runs[run];
  int2 *stage = reinterpret_cast<int2 *>(B.rtmp);  // free after the grid stage
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const UnitDev U = B.units[ch.unit];
    const int cb = U.cl_begin + ch.begin;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    // a thread's hits: links first, then the partners' links, all in flight together
    int lu[kPer], ld[kPer], pu[kPer], pd[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kBlock;
      const int g = cb + (i < ch.count ? i : 0);
      lu[q] = i < ch.count ? B.up[g] : -1;
      ld[q] = i < ch.count ? B.dn[g] : -1;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      pu[q] = lu[q] >= 0 ? B.dn[lu[q]] : -1;
      pd[q] = ld[q] >= 0 ? B.up[ld[q]] : -1;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kBlock;
      if (i >= ch.count) break;
      const int g = cb + i;
      const int uc = (lu[q] >= 0 && pu[q] == g) ? lu[q] : -1;
      const int dc = (ld[q] >= 0 && pd[q] == g) ? ld[q] : -1;
      B.upc[g] = uc;
      B.dnc[g] = dc;
      if (uc >= 0 && dc < 0) stage[cb + atomicAdd(&cnt, 1)] = make_int2(g, U.cl_begin + B.sid[g]);
    }
    __syncthreads();
    if (threadIdx.x == 0) B.scan_tmp[c - rd.c0] = cnt;
    __syncthreads();
  }
}

// The chunks' start lists, concatenated into the run's list at the scanned
// offsets (block per chunk).
__global__ __launch_bounds__(kBlock) void k_starts_compact(Bufs B, int run) {
  RunDev &rd = B.runs[run];
  const int2 *stage = reinterpret_cast<const int2 *>(B.rtmp);
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const int cb = B.units[ch.unit].cl_begin + ch.begin;
    const int64_t off = B.scan_tmp[c - rd.c0];
    const int n = (int)(B.scan_tmp[c - rd.c0 + 1] - off);
    for (int k = threadIdx.x; k < n; k += blockDim.x) B.starts[rd.cl0 + off + k] = stage[cb + k];
    if (c == rd.c1 - 1 && threadIdx.x == 0) rd.n_starts = (int32_t)B.scan_tmp[rd.c1 - rd.c0];
  }
}


// Chains: follow the cleaned up links from every start hit; a chain of at
// least min_chain hits marks its start in cluster-ID order (flag = sorted
// index + 1) and records (last hit, length).  Thread per start hit of the
// run's list, so that every resident lane chases a chain.
__global__ __launch_bounds__(kBlock) void k_chain(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int2 pc = order_piece(rd.n_starts);
  for (int k = pc.x + (int)threadIdx.x; k < pc.y; k += (int)blockDim.x) {
    const int2 st = B.starts[rd.cl0 + k];
    const int g = st.x;
    int n = 1, last = g, nx = B.upc[g];
    for (int s = 0; nx >= 0 && s < P.n_rows; ++s) {
      ++n;
      last = nx;
      nx = B.upc[nx];
    }
    if (n >= P.min_chain) {
      B.flag[st.y] = g + 1;
      B.cinfo[g] = make_int2(last, n);
      // 2: a long chain, fitted in the first part of the processing order
      B.sval[g] = (P.kf_split > 0 && P.kf_bands == 0 && n >= P.kf_split) ? 2 : 1;
    }
  }
}

// ---------------------------------------------------------------- scans ---
// Exclusive scan of n tile sums in place (one block); sums[n] = total.
__global__ __launch_bounds__(1024) void k_scan_tiles(int64_t *sums, int64_t n) {
  // one pass covers kSpan values: loaded and stored coalesced through LDS,
  // scanned kPerT consecutive values per thread (LDS index padded by one
  // word per 32 against bank conflicts)
  constexpr int kPerT = 8, kSpan = 1024 * kPerT;
  __shared__ int64_t buf[kSpan + kSpan / 32];
  __shared__ int64_t lds[1024 / 64 + 1];
  auto pad = [](int i) { return i + (i >> 5); };
  int64_t carry = 0;
  for (int64_t s = 0; s < n; s += kSpan) {
#pragma unroll
    for (int q = 0; q < kPerT; ++q) {
      const int i = q * 1024 + (int)threadIdx.x;
      buf[pad(i)] = s + i < n ? sums[s + i] : 0;
    }
    __syncthreads();
    int64_t v[kPerT];
    int64_t loc = 0;
#pragma unroll
    for (int q = 0; q < kPerT; ++q) {
      v[q] = buf[pad((int)threadIdx.x * kPerT + q)];
      loc += v[q];
    }
    int64_t tot;
    int64_t ex = carry + block_exclusive_scan<int64_t>(loc, lds, &tot);  // ends with a barrier
#pragma unroll
    for (int q = 0; q < kPerT; ++q) {
      buf[pad((int)threadIdx.x * kPerT + q)] = ex;
      ex += v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPerT; ++q) {
      const int i = q * 1024 + (int)threadIdx.x;
      if (s + i < n) sums[s + i] = buf[pad(i)];
    }
    __syncthreads();  // the next pass refills buf
    carry += tot;
  }
  if (threadIdx.x == 0) sums[n] = carry;
}

// Tracklet compaction: per chunk, count flags (tile = chunk).
__global__ __launch_bounds__(kBlock) void k_flag_sums(Bufs B, int run) {
  __shared__ int64_t part[kBlock / 64];
  const RunDev &rd = B.runs[run];
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const int base = B.units[ch.unit].cl_begin + ch.begin;
    int64_t v = 0;
    for (int i = threadIdx.x; i < ch.count; i += blockDim.x) v += B.flag[base + i] != 0;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int w = 0; w < kBlock / 64; ++w) tot += part[w];
      B.scan_tmp[c - rd.c0] = tot;
    }
    __syncthreads();
  }
}

// Tracklet compaction: slots in cluster-ID order (ascending start IDs).
__global__ __launch_bounds__(kBlock) void k_flag_apply(Bufs B, int run) {
  __shared__ int64_t lds[kBlock / 64 + 1];
  RunDev &rd = B.runs[run];
  constexpr int per = kChunk / kBlock;
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const int base = B.units[ch.unit].cl_begin + ch.begin;
    int32_t f[per];
    int64_t loc = 0;
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x * per + k;
      f[k] = i < ch.count ? B.flag[base + i] : 0;
      loc += f[k] != 0;
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(loc, lds, &tot) + B.scan_tmp[c - rd.c0];
    if (ch.begin == 0 && threadIdx.x == 0) B.unit_tbegin[ch.unit] = rd.trk0 + (int32_t)ex;
    for (int k = 0; k < per; ++k) {
      if (f[k]) {
        const int t = rd.trk0 + (int32_t)ex;
        B.trk_start[t] = f[k] - 1;
        B.trk_unit[t] = ch.unit;
        B.tofg[f[k] - 1] = t;
        ++ex;
      }
    }
    if (c == rd.c1 - 1 && threadIdx.x == 0) rd.n_trk = (int32_t)B.scan_tmp[rd.c1 - rd.c0];
  }
}

// Processing order of the fit: tracklets ranked by the grid position
// (unit, row, z bin) of their start hit, so that the lanes of a wave follow
// nearby tracks and share cache lines.  Per chunk of sorted hits: count,
// then (after the tile scan) write the ranks.
// Processing order of the fit: the start hits in grid order, tracklets of
// long chains (sval 2) before the others (sval 1) when a split is set.
// Per chunk the two counts, scanned as one array [long..., short...].
__global__ __launch_bounds__(kBlock) void k_order_sums(Bufs B, int run) {
  __shared__ int64_t part[2][kBlock / 64];
  const RunDev &rd = B.runs[run];
  const int nch = rd.c1 - rd.c0;
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const int base = B.units[ch.unit].cl_begin + ch.begin;
    int64_t a = 0, b = 0;
    for (int i = threadIdx.x; i < ch.count; i += blockDim.x) {
      const int v = B.sval[base + i];
      a += v == 2;
      b += v == 1;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
      part[0][threadIdx.x >> 6] = a;
      part[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t ta = 0, tb = 0;
      for (int w = 0; w < kBlock / 64; ++w) {
        ta += part[0][w];
        tb += part[1][w];
      }
      B.scan_tmp[c - rd.c0] = ta;
      B.scan_tmp[nch + c - rd.c0] = tb;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_order_apply(Bufs B, int run, int32_t *dst) {
  __shared__ int64_t lds[kBlock / 64 + 1];
  const RunDev &rd = B.runs[run];
  const int nch = rd.c1 - rd.c0;
  constexpr int per = kChunk / kBlock;
  for (int c = rd.c0 + blockIdx.x; c < rd.c1; c += gridDim.x) {
    const Chunk ch = B.chunks[c];
    const int base = B.units[ch.unit].cl_begin + ch.begin;
    int f[per];
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x * per + k;
      f[k] = i < ch.count ? B.sval[base + i] : 0;
    }
    for (int cls = 2; cls >= 1; --cls) {
      int64_t loc = 0;
      for (int k = 0; k < per; ++k) loc += f[k] == cls;
      int64_t tot;
      int64_t ex = block_exclusive_scan<int64_t>(loc, lds, &tot) +
                   B.scan_tmp[(cls == 2 ? 0 : nch) + c - rd.c0];
      for (int k = 0; k < per; ++k) {
        if (f[k] == cls) {
          dst[rd.trk0 + (int32_t)ex] = B.tofg[base + threadIdx.x * per + k];
          ++ex;
        }
      }
      __syncthreads();  // lds is reused by the next class's scan
    }
  }
}

// Optional start-row bands of the fit's processing order: (band of the start
// row, unit, grid order) instead of (unit, grid order).  Tracklets that
// start at outer rows cannot run long, so when they come last the fit's
// drain is short; and the tracklets in flight together sweep neighbouring
// rows of all units.  In the unit-major order each (unit, band) bucket is
// contiguous, so a tracklet's new position is its bucket's band-major offset
// plus its rank inside the bucket.
__device__ __forceinline__ int start_band(const Bufs &B, int t, int nb, int R) {
  return (int)B.srow[B.trk_start[t]] * nb / R;
}

__global__ void k_band_count(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int nu = rd.u1 - rd.u0, nb = P.kf_bands;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rd.n_trk; i += gridDim.x * blockDim.x) {
    const int t = B.kf_tmp[rd.trk0 + i];
    atomicAdd(&B.band_tmp[start_band(B, t, nb, P.n_rows) * nu + (B.trk_unit[t] - rd.u0)], 1);
  }
}

// One block: exclusive scans of the bucket counts in the new order and in
// the unit-major order.  The new order keeps the first units unit-major and
// takes the last kf_tail units (all with kf_tail = 0) band by band.
__global__ __launch_bounds__(1024) void k_band_scan(Bufs B, ParamsDev P, int run) {
  __shared__ int32_t lds[1024 / 64 + 1];
  const RunDev &rd = B.runs[run];
  const int nu = rd.u1 - rd.u0, nb = P.kf_bands, n = nu * nb;
  const int nt = (P.kf_tail > 0 && P.kf_tail < nu) ? P.kf_tail : nu;  // units taken band by band
  const int u0 = nu - nt;
  const int32_t *cnt = B.band_tmp;
  int32_t *off_bm = B.band_tmp + n, *off_um = B.band_tmp + 2 * n;
  for (int order = 0; order < 2; ++order) {
    int32_t carry = 0;
    for (int s0 = 0; s0 < n; s0 += 1024) {
      const int k = s0 + threadIdx.x;  // position in the scan order
      int j = 0;                        // bucket index (band * nu + unit)
      if (k < n) {
        if (order == 1 || k < u0 * nb) {  // unit-major part
          j = (k % nb) * nu + k / nb;
        } else {                          // band-major part over the last nt units
          const int kk = k - u0 * nb;
          j = (kk / nt) * nu + u0 + kk % nt;
        }
      }
      const int32_t v = k < n ? cnt[j] : 0;
      int32_t tot;
      const int32_t ex = block_exclusive_scan<int32_t>(v, lds, &tot);
      if (k < n) (order == 0 ? off_bm : off_um)[j] = carry + ex;
      carry += tot;
      __syncthreads();
    }
  }
}

__global__ void k_band_apply(Bufs B, ParamsDev P, int run) {
  RunDev &rd = B.runs[run];
  const int nu = rd.u1 - rd.u0, nb = P.kf_bands, n = nu * nb;
  const int n_trk = rd.n_trk;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_trk; i += gridDim.x * blockDim.x) {
    const int t = B.kf_tmp[rd.trk0 + i];
    const int j = start_band(B, t, nb, P.n_rows) * nu + (B.trk_unit[t] - rd.u0);
    const int pos = B.band_tmp[n + j] + (i - B.band_tmp[2 * n + j]);
    if (pos < 0 || pos >= n_trk) {  // never write outside the run's slots
      atomicOr(&rd.err, 2);
      continue;
    }
    B.kf_order[rd.trk0 + pos] = t;
  }
}

// Units without clusters have no chunk: their first tracklet is the one of
// the next non-empty unit of the run (or the run's end).
__global__ void k_empty_units(Bufs B, int run) {
  const RunDev &rd = B.runs[run];
  for (int u = rd.u0 + blockIdx.x * blockDim.x + threadIdx.x; u < rd.u1;
       u += gridDim.x * blockDim.x) {
    if (B.units[u].n != 0) continue;
    int t = rd.trk0 + rd.n_trk;
    for (int v = u + 1; v < rd.u1; ++v)
      if (B.units[v].n != 0) {
        t = B.unit_tbegin[v];
        break;
      }
    B.unit_tbegin[u] = t;
  }
}

// ------------------------------------------------------------ tracklets ---
// Nearest hit (dy^2 + dz^2, ties to the lower ID) of the row described by t
// inside the prediction window; -1 if none; its coordinates are returned
// in bc.
// The state's z is relative to zr (see k_kf); the bins are looked up around
// the absolute prediction zr + z with a margin that covers its rounding.
__device__ __forceinline__ int kf_search(const Bufs &B, const ParamsDev &P, const RowTab &t,
                                         const KState &s, float zr, unsigned int &cands, float2 &bc) {
  float wy = P.nsig * sqrtf(s.C[0] + P.ery);
  float wz = P.nsig * sqrtf(s.C[2] + P.erz);
  if (wy > P.wmax) wy = P.wmax;
  if (wz > P.wmax) wz = P.wmax;
  int b, e;
  bin_range(t, B.binbeg, zr + s.p[1], wz, b, e);
  int best = -1;
  float bd2 = __builtin_inff();
  cands += (unsigned int)(e - b);
  // candidates in ascending sorted index, loaded two at a time (independent
  // loads in flight); the evaluation order is unchanged
  for (int i0 = b; i0 < e; i0 += 2) {
    float2 c[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) c[q] = i0 + q < e ? B.yz[i0 + q] : make_float2(0.0f, 0.0f);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = i0 + q;
      if (!(i < e && fabsf(c[q].x - s.p[0]) <= wy && fabsf((c[q].y - zr) - s.p[1]) <= wz)) continue;
      const float dy = c[q].x - s.p[0];
      const float dz = (c[q].y - zr) - s.p[1];
      const float d2 = __builtin_fmaf(dy, dy, dz * dz);
      // equal distances (rare) are decided by the lower cluster ID
      if (d2 < bd2 || (d2 == bd2 && B.sid[i] < B.sid[best])) {
        bd2 = d2;
        best = i;
        bc = c[q];
      }
    }
  }
  return best;
}

// Track following with the Kalman filter (Fig. 1c), one tracklet per lane:
// seed on the chain's first hit with the direction of its end points; pass 1
// updates with the chain and follows outward picking the nearest window hit
// with chi2 <= pick_chi2 (stop after max_miss empty rows); pass 2 restarts at
// the outermost hit with the pass-1 covariance x refit_inflate, refits inward
// through all pass-1 hits and continues below the chain start.
//
// The state's z is kept relative to zr, the z of the chain's first hit:
// measurements enter as z_hit - zr (exact for a track's own hits) and the
// outputs add zr back.  Time frames place z' tens of metres from the
// sector's origin (Sec. 5), where an absolute FP32 z would carry rounding
// errors comparable with the fit's resolution.
//
// The kernel is persistent and written as a per-lane state machine: every
// loop iteration performs one row step (propagate, search or take the given
// hit, update) of whatever phase the lane is in, and a lane whose tracklet
// is done takes the next one from a device work counter (one atomic per
// wave).  Lanes of a wave therefore stay busy while tracklets of very
// different lengths and phases share it; each tracklet still sees exactly
// the operation sequence of the sequential description above.
template <int kMinWaves, int kBlk>
__global__ __launch_bounds__(kBlk, kMinWaves) void k_kf(Bufs B, ParamsDev P, int run) {
  RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  const int n_trk = rd.n_trk;
  const int lane = threadIdx.x & 63;
  int phase = kIdle;
  bool exhausted = false;
  const int kPool = P.kf_pool;
  int t = 0, start_id = 0, n_chain = 0, r0 = 0, k = 0, r = 0, miss = 0, n1 = 0, ne = 0;
  int prev = 0;
  int u = 0, ucl = 0;  // the tracklet's unit and its first global cluster index
  float zr = 0.0f;     // z of the chain's first hit: the origin of the state's z
  // the row positions, staged once per block
  __shared__ float s_rx[kMaxRows + 1];
  for (int i = threadIdx.x; i < R; i += blockDim.x) s_rx[i] = B.row_x[i];
  __syncthreads();
  KState st;
  // aux state in LDS (frees registers for occupancy): the pass-1 state at
  // the outermost hit, then the pass-2 state at the innermost hit
  __shared__ float s_aux[21][kBlk];
  const int tid = threadIdx.x;
  // hit slots go to memory eight at a time (one aligned 32-B group): a lane
  // collects a group in LDS and writes it when complete or when its phase
  // ends; the refit reads them back a group at a time.  Scattered stores
  // narrower than a memory segment cost a read-modify-write each, so fewer,
  // wider ones matter.
  constexpr int G = kSlotGrp, GM = kSlotGrp - 1;
  __shared__ int32_t s_slot[G][kBlk];
  const int Rs = slot_stride(R);
  auto slot_flush = [&](int j) {  // the group holding slot j
    int4 *dst = reinterpret_cast<int4 *>(B.trk_hits + (int64_t)t * Rs + (j & ~GM));
    dst[0] = make_int4(s_slot[0][tid], s_slot[1][tid], s_slot[2][tid], s_slot[3][tid]);
    dst[1] = make_int4(s_slot[4][tid], s_slot[5][tid], s_slot[6][tid], s_slot[7][tid]);
  };
  auto slot_put = [&](int j, int32_t v) {
    s_slot[j & GM][tid] = v;
    if ((j & GM) == GM) slot_flush(j);
  };
  auto save_aux = [&]() {
#pragma unroll
    for (int q = 0; q < 5; ++q) s_aux[q][tid] = st.p[q];
#pragma unroll
    for (int q = 0; q < 15; ++q) s_aux[5 + q][tid] = st.C[q];
    s_aux[20][tid] = st.x;
  };
  float chi2 = 0.0f;
  unsigned int cands = 0;
  unsigned int steps = 0, tests = 0, updates = 0, iters = 0;  // wave totals (scalar)
  const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();
  int pnext = 0, pend = 0;  // wave-private pool of claimed tracklets
  // The processing order is cut into one slice per XCD.  Block b runs on
  // XCD b mod 8, whose waves drain that slice first (its L2 then holds the
  // hits of a few sectors rather than of all of them) and then help drain
  // the following slices.
  const int nsl = P.kf_xcd ? kXcds : 1;
  int part = blockIdx.x % nsl, tried = 0;
  int seen = 0;  // the work counter as of this wave's last claim
  for (;;) {
    const unsigned long long idle = __ballot(phase == kIdle);
    while (idle && pnext == pend && !exhausted) {
      // claim the next tracklets of the slice with one atomic per wave:
      // kPool neighbouring ones while many remain; in the last stretch
      // (less than a quarter pool per wave left, judged from this wave's
      // previous claim) fewer, but never fewer than the idle lanes, so that
      // at the end no wave holds a private backlog
      const int lo = (int)((int64_t)n_trk * part / nsl);
      const int hi = (int)((int64_t)n_trk * (part + 1) / nsl);
      const int nw = (int)((gridDim.x * blockDim.x) >> 6);
      const int want = max(__popcll(idle), min(kPool, 4 * (((hi - lo) - seen) / nw)));
      int base = 0;
      if (lane == 0) base = atomicAdd(&rd.kf_next[part], want);
      base = __shfl(base, 0, 64);
      seen = base + want;
      if (base < hi - lo) {
        pnext = lo + base;
        pend = min(pnext + want, hi);
      } else if (++tried == nsl) {
        exhausted = true;
        if (lane == 0) atomicMin(&rd.kf_t_drain, (unsigned long long)__builtin_amdgcn_s_memrealtime());
      } else {
        part = (part + 1) % nsl;
        seen = 0;
      }
    }
    if (idle && pnext < pend) {
      const int take = min(__popcll(idle), pend - pnext);
      const int rank = __popcll(idle & ((1ull << lane) - 1));
      const int mine = pnext + rank;
      pnext += take;
      {
        if (phase == kIdle) {
          const int tl = mine;
          if (rank < take) {
            t = B.kf_order[rd.trk0 + tl];
            const int g0 = B.trk_start[t];
            u = B.trk_unit[t];
            ucl = B.units[u].cl_begin;
            const int2 ci = B.cinfo[g0];
            const int gL = ci.x;
            n_chain = ci.y;
            r0 = B.srow[g0];
            start_id = B.sid[g0];
            const float2 h0 = B.yz[g0], hL = B.yz[gL];
            const float x0 = s_rx[r0], xL = s_rx[r0 + n_chain - 1];
            const float dxs = xL - x0;
            const float ty = (hL.x - h0.x) / dxs;
            const float sn = ty / sqrtf(__builtin_fmaf(ty, ty, 1.0f));
            const float tz = (hL.y - h0.y) / dxs;
            const float tl2 = tz * sqrtf(__builtin_fmaf(-sn, sn, 1.0f));
            zr = h0.y;
            st.p[0] = h0.x;
            st.p[1] = h0.y - zr;
            st.p[2] = sn;
            st.p[3] = tl2;
            st.p[4] = 0.0f;
#pragma unroll
            for (int q = 0; q < 15; ++q) st.C[q] = 0.0f;
            st.C[0] = P.ery;
            st.C[2] = P.erz;
            st.C[5] = P.c22;
            st.C[9] = P.c33;
            st.C[14] = P.c44;
            st.x = x0;
            s_slot[0][tid] = slot_enc(g0, ucl, r0);
            prev = g0;
            k = 1;
            chi2 = 0.0f;
            phase = kChain;
          }
        }
      }
    }
    if (!__any(phase != kIdle) && exhausted && pnext == pend) break;
    // ---- inputs of this row step: a given hit to update with, or a search
    bool act = phase != kIdle;
    bool prop = act;
    bool end = false;  // FOLLOW / EXTEND ran out of rows
    int given = -1;
    int row = 0;
    if (phase == kChain) {
      given = B.upc[prev];
      row = r0 + k;
    } else if (phase == kRefit) {
      if (k == n1 - 1 || (k & GM) == GM) {
        const int4 *src = reinterpret_cast<const int4 *>(B.trk_hits + (int64_t)t * Rs + (k & ~GM));
        const int4 q0 = src[0], q1 = src[1];
        s_slot[0][tid] = q0.x;
        s_slot[1][tid] = q0.y;
        s_slot[2][tid] = q0.z;
        s_slot[3][tid] = q0.w;
        s_slot[4][tid] = q1.x;
        s_slot[5][tid] = q1.y;
        s_slot[6][tid] = q1.z;
        s_slot[7][tid] = q1.w;
      }
      const int32_t v = s_slot[k & GM][tid];
      given = slot_hit(v, ucl);
      row = slot_row(v);
      prop = k < n1 - 1;
    } else if (phase == kFollow || phase == kExtend) {
      end = phase == kFollow ? r >= R : r < 0;
      row = r;
      if (end) act = prop = false;
    }
    // loads that do not depend on the propagation are issued before it, so
    // that their latency overlaps its arithmetic: the given hit, or the
    // grid description of the row to search
    float2 c = make_float2(0.0f, 0.0f);
    RowTab trow;
    if (given >= 0) c = B.yz[given];
    else if (act) trow = B.rowtab[(int64_t)u * (R + 1) + row];
    // ---- the step: one propagation, one search, one test, one update
    bool ok = true;
    steps += __popcll(__ballot(prop));
    ++iters;
    if (prop) ok = kf_propagate(P, st, s_rx[row]);
    int h = given;
    const bool search = act && ok && given < 0;
    if (search) h = kf_search(B, P, trow, st, zr, cands, c);
    const float zm = c.y - zr;
    bool acc = act && ok && h >= 0;
    tests += __popcll(__ballot(acc && search));
    if (acc && search) {
      float cc2;
      acc = kf_chi2(P, st, c.x, zm, cc2) && cc2 <= P.pick_chi2;
    }
    float c2 = 0.0f;
    updates += __popcll(__ballot(acc));
    const bool upd = acc && kf_update(P, st, c.x, zm, c2);
    bool fin = false;  // a tracklet fit ended with enough hits: claim them
    // ---- bookkeeping
    if (phase == kChain) {
      if (!upd) {
        kf_fail(B, t, start_id, n_chain);
        phase = kIdle;
      } else {
        slot_put(k, slot_enc(h, ucl, row));
        prev = h;
        if (++k == n_chain) {
          save_aux();
          r = r0 + n_chain;
          miss = 0;
          n1 = n_chain;
          phase = kFollow;
        }
      }
    } else if (phase == kRefit) {
      if (!upd) {
        kf_fail(B, t, start_id, n_chain);
        phase = kIdle;
      } else {
        chi2 = chi2 + c2;
        if (--k < 0) {
          save_aux();
          ne = 0;
          miss = 0;
          r = r0 - 1;
          phase = kExtend;
        }
      }
    } else if (phase == kFollow || phase == kExtend) {
      const bool fwd = phase == kFollow;
      if (!end) {
        if (!ok) {
          end = true;
        } else {
          if (upd) {
            if (fwd) {
              slot_put(n1, slot_enc(h, ucl, r));
              ++n1;
            } else {
              chi2 = chi2 + c2;
              const int j = n1 + ne;
              if ((j & ~GM) < n1)  // a group shared with pass-1 slots: this slot alone
                B.trk_hits[(int64_t)t * Rs + j] = slot_enc(h, ucl, r);
              else
                slot_put(j, slot_enc(h, ucl, r));
              ++ne;
            }
            save_aux();
            miss = 0;
          } else if (++miss >= P.max_miss) {
            end = true;
          }
          r += fwd ? 1 : -1;
        }
      }
      if (end && fwd) {
        // end of pass 1: its last (partial) slot group goes to memory (the
        // slots after n1 are written again by pass 2 or never read); keep
        // the pass-1 state in the record, restart for pass 2
        if (n1 & GM) slot_flush(n1 - 1);
        tpcca_tracklet_t &o = B.trk[t];
#pragma unroll
        for (int q = 0; q < 5; ++q) o.p_out[q] = st.p[q] = s_aux[q][tid];
        o.p_out[1] = st.p[1] + zr;
#pragma unroll
        for (int q = 0; q < 15; ++q) o.cov_out[q] = st.C[q] = s_aux[5 + q][tid];
        o.x_out = st.x = s_aux[20][tid];
        kf_restart(P, st);
        chi2 = 0.0f;
        k = n1 - 1;
        phase = kRefit;
      } else if (end) {
        tpcca_tracklet_t &o = B.trk[t];
        o.start_id = start_id;
        o.n_chain = n_chain;
        o.n_hits = n1 + ne;
        o.n_pass1 = n1;
        o.ndf = 2 * (n1 + ne) - 5;
        // the last partial group of pass-2 slots (one that does not share
        // pass-1 slots) goes to memory
        const int jl = n1 + ne - 1;
        if (ne > 0 && (jl & GM) != GM && (jl & ~GM) >= n1) slot_flush(jl);
        // outermost pass-1 hit and innermost hit, from their slots' rows
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
    // ---- the selection's claims of the tracklets that ended in this step:
    // the wave writes the claim key of each into the owner word of its hits
    // (one tracklet at a time, hit slots read by all lanes)
    unsigned long long fm = P.kf_claims ? __ballot(fin) : 0ull;
    if (fm) {
      // the hit slots were written by other lanes of this wave
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      while (fm) {
        const int src = __builtin_ctzll(fm);
        fm &= fm - 1;
        // wave-uniform values of the source lane (scalar registers)
        const int tt = __builtin_amdgcn_readlane(t, src);
        const int nn = __builtin_amdgcn_readlane(n1 + ne, src);
        const unsigned long long kk = claim_key(
            nn, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(chi2), src)),
            __builtin_amdgcn_readlane(start_id, src));
        const int uc = __builtin_amdgcn_readlane(ucl, src);
        const int32_t *hh = B.trk_hits + (int64_t)tt * Rs;
        for (int j = lane; j < nn; j += 64) atomicMax(&B.owner[slot_hit(hh[j], uc)], kk);
      }
    }
  }
  // work counters (one atomic per wave)
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

// ------------------------------------------------------------ selection ---
__device__ __forceinline__ unsigned long long select_key(const tpcca_tracklet_t &o) {
  return claim_key(o.n_hits, o.chi2, o.start_id);
}

// Thread per tracklet (64 neighbouring tracklets of the processing order
// per wave): claim its hits with its key (used when the fit does not write
// the claims itself); hit slots are read eight at a time.
__global__ __launch_bounds__(kBlock) void k_claim(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rd.n_trk; i += gridDim.x * blockDim.x) {
    const int t = B.kf_order[rd.trk0 + i];
    const tpcca_tracklet_t &o = B.trk[t];
    if (o.status != 0) continue;
    const unsigned long long key = select_key(o);
    const int32_t *hl = B.trk_hits + (int64_t)t * slot_stride(R);
    const int ucl = B.units[B.trk_unit[t]].cl_begin;
    const int n = o.n_hits;
    for (int j0 = 0; j0 < n; j0 += 8) {
      int h[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) h[q] = j0 + q < n ? slot_hit(hl[j0 + q], ucl) : -1;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (h[q] >= 0) atomicMax(&B.owner[h[q]], key);
    }
  }
}

// The selection kernels give each tracklet a group of lanes (eight
// neighbouring tracklets of the processing order per wave): the group walks
// the tracklet's hit slots a group width at a time, so a wave's trip count
// follows the lengths of eight tracklets rather than of sixty-four (groups
// of 16 lanes measured 2 % slower in the output pass).  In the acceptance
// pass a tracklet that loses its first hits is rejected after fewer owner
// reads.
constexpr int kGrp = 8;
constexpr int kWonGrp = 8;

// Count the hits a tracklet won, record which, accept or reject (a tracklet
// that has already lost too many hits is rejected without reading the rest).
template <int kG>
__global__ __launch_bounds__(kBlock) void k_won(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (kG - 1), g0 = lane & ~(kG - 1);
  const int2 pc = order_piece(rd.n_trk);
  for (int i = pc.x + (int)threadIdx.x / kG; i < pc.y; i += (int)blockDim.x / kG) {
    const int t = B.kf_order[rd.trk0 + i];
    const int tl = t - rd.trk0;
    const tpcca_tracklet_t &o = B.trk[t];
    unsigned long long v = 0;
    if (o.status == 0) {
      const unsigned long long key = select_key(o);
      const int32_t *hl = B.trk_hits + (int64_t)t * slot_stride(R);
      const int ucl = B.units[B.trk_unit[t]].cl_begin;
      unsigned long long *wm = B.wonmask + (int64_t)t * 4;
      const int n = o.n_hits;
      unsigned long long cur = 0;
      int won = 0;
      for (int j0 = 0; j0 < n; j0 += kG) {
        const int j = j0 + gl;
        const bool w = j < n && B.owner[slot_hit(hl[j], ucl)] == key;
        const unsigned int bits = (unsigned int)(__ballot(w) >> g0) & ((1u << kG) - 1);
        won += __popc(bits);
        cur |= (unsigned long long)bits << (j0 & 63);
        if (((j0 + kG) & 63) == 0 || j0 + kG >= n) {  // a 64-slot word is complete
          if (gl == 0) wm[j0 >> 6] = cur;
          cur = 0;
        }
        // stop once even winning every remaining hit could not reach the
        // acceptance bounds (the won mask is read for accepted tracks only)
        const int most = won + (n - (j0 + kG));
        if (j0 + kG < n && (most < P.min_hits || most * 100 < P.own_pct * n)) break;
      }
      if (won >= P.min_hits && won * 100 >= P.own_pct * n)
        v = (1ull << 40) | (unsigned long long)won;
    }
    if (gl == 0) B.accv[tl] = v;
  }
}

// Scan of accv over the run's tracklets (count read on the device).
__global__ __launch_bounds__(kBlock) void k_acc_sums(Bufs B, int run) {
  __shared__ unsigned long long part[kBlock / 64];
  const RunDev &rd = B.runs[run];
  const int64_t n = rd.n_trk;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    unsigned long long v = 0;
    for (int64_t i = t * kScanTile + threadIdx.x; i < min(n, (t + 1) * kScanTile); i += blockDim.x)
      v += B.accv[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (int w = 0; w < kBlock / 64; ++w) tot += part[w];
      B.scan_tmp[t] = (int64_t)tot;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_acc_tiles(Bufs B, int run) {
  __shared__ int64_t lds[1024 / 64 + 1];
  RunDev &rd = B.runs[run];
  const int64_t n = (rd.n_trk + kScanTile - 1) / kScanTile;
  int64_t carry = 0;
  for (int64_t s = 0; s < n; s += 1024) {
    const int64_t i = s + threadIdx.x;
    const int64_t v = i < n ? B.scan_tmp[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<int64_t>(v, lds, &tot);
    if (i < n) B.scan_tmp[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    B.scan_tmp[n] = carry;
    rd.n_acc = (int32_t)((unsigned long long)carry >> 40);
    rd.n_acc_hits = (int64_t)((unsigned long long)carry & ((1ull << 40) - 1));
    B.accx[rd.n_trk] = (unsigned long long)carry;
  }
}

__global__ __launch_bounds__(kBlock) void k_acc_apply(Bufs B, int run) {
  __shared__ int64_t lds[kBlock / 64 + 1];
  const RunDev &rd = B.runs[run];
  const int64_t n = rd.n_trk;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  constexpr int per = kScanTile / kBlock;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t s = t * kScanTile;
    unsigned long long v[per];
    int64_t loc = 0;
    for (int k = 0; k < per; ++k) {
      const int64_t i = s + threadIdx.x * per + k;
      v[k] = i < n ? B.accv[i] : 0;
      loc += (int64_t)v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(loc, lds, &tot) + B.scan_tmp[t];
    for (int k = 0; k < per; ++k) {
      const int64_t i = s + threadIdx.x * per + k;
      if (i < n) B.accx[i] = (unsigned long long)ex;
      ex += (int64_t)v[k];
    }
  }
}

__device__ __forceinline__ int acc_count(unsigned long long v) { return (int)(v >> 40); }
__device__ __forceinline__ int64_t acc_hits(unsigned long long v) {
  return (int64_t)(v & ((1ull << 40) - 1));
}

// Per-unit result table (after the accepted-track scan).
__global__ void k_unit_results(Bufs B, int run) {
  const RunDev &rd = B.runs[run];
  for (int u = rd.u0 + blockIdx.x * blockDim.x + threadIdx.x; u < rd.u1;
       u += gridDim.x * blockDim.x) {
    const UnitDev U = B.units[u];
    const int tb = B.unit_tbegin[u] - rd.trk0;
    const int te = (u + 1 < rd.u1) ? B.unit_tbegin[u + 1] - rd.trk0 : rd.n_trk;
    const unsigned long long a = B.accx[tb], b = B.accx[te];
    tpcca_unit_result_t r;
    r.slot = U.slot;
    r.sector = U.sector;
    r.n_clusters = U.n;
    r.n_tracklets = te - tb;
    r.n_tracks = acc_count(b) - acc_count(a);
    r.n_track_hits = (int32_t)(acc_hits(b) - acc_hits(a));
    r.cluster_begin = U.cl_begin;
    r.track_begin = rd.trk0 + acc_count(a);
    r.hit_begin = rd.cl0 + acc_hits(a);
    B.unit_res[u] = r;
  }
}

// Compaction of accepted tracks, a group of kGrp lanes per tracklet:
// parameters, won hits in ascending rows (inward hits were stored after the
// pass-1 hits, in descending rows) and the per-cluster assignment
// (unit-local track index).
__global__ __launch_bounds__(kBlock) void k_output(Bufs B, ParamsDev P, int run) {
  const RunDev &rd = B.runs[run];
  const int R = P.n_rows;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (kGrp - 1), g0 = lane & ~(kGrp - 1);
  // a grid-stride walk: its scattered assignment stores, not its reads, set
  // its time, and contiguous pieces per XCD measured slower here
  const int ng = (gridDim.x * blockDim.x) / kGrp;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) / kGrp; i < rd.n_trk; i += ng) {
    const int t = B.kf_order[rd.trk0 + i];
    const int tl = t - rd.trk0;
    if (B.accv[tl] == 0) continue;
    const tpcca_tracklet_t &o = B.trk[t];
    const int u = B.trk_unit[t];
    const int ucl = B.units[u].cl_begin;
    const int32_t tb = B.unit_res[u].track_begin;
    const int32_t hb = B.unit_res[u].hit_begin;
    const unsigned long long ex = B.accx[tl];
    const int k = rd.trk0 + acc_count(ex);
    const int64_t h0 = rd.cl0 + acc_hits(ex);
    const int32_t *hl = B.trk_hits + (int64_t)t * slot_stride(R);
    const int n1 = o.n_pass1, nh = o.n_hits, ne = nh - n1;
    const int local_track = k - tb;
    const unsigned long long *wmp = B.wonmask + (int64_t)t * 4;
    const unsigned long long m0 = wmp[0];
    const unsigned long long m1 = nh > 64 ? wmp[1] : 0ull;
    const unsigned long long m2 = nh > 128 ? wmp[2] : 0ull;
    const unsigned long long m3 = nh > 192 ? wmp[3] : 0ull;
    int w = 0;
    for (int j0 = 0; j0 < nh; j0 += kGrp) {
      const int j = j0 + gl;
      // slot of the j-th hit in row order
      const int slot = j < ne ? n1 + ne - 1 - j : j - ne;
      const unsigned long long m = slot < 64 ? m0 : slot < 128 ? m1 : slot < 192 ? m2 : m3;
      const bool won = j < nh && ((m >> (slot & 63)) & 1ull);
      const unsigned int bits = (unsigned int)(__ballot(won) >> g0) & ((1u << kGrp) - 1);
      if (won) {
        const int id = B.sid[slot_hit(hl[slot], ucl)];
        B.hits_out[h0 + w + __popc(bits & ((1u << gl) - 1))] = id;
        B.assign[ucl + id] = local_track;
      }
      w += __popc(bits);
    }
    if (gl == 0) {
      tpcca_track_t tr;
      tr.x_ref = o.x_ref;
      for (int q = 0; q < 5; ++q) tr.p[q] = o.p[q];
      for (int q = 0; q < 15; ++q) tr.cov[q] = o.cov[q];
      tr.chi2 = o.chi2;
      tr.ndf = o.ndf;
      tr.n_hits = w;
      tr.hit_offset = (int32_t)(h0 - hb);
      tr.sector = B.units[u].sector;
      tr.start_id = o.start_id;
      B.tracks[k] = tr;
    }
  }
}

// Sorted indices -> unit-local cluster IDs (for the parity getters).
__global__ void k_to_ids(const int32_t *sid, const int32_t *in, int32_t *out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = in[i];
    out[i] = v >= 0 ? sid[v] : -1;
  }
}

// Links of one unit in cluster-ID space.
__global__ void k_links_by_id(const int32_t *sid, const int32_t *up, const int32_t *dn, int32_t *out_up,
                              int32_t *out_dn, int32_t cl_begin, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = cl_begin + i;
    const int id = sid[g];
    const int a = up[g], b = dn[g];
    out_up[id] = a >= 0 ? sid[a] : -1;
    out_dn[id] = b >= 0 ? sid[b] : -1;
  }
}


// ============================================================ launchers ===
static inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;  // never an empty grid
  return (int)g;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<grid_for(n, 256 * 8, 4096), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_u64<<<grid_for(n, 256 * 8, 4096), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_scan_tiles(int64_t *sums, int64_t n, hipStream_t s) {
  if (n < 0) return hipSuccess;
  k_scan_tiles<<<1, 1024, 0, s>>>(sums, n);
  return hipGetLastError();
}

hipError_t launch_grid(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                       hipStream_t s) {
  const int R = P.n_rows;
  const int nch = h.c1 - h.c0, nu = h.u1 - h.u0;
  k_run_reset<<<grid_for((int64_t)nu * (R + 1), 256, 1024), 256, 0, s>>>(B, run, R);
  if (nch > 0) k_count<<<grid_for(nch, 1, 2048), kBlock, 0, s>>>(B, run, R);
  if (nu > 0) k_plan<<<grid_for(nu, 1, 4096), kBlock, 0, s>>>(B, run, R, P.hits_per_bin, link_tile_of(P));
  if (nch > 0) k_rowscatter<<<grid_for((nch + kGroup - 1) / kGroup, 1, 8192), kBlock, 0, s>>>(B, run, R);
  if (nu > 0) {
    // dense rows (time frames): the staged sort, one 1024-thread block per CU
    const int64_t rows = (int64_t)nu * (R + 1);
    if (h.dense)
      k_rowsort<1024, true><<<grid_for(rows, 1, 16384), 1024, 0, s>>>(B, run, R);
    else
      k_rowsort<kBlock, false><<<grid_for(rows, 1, 16384), kBlock, 0, s>>>(B, run, R);
  }
  return hipGetLastError();
}

hipError_t launch_links(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                        hipStream_t s) {
  const int nt = h.tile1 - h.tile0;
  if (nt > 0) {
    int g = grid_for(nt, 1, 256 * (P.link_blocks_per_cu > 0 ? P.link_blocks_per_cu : 32));
    g = (g + 7) & ~7;  // a multiple of the 8 XCDs
    const int tile = link_tile_of(P);
#define TPCCA_LINKS(V, T) k_links<V, T><<<g, T, 0, s>>>(B, P, run)
    switch (P.link_stage * 4 + (tile == 128 ? 0 : tile == 512 ? 2 : 1)) {
      case 8: TPCCA_LINKS(2, 128); break;
      case 9: TPCCA_LINKS(2, 256); break;
      case 10: TPCCA_LINKS(2, 512); break;
      case 4: TPCCA_LINKS(1, 128); break;
      case 5: TPCCA_LINKS(1, 256); break;
      case 6: TPCCA_LINKS(1, 512); break;
      case 0: TPCCA_LINKS(0, 128); break;
      case 2: TPCCA_LINKS(0, 512); break;
      default: TPCCA_LINKS(0, 256); break;
    }
#undef TPCCA_LINKS
  }
  return hipGetLastError();
}

hipError_t launch_clean(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                        hipStream_t s) {
  (void)P;
  const int nch = h.c1 - h.c0;
  if (nch > 0) {
    k_clean<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run);
    k_scan_tiles<<<1, 1024, 0, s>>>(B.scan_tmp, nch);
    k_starts_compact<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run);
  }
  return hipGetLastError();
}

hipError_t launch_chains(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                         hipStream_t s) {
  const int nch = h.c1 - h.c0, nu = h.u1 - h.u0;
  hipError_t e = launch_fill_i32(B.flag + h.cl0, h.cl1 - h.cl0, 0, s);
  if (e != hipSuccess) return e;
  // sval is a byte array: clear it as 32-bit words (its range is padded)
  e = launch_fill_i32(reinterpret_cast<int32_t *>(B.sval + (h.cl0 & ~3)),
                      ((int64_t)h.cl1 - (h.cl0 & ~3) + 3) / 4, 0, s);
  if (e != hipSuccess) return e;
  if (nch > 0) {
    k_chain<<<grid_for(h.cl1 - h.cl0, kBlock, 4096), kBlock, 0, s>>>(B, P, run);
    k_flag_sums<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run);
    k_scan_tiles<<<1, 1024, 0, s>>>(B.scan_tmp, nch);
    k_flag_apply<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run);
    if (P.kf_rows <= 0) {  // the row-synchronous fit orders its tracklets itself (below)
    k_order_sums<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run);
    k_scan_tiles<<<1, 1024, 0, s>>>(B.scan_tmp, 2 * (int64_t)nch);
    const bool bands = P.kf_bands > 0 && h.trk_cap > 0;
    k_order_apply<<<grid_for(nch, 1, 8192), kBlock, 0, s>>>(B, run, bands ? B.kf_tmp : B.kf_order);
    if (bands) {
      const int64_t nbk = (int64_t)nu * P.kf_bands;
      e = launch_fill_i32(B.band_tmp, nbk, 0, s);
      if (e != hipSuccess) return e;
      k_band_count<<<grid_for(h.trk_cap, kBlock, 4096), kBlock, 0, s>>>(B, P, run);
      k_band_scan<<<1, 1024, 0, s>>>(B, P, run);
      k_band_apply<<<grid_for(h.trk_cap, kBlock, 4096), kBlock, 0, s>>>(B, P, run);
    }
    }
  }
  if (nu > 0) k_empty_units<<<grid_for(nu, 64, 1024), 64, 0, s>>>(B, run);
  if (P.kf_rows > 0) return launch_kf_order_rows(B, P, run, h, s);
  return hipGetLastError();
}

// Compute units and resident fit blocks per CU of the current device, for
// each register variant and block size; queried once per device (contexts
// on several host threads launch concurrently, hence the lock).
struct KfOccupancy {
  int cus = 1;
  int per[3][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}};  // [register variant][64, 128, 256 threads]
};

template <int kBlk>
static void kf_occ_row(int per[3]) {
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[0], k_kf<5, kBlk>, kBlk, 0);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[1], k_kf<4, kBlk>, kBlk, 0);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[2], k_kf<6, kBlk>, kBlk, 0);
}

static const KfOccupancy &kf_occupancy() {
  static std::mutex mu;
  static std::map<int, KfOccupancy> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  KfOccupancy o;
  int cus = 0, per[3][3] = {};
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  kf_occ_row<64>(per[0]);
  kf_occ_row<128>(per[1]);
  kf_occ_row<256>(per[2]);
  o.cus = std::max(1, cus);
  for (int v = 0; v < 3; ++v)
    for (int b = 0; b < 3; ++b) o.per[v][b] = std::max(1, per[b][v]);
  return cache.emplace(dev, o).first->second;
}

hipError_t launch_kf(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s) {
  // persistent: exactly the resident capacity of the chip, work taken from a
  // counter
  // register budgets: 5 (default), 4 or 6 resident waves per SIMD; block
  // sizes 64, 128 (default) or 256 threads
  const int v = P.kf_min_waves >= 6 ? 2 : P.kf_min_waves == 4 ? 1 : 0;
  const int blk = kf_block_of(P);
  const int bi = blk == 64 ? 0 : blk == 256 ? 2 : 1;
  const KfOccupancy &o = kf_occupancy();
  const int cus = o.cus;
  const int bpc = P.kf_blocks_per_cu > 0 ? std::min(P.kf_blocks_per_cu, o.per[v][bi]) : o.per[v][bi];
  const int g = grid_for(h.trk_cap, blk, cus * bpc);
  // the claim words of the selection start at zero (the fit may write them
  // as its tracklets end)
  hipError_t e = launch_fill_u64(B.owner + h.cl0, h.cl1 - h.cl0, 0ull, s);
  if (e != hipSuccess) return e;
  if (P.kf_rows > 0) return launch_kf_rows(B, P, run, h, s);
  if (h.trk_cap > 0) {
#define TPCCA_KF(W, T) k_kf<W, T><<<g, T, 0, s>>>(B, P, run)
    switch (v * 3 + bi) {
      case 0: TPCCA_KF(5, 64); break;
      case 2: TPCCA_KF(5, 256); break;
      case 3: TPCCA_KF(4, 64); break;
      case 4: TPCCA_KF(4, 128); break;
      case 5: TPCCA_KF(4, 256); break;
      case 6: TPCCA_KF(6, 64); break;
      case 7: TPCCA_KF(6, 128); break;
      case 8: TPCCA_KF(6, 256); break;
      default: TPCCA_KF(5, 128); break;
    }
#undef TPCCA_KF
  }
  return hipGetLastError();
}

hipError_t launch_select(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                         hipStream_t s) {
  const int64_t n = h.cl1 - h.cl0;
  hipError_t e = launch_fill_i32(B.assign + h.cl0, n, -1, s);
  if (e != hipSuccess) return e;
  const int nu = h.u1 - h.u0;
  const int tg = grid_for((int64_t)h.trk_cap, kBlock, 8192);  // thread per tracklet (claims)
  const int gg = grid_for((int64_t)h.trk_cap * kGrp, kBlock, 8192);  // lane group per tracklet
  const int64_t tiles = (h.trk_cap + kScanTile - 1) / kScanTile;
  if (h.trk_cap > 0) {
    if (!P.kf_claims) k_claim<<<tg, kBlock, 0, s>>>(B, P, run);
    k_won<kWonGrp><<<gg, kBlock, 0, s>>>(B, P, run);
    k_acc_sums<<<grid_for(tiles, 1, 8192), kBlock, 0, s>>>(B, run);
  }
  k_acc_tiles<<<1, 1024, 0, s>>>(B, run);
  if (h.trk_cap > 0) k_acc_apply<<<grid_for(tiles, 1, 8192), kBlock, 0, s>>>(B, run);
  if (nu > 0) k_unit_results<<<grid_for(nu, 64, 1024), 64, 0, s>>>(B, run);
  if (h.trk_cap > 0) k_output<<<gg, kBlock, 0, s>>>(B, P, run);
  return hipGetLastError();
}

hipError_t launch_links_by_id(const Bufs &B, const int32_t *up, const int32_t *dn, int32_t *out_up,
                              int32_t *out_dn, int32_t cl_begin, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_links_by_id<<<grid_for(n, 256, 4096), 256, 0, s>>>(B.sid, up, dn, out_up, out_dn, cl_begin, n);
  return hipGetLastError();
}

hipError_t launch_to_ids(const Bufs &B, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_to_ids<<<grid_for(n, 256, 4096), 256, 0, s>>>(B.sid, in, out, n);
  return hipGetLastError();
}

}  // namespace tpcca
