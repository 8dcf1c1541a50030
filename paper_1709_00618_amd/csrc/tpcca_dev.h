// Wave and block primitives of the gfx950 kernels (GPU library internal).
#pragma once
#include <hip/hip_runtime.h>

namespace tpcca {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Minimum and maximum over the 64 lanes of a wave (all lanes active),
// returned to every lane, through data-parallel-primitive moves instead of
// LDS permutes: shifts by 1, 2, 4 and 8 within each row of 16 lanes leave
// the row's extreme in its lane 15, two row broadcasts carry it to lane 63.
// A lane whose source lies outside its row, or a row the mask leaves out,
// receives the identity.
__device__ __forceinline__ int wave_min_dpp(int v) {
  constexpr int id = 0x7FFFFFFF;
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_dpp(int v) {
  constexpr int id = (int)0x80000000;
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024,
// multiple of 64).  Returns the exclusive prefix; *total gets the sum.
template <typename T>
__device__ T block_exclusive_scan(T v, T *lds /* >= 16 */, T *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    T n = __shfl_up(incl, o, 64);
    if (lane >= o) incl += n;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < nw; ++w) {
      T t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[nw] = run;
  }
  __syncthreads();
  T res = incl - v + lds[wid];
  if (total) *total = lds[nw];
  __syncthreads();
  return res;
}

// The block's contiguous piece [x, y) of a run-ordered list [0, n) (start
// hits, tracklets, blocks of track hits): the list is cut into one slice per
// XCD (block b runs on XCD b mod 8) and each block of a slice takes a
// contiguous piece of it, so that the blocks resident on an XCD work on
// neighbouring items (one or two sectors at a time, whose links, owner words
// or clusters are then shared in that XCD's L2) instead of strides spread
// over the whole run.  The pieces partition [0, n) for any grid size.  (The
// cleaning and row-scatter passes measured no gain from it: their accesses
// are local already.)
template <typename I>
__device__ __forceinline__ void order_range(I n, I &lo, I &hi) {
  const int nb = (int)gridDim.x;
  const int nsl = nb < 8 ? nb : 8;  // the chip's eight XCDs
  const int x = (int)blockIdx.x % nsl, j = (int)blockIdx.x / nsl;
  const int nbx = (nb - x + nsl - 1) / nsl;  // blocks of slice x
  const I s0 = (I)((int64_t)n * x / nsl), s1 = (I)((int64_t)n * (x + 1) / nsl);
  const I per = (s1 - s0 + nbx - 1) / nbx;
  const int64_t l = (int64_t)s0 + (int64_t)j * per;
  lo = l < (int64_t)s1 ? (I)l : s1;
  hi = lo + per < s1 ? lo + per : s1;
}
__device__ __forceinline__ int2 order_piece(int n) {
  int lo, hi;
  order_range(n, lo, hi);
  return make_int2(lo, hi);
}

}  // namespace tpcca
