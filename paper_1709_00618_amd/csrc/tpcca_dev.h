// Wave and block primitives of the gfx950 kernels (GPU library internal).
#pragma once
#include <hip/hip_runtime.h>

namespace tpcca {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

}  // namespace tpcca
