// Host-side launchers of the gfx950 kernels (GPU library internal).
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca_internal.h"

namespace tpcca {

// Static description of a run as the host knows it (grid sizing).
struct RunHost {
  int32_t u0, u1, c0, c1, cl0, cl1;
  int64_t bin0, bin1;
  int32_t trk0, trk_cap;
  int32_t tile0, tile1;
  int32_t dense;  // mean pad-row occupancy of the batch's units >= 1024 (row sort variant)
};

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_grid(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
hipError_t launch_links(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
hipError_t launch_clean(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
hipError_t launch_chains(const Bufs &B, const ParamsDev &P, int run, const RunHost &h,
                         hipStream_t s);
hipError_t launch_kf(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
// Row-synchronous fit (tpcca_fit_rows.hip): its processing order and chunks
// (called by launch_chains), the fit itself (called by launch_kf).
hipError_t launch_kf_order_rows(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
hipError_t launch_kf_rows(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
// Exclusive scan of n int64 values in place (one block); sums[n] = total.
hipError_t launch_scan_tiles(int64_t *sums, int64_t n, hipStream_t s);
hipError_t launch_select(const Bufs &B, const ParamsDev &P, int run, const RunHost &h, hipStream_t s);
hipError_t launch_links_by_id(const Bufs &B, const int32_t *up, const int32_t *dn, int32_t *out_up,
                              int32_t *out_dn, int32_t cl_begin, int32_t n, hipStream_t s);
hipError_t launch_to_ids(const Bufs &B, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);

}  // namespace tpcca
