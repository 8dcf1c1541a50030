// Internal layout shared by the gfx950 kernels and the host runtime of the
// GPU library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpcca.h"

namespace tpcca {

constexpr int kMaxRows = 255;
constexpr int kChunk = 1024;        // clusters per chunk (block work unit)
constexpr int kBlock = 256;         // threads per block of the cluster kernels
constexpr int kScanTile = 2048;     // elements per tile of the device scans
constexpr int kKfBlock = 128;       // threads per block of the Kalman filter
constexpr int kXcds = 8;            // XCDs of the chip (blocks are dealt round-robin)

// One (slot, sector) unit.  Work arrays are indexed by global cluster index:
// the unit owns [cl_begin, cl_begin + n) of every per-cluster array.
struct UnitDev {
  const float4 *cl;      // input clusters (device address)
  const uint8_t *row;    // input pad rows (device address)
  int64_t bin_base;      // first entry of the unit's bin-begin table
  int32_t cl_begin;
  int32_t n;
  int32_t trk_base;      // first tracklet slot reserved for the unit
  int32_t slot, sector;
  int32_t tile_base;     // first row tile slot reserved for the unit
};

constexpr int kTile = 256;     // hits of one row per neighbour-finding tile (default)
constexpr int kTileMin = 128;  // smallest tile the schedule may ask for (tile table capacity)
constexpr int kMaxBinsRow = 8192;  // z bins per row (the row sort keeps them in LDS)

// A chunk of <= kChunk consecutive clusters of one unit.
struct Chunk {
  int32_t unit;
  int32_t begin;  // unit-local
  int32_t count;
  int32_t pad_;
};

// Per (unit, row) grid description; row n_rows is the dump row of invalid
// clusters.  Bins split the row in z; entries bin0 .. bin0 + nb hold the
// sorted index where each bin starts (the last one is the row's end).
struct RowTab {
  int32_t begin;  // global sorted index of the row's first hit
  int32_t count;
  int32_t nb;
  int32_t bin0;   // first bin-begin entry of the row (the bin table has < 2^31 entries)
  float z0, inv;  // bin(z) = clamp(floor((z - z0) * inv), 0, nb - 1)
  int32_t pad_[2];
};

// Everything one launch needs to know about the units it processes.  The
// host writes the static part; the device fills the counters.
struct RunDev {
  int32_t u0, u1;       // units [u0, u1)
  int32_t c0, c1;       // chunks [c0, c1)
  int32_t cl0, cl1;     // global clusters [cl0, cl1)
  int64_t bin0, bin1;   // bin-begin entries [bin0, bin1)
  int32_t trk0;         // first tracklet slot of the run
  int32_t trk_cap;      // tracklet slots reserved for the run
  int32_t tile0, tile1; // row tile slots [tile0, tile1)
  // device-written
  int32_t n_trk;
  int32_t n_acc;
  int64_t n_acc_hits;
  int32_t err;          // 1: invalid cluster seen; 2: inconsistent fit order (internal)
  int32_t kf_next[8];   // work counters of the fit kernel, one per slice of the order
  int32_t n_starts;     // chain start hits found by the cleaning kernel
  unsigned long long kf_steps;   // row steps of the fit (propagations)
  unsigned long long kf_cands;   // candidate hits examined by the fit's searches
  unsigned long long kf_tests;   // chi2 tests of searched hits
  unsigned long long kf_updates; // Kalman updates
  unsigned long long kf_iters;   // state-machine iterations summed over the fit's waves
  // fit timeline on the 100 MHz constant clock: first wave start, first wave
  // to find the work counter exhausted, last wave end
  unsigned long long kf_t_start, kf_t_drain, kf_t_end;
};

// Device-side parameters (FP32 copies of tpcca_params_t).
struct ParamsDev {
  int32_t n_rows;
  float wy, wz, link_chi2;
  int32_t min_chain;
  float kB, ery, erz, max_sin, c22, c33, c44, r00, r11, nsig, wmax, pick_chi2;
  int32_t max_miss, min_hits, own_pct;
  float inflate;
  int32_t hits_per_bin;
  // schedule (no effect on results)
  int32_t kf_pool;
  int32_t kf_blocks_per_cu;
  int32_t link_blocks_per_cu;
  int32_t kf_min_waves;
  int32_t kf_claims;   // 1: the fit writes the selection's claims, 0: a kernel of its own
  int32_t kf_xcd;      // 1: the fit's order is cut into one slice per XCD
  int32_t link_stage;  // staging capacity variant of the neighbour kernel (0..2)
  int32_t kf_split;    // chains of at least this many hits are fitted first (0: off)
  int32_t kf_bands;    // fit order by (start-row band, unit) with this many bands (0: unit-major)
  int32_t kf_tail;     // with bands: only the last this many units are reordered (0: all)
  int32_t kf_rows;     // row-synchronous fit with chunks of at most this many tracklets (0: per-lane fit)
  int32_t link_tile;   // hits per neighbour-finding tile (128, 256 or 512)
  int32_t kf_block;    // threads per block of the per-lane fit (64, 128 or 256)
};

// Schedule knobs with defaults (0 in the tuning means the default).
__host__ __device__ inline int link_tile_of(const ParamsDev &P) { return P.link_tile > 0 ? P.link_tile : kTile; }
__host__ __device__ inline int kf_block_of(const ParamsDev &P) { return P.kf_block > 0 ? P.kf_block : kKfBlock; }

// Hit slots per tracklet: n_rows rounded up to whole 32-B groups, so that
// every tracklet's slots start 32-B aligned and move eight at a time.
constexpr int kSlotGrp = 8;
__host__ __device__ inline int slot_stride(int R) { return (R + kSlotGrp - 1) & ~(kSlotGrp - 1); }

// Device buffers of a context (all indices global).
struct Bufs {
  const float *row_x;
  UnitDev *units;
  Chunk *chunks;
  RunDev *runs;
  RowTab *rowtab;        // units x (n_rows + 1)
  int32_t *row_cnt;      // units x (n_rows + 1)
  int32_t *row_fill;     // units x (n_rows + 1): reservation cursors of the row scatter
  int32_t *chunk_hist;   // chunks x (n_rows + 1): clusters of each chunk per row (count pass)
  int4 *rtmp;            // row-grouped staging records (y, z, id, row) by global index
  int32_t *zmm;          // units x 2 (ordered-int min, max)
  int32_t *binbeg;       // bins
  float2 *yz;            // sorted hits
  int32_t *sid;          // sorted -> unit-local cluster ID
  uint8_t *srow;         // sorted -> pad row
  int2 *cinfo;           // sorted start hit -> (last hit, chain length)
  int32_t *up, *dn;      // raw links (sorted indices)
  int32_t *upc, *dnc;    // cleaned links
  int32_t *flag;         // by global cluster index: start sorted index + 1, or 0
  int2 *starts;          // chain start hits of a run: (sorted index, flag index)
  int4 *tiles;           // (unit, row, first sorted hit, count) row tiles
  uint8_t *sval;         // sorted: 1 if the hit starts a tracklet
  int32_t *tofg;         // sorted start hit -> tracklet
  int32_t *kf_order;     // processing rank -> tracklet (grid order of start hits)
  int32_t *kf_tmp;       // the unit-major order while start-row bands reorder it
  int32_t *band_tmp;     // 3 x units x (n_rows + 1): band counts, band-major and unit-major offsets
  int32_t *trk_start;    // tracklet -> sorted index of its start hit
  int32_t *trk_unit;     // tracklet -> unit
  int32_t *unit_tbegin;  // unit -> first tracklet
  tpcca_tracklet_t *trk; // tracklet fits
  int32_t *trk_hits;     // tracklet x slot_stride(n_rows) hit slots
  unsigned long long *owner;  // by sorted index
  unsigned long long *accv;   // by tracklet: accepted << 40 | won hits
  unsigned long long *wonmask;  // by tracklet: 4 x 64 bits, slot k won its hit (the row-synchronous
                                // fit's seed records before the selection)
  unsigned long long *accx;   // exclusive scan of accv (+ total)
  tpcca_track_t *tracks;      // by tracklet slot of the run (compacted)
  int32_t *hits_out;          // by global cluster index (compacted per run)
  int32_t *assign;            // by global cluster index
  tpcca_unit_result_t *unit_res;
  int64_t *scan_tmp;          // tile sums
  int32_t *ids_tmp;           // translation scratch
  // row-synchronous fit: (bucket, rank) per tracklet, bucket counts, chunks
  // (unit, first position in the run's order, count, -)
  int2 *zo_tmp;
  int64_t *zo_cnt;
  int4 *kf_chunks;
};

}  // namespace tpcca
