// Second phase of the gfx950 tracker (GPU library internal): merging of the
// sector segments into final tracks and their refit (Rohr, LHCP 2017,
// Sec. 2), vertex times from the tracks (Sec. 5), track-model compression
// and the flags of clusters not used for physics (Sec. 3).
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca_internal.h"

namespace tpcca {

constexpr int kP2Tile = 2048;   // elements per tile of the phase's scans

// Device copy of tpcca_phase2_params_t.
struct P2Params {
  float cs, sn, max_sin, dz_ends;
  int32_t max_gap;
  float wy, wz, chi2, inflate;
  int32_t dca_steps;
  float vdrift, gap_us;
  int32_t vtx_min_tracks, vtx_min_hits;
  float attach_us, qy, qz, c22, c33, c44, rej_qpt, rej_looper, rej_sin;
};

// Per unit: compact slot index, sector, and the units of the neighbouring
// sectors of the same slot and side (-1 if not loaded).
struct P2Unit {
  int32_t slot, sector, prev, next;
};

// Outer end of a segment: its state propagated to its outermost won hit
// (z relative to the segment's inner z).
struct P2Out {
  float x;
  float p[5];
  float C[15];
  int32_t ok;
};

// Device-side counts of the phase.
struct P2Counts {
  int32_t n_seg, n_final, n_cand, n_group, n_vtx, n_slots;
  int64_t n_final_hits;
  int64_t n_pairs;               // candidate pairs of the merge
  int32_t seg_next, fin_next;    // work counters of the per-lane segment and refit kernels
  int32_t pad_[2];
};

struct P2Bufs {
  const P2Unit *units;
  int32_t n_units;
  int32_t *seg_begin;            // units + 1: first segment of each unit
  int32_t *seg_unit;             // per segment
  int32_t *seg_nh;               // per segment: won hits
  int64_t *seg_hb;               // per segment: first won hit in the track hit array
  int2 *seg_rows;                // (row of the first won hit, row of the last)
  float *seg_zin;                // absolute z of the inner state
  float *seg_zout;               // absolute z of the outer end
  P2Out *seg_out;
  int2 *zmm;                     // per unit: ordered-int min, max of seg_zin
  int32_t *unit_nz;              // per unit: z bins per row of its pairing grid
  int64_t *unit_bbase;           // per unit: first cell of its pairing grid
  int32_t *bin_cnt;              // cells of all units' grids (row-major per unit)
  int32_t *bin_beg;              // cell starts (unit-local offsets), one extra entry per unit
  int32_t *bin_seg;              // segments in bin order (unit u at seg_begin[u])
  int2 *bin_rz;                  // (first won row, bits of inner z) in bin order
  float4 *hrec;                  // per hit position: y, z, row and cluster ID (as bits)
  float4 *seg_flag;              // per segment: kB q/pT, x_ref, sin phi, final-track flags (bits)
  unsigned long long *best_b;    // per A: (chi2 bits << 32) | key of its best B
  unsigned long long *best_a;    // per B: (chi2 bits << 32) | key of its best A
  int32_t *next, *prev;          // merge links (segment indices)
  int32_t *final_of;             // per segment
  int32_t *seg_fpos;             // per segment: first position of its hits in its final's hit list
  int32_t *final_start;          // per final: innermost segment
  int32_t *final_nhits;
  int64_t *final_hbeg;           // per final: first entry in final_hits
  tpcca_final_t *finals;
  int32_t *final_hits;           // sector << 24 | cluster ID
  unsigned long long *vkey[2];   // vertex sort keys (slot << 32 | ordered t0)
  int32_t *vval[2];              // vertex sort values (final index)
  int32_t *gstart;               // per sorted candidate: group start flag, then group index
  int32_t *group_pos;            // per group: first sorted position
  tpcca_vertex_t *vertices;      // slot field holds the compact slot index
  int32_t *slot_first;           // per slot: first sorted candidate position
  int32_t *slot_vbeg, *slot_vend;// per slot: vertex range
  uint8_t *flags;                // per global cluster index
  int32_t *rec;                  // 6 per segment
  int32_t *res;                  // 4 per hit (global hit index of hits_out), 16-B aligned
  int32_t *order;                // processing order of the per-lane kernels (longest first)
  int32_t *len_hist, *len_cursor; // length-class counts and cursors of that order
  int64_t *scan_tmp;
  P2Counts *cnt;
};

hipError_t p2_launch_merge(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q,
                           int n_units, int64_t seg_cap, int64_t hit_span, hipStream_t s);
// the candidate pairs (after p2_launch_merge counted them), merge links,
// final tracks and their refit, vertex candidates
hipError_t p2_launch_pairs(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q, int64_t seg_cap,
                           int2 *pairs, int64_t n_pairs, hipStream_t s);
hipError_t p2_launch_vertices(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q,
                              int32_t n_final, int32_t n_cand, int32_t n_slots, void *sort_tmp,
                              size_t sort_tmp_bytes, hipStream_t s);
hipError_t p2_launch_finish(const Bufs &B, const P2Bufs &Q, const ParamsDev &P, const P2Params &q,
                            int32_t n_seg, int32_t n_final, int64_t n_clusters, hipStream_t s);
size_t p2_sort_tmp_bytes(int32_t n);
int64_t p2_grid_cells(int64_t seg_cap, int64_t n_units, int R);
hipError_t p2_launch_decompress(const ParamsDev &P, const P2Params &q, const float *row_x, int32_t n_seg,
                                const int32_t *n_hits, const int64_t *hit_begin, const int32_t *rec,
                                const int32_t *res, int32_t *yq, int32_t *zq, uint8_t *rows, hipStream_t s);

}  // namespace tpcca
