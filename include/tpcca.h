/*
 * tpcca.h - C ABI of the MI355X (gfx950) TPC sector tracker.
 *
 * The library implements the first phase of the online TPC track finder of
 * Rohr, "Tracking performance in high multiplicities environment at ALICE"
 * (LHCP 2017), Sec. 2: per TPC sector, a Cellular Automaton forms links of
 * hits in adjacent pad rows that are nearly collinear (Fig. 1a) and
 * concatenates them into short track candidates (Fig. 1b); track following
 * fits every candidate with a simplified Kalman filter, extrapolates through
 * the sector and picks up further clusters (Fig. 1c); the last step selects
 * good tracks and assigns each cluster to at most one track.  The paper gives
 * the steps in prose; the cuts and formulas (the "readings") are fixed by the
 * parameters below and documented with the kernels.
 *
 * Units of work are (slot, sector) pairs: a slot is an event or a time frame,
 * a sector one of the 36 TPC sectors.  Several units are processed in one
 * launch per stage; Sec. 2 notes that even a central Pb-Pb event is too small
 * to fill a GPU, and Sec. 5 that time frames of continuous read-out will be
 * tracked as a whole.
 *
 * Conventions
 *   - Cluster IDs are positions 0..n-1 inside the unit's input array.
 *   - Coordinates are FP32 in the sector frame (cm); x must equal the pad
 *     row's radius row_x[row] (within 1e-3 cm).
 *   - Every call returns a status code (TPCCA_OK or a negative error).
 *   - A context is used by one host thread at a time; a server is thread-safe.
 *   - Work is queued on the context's HIP stream; results are only defined
 *     after tpcca_sync() (the get functions synchronise themselves).
 */
#ifndef TPCCA_H
#define TPCCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status --- */
#define TPCCA_OK 0
#define TPCCA_EINVAL (-1)    /* bad argument, row >= n_rows, |x - row_x| > 1e-3, non-finite */
#define TPCCA_ENOMEM (-2)    /* device budget exceeded */
#define TPCCA_ECAPACITY (-3) /* output buffer too small; *_out holds the size needed */
#define TPCCA_EDEVICE (-4)   /* HIP runtime error; text in tpcca_last_error() */
#define TPCCA_ESTATE (-5)    /* stage called out of order, or unit not loaded */
#define TPCCA_EBUSY (-6)     /* server queue full; retry later */
#define TPCCA_ENOTFOUND (-7) /* unknown request id */

/* where input pointers live */
#define TPCCA_MEM_HOST 0
#define TPCCA_MEM_DEVICE 1
/* run_batch option: replay the stage sequence as a captured HIP graph */
#define TPCCA_BATCH_GRAPH 2

/* ------------------------------------------------------------- types --- */
typedef struct {
  float x, y, z, q; /* sector frame (cm); q is carried, not used */
} tpcca_cluster_t;  /* 16 B */

typedef struct {
  int32_t n_sectors;  /* 36 */
  int32_t n_rows;     /* pad rows, 3..255 (159) */
  const float *row_x; /* host array of n_rows radii (cm), copied at create */
} tpcca_geometry_t;

/* Cuts and constants of the reading of Sec. 2; defaults from
   tpcca_params_default().  Field order is part of the ABI. */
typedef struct {
  int32_t n_rows;          /* must equal the geometry's n_rows */
  float link_wy, link_wz;  /* neighbour windows |dy|, |dz| <= W * row distance (2.0) */
  float link_chi2;         /* max straight-line deviation^2 of a link triplet (0.2 cm^2) */
  int32_t min_chain_hits;  /* shortest chain that seeds a tracklet (3) */
  float kB;                /* curvature per q/pT: -Bz * 0.299792458e-2 (Bz = 0.5 T) */
  float err2_y, err2_z;    /* cluster variances (0.01 cm^2) */
  float max_sinphi;        /* propagation fails beyond |sin phi| (0.95) */
  float seed_c22, seed_c33, seed_c44; /* seed variances of sin phi, tan lambda, q/pT */
  float reset_c00, reset_c11;         /* hard-restart variances (refit_inflate = 0) */
  float pick_nsig;         /* search window in predicted sigmas (3) */
  float pick_win_max;      /* cap of the search half-window (4 cm) */
  float pick_chi2;         /* accept a picked cluster if chi2 <= this (16) */
  int32_t max_miss;        /* stop following after this many empty rows (10) */
  int32_t min_track_hits;  /* minimum hits of a tracklet and won hits of a track (10) */
  int32_t own_frac_pct;    /* a track must win this percentage of its hits (90) */
  float refit_inflate;     /* pass-2 restart: pass-1 covariance x this (100); 0 = hard */
  int32_t grid_hits_per_bin; /* z-bin occupancy target of the row grid (1; tuning only) */
} tpcca_params_t;

/* An accepted track (FP32).  Parameters at plane x_ref (the innermost hit's
   row): y, z, sin phi, tan lambda, q/pT; cov is the lower triangle, row-major
   (00,10,11,20,21,22,30,...,44).  hit_offset indexes the unit's hit list
   returned with the tracks; n_hits counts the won (assigned) clusters. */
typedef struct {
  float x_ref;
  float p[5];
  float cov[15];
  float chi2;
  int32_t ndf;        /* 2 * (hits in the fit) - 5 */
  int32_t n_hits;
  int32_t hit_offset;
  int32_t sector;
  int32_t start_id;   /* cluster ID of the seeding chain's first hit */
} tpcca_track_t;      /* 108 B */

/* A fitted candidate before selection (parity and diagnostics). */
typedef struct {
  int32_t start_id, n_chain, status; /* status: 0 fitted, 1 < min_track_hits, 2 failure */
  int32_t n_hits, n_pass1, ndf, row_ref, row_out;
  float x_ref, chi2, x_out;
  float p[5];
  float cov[15];
  float p_out[5];     /* pass-1 state at the outermost hit */
  float cov_out[15];  /* pass-1 covariance there */
} tpcca_tracklet_t;

/* Per-unit summary of a processed batch. */
typedef struct {
  int32_t slot, sector, n_clusters, n_tracklets;
  int32_t n_tracks, n_track_hits;
  int64_t cluster_begin; /* unit's first cluster in the batch's assignment array */
  int64_t track_begin;   /* unit's first track in the batch's track array */
  int64_t hit_begin;     /* unit's first hit in the batch's hit array */
} tpcca_unit_result_t;

/* Many units in one call.  Unit u's clusters are cl[begin[u] .. begin[u]+n[u])
   and rows row[begin[u] ..]; cl/row are host or device pointers (flags). */
typedef struct {
  int32_t n_units;
  const int32_t *slot;   /* host arrays of n_units entries */
  const int32_t *sector;
  const int64_t *begin;
  const int32_t *n;
  const tpcca_cluster_t *cl;
  const uint8_t *row;
  int32_t flags;         /* TPCCA_MEM_HOST or TPCCA_MEM_DEVICE, | TPCCA_BATCH_GRAPH */
} tpcca_batch_t;

/* Device views of a processed batch (valid until the next load/reset). */
typedef struct {
  const tpcca_track_t *tracks; /* all units, in unit order */
  const int32_t *hits;         /* cluster IDs (unit-local) of the tracks' won hits */
  const int32_t *assignment;   /* per input cluster, unit-local track index or -1 */
  const tpcca_unit_result_t *units;
  int32_t n_units;
} tpcca_device_results_t;

typedef struct tpcca_ctx tpcca_ctx_t;

/* ----------------------------------------------------------- context --- */
void tpcca_params_default(tpcca_params_t *p);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to
   queue work on (e.g. torch.cuda.Stream().cuda_stream) or NULL for a
   context-owned stream.  device_budget_bytes caps the device memory the
   context allocates (0 = 64 GiB).  Errors: EINVAL, EDEVICE. */
int tpcca_create(const tpcca_geometry_t *geo, const tpcca_params_t *params, int device,
                 void *hip_stream, size_t device_budget_bytes, tpcca_ctx_t **out);
int tpcca_destroy(tpcca_ctx_t *ctx);

/* Forget every loaded unit (device memory is kept for reuse). */
int tpcca_reset(tpcca_ctx_t *ctx);

/* Append unit (slot, sector) with n clusters.  flags = TPCCA_MEM_HOST: the
   clusters are copied (asynchronously from a pinned staging buffer) and the
   caller may reuse its buffers on return.  TPCCA_MEM_DEVICE: the pointers are
   device addresses read in place; they must stay valid until tpcca_sync().
   Validation of rows and coordinates happens on the device; a bad cluster
   makes the next stage call's tpcca_sync() return EINVAL.  A (slot, sector)
   may be loaded once per reset.  A unit holds at most 2^24 - 1 clusters (hit
   slots keep a unit-local index in 24 bits); n beyond that is EINVAL and
   nothing is read.  Errors: EINVAL, ENOMEM, ESTATE. */
int tpcca_load_sector(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, const tpcca_cluster_t *cl,
                      const uint8_t *row, int32_t n, int32_t flags);

/* Stages (Sec. 2).  slot / sector = -1 select every loaded value; all
   selected units go through one launch per kernel.  Each stage requires the
   previous one on the same units (ESTATE otherwise). */
int tpcca_find_links(tpcca_ctx_t *ctx, int32_t slot, int32_t sector);      /* Fig. 1a */
int tpcca_clean_links(tpcca_ctx_t *ctx, int32_t slot, int32_t sector);     /* Fig. 1b */
int tpcca_build_tracklets(tpcca_ctx_t *ctx, int32_t slot, int32_t sector); /* Fig. 1c */
int tpcca_select_tracks(tpcca_ctx_t *ctx, int32_t slot, int32_t sector);   /* selection */

/* Wait for queued work; report deferred device-side validation errors. */
int tpcca_sync(tpcca_ctx_t *ctx);

/* Links of one unit in cluster-ID space (-1 = none).  which = 0: as found,
   1: after cleaning.  n must equal the unit's cluster count. */
int tpcca_get_links(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, int32_t which, int32_t *up,
                    int32_t *down, int32_t n);

/* Tracklets of one unit in ascending start_id; hits (cluster IDs, ascending
   rows) concatenated, hit_begin has n+1 entries.  ECAPACITY with the needed
   sizes in *n_out / *n_hits_out when cap or hits_cap is too small. */
int tpcca_get_tracklets(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, tpcca_tracklet_t *out,
                        int32_t cap, int32_t *n_out, int64_t *hit_begin, int32_t *hits,
                        int64_t hits_cap, int64_t *n_hits_out);

/* Accepted tracks of one unit (ascending start_id) and their won hits. */
int tpcca_get_tracks(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, tpcca_track_t *out,
                     int32_t cap, int32_t *n_out, int32_t *hits, int64_t hits_cap,
                     int64_t *n_hits_out);

/* Per cluster ID: index into the unit's track list, or -1. */
int tpcca_get_assignment(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, int32_t *track_of_cluster,
                         int32_t n);

/* Reset, load every unit of the batch and run all stages on all of them in
   one launch per kernel (TPCCA_BATCH_GRAPH: as a replayed HIP graph of
   persistent kernels whose work counts live in device memory).  Does not
   synchronise.  Errors: EINVAL, ENOMEM, EDEVICE. */
int tpcca_run_batch(tpcca_ctx_t *ctx, const tpcca_batch_t *batch);

/* Copy the whole batch's results to the host: units (n_units entries),
   tracks, hits and assignment (total clusters).  Any pointer may be NULL. */
int tpcca_get_batch_results(tpcca_ctx_t *ctx, tpcca_unit_result_t *units, tpcca_track_t *tracks,
                            int64_t tracks_cap, int32_t *hits, int64_t hits_cap,
                            int32_t *assignment, int64_t n_clusters);
int tpcca_batch_totals(tpcca_ctx_t *ctx, int32_t *n_units, int64_t *n_clusters, int64_t *n_tracks,
                       int64_t *n_hits);
/* Work counters of everything processed since the last reset (synchronises):
   clusters, tracklets (fitted candidates), accepted tracks and their hits,
   Kalman row steps (propagations), candidate clusters examined by the
   track-following searches, chi2 tests of the hits those searches picked,
   Kalman updates, the fit kernel's loop iterations summed over its 64-lane
   waves (fit_steps / (64 x fit_wave_iterations) is its lane use), and, from
   the GPU's constant clock, the fit kernel's span and the part of it after
   the first wave found no more tracklets to start (the drain), in ns, summed
   over runs; and the batches since the context was created that ran without
   their graph because its capture failed (TPCCA_BATCH_GRAPH falls back to
   plain launches; results are the same). */
typedef struct {
  int64_t clusters, tracklets, tracks, track_hits, fit_steps, fit_candidates, fit_tests, fit_updates,
      fit_wave_iterations, fit_ns, fit_drain_ns, graph_fallbacks;
} tpcca_work_stats_t;
int tpcca_work_stats(tpcca_ctx_t *ctx, tpcca_work_stats_t *out);

/* Device pointers to the batch results (no copy; synchronises). */
int tpcca_device_results(tpcca_ctx_t *ctx, tpcca_device_results_t *out);

/* For callers that cannot allocate device memory (serving loops and
   harnesses that forbid hipMalloc, code that must not synchronise the
   device through the allocator): tpcca_run_batch on device-resident inputs
   without a context and without any allocation.  Every work buffer and the
   run tables live in one fixed device array of TPCCA_NOALLOC_SCRATCH_BYTES
   that the library holds on each device it runs on until the process ends
   (about 390 B per cluster: up to roughly 1.6e5 clusters, e.g. five sectors
   of a central Pb-Pb event).  The caller owns inputs and outputs:
     bt          units as for tpcca_run_batch; flags must be TPCCA_MEM_DEVICE
                 (cl/row are device addresses; TPCCA_BATCH_GRAPH is EINVAL);
     tracks      device array of tracks_cap >= sum over units of
                 (n / min_chain_hits + 1) entries (worst-case capacity; the
                 accepted tracks come first, in unit order);
     hits        device array of hits_cap >= total clusters (won hits);
     assignment  device array of n_assignment >= total clusters;
     units       device array of n_units tpcca_unit_result_t;
   with the layout of tpcca_device_results.  *n_tracks_out / *n_hits_out
   (host, may be NULL) receive the totals.  The call queues the stages on
   hip_stream (NULL: the null stream) of `device` and returns when they are
   done.  Errors: EINVAL (bad arguments, or an invalid cluster, as the sync
   of tpcca_run_batch reports it), ECAPACITY (an output too small), ENOMEM
   (the units need more than TPCCA_NOALLOC_SCRATCH_BYTES), EDEVICE.  Calls
   for one device are serialised by the library; the array keeps the last
   call's contents, and every buffer that must start cleared is cleared by
   the stages themselves. */
#define TPCCA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tpcca_run_batch_noalloc(const tpcca_geometry_t *geo, const tpcca_params_t *params, int device,
                            void *hip_stream, const tpcca_batch_t *bt, tpcca_track_t *tracks,
                            int64_t tracks_cap, int32_t *hits, int64_t hits_cap, int32_t *assignment,
                            int64_t n_assignment, tpcca_unit_result_t *units, int64_t *n_tracks_out,
                            int64_t *n_hits_out);

/* Launch schedule knobs.  None of them changes any result (every decision
   compares cluster IDs and the same operation sequence runs per tracklet);
   they only trade occupancy, load balance and grid granularity.  Picked by
   the autotuner (paper_1709_00618_amd/autotune.py); 0 = default. */
typedef struct {
  int32_t fit_pool;          /* tracklets a wave of the fit kernel claims at once (64) */
  int32_t fit_blocks_per_cu; /* resident fit blocks per CU (0: occupancy limit) */
  int32_t grid_hits_per_bin; /* z-bin occupancy of the row grid (1); applies after reset */
  int32_t link_blocks_per_cu;/* resident neighbour-finding blocks per CU (0: 32) */
  int32_t fit_min_waves;     /* register budget of the fit kernel in resident waves per SIMD:
                                0 (5), 4 or 6 (larger values act as 6) */
  int32_t fit_claims;        /* 1: the fit kernel writes the selection's claims as tracklets end
                                (default); 0: a claim kernel of its own */
  int32_t fit_xcd_slices;    /* 1: the fit's processing order is cut into one slice per XCD;
                                0: one shared work counter (default) */
  int32_t link_stage;        /* LDS staging capacity of the neighbour kernel: 0 default (1024
                                hits, 768 bins), 1 large (1536, 1024: fewer global fallbacks),
                                2 small (768, 512: less LDS per block); EINVAL outside 0..2 */
  int32_t fit_long_first;    /* tracklets whose chain has at least this many hits are fitted
                                first (shorter fits drain the end of the kernel); 0: off */
  int32_t fit_row_bands;     /* fit order by (start-row band, unit) with this many bands of
                                rows (1..n_rows; overrides fit_long_first); 0: by unit */
  int32_t fit_tail_units;    /* with fit_row_bands: only the last this many units of a run are
                                taken band by band, the others stay unit by unit; 0: all */
  int32_t fit_rows;          /* 0: per-lane fit (each lane at its own row); 64..1024: row-
                                synchronous fit, the lanes of a wave step through the rows
                                together over chunks of at most this many tracklets (ordered
                                by z), the rows' hits read once into LDS; EINVAL otherwise.
                                The order knobs above (long first, row bands, XCD slices, pool)
                                do not apply to it. */
  int32_t link_tile;         /* hits of one pad row per neighbour-finding block: 0 (256), 128,
                                256 or 512; set before loading units (ESTATE if it would change
                                the tile reservations of loaded units); EINVAL otherwise */
  int32_t fit_block;         /* threads per block of the per-lane fit: 0 (128), 64, 128 or 256;
                                EINVAL otherwise */
} tpcca_tuning_t;
int tpcca_set_tuning(tpcca_ctx_t *ctx, const tpcca_tuning_t *t);
/* The schedule a new context starts with (pool 64, claims in the fit,
   every other knob 0). */
void tpcca_tuning_default(tpcca_tuning_t *t);
int tpcca_get_tuning(tpcca_ctx_t *ctx, tpcca_tuning_t *t);

/* Error text of a status code, and the last HIP/runtime message of ctx. */
const char *tpcca_error_string(int status);
const char *tpcca_last_error(tpcca_ctx_t *ctx);

/* Stage timing of the last full stage sequence on ctx's stream, via HIP
   events (ms): 0 grid, 1 links (the neighbour kernel alone), 2 clean,
   3 chains (compaction), 4 Kalman fit (the fit kernel and the clearing of
   the claim words it writes), 5 selection.  With timing on, a graph run of
   tpcca_run_batch replays one graph per stage with the events between them
   on ctx's stream, so each replay times its own stages (the graphs are
   captured again when timing is switched).  Valid after tpcca_sync; returns
   the number of entries written (0 if timing was off). */
int tpcca_stage_times(tpcca_ctx_t *ctx, float *ms, int32_t cap);
/* Enable/disable per-stage event recording (off by default). */
int tpcca_set_timing(tpcca_ctx_t *ctx, int32_t enable);

/* ------------------------------------------------------ second phase --- */
/* The steps after the sector tracker, on the accepted tracks of every unit
   of a context ("segments"):
   - Sec. 2, second phase: the segments found in the individual sectors are
     merged into final tracks, which are refitted.  Reading: segment A (in
     sector s) and B (in the neighbouring sector s +- 1 of the same side and
     slot) are a candidate pair if B's first won row follows A's last by 1 to
     merge_max_gap rows and their facing ends lie within merge_dz_ends in z;
     B's inner state is rotated into A's frame, A's outer end (its fitted
     state propagated along its won hits) propagated to that plane, and the
     five-parameter difference must lie within the y, z windows and the
     chi^2 cut.  Mutual best partners (smallest chi^2, then (sector, index))
     merge; a final track is a chain of merged segments, refitted inward from
     the outermost segment's outer end (covariance x refit_inflate) through
     every won hit, the state rotated between sector frames.
   - Sec. 5, continuous read-out: the time of a vertex is known only after
     tracking, so tracking runs in the drift coordinate z' and each refitted
     track is extrapolated (dca_steps propagation steps) to the plane x = 0
     of its frame, which holds the beam axis, for z0 and a time estimate
     t0 = -z0 / v (A side), z0 / v (C side).  Sorted t0 of tracks with at
     least vtx_min_hits hits and |q/pT| <= rej_looper_qpt form vertices
     (estimates closer than vtx_gap_us chain; at least vtx_min_tracks; time
     = lower median); every track joins the nearest vertex within
     vtx_attach_us and gets z = z' + v t0 (A), z' - v t0 (C).
   - Sec. 3, compression: per segment, the first won cluster quantised
     (rint(y / cmp_qy), rint(z / cmp_qz)) and sin phi, tan lambda, q/pT as
     FP32; per further hit the row step and the residuals of the quantised
     cluster to the quantised prediction of an FP32 Kalman fit over the
     quantised values; decompression runs the same fit and is exact.
   - Sec. 3, rejection: flags per cluster of a final track: 1 |q/pT| >
     rej_qpt (pT < 50 MeV), 2 later leg of a looping track (|q/pT| >
     rej_looper_qpt and no vertex), 4 local |sin phi| > rej_sinphi.
   The phase's propagations and rotations fail beyond |sin phi| > max_sinphi.
   Defaults from tpcca_phase2_params_default(); field order is part of the
   ABI. */
typedef struct {
  float sector_cos, sector_sin; /* cos, sin of the 20-degree sector width */
  float max_sinphi;             /* 0.99 */
  float merge_dz_ends;          /* 40 cm */
  int32_t merge_max_gap;        /* 10 rows */
  float merge_wy, merge_wz;     /* 4 cm */
  float merge_chi2;             /* 50 */
  float refit_inflate;          /* 100 */
  int32_t dca_steps;            /* 16 */
  float vdrift;                 /* 2.58 cm/us */
  float vtx_gap_us;             /* 0.1 */
  int32_t vtx_min_tracks;       /* 3 */
  int32_t vtx_min_hits;         /* 20 */
  float vtx_attach_us;          /* 0.25 */
  float cmp_qy, cmp_qz;         /* 0.01 cm */
  float cmp_c22, cmp_c33, cmp_c44; /* 1e-4, 1e-4, 1 */
  float rej_qpt;                /* 20 c/GeV (50 MeV) */
  float rej_looper_qpt;         /* 5.4 c/GeV: the circle turns back inside 247 cm */
  float rej_sinphi;             /* 0.8 */
} tpcca_phase2_params_t;

/* A final track: state at its innermost hit in the frame of its innermost
   segment's sector. */
typedef struct {
  int32_t slot, sector;
  int32_t status;     /* 0 refitted, 2 numerical failure of the refit */
  int32_t n_seg, n_hits, ndf, row_ref;
  int32_t vertex;     /* index into the slot's vertices, or -1 */
  int32_t z0_ok;      /* 1 if the extrapolation to the axis succeeded */
  int32_t first_seg;  /* innermost segment: sector << 24 | index among its unit's tracks */
  int64_t hit_begin;  /* first entry in the hit list returned with the finals */
  float x_ref, chi2;
  float p[5];         /* y, z', sin phi, tan lambda, q/pT */
  float cov[15];
  float z0, t0;       /* z' at the axis, time estimate (us) */
  float z_conv;       /* p[1] converted with the vertex time (p[1] without vertex) */
  int32_t pad_;
} tpcca_final_t;      /* 152 B */

typedef struct {
  int32_t slot, n_tracks;
  int32_t first;      /* first member's position among the slot's sorted t0 estimates */
  float t0;           /* us */
} tpcca_vertex_t;

/* Device views of the phase's results (valid until the next load/reset). */
typedef struct {
  int32_t n_seg, n_final, n_vertices;
  int32_t pad_;
  int64_t n_final_hits;
  const tpcca_final_t *finals;  /* all slots, in the order of their innermost segment */
  const int32_t *final_hits;    /* sector << 24 | cluster ID */
  const tpcca_vertex_t *vertices; /* slot field = compact slot index */
  const uint8_t *flags;         /* per cluster, batch order (as the assignment) */
  const int32_t *rec;           /* 6 per segment */
  const int32_t *res;           /* 4 per hit (16-B aligned), at the hit's position in the track hit array */
  const int32_t *seg_n_hits;    /* per segment */
  const int64_t *seg_hit_begin; /* per segment: first hit in the track hit array */
} tpcca_phase2_view_t;

void tpcca_phase2_params_default(tpcca_phase2_params_t *q);
/* Parameters of the phase for ctx (copied). EINVAL on out-of-range values. */
int tpcca_set_phase2_params(tpcca_ctx_t *ctx, const tpcca_phase2_params_t *q);
/* Run the phase on every unit of ctx (all must have been selected; ESTATE
   otherwise).  Reads the units' inputs again: device inputs must still be
   valid.  Queues its kernels and waits once for the number of final tracks
   (to size the sort of the time estimates).  Errors: ESTATE, ENOMEM,
   EDEVICE. */
int tpcca_phase2(tpcca_ctx_t *ctx);
/* Final tracks of one slot (order of their innermost segment) with their
   hits (sector << 24 | cluster ID, inner to outer); ECAPACITY with the sizes. */
int tpcca_get_finals(tpcca_ctx_t *ctx, int32_t slot, tpcca_final_t *out, int32_t cap, int32_t *n_out,
                     int32_t *hits, int64_t hits_cap, int64_t *n_hits_out);
/* Per track of unit (slot, sector), n = its number of tracks: the merge
   partners (sector << 24 | index among that unit's tracks, -1 if none) and
   the index of its final track among the slot's finals. */
int tpcca_get_segment_links(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, int32_t *next,
                            int32_t *prev, int32_t *final_of, int32_t n);
int tpcca_get_vertices(tpcca_ctx_t *ctx, int32_t slot, tpcca_vertex_t *out, int32_t cap, int32_t *n_out);
/* Rejection flags of the unit's clusters (n = cluster count). */
int tpcca_get_flags(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, uint8_t *flags, int32_t n);
/* Compressed form of the unit's tracks (ascending start_id): 6 int32 per
   track (row, y and z step counts of the first won cluster, FP32 bits of
   sin phi, tan lambda, q/pT) and 4 int32 per won hit (row step, residual of
   y, of z, 0; zeros for the first); hits_cap counts hits. */
int tpcca_get_compressed(tpcca_ctx_t *ctx, int32_t slot, int32_t sector, int32_t *rec, int32_t seg_cap,
                         int32_t *res, int64_t hits_cap, int32_t *n_seg, int64_t *n_hits);
int tpcca_phase2_view(tpcca_ctx_t *ctx, tpcca_phase2_view_t *out);
/* Decompression (device pointers, queued on ctx's stream): n_seg records
   (6 int32), their hits' residuals (4 int32 per hit, 16-B aligned, hit_begin / n_hits per
   record) -> the quantised coordinates yq, zq and the rows of every hit, at
   the same positions.  Uses ctx's geometry and phase parameters.  EINVAL if
   res is not 16-B aligned. */
int tpcca_decompress(tpcca_ctx_t *ctx, int32_t n_seg, const int32_t *n_hits, const int64_t *hit_begin,
                     const int32_t *rec, const int32_t *res, int32_t *yq, int32_t *zq, uint8_t *rows);

/* ------------------------------------------------------------ server --- */
/* Continuous batching of time frames (Sec. 5: time frames are tracked as a
   whole; GPU memory is the limit, a frame larger than memory is sliced, here
   by sector).  Requests are admitted while their bytes fit the device
   budget; admitted units of all waiting frames are packed into batches that
   run on n_streams streams concurrently. */
typedef struct tpcca_server tpcca_server_t;

typedef struct {
  int32_t n_units;
  const int32_t *sector;        /* host arrays */
  const int64_t *begin;
  const int32_t *n;
  const tpcca_cluster_t *cl;    /* host memory; must stay valid until done */
  const uint8_t *row;
  /* outputs (host, caller-owned, valid until the request completes):
     tracks, hits: capacity-checked; assignment: sum(n) entries */
  tpcca_track_t *tracks;
  int64_t tracks_cap;
  int32_t *hits;
  int64_t hits_cap;
  int32_t *assignment;
  tpcca_unit_result_t *units;   /* n_units entries */
  double arrival_s;             /* caller's arrival stamp (steady clock, s); 0 = now */
} tpcca_timeframe_t;

typedef struct {
  int32_t status;       /* TPCCA_OK or error of this request */
  int32_t done;         /* 1 when complete */
  int64_t n_tracks, n_hits;
  double arrival_s, start_s, end_s; /* steady-clock seconds */
} tpcca_result_t;

typedef struct {
  int64_t submitted, completed, rejected, clusters_done, tracks_done;
  int64_t bytes_in_flight, bytes_budget;
  int32_t queue_depth, batches_run;
  double busy_s;        /* wall time with at least one batch in flight */
  double p50_ms, p99_ms, mean_ms; /* latency = end - arrival over completed requests */
} tpcca_stats_t;

/* A server on `device`: n_streams lanes (1..16), each a worker thread with
   its own context and an equal share of budget_bytes of device memory (0:
   64 GiB); at most max_queue (>= 1) frames wait for a lane.  The geometry
   and parameters are copied.  EINVAL on bad arguments, EDEVICE if the
   device cannot be selected; if a lane cannot create its context, the lanes
   are stopped and that lane's status (EDEVICE, ENOMEM) is returned.  Each
   lane launches on a stream of its own; HIP gives a process a few hardware
   queues (GPU_MAX_HW_QUEUES, 4 by default) and streams beyond them share a
   queue, so lanes whose streams share one run one after the other: keep
   the lanes plus the process's other busy streams within that number
   (three lanes measured best beside the default stream). */
int tpcca_server_create(const tpcca_geometry_t *geo, const tpcca_params_t *params, int device,
                        size_t budget_bytes, int32_t n_streams, int32_t max_queue,
                        tpcca_server_t **out);
/* Non-blocking; EBUSY when the queue is full, ENOMEM when one unit alone
   exceeds the budget, EINVAL on bad descriptors. */
int tpcca_server_submit(tpcca_server_t *srv, const tpcca_timeframe_t *tf, uint64_t *req_id);
/* Current state of a request (done flag, status, times); ENOTFOUND for an
   unknown or released id. */
int tpcca_server_poll(tpcca_server_t *srv, uint64_t req_id, tpcca_result_t *res);
/* Block until done or timeout_s elapses (returns EBUSY on timeout). */
int tpcca_server_wait(tpcca_server_t *srv, uint64_t req_id, double timeout_s, tpcca_result_t *res);
/* Forget a completed request's record. */
int tpcca_server_release(tpcca_server_t *srv, uint64_t req_id);
/* Counters since creation or the last reset, and latency percentiles over
   the requests completed in that time. */
int tpcca_server_stats(tpcca_server_t *srv, tpcca_stats_t *st);
/* Text of the last failed batch (lane, size, failing step and HIP error),
   "" if none; the pointer stays valid until the calling thread's next call. */
const char *tpcca_server_last_error(tpcca_server_t *srv);
int tpcca_server_reset_stats(tpcca_server_t *srv);
/* Launch schedule of every lane's context (tpcca_set_tuning), applied by
   each lane from its next batch on; results do not depend on it.  EINVAL
   for knobs out of range. */
int tpcca_server_set_tuning(tpcca_server_t *srv, const tpcca_tuning_t *t);
/* Stop accepting, finish in-flight work, free everything. */
int tpcca_server_destroy(tpcca_server_t *srv);

/* Seconds on the steady clock the server stamps with. */
double tpcca_now(void);

#ifdef __cplusplus
}
#endif
#endif /* TPCCA_H */
