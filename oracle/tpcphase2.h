/*
 * tpcphase2: plain CPU oracle of the steps that follow the sector tracker
 * (TEST INFRASTRUCTURE: only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; it shares no code with the GPU
 * library).
 *
 * Rohr, "Tracking performance in high multiplicities environment at ALICE"
 * (LHCP 2017):
 *   - Sec. 2, second phase: the track segments found in the individual
 *     sectors are merged into final tracks, which are refitted;
 *   - Sec. 5: in continuous read-out the drift time cannot be turned into z
 *     before the vertex time is known, so tracks are found in the time
 *     coordinate, the vertices estimated from them, and only then z
 *     computed;
 *   - Sec. 3: track-model compression stores, for clusters attached to
 *     tracks, the residual of the cluster to the refitted track in the
 *     stored (integer) coordinates, so that decompression, running the same
 *     fit, is exact; and clusters of tracks below 50 MeV, of further legs of
 *     looping tracks and of highly inclined segments are marked for removal.
 * The paper states these steps in prose; every cut and formula is a reading
 * written out in tpcphase2.cpp next to the code that applies it.
 *
 * Precision: 32 or 64 as in tpcref.h.  All cluster IDs are positions inside
 * one sector's input array.
 */
#ifndef TPCPHASE2_H
#define TPCPHASE2_H
#include <stdint.h>

#include "tpcref.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float sector_cos, sector_sin; /* cos and sin of the 20-degree sector width (FP64, rounded once) */
  float max_sinphi;      /* propagations and rotations of this phase fail beyond |sin phi| */
  float merge_dz_ends;   /* facing segment ends more than this apart in z are never paired (cm) */
  int32_t merge_max_gap; /* B's innermost won row - A's outermost won row must lie in [1, this] */
  float merge_wy, merge_wz; /* |dy|, |dz| windows of a pair at B's plane (cm) */
  float merge_chi2;      /* max chi^2 of the 5-parameter difference of a pair */
  float refit_inflate;   /* the refit starts from the outer end's covariance times this */
  int32_t dca_steps;     /* equal steps of the extrapolation to the plane x = 0 */
  float vdrift;          /* drift velocity, cm/us */
  float vtx_gap_us;      /* sorted t0 estimates closer than this join one vertex */
  int32_t vtx_min_tracks;/* a vertex needs at least this many tracks */
  int32_t vtx_min_hits;  /* tracks with fewer hits take no part in finding vertices */
  float vtx_attach_us;   /* a track joins the nearest vertex within this time (us) */
  float cmp_qy, cmp_qz;  /* quantisation steps of the stored cluster coordinates (cm) */
  float cmp_c22, cmp_c33, cmp_c44; /* start variances of sin phi, tan lambda, q/pT of the
                                      compression fit */
  float rej_qpt;         /* |q/pT| above this (pT < 50 MeV) marks a track's clusters */
  float rej_looper_qpt;  /* |q/pT| above this: the track turns back inside the TPC */
  float rej_sinphi;      /* local |sin phi| above this marks a cluster (high inclination) */
} tpcref_p2params_t;

void tpcref_p2params_default(tpcref_p2params_t *q);

/* A segment: an accepted sector track of one slot (event or time frame). */
typedef struct {
  int32_t sector;
  int32_t start_id;    /* tie-break key together with the sector */
  int32_t n_hits;      /* won hits (hit list below, ascending rows) */
  int32_t pad_;
  double x_ref;        /* plane of p, cov (the tracklet's innermost hit row) */
  double p[5];         /* y, z (absolute), sin phi, tan lambda, q/pT */
  double cov[15];
} tpcref_segment_t;

/* A final track of the second phase (state at its innermost hit, in the
   frame of its innermost segment's sector). */
typedef struct {
  int32_t status;      /* 0 refitted, 2 numerical failure of the refit */
  int32_t n_seg;       /* segments merged */
  int32_t seg_begin;   /* first entry in the segment-order list */
  int32_t sector;      /* sector of the innermost segment (frame of p, cov) */
  int32_t n_hits, ndf, row_ref;
  int32_t vertex;      /* nearest vertex within vtx_attach_us (Sec. 5), or -1 */
  double x_ref, chi2;
  double p[5];
  double cov[15];
  double z0;           /* z at the plane x = 0 (time coordinate of the input) */
  double t0;           /* vertex-time estimate of this track (us) */
  int32_t z0_ok;       /* 1 if the extrapolation to x = 0 succeeded */
  int32_t pad_;
  double z_conv;       /* p[1] converted with the vertex time (p[1] if no vertex) */
} tpcref_final_t;

typedef struct {
  double t0;           /* lower median of the members' t0 estimates (us) */
  int32_t n_tracks;
  int32_t first;       /* first member in t0 order */
} tpcref_vertex_t;

/*
 * Second phase of one slot.  Inputs: the slot's clusters per sector
 * (cl / row concatenated, sector s owns [sec_begin[s], sec_begin[s+1]) ),
 * and its segments (any order) with their won hits (sector-local IDs,
 * ascending rows) concatenated at seg_hit_begin.  Returns an opaque result,
 * NULL on bad input.  brute != 0 pairs segments by testing every pair
 * instead of the z-sorted enumeration (same definition; for the pins).
 */
void *tpcref_phase2(const tpcref_params_t *p, const tpcref_p2params_t *q, const float *row_x,
                    int32_t n_sectors, const int64_t *sec_begin, const float *cl,
                    const uint8_t *row, int32_t n_seg, const tpcref_segment_t *seg,
                    const int64_t *seg_hit_begin, const int32_t *seg_hits, int32_t precision,
                    int32_t brute);
void tpcref_phase2_free(void *r);

int32_t tpcref_p2_n_final(const void *r);
int32_t tpcref_p2_n_vertices(const void *r);
int64_t tpcref_p2_n_final_hits(const void *r);
/* per segment: outer partner (next), inner partner (prev), final track */
void tpcref_p2_links(const void *r, int32_t *next, int32_t *prev, int32_t *final_of_seg);
/* final tracks in the order of their innermost segment in the input list;
   seg_order: segments of each final track, inner to outer (n_seg entries
   from seg_begin); hits: (sector << 24 | cluster ID), inner to outer. */
void tpcref_p2_finals(const void *r, tpcref_final_t *out, int32_t *seg_order, int64_t *hit_begin,
                      int32_t *hits);
void tpcref_p2_vertices(const void *r, tpcref_vertex_t *out);
/* per cluster of the slot (sec_begin indexing): rejection flags
   (1 low pT, 2 further looper leg, 4 high inclination) */
void tpcref_p2_flags(const void *r, uint8_t *flags);
/* outer-end states of the segments (for the pins): x, p, cov, ok */
void tpcref_p2_outer(const void *r, double *x, double *p, double *cov, int32_t *ok);
void tpcref_p2_stats(const void *r, int64_t *pair_tests, int64_t *near_ties, double *min_margin);

/*
 * Track-model compression (Sec. 3) of one sector's accepted tracks: for each
 * segment its record (first row, quantised first cluster, sin phi,
 * tan lambda, q/pT) and per further hit (row step, residual in y, in z).
 * rec: 6 int32 per segment (row0, yq0, zq0, bits(s), bits(t), bits(q/pT));
 * res: 3 int32 per hit (row step, ry, rz), hit 0 of each segment gets 0s.
 * The stored format is FP32 and so is the fit that defines it: precision
 * must be 32.
 */
int32_t tpcref_compress(const tpcref_params_t *p, const tpcref_p2params_t *q, const float *row_x,
                        const float *cl, const uint8_t *row, int32_t n_seg,
                        const tpcref_segment_t *seg, const int64_t *seg_hit_begin,
                        const int32_t *seg_hits, int32_t precision, int32_t *rec, int32_t *res);
/* The inverse: from rec and res, the quantised coordinates (yq, zq) and rows
   of every hit (hit order as in compression). */
int32_t tpcref_decompress(const tpcref_params_t *p, const tpcref_p2params_t *q,
                          const float *row_x, int32_t n_seg, const int32_t *n_hits,
                          const int32_t *rec, const int32_t *res, int32_t precision,
                          int32_t *yq, int32_t *zq, uint8_t *rows);

/* Single steps for the pins: rotate a state from the frame of a sector at
   angle alpha' to the frame at alpha = alpha' - delta (cs = cos delta,
   sn = sin delta); x in/out. */
int32_t tpcref_rotate(const tpcref_params_t *p, int32_t precision, double cs, double sn,
                      double *state, double *cov, double *x);
/* z at the plane x = 0 of a state at plane x whose z is relative to zr
   (the extrapolation of the second phase); -1 if the propagation fails. */
int32_t tpcref_z0(const tpcref_params_t *p, const tpcref_p2params_t *q, int32_t precision,
                  const double *state, double x, double zr, double *z0);
/* The vertex grouping alone, in FP32, on given t0 estimates and tie-break
   keys: group_of[i] = vertex index or -1; returns the number of vertices. */
int32_t tpcref_vertex_groups(int32_t n, const double *t0, const int64_t *key, double gap,
                             int32_t min_n, int32_t *group_of, tpcref_vertex_t *out);
/* chi^2 of a 5-parameter difference against the sum of two covariances */
int32_t tpcref_chi2_5(int32_t precision, const double *d, const double *c1, const double *c2,
                      double *chi2);

#ifdef __cplusplus
}
#endif
#endif
