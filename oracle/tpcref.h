/*
 * tpcref: plain CPU oracle of the TPC sector tracker (TEST INFRASTRUCTURE).
 *
 * This library exists to check the GPU library.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never does.  It shares no code, header or table with the GPU library.
 *
 * It follows the sector tracker of Rohr, "Tracking performance in high
 * multiplicities environment at ALICE" (LHCP 2017), Sec. 2: a Cellular
 * Automaton links hits of adjacent rows that are nearly collinear with one
 * another and joins the links into short candidates (Fig. 1a, 1b); track following
 * fits each candidate with a simplified Kalman filter, extrapolates through
 * the sector and picks up clusters (Fig. 1c); finally good tracks are
 * selected and every cluster is assigned to at most one track.  The paper
 * states these steps in prose only, so every cut, formula and tie-break is a
 * reading; they are written out in tpcref.cpp next to the code that applies
 * them.  Propagation uses Bz only (Sec. 2 names the neglect of Bx, By).
 *
 * Precision: every routine runs in FP32 (precision = 32) or FP64 (64).
 * All cluster IDs are input positions 0..n-1 inside one sector.
 */
#ifndef TPCREF_H
#define TPCREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_rows;          /* pad rows (159) */
  float link_wy, link_wz;  /* neighbour window slope: |dy|, |dz| <= W * dx */
  float link_chi2;         /* max straight-line deviation^2 of a link triplet, cm^2 */
  int32_t min_chain_hits;  /* shortest chain that seeds a tracklet */
  float kB;                /* curvature per unit q/pT: -Bz * 0.299792458e-2 (1/cm per c/GeV) */
  float err2_y, err2_z;    /* cluster variance, cm^2 */
  float max_sinphi;        /* propagation fails beyond this |sin phi| */
  float seed_c22, seed_c33, seed_c44; /* initial variances of sin phi, tan lambda, q/pT */
  float reset_c00, reset_c11;         /* pass-2 restart variances of y, z */
  float pick_nsig;         /* search window in predicted sigmas */
  float pick_win_max;      /* cap of the search half-window, cm */
  float pick_chi2;         /* accept a picked cluster if its 2-D chi^2 is below */
  int32_t max_miss;        /* stop following after this many rows without a hit */
  int32_t min_track_hits;  /* minimum hits of a tracklet and won hits of a track */
  int32_t own_frac_pct;    /* a track must win this percentage of its hits */
  float refit_inflate;     /* > 0: pass 2 restarts from the pass-1 covariance times
                              this factor; 0: from diag(reset_c00, reset_c11, c22, c33, c44) */
} tpcref_params_t;

typedef struct {
  int32_t start_id;   /* input ID of the chain's first (innermost) hit */
  int32_t n_chain;    /* hits in the CA chain */
  int32_t status;     /* 0 fitted, 1 fewer than min_track_hits, 2 numerical failure */
  int32_t n_hits;     /* hits after following (pass 1 + inward extension) */
  int32_t n_pass1;    /* chain hits + hits picked up outward */
  int32_t ndf;        /* 2 n_hits - 5 */
  int32_t row_ref;    /* row of the innermost hit (where p, cov are given) */
  int32_t row_out;    /* row of the outermost hit */
  double x_ref, chi2, x_out;
  double p[5];        /* y, z, sin phi, tan lambda, q/pT at x_ref */
  double cov[15];     /* lower triangle, row-major: 00,10,11,20,21,22,30,...,44 */
  double p_out[5];    /* pass-1 state at the outermost hit (start of pass 2) */
  double cov_out[15]; /* pass-1 covariance there (before the pass-2 restart) */
} tpcref_tracklet_t;

typedef struct {
  int64_t decisions;  /* comparisons whose outcome shaped the result */
  int64_t near_ties;  /* of those, relative margin below 1e-6 */
  double min_margin;
  int64_t propagations; /* Kalman row steps of the fits (incl. failed ones) */
  int64_t tests;        /* chi2 tests of hits picked by the searches */
  int64_t updates;      /* Kalman updates attempted */
} tpcref_stats_t;

void tpcref_params_default(tpcref_params_t *p);

/* Run all stages on one sector.  cl is n x {x, y, z, q}; row[i] < n_rows.
   Returns an opaque result or NULL; *err = 0 ok, -1 bad input. */
void *tpcref_run(const tpcref_params_t *p, const float *row_x, const float *cl,
                 const uint8_t *row, int32_t n, int32_t precision, int32_t *err);
void tpcref_free(void *res);

int32_t tpcref_n_clusters(const void *res);
int32_t tpcref_n_tracklets(const void *res);   /* chains >= min_chain_hits */
int32_t tpcref_n_tracks(const void *res);
int64_t tpcref_n_tracklet_hits(const void *res);
int64_t tpcref_n_track_hits(const void *res);

/* which = 0: links as found; 1: after cleaning.  -1 = no link. */
void tpcref_get_links(const void *res, int32_t which, int32_t *up, int32_t *down);
/* tracklets in ascending start_id; hit_begin has n_tracklets + 1 entries */
void tpcref_get_tracklets(const void *res, tpcref_tracklet_t *out, int64_t *hit_begin,
                          int32_t *hits);
/* accepted tracks in ascending start_id: index of their tracklet, won hits */
void tpcref_get_tracks(const void *res, int32_t *tracklet_index, int64_t *hit_begin,
                       int32_t *hits);
void tpcref_get_assignment(const void *res, int32_t *track_of_cluster);
void tpcref_get_stats(const void *res, tpcref_stats_t *s);

/* Replay the fit of one tracklet along a given hit list (ascending rows;
   the chain occupies hits[k0 .. k0 + n_chain - 1] where hits[k0] is the chain
   start; hits before k0 came from the inward extension).  All decisions are
   taken from the list; only arithmetic is redone at the given precision.
   *min_margin (may be NULL) receives the smallest relative margin of the
   replay's |sin phi| <= max_sinphi tests (a replay that fails on a margin
   below 1e-6 met a near-tie, not an error). */
int32_t tpcref_refit(const tpcref_params_t *p, const float *row_x, const float *cl,
                     const uint8_t *row, const int32_t *hits, int32_t n_hits, int32_t k0,
                     int32_t n_chain, int32_t precision, tpcref_tracklet_t *out,
                     double *min_margin);

/* Single steps, for the unit pins.  State p[5], cov[15] in/out, *x in/out. */
int32_t tpcref_propagate(const tpcref_params_t *p, int32_t precision, double *state,
                         double *cov, double *x, double x1);
int32_t tpcref_update(const tpcref_params_t *p, int32_t precision, double *state, double *cov,
                      double ym, double zm, double *chi2);
/* The 2-D chi^2 the track-following searches test a picked hit with. */
int32_t tpcref_chi2(const tpcref_params_t *p, int32_t precision, const double *state,
                    const double *cov, double ym, double zm, double *chi2);
/* The hit the track-following search picks in row r for a state at plane
   row_x[r] whose z is relative to zr; -1 if none, -2 on bad input. */
int32_t tpcref_search_row(const tpcref_params_t *p, int32_t precision, const float *row_x,
                          const float *cl, const uint8_t *row, int32_t n, int32_t r,
                          const double *state, const double *cov, double zr);
/* The selection alone on given candidates: accepted[t] = index of the
   accepted track or -1, assignment[i] = track index or -1.  Returns the
   number of accepted tracks, -1 on bad input. */
int32_t tpcref_select(const tpcref_params_t *p, int32_t n_clusters, int32_t n_tracklets,
                      const int32_t *n_hits, const float *chi2, const int32_t *start_id,
                      const int32_t *status, const int64_t *hit_begin, const int32_t *hits,
                      int32_t *accepted, int32_t *assignment);

#ifdef __cplusplus
}
#endif
#endif
