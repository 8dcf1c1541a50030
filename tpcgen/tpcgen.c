/*
 * Seeded synthetic TPC events for the sector tracker.
 *
 * This module only produces inputs: helices of charged particles from the
 * origin in a uniform solenoid field, intersected in double precision with
 * the pad-row planes of the 36 TPC sectors, smeared, and written out as FP32
 * clusters {x, y, z, q} in each sector's local frame plus a pad-row index.
 * It holds none of the tracker's arithmetic.
 *
 * Conventions (shared by construction with whatever consumes the data):
 *   sector s in 0..35, s < 18 is the A side (z > 0), others the C side;
 *   sector centre angle alpha_s = ((s mod 18) + 0.5) * 20 deg;
 *   local frame x = X cos(a) + Y sin(a), y = -X sin(a) + Y cos(a), z = Z;
 *   pad rows at x_i = 85 + i * 162/158 cm, i = 0..158;
 *   signed curvature of the transverse circle kappa = kB * q / pT with
 *   kB = -Bz * 0.299792458e-2 cm^-1 (GeV/c)^-1, so dphi/dl = kappa;
 *   tan(lambda) = dz/dl (l = transverse arc length) = sinh(eta).
 *
 * Random numbers come from a counter-based generator: SplitMix64's finaliser
 * (Steele, Lea, Flood 2014) chained over (seed, stream, event, track, draw),
 * so every draw is a pure function of its coordinates.  Gaussians use the
 * Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TPCGEN_NROWS 159
#define TPCGEN_NSECT 36

static const double kPi = 3.14159265358979323846;

/* ---------------------------------------------------------------- RNG --- */
static uint64_t sm_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t tpcgen_hash(uint64_t seed, uint64_t stream, uint64_t event, uint64_t track,
                     uint64_t draw) {
  uint64_t h = sm_mix(seed);
  h = sm_mix(h ^ stream);
  h = sm_mix(h ^ event);
  h = sm_mix(h ^ track);
  return sm_mix(h ^ draw);
}

/* uniform in [0, 1) with 53 random bits */
static double u01(uint64_t seed, uint64_t st, uint64_t ev, uint64_t tr, uint64_t d) {
  return (double)(tpcgen_hash(seed, st, ev, tr, d) >> 11) * (1.0 / 9007199254740992.0);
}

/* standard normal from draws d and d+1 (Box-Muller, cosine branch) */
static double gauss(uint64_t seed, uint64_t st, uint64_t ev, uint64_t tr, uint64_t d) {
  double u1 = 1.0 - u01(seed, st, ev, tr, d); /* (0, 1] */
  double u2 = u01(seed, st, ev, tr, d + 1);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
}

/* ------------------------------------------------------------ geometry --- */
void tpcgen_row_x(int n_rows, float *out) {
  for (int i = 0; i < n_rows; ++i) out[i] = (float)(85.0 + (double)i * 162.0 / 158.0);
}

static double row_x64(int i) { return (double)(float)(85.0 + (double)i * 162.0 / 158.0); }

static double sector_alpha(int s) { return ((double)(s % 18) + 0.5) * (20.0 * kPi / 180.0); }

/* ------------------------------------------------------------- config --- */
typedef struct {
  uint64_t seed;
  uint64_t stream;   /* workload id: separates configurations */
  uint64_t event;    /* event index inside the stream */
  int32_t n_tracks;  /* primaries, loopers included */
  int32_t only_sector; /* -1: all 36 sectors; else keep clusters of this sector only */
  double looper_frac;  /* fraction of tracks drawn as low-pT loopers */
  double noise_frac;   /* noise clusters as a fraction of signal clusters */
  double sigma_y, sigma_z;
  double pt_min, pt_max;      /* power-law pT range, density ~ pT^-pt_index */
  double pt_index;            /* 2.0 */
  double eta_min, eta_max;
  double phi_min, phi_max;    /* global azimuth range of the initial direction */
  double looper_pt_min, looper_pt_max;
  double looper_turns;        /* full turns simulated for loopers */
  double normal_turns;        /* 0.5: outgoing half-turn only */
  double bz;                  /* tesla */
  double zmax;                /* |z| acceptance, cm */
  double t0_us;               /* event time inside a time frame */
  double vdrift;              /* cm/us */
  double q_min, q_max;        /* charge amplitude range (unused by tracking) */
} tpcgen_cfg_t;

void tpcgen_cfg_default(tpcgen_cfg_t *c) {
  memset(c, 0, sizeof(*c));
  c->n_tracks = 200;
  c->only_sector = -1;
  c->looper_frac = 0.0;
  c->noise_frac = 0.0;
  c->sigma_y = 0.1;
  c->sigma_z = 0.1;
  c->pt_min = 0.1;
  c->pt_max = 20.0;
  c->pt_index = 2.0;
  c->eta_min = -0.9;
  c->eta_max = 0.9;
  c->phi_min = 0.0;
  c->phi_max = 2.0 * kPi;
  c->looper_pt_min = 0.07;
  c->looper_pt_max = 0.185;
  c->looper_turns = 2.0;
  c->normal_turns = 0.5;
  c->bz = 0.5;
  c->zmax = 250.0;
  c->t0_us = 0.0;
  c->vdrift = 2.58;
  c->q_min = 20.0;
  c->q_max = 500.0;
}

/* per-track truth */
typedef struct {
  double pt, eta, phi0, tanl, kappa;
  int32_t charge, looper, side;
} tpcgen_track_t;

/* per-cluster truth: exact local state at the crossing (before smearing) */
typedef struct {
  double y, z, sinphi, tanl, qpt; /* qpt = q/pT */
  int32_t track;                  /* generating track, -1 for noise */
  int32_t leg;                    /* half-turns completed before the crossing; -1 noise */
  int32_t branch;                 /* 0: moving to larger x (cos > 0), 1: cos < 0 */
  int32_t pad_;
} tpcgen_truth_t;

typedef struct {
  float x, y, z, q;
} tpcgen_cluster_t;

typedef struct {
  int64_t n, cap;
  tpcgen_cluster_t *cl;
  uint8_t *row;
  uint8_t *sector;
  tpcgen_truth_t *truth;
  int32_t n_tracks;
  tpcgen_track_t *tracks;
  int64_t n_signal, n_noise;
} tpcgen_event_t;

static int ev_push(tpcgen_event_t *e, tpcgen_cluster_t c, int row, int sec, tpcgen_truth_t t) {
  if (e->n == e->cap) {
    int64_t nc = e->cap ? e->cap * 2 : 4096;
    void *a = realloc(e->cl, (size_t)nc * sizeof(tpcgen_cluster_t));
    if (!a) return -1;
    e->cl = (tpcgen_cluster_t *)a;
    a = realloc(e->row, (size_t)nc);
    if (!a) return -1;
    e->row = (uint8_t *)a;
    a = realloc(e->sector, (size_t)nc);
    if (!a) return -1;
    e->sector = (uint8_t *)a;
    a = realloc(e->truth, (size_t)nc * sizeof(tpcgen_truth_t));
    if (!a) return -1;
    e->truth = (tpcgen_truth_t *)a;
    e->cap = nc;
  }
  e->cl[e->n] = c;
  e->row[e->n] = (uint8_t)row;
  e->sector[e->n] = (uint8_t)sec;
  e->truth[e->n] = t;
  e->n++;
  return 0;
}

/* draw indices per track (stable meaning across versions) */
enum { D_LOOPER = 0, D_PT = 1, D_ETA = 2, D_PHI = 3, D_Q = 4, D_SMEAR = 16 };

/*
 * All crossings of one track with row plane x_r of sector s.  For a circle
 * through the origin with initial direction psi0 in the local frame, the local
 * direction at local x satisfies sin(psi) = sin(psi0) + kappa * x.  Two
 * branches: cos(psi) > 0 (moving to larger x) and cos(psi) < 0.  Each solution
 * repeats every full turn; the transverse arc length is dpsi / |kappa|.
 */
static int cross_row(tpcgen_event_t *e, const tpcgen_cfg_t *c, const tpcgen_track_t *t,
                     int itrk, int s, int r, double max_dpsi, int *draw_ctr) {
  const double a = sector_alpha(s);
  const double psi0 = t->phi0 - a;
  const double s0 = sin(psi0), c0 = cos(psi0);
  const double k = t->kappa;
  const double sgn = k >= 0 ? 1.0 : -1.0;
  const double tan10 = tan(10.0 * kPi / 180.0);
  const double xr = row_x64(r);
  if (k == 0.0) {
    /* no field: a straight line, one crossing if it heads to larger x */
    if (!(c0 > 0.0)) return 0;
    const double y = xr * s0 / c0;
    if (!(fabs(y) <= xr * tan10)) return 0;
    const double l = xr / c0;
    const double z = t->tanl * l;
    if (!(fabs(z) <= c->zmax)) return 0;
    const double zs = z - (z >= 0 ? 1.0 : -1.0) * c->vdrift * c->t0_us;
    int d = (*draw_ctr);
    *draw_ctr += 4;
    double gy = gauss(c->seed, c->stream, c->event, (uint64_t)itrk, D_SMEAR + d);
    double gz = gauss(c->seed, c->stream, c->event, (uint64_t)itrk, D_SMEAR + d + 2);
    tpcgen_cluster_t cl;
    cl.x = (float)xr;
    cl.y = (float)(y + c->sigma_y * gy);
    cl.z = (float)(zs + c->sigma_z * gz);
    cl.q = (float)c->q_min;
    tpcgen_truth_t tr;
    tr.y = y;
    tr.z = zs;
    tr.sinphi = s0;
    tr.tanl = t->tanl;
    tr.qpt = (double)t->charge / t->pt;
    tr.track = itrk;
    tr.leg = 0;
    tr.branch = 0;
    tr.pad_ = 0;
    return ev_push(e, cl, r, s, tr);
  }
  const double s1 = s0 + k * xr;
  if (!(fabs(s1) < 1.0)) return 0;
  const double cabs = sqrt((1.0 - s1) * (1.0 + s1));
  for (int br = 0; br < 2; ++br) {
    const double c1 = br == 0 ? cabs : -cabs;
    /* local y at the crossing: stable forms for each branch */
    double y;
    if (c0 + c1 > 0.5) y = xr * (s0 + s1) / (c0 + c1);
    else y = (c0 - c1) / k;
    if (!(fabs(y) <= xr * tan10)) continue;
    /* direction change psi1 - psi0 in (-pi, pi], then oriented by kappa */
    double dpsi = atan2(s1 * c0 - c1 * s0, c1 * c0 + s1 * s0);
    dpsi *= sgn;
    if (dpsi < 0) dpsi += 2.0 * kPi;
    for (int turn = 0;; ++turn) {
      double dp = dpsi + 2.0 * kPi * turn;
      if (dp > max_dpsi) break;
      const double l = dp / fabs(k);
      const double z = t->tanl * l;
      if (!(fabs(z) <= c->zmax)) break;
      const double zs = z - (z >= 0 ? 1.0 : -1.0) * c->vdrift * c->t0_us;
      int d = (*draw_ctr);
      *draw_ctr += 4;
      double gy = gauss(c->seed, c->stream, c->event, (uint64_t)itrk, D_SMEAR + d);
      double gz = gauss(c->seed, c->stream, c->event, (uint64_t)itrk, D_SMEAR + d + 2);
      double qa = c->q_min + (c->q_max - c->q_min) *
                                 u01(c->seed, c->stream, c->event, (uint64_t)itrk,
                                     (uint64_t)(D_SMEAR + d) + (1ULL << 40));
      tpcgen_cluster_t cl;
      cl.x = (float)xr;
      cl.y = (float)(y + c->sigma_y * gy);
      cl.z = (float)(zs + c->sigma_z * gz);
      cl.q = (float)qa;
      tpcgen_truth_t tr;
      tr.y = y;
      tr.z = zs;
      tr.sinphi = s1;
      tr.tanl = t->tanl;
      tr.qpt = (double)t->charge / t->pt;
      tr.track = itrk;
      tr.leg = (int32_t)floor(dp / kPi);
      tr.branch = br;
      tr.pad_ = 0;
      if (ev_push(e, cl, r, s, tr)) return -1;
    }
  }
  return 0;
}

static int sector_allowed(const tpcgen_cfg_t *c, int s) {
  return c->only_sector < 0 || c->only_sector == s;
}

tpcgen_event_t *tpcgen_make_event(const tpcgen_cfg_t *c) {
  tpcgen_event_t *e = (tpcgen_event_t *)calloc(1, sizeof(tpcgen_event_t));
  if (!e) return NULL;
  const int nt = c->n_tracks;
  e->n_tracks = nt;
  e->tracks = (tpcgen_track_t *)calloc((size_t)(nt > 0 ? nt : 1), sizeof(tpcgen_track_t));
  if (!e->tracks) return NULL;
  const double kB = -c->bz * 0.299792458e-2;
  for (int i = 0; i < nt; ++i) {
    tpcgen_track_t *t = &e->tracks[i];
    const uint64_t S = c->seed, st = c->stream, ev = c->event, tr = (uint64_t)i;
    t->looper = u01(S, st, ev, tr, D_LOOPER) < c->looper_frac;
    double u = u01(S, st, ev, tr, D_PT);
    if (t->looper) {
      t->pt = c->looper_pt_min + (c->looper_pt_max - c->looper_pt_min) * u;
    } else if (fabs(c->pt_index - 1.0) < 1e-12) {
      t->pt = c->pt_min * pow(c->pt_max / c->pt_min, u);
    } else {
      /* inverse CDF of a truncated power law with density ~ pT^-n */
      const double g = 1.0 - c->pt_index;
      const double a = pow(c->pt_min, g), b = pow(c->pt_max, g);
      t->pt = pow(a + (b - a) * u, 1.0 / g);
    }
    t->eta = c->eta_min + (c->eta_max - c->eta_min) * u01(S, st, ev, tr, D_ETA);
    t->tanl = sinh(t->eta);
    t->phi0 = c->phi_min + (c->phi_max - c->phi_min) * u01(S, st, ev, tr, D_PHI);
    t->charge = u01(S, st, ev, tr, D_Q) < 0.5 ? -1 : 1;
    t->kappa = kB * (double)t->charge / t->pt;
    t->side = t->tanl >= 0 ? 0 : 1;
  }
  for (int i = 0; i < nt; ++i) {
    const tpcgen_track_t *t = &e->tracks[i];
    const double max_dpsi = 2.0 * kPi * (t->looper ? c->looper_turns : c->normal_turns);
    int draw = 0;
    const int base = t->side * 18;
    const double sw = 20.0 * kPi / 180.0;
    if (t->looper) {
      for (int ss = 0; ss < 18; ++ss) {
        if (!sector_allowed(c, base + ss)) continue;
        for (int r = 0; r < TPCGEN_NROWS; ++r)
          if (cross_row(e, c, t, i, base + ss, r, max_dpsi, &draw)) return NULL;
      }
    } else {
      /* On the outgoing half-turn a circle through the origin is at azimuth
         phi0 + asin(kappa rho / 2) when at radius rho.  A crossing of row
         plane x_r lies at rho in [x_r, x_r / cos 10deg], so its sector is
         within one of the sectors holding those two azimuths. */
      const double inv_c10 = 1.0 / cos(10.0 * kPi / 180.0);
      for (int r = 0; r < TPCGEN_NROWS; ++r) {
        const double xr = row_x64(r);
        const double a0 = t->kappa * xr * 0.5;
        if (!(fabs(a0) < 1.0)) break;
        double a1 = t->kappa * xr * inv_c10 * 0.5;
        if (a1 > 1.0) a1 = 1.0;
        if (a1 < -1.0) a1 = -1.0;
        int sa = (int)floor((t->phi0 + asin(a0)) / sw);
        int sb = (int)floor((t->phi0 + asin(a1)) / sw);
        int lo = sa < sb ? sa : sb, hi = sa < sb ? sb : sa;
        for (int q = lo - 1; q <= hi + 1; ++q) {
          int ss = ((q % 18) + 18) % 18;
          if (!sector_allowed(c, base + ss)) continue;
          if (cross_row(e, c, t, i, base + ss, r, max_dpsi, &draw)) return NULL;
        }
      }
    }
  }
  e->n_signal = e->n;
  /* uniform noise clusters */
  int64_t nn = (int64_t)floor(c->noise_frac * (double)e->n_signal + 0.5);
  const uint64_t NOISE_TRACK = 0xFFFFFFFFULL;
  for (int64_t j = 0; j < nn; ++j) {
    const uint64_t S = c->seed, st = c->stream, ev = c->event;
    uint64_t d = (uint64_t)j * 8;
    int s = c->only_sector >= 0 ? c->only_sector
                                : (int)floor(36.0 * u01(S, st, ev, NOISE_TRACK, d));
    if (s > 35) s = 35;
    int r = (int)floor(159.0 * u01(S, st, ev, NOISE_TRACK, d + 1));
    if (r > 158) r = 158;
    double xr = row_x64(r);
    double ymax = xr * tan(10.0 * kPi / 180.0);
    double y = ymax * (2.0 * u01(S, st, ev, NOISE_TRACK, d + 2) - 1.0);
    double z = c->zmax * u01(S, st, ev, NOISE_TRACK, d + 3);
    if (s >= 18) z = -z;
    double zs = z - (z >= 0 ? 1.0 : -1.0) * c->vdrift * c->t0_us;
    tpcgen_cluster_t cl;
    cl.x = (float)xr;
    cl.y = (float)y;
    cl.z = (float)zs;
    cl.q = (float)(c->q_min + (c->q_max - c->q_min) * u01(S, st, ev, NOISE_TRACK, d + 4));
    tpcgen_truth_t tr;
    memset(&tr, 0, sizeof(tr));
    tr.y = y;
    tr.z = zs;
    tr.track = -1;
    tr.leg = -1;
    tr.branch = -1;
    if (ev_push(e, cl, r, s, tr)) return NULL;
  }
  e->n_noise = e->n - e->n_signal;
  return e;
}

int64_t tpcgen_count(const tpcgen_event_t *e) { return e ? e->n : -1; }
int64_t tpcgen_count_signal(const tpcgen_event_t *e) { return e ? e->n_signal : -1; }
int32_t tpcgen_n_tracks(const tpcgen_event_t *e) { return e ? e->n_tracks : -1; }

/*
 * Copy the event out grouped by sector (sector-major, stable inside a
 * sector).  sector_begin has 37 entries.  Any output pointer may be NULL.
 */
int tpcgen_copy(const tpcgen_event_t *e, tpcgen_cluster_t *cl, uint8_t *row, uint8_t *sector,
                tpcgen_truth_t *truth, int64_t *sector_begin, tpcgen_track_t *tracks) {
  if (!e) return -1;
  int64_t cnt[TPCGEN_NSECT + 1];
  memset(cnt, 0, sizeof(cnt));
  for (int64_t i = 0; i < e->n; ++i) cnt[e->sector[i] + 1]++;
  for (int s = 0; s < TPCGEN_NSECT; ++s) cnt[s + 1] += cnt[s];
  if (sector_begin)
    for (int s = 0; s <= TPCGEN_NSECT; ++s) sector_begin[s] = cnt[s];
  int64_t pos[TPCGEN_NSECT];
  for (int s = 0; s < TPCGEN_NSECT; ++s) pos[s] = cnt[s];
  for (int64_t i = 0; i < e->n; ++i) {
    int64_t p = pos[e->sector[i]]++;
    if (cl) cl[p] = e->cl[i];
    if (row) row[p] = e->row[i];
    if (sector) sector[p] = e->sector[i];
    if (truth) truth[p] = e->truth[i];
  }
  if (tracks) memcpy(tracks, e->tracks, (size_t)e->n_tracks * sizeof(tpcgen_track_t));
  return 0;
}

void tpcgen_free(tpcgen_event_t *e) {
  if (!e) return;
  free(e->cl);
  free(e->row);
  free(e->sector);
  free(e->truth);
  free(e->tracks);
  free(e);
}

/* Fisher-Yates permutation of 0..n-1 from the counter-based generator. */
void tpcgen_permutation(uint64_t seed, uint64_t stream, uint64_t key, int64_t n, int32_t *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t h = tpcgen_hash(seed, stream, key, 0xABCDEF01ULL, (uint64_t)i);
    int64_t j = (int64_t)(h % (uint64_t)(i + 1));
    int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

/* Uniform draws exposed for higher-level recipes (multiplicity, arrivals). */
double tpcgen_uniform(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b, uint64_t draw) {
  return u01(seed, stream, a, b, draw);
}
