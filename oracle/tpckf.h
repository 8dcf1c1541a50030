/*
 * tpckf.h: Kalman-filter primitives of the CPU oracle (TEST INFRASTRUCTURE),
 * shared by the sector tracker (tpcref.cpp) and the second phase
 * (tpcphase2.cpp).  Nothing of the GPU library includes this file.
 *
 * Track model of Sec. 2 (Rohr, LHCP 2017): state (y, z, sin phi, tan lambda,
 * q/pT) at a pad-row plane x of a sector frame, propagated with Bz only.
 */
#ifndef TPCKF_H
#define TPCKF_H

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>

#include "tpcref.h"

namespace tpcref_kf {

/* ------------------------------------------------------------ margins --- */
/* A decision a <= b has relative margin |a - b| / max(|a|, |b|, 1e-30).
   Decisions closer than 1e-6 are counted: they are the ones where a
   different rounding could flip the outcome. */
struct Margins {
  int64_t decisions = 0, near = 0;
  /* work of the fits: propagations, chi2 tests of searched hits, updates */
  int64_t props = 0, tests = 0, updates = 0;
  double min_margin = std::numeric_limits<double>::infinity();
  void note(double a, double b) {
    double d = std::fabs(a - b);
    double s = std::max(std::max(std::fabs(a), std::fabs(b)), 1e-30);
    double m = d / s;
    ++decisions;
    if (m < 1e-6) ++near;
    if (m < min_margin) min_margin = m;
  }
};

/* lower-triangular index of a symmetric 5x5 matrix */
inline int ci(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <typename F>
struct Par {
  int n_rows;
  F wy, wz, link_chi2;
  int min_chain;
  F kB, ery, erz, max_sin, c22, c33, c44, r00, r11, nsig, wmax, pick_chi2;
  int max_miss, min_hits, own_pct;
  F inflate;
  explicit Par(const tpcref_params_t &p)
      : n_rows(p.n_rows), wy(p.link_wy), wz(p.link_wz), link_chi2(p.link_chi2),
        min_chain(p.min_chain_hits), kB(p.kB), ery(p.err2_y), erz(p.err2_z),
        max_sin(p.max_sinphi), c22(p.seed_c22), c33(p.seed_c33), c44(p.seed_c44),
        r00(p.reset_c00), r11(p.reset_c11), nsig(p.pick_nsig), wmax(p.pick_win_max),
        pick_chi2(p.pick_chi2), max_miss(p.max_miss), min_hits(p.min_track_hits),
        own_pct(p.own_frac_pct), inflate(p.refit_inflate) {}
};

/* Track state at plane x: p = (y, z, sin phi, tan lambda, q/pT), cov C. */
template <typename F>
struct State {
  F p[5];
  F C[15];
  F x;
};

/*
 * Propagation of the state from its plane x to plane x1 in a field along z
 * (Sec. 2: the online tracker propagates with Bz only).  In the transverse
 * plane the trajectory is a circle of curvature k = kB * q/pT, so sin(phi)
 * grows linearly in x; the y step over dx is dx * tan of the mean direction,
 * which equals dx (s0 + s1) / (c0 + c1) exactly; the transverse arc length is
 * the chord (signed like dx) times asin(u)/u with u = chord * |k| / 2,
 * evaluated with the Maclaurin series of asin(u)/u to the u^8 term (one row
 * step has u < 0.02).
 *
 * Reading of "simplified" Kalman filter: the Jacobian drops the curvature
 * term of the arc length, i.e. dz/d(sin phi) and dz/d(q/pT) are taken as
 * tan(lambda) * d(chord)/d(.) with d(chord) = (dy / chord) d(dy).
 */
template <typename F>
bool propagate(const Par<F> &P, State<F> &s, F x1, Margins *mg) {
  const F dx = x1 - s.x;
  const F kk = P.kB * s.p[4];
  const F s0 = s.p[2];
  const F s1 = std::fma(kk, dx, s0);
  if (mg) mg->note((double)std::fabs(s1), (double)P.max_sin);
  if (!(std::fabs(s1) <= P.max_sin)) return false;
  const F one = (F)1;
  const F c0 = std::sqrt(std::fma(-s0, s0, one));
  const F c1 = std::sqrt(std::fma(-s1, s1, one));
  const F cc = c0 + c1;
  const F tt = (s0 + s1) / cc;
  const F dy = dx * tt;
  const F ch2 = std::fma(dy, dy, dx * dx);
  const F ch = std::sqrt(ch2);
  const F chs = dx < (F)0 ? -ch : ch; /* the arc length has the sign of the step */
  const F u2 = ch2 * kk * kk * (F)0.25;
  F h = (F)(35.0 / 1152.0);
  h = std::fma(u2, h, (F)(5.0 / 112.0));
  h = std::fma(u2, h, (F)(3.0 / 40.0));
  h = std::fma(u2, h, (F)(1.0 / 6.0));
  h = std::fma(u2, h, one);
  const F dS = chs * h;
  const F t = s.p[3];

  /* Jacobian entries (all others identity or zero) */
  const F a = dx * ((F)2 + tt * (s0 / c0 + s1 / c1)) / cc; /* dy/ds0 */
  const F b = dx * P.kB * dx * (one + tt * s1 / c1) / cc;  /* dy/dQ  */
  const F g = ch > (F)0 ? t * (dy / chs) : (F)0;
  const F cz = g * a;    /* dz/ds0 */
  const F dzq = g * b;   /* dz/dQ  */
  const F e = dS;        /* dz/dt  */
  const F f = P.kB * dx; /* ds/dQ  */

  s.p[0] = s.p[0] + dy;
  s.p[1] = s.p[1] + t * dS;
  s.p[2] = s1;
  s.x = x1;

  /* C <- F C F^T, expanded for the sparse F above. */
  const F *C = s.C;
  const F c00 = C[0], c10 = C[1], c11 = C[2], c20 = C[3], c21 = C[4], c22 = C[5];
  const F c30 = C[6], c31 = C[7], c32 = C[8], c33 = C[9];
  const F c40 = C[10], c41 = C[11], c42 = C[12], c43 = C[13], c44 = C[14];
  /* rows 0..2 of F*C that are needed */
  const F fc00 = c00 + a * c20 + b * c40;
  const F fc02 = c20 + a * c22 + b * c42;
  const F fc04 = c40 + a * c42 + b * c44;
  const F fc10 = c10 + cz * c20 + e * c30 + dzq * c40;
  const F fc11 = c11 + cz * c21 + e * c31 + dzq * c41;
  const F fc12 = c21 + cz * c22 + e * c32 + dzq * c42;
  const F fc13 = c31 + cz * c32 + e * c33 + dzq * c43;
  const F fc14 = c41 + cz * c42 + e * c43 + dzq * c44;
  const F fc20 = c20 + f * c40;
  const F fc21 = c21 + f * c41;
  const F fc22 = c22 + f * c42;
  const F fc23 = c32 + f * c43;
  const F fc24 = c42 + f * c44;
  F *O = s.C;
  O[0] = fc00 + a * fc02 + b * fc04;
  O[1] = fc10 + a * fc12 + b * fc14;
  O[2] = fc11 + cz * fc12 + e * fc13 + dzq * fc14;
  O[3] = fc20 + a * fc22 + b * fc24;
  O[4] = fc21 + cz * fc22 + e * fc23 + dzq * fc24;
  O[5] = fc22 + f * fc24;
  O[6] = c30 + a * c32 + b * c43;
  O[7] = c31 + cz * c32 + e * c33 + dzq * c43;
  O[8] = c32 + f * c43;
  O[9] = c33;
  O[10] = c40 + a * c42 + b * c44;
  O[11] = c41 + cz * c42 + e * c43 + dzq * c44;
  O[12] = c42 + f * c44;
  O[13] = c43;
  O[14] = c44;
  return true;
}

/* chi^2 of measurement (ym, zm) against the state: r^T S^-1 r with
   S = C[y,z block] + diag(err2_y, err2_z).  Returns false if S is singular. */
template <typename F>
bool chi2_2d(const Par<F> &P, const State<F> &s, F ym, F zm, F &chi2) {
  const F r0 = ym - s.p[0];
  const F r1 = zm - s.p[1];
  const F s00 = s.C[0] + P.ery;
  const F s10 = s.C[1];
  const F s11 = s.C[2] + P.erz;
  const F det = s00 * s11 - s10 * s10;
  if (!(det > (F)0)) return false;
  const F inv = (F)1 / det;
  const F i00 = s11 * inv, i10 = -s10 * inv, i11 = s00 * inv;
  const F v0 = i00 * r0 + i10 * r1;
  const F v1 = i10 * r0 + i11 * r1;
  chi2 = r0 * v0 + r1 * v1;
  return true;
}

/* Kalman update with a 2-D measurement of (y, z): gain K = C H^T S^-1,
   p += K r, C -= K H C (standard form, lower triangle kept). */
template <typename F>
bool update(const Par<F> &P, State<F> &s, F ym, F zm, F &chi2) {
  const F r0 = ym - s.p[0];
  const F r1 = zm - s.p[1];
  const F s00 = s.C[0] + P.ery;
  const F s10 = s.C[1];
  const F s11 = s.C[2] + P.erz;
  const F det = s00 * s11 - s10 * s10;
  if (!(det > (F)0)) return false;
  const F inv = (F)1 / det;
  const F i00 = s11 * inv, i10 = -s10 * inv, i11 = s00 * inv;
  const F v0 = i00 * r0 + i10 * r1;
  const F v1 = i10 * r0 + i11 * r1;
  chi2 = r0 * v0 + r1 * v1;
  F k0[5], k1[5], cj0[5], cj1[5];
  for (int k = 0; k < 5; ++k) {
    cj0[k] = s.C[ci(k, 0)];
    cj1[k] = s.C[ci(k, 1)];
  }
  for (int k = 0; k < 5; ++k) {
    k0[k] = cj0[k] * i00 + cj1[k] * i10;
    k1[k] = cj0[k] * i10 + cj1[k] * i11;
  }
  for (int k = 0; k < 5; ++k) s.p[k] = s.p[k] + k0[k] * r0 + k1[k] * r1;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j)
      s.C[ci(i, j)] = s.C[ci(i, j)] - (k0[i] * cj0[j] + k1[i] * cj1[j]);
  return true;
}

}  // namespace tpcref_kf

#endif
