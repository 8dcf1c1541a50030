/*
 * tpcref: plain CPU oracle of the TPC sector tracker.  TEST INFRASTRUCTURE:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the GPU library.
 *
 * Method: Rohr, LHCP 2017, Sec. 2 (sector tracker, Fig. 1a-c).  The paper
 * gives the steps in prose; the formulas, cuts and tie-breaks below are the
 * readings this project fixes, stated next to the code that applies them.
 * The code favours being checkable by eye over speed: rows are kept sorted by
 * z so that a window lookup is a binary search followed by an exact test of
 * every hit in a slightly wider z range.
 *
 * Floating point: compiled without contraction (-ffp-contract=off) and without
 * fast-math; std::fma appears exactly where the reading prescribes a fused
 * multiply-add; / and sqrt are the correctly rounded IEEE operations.
 */
#include "tpcref.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>

#include "tpckf.h"

namespace {

using namespace tpcref_kf;

/* ------------------------------------------------------------- sector --- */
template <typename F>
struct Sector {
  const Par<F> &P;
  std::vector<F> rx;            /* row radii */
  int n;
  std::vector<F> y, z;
  std::vector<int> row;
  std::vector<std::vector<int>> ids; /* per row, ids sorted by (z, id) */
  std::vector<std::vector<F>> zs;    /* per row, z in the same order */

  Sector(const Par<F> &P_, const float *row_x, const float *cl, const uint8_t *rw, int n_)
      : P(P_), rx(P_.n_rows), n(n_), y(n_), z(n_), row(n_), ids(P_.n_rows), zs(P_.n_rows) {
    for (int r = 0; r < P.n_rows; ++r) rx[r] = (F)row_x[r];
    for (int i = 0; i < n; ++i) {
      y[i] = (F)cl[4 * i + 1];
      z[i] = (F)cl[4 * i + 2];
      row[i] = rw[i];
      ids[row[i]].push_back(i);
    }
    for (int r = 0; r < P.n_rows; ++r) {
      auto &v = ids[r];
      std::sort(v.begin(), v.end(), [&](int a, int b) {
        return z[a] < z[b] || (z[a] == z[b] && a < b);
      });
      zs[r].resize(v.size());
      for (size_t k = 0; k < v.size(); ++k) zs[r][k] = z[v[k]];
    }
  }

  /* All hits of row r with |y_h - yc| <= ly and |z_h - zc| <= lz.  The binary
     search brackets a z range a little wider than the window; the exact test
     is applied to each hit in it. */
  template <typename Fn>
  void window(int r, F yc, F zc, F ly, F lz, Fn &&fn) const {
    const auto &zv = zs[r];
    const double pad = 1e-3 + 1e-6 * std::fabs((double)zc) + 1e-3 * (double)lz;
    const double lo = (double)zc - (double)lz - pad, hi = (double)zc + (double)lz + pad;
    auto it = std::lower_bound(zv.begin(), zv.end(), lo,
                               [](F a, double b) { return (double)a < b; });
    for (size_t k = (size_t)(it - zv.begin()); k < zv.size() && (double)zv[k] <= hi; ++k) {
      const int h = ids[r][k];
      if (std::fabs(y[h] - yc) <= ly && std::fabs(z[h] - zc) <= lz) fn(h);
    }
  }

  /* The same for a track state whose z is kept relative to zr: the window
     is |y_h - yc| <= ly and |(z_h - zr) - zc| <= lz.  The bracket is taken
     around the absolute z in FP64 (a superset), the test in F. */
  template <typename Fn>
  void window_rel(int r, F yc, F zr, F zc, F ly, F lz, Fn &&fn) const {
    const double za = (double)zr + (double)zc;
    const auto &zv = zs[r];
    const double pad = 1e-3 + 1e-6 * std::fabs(za) + 1e-3 * (double)lz;
    const double lo = za - (double)lz - pad, hi = za + (double)lz + pad;
    auto it = std::lower_bound(zv.begin(), zv.end(), lo,
                               [](F a, double b) { return (double)a < b; });
    for (size_t k = (size_t)(it - zv.begin()); k < zv.size() && (double)zv[k] <= hi; ++k) {
      const int h = ids[r][k];
      if (std::fabs(y[h] - yc) <= ly && std::fabs((z[h] - zr) - zc) <= lz) fn(h);
    }
  }
};

template <typename F>
struct Tracklet {
  tpcref_tracklet_t t;
  std::vector<int> hits; /* ascending rows */
};

/*
 * CA neighbour finding (Fig. 1a): for a hit in row i (1 <= i <= n_rows - 2)
 * consider every pair (u in row i+1, d in row i-1) inside windows
 * |dy| <= W dx, |dz| <= W dx around the hit.  The pair's deviation from a
 * straight line is measured at x_i: e = (y, z)_h - interpolation of d -> u,
 * evaluated from coordinate differences, e = (h - d) - w (u - d), with one
 * rounding: in a time frame z' reaches tens of metres (Sec. 5), where the
 * FP32 spacing of an absolute coordinate is a sizeable part of the
 * deviations, while differences of nearby hits are exact.
 * The best pair minimises (chi2, id_u, id_d) lexicographically; it becomes
 * the hit's (up, down) links if chi2 <= link_chi2.  Edge rows get no links.
 */
template <typename F>
void find_links(const Sector<F> &S, std::vector<int> &up, std::vector<int> &dn, Margins &mg) {
  const auto &P = S.P;
  up.assign(S.n, -1);
  dn.assign(S.n, -1);
  for (int h = 0; h < S.n; ++h) {
    const int i = S.row[h];
    if (i < 1 || i > P.n_rows - 2) continue;
    const F dxu = S.rx[i + 1] - S.rx[i];
    const F dxd = S.rx[i] - S.rx[i - 1];
    const F w = dxd / (dxd + dxu);
    const F luy = P.wy * dxu, luz = P.wz * dxu, ldy = P.wy * dxd, ldz = P.wz * dxd;
    const F yh = S.y[h], zh = S.z[h];
    std::vector<int> U, D;
    S.window(i + 1, yh, zh, luy, luz, [&](int u) { U.push_back(u); });
    if (U.empty()) continue;
    S.window(i - 1, yh, zh, ldy, ldz, [&](int d) { D.push_back(d); });
    if (D.empty()) continue;
    F best = std::numeric_limits<F>::infinity(), second = best;
    int bu = -1, bd = -1;
    for (int u : U)
      for (int d : D) {
        const F ey = std::fma(-(S.y[u] - S.y[d]), w, yh - S.y[d]);
        const F ez = std::fma(-(S.z[u] - S.z[d]), w, zh - S.z[d]);
        const F c2 = std::fma(ey, ey, ez * ez);
        bool better = c2 < best || (c2 == best && (u < bu || (u == bu && d < bd)));
        if (better) {
          second = best;
          best = c2;
          bu = u;
          bd = d;
        } else if (c2 < second) {
          second = c2;
        }
      }
    mg.note((double)best, (double)P.link_chi2);
    if (second < std::numeric_limits<F>::infinity()) mg.note((double)best, (double)second);
    mg.note((double)std::fabs(S.y[bu] - yh), (double)luy);
    mg.note((double)std::fabs(S.z[bu] - zh), (double)luz);
    mg.note((double)std::fabs(S.y[bd] - yh), (double)ldy);
    mg.note((double)std::fabs(S.z[bd] - zh), (double)ldz);
    if (best <= P.link_chi2) {
      up[h] = bu;
      dn[h] = bd;
    }
  }
}

/*
 * Link cleaning (Fig. 1b): a link survives only if it is reciprocal, i.e.
 * up'[h] = u iff down[u] = h, and down'[h] = d iff up[d] = h.
 */
void clean_links(const std::vector<int> &up, const std::vector<int> &dn, std::vector<int> &upc,
                 std::vector<int> &dnc) {
  const int n = (int)up.size();
  upc.assign(n, -1);
  dnc.assign(n, -1);
  for (int h = 0; h < n; ++h) {
    if (up[h] >= 0 && dn[up[h]] == h) upc[h] = up[h];
    if (dn[h] >= 0 && up[dn[h]] == h) dnc[h] = dn[h];
  }
}

/* Nearest hit to the predicted (y, z) inside nsig predicted sigmas (capped),
   by dy^2 + dz^2 with ties to the lower ID. */
template <typename F>
int search_row(const Sector<F> &S, const State<F> &st, F zr, int r, Margins &mg) {
  const auto &P = S.P;
  F wy = P.nsig * std::sqrt(st.C[0] + P.ery);
  F wz = P.nsig * std::sqrt(st.C[2] + P.erz);
  if (wy > P.wmax) wy = P.wmax;
  if (wz > P.wmax) wz = P.wmax;
  int best = -1;
  F bd2 = std::numeric_limits<F>::infinity(), second = bd2;
  S.window_rel(r, st.p[0], zr, st.p[1], wy, wz, [&](int h) {
    const F dy = S.y[h] - st.p[0];
    const F dz = (S.z[h] - zr) - st.p[1];
    const F d2 = std::fma(dy, dy, dz * dz);
    if (d2 < bd2 || (d2 == bd2 && h < best)) {
      second = bd2;
      bd2 = d2;
      best = h;
    } else if (d2 < second) {
      second = d2;
    }
  });
  if (best >= 0) {
    if (second < std::numeric_limits<F>::infinity()) mg.note((double)bd2, (double)second);
    mg.note((double)std::fabs(S.y[best] - st.p[0]), (double)wy);
    mg.note((double)std::fabs((S.z[best] - zr) - st.p[1]), (double)wz);
  }
  return best;
}

template <typename F>
void to_out(const State<F> &s, double *p, double *C, F zr = (F)0) {
  for (int k = 0; k < 5; ++k) p[k] = (double)s.p[k];
  p[1] = (double)(s.p[1] + zr); /* back to the absolute z of the sector frame */
  if (C)
    for (int k = 0; k < 15; ++k) C[k] = (double)s.C[k];
}

/*
 * Track following with the Kalman filter (Fig. 1c).  Reading:
 *  seed  at the chain's first hit: y, z measured; sin phi from the slope of
 *        the chain's end points, tan lambda from their z slope times cos phi,
 *        q/pT = 0; C = diag(err2_y, err2_z, c22, c33, c44).
 *  pass 1 (outward) updates with the remaining chain hits, then visits every
 *        further row: propagate, take the nearest hit inside the window and
 *        accept it if chi2 <= pick_chi2; stop after max_miss rows in a row
 *        without a hit, at the last row, or when propagation fails.
 *  pass 2 (inward) restarts at the outermost hit from the pass-1 state and
 *        the pass-1 covariance multiplied by refit_inflate (a soft restart:
 *        the first hits of the refit cannot swing the direction far from the
 *        pass-1 estimate, which keeps the linearisation honest; a hard restart
 *        C = diag(reset_c00, reset_c11, c22, c33, c44) is used when
 *        refit_inflate = 0), updates with all pass-1 hits in decreasing row
 *        order (no cut), then continues below the chain start row by row as
 *        in pass 1.
 *  output the state after the last pass-2 update (innermost hit), the pass-2
 *        chi2 and ndf = 2 n_hits - 5; tracklets with fewer than
 *        min_track_hits hits are kept but flagged (status 1).
 *  z     the state's z is kept relative to zr, the z of the chain's first
 *        hit: every measurement enters as z_h - zr and the output adds zr
 *        back.  In a time frame z' spans tens of metres (Sec. 5) and an
 *        absolute FP32 z would carry rounding errors comparable with the
 *        fit's z resolution; differences of a track's own hits are exact.
 *  `replay`, when given, lists the hits to use instead of searching: the
 *        pass-1 extra hits and the inward hits, each with its row.
 */
struct Replay {
  std::vector<int> outward; /* pass-1 hits beyond the chain, ascending rows */
  std::vector<int> inward;  /* inward hits, descending rows */
};

template <typename F>
void fit_tracklet(const Sector<F> &S, const std::vector<int> &chain, Tracklet<F> &T, Margins &mg,
                  const Replay *rp) {
  const auto &P = S.P;
  tpcref_tracklet_t &o = T.t;
  std::memset(&o, 0, sizeof(o));
  o.start_id = chain[0];
  o.n_chain = (int)chain.size();
  o.status = 2;
  const int L = (int)chain.size() - 1;
  const int h0 = chain[0], hL = chain[L];
  State<F> st;
  const F one = (F)1;
  const F zr = S.z[h0];
  auto zm = [&](int h) { return S.z[h] - zr; };
  {
    const F x0 = S.rx[S.row[h0]], xL = S.rx[S.row[hL]];
    const F dxs = xL - x0;
    const F ty = (S.y[hL] - S.y[h0]) / dxs;
    const F sn = ty / std::sqrt(std::fma(ty, ty, one));
    const F tz = (S.z[hL] - S.z[h0]) / dxs;
    const F tl = tz * std::sqrt(std::fma(-sn, sn, one));
    st.p[0] = S.y[h0];
    st.p[1] = zm(h0);
    st.p[2] = sn;
    st.p[3] = tl;
    st.p[4] = (F)0;
    for (int k = 0; k < 15; ++k) st.C[k] = (F)0;
    st.C[0] = P.ery;
    st.C[2] = P.erz;
    st.C[5] = P.c22;
    st.C[9] = P.c33;
    st.C[14] = P.c44;
    st.x = x0;
  }
  std::vector<int> pass1(chain.begin(), chain.end());
  F c2;
  for (int k = 1; k <= L; ++k) {
    const int h = chain[k];
    ++mg.props;
    if (!propagate(P, st, S.rx[S.row[h]], &mg)) return;
    ++mg.updates;
    if (!update(P, st, S.y[h], zm(h), c2)) return;
  }
  State<F> saved = st;
  int row_out = S.row[hL];
  /* pass 1: follow outward */
  if (!rp) {
    int miss = 0;
    for (int r = row_out + 1; r < P.n_rows; ++r) {
      ++mg.props;
      if (!propagate(P, st, S.rx[r], &mg)) break;
      const int h = search_row(S, st, zr, r, mg);
      bool took = false;
      if (h >= 0) {
        F c;
        ++mg.tests;
        if (chi2_2d(P, st, S.y[h], zm(h), c)) {
          mg.note((double)c, (double)P.pick_chi2);
          if (c <= P.pick_chi2) ++mg.updates;
          if (c <= P.pick_chi2 && update(P, st, S.y[h], zm(h), c2)) {
            pass1.push_back(h);
            saved = st;
            row_out = r;
            took = true;
          }
        }
      }
      if (took) {
        miss = 0;
      } else if (++miss >= P.max_miss) {
        break;
      }
    }
  } else {
    size_t k = 0;
    for (int r = row_out + 1; r < P.n_rows && k < rp->outward.size(); ++r) {
      if (!propagate(P, st, S.rx[r], &mg)) return;
      const int h = rp->outward[k];
      if (S.row[h] == r) {
        if (!update(P, st, S.y[h], zm(h), c2)) return;
        pass1.push_back(h);
        saved = st;
        row_out = r;
        ++k;
      }
    }
    if (k != rp->outward.size()) return;
  }
  /* pass 2: restart at the outermost hit and refit inward */
  st = saved;
  if (P.inflate > (F)0) {
    for (int k = 0; k < 15; ++k) st.C[k] = st.C[k] * P.inflate;
  } else {
    for (int k = 0; k < 15; ++k) st.C[k] = (F)0;
    st.C[0] = P.r00;
    st.C[2] = P.r11;
    st.C[5] = P.c22;
    st.C[9] = P.c33;
    st.C[14] = P.c44;
  }
  F chi2 = (F)0;
  State<F> out_state;
  const int n1 = (int)pass1.size();
  for (int k = n1 - 1; k >= 0; --k) {
    const int h = pass1[k];
    if (k < n1 - 1) ++mg.props;
    if (k < n1 - 1 && !propagate(P, st, S.rx[S.row[h]], &mg)) return;
    ++mg.updates;
    if (!update(P, st, S.y[h], zm(h), c2)) return;
    chi2 = chi2 + c2;
  }
  out_state = st;
  std::vector<int> inward;
  if (!rp) {
    int miss = 0;
    for (int r = S.row[h0] - 1; r >= 0; --r) {
      ++mg.props;
      if (!propagate(P, st, S.rx[r], &mg)) break;
      const int h = search_row(S, st, zr, r, mg);
      bool took = false;
      if (h >= 0) {
        F c;
        ++mg.tests;
        if (chi2_2d(P, st, S.y[h], zm(h), c)) {
          mg.note((double)c, (double)P.pick_chi2);
          if (c <= P.pick_chi2) ++mg.updates;
          if (c <= P.pick_chi2 && update(P, st, S.y[h], zm(h), c2)) {
            chi2 = chi2 + c2;
            inward.push_back(h);
            out_state = st;
            took = true;
          }
        }
      }
      if (took) {
        miss = 0;
      } else if (++miss >= P.max_miss) {
        break;
      }
    }
  } else {
    size_t k = 0;
    for (int r = S.row[h0] - 1; r >= 0 && k < rp->inward.size(); --r) {
      if (!propagate(P, st, S.rx[r], &mg)) return;
      const int h = rp->inward[k];
      if (S.row[h] == r) {
        if (!update(P, st, S.y[h], zm(h), c2)) return;
        chi2 = chi2 + c2;
        inward.push_back(h);
        out_state = st;
        ++k;
      }
    }
    if (k != rp->inward.size()) return;
  }
  /* hits in ascending row order: inward hits reversed, then pass 1 */
  T.hits.assign(inward.rbegin(), inward.rend());
  T.hits.insert(T.hits.end(), pass1.begin(), pass1.end());
  o.n_hits = (int)T.hits.size();
  o.n_pass1 = n1;
  o.ndf = 2 * o.n_hits - 5;
  o.row_ref = S.row[T.hits.front()];
  o.row_out = row_out;
  o.x_ref = (double)out_state.x;
  o.x_out = (double)saved.x;
  o.chi2 = (double)chi2;
  to_out(out_state, o.p, o.cov, zr);
  to_out(saved, o.p_out, o.cov_out, zr);
  o.status = o.n_hits < P.min_hits ? 1 : 0;
}

struct Result {
  int n = 0;
  std::vector<int> up, dn, upc, dnc;
  std::vector<tpcref_tracklet_t> trk;
  std::vector<std::vector<int>> trk_hits;
  std::vector<int> acc_index;             /* accepted tracklet indices */
  std::vector<std::vector<int>> acc_hits; /* won hits, ascending rows */
  std::vector<int> assign;
  Margins mg;
};

/*
 * Selection (end of Sec. 2's sector tracker): every fitted tracklet claims
 * its hits with a key ordered by more hits, then smaller chi2, then smaller
 * start_id; a hit belongs to the largest key claiming it (one round, so the
 * result does not depend on any order).  A tracklet is accepted if it wins at
 * least min_track_hits hits and at least own_frac_pct percent of its hits;
 * it keeps the hits it won, its parameters are not refitted.  Accepted tracks
 * are listed in ascending start_id.
 *
 * The key packs n_hits (8 bits), the inverted FP32 bit pattern of chi2
 * (32 bits; the bits of a non-negative float order like its value) and the
 * inverted start_id (24 bits) into one 64-bit integer.
 */
uint64_t select_key(int n_hits, float chi2, int start_id) {
  float c = chi2 > 0.0f ? chi2 : 0.0f;
  uint32_t bits;
  std::memcpy(&bits, &c, sizeof(bits));
  return ((uint64_t)(uint32_t)n_hits << 56) | ((uint64_t)(0xFFFFFFFFu - bits) << 24) |
         (uint64_t)(0xFFFFFFu - (uint32_t)start_id);
}

void select_tracks(int min_hits, int own_pct, int n, Result &R) {
  std::vector<uint64_t> owner(n, 0);
  const int T = (int)R.trk.size();
  auto key = [&](int t) {
    return select_key(R.trk[t].n_hits, (float)R.trk[t].chi2, R.trk[t].start_id);
  };
  for (int t = 0; t < T; ++t) {
    if (R.trk[t].status != 0) continue;
    for (int h : R.trk_hits[t]) owner[h] = std::max(owner[h], key(t));
  }
  R.assign.assign(n, -1);
  for (int t = 0; t < T; ++t) {
    if (R.trk[t].status != 0) continue;
    std::vector<int> won;
    for (int h : R.trk_hits[t])
      if (owner[h] == key(t)) won.push_back(h);
    const int nw = (int)won.size();
    if (nw >= min_hits && nw * 100 >= own_pct * R.trk[t].n_hits) {
      const int idx = (int)R.acc_index.size();
      R.acc_index.push_back(t);
      for (int h : won) R.assign[h] = idx;
      R.acc_hits.push_back(std::move(won));
    }
  }
}

template <typename F>
Result *run(const tpcref_params_t &pp, const float *row_x, const float *cl, const uint8_t *rw,
            int n) {
  Par<F> P(pp);
  Sector<F> S(P, row_x, cl, rw, n);
  auto R = std::make_unique<Result>();
  R->n = n;
  find_links(S, R->up, R->dn, R->mg);
  clean_links(R->up, R->dn, R->upc, R->dnc);
  /* chains start at hits with an up link and no down link (ascending ID) */
  for (int h = 0; h < n; ++h) {
    if (!(R->upc[h] >= 0 && R->dnc[h] < 0)) continue;
    std::vector<int> chain;
    for (int k = h; k >= 0; k = R->upc[k]) chain.push_back(k);
    if ((int)chain.size() < P.min_chain) continue;
    Tracklet<F> T;
    fit_tracklet(S, chain, T, R->mg, nullptr);
    R->trk.push_back(T.t);
    R->trk_hits.push_back(std::move(T.hits));
  }
  select_tracks(P.min_hits, P.own_pct, n, *R);
  return R.release();
}

template <typename F>
void set_state(State<F> &s, const double *p, const double *C, double x) {
  for (int k = 0; k < 5; ++k) s.p[k] = (F)p[k];
  for (int k = 0; k < 15; ++k) s.C[k] = (F)C[k];
  s.x = (F)x;
}

template <typename F>
int32_t refit_impl(const tpcref_params_t &pp, const float *row_x, const float *cl,
                          const uint8_t *rw, int32_t n, const int32_t *hits, int32_t nh, int32_t k0,
                          int32_t n_chain, tpcref_tracklet_t *out, double *min_margin) {
  Par<F> P(pp);
  Sector<F> S(P, row_x, cl, rw, n);
  std::vector<int> chain(hits + k0, hits + k0 + n_chain);
  Replay rp;
  for (int k = k0 + n_chain; k < nh; ++k) rp.outward.push_back(hits[k]);
  for (int k = k0 - 1; k >= 0; --k) rp.inward.push_back(hits[k]);
  Tracklet<F> T;
  Margins mg;
  fit_tracklet(S, chain, T, mg, &rp);
  *out = T.t;
  if (min_margin) *min_margin = mg.min_margin;
  return T.t.status == 2 ? -1 : 0;
}

}  // namespace

extern "C" {

void tpcref_params_default(tpcref_params_t *p) {
  p->n_rows = 159;
  p->link_wy = 2.0f;
  p->link_wz = 2.0f;
  p->link_chi2 = 0.2f;
  p->min_chain_hits = 3;
  p->kB = (float)(-0.5 * 0.299792458e-2);
  p->err2_y = 0.01f;
  p->err2_z = 0.01f;
  p->max_sinphi = 0.95f;
  p->seed_c22 = 0.25f;
  p->seed_c33 = 0.25f;
  p->seed_c44 = 400.0f;
  p->reset_c00 = 1.0f;
  p->reset_c11 = 1.0f;
  p->pick_nsig = 3.0f;
  p->pick_win_max = 4.0f;
  p->pick_chi2 = 16.0f;
  p->max_miss = 10;
  p->min_track_hits = 10;
  p->own_frac_pct = 90;
  p->refit_inflate = 100.0f;
}

static bool valid_input(const tpcref_params_t *p, const float *row_x, const float *cl,
                        const uint8_t *row, int32_t n) {
  if (!p || !row_x || n < 0 || (n > 0 && (!cl || !row))) return false;
  if (p->n_rows < 3 || p->n_rows > 255) return false;
  if (n > 0xFFFFFF) return false; /* IDs must fit the 24 bits of the selection key */
  for (int32_t i = 0; i < n; ++i) {
    if (row[i] >= p->n_rows) return false;
    const float *c = cl + 4 * i;
    if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2])) return false;
    if (std::fabs(c[0] - row_x[row[i]]) > 1e-3f) return false;
  }
  return true;
}

void *tpcref_run(const tpcref_params_t *p, const float *row_x, const float *cl, const uint8_t *row,
                 int32_t n, int32_t precision, int32_t *err) {
  if (err) *err = 0;
  if (!valid_input(p, row_x, cl, row, n) || (precision != 32 && precision != 64)) {
    if (err) *err = -1;
    return nullptr;
  }
  if (precision == 32) return run<float>(*p, row_x, cl, row, n);
  return run<double>(*p, row_x, cl, row, n);
}

void tpcref_free(void *r) { delete static_cast<Result *>(r); }

int32_t tpcref_n_clusters(const void *r) { return static_cast<const Result *>(r)->n; }
int32_t tpcref_n_tracklets(const void *r) {
  return (int32_t) static_cast<const Result *>(r)->trk.size();
}
int32_t tpcref_n_tracks(const void *r) {
  return (int32_t) static_cast<const Result *>(r)->acc_index.size();
}
int64_t tpcref_n_tracklet_hits(const void *r) {
  int64_t s = 0;
  for (auto &v : static_cast<const Result *>(r)->trk_hits) s += (int64_t)v.size();
  return s;
}
int64_t tpcref_n_track_hits(const void *r) {
  int64_t s = 0;
  for (auto &v : static_cast<const Result *>(r)->acc_hits) s += (int64_t)v.size();
  return s;
}

void tpcref_get_links(const void *r, int32_t which, int32_t *up, int32_t *down) {
  const Result *R = static_cast<const Result *>(r);
  const auto &u = which ? R->upc : R->up;
  const auto &d = which ? R->dnc : R->dn;
  for (int i = 0; i < R->n; ++i) {
    if (up) up[i] = u[i];
    if (down) down[i] = d[i];
  }
}

void tpcref_get_tracklets(const void *r, tpcref_tracklet_t *out, int64_t *hit_begin,
                          int32_t *hits) {
  const Result *R = static_cast<const Result *>(r);
  int64_t off = 0;
  for (size_t t = 0; t < R->trk.size(); ++t) {
    if (out) out[t] = R->trk[t];
    if (hit_begin) hit_begin[t] = off;
    for (int h : R->trk_hits[t]) {
      if (hits) hits[off] = h;
      ++off;
    }
  }
  if (hit_begin) hit_begin[R->trk.size()] = off;
}

void tpcref_get_tracks(const void *r, int32_t *tracklet_index, int64_t *hit_begin, int32_t *hits) {
  const Result *R = static_cast<const Result *>(r);
  int64_t off = 0;
  for (size_t t = 0; t < R->acc_index.size(); ++t) {
    if (tracklet_index) tracklet_index[t] = R->acc_index[t];
    if (hit_begin) hit_begin[t] = off;
    for (int h : R->acc_hits[t]) {
      if (hits) hits[off] = h;
      ++off;
    }
  }
  if (hit_begin) hit_begin[R->acc_index.size()] = off;
}

void tpcref_get_assignment(const void *r, int32_t *a) {
  const Result *R = static_cast<const Result *>(r);
  for (int i = 0; i < R->n; ++i) a[i] = R->assign[i];
}

void tpcref_get_stats(const void *r, tpcref_stats_t *s) {
  const Result *R = static_cast<const Result *>(r);
  s->decisions = R->mg.decisions;
  s->near_ties = R->mg.near;
  s->min_margin = R->mg.min_margin;
  s->propagations = R->mg.props;
  s->tests = R->mg.tests;
  s->updates = R->mg.updates;
}

int32_t tpcref_refit(const tpcref_params_t *p, const float *row_x, const float *cl,
                     const uint8_t *row, const int32_t *hits, int32_t n_hits, int32_t k0,
                     int32_t n_chain, int32_t precision, tpcref_tracklet_t *out,
                     double *min_margin) {
  if (!p || !row_x || !cl || !row || !hits || !out || n_chain < 2 || k0 < 0 ||
      k0 + n_chain > n_hits)
    return -1;
  /* the sector is rebuilt from the hits only: enough for a replay */
  std::vector<float> c(4 * (size_t)n_hits);
  std::vector<uint8_t> r(n_hits);
  std::vector<int32_t> local(n_hits);
  for (int32_t k = 0; k < n_hits; ++k) {
    std::memcpy(&c[4 * (size_t)k], cl + 4 * (size_t)hits[k], 4 * sizeof(float));
    r[k] = row[hits[k]];
    local[k] = k;
  }
  if (precision == 32)
    return refit_impl<float>(*p, row_x, c.data(), r.data(), n_hits, local.data(), n_hits, k0,
                             n_chain, out, min_margin);
  if (precision == 64)
    return refit_impl<double>(*p, row_x, c.data(), r.data(), n_hits, local.data(), n_hits, k0,
                              n_chain, out, min_margin);
  return -1;
}

int32_t tpcref_propagate(const tpcref_params_t *p, int32_t precision, double *state, double *cov,
                         double *x, double x1) {
  if (precision == 32) {
    Par<float> P(*p);
    State<float> s;
    set_state(s, state, cov, *x);
    bool ok = propagate(P, s, (float)x1, nullptr);
    to_out(s, state, cov);
    *x = s.x;
    return ok ? 0 : -1;
  }
  Par<double> P(*p);
  State<double> s;
  set_state(s, state, cov, *x);
  bool ok = propagate(P, s, x1, nullptr);
  to_out(s, state, cov);
  *x = s.x;
  return ok ? 0 : -1;
}

int32_t tpcref_chi2(const tpcref_params_t *p, int32_t precision, const double *state,
                    const double *cov, double ym, double zm, double *chi2) {
  if (precision == 32) {
    Par<float> P(*p);
    State<float> s;
    set_state(s, state, cov, 0.0);
    float c = 0;
    bool ok = chi2_2d(P, s, (float)ym, (float)zm, c);
    *chi2 = c;
    return ok ? 0 : -1;
  }
  Par<double> P(*p);
  State<double> s;
  set_state(s, state, cov, 0.0);
  double c = 0;
  bool ok = chi2_2d(P, s, ym, zm, c);
  *chi2 = c;
  return ok ? 0 : -1;
}

int32_t tpcref_search_row(const tpcref_params_t *p, int32_t precision, const float *row_x,
                          const float *cl, const uint8_t *row, int32_t n, int32_t r,
                          const double *state, const double *cov, double zr) {
  if (!valid_input(p, row_x, cl, row, n) || r < 0 || r >= p->n_rows) return -2;
  if (precision == 32) {
    Par<float> P(*p);
    Sector<float> S(P, row_x, cl, row, n);
    State<float> s;
    set_state(s, state, cov, (double)row_x[r]);
    Margins mg;
    return search_row(S, s, (float)zr, r, mg);
  }
  Par<double> P(*p);
  Sector<double> S(P, row_x, cl, row, n);
  State<double> s;
  set_state(s, state, cov, (double)row_x[r]);
  Margins mg;
  return search_row(S, s, zr, r, mg);
}

int32_t tpcref_select(const tpcref_params_t *p, int32_t n_clusters, int32_t n_tracklets,
                      const int32_t *n_hits, const float *chi2, const int32_t *start_id,
                      const int32_t *status, const int64_t *hit_begin, const int32_t *hits,
                      int32_t *accepted, int32_t *assignment) {
  if (!p || n_clusters < 0 || n_tracklets < 0) return -1;
  Result R;
  R.n = n_clusters;
  for (int32_t t = 0; t < n_tracklets; ++t) {
    tpcref_tracklet_t o;
    std::memset(&o, 0, sizeof(o));
    o.n_hits = n_hits[t];
    o.chi2 = chi2[t];
    o.start_id = start_id[t];
    o.status = status[t];
    if (hit_begin[t + 1] - hit_begin[t] != n_hits[t]) return -1;
    std::vector<int> hl(hits + hit_begin[t], hits + hit_begin[t + 1]);
    for (int h : hl)
      if (h < 0 || h >= n_clusters) return -1;
    R.trk.push_back(o);
    R.trk_hits.push_back(std::move(hl));
  }
  select_tracks(p->min_track_hits, p->own_frac_pct, n_clusters, R);
  for (int32_t t = 0; t < n_tracklets; ++t) accepted[t] = -1;
  for (size_t k = 0; k < R.acc_index.size(); ++k) accepted[R.acc_index[k]] = (int32_t)k;
  for (int32_t i = 0; i < n_clusters; ++i) assignment[i] = R.assign[i];
  return (int32_t)R.acc_index.size();
}

int32_t tpcref_update(const tpcref_params_t *p, int32_t precision, double *state, double *cov,
                      double ym, double zm, double *chi2) {
  if (precision == 32) {
    Par<float> P(*p);
    State<float> s;
    set_state(s, state, cov, 0.0);
    float c = 0;
    bool ok = update(P, s, (float)ym, (float)zm, c);
    to_out(s, state, cov);
    *chi2 = c;
    return ok ? 0 : -1;
  }
  Par<double> P(*p);
  State<double> s;
  set_state(s, state, cov, 0.0);
  double c = 0;
  bool ok = update(P, s, ym, zm, c);
  to_out(s, state, cov);
  *chi2 = c;
  return ok ? 0 : -1;
}

}  // extern "C"
