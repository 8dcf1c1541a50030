/*
 * tpcphase2: plain CPU oracle of the steps after the sector tracker.
 * TEST INFRASTRUCTURE: only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it; it shares no code with the GPU
 * library.
 *
 * Rohr, LHCP 2017: Sec. 2 (second phase: merging of sector segments and
 * refit), Sec. 5 (vertex time from tracks found in the time coordinate),
 * Sec. 3 (track-model compression; rejection of clusters not used for
 * physics).  The paper gives these steps in prose only: every cut, formula
 * and tie-break below is a reading, stated next to the code that applies it.
 * The code is written to be checked by eye, not to be fast.
 *
 * Floating point as in tpcref.cpp: no contraction, no fast-math, std::fma
 * only where a reading prescribes it, correctly rounded / and sqrt.
 */
#include "tpcphase2.h"

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

template <typename F>
struct Par2 {
  F cs, sn, dz_ends, wy, wz, chi2, inflate, vdrift, gap_us, attach_us, qy, qz, c22, c33, c44,
      rej_qpt, rej_looper, rej_sin;
  int max_gap, dca_steps, vtx_min_tracks, vtx_min_hits;
  explicit Par2(const tpcref_p2params_t &q)
      : cs(q.sector_cos), sn(q.sector_sin), dz_ends(q.merge_dz_ends), wy(q.merge_wy),
        wz(q.merge_wz), chi2(q.merge_chi2), inflate(q.refit_inflate), vdrift(q.vdrift),
        gap_us(q.vtx_gap_us), attach_us(q.vtx_attach_us), qy(q.cmp_qy), qz(q.cmp_qz), c22(q.cmp_c22), c33(q.cmp_c33),
        c44(q.cmp_c44), rej_qpt(q.rej_qpt), rej_looper(q.rej_looper_qpt), rej_sin(q.rej_sinphi),
        max_gap(q.merge_max_gap), dca_steps(q.dca_steps), vtx_min_tracks(q.vtx_min_tracks),
        vtx_min_hits(q.vtx_min_hits) {}
};

/* Sectors 0..17 lie on the A side (z > 0), 18..35 on the C side; sector s is
   centred at ((s mod 18) + 1/2) * 20 degrees, so s and (s mod 18) + 1 on the
   same side are neighbours, the second one at the larger angle. */
int side_of(int s) { return s < 18 ? 0 : 1; }
int next_sector(int s) { return side_of(s) * 18 + ((s % 18) + 1) % 18; }
int prev_sector(int s) { return side_of(s) * 18 + ((s % 18) + 17) % 18; }

/*
 * Rotation of a state from the frame of a sector at angle alpha' into the
 * frame at alpha = alpha' - delta (cs = cos delta, sn = sin delta).  The
 * track point keeps its place: x = x' cs - y' sn, y = x' sn + y' cs, and
 * the direction turns by delta: sin phi = s' cs + c' sn,
 * cos phi = c' cs - s' sn with c' = sqrt(1 - s'^2) (the tracks run towards
 * larger x).  z, tan lambda and q/pT do not change.  The state then lies on
 * the plane x of the new frame; its covariance moves with the Jacobian of
 * this map at a fixed plane: a shift dy' of the point along the old plane
 * is a shift along the track of dl = sn dy' / cos phi back onto the new
 * plane, so dy = (c' / cos phi) dy', dz = (tan lambda sn / cos phi) dy' and
 * d sin phi = (cos phi / c') d sin phi'.  The curvature term of the turn
 * along dl (k sn dy' in d sin phi) is dropped, as the propagation's
 * Jacobian drops the curvature term of the arc length.  Fails if the track
 * would not cross the new plane towards larger x (cos phi <= 0) or
 * |sin phi| > max_sinphi.
 */
template <typename F>
bool rotate(const Par<F> &P, F cs, F sn, State<F> &st) {
  const F one = (F)1;
  const F x0 = st.x, y0 = st.p[0], s0 = st.p[2], t = st.p[3];
  const F c0 = std::sqrt(std::fma(-s0, s0, one));
  const F s1 = s0 * cs + c0 * sn;
  const F c1 = c0 * cs - s0 * sn;
  if (!(c1 > (F)0) || !(std::fabs(s1) <= P.max_sin)) return false;
  const F j00 = c0 / c1;
  const F j10 = t * sn / c1;
  const F j22 = c1 / c0;
  st.x = x0 * cs - y0 * sn;
  st.p[0] = x0 * sn + y0 * cs;
  st.p[2] = s1;
  F *C = st.C;
  const F c00 = C[0], c10 = C[1], c11 = C[2], c20 = C[3], c21 = C[4], c22 = C[5];
  const F c30 = C[6], c31 = C[7], c32 = C[8];
  const F c40 = C[10], c41 = C[11], c42 = C[12];
  /* C <- J C J^T for J = identity but J00, J10 (row z, column y), J22 */
  C[0] = j00 * j00 * c00;
  C[1] = j00 * (c10 + j10 * c00);
  C[2] = c11 + (F)2 * j10 * c10 + j10 * j10 * c00;
  C[3] = j22 * j00 * c20;
  C[4] = j22 * (c21 + j10 * c20);
  C[5] = j22 * j22 * c22;
  C[6] = j00 * c30;
  C[7] = c31 + j10 * c30;
  C[8] = j22 * c32;
  C[10] = j00 * c40;
  C[11] = c41 + j10 * c40;
  C[12] = j22 * c42;
  return true;
}

/* chi^2 = d^T (C1 + C2)^-1 d by a Cholesky factorisation S = L L^T (row by
   row, left to right), forward substitution L w = d and the sum of w_i^2 in
   index order.  Fails on a pivot that is not positive. */
template <typename F>
bool chi2_5(const F *d, const F *C1, const F *C2, F &chi2) {
  F L[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      F sum = C1[ci(i, j)] + C2[ci(i, j)];
      for (int k = 0; k < j; ++k) sum = sum - L[i][k] * L[j][k];
      if (i == j) {
        if (!(sum > (F)0)) return false;
        L[i][i] = std::sqrt(sum);
      } else {
        L[i][j] = sum / L[j][j];
      }
    }
  F w[5];
  for (int i = 0; i < 5; ++i) {
    F sum = d[i];
    for (int k = 0; k < i; ++k) sum = sum - L[i][k] * w[k];
    w[i] = sum / L[i][i];
  }
  F c = w[0] * w[0];
  for (int i = 1; i < 5; ++i) c = c + w[i] * w[i];
  chi2 = c;
  return true;
}

template <typename F>
struct Seg {
  int sector, start_id, n_hits;
  int64_t hb;          /* first hit in the hit list */
  int row_in, row_out; /* rows of the first and last won hit */
  F zr;                /* absolute z of the inner state (z reference of its end states) */
  State<F> in;         /* inner state, z relative to zr */
  bool out_ok;
  State<F> out;        /* outer end, z relative to zr */
  int64_t key() const { return ((int64_t)sector << 24) | start_id; }
};

template <typename F>
struct SlotData {
  const float *row_x;
  int n_sectors;
  const int64_t *sec_begin;
  const float *cl;
  const uint8_t *row;
  F y(int s, int id) const { return (F)cl[4 * (sec_begin[s] + id) + 1]; }
  F z(int s, int id) const { return (F)cl[4 * (sec_begin[s] + id) + 2]; }
  int r(int s, int id) const { return row[sec_begin[s] + id]; }
};

struct Result2 {
  std::vector<int> next, prev, final_of;
  std::vector<tpcref_final_t> finals;
  std::vector<int> seg_order;
  std::vector<int64_t> hit_begin;
  std::vector<int32_t> hits;
  std::vector<tpcref_vertex_t> vertices;
  std::vector<uint8_t> flags;
  std::vector<double> out_x, out_p, out_c;
  std::vector<int32_t> out_ok;
  int64_t pair_tests = 0;
  Margins mg;
};

/*
 * Outer end of a segment: its fitted state (at the tracklet's innermost hit,
 * where the fit ends) propagated, without updates, to the row of each of
 * its won hits in ascending order.  The fit has no process noise, so the
 * state at one end carries the information of every hit and its
 * propagation is the estimate at the other end.
 */
template <typename F>
void outer_end(const Par<F> &P, const SlotData<F> &D, const int32_t *hits, Seg<F> &g) {
  g.out = g.in;
  g.out_ok = true;
  for (int k = 0; k < g.n_hits; ++k) {
    const int r = D.r(g.sector, hits[g.hb + k]);
    if (!propagate(P, g.out, (F)D.row_x[r], nullptr)) {
      g.out_ok = false;
      return;
    }
  }
}

/*
 * Pair test (reading of Sec. 2's merging): A ends in sector s, B starts in a
 * neighbouring sector s' of the same side.  Candidates need
 *   1 <= row_in(B) - row_out(A) <= merge_max_gap and
 *   |z(B's inner state) - z(A's outer end)| <= merge_dz_ends (absolute z);
 * B's inner state is rotated into A's frame, A's outer end propagated to
 * that plane, and the difference d of the five parameters must satisfy
 * |d_y| <= merge_wy, |d_z| <= merge_wz and d^T (C_A + C_B)^-1 d <=
 * merge_chi2.  z is compared as (zr_B - zr_A) - z_A: each end keeps z
 * relative to its own segment's inner z (zr), and B's inner state sits at
 * relative z = 0.
 */
template <typename F>
bool pair_chi2(const Par<F> &P, const Par2<F> &Q, const Seg<F> &A, const Seg<F> &B, F &chi2,
               Margins &mg) {
  const F zA = A.out.p[1] + A.zr;
  if (!(std::fabs(B.zr - zA) <= Q.dz_ends)) return false;
  State<F> b = B.in;
  const F sn = next_sector(A.sector) == B.sector ? Q.sn : -Q.sn;
  if (!rotate(P, Q.cs, sn, b)) return false;
  State<F> a = A.out;
  if (!propagate(P, a, b.x, nullptr)) return false;
  F d[5];
  d[0] = b.p[0] - a.p[0];
  d[1] = (B.zr - A.zr) - a.p[1];
  d[2] = b.p[2] - a.p[2];
  d[3] = b.p[3] - a.p[3];
  d[4] = b.p[4] - a.p[4];
  if (!(std::fabs(d[0]) <= Q.wy) || !(std::fabs(d[1]) <= Q.wz)) return false;
  F c;
  if (!chi2_5(d, a.C, b.C, c)) return false;
  mg.note((double)c, (double)Q.chi2);
  if (!(c <= Q.chi2)) return false;
  chi2 = c;
  return true;
}

/* (chi2, key) lexicographic minimum */
template <typename F>
struct Best {
  F chi2 = std::numeric_limits<F>::infinity();
  int64_t key = std::numeric_limits<int64_t>::max();
  int idx = -1;
  void offer(F c, int64_t k, int i) {
    if (c < chi2 || (c == chi2 && k < key)) {
      chi2 = c;
      key = k;
      idx = i;
    }
  }
};

/*
 * Refit of a final track (reading of Sec. 2's "track refit"): a Kalman
 * filter inward through the won hits of all its segments, from the outer
 * end of the outermost segment with its covariance times refit_inflate (the
 * soft restart of the sector tracker's pass 2).  Inside a segment the state
 * is propagated from hit to hit and updated with each; between segments it
 * is rotated into the next inner segment's frame and propagated to that
 * segment's outermost hit.  z stays relative to the outermost segment's
 * inner z.  The result is the state at the innermost hit, the sum of the
 * updates' chi^2 and ndf = 2 n - 5.
 */
template <typename F>
void refit(const Par<F> &P, const Par2<F> &Q, const SlotData<F> &D, const int32_t *hits,
           const std::vector<Seg<F>> &S, const std::vector<int> &chain, tpcref_final_t &o,
           F &zr_out, State<F> &st_out) {
  o.status = 2;
  const Seg<F> &last = S[chain.back()];
  if (!last.out_ok) return;
  State<F> st = last.out;
  const F zr = last.zr;
  for (int k = 0; k < 15; ++k) st.C[k] = st.C[k] * Q.inflate;
  F chi2 = (F)0, c2;
  int n = 0, row_ref = -1;
  for (int m = (int)chain.size() - 1; m >= 0; --m) {
    const Seg<F> &g = S[chain[m]];
    if (m < (int)chain.size() - 1) {
      const Seg<F> &outer = S[chain[m + 1]];
      const F sn = next_sector(g.sector) == outer.sector ? Q.sn : -Q.sn;
      if (!rotate(P, Q.cs, sn, st)) return;
    }
    for (int k = g.n_hits - 1; k >= 0; --k) {
      const int id = hits[g.hb + k];
      const int r = D.r(g.sector, id);
      if (n > 0 && !propagate(P, st, (F)D.row_x[r], nullptr)) return;
      if (!update(P, st, D.y(g.sector, id), D.z(g.sector, id) - zr, c2)) return;
      chi2 = chi2 + c2;
      ++n;
      row_ref = r;
    }
  }
  o.status = 0;
  o.n_hits = n;
  o.ndf = 2 * n - 5;
  o.row_ref = row_ref;
  o.x_ref = (double)st.x;
  o.chi2 = (double)chi2;
  for (int k = 0; k < 5; ++k) o.p[k] = (double)st.p[k];
  o.p[1] = (double)(st.p[1] + zr);
  for (int k = 0; k < 15; ++k) o.cov[k] = (double)st.C[k];
  zr_out = zr;
  st_out = st;
}

/*
 * z at the beam axis (reading of Sec. 5): the refitted state is extrapolated
 * to the plane x = 0 of its sector frame, which holds the beam axis, in
 * dca_steps equal steps (x_k = x_ref (N - k) / N) of the tracker's
 * propagation (a step's arc stays short enough for its series).  For a track
 * from the beam axis this is its production z, in the time coordinate of
 * the input.  Fails where the propagation fails.
 */
template <typename F>
bool z_at_axis(const Par<F> &P, const Par2<F> &Q, State<F> st, F zr, F &z0) {
  const int N = Q.dca_steps;
  const F x0 = st.x;
  for (int k = 1; k <= N; ++k) {
    const F xk = (x0 * (F)(N - k)) / (F)N;
    if (!propagate(P, st, xk, nullptr)) return false;
  }
  z0 = st.p[1] + zr;
  return true;
}

/* Sort t0 estimates by (t0, key); consecutive estimates closer than gap
   join one group; groups of at least min_n members are vertices at the
   lower median of their members.  order receives the sorted positions. */
template <typename F>
std::vector<tpcref_vertex_t> vertex_groups(const std::vector<F> &t, const std::vector<int64_t> &key,
                                           F gap, int min_n, std::vector<int> &order, Margins &mg) {
  order.resize(t.size());
  for (size_t i = 0; i < t.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return t[a] < t[b] || (t[a] == t[b] && key[a] < key[b]);
  });
  std::vector<tpcref_vertex_t> out;
  for (size_t i = 0; i < order.size();) {
    size_t j = i + 1;
    while (j < order.size()) {
      const F d = t[order[j]] - t[order[j - 1]];
      mg.note((double)d, (double)gap);
      if (!(d <= gap)) break;
      ++j;
    }
    const int cnt = (int)(j - i);
    if (cnt >= min_n) {
      tpcref_vertex_t v;
      v.first = (int)i;
      v.n_tracks = cnt;
      v.t0 = (double)t[order[i + (size_t)(cnt - 1) / 2]];
      out.push_back(v);
    }
    i = j;
  }
  return out;
}

template <typename F>
Result2 *phase2(const tpcref_params_t &pp, const tpcref_p2params_t &qq, const float *row_x,
                int n_sectors, const int64_t *sec_begin, const float *cl, const uint8_t *row,
                int n_seg, const tpcref_segment_t *seg, const int64_t *seg_hit_begin,
                const int32_t *seg_hits, bool brute) {
  Par<F> P(pp);
  P.max_sin = (F)qq.max_sinphi; /* this phase's own limit */
  Par2<F> Q(qq);
  SlotData<F> D{row_x, n_sectors, sec_begin, cl, row};
  auto R = std::make_unique<Result2>();
  std::vector<Seg<F>> S(n_seg);
  for (int i = 0; i < n_seg; ++i) {
    const tpcref_segment_t &t = seg[i];
    Seg<F> &g = S[i];
    g.sector = t.sector;
    g.start_id = t.start_id;
    g.n_hits = t.n_hits;
    g.hb = seg_hit_begin[i];
    g.row_in = D.r(t.sector, seg_hits[g.hb]);
    g.row_out = D.r(t.sector, seg_hits[g.hb + g.n_hits - 1]);
    g.zr = (F)t.p[1];
    for (int k = 0; k < 5; ++k) g.in.p[k] = (F)t.p[k];
    g.in.p[1] = (F)0;
    for (int k = 0; k < 15; ++k) g.in.C[k] = (F)t.cov[k];
    g.in.x = (F)t.x_ref;
    outer_end(P, D, seg_hits, g);
  }
  /* per sector, the segments ordered by (inner z, key) for the z window */
  std::vector<std::vector<int>> by_z(n_sectors);
  for (int i = 0; i < n_seg; ++i) by_z[S[i].sector].push_back(i);
  for (auto &v : by_z)
    std::sort(v.begin(), v.end(), [&](int a, int b) {
      return S[a].zr < S[b].zr || (S[a].zr == S[b].zr && S[a].key() < S[b].key());
    });
  std::vector<Best<F>> bestB(n_seg), bestA(n_seg);
  for (int a = 0; a < n_seg; ++a) {
    const Seg<F> &A = S[a];
    if (!A.out_ok) continue;
    const F zA = A.out.p[1] + A.zr;
    for (int nb : {prev_sector(A.sector), next_sector(A.sector)}) {
      if (nb >= n_sectors || nb == A.sector) continue;
      const auto &v = by_z[nb];
      size_t k0 = 0, k1 = v.size();
      if (!brute) {
        /* a bracket a little wider than the window, in FP64; the exact
           test is pair_chi2's */
        const double pad = 1e-3 + 1e-6 * std::fabs((double)zA);
        const double lo = (double)zA - (double)Q.dz_ends - pad;
        const double hi = (double)zA + (double)Q.dz_ends + pad;
        k0 = (size_t)(std::lower_bound(v.begin(), v.end(), lo,
                                       [&](int i, double z) { return (double)S[i].zr < z; }) -
                      v.begin());
        k1 = (size_t)(std::upper_bound(v.begin(), v.end(), hi,
                                       [&](double z, int i) { return z < (double)S[i].zr; }) -
                      v.begin());
      }
      for (size_t k = k0; k < k1; ++k) {
        const int b = v[k];
        const Seg<F> &B = S[b];
        const int gap = B.row_in - A.row_out;
        if (gap < 1 || gap > Q.max_gap) continue;
        ++R->pair_tests;
        F c;
        if (!pair_chi2(P, Q, A, B, c, R->mg)) continue;
        bestB[a].offer(c, B.key(), b);
        bestA[b].offer(c, A.key(), a);
      }
    }
  }
  /* mutual best partners are merged */
  R->next.assign(n_seg, -1);
  R->prev.assign(n_seg, -1);
  for (int a = 0; a < n_seg; ++a) {
    const int b = bestB[a].idx;
    if (b >= 0 && bestA[b].idx == a) {
      R->next[a] = b;
      R->prev[b] = a;
    }
  }
  /* final tracks: chains of segments from those without an inner partner */
  R->final_of.assign(n_seg, -1);
  R->hit_begin.push_back(0);
  for (int i = 0; i < n_seg; ++i) {
    if (R->prev[i] >= 0) continue;
    std::vector<int> chain;
    for (int k = i; k >= 0; k = R->next[k]) chain.push_back(k);
    tpcref_final_t o;
    std::memset(&o, 0, sizeof(o));
    o.n_seg = (int)chain.size();
    o.seg_begin = (int)R->seg_order.size();
    o.sector = S[i].sector;
    o.vertex = -1;
    const int f = (int)R->finals.size();
    for (int k : chain) {
      R->seg_order.push_back(k);
      R->final_of[k] = f;
      for (int j = 0; j < S[k].n_hits; ++j)
        R->hits.push_back((S[k].sector << 24) | seg_hits[S[k].hb + j]);
    }
    R->hit_begin.push_back((int64_t)R->hits.size());
    F zr = (F)0;
    State<F> st{};
    refit(P, Q, D, seg_hits, S, chain, o, zr, st);
    if (o.status != 0) {
      o.n_hits = 0;
      for (int k : chain) o.n_hits += S[k].n_hits;
    }
    /* Sec. 5: z at the beam axis and the track's own vertex-time estimate;
       z' = z - v t0 on the A side and z + v t0 on the C side, so a track
       from the axis has t0 = -z0 / v (A) or z0 / v (C). */
    F z0 = (F)0;
    if (o.status == 0 && z_at_axis(P, Q, st, zr, z0)) {
      o.z0_ok = 1;
      o.z0 = (double)z0;
      const F t0 = side_of(o.sector) == 0 ? -z0 / Q.vdrift : z0 / Q.vdrift;
      o.t0 = (double)t0;
    }
    o.z_conv = o.p[1];
    R->finals.push_back(o);
  }
  /*
   * Vertices (reading of Sec. 5).  The t0 estimates of the refitted tracks
   * with at least vtx_min_hits hits and |q/pT| <= rej_looper_qpt (tracks
   * that cannot turn back inside the TPC, so their only leg starts at the
   * vertex) are sorted (ties by the innermost segment's key); consecutive
   * estimates closer than vtx_gap_us join one group, and a group of at least
   * vtx_min_tracks tracks is a vertex whose time is the lower median of its
   * members.  Every track with a t0 estimate then joins the nearest vertex
   * (the earlier one on a tie) if it lies within vtx_attach_us, and gets z
   * from z': z = z' + v t0 on the A side, z' - v t0 on the C side.
   */
  std::vector<int> cand;
  for (int f = 0; f < (int)R->finals.size(); ++f) {
    const auto &o = R->finals[f];
    if (o.status == 0 && o.z0_ok && o.n_hits >= Q.vtx_min_hits &&
        std::fabs((F)o.p[4]) <= Q.rej_looper)
      cand.push_back(f);
  }
  std::vector<F> tv;
  std::vector<int64_t> kv;
  for (int f : cand) {
    tv.push_back((F)R->finals[f].t0);
    kv.push_back(S[R->seg_order[R->finals[f].seg_begin]].key());
  }
  std::vector<int> order;
  R->vertices = vertex_groups(tv, kv, Q.gap_us, Q.vtx_min_tracks, order, R->mg);
  /* vertex times ascend with the groups; the nearest one by a plain scan */
  for (auto &o : R->finals) {
    if (!o.z0_ok) continue;
    const F t = (F)o.t0;
    int best = -1;
    F bd = (F)0;
    for (int v = 0; v < (int)R->vertices.size(); ++v) {
      const F d = std::fabs(t - (F)R->vertices[v].t0);
      if (best < 0 || d < bd) {
        best = v;
        bd = d;
      }
    }
    if (best < 0) continue;
    R->mg.note((double)bd, (double)Q.attach_us);
    if (!(bd <= Q.attach_us)) continue;
    o.vertex = best;
    const F shift = Q.vdrift * (F)R->vertices[best].t0;
    const F zp = (F)o.p[1];
    o.z_conv = (double)(side_of(o.sector) == 0 ? zp + shift : zp - shift);
  }
  /*
   * Rejection flags (reading of Sec. 3), per cluster of a final track:
   *   1  the track's |q/pT| > rej_qpt (pT below 50 MeV);
   *   2  a further leg of a looping track: |q/pT| > rej_looper_qpt (the
   *      circle turns back inside the TPC) and the track joined no vertex
   *      (a later leg extrapolates to the axis a full turn's z away from
   *      where the particle was produced);
   *   4  high inclination: the segment's local |sin phi| at the cluster's
   *      row, fma(kB q/pT, x_row - x_ref, sin phi) with the segment's own
   *      state, exceeds rej_sinphi.
   * q/pT is the refit's, or each segment's own where the refit failed.
   */
  const int64_t n_cl = sec_begin[n_sectors];
  R->flags.assign((size_t)n_cl, 0);
  for (int f = 0; f < (int)R->finals.size(); ++f) {
    const auto &o = R->finals[f];
    for (int m = 0; m < o.n_seg; ++m) {
      const Seg<F> &g = S[R->seg_order[o.seg_begin + m]];
      const F q = o.status == 0 ? (F)o.p[4] : g.in.p[4];
      uint8_t fl = 0;
      if (std::fabs(q) > Q.rej_qpt) fl |= 1;
      if (std::fabs(q) > Q.rej_looper && o.vertex < 0) fl |= 2;
      const F kk = P.kB * g.in.p[4];
      for (int j = 0; j < g.n_hits; ++j) {
        const int id = seg_hits[g.hb + j];
        const F dx = (F)D.row_x[D.r(g.sector, id)] - g.in.x;
        const F s = std::fma(kk, dx, g.in.p[2]);
        R->flags[(size_t)(sec_begin[g.sector] + id)] =
            (uint8_t)(fl | (std::fabs(s) > Q.rej_sin ? 4 : 0));
      }
    }
  }
  R->out_x.resize(n_seg);
  R->out_p.resize(5 * (size_t)n_seg);
  R->out_c.resize(15 * (size_t)n_seg);
  R->out_ok.resize(n_seg);
  for (int i = 0; i < n_seg; ++i) {
    R->out_ok[i] = S[i].out_ok ? 1 : 0;
    R->out_x[i] = (double)S[i].out.x;
    for (int k = 0; k < 5; ++k) R->out_p[5 * i + k] = (double)S[i].out.p[k];
    R->out_p[5 * i + 1] = (double)(S[i].out.p[1] + S[i].zr);
    for (int k = 0; k < 15; ++k) R->out_c[15 * i + k] = (double)S[i].out.C[k];
  }
  return R.release();
}

/* ------------------------------------------------------- compression --- */
/*
 * Track-model compression (reading of Sec. 3).  Stored coordinates are
 * integers: yq = rint(y / cmp_qy), zq = rint(z / cmp_qz) (FP32 division,
 * round half to even); their values are yd = yq * cmp_qy, zd = zq * cmp_qz.
 * A segment's record holds its first (innermost) won hit's row and (yq, zq)
 * and the segment's sin phi, tan lambda, q/pT as FP32.  The fit starts at
 * that hit with y = yd, z = 0 relative to zr = zd and C = diag(err2_y,
 * err2_z, cmp_c22, cmp_c33, cmp_c44); for every further hit, in ascending
 * rows, it propagates to the hit's row, predicts (y, z + zr), stores the
 * row step and the residuals yq - rint(y / cmp_qy), zq - rint(z / cmp_qz),
 * and updates with (yd, zd - zr).  A failed propagation leaves the state
 * where it was (the prediction is the previous state) and skips the update.
 * Decompression runs the same fit on the reconstructed values, so it
 * recovers every stored coordinate exactly.  A prediction beyond 2^30 steps
 * (a diverged fit) quantises to 0.
 */
int32_t quant(float v, float q) {
  const float r = std::nearbyint(v / q);
  return std::fabs(r) < 1073741824.0f ? (int32_t)r : 0;
}

uint32_t fbits(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}
float bitsf(uint32_t b) {
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

struct CmpFit {
  const Par<float> &P;
  const Par2<float> &Q;
  const float *row_x;
  State<float> st;
  float zr;
  void start(int row0, int32_t yq0, int32_t zq0, float s, float t, float qpt) {
    st.x = row_x[row0];
    st.p[0] = (float)yq0 * Q.qy;
    zr = (float)zq0 * Q.qz;
    st.p[1] = 0.0f;
    st.p[2] = s;
    st.p[3] = t;
    st.p[4] = qpt;
    for (int k = 0; k < 15; ++k) st.C[k] = 0.0f;
    st.C[0] = P.ery;
    st.C[2] = P.erz;
    st.C[5] = Q.c22;
    st.C[9] = Q.c33;
    st.C[14] = Q.c44;
  }
  /* propagate to row r and return the quantised prediction */
  bool predict(int r, int32_t &py, int32_t &pz) {
    const bool ok = propagate(P, st, row_x[r], nullptr);
    py = quant(st.p[0], Q.qy);
    pz = quant(st.p[1] + zr, Q.qz);
    return ok;
  }
  void take(bool ok, int32_t yq, int32_t zq) {
    if (!ok) return;
    float c2;
    (void)update(P, st, (float)yq * Q.qy, (float)zq * Q.qz - zr, c2);
  }
};

}  // namespace

extern "C" {

void tpcref_p2params_default(tpcref_p2params_t *q) {
  const double w = 20.0 * 3.14159265358979323846 / 180.0;
  q->sector_cos = (float)std::cos(w);
  q->sector_sin = (float)std::sin(w);
  q->max_sinphi = 0.99f;
  q->merge_dz_ends = 40.0f;
  q->merge_max_gap = 10;
  q->merge_wy = 4.0f;
  q->merge_wz = 4.0f;
  q->merge_chi2 = 50.0f;
  q->refit_inflate = 100.0f;
  q->dca_steps = 16;
  q->vdrift = 2.58f;
  q->vtx_gap_us = 0.1f;
  q->vtx_min_tracks = 3;
  q->vtx_min_hits = 20;
  q->vtx_attach_us = 0.25f;
  q->cmp_qy = 0.01f;
  q->cmp_qz = 0.01f;
  q->cmp_c22 = 1e-4f;
  q->cmp_c33 = 1e-4f;
  q->cmp_c44 = 1.0f;
  q->rej_qpt = 20.0f;
  q->rej_looper_qpt = 5.4f;
  q->rej_sinphi = 0.8f;
}

void *tpcref_phase2(const tpcref_params_t *p, const tpcref_p2params_t *q, const float *row_x,
                    int32_t n_sectors, const int64_t *sec_begin, const float *cl,
                    const uint8_t *row, int32_t n_seg, const tpcref_segment_t *seg,
                    const int64_t *seg_hit_begin, const int32_t *seg_hits, int32_t precision,
                    int32_t brute) {
  if (!p || !q || !row_x || !sec_begin || n_sectors < 1 || n_sectors > 36 || n_seg < 0) return nullptr;
  if (n_seg > 0 && (!seg || !seg_hit_begin || !seg_hits || !cl || !row)) return nullptr;
  for (int32_t i = 0; i < n_seg; ++i) {
    const auto &t = seg[i];
    if (t.sector < 0 || t.sector >= n_sectors || t.n_hits < 1) return nullptr;
    if (seg_hit_begin[i + 1] - seg_hit_begin[i] != t.n_hits) return nullptr;
    const int64_t n_s = sec_begin[t.sector + 1] - sec_begin[t.sector];
    int prev_row = -1;
    for (int64_t k = seg_hit_begin[i]; k < seg_hit_begin[i + 1]; ++k) {
      if (seg_hits[k] < 0 || seg_hits[k] >= n_s) return nullptr;
      const int r = row[sec_begin[t.sector] + seg_hits[k]];
      if (r <= prev_row || r >= p->n_rows) return nullptr;
      prev_row = r;
    }
  }
  if (precision == 32)
    return phase2<float>(*p, *q, row_x, n_sectors, sec_begin, cl, row, n_seg, seg, seg_hit_begin,
                         seg_hits, brute != 0);
  if (precision == 64)
    return phase2<double>(*p, *q, row_x, n_sectors, sec_begin, cl, row, n_seg, seg, seg_hit_begin,
                          seg_hits, brute != 0);
  return nullptr;
}

void tpcref_phase2_free(void *r) { delete static_cast<Result2 *>(r); }

int32_t tpcref_p2_n_final(const void *r) {
  return (int32_t) static_cast<const Result2 *>(r)->finals.size();
}
int32_t tpcref_p2_n_vertices(const void *r) {
  return (int32_t) static_cast<const Result2 *>(r)->vertices.size();
}
int64_t tpcref_p2_n_final_hits(const void *r) {
  return (int64_t) static_cast<const Result2 *>(r)->hits.size();
}

void tpcref_p2_links(const void *r, int32_t *next, int32_t *prev, int32_t *final_of_seg) {
  const Result2 *R = static_cast<const Result2 *>(r);
  for (size_t i = 0; i < R->next.size(); ++i) {
    if (next) next[i] = R->next[i];
    if (prev) prev[i] = R->prev[i];
    if (final_of_seg) final_of_seg[i] = R->final_of[i];
  }
}

void tpcref_p2_finals(const void *r, tpcref_final_t *out, int32_t *seg_order, int64_t *hit_begin,
                      int32_t *hits) {
  const Result2 *R = static_cast<const Result2 *>(r);
  for (size_t f = 0; f < R->finals.size(); ++f)
    if (out) out[f] = R->finals[f];
  if (seg_order)
    for (size_t k = 0; k < R->seg_order.size(); ++k) seg_order[k] = R->seg_order[k];
  if (hit_begin)
    for (size_t k = 0; k < R->hit_begin.size(); ++k) hit_begin[k] = R->hit_begin[k];
  if (hits)
    for (size_t k = 0; k < R->hits.size(); ++k) hits[k] = R->hits[k];
}

void tpcref_p2_vertices(const void *r, tpcref_vertex_t *out) {
  const Result2 *R = static_cast<const Result2 *>(r);
  for (size_t k = 0; k < R->vertices.size(); ++k) out[k] = R->vertices[k];
}

void tpcref_p2_flags(const void *r, uint8_t *flags) {
  const Result2 *R = static_cast<const Result2 *>(r);
  for (size_t k = 0; k < R->flags.size(); ++k) flags[k] = R->flags[k];
}

void tpcref_p2_outer(const void *r, double *x, double *p, double *cov, int32_t *ok) {
  const Result2 *R = static_cast<const Result2 *>(r);
  for (size_t i = 0; i < R->out_ok.size(); ++i) {
    if (x) x[i] = R->out_x[i];
    if (ok) ok[i] = R->out_ok[i];
    for (int k = 0; k < 5 && p; ++k) p[5 * i + k] = R->out_p[5 * i + k];
    for (int k = 0; k < 15 && cov; ++k) cov[15 * i + k] = R->out_c[15 * i + k];
  }
}

void tpcref_p2_stats(const void *r, int64_t *pair_tests, int64_t *near_ties, double *min_margin) {
  const Result2 *R = static_cast<const Result2 *>(r);
  if (pair_tests) *pair_tests = R->pair_tests;
  if (near_ties) *near_ties = R->mg.near;
  if (min_margin) *min_margin = R->mg.min_margin;
}

int32_t tpcref_compress(const tpcref_params_t *p, const tpcref_p2params_t *q, const float *row_x,
                        const float *cl, const uint8_t *row, int32_t n_seg,
                        const tpcref_segment_t *seg, const int64_t *seg_hit_begin,
                        const int32_t *seg_hits, int32_t precision, int32_t *rec, int32_t *res) {
  if (!p || !q || !row_x || precision != 32 || n_seg < 0) return -1;
  Par<float> P(*p);
  P.max_sin = q->max_sinphi;
  Par2<float> Q(*q);
  for (int32_t i = 0; i < n_seg; ++i) {
    const int64_t hb = seg_hit_begin[i], he = seg_hit_begin[i + 1];
    if (he <= hb) return -1;
    const int h0 = seg_hits[hb];
    const int row0 = row[h0];
    const int32_t yq0 = quant(cl[4 * h0 + 1], Q.qy), zq0 = quant(cl[4 * h0 + 2], Q.qz);
    const float s = (float)seg[i].p[2], t = (float)seg[i].p[3], qpt = (float)seg[i].p[4];
    int32_t *rc = rec + 6 * (size_t)i;
    rc[0] = row0;
    rc[1] = yq0;
    rc[2] = zq0;
    rc[3] = (int32_t)fbits(s);
    rc[4] = (int32_t)fbits(t);
    rc[5] = (int32_t)fbits(qpt);
    CmpFit fit{P, Q, row_x, {}, 0.0f};
    fit.start(row0, yq0, zq0, s, t, qpt);
    int prev = row0;
    res[3 * hb] = res[3 * hb + 1] = res[3 * hb + 2] = 0;
    for (int64_t k = hb + 1; k < he; ++k) {
      const int h = seg_hits[k];
      const int r = row[h];
      if (r <= prev) return -1;
      int32_t py, pz;
      const bool ok = fit.predict(r, py, pz);
      const int32_t yq = quant(cl[4 * h + 1], Q.qy), zq = quant(cl[4 * h + 2], Q.qz);
      res[3 * k] = r - prev;
      res[3 * k + 1] = yq - py;
      res[3 * k + 2] = zq - pz;
      fit.take(ok, yq, zq);
      prev = r;
    }
  }
  return 0;
}

int32_t tpcref_decompress(const tpcref_params_t *p, const tpcref_p2params_t *q,
                          const float *row_x, int32_t n_seg, const int32_t *n_hits,
                          const int32_t *rec, const int32_t *res, int32_t precision,
                          int32_t *yq, int32_t *zq, uint8_t *rows) {
  if (!p || !q || !row_x || precision != 32 || n_seg < 0) return -1;
  Par<float> P(*p);
  P.max_sin = q->max_sinphi;
  Par2<float> Q(*q);
  int64_t hb = 0;
  for (int32_t i = 0; i < n_seg; ++i) {
    const int32_t *rc = rec + 6 * (size_t)i;
    CmpFit fit{P, Q, row_x, {}, 0.0f};
    int r = rc[0];
    fit.start(r, rc[1], rc[2], bitsf((uint32_t)rc[3]), bitsf((uint32_t)rc[4]),
              bitsf((uint32_t)rc[5]));
    yq[hb] = rc[1];
    zq[hb] = rc[2];
    rows[hb] = (uint8_t)r;
    for (int32_t k = 1; k < n_hits[i]; ++k) {
      const int64_t j = hb + k;
      r += res[3 * j];
      if (r >= p->n_rows) return -1;
      int32_t py, pz;
      const bool ok = fit.predict(r, py, pz);
      yq[j] = res[3 * j + 1] + py;
      zq[j] = res[3 * j + 2] + pz;
      rows[j] = (uint8_t)r;
      fit.take(ok, yq[j], zq[j]);
    }
    hb += n_hits[i];
  }
  return 0;
}

int32_t tpcref_rotate(const tpcref_params_t *p, int32_t precision, double cs, double sn,
                      double *state, double *cov, double *x) {
  if (precision == 32) {
    Par<float> P(*p);
    State<float> s;
    for (int k = 0; k < 5; ++k) s.p[k] = (float)state[k];
    for (int k = 0; k < 15; ++k) s.C[k] = (float)cov[k];
    s.x = (float)*x;
    const bool ok = rotate(P, (float)cs, (float)sn, s);
    for (int k = 0; k < 5; ++k) state[k] = s.p[k];
    for (int k = 0; k < 15; ++k) cov[k] = s.C[k];
    *x = s.x;
    return ok ? 0 : -1;
  }
  Par<double> P(*p);
  State<double> s;
  for (int k = 0; k < 5; ++k) s.p[k] = state[k];
  for (int k = 0; k < 15; ++k) s.C[k] = cov[k];
  s.x = *x;
  const bool ok = rotate(P, cs, sn, s);
  for (int k = 0; k < 5; ++k) state[k] = s.p[k];
  for (int k = 0; k < 15; ++k) cov[k] = s.C[k];
  *x = s.x;
  return ok ? 0 : -1;
}

int32_t tpcref_z0(const tpcref_params_t *p, const tpcref_p2params_t *q, int32_t precision,
                  const double *state, double x, double zr, double *z0) {
  if (!p || !q || !state || !z0) return -1;
  if (precision == 32) {
    Par<float> P(*p);
    P.max_sin = q->max_sinphi;
    Par2<float> Q(*q);
    State<float> s{};
    for (int k = 0; k < 5; ++k) s.p[k] = (float)state[k];
    s.x = (float)x;
    float z = 0;
    const bool ok = z_at_axis(P, Q, s, (float)zr, z);
    *z0 = z;
    return ok ? 0 : -1;
  }
  Par<double> P(*p);
  P.max_sin = q->max_sinphi;
  Par2<double> Q(*q);
  State<double> s{};
  for (int k = 0; k < 5; ++k) s.p[k] = state[k];
  s.x = x;
  double z = 0;
  const bool ok = z_at_axis(P, Q, s, zr, z);
  *z0 = z;
  return ok ? 0 : -1;
}

int32_t tpcref_vertex_groups(int32_t n, const double *t0, const int64_t *key, double gap,
                             int32_t min_n, int32_t *group_of, tpcref_vertex_t *out) {
  if (n < 0 || (n > 0 && (!t0 || !key || !group_of))) return -1;
  std::vector<float> t(t0, t0 + n);
  std::vector<int64_t> k(key, key + n);
  std::vector<int> order;
  Margins mg;
  auto v = vertex_groups(t, k, (float)gap, min_n, order, mg);
  for (int32_t i = 0; i < n; ++i) group_of[i] = -1;
  for (size_t g = 0; g < v.size(); ++g) {
    for (int m = 0; m < v[g].n_tracks; ++m) group_of[order[(size_t)v[g].first + m]] = (int32_t)g;
    if (out) out[g] = v[g];
  }
  return (int32_t)v.size();
}

int32_t tpcref_chi2_5(int32_t precision, const double *d, const double *c1, const double *c2,
                      double *chi2) {
  if (precision == 32) {
    float df[5], a[15], b[15], c = 0;
    for (int k = 0; k < 5; ++k) df[k] = (float)d[k];
    for (int k = 0; k < 15; ++k) {
      a[k] = (float)c1[k];
      b[k] = (float)c2[k];
    }
    const bool ok = chi2_5(df, a, b, c);
    *chi2 = c;
    return ok ? 0 : -1;
  }
  double c = 0;
  const bool ok = chi2_5(d, c1, c2, c);
  *chi2 = c;
  return ok ? 0 : -1;
}

}  // extern "C"
