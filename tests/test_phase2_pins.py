"""Pins of the second-phase oracle (oracle/tpcphase2.cpp) against facts that
do not come from it.

Rohr, LHCP 2017: Sec. 2 (merging of the sector segments into final tracks
and their refit), Sec. 5 (vertex times from tracks found in the time
coordinate), Sec. 3 (track-model compression; rejection of clusters not
used for physics).  The paper prints no worked example, so:
  * rotation       - the generator's exact helix crossings in two sector
                     frames, and a finite-difference Jacobian at B = 0;
  * pair chi^2     - a linear solve of the same system;
  * merging        - Monte-Carlo truth (exact for noise-free helices) and a
                     brute-force pairing without the z window;
  * refit          - nonlinear least squares of straight lines across two
                     sectors (B = 0) and pull distributions of merged tracks;
  * z at the axis  - the production z of exact truth states;
  * vertices       - connected components by brute force, the generator's
                     event times;
  * compression    - exact round trip, residual spread of the measurement
                     model, entropy below that of absolute coordinates;
  * rejection      - truth legs and truth inclination.
"""
import math

import numpy as np
import pytest

import oracle
import tpcgen
from tests import _slots

F32 = np.float32
SIN20 = float(F32(math.sin(math.radians(20.0))))
COS20 = float(F32(math.cos(math.radians(20.0))))
ALPHA = [((s % 18) + 0.5) * math.radians(20.0) for s in range(36)]


def _adjacent(sa, sb):
    return sa // 18 == sb // 18 and ((sb % 18) - (sa % 18)) % 18 in (1, 17)


def _crossings(ev):
    """Consecutive crossings (row r in sector sa, row r' in sector sb) of one
    track's outgoing first half-turn across a sector boundary."""
    t, row, sec = ev.truth, ev.row, ev.sector
    ok = np.nonzero((t["track"] >= 0) & (t["leg"] == 0) & (t["branch"] == 0))[0]
    out = []
    by = {}
    for i in ok:
        by.setdefault(int(t["track"][i]), []).append(i)
    for ids in by.values():
        ids = sorted(ids, key=lambda i: row[i])
        for a, b in zip(ids[:-1], ids[1:]):
            if sec[a] != sec[b] and _adjacent(int(sec[a]), int(sec[b])) and row[b] > row[a]:
                out.append((a, b))
    return out


# --------------------------------------------------------------- rotation ---
@pytest.mark.parametrize("bz", [0.5, -0.5])
def test_rotation_moves_exact_states_between_sector_frames(row_x, bz):
    """The truth state of a noise-free helix at its first row in the next
    sector, rotated into the previous sector's frame and propagated (FP64,
    pinned to the exact crossings) to the last row there, is the truth state
    at that row."""
    ev = tpcgen.make_event(seed=21, stream=31, n_tracks=600, sigma=0.0, bz=bz)
    P = oracle.default_params(kB=float(F32(-bz * 0.299792458e-2)), max_sinphi=0.99)
    pairs = _crossings(ev)
    assert len(pairs) > 200
    t = ev.truth
    worst = 0.0
    for a, b in pairs:
        sa, sb = int(ev.sector[a]), int(ev.sector[b])
        sn = SIN20 if (sb % 18) == (sa % 18 + 1) % 18 else -SIN20
        state = [t["y"][b], t["z"][b], t["sinphi"][b], t["tanl"][b], t["qpt"][b]]
        rc, s1, _, x1 = oracle.rotate(state, np.eye(5)[np.tril_indices(5)], float(row_x[ev.row[b]]),
                                      math.cos(math.radians(20.0)), math.copysign(math.sin(math.radians(20.0)), sn),
                                      P, 64)
        if rc != 0:
            continue
        rc, s2, _, _ = oracle.propagate(s1, np.eye(5)[np.tril_indices(5)], x1, float(row_x[ev.row[a]]), P, 64)
        if rc != 0:
            continue
        for got, want in ((s2[0], t["y"][a]), (s2[1], t["z"][a]), (s2[2], t["sinphi"][a])):
            worst = max(worst, abs(got - want) / max(abs(want), 1.0))
        assert s2[3] == t["tanl"][a] and s2[4] == t["qpt"][a]
    assert worst <= 1e-8, worst


def _spd(rng, d):
    a = rng.normal(size=(5, 5)) * d[None, :]
    return a.T @ a + np.diag(d * d)


def test_rotation_covariance_matches_numeric_jacobian(row_x):
    """At B = 0 (where the dropped curvature term vanishes) the rotated
    covariance is J C J^T for the Jacobian of rotation followed by the exact
    straight-line move back to the nominal plane, by central differences."""
    rng = np.random.default_rng(3)
    P = oracle.default_params(kB=0.0, max_sinphi=0.99)
    for case in range(40):
        x = float(row_x[rng.integers(0, 159)])
        sgn = 1.0 if case % 2 else -1.0
        state = np.array([sgn * rng.uniform(0.5, 1.0) * x * math.tan(math.radians(10)), rng.uniform(-200, 200),
                          rng.uniform(-0.6, 0.6), rng.uniform(-1, 1), rng.uniform(-5, 5)])
        cs, sn = math.cos(math.radians(20)), sgn * math.sin(math.radians(20))
        C = _spd(rng, np.array([0.05, 0.05, 0.002, 0.002, 0.05]))
        c15 = oracle.cov_lower(C)
        rc, s0, got, xn = oracle.rotate(state, c15, x, cs, sn, P, 64)
        assert rc == 0
        J = np.zeros((5, 5))
        for j in range(5):
            h = 1e-6 * max(1.0, abs(state[j]))
            out = []
            for d in (h, -h):
                st = state.copy()
                st[j] += d
                rc, s1, _, x1 = oracle.rotate(st, c15, x, cs, sn, P, 64)
                rc2, s2, _, _ = oracle.propagate(s1, c15, x1, xn, P, 64)
                assert rc == 0 and rc2 == 0
                out.append(s2)
            J[:, j] = (out[0] - out[1]) / (2 * h)
        want = J @ C @ J.T
        d = np.sqrt(np.diag(want))
        err = np.abs(oracle.cov_matrix(got) - want) / np.outer(d, d)
        assert err.max() <= 1e-6, err.max()


def test_pair_chi2_equals_linear_solve():
    rng = np.random.default_rng(5)
    for _ in range(200):
        C1 = _spd(rng, rng.uniform(0.01, 1, 5))
        C2 = _spd(rng, rng.uniform(0.01, 1, 5))
        d = rng.normal(size=5) * 0.3
        want = d @ np.linalg.solve(C1 + C2, d)
        rc, got = oracle.chi2_5(d, oracle.cov_lower(C1), oracle.cov_lower(C2), 64)
        assert rc == 0 and abs(got - want) <= 1e-10 * max(1.0, want)
        rc, got32 = oracle.chi2_5(d, oracle.cov_lower(C1), oracle.cov_lower(C2), 32)
        assert rc == 0 and abs(got32 - want) <= 1e-3 * max(1.0, want)
    bad = -np.eye(5)[np.tril_indices(5)]
    assert oracle.chi2_5(np.ones(5), bad, bad, 64)[0] != 0


# ---------------------------------------------------------------- merging ---
def _segment_labels(trs, seg, hb, hits, pure=False):
    """(track, leg) majority label of every segment, -1 for noise-led ones
    (pure: -1 unless every hit carries the label)."""
    lab = np.full(seg.shape[0], -1, np.int64)
    for i in range(seg.shape[0]):
        tr = trs[seg[i]["sector"]]
        h = hits[hb[i]:hb[i + 1]]
        k = np.where(tr["track"][h] >= 0, tr["track"][h].astype(np.int64) * 8 + tr["leg"][h], -1)
        v, c = np.unique(k, return_counts=True)
        if not pure or v.shape[0] == 1:
            lab[i] = v[np.argmax(c)]
    return lab


def _true_pairs(rows, seg, hb, hits, lab, max_gap=10):
    out = set()
    by = {}
    for i, l in enumerate(lab):
        if l >= 0:
            by.setdefault(int(l), []).append(i)
    for v in by.values():
        for a in v:
            for b in v:
                sa, sb = int(seg[a]["sector"]), int(seg[b]["sector"])
                if a == b or not _adjacent(sa, sb):
                    continue
                gap = int(rows[sb][hits[hb[b]]]) - int(rows[sa][hits[hb[a + 1] - 1]])
                if 1 <= gap <= max_gap:
                    out.add((a, b))
    return out


def test_merge_exact_recovery_noise_free(row_x):
    """Noise-free helices: every pair of pure segments (all hits from one
    track) of one track that meets the candidate rules is merged, and no
    merge joins segments led by different tracks."""
    ev = tpcgen.make_event(seed=7, stream=41, n_tracks=3000, sigma=0.0)
    cls, rows, trs = _slots.event_arrays(ev)
    _, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x)
    pairs = _true_pairs(rows, seg, hb, hits, _segment_labels(trs, seg, hb, hits, pure=True))
    assert len(pairs) > 1000
    lab = _segment_labels(trs, seg, hb, hits)
    merged = {(a, int(b)) for a, b in enumerate(r.next) if b >= 0}
    assert pairs <= merged, len(pairs - merged)
    assert all(lab[a] == lab[b] and lab[a] >= 0 for a, b in merged)


def test_merge_with_smearing(row_x):
    """Central event (sigma 0.1 cm, loopers, noise): >= 99 % of the true
    pairs merged, no merge of segments of different particles."""
    b = tpcgen.central_event(seed=1)
    cls, rows, trs = _slots.slot_arrays(b.cl, b.row, b.units, b.truth)
    _, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x)
    lab = _segment_labels(trs, seg, hb, hits)
    pairs = _true_pairs(rows, seg, hb, hits, lab)
    merged = {(a, int(b)) for a, b in enumerate(r.next) if b >= 0}
    wrong = [(a, b) for a, b in merged if lab[a] != lab[b] or lab[a] < 0]
    assert not wrong
    assert len(merged & pairs) >= 0.99 * len(pairs), (len(merged & pairs), len(pairs))
    print(f"\ncentral event: {seg.shape[0]} segments, {r.finals.shape[0]} final tracks, "
          f"{len(merged)} merges of {len(pairs)} true pairs, near-ties {r.near_ties}")


def test_windowed_pairing_equals_brute_force(row_x):
    b = tpcgen.central_event(seed=2, n_tracks=4000)
    cls, rows, _ = _slots.slot_arrays(b.cl, b.row, b.units)
    res, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x)
    _, _, _, _, rb = _slots.run_slot(cls, rows, row_x, brute=True, results=res)
    assert np.array_equal(r.next, rb.next) and np.array_equal(r.prev, rb.prev)
    assert r.finals.tobytes() == rb.finals.tobytes()
    assert rb.pair_tests > r.pair_tests


def test_second_phase_invariants(row_x):
    b = tpcgen.central_event(seed=3, n_tracks=4000)
    cls, rows, _ = _slots.slot_arrays(b.cl, b.row, b.units)
    res, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x)
    n = seg.shape[0]
    # every segment in exactly one final track, chains follow next links
    assert np.array_equal(np.sort(r.seg_order), np.arange(n))
    firsts = []
    for f, o in enumerate(r.finals):
        chain = r.seg_order[o["seg_begin"]:o["seg_begin"] + o["n_seg"]]
        assert np.all(r.final_of_seg[chain] == f)
        assert r.prev[chain[0]] == -1 and r.next[chain[-1]] == -1
        for a, c in zip(chain[:-1], chain[1:]):
            assert r.next[a] == c and r.prev[c] == a
            sa, sc = int(seg[a]["sector"]), int(seg[c]["sector"])
            assert _adjacent(sa, sc)
            assert rows[sc][hits[hb[c]]] > rows[sa][hits[hb[a + 1] - 1]]
        want = np.concatenate([(int(seg[k]["sector"]) << 24) | hits[hb[k]:hb[k + 1]] for k in chain])
        assert np.array_equal(r.hits[r.hit_begin[f]:r.hit_begin[f + 1]], want)
        assert o["sector"] == seg[chain[0]]["sector"]
        firsts.append(chain[0])
        if o["status"] == 0:
            assert o["n_hits"] == want.shape[0] and o["ndf"] == 2 * o["n_hits"] - 5
    assert firsts == sorted(firsts)
    # a merged track is inside one side, and every cluster is in one track
    allh = r.hits
    assert np.unique(allh).shape[0] == allh.shape[0]


def _line_event(rng, row_x, n_lines=60, sigma=0.1):
    """Straight lines (no field) that start near radius 70 cm and cross one
    sector boundary, with their clusters in each sector's frame.  Returns
    per-sector lists and, per line, (global point, direction angle, z0, tan
    lambda)."""
    cls = [[] for _ in range(36)]
    rows = [[] for _ in range(36)]
    lines = []
    tan10 = math.tan(math.radians(10))
    for k in range(n_lines):
        edge = (k % 18) * math.radians(20)  # boundary between sectors k-1 and k (A side)
        r0 = 70.0
        phi_p = edge - math.radians(rng.uniform(2.0, 8.0))
        X0, Y0 = r0 * math.cos(phi_p), r0 * math.sin(phi_p)
        psi = edge + math.radians(rng.uniform(4.0, 12.0))
        z0, tl = rng.uniform(10, 60), rng.uniform(0.05, 0.6)
        lines.append((X0, Y0, psi, z0, tl))
        for s in range(18):
            a = ALPHA[s]
            x0s = X0 * math.cos(a) + Y0 * math.sin(a)
            y0s = -X0 * math.sin(a) + Y0 * math.cos(a)
            cp, sp = math.cos(psi - a), math.sin(psi - a)
            if cp <= 0.2:
                continue
            for r in range(159):
                xr = float(row_x[r])
                l = (xr - x0s) / cp
                if l <= 0:
                    continue
                y = y0s + l * sp
                if abs(y) > xr * tan10:
                    continue
                z = z0 + tl * l
                if z > 250:
                    continue
                cls[s].append([xr, y + sigma * rng.normal(), z + sigma * rng.normal(), 100.0])
                rows[s].append(r)
    cls = [np.array(c, np.float32).reshape(-1, 4) for c in cls]
    rows = [np.array(r, np.uint8) for r in rows]
    return cls, rows, lines


def _line_frame_state(theta, x_ref, s1, s, x):
    """State (y, z, sin phi, tan lambda) at plane x of sector s of the line
    given by theta = (y, z, sin phi, tan lambda) at plane x_ref of sector
    s1, through global coordinates."""
    y, z, sp, tl = theta
    a1 = ALPHA[s1]
    X = x_ref * math.cos(a1) - y * math.sin(a1)
    Y = x_ref * math.sin(a1) + y * math.cos(a1)
    psi = a1 + math.asin(sp)
    a = ALPHA[s]
    xs = X * math.cos(a) + Y * math.sin(a)
    ys = -X * math.sin(a) + Y * math.cos(a)
    cp, spp = math.cos(psi - a), math.sin(psi - a)
    l = (x - xs) / cp
    return np.array([ys + l * spp, z + tl * l, spp, tl])


def test_refit_across_sectors_equals_least_squares(row_x):
    """B = 0: straight lines crossing a sector boundary.  The refit of a
    merged track is the maximum of its posterior: least squares over every
    hit, each measured in its own sector's frame, plus the refit's Gaussian
    prior (the outermost segment's outer end, covariance times
    refit_inflate), solved by Gauss-Newton on the exact geometry in FP64."""
    rng = np.random.default_rng(11)
    cls, rows, lines = _line_event(rng, row_x)
    P = oracle.default_params(kB=0.0)
    Q = oracle.default_p2params()
    res, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x, P, Q, precision=64)
    checked = 0
    worst = 0.0
    for f, o in enumerate(r.finals):
        if o["n_seg"] < 2 or o["status"] != 0:
            continue
        h = r.hits[r.hit_begin[f]:r.hit_begin[f + 1]]
        sec, cid = h >> 24, h & 0xFFFFFF
        s1 = int(o["sector"])
        last = r.seg_order[o["seg_begin"] + o["n_seg"] - 1]
        sm = int(seg[last]["sector"])
        prior_mean = r.out_p[last][:4]
        prior_cov = oracle.cov_matrix(r.out_cov[last])[:4, :4] * float(F32(Q.refit_inflate))
        Wp = np.linalg.cholesky(np.linalg.inv(prior_cov)).T
        meas = np.concatenate([[cls[s][c, 1], cls[s][c, 2]] for s, c in zip(sec, cid)]).astype(np.float64)

        def resid(th):
            pred = np.concatenate([_line_frame_state(th, o["x_ref"], s1, int(s), float(row_x[rows[s][c]]))[:2]
                                   for s, c in zip(sec, cid)])
            pri = _line_frame_state(th, o["x_ref"], s1, sm, r.out_x[last]) - prior_mean
            return np.r_[(pred - meas) / 0.1, Wp @ pri]

        theta = np.array(o["p"][:4], np.float64)
        for _ in range(8):
            J = np.zeros((resid(theta).shape[0], 4))
            for j in range(4):
                d = np.zeros(4)
                d[j] = 1e-6
                J[:, j] = (resid(theta + d) - resid(theta - d)) / 2e-6
            theta = theta - np.linalg.lstsq(J, resid(theta), rcond=None)[0]
        sig = np.sqrt(np.diag(np.linalg.inv(J.T @ J)))
        got = np.array(o["p"][:4])
        worst = max(worst, float(np.max(np.abs(got - theta) / sig)))
        checked += 1
    print(f"\nworst |refit - least squares| / sigma: {worst:.2e} over {checked} merged lines")
    # what is left is the filter's linearisation at its running estimate
    # (tan phi of a 0.3-rad line is not linear in sin phi): ~1e-3 sigma
    assert checked >= 20 and worst <= 3e-3, (checked, worst)


def test_refit_pulls_of_merged_tracks(row_x):
    """Merged, pure tracks of central events (sigma 0.1): pulls of the
    refitted parameters at the innermost hit have mean 0 +- 0.05 and width
    1 +- 0.05."""
    pulls = []
    ev_i = 0
    while len(pulls) < 10000:
        ev = tpcgen.make_event(seed=500 + ev_i, stream=43, n_tracks=6000, sigma=0.1)
        ev_i += 1
        cls, rows, trs = _slots.event_arrays(ev)
        _, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x, precision=64)
        for f, o in enumerate(r.finals):
            if o["n_seg"] < 2 or o["status"] != 0:
                continue
            h = r.hits[r.hit_begin[f]:r.hit_begin[f + 1]]
            sec, cid = h >> 24, h & 0xFFFFFF
            tk = np.array([trs[s]["track"][c] for s, c in zip(sec, cid)])
            lg = np.array([trs[s]["leg"][c] * 2 + trs[s]["branch"][c] for s, c in zip(sec, cid)])
            if np.any(tk != tk[0]) or np.any(lg != 0) or tk[0] < 0:
                continue
            t = trs[sec[0]][cid[0]]
            truth = np.array([t["y"], t["z"], t["sinphi"], t["tanl"], t["qpt"]])
            sig = np.sqrt(np.diag(oracle.cov_matrix(o["cov"])))
            pulls.append((o["p"] - truth) / sig)
    pulls = np.array(pulls)
    mean, width = pulls.mean(0), pulls.std(0)
    assert np.all(np.abs(mean) <= 0.05), mean
    assert np.all(np.abs(width - 1) <= 0.05), width


def test_fp32_second_phase_within_1e4_of_fp64(row_x):
    """The FP32 second phase against an FP64 run on the same segments: the
    same merges (up to counted near-ties) and refitted parameters meeting
    the precision criterion of the sector tracker (tests/_fp64.py): every
    final track within 0.1 sigma64, at most 0.5 % of them missing
    1e-4 max(|p64|, sigma64)."""
    from tests import _fp64
    b = tpcgen.central_event(seed=4, n_tracks=6000)
    cls, rows, _ = _slots.slot_arrays(b.cl, b.row, b.units)
    res, seg, hb, hits, r32 = _slots.run_slot(cls, rows, row_x)
    r64 = oracle.phase2(cls, rows, row_x, seg, hb, hits, precision=64)
    diff = int((r32.next != r64.next).sum())
    assert diff <= 2 * (r32.near_ties + r64.near_ties), diff
    same, fails = 0, 0
    dev = np.zeros(5)
    for f, o in enumerate(r32.finals):
        chain = r32.seg_order[o["seg_begin"]:o["seg_begin"] + o["n_seg"]]
        o64 = r64.finals[r64.final_of_seg[chain[0]]]
        if o64["n_seg"] != o["n_seg"] or o["status"] or o64["status"]:
            continue
        if not np.array_equal(r64.seg_order[o64["seg_begin"]:o64["seg_begin"] + o64["n_seg"]], chain):
            continue
        sig = np.sqrt(np.diag(oracle.cov_matrix(o64["cov"])))
        d = np.abs(o["p"] - o64["p"])
        dev = np.maximum(dev, d / sig)
        fails += int(np.any(d > _fp64.SIGMA_FLOOR_TOL * np.maximum(np.abs(o64["p"]), sig)))
        same += 1
    print(f"\nsecond phase FP32 vs FP64: {same} final tracks, max |dp|/sigma64 {np.array2string(dev, precision=4)}, "
          f"missing 1e-4*max(|p|,sigma): {fails}, merge differences {diff}")
    assert same >= 0.99 * r32.finals.shape[0]
    assert np.all(dev <= _fp64.MAX_DEV_SIGMA), dev
    assert fails <= _fp64.MAX_FAIL_FRAC * same, fails


# -------------------------------------------------------------- vertices ---
def test_z_at_axis_of_exact_states(row_x):
    """Exact truth states of primaries (|sin phi| <= 0.9; production at z = 0
    shifted by the event time in a time frame) extrapolate to their
    production z."""
    P = oracle.default_params()
    for t0 in (0.0, 37.5):
        ev = tpcgen.make_event(seed=9, stream=45, n_tracks=400, sigma=0.0, t0_us=t0)
        t = ev.truth
        ok = np.nonzero((t["track"] >= 0) & (t["leg"] == 0) & (t["branch"] == 0) & (np.abs(t["sinphi"]) <= 0.9))[0][::5]
        worst, n = 0.0, 0
        for i in ok:
            side = 0 if ev.sector[i] < 18 else 1
            want = -2.58 * t0 if side == 0 else 2.58 * t0
            st = [t["y"][i], 0.0, t["sinphi"][i], t["tanl"][i], t["qpt"][i]]
            rc, z = oracle.z0(st, float(row_x[ev.row[i]]), float(t["z"][i]), P, precision=64)
            if rc != 0:
                continue
            worst = max(worst, abs(z - want))
            n += 1
        # kB is an FP32 parameter (relative rounding <= 6e-8 against the
        # generator's FP64 curvature): over arcs of up to 2.5 m that moves z0
        # by up to ~1e-5 cm; any error of the extrapolation itself is far larger
        assert n > 500 and worst <= 2e-5, (n, worst)


def test_vertex_groups_equal_connected_components():
    """Grouping of sorted t0 estimates = connected components of the graph
    |t_i - t_j| <= gap (FP32 differences), groups of >= min_n members, at
    the lower median."""
    rng = np.random.default_rng(13)
    for case in range(30):
        n = int(rng.integers(1, 120))
        centers = rng.uniform(0, 50, int(rng.integers(1, 8)))
        t = F32(centers[rng.integers(0, centers.shape[0], n)] + rng.normal(0, 0.05, n))
        if case % 3 == 0:
            t[: n // 3] = t[0]  # exact duplicates
        key = rng.permutation(n).astype(np.int64)
        gap = float(F32(rng.choice([0.02, 0.1, 0.3])))
        min_n = int(rng.integers(1, 5))
        parent = list(range(n))

        def find(i):
            while parent[i] != i:
                parent[i] = parent[parent[i]]
                i = parent[i]
            return i
        for i in range(n):
            for j in range(n):
                if abs(F32(t[i]) - F32(t[j])) <= F32(gap):
                    parent[find(i)] = find(j)
        comps = {}
        for i in range(n):
            comps.setdefault(find(i), []).append(i)
        want = []
        for members in comps.values():
            if len(members) >= min_n:
                order = sorted(members, key=lambda i: (t[i], key[i]))
                want.append((float(t[order[(len(order) - 1) // 2]]), sorted(members)))
        want.sort()
        g, v = oracle.vertex_groups(t.astype(np.float64), key, gap, min_n)
        got = sorted((float(v["t0"][k]), sorted(np.nonzero(g == k)[0].tolist())) for k in range(v.shape[0]))
        assert got == want


def _frame_finals(b, row_x, p2=None):
    cls, rows, trs = _slots.slot_arrays(b.cl, b.row, b.units, b.truth)
    _, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x, p2=p2)
    ev = np.full(r.finals.shape[0], -1)
    pure = np.zeros(r.finals.shape[0], bool)
    for f in range(r.finals.shape[0]):
        h = r.hits[r.hit_begin[f]:r.hit_begin[f + 1]]
        sec, cid = h >> 24, h & 0xFFFFFF
        e = np.array([trs[s]["pad"][c] if trs[s]["track"][c] >= 0 else -1 for s, c in zip(sec, cid)])
        k = np.array([trs[s]["track"][c] * 8 + trs[s]["leg"][c] * 2 + trs[s]["branch"][c] for s, c in zip(sec, cid)])
        ev[f] = np.bincount(e[e >= 0]).argmax() if np.any(e >= 0) else -1
        pure[f] = np.all(k == k[0]) and np.all(e == e[0]) and k[0] % 8 == 0
    return cls, rows, trs, seg, hb, hits, r, ev, pure


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_vertices_recover_event_times(row_x, sigma):
    """Time frame of 12 events: every event with at least 3 long, stiff
    tracks is a vertex at its time (1e-3 us without smearing, 0.02 us with),
    unless another event lies within 1 us; attached pure tracks convert to
    their true z."""
    b = tpcgen.timeframe(seed=5, n_events=12, keep_truth=True)
    if sigma == 0.0:
        t0 = tpcgen.arrival_times_us(5, tpcgen.STREAM_TIMEFRAME, 0, 12)
        evs = [tpcgen.make_event(seed=5, stream=tpcgen.STREAM_TIMEFRAME, event=i,
                                 n_tracks=tpcgen.minbias_multiplicity(5, tpcgen.STREAM_TIMEFRAME, i),
                                 looper_frac=0.05, sigma=0.0, t0_us=float(t0[i])) for i in range(12)]
        parts = []
        for i, ev in enumerate(evs):
            for (sl, s, c, r, tr) in tpcgen.event_units(ev, 0):
                tr = tr.copy()
                tr["pad"] = i
                parts.append((0, s, c, r, tr))
        merged = {}
        for sl, s, c, r, tr in parts:
            merged.setdefault(s, []).append((c, r, tr))
        cl = np.concatenate([np.concatenate([x[0] for x in merged[s]]) for s in range(36)])
        row = np.concatenate([np.concatenate([x[1] for x in merged[s]]) for s in range(36)])
        truth = np.concatenate([np.concatenate([x[2] for x in merged[s]]) for s in range(36)])
        n = [sum(x[0].shape[0] for x in merged[s]) for s in range(36)]
        begin = np.r_[0, np.cumsum(n)[:-1]]
        units = np.array([(begin[s], n[s], 0, s) for s in range(36)], np.int64)
        b = tpcgen.Batch(cl, row, units, truth, {"t0_us": t0})
    t0 = b.meta["t0_us"]
    cls, rows, trs, seg, hb, hits, r, ev, pure = _frame_finals(b, row_x)
    f = r.finals
    stiff = (f["status"] == 0) & (f["z0_ok"] == 1) & (f["n_hits"] >= 20) & (np.abs(f["p"][:, 4]) <= 5.4)
    tol = 1e-3 if sigma == 0.0 else 0.02
    vt = r.vertices["t0"]
    checked = 0
    for e in range(len(t0)):
        if ((ev == e) & stiff & pure).sum() < 3 or np.min(np.abs(np.delete(t0, e) - t0[e])) < 1.0:
            continue
        assert np.min(np.abs(vt - t0[e])) <= tol, (e, t0[e], vt)
        checked += 1
    assert checked >= 8
    att = np.nonzero((f["vertex"] >= 0) & pure & (ev >= 0))[0]
    right = np.abs(vt[f["vertex"][att]] - t0[ev[att]]) <= tol
    assert right.mean() >= 0.98
    for i in att[right][::7]:
        h = r.hits[r.hit_begin[i]]
        s, c = h >> 24, h & 0xFFFFFF
        tz = trs[s]["z"][c] + (1 if s < 18 else -1) * 2.58 * t0[ev[i]]  # the unshifted z of the innermost hit
        assert abs(f["z_conv"][i] - tz) <= (1e-2 if sigma == 0.0 else 1.0), (f["z_conv"][i], tz)


# ------------------------------------------------------------ compression ---
def _entropy_bits(v):
    _, c = np.unique(v, return_counts=True)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def test_compression_round_trip_and_residuals(row_x):
    """Decompression recovers every stored coordinate exactly; the residuals
    of the track model spread like the measurement error (sigma 0.1 cm plus
    the prediction's), and carry fewer bits than absolute coordinates."""
    Q = oracle.default_p2params()
    b = tpcgen.central_event(seed=6, n_tracks=6000)
    tf = tpcgen.timeframe(seed=6, n_events=6)
    for batch, sectors in ((b, range(0, 36, 5)), (tf, (3, 30))):
        for s in sectors:
            cls, rows, _ = _slots.slot_arrays(batch.cl, batch.row, batch.units)
            res = oracle.run_sector(cls[s], rows[s], row_x)
            seg, hb, hits = oracle.segments_of([None] * s + [res])
            rec, rs = oracle.compress(cls[s], rows[s], row_x, seg, hb, hits)
            yq, zq, rr = oracle.decompress(row_x, seg["n_hits"], rec, rs)
            cl = cls[s][hits]
            want_y = np.array([oracle_quant(v, Q.cmp_qy) for v in cl[:, 1]])
            want_z = np.array([oracle_quant(v, Q.cmp_qz) for v in cl[:, 2]])
            assert np.array_equal(yq, want_y) and np.array_equal(zq, want_z)
            assert np.array_equal(rr, rows[s][hits])
            first = np.zeros(hits.shape[0], bool)
            first[hb[:-1]] = True
            ry = rs[~first, 1] * float(F32(Q.cmp_qy))
            rz = rs[~first, 2] * float(F32(Q.cmp_qz))
            assert 0.09 <= np.std(ry) <= 0.2 and 0.09 <= np.std(rz) <= 0.2, (np.std(ry), np.std(rz))
            assert abs(np.mean(ry)) <= 0.01 and abs(np.mean(rz)) <= 0.01
            assert _entropy_bits(rs[~first, 1]) + 4 <= _entropy_bits(want_y)


def oracle_quant(v, q):
    r = np.rint(F32(v) / F32(q))
    return int(r) if abs(r) < 2 ** 30 else 0


# -------------------------------------------------------------- rejection ---
def test_rejection_flags_follow_truth(row_x):
    """Noise-free event with loopers: clusters of later legs of loopers are
    flagged as such, first legs are not; the inclination flag follows the
    truth |sin phi| away from the threshold."""
    ev = tpcgen.make_event(seed=15, stream=47, n_tracks=3000, looper_frac=0.3, sigma=0.0)
    cls, rows, trs = _slots.event_arrays(ev)
    _, seg, hb, hits, r = _slots.run_slot(cls, rows, row_x)
    fl = r.flags
    t = ev.truth
    assigned = np.zeros(fl.shape[0], bool)
    for h in r.hits:
        assigned[ev.sector_begin[h >> 24] + (h & 0xFFFFFF)] = True
    loop = ev.tracks["looper"][np.maximum(t["track"], 0)] == 1
    later = assigned & (t["track"] >= 0) & loop & (t["leg"] >= 1) & (np.abs(t["tanl"]) >= 0.01)
    first = assigned & (t["track"] >= 0) & (t["leg"] == 0) & (t["branch"] == 0)
    assert later.sum() > 1000
    assert (fl[later] & oracle.FLAG_LEG).astype(bool).mean() >= 0.95
    assert (fl[first] & oracle.FLAG_LEG).astype(bool).mean() <= 0.02
    s = np.abs(t["sinphi"])
    hi = assigned & (t["track"] >= 0) & (s >= 0.82) & (t["branch"] == 0)
    lo = assigned & (t["track"] >= 0) & (s <= 0.78) & (t["branch"] == 0)
    assert hi.sum() > 100
    assert (fl[hi] & oracle.FLAG_INCL).astype(bool).mean() >= 0.99
    assert (fl[lo] & oracle.FLAG_INCL).astype(bool).mean() <= 0.01
    assert not np.any(fl[~assigned])


def test_low_pt_flag_threshold(row_x):
    """Constructed segments on helices of |q/pT| just above and just below
    20 c/GeV (pT = 50 MeV): only the first gets the low-pT flag."""
    P = oracle.default_params()
    eye = np.eye(5)[np.tril_indices(5)]
    for qpt, want in ((21.0, oracle.FLAG_LOWPT), (19.0, 0)):
        # noise-free hits on rows 40..51 of sector 0 from the (pinned) FP64
        # propagation of a state starting at sin phi = -0.2
        n = 12
        st, x = np.array([1.0, 5.0, -0.2, 0.1, qpt]), float(row_x[40])
        pts = []
        for k in range(n):
            rc, st, _, x = oracle.propagate(st, eye, x, float(row_x[40 + k]), P, 64)
            assert rc == 0
            pts.append([x, st[0], st[1], 50.0])
        cl = np.array(pts, np.float32)
        row = np.arange(40, 40 + n).astype(np.uint8)
        seg = np.zeros(1, oracle.SEGMENT_DTYPE)
        seg["sector"], seg["n_hits"], seg["x_ref"] = 0, n, row_x[40]
        seg["p"] = [pts[0][1], pts[0][2], -0.2, 0.1, qpt]
        seg["cov"] = np.diag([0.01, 0.01, 1e-4, 1e-4, 1.0])[np.tril_indices(5)]
        cls = [cl] + [np.zeros((0, 4), np.float32)] * 35
        rows = [row] + [np.zeros(0, np.uint8)] * 35
        r = oracle.phase2(cls, rows, row_x, seg, np.array([0, n]), np.arange(n, dtype=np.int32), P)
        assert r.finals["status"][0] == 0 and abs(r.finals["p"][0][4] - qpt) < 0.5
        assert np.all((r.flags & oracle.FLAG_LOWPT) == want)
