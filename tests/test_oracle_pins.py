"""Pins of the CPU oracle against facts that do not come from the oracle.

The paper (Rohr, LHCP 2017, Sec. 2) prints no worked example, so each stage
is pinned by mathematics instead:
  * propagation    - the exact FP64 helix crossings of the generator;
  * update         - the information form of the Gaussian posterior;
  * covariance     - a finite-difference Jacobian of the pinned propagation;
  * links          - brute-force triplet enumeration with exact FP32 rounding;
  * whole tracker  - exact recovery of noise-free helices, the Bayesian
                     least-squares line in the linear limit, pull widths,
                     structural invariants and permutation invariance.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import _fp64
import tpcgen
from tests import _truth

F32 = np.float32


# ------------------------------------------------------------ propagation ---
def _truth_pairs(batch):
    """Consecutive-row crossings of one track on its outgoing branch."""
    cl, row, _, _, tr = batch.unit(0)
    ok = (tr["track"] >= 0) & (tr["leg"] == 0) & (tr["branch"] == 0)
    ids = np.nonzero(ok)[0]
    key = tr["track"][ids].astype(np.int64) * 1000 + row[ids]
    order = np.argsort(key)
    ids, key = ids[order], key[order]
    nxt = np.nonzero(np.diff(key) == 1)[0]
    return tr, row, ids[nxt], ids[nxt + 1]


@pytest.mark.parametrize("bz", [0.5, -0.5])
def test_propagation_hits_exact_helix(row_x, bz):
    b = tpcgen.one_sector(seed=3, sigma=0.0, bz=bz, shuffle=False)
    tr, row, a, c = _truth_pairs(b)
    assert a.shape[0] > 1000
    P = oracle.default_params(kB=float(F32(-bz * 0.299792458e-2)))
    worst = 0.0
    for i, j in zip(a[::7], c[::7]):
        s = [tr["y"][i], tr["z"][i], tr["sinphi"][i], tr["tanl"][i], tr["qpt"][i]]
        cov = np.eye(5).ravel()[[0, 5, 6, 10, 11, 12, 15, 16, 17, 18, 20, 21, 22, 23, 24]]
        rc, s1, _, x1 = oracle.propagate(s, cov, float(row_x[row[i]]), float(row_x[row[j]]), P, 64)
        if abs(tr["sinphi"][j]) > P.max_sinphi:
            continue
        assert rc == 0
        for got, want in ((s1[0], tr["y"][j]), (s1[1], tr["z"][j]), (s1[2], tr["sinphi"][j])):
            err = abs(got - want) / max(abs(want), 1.0)
            worst = max(worst, err)
    assert worst <= 1e-9, worst


def test_propagation_inward_is_inverse(row_x):
    """Stepping back over the same rows returns to the start state (the arc
    length carries the sign of the step)."""
    b = tpcgen.one_sector(seed=5, sigma=0.0, shuffle=False)
    tr, row, a, c = _truth_pairs(b)
    i, j = a[10], c[10]
    s = np.array([tr["y"][j], tr["z"][j], tr["sinphi"][j], tr["tanl"][j], tr["qpt"][j]])
    cov = oracle.cov_lower(np.eye(5))
    rc, s1, _, _ = oracle.propagate(s, cov, float(row_x[row[j]]), float(row_x[row[i]]), precision=64)
    assert rc == 0
    np.testing.assert_allclose(s1[:3], [tr["y"][i], tr["z"][i], tr["sinphi"][i]], rtol=1e-9, atol=1e-9)


def _spd(rng, scale):
    a = rng.normal(size=(5, 5))
    m = a @ a.T + 5 * np.eye(5)
    d = np.sqrt(np.diag(m))
    m = m / np.outer(d, d)
    return m * np.outer(scale, scale)


def test_covariance_propagation_matches_numeric_jacobian():
    """C' = J C J^T with J from central differences of the state propagation,
    which is pinned to the exact helix above.  The reading drops the curvature
    term of the arc length in dz/d(.), an O(u^2) ~ 1e-4 relative change for
    one row, so 2e-3 relative still catches any wrong or dropped term."""
    rng = np.random.default_rng(1)
    P = oracle.default_params()
    for trial in range(20):
        s = np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.6, 0.6),
                      rng.uniform(-1, 1), rng.uniform(-8, 8)])
        C = _spd(rng, np.array([0.3, 0.3, 0.01, 0.01, 0.5]))
        x0 = 120.0
        x1 = x0 + (1.0253 if trial % 2 == 0 else -1.0253)
        J = np.zeros((5, 5))
        for k in range(5):
            h = 1e-6 * max(1.0, abs(s[k]))
            sp, sm = s.copy(), s.copy()
            sp[k] += h
            sm[k] -= h
            _, a, _, _ = oracle.propagate(sp, oracle.cov_lower(np.eye(5)), x0, x1, P, 64)
            _, b, _, _ = oracle.propagate(sm, oracle.cov_lower(np.eye(5)), x0, x1, P, 64)
            J[:, k] = (a - b) / (2 * h)
        rc, _, c1, _ = oracle.propagate(s, oracle.cov_lower(C), x0, x1, P, 64)
        assert rc == 0
        want = J @ C @ J.T
        got = oracle.cov_matrix(c1)
        scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
        assert np.max(np.abs(got - want) / scale) < 2e-3


# ----------------------------------------------------------------- update ---
def test_update_equals_information_form():
    rng = np.random.default_rng(7)
    P = oracle.default_params()
    R = np.diag([P.err2_y, P.err2_z]).astype(np.float64)
    H = np.zeros((2, 5))
    H[0, 0] = H[1, 1] = 1
    for _ in range(50):
        p = rng.normal(size=5)
        C = _spd(rng, rng.uniform(0.05, 3.0, size=5))
        m = p[:2] + rng.normal(scale=0.3, size=2)
        rc, p1, c1, chi2 = oracle.update(p, oracle.cov_lower(C), m[0], m[1], P, 64)
        assert rc == 0
        Ci = np.linalg.inv(C)
        post = np.linalg.inv(Ci + H.T @ np.linalg.inv(R) @ H)
        mean = post @ (Ci @ p + H.T @ np.linalg.inv(R) @ m)
        r = m - p[:2]
        want_chi2 = r @ np.linalg.solve(H @ C @ H.T + R, r)
        np.testing.assert_allclose(p1, mean, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(oracle.cov_matrix(c1), post, rtol=1e-8, atol=1e-12)
        assert abs(chi2 - want_chi2) <= 1e-9 * max(1.0, want_chi2)


def test_update_rejects_singular_innovation():
    P = oracle.default_params(err2_y=0.0, err2_z=0.0)
    rc, *_ = oracle.update(np.zeros(5), np.zeros(15), 0.1, 0.1, P, 64)
    assert rc != 0


# ------------------------------------------------------ links: brute force ---
def _rnd32(q: Fr):
    """Round a rational to the nearest float32, ties to even."""
    r = F32(float(q))
    best = None
    for c in (np.nextafter(r, F32(-np.inf)), r, np.nextafter(r, F32(np.inf))):
        if not np.isfinite(c):
            continue
        d = abs(Fr(float(c)) - q)
        even = int(np.array([c], F32).view(np.uint32)[0]) % 2 == 0
        if best is None or d < best[0] or (d == best[0] and even):
            best = (d, c)
    return best[1]


def _fma32(a, b, c):
    return _rnd32(Fr(float(a)) * Fr(float(b)) + Fr(float(c)))


def _brute_links(cl, row, row_x, P, n_rows):
    """Every (down, hit, up) triplet, no grid, FP32 with exactly rounded fma:
    window |dy|, |dz| <= W dx; deviation of the hit from the straight line
    through the pair, measured at the hit's row as (h - d) - w (u - d) with
    one rounding; best = min (chi2, id_u, id_d)."""
    y = cl[:, 1].astype(F32)
    z = cl[:, 2].astype(F32)
    n = cl.shape[0]
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    rows = [np.nonzero(row == r)[0] for r in range(n_rows)]
    for h in range(n):
        i = int(row[h])
        if i < 1 or i > n_rows - 2:
            continue
        dxu = F32(row_x[i + 1]) - F32(row_x[i])
        dxd = F32(row_x[i]) - F32(row_x[i - 1])
        w = dxd / (dxd + dxu)
        luy, luz = F32(P.link_wy) * dxu, F32(P.link_wz) * dxu
        ldy, ldz = F32(P.link_wy) * dxd, F32(P.link_wz) * dxd
        U = [u for u in rows[i + 1] if abs(y[u] - y[h]) <= luy and abs(z[u] - z[h]) <= luz]
        D = [d for d in rows[i - 1] if abs(y[d] - y[h]) <= ldy and abs(z[d] - z[h]) <= ldz]
        best = None
        for u in U:
            for d in D:
                # deviation from coordinate differences, one rounding
                ey = _fma32(-(y[u] - y[d]), w, y[h] - y[d])
                ez = _fma32(-(z[u] - z[d]), w, z[h] - z[d])
                c2 = _fma32(ey, ey, ez * ez)
                cand = (float(c2), int(u), int(d))
                if best is None or cand < best:
                    best = cand
        if best is not None and best[0] <= float(F32(P.link_chi2)):
            up[h], dn[h] = best[1], best[2]
    return up, dn


def _tiny_sector(rng, n_rows, per_row, spread, row_x, ties=False, edges=False):
    cls, rows = [], []
    for r in range(n_rows):
        k = int(rng.integers(per_row[0], per_row[1] + 1))
        y = rng.uniform(-spread, spread, k)
        z = rng.uniform(-spread, spread, k) + 40.0
        for j in range(k):
            cls.append((row_x[r], y[j], z[j], 100.0))
            rows.append(r)
        if ties and k:
            # exact duplicates: equal chi2, decided by the IDs
            cls.append(cls[-1])
            rows.append(r)
    if edges:
        # hits exactly on and just beyond a window edge around a centre hit
        r = n_rows // 2
        yc, zc = F32(0.25), F32(40.0)
        dxu = F32(row_x[r + 1]) - F32(row_x[r])
        lim = F32(2.0) * dxu
        cls.append((row_x[r], yc, zc, 1.0)); rows.append(r)
        cls.append((row_x[r + 1], F32(yc + lim), zc, 1.0)); rows.append(r + 1)
        cls.append((row_x[r + 1], np.nextafter(F32(yc + lim), F32(np.inf)), zc, 1.0)); rows.append(r + 1)
        cls.append((row_x[r - 1], yc, zc, 1.0)); rows.append(r - 1)
    cl = np.array(cls, F32).reshape(-1, 4)
    return cl, np.array(rows, np.uint8)


@pytest.mark.parametrize("case", range(8))
def test_links_equal_bruteforce(row_x, case):
    rng = np.random.default_rng(100 + case)
    n_rows = int(rng.integers(5, 10))
    dense = case % 2 == 0
    per_row = (5, 14) if dense else (5, 40)
    spread = 2.5 if dense else 12.0
    cl, row = _tiny_sector(rng, n_rows, per_row, spread, row_x, ties=case in (2, 5), edges=case in (3, 6))
    P = oracle.default_params(n_rows=n_rows, link_chi2=0.5 if dense else 0.2)
    want_up, want_dn = _brute_links(cl, row, row_x, P, n_rows)
    res = oracle.run_sector(cl, row, row_x, P, precision=32)
    np.testing.assert_array_equal(res.up_raw, want_up)
    np.testing.assert_array_equal(res.dn_raw, want_dn)
    if dense:
        assert (want_up >= 0).sum() > 5


# ------------------------------------------------------- whole-tracker pins ---
def _accepted_hit_lists(res):
    return [res.track_hit_list(k) for k in range(res.n_tracks)]


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_exact_recovery_noise_free(row_x, seed):
    """sigma = 0, no noise: every findable segment is found with exactly its
    clusters; every accepted track is pure; no clones."""
    b = tpcgen.one_sector(seed=seed, sigma=0.0)
    cl, row, _, _, tr = b.unit(0)
    res = oracle.run_sector(cl, row, row_x)
    m = _truth.match_tracks(tr, row, _accepted_hit_lists(res), purity=1.0)
    assert m["findable"] > 20
    assert m["fakes"] == 0
    assert m["clones"] == 0
    assert m["found"] == m["findable"]
    assert m["exact"] == m["findable"]


def test_efficiency_with_smearing(row_x):
    tot = {"findable": 0, "found": 0, "fakes": 0, "clones": 0}
    for seed in range(10):
        b = tpcgen.one_sector(seed=seed, sigma=0.1)
        cl, row, _, _, tr = b.unit(0)
        res = oracle.run_sector(cl, row, row_x)
        m = _truth.match_tracks(tr, row, _accepted_hit_lists(res))
        for k in tot:
            tot[k] += m[k]
    assert tot["found"] >= 0.99 * tot["findable"], tot
    assert tot["clones"] == 0 and tot["fakes"] <= 2, tot


def test_linear_limit_equals_bayesian_least_squares(row_x):
    """B = 0, |phi| < 5 mrad, lambda = 0: pass 2 of the Kalman filter is the
    Bayesian linear regression y = y_ref + s (x - x_ref), z = z_ref + t (x -
    x_ref) with the Gaussian prior it restarts from: mean = the pass-1 state at
    the outermost hit, covariance = the pass-1 covariance times refit_inflate
    (or the hard-restart diagonal).  What is left is the small-angle
    nonlinearity of tan(phi) and the arc-length coupling of z to phi
    (proportional to tan(lambda) tan(phi), ~1e-7 here): far below 1e-3 sigma."""
    a0 = 10.0 * np.pi / 180.0
    runs = []
    for e in range(40):
        # one track per event: tracks from one vertex within 5 mrad would overlap
        ev = tpcgen.make_event(seed=11, stream=77, event=e, n_tracks=1, only_sector=0, sigma=0.1,
                               phi_range=(a0 - 0.005, a0 + 0.005), bz=0.0, eta_max=0.0, eta_min=0.0)
        parts = tpcgen.event_units(ev, 0, sectors=[0])
        runs.append((parts[0][2], parts[0][3]))
    # soft restart (default), and the hard restart with a tight slope prior so
    # that the first hits cannot move the direction out of the small-angle regime
    for P in (oracle.default_params(kB=0.0),
              oracle.default_params(kB=0.0, refit_inflate=0.0, seed_c22=1e-4, seed_c33=1e-4)):
        checked = 0
        for cl, row in runs:
            res = oracle.run_sector(cl, row, row_x, P, precision=64)
            for t in range(res.tracklets.shape[0]):
                T = res.tracklets[t]
                if T["status"] != 0:
                    continue
                hits = res.tracklet_hit_list(t)
                x = row_x[row[hits]].astype(np.float64)
                xr, xo = T["x_ref"], T["x_out"]
                n = hits.shape[0]
                # theta = (y_ref, z_ref, s, t); observations of y then z
                A = np.zeros((2 * n, 4))
                A[:n, 0] = 1
                A[:n, 2] = x - xr
                A[n:, 1] = 1
                A[n:, 3] = x - xr
                meas = np.r_[cl[hits, 1], cl[hits, 2]].astype(np.float64)
                w = np.r_[np.full(n, 1 / float(F32(P.err2_y))), np.full(n, 1 / float(F32(P.err2_z)))]
                # prior on the values at x_out: B theta
                B = np.eye(4)
                B[0, 2] = B[1, 3] = xo - xr
                if P.refit_inflate > 0:
                    prior_cov = oracle.cov_matrix(T["cov_out"])[:4, :4] * float(F32(P.refit_inflate))
                else:
                    prior_cov = np.diag([float(F32(v)) for v in (P.reset_c00, P.reset_c11, P.seed_c22, P.seed_c33)])
                prior_mean = T["p_out"][:4]
                Pinv = np.linalg.inv(prior_cov)
                info = B.T @ Pinv @ B + A.T @ (A * w[:, None])
                rhs = B.T @ Pinv @ prior_mean + A.T @ (meas * w)
                theta = np.linalg.solve(info, rhs)
                cov = np.linalg.inv(info)
                got = T["p"][:4]
                sig = np.sqrt(np.diag(cov))
                assert np.all(np.abs(got - theta) <= np.maximum(1e-3 * sig, 1e-4 * np.abs(theta))), (got, theta, sig)
                d = np.sqrt(np.diag(cov))
                dc = np.abs(oracle.cov_matrix(T["cov"])[:4, :4] - cov) / np.outer(d, d)
                assert dc.max() <= 2e-3, dc
                checked += 1
        assert checked >= 30


def test_pull_distributions(row_x):
    """>= 1e4 pure, complete tracks (one-sector law, sigma = 0.1): pulls of all
    five parameters at the reference row have mean 0 +- 0.05, width 1 +- 0.05."""
    pulls = []
    seed = 0
    while len(pulls) < 10000:
        b = tpcgen.one_sector(seed=1000 + seed, sigma=0.1, n_tracks=400)
        seed += 1
        cl, row, _, _, tr = b.unit(0)
        res = oracle.run_sector(cl, row, row_x, precision=64)
        hl = _accepted_hit_lists(res)
        m = _truth.match_tracks(tr, row, hl, purity=1.0)
        for fk, ts in m["matched"].items():
            if len(ts) != 1:
                continue
            k = ts[0]
            hits = hl[k]
            if not np.array_equal(np.sort(hits), m["segments"][fk]):
                continue
            T = res.tracklets[res.track_tracklet[k]]
            ref = hits[np.argmin(row[hits])]
            truth = np.array([tr["y"][ref], tr["z"][ref], tr["sinphi"][ref], tr["tanl"][ref], tr["qpt"][ref]])
            sig = np.sqrt(np.diag(oracle.cov_matrix(T["cov"])))
            pulls.append((T["p"] - truth) / sig)
    pulls = np.array(pulls)
    mean = pulls.mean(0)
    width = pulls.std(0)
    assert np.all(np.abs(mean) <= 0.05), mean
    assert np.all(np.abs(width - 1) <= 0.05), width


def _select_key(T):
    """more hits, then smaller chi2 (as FP32), then smaller start_id"""
    c = max(float(F32(T["chi2"])), 0.0)
    bits = int(np.array([c], F32).view(np.uint32)[0])
    return (int(T["n_hits"]) << 56) | ((0xFFFFFFFF - bits) << 24) | (0xFFFFFF - int(T["start_id"]))


def _invariants(res, cl, row, P):
    n = cl.shape[0]
    up, dn = res.up, res.dn
    for h in range(n):
        if up[h] >= 0:
            assert dn[up[h]] == h and row[up[h]] == row[h] + 1
        if dn[h] >= 0:
            assert up[dn[h]] == h and row[dn[h]] == row[h] - 1
    # raw links also obey the row rule; cleaning only removes links
    for h in np.nonzero(res.up_raw >= 0)[0]:
        assert row[res.up_raw[h]] == row[h] + 1 and row[res.dn_raw[h]] == row[h] - 1
    assert np.all((up < 0) | (up == res.up_raw))
    assert np.all((dn < 0) | (dn == res.dn_raw))
    # chains are disjoint row-increasing paths
    starts = np.nonzero((up >= 0) & (dn < 0))[0]
    seen = np.zeros(n, bool)
    for s in starts:
        k = s
        while k >= 0:
            assert not seen[k]
            seen[k] = True
            k = up[k]
    # tracklets: one per chain of >= min_chain_hits, ascending start ids
    chain_len = {}
    for s in starts:
        c, k = 0, s
        while k >= 0:
            c, k = c + 1, up[k]
        chain_len[int(s)] = c
    want = sorted(s for s, c in chain_len.items() if c >= P.min_chain_hits)
    assert list(res.tracklets["start_id"]) == want
    # tracklet hit lists: one hit per row, ascending, include the chain
    for t in range(res.tracklets.shape[0]):
        T = res.tracklets[t]
        hits = res.tracklet_hit_list(t)
        if T["status"] == 2:
            continue
        assert np.all(np.diff(row[hits].astype(int)) > 0)
        assert T["start_id"] in hits and T["n_hits"] == hits.shape[0]
        assert T["ndf"] == 2 * T["n_hits"] - 5
    # selection: each cluster at most once; owner rule; acceptance rule
    key = {}
    for t in range(res.tracklets.shape[0]):
        T = res.tracklets[t]
        if T["status"] != 0:
            continue
        kk = _select_key(T)
        for h in res.tracklet_hit_list(t):
            key[int(h)] = max(key.get(int(h), 0), kk)
    used = np.zeros(n, int)
    for k in range(res.n_tracks):
        T = res.tracklets[res.track_tracklet[k]]
        kk = _select_key(T)
        won = res.track_hit_list(k)
        assert won.shape[0] >= P.min_track_hits and won.shape[0] * 100 >= P.own_frac_pct * T["n_hits"]
        for h in won:
            assert key[int(h)] == kk
            used[h] += 1
            assert res.assignment[h] == k
    assert used.max(initial=0) <= 1
    assert np.all((res.assignment >= 0) == (used == 1))
    assert np.all(np.diff(res.tracklets["start_id"][res.track_tracklet]) > 0)


def _predicted_work(res, row, P):
    """Propagations and updates each fitted tracklet takes by the row rules
    of the fit (Fig. 1c): the chain's hits one by one, outward until
    max_miss empty rows follow the outermost hit or the last row, the refit
    through the pass-1 hits, inward likewise; every update succeeds (S is
    positive definite).  Valid when no propagation leaves the sector."""
    R, mm = P.n_rows, P.max_miss
    props = upd = acc_search = 0
    for T in res.tracklets:
        assert T["status"] != 2
        r0 = int(row[T["start_id"]])
        nc, n1, ne = int(T["n_chain"]), int(T["n_pass1"]), int(T["n_hits"] - T["n_pass1"])
        chain_end = r0 + nc - 1
        props += (nc - 1) + (min(int(T["row_out"]) + mm, R - 1) - chain_end)
        props += (n1 - 1) + (r0 - max(int(T["row_ref"]) - mm, 0))
        upd += (nc - 1) + (n1 - nc) + n1 + ne
        acc_search += (n1 - nc) + ne
    return props, upd, acc_search


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_fit_work_counts_follow_the_row_rules(row_x, sigma):
    """The oracle's work counters (the basis of the fit's FLOP count) equal
    what the row rules predict from the tracklets it returns."""
    P = oracle.default_params()
    for seed in (2, 3):
        b = tpcgen.one_sector(seed=seed, sigma=sigma, n_tracks=120)
        cl, row, _, _, _ = b.unit(0)
        res = oracle.run_sector(cl, row, row_x, P)
        props, upd, acc_search = _predicted_work(res, row, P)
        assert res.tracklets.shape[0] > 20
        assert res.work["propagations"] == props
        assert res.work["updates"] == upd
        # every searched hit that was taken passed one chi2 test
        assert res.work["tests"] >= acc_search
        if sigma == 0.0:
            assert res.work["tests"] == acc_search


def test_invariants_central_sector(row_x):
    b = tpcgen.central_event(seed=1, n_tracks=8000)
    P = oracle.default_params()
    for u in (0, 20):
        cl, row, _, _, _ = b.unit(u)
        res = oracle.run_sector(cl, row, row_x, P)
        assert res.n_tracks > 200
        _invariants(res, cl, row, P)


def test_permutation_invariance(row_x):
    b = tpcgen.central_event(seed=2, n_tracks=3000, shuffle=False)
    cl, row, _, _, _ = b.unit(5)
    perm = np.random.default_rng(0).permutation(cl.shape[0])
    inv = np.argsort(perm)
    r0 = oracle.run_sector(cl, row, row_x)
    r1 = oracle.run_sector(cl[perm], row[perm], row_x)
    # links map through the permutation
    m = lambda a: np.where(a >= 0, perm[np.maximum(a, 0)], -1)
    np.testing.assert_array_equal(m(r1.up_raw)[inv], r0.up_raw)
    np.testing.assert_array_equal(m(r1.dn_raw)[inv], r0.dn_raw)
    # accepted tracks: same hit sets with bit-identical parameters
    def tracks(r, ids):
        out = {}
        for k in range(r.n_tracks):
            T = r.tracklets[r.track_tracklet[k]]
            out[tuple(sorted(ids[r.track_hit_list(k)]))] = (tuple(T["p"]), tuple(T["cov"]), T["chi2"])
        return out
    t0 = tracks(r0, np.arange(cl.shape[0]))
    t1 = tracks(r1, perm)
    # IDs only break exact ties (equal chi2, equal distances), which random
    # data does not produce: the result is the same up to relabelling.
    assert t0 == t1


def test_internal_order_invariance(row_x):
    """Reordering the input while keeping every pairwise ID order (i.e. moving
    clusters around rows without relabelling) cannot change anything: the
    result depends on IDs only through comparisons."""
    b = tpcgen.central_event(seed=2, n_tracks=3000, shuffle=False)
    cl, row, _, _, _ = b.unit(5)
    r0 = oracle.run_sector(cl, row, row_x)
    # reverse the z order inside every row but keep IDs: the oracle sorts by
    # (z, id), so flipping z signs exercises a different internal order
    flipped = cl.copy()
    flipped[:, 2] = -flipped[:, 2]
    r1 = oracle.run_sector(flipped, row, row_x)
    np.testing.assert_array_equal(r0.up_raw, r1.up_raw)
    np.testing.assert_array_equal(r0.dn_raw, r1.dn_raw)
    np.testing.assert_array_equal(r0.assignment, r1.assignment)
    np.testing.assert_array_equal(r0.tracklets["start_id"], r1.tracklets["start_id"])
    np.testing.assert_array_equal(r0.tracklets["n_hits"], r1.tracklets["n_hits"])


def _fp32_fp64(cl, row, row_x, name):
    r32 = oracle.run_sector(cl, row, row_x, precision=32)
    r64 = oracle.run_sector(cl, row, row_x, precision=64)
    # links: identical away from decisions with a relative margin below 1e-6
    # (a hit whose link decision flips counts once)
    diff = int(np.count_nonzero((r32.up_raw != r64.up_raw) | (r32.dn_raw != r64.dn_raw)))
    st = _fp64.compare(cl, row, row_x, r32.tracklets, r32.tracklet_hit_begin, r32.tracklet_hits)
    print(_fp64.summary(name, st) + f"; link differences {diff}, near-ties FP32 {r32.near_ties} "
          f"FP64 {r64.near_ties}, min margin {r32.min_margin:.2e}")
    assert diff <= r32.near_ties + r64.near_ties, (diff, r32.near_ties, r64.near_ties)
    _fp64.check(st)
    return st


def test_fp32_and_fp64_runs_agree(row_x):
    """Central event: links of the FP32 run equal the FP64 run's except at
    counted near-ties, and every FP32 tracklet meets the precision criterion
    against the FP64 replay of its own decisions (tests/_fp64.py)."""
    b = tpcgen.central_event(seed=3, n_tracks=8000)
    cl, row, _, _, _ = b.unit(7)
    st = _fp32_fp64(cl, row, row_x, "central event, sector 7")
    assert st["tracklets"] > 500


@pytest.mark.slow
def test_fp32_and_fp64_time_frame_sector(row_x):
    """A sector of the 128-event time frame: z' spans tens of metres
    (Sec. 5).  With the CA deviation and the fit's z formed relative to the
    hits, FP32 keeps its precision there: the same criterion holds."""
    tf = tpcgen.timeframe(seed=0, n_events=128)
    cl, row, _, _, _ = tf.unit(30)
    assert np.ptp(cl[:, 2]) > 5000.0
    st = _fp32_fp64(cl, row, row_x, "128-event time frame, unit 30")
    assert st["tracklets"] > 20000


def test_fp32_precision_does_not_depend_on_a_z_offset(row_x):
    """The same sector shifted by -60 m in z (the far end of a time frame):
    the FP32 fit stays as close to FP64 as unshifted.  An absolute FP32 z at
    60 m has a spacing of 5e-4 cm and moved tan lambda by up to 0.5 sigma."""
    b = tpcgen.central_event(seed=3, n_tracks=8000)
    cl, row, _, _, _ = b.unit(7)
    shifted = cl.copy()
    shifted[:, 2] -= 6000.0
    st = _fp32_fp64(shifted, row, row_x, "central sector 7 shifted by -60 m")
    assert st["max_dev_sigma"][3] < 0.05


def test_fp32_and_fp64_minimum_bias(row_x):
    """Units of the largest and the smallest event of a 64-event minimum-bias batch."""
    b = tpcgen.minbias_batch(seed=0, n_events=64)
    sizes = np.bincount(b.units[:, 2], weights=b.units[:, 1])
    for ev in (int(np.argmax(sizes)), int(np.argmin(sizes))):
        for u in np.nonzero(b.units[:, 2] == ev)[0][:2]:
            cl, row, _, _, _ = b.unit(int(u))
            _fp32_fp64(cl, row, row_x, f"minimum-bias event {ev} ({int(sizes[ev])} clusters), unit {u}")


def test_refit_replays_fp64_run(row_x):
    """The FP64 replay along the FP64 run's own decisions reproduces it bit for bit."""
    b = tpcgen.one_sector(seed=9)
    cl, row, _, _, _ = b.unit(0)
    r = oracle.run_sector(cl, row, row_x, precision=64)
    for t in range(r.tracklets.shape[0]):
        T = r.tracklets[t]
        if T["status"] != 0:
            continue
        hits = r.tracklet_hit_list(t)
        k0 = int(np.nonzero(hits == T["start_id"])[0][0])
        rc, R = oracle.refit(cl, row, row_x, hits, k0, T["n_chain"], precision=64)
        assert rc == 0
        assert np.array_equal(R["p"], T["p"]) and np.array_equal(R["cov"], T["cov"]) and R["chi2"] == T["chi2"]


def test_rejects_bad_input(row_x):
    cl = np.array([[row_x[3], 0, 10, 1]], np.float32)
    with pytest.raises(ValueError):
        oracle.run_sector(cl, np.array([200], np.uint8), row_x)
    bad = cl.copy()
    bad[0, 0] += 0.5
    with pytest.raises(ValueError):
        oracle.run_sector(bad, np.array([3], np.uint8), row_x)
    nan = cl.copy()
    nan[0, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.run_sector(nan, np.array([3], np.uint8), row_x)
    empty = oracle.run_sector(np.zeros((0, 4), np.float32), np.zeros(0, np.uint8), row_x)
    assert empty.n_tracks == 0


# ----------------------------------------------------- single-decision pins ---
def test_chi2_equals_closed_form():
    """The pickup test's chi^2 is r^T S^-1 r with S = C_yz + diag(err2): against
    numpy's solve in FP64, and equal to the chi^2 the update reports (FP32 and
    FP64); a singular S is refused."""
    rng = np.random.default_rng(5)
    P = oracle.default_params()
    for _ in range(200):
        A = rng.normal(size=(5, 5))
        C = A @ A.T * rng.uniform(1e-4, 1.0) + np.eye(5) * 1e-6
        p = rng.normal(size=5) * [10, 50, 0.3, 0.5, 2]
        ym, zm = p[0] + rng.normal() * 0.3, p[1] + rng.normal() * 0.3
        c15 = oracle.cov_lower(C)
        rc, c2 = oracle.chi2(p, c15, ym, zm, precision=64)
        assert rc == 0
        S = C[:2, :2] + np.diag([P.err2_y, P.err2_z]).astype(np.float64)
        r = np.array([ym - p[0], zm - p[1]])
        want = float(r @ np.linalg.solve(S, r))
        assert abs(c2 - want) <= 1e-10 * max(1.0, want)
        for prec in (32, 64):
            rc1, c_test = oracle.chi2(p, c15, ym, zm, precision=prec)
            rc2, _, _, c_upd = oracle.update(p, c15, ym, zm, precision=prec)
            assert rc1 == rc2 == 0 and c_test == c_upd
    # S singular: C_yz = -R makes det(S) = 0
    C = np.zeros(15)
    C[0], C[2] = -P.err2_y, -P.err2_z
    assert oracle.chi2(np.zeros(5), C, 1.0, 1.0)[0] != 0


def _search_case(row_x, hits_yz, r=50):
    """A one-row sector: hits (y, z) in row r, in ID order."""
    cl = np.array([[row_x[r], y, z, 1.0] for y, z in hits_yz], np.float32).reshape(-1, 4)
    return cl, np.full(cl.shape[0], r, np.uint8)


def test_search_row_tie_rule_and_window_cap(row_x):
    """Track following picks the nearest hit by dy^2 + dz^2 inside
    nsig predicted sigmas capped at pick_win_max; equal distances go to the
    lower cluster ID.  Expected picks follow from the rule alone."""
    P = oracle.default_params()
    small = np.zeros(15)
    small[0] = small[2] = 0.01          # window 3 sqrt(0.02) = 0.424 cm
    wide = np.zeros(15)
    wide[0] = wide[2] = 100.0           # 3 sqrt(100.01) = 30 cm, capped at 4 cm
    zr = 6000.0                          # the state's z is relative to zr
    st = np.array([10.0, 0.25, 0.0, 0.0, 0.0])
    zc = zr + 0.25                       # absolute predicted z (exact in FP32)
    for prec in (32, 64):
        def pick(hits, cov):
            cl, row = _search_case(row_x, hits)
            return oracle.search_row(cl, row, row_x, 50, st, cov, zr=zr, params=P, precision=prec)
        # equal distances (exact in FP32): the lower ID wins, whichever side
        assert pick([(10.25, zc), (9.75, zc)], small) == 0
        assert pick([(9.75, zc), (10.25, zc)], small) == 0
        assert pick([(10.0, zc + 0.25), (10.25, zc), (10.0, zc - 0.25)], small) == 0
        # the nearer hit wins over the lower ID
        assert pick([(10.375, zc), (10.25, zc)], small) == 1
        assert pick([(10.0, zc + 0.375), (10.0, zc - 0.25)], small) == 1
        # window edges: 0.4 inside, 0.5 outside the 0.424 cm window
        assert pick([(10.5, zc)], small) == -1
        assert pick([(10.4, zc)], small) == 0
        assert pick([(10.0, zc + 0.5)], small) == -1
        # the cap binds: 4.5 cm is inside 3 sigma (30 cm) but beyond 4 cm
        assert pick([(14.5, zc)], wide) == -1
        assert pick([(10.0, zc - 4.5)], wide) == -1
        assert pick([(14.0, zc), (14.5, zc)], wide) == 0   # exactly on the cap is inside
        assert pick([(14.5, zc), (13.75, zc)], wide) == 1
        # an empty row
        assert pick([(10.0, zc + 50.0)], wide) == -1


def test_selection_claim_order():
    """Selection on hand-made candidates: a hit belongs to the candidate with
    more hits, then the smaller chi^2, then the smaller start ID; a candidate
    is accepted with >= min_track_hits won hits and >= 90 % of its hits.
    Expected outcomes are worked out from that rule by hand."""
    P = oracle.default_params()
    h10 = list(range(10))
    # equal length, equal hits: the smaller chi^2 takes every hit
    acc, asg = oracle.select(30, [10, 10], [2.0, 1.0], [3, 5], [0, 0], [h10, h10], P)
    assert acc.tolist() == [-1, 0] and np.all(asg[:10] == 0) and np.all(asg[10:] == -1)
    # equal length and bit-equal chi^2: the smaller start ID
    acc, _ = oracle.select(30, [10, 10], [1.5, 1.5], [7, 4], [0, 0], [h10, h10], P)
    assert acc.tolist() == [-1, 0]
    acc, _ = oracle.select(30, [10, 10], [1.5, 1.5], [4, 7], [0, 0], [h10, h10], P)
    assert acc.tolist() == [0, -1]
    # more hits beats a smaller chi^2
    acc, _ = oracle.select(30, [11, 10], [50.0, 1.0], [9, 1], [0, 0], [list(range(11)), h10], P)
    assert acc.tolist() == [0, -1]
    # chi^2 = 0 is the best chi^2
    acc, _ = oracle.select(30, [10, 10], [0.0, 1e-30], [9, 1], [0, 0], [h10, h10], P)
    assert acc.tolist() == [0, -1]
    # 90 % boundary: B (20 hits) loses 2 shared hits to A -> 18/20 = 90 %: kept
    A = list(range(20))
    B = [18, 19] + list(range(100, 118))
    acc, asg = oracle.select(200, [20, 20], [1.0, 2.0], [0, 1], [0, 0], [A, B], P)
    assert acc.tolist() == [0, 1] and asg[18] == 0 and asg[100] == 1 and (asg == 1).sum() == 18
    # losing 3 of 20 (85 %): rejected, its other hits stay unassigned
    B = [17, 18, 19] + list(range(100, 117))
    acc, asg = oracle.select(200, [20, 20], [1.0, 2.0], [0, 1], [0, 0], [A, B], P)
    assert acc.tolist() == [0, -1] and np.all(asg[100:117] == -1)
    # 9 hits won is below min_track_hits even at 100 %
    acc, _ = oracle.select(30, [9], [1.0], [0], [0], [list(range(9))], P)
    assert acc.tolist() == [-1]
    # a candidate that is not fitted (status != 0) does not claim
    acc, _ = oracle.select(30, [12, 10], [1.0, 1.0], [0, 1], [1, 0], [list(range(12)), h10], P)
    assert acc.tolist() == [-1, 0]
