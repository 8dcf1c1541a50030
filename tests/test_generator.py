"""The synthetic input recipes: determinism, geometry and sizes."""
import math

import numpy as np

import tpcgen


def test_row_geometry():
    rx = tpcgen.row_x()
    assert rx.dtype == np.float32 and rx.shape == (159,)
    assert rx[0] == np.float32(85.0) and rx[-1] == np.float32(247.0)
    np.testing.assert_allclose(np.diff(rx.astype(np.float64)), 162.0 / 158.0, rtol=3e-5)


def test_deterministic_per_seed():
    a = tpcgen.one_sector(seed=4)
    b = tpcgen.one_sector(seed=4)
    c = tpcgen.one_sector(seed=5)
    np.testing.assert_array_equal(a.cl, b.cl)
    np.testing.assert_array_equal(a.row, b.row)
    assert a.cl.shape != c.cl.shape or not np.array_equal(a.cl, c.cl)


def test_clusters_lie_on_rows_and_in_sector():
    b = tpcgen.central_event(seed=0, n_tracks=2000)
    rx = tpcgen.row_x()
    np.testing.assert_array_equal(b.cl[:, 0], rx[b.row])
    tan10 = math.tan(math.radians(10))
    sig = b.truth["track"] >= 0
    assert np.all(np.abs(b.truth["y"][sig]) <= rx[b.row[sig]] * tan10 + 1e-9)
    for u in range(b.units.shape[0]):
        _, _, _, sec, tr = b.unit(u)
        z = tr["z"]
        assert np.all(z >= 0) if sec < 18 else np.all(z <= 0)


def test_truth_is_on_the_circle():
    """sin(phi) grows linearly with x along each helix: ds/dx = kappa."""
    b = tpcgen.one_sector(seed=1, sigma=0.0, shuffle=False)
    tr, row = b.truth, b.row
    kappa = b.meta["tracks"]["kappa"]
    rx = tpcgen.row_x().astype(np.float64)
    for t in range(20):
        m = (tr["track"] == t) & (tr["branch"] == 0) & (tr["leg"] == 0)
        if m.sum() < 3:
            continue
        x = rx[row[m]]
        s = tr["sinphi"][m]
        slope = np.polyfit(x, s, 1)[0]
        assert abs(slope - kappa[t]) <= 1e-9 + 1e-7 * abs(kappa[t])


def test_workload_sizes():
    one = tpcgen.one_sector(seed=0)
    assert 3000 < one.n_clusters < 8000
    ev = tpcgen.central_event(seed=0)
    assert ev.units.shape == (36, 4)
    assert 0.9e6 < ev.n_clusters < 1.3e6
    noise = (ev.truth["track"] < 0).sum()
    assert abs(noise - 0.01 * (ev.n_clusters - noise)) <= 1
    mult = [tpcgen.minbias_multiplicity(0, tpcgen.STREAM_MINBIAS, e) for e in range(2000)]
    assert min(mult) >= 10 and max(mult) <= 8000
    assert 1800 < np.mean(mult) < 2200   # mean of the overlap-area law: 8000/4


def test_timeframe_shift():
    tf = tpcgen.timeframe(seed=0, n_events=6)
    t0 = tf.meta["t0_us"]
    assert t0.shape == (6,) and np.all(np.diff(t0) > 0)
    # A side z' = z - v t0 can only go down, C side up
    a = tf.units[:, 3] < 18
    for u in range(tf.units.shape[0]):
        c, _, _, sec, _ = tf.unit(u)
        if c.shape[0]:
            if sec < 18:
                assert c[:, 2].max() <= 250.5
            else:
                assert c[:, 2].min() >= -250.5
    assert a.sum() == 18


def test_served_stream_law():
    sizes, arrivals, mean = tpcgen.served_stream(seed=0, n_tf=400)
    assert sizes.min() >= 8 and sizes.max() <= 256
    assert abs(mean - 71.6) < 0.1
    rate = 1e6 / np.mean(np.diff(arrivals))       # TF per second
    assert 500 < rate < 900                       # 50 kHz / 71.6 = 698 per s
