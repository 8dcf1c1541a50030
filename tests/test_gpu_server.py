"""The continuous-batching server: each time frame's result is the same
alone and in a mix of concurrent frames, and equals the batch path and the
oracle; admission errors are reported at submit."""
import numpy as np
import pytest

import tpcgen
from tests import _parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_00618_amd import serving, tpcca
    tpcca.lib()
    return tpcca, serving


@pytest.fixture(scope="module")
def frames():
    pool = tpcgen.minbias_pool(seed=3, n=12)
    out = []
    for i, k in enumerate((8, 13, 21)):
        out.append(tpcgen.timeframe(seed=3, n_events=k, tf_index=i, event_pool=pool, stream=tpcgen.STREAM_SERVED))
    return out


def _results(serving, srv, tfs, pinned):
    fr = [serving.Frame(t.cl, t.row, t.units, pinned=pinned) for t in tfs]
    outs = [serving.Outputs(f.n_clusters, f.n_units) for f in fr]
    rids = [srv.submit(f, o) for f, o in zip(fr, outs)]
    res = []
    for rid, f, o in zip(rids, fr, outs):
        r = srv.wait(rid, 300)
        assert r.status == 0 and r.done == 1
        assert r.end_s >= r.start_s >= r.arrival_s - 1e-3
        res.append([(a.copy(), b.copy(), c.copy()) for a, b, c in serving.unit_results(f, o)])
        srv.release(rid)
    return res


def test_alone_equals_mix_equals_batch(mods, frames, row_x):
    tpcca, serving = mods
    with serving.Server(row_x, n_streams=2, budget_bytes=8 << 30) as srv:
        alone = [_results(serving, srv, [t], pinned=True)[0] for t in frames]
        print("alone done", flush=True)
        mix_tfs = [frames[0], frames[1], frames[2], frames[0], frames[1]]
        mix = _results(serving, srv, mix_tfs, pinned=False)
        st = srv.stats()
        assert st.completed == 3 + 5 and st.batches_run >= 2
    for k, m in zip((0, 1, 2, 0, 1), mix):
        for (ta, ha, aa), (tm, hm, am) in zip(alone[k], m):
            assert ta.tobytes() == tm.tobytes()
            assert np.array_equal(ha, hm) and np.array_equal(aa, am)
    # the batch path gives the same per-unit results
    with tpcca.Context(row_x) as ctx:
        for k, t in enumerate(frames):
            ctx.run_batch(t.cl, t.row, t.units, graph=True)
            units, tracks, hits, asg = ctx.get_batch_results()
            for u in range(t.units.shape[0]):
                ur = units[u]
                t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
                h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
                c0, n = int(ur["cluster_begin"]), int(t.units[u, 1])
                assert alone[k][u][0].tobytes() == tracks[t0:t0 + nt].tobytes()
                assert np.array_equal(alone[k][u][1], hits[h0:h0 + nh])
                assert np.array_equal(alone[k][u][2], asg[c0:c0 + n])
    # and the oracle, on a few sectors of the largest frame
    t = frames[2]
    refs = _parity.oracle_units(t, row_x, which={0, 17, 35})
    for u in (0, 17, 35):
        tr, h, a = alone[2][u]
        _parity.compare_tracks(tr, h, refs[u])
        assert np.array_equal(a, refs[u].assignment)


def test_admission_errors(mods, frames, row_x):
    tpcca, serving = mods
    t = frames[0]
    with serving.Server(row_x, n_streams=1, budget_bytes=1 << 20) as srv:
        f = serving.Frame(t.cl, t.row, t.units)
        o = serving.Outputs(f.n_clusters, f.n_units)
        with pytest.raises(tpcca.TpccaError) as ei:
            srv.submit(f, o)  # one sector alone exceeds a 1 MiB lane
        assert ei.value.status == tpcca.ENOMEM
    with serving.Server(row_x, n_streams=1, budget_bytes=4 << 30) as srv:
        units = t.units.copy()
        units[0, 3] = 77
        f = serving.Frame(t.cl, t.row, units)
        with pytest.raises(tpcca.TpccaError) as ei:
            srv.submit(f, serving.Outputs(f.n_clusters, f.n_units))
        assert ei.value.status == tpcca.EINVAL
        # an empty frame completes at once
        f = serving.Frame(np.zeros((0, 4), np.float32), np.zeros(0, np.uint8), np.zeros((0, 4), np.int64))
        rid = srv.submit(f, serving.Outputs(1, 1))
        assert srv.wait(rid, 10).done == 1


def test_large_frame_sliced_across_lane_batches(mods, row_x):
    """A frame larger than a lane's share is split by sector over several
    batches and lanes; the result equals one batch of the whole frame."""
    tpcca, serving = mods
    tf = tpcgen.timeframe(seed=8, n_events=40)
    print(f"large frame: {tf.n_clusters} clusters", flush=True)
    # 2 lanes of 1.5 GiB: about 2M clusters per lane batch
    with serving.Server(row_x, n_streams=2, budget_bytes=3 << 30) as srv:
        f = serving.Frame(tf.cl, tf.row, tf.units, pinned=True)
        o = serving.Outputs(f.n_clusters, f.n_units)
        rid = srv.submit(f, o)
        r = srv.wait(rid, 300)
        assert r.status == 0 and r.done == 1
        st = srv.stats()
        assert st.batches_run >= 3
        got = serving.unit_results(f, o)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(tf.cl, tf.row, tf.units, graph=True)
        units, tracks, hits, asg = ctx.get_batch_results()
    for u in range(tf.units.shape[0]):
        ur = units[u]
        t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
        h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
        c0, n = int(ur["cluster_begin"]), int(tf.units[u, 1])
        assert got[u][0].tobytes() == tracks[t0:t0 + nt].tobytes()
        assert np.array_equal(got[u][1], hits[h0:h0 + nh])
        assert np.array_equal(got[u][2], asg[c0:c0 + n])


def test_tuned_lanes_give_the_same_results(mods, frames, row_x):
    """A schedule set on the server (applied by every lane from its next
    batch) changes no result; knobs out of range are refused."""
    tpcca, serving = mods
    with serving.Server(row_x, n_streams=2, budget_bytes=8 << 30) as srv:
        base = _results(serving, srv, frames[:2], pinned=True)
        srv.set_tuning(fit_pool=128, fit_blocks_per_cu=6, link_stage=1, fit_min_waves=4)
        print("tuned lanes", flush=True)
        tuned = _results(serving, srv, frames[:2], pinned=True)
        with pytest.raises(tpcca.TpccaError):
            srv.set_tuning(link_stage=7)
        assert srv.last_error() == ""
    for a, b in zip(base, tuned):
        for (ta, ha, aa), (tb, hb, ab) in zip(a, b):
            assert ta.tobytes() == tb.tobytes()
            assert np.array_equal(ha, hb) and np.array_equal(aa, ab)


def test_full_queue_returns_ebusy(mods, frames, row_x):
    """With room for one waiting frame, frames submitted back to back while
    the lane works are refused with EBUSY (counted as rejected); every
    admitted frame still completes with the batch path's results."""
    tpcca, serving = mods
    t = frames[2]
    with serving.Server(row_x, n_streams=1, budget_bytes=8 << 30, max_queue=1) as srv:
        fr = serving.Frame(t.cl, t.row, t.units, pinned=True)
        admitted, busy = [], 0
        for _ in range(12):
            o = serving.Outputs(fr.n_clusters, fr.n_units)
            try:
                admitted.append((srv.submit(fr, o), o))
            except tpcca.TpccaError as e:
                assert e.status == tpcca.EBUSY
                busy += 1
        print(f"admitted {len(admitted)}, refused {busy}", flush=True)
        assert busy >= 1 and len(admitted) >= 1
        assert srv.stats().rejected == busy
        res = []
        for rid, o in admitted:
            r = srv.wait(rid, 300)
            assert r.status == 0 and r.done == 1
            res.append(serving.unit_results(fr, o))
            srv.release(rid)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(t.cl, t.row, t.units, graph=True)
        units, tracks, hits, asg = ctx.get_batch_results()
    for got in res:
        for u in range(t.units.shape[0]):
            ur = units[u]
            t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
            h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
            c0, n = int(ur["cluster_begin"]), int(t.units[u, 1])
            assert got[u][0].tobytes() == tracks[t0:t0 + nt].tobytes()
            assert np.array_equal(got[u][1], hits[h0:h0 + nh])
            assert np.array_equal(got[u][2], asg[c0:c0 + n])


def test_three_lanes_eight_outstanding_equal_the_batch_path(mods, frames, row_x):
    """The served configuration of the benchmark (three lanes, up to eight
    frames outstanding, frames of different sizes batched together and
    graphs replayed from the lanes' caches): every served frame equals the
    batch path's results for it."""
    tpcca, serving = mods
    want = []
    with tpcca.Context(row_x) as ctx:
        for t in frames:
            ctx.run_batch(t.cl, t.row, t.units, graph=True)
            units, tracks, hits, asg = ctx.get_batch_results()
            per = []
            for u in range(t.units.shape[0]):
                ur = units[u]
                t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
                h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
                c0, n = int(ur["cluster_begin"]), int(t.units[u, 1])
                per.append((tracks[t0:t0 + nt].tobytes(), hits[h0:h0 + nh].copy(), asg[c0:c0 + n].copy()))
            want.append(per)
    fr = [serving.Frame(t.cl, t.row, t.units, pinned=True) for t in frames]
    maxc = max(f.n_clusters for f in fr)
    outs = [serving.Outputs(maxc, 36, pinned=True) for _ in range(8)]
    order = [0, 1, 2, 2, 0, 1, 1, 0, 2, 0, 0, 2, 1, 2, 0, 1]
    checked = 0
    with serving.Server(row_x, n_streams=3, budget_bytes=16 << 30) as srv:
        free, inflight = list(range(8)), []

        def finish():
            nonlocal checked
            rid, oi, k = inflight.pop(0)
            r = srv.wait(rid, 300)
            assert r.status == 0 and r.done == 1
            for (tb, hb, ab), (tg, hg, ag) in zip(want[k], serving.unit_results(fr[k], outs[oi])):
                assert tg.tobytes() == tb and np.array_equal(hg, hb) and np.array_equal(ag, ab)
            srv.release(rid)
            free.append(oi)
            checked += 1

        for k in order:
            if not free:
                finish()
            oi = free.pop()
            inflight.append((srv.submit(fr[k], outs[oi]), oi, k))
        while inflight:
            finish()
        st = srv.stats()
    print(f"served {checked} frames on three lanes in {st.batches_run} batches", flush=True)
    assert checked == len(order) and st.completed >= len(order)
