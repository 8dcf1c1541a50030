"""GPU parity: the gfx950 path against the FP32 oracle, element by element.

Sizes span several chunks (1024 clusters) and a ragged tail; the workloads
are the one-sector, central-event and minimum-bias recipes of tpcgen, plus
edge cases (empty unit, one cluster, one row, edge rows only, bad input).
"""
import numpy as np
import pytest

import oracle
import tpcgen
from tests import _parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def tpcca(torch_cuda):
    from paper_1709_00618_amd import tpcca as m
    m.lib()
    return m


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_one_sector_stagewise_host_input(tpcca, row_x):
    b = tpcgen.one_sector(seed=0)
    cl, row, slot, sec, _ = b.unit(0)
    print(f"one sector: {cl.shape[0]} clusters", flush=True)
    ref = oracle.run_sector(cl, row, row_x)
    with tpcca.Context(row_x) as ctx:
        ctx.load_sector(slot, sec, cl, row)
        ctx.find_links(slot, sec)
        ctx.clean_links(slot, sec)
        ctx.build_tracklets(slot, sec)
        ctx.select_tracks(slot, sec)
        ctx.sync()
        _parity.compare_unit_stagewise(ctx, slot, sec, cl, row, ref)
    assert ref.n_tracks > 20


def test_central_event_one_launch_per_stage(tpcca, torch_cuda, row_x):
    """All 36 sectors of a central event in one launch per kernel, inputs in HBM."""
    torch = torch_cuda
    b = tpcgen.central_event(seed=0, keep_truth=False)
    print(f"central event: {b.n_clusters} clusters", flush=True)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    refs = _parity.oracle_units(b, row_x)
    with tpcca.Context(row_x) as ctx:
        for u in range(b.units.shape[0]):
            beg, n, slot, sec = (int(v) for v in b.units[u])
            ctx.load_sector(slot, sec, dcl[beg:beg + n], drow[beg:beg + n], device=True)
        ctx.run_all(0, -1)
        ctx.sync()
        for u in range(b.units.shape[0]):
            cl, row, slot, sec, _ = b.unit(u)
            _parity.compare_unit_stagewise(ctx, slot, sec, cl, row, refs[u])
        # the fit's work counters (the basis of its FLOP count) are the oracle's
        w = ctx.work_stats()
        assert w["fit_steps"] == sum(r.work["propagations"] for r in refs)
        assert w["fit_tests"] == sum(r.work["tests"] for r in refs)
        assert w["fit_updates"] == sum(r.work["updates"] for r in refs)
        assert w["tracklets"] == sum(r.tracklets.shape[0] for r in refs)
    assert sum(r.n_tracks for r in refs) > 15000


@pytest.mark.parametrize("graph", [False, True])
def test_minbias_batch(tpcca, torch_cuda, row_x, graph):
    torch = torch_cuda
    b = tpcgen.minbias_batch(seed=1, n_events=6)
    print(f"batch: {b.units.shape[0]} units, {b.n_clusters} clusters, graph={graph}", flush=True)
    refs = _parity.oracle_units(b, row_x)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(dcl, drow, b.units, device=True, graph=graph)
        units, tracks, hits, asg = ctx.get_batch_results()
    _parity.compare_batch(units, tracks, hits, asg, b, refs)


def _crowded_rows_unit(row_x, n, seed, r=60):
    """Rows r-1 and r+1 with n hits each at almost the same z (so every hit of
    row r has all n in its candidate range) spread in y (so only a few lie
    inside its window), and three hits in row r."""
    rng = np.random.default_rng(seed)
    parts, rows = [], []
    for rr, k in ((r - 1, n), (r, 3), (r + 1, n)):
        y = rng.uniform(-40.0, 40.0, k).astype(np.float32)
        if rr == r:
            y = np.array([0.0, 0.4, -0.3], np.float32)
        else:
            y[:3] = rng.uniform(-0.5, 0.5, 3)  # some inside the window
        z = (10.0 + rng.uniform(-0.05, 0.05, k)).astype(np.float32)
        c = np.stack([np.full(k, row_x[rr], np.float32), y, z, np.ones(k, np.float32)], axis=1)
        parts.append(c)
        rows.append(np.full(k, rr, np.uint8))
    cl = np.concatenate(parts).astype(np.float32)
    row = np.concatenate(rows)
    perm = rng.permutation(cl.shape[0])
    return np.ascontiguousarray(cl[perm]), np.ascontiguousarray(row[perm])


def test_link_candidate_ranges_around_the_mask_limit(tpcca, torch_cuda, row_x):
    """Candidate ranges of 63, 64 and 65 hits per side (the bit-mask scan
    takes up to 64, longer ranges take the full double loop) and of 130:
    links equal the oracle's on both paths."""
    torch = torch_cuda
    cls, rows, units, b0 = [], [], [], 0
    for k, n in enumerate((63, 64, 65, 130)):
        cl, row = _crowded_rows_unit(row_x, n, seed=20 + k)
        cls.append(cl)
        rows.append(row)
        units.append((b0, cl.shape[0], k, k))
        b0 += cl.shape[0]
    cl = np.concatenate(cls)
    row = np.concatenate(rows)
    units = np.array(units, np.int64)
    b = tpcgen.Batch(cl, row, units)
    refs = _parity.oracle_units(b, row_x)
    print(f"crowded rows: {cl.shape[0]} clusters in {units.shape[0]} units", flush=True)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(_dev(torch, cl), _dev(torch, row), units, device=True, graph=False)
        units_r, tracks, hits, asg = ctx.get_batch_results()
        _parity.compare_batch(units_r, tracks, hits, asg, b, refs)
        for u in range(units.shape[0]):
            slot, sec, n = int(units[u, 2]), int(units[u, 3]), int(units[u, 1])
            up, dn = ctx.get_links(slot, sec, n, which=0)  # as found by the neighbour kernel
            assert np.array_equal(up, refs[u].up_raw) and np.array_equal(dn, refs[u].dn_raw), f"unit {u}"
            assert (up >= 0).sum() == 3, f"unit {u}: each hit of the middle row links"
            up, dn = ctx.get_links(slot, sec, n, which=1)
            assert np.array_equal(up, refs[u].up) and np.array_equal(dn, refs[u].dn), f"unit {u}"


def test_dense_rows_time_frame(tpcca, torch_cuda, row_x):
    """Three sector units of a 32-event time frame (about 1400 hits per pad
    row, the dense-row sort that stages a row in LDS), graph and eager."""
    torch = torch_cuda
    tf = tpcgen.timeframe(seed=3, n_events=32)
    parts = [tf.unit(u) for u in (0, 7, 30)]
    off = np.cumsum([0] + [p[0].shape[0] for p in parts])
    units = np.array([(off[i], parts[i][0].shape[0], parts[i][2], parts[i][3]) for i in range(3)], np.int64)
    b = tpcgen.Batch(np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]), units)
    assert b.n_clusters / (3 * (row_x.shape[0] + 1)) >= 1024
    print(f"dense batch: {b.n_clusters} clusters", flush=True)
    refs = _parity.oracle_units(b, row_x)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        for graph in (True, False):
            ctx.run_batch(dcl, drow, b.units, device=True, graph=graph)
            units_r, tracks, hits, asg = ctx.get_batch_results()
            _parity.compare_batch(units_r, tracks, hits, asg, b, refs)


def test_dense_unit_with_an_overfull_row(tpcca, torch_cuda, row_x):
    """A dense unit (mean row above 1024 hits) with one pad row holding more
    hits than the LDS-staged row sort takes (8192): that row takes the
    scatter path inside the same kernel; the result is the oracle's."""
    torch = torch_cuda
    tf = tpcgen.timeframe(seed=4, n_events=32)
    cl, row, slot, sec, _ = tf.unit(5)
    r_full = 80
    base = cl[row == r_full]
    rng = np.random.default_rng(4)
    extra = np.repeat(base, 9000 // base.shape[0] + 1, axis=0)[:9000].copy()
    extra[:, 1] += rng.uniform(-3.0, 3.0, extra.shape[0]).astype(np.float32)  # y
    extra[:, 2] += rng.uniform(-3.0, 3.0, extra.shape[0]).astype(np.float32)  # z
    cl2 = np.concatenate([cl, extra]).astype(np.float32)
    row2 = np.concatenate([row, np.full(extra.shape[0], r_full, np.uint8)])
    perm = rng.permutation(cl2.shape[0])
    cl2, row2 = np.ascontiguousarray(cl2[perm]), np.ascontiguousarray(row2[perm])
    assert (row2 == r_full).sum() > 8192 and cl2.shape[0] / (row_x.shape[0] + 1) >= 1024
    units = np.array([(0, cl2.shape[0], slot, sec)], np.int64)
    b = tpcgen.Batch(cl2, row2, units)
    print(f"overfull row: {cl2.shape[0]} clusters, {(row2 == r_full).sum()} in row {r_full}", flush=True)
    refs = _parity.oracle_units(b, row_x)
    dcl, drow = _dev(torch, cl2), _dev(torch, row2)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(dcl, drow, units, device=True, graph=True)
        units_r, tracks, hits, asg = ctx.get_batch_results()
        _parity.compare_batch(units_r, tracks, hits, asg, b, refs)
        up, dn = ctx.get_links(slot, sec, cl2.shape[0], which=1)
    assert np.array_equal(up, refs[0].up) and np.array_equal(dn, refs[0].dn)


def test_graph_replays_track_changing_batches(tpcca, torch_cuda, row_x):
    """One context, graph replays of different batches, host work between;
    batches of earlier sizes come back (their graphs are replayed from the
    context's cache of captured graphs)."""
    torch = torch_cuda
    batches = [tpcgen.minbias_batch(seed=s, n_events=k) for s, k in ((2, 5), (3, 3), (4, 5))]
    refs = [_parity.oracle_units(b, row_x) for b in batches]
    with tpcca.Context(row_x) as ctx:
        for i in (0, 1, 2, 0, 1, 1, 2):
            b = batches[i]
            print(f"replay batch {i}: {b.n_clusters} clusters", flush=True)
            ctx.run_batch(b.cl, b.row, b.units, device=False, graph=True)
            units, tracks, hits, asg = ctx.get_batch_results()
            _parity.compare_batch(units, tracks, hits, asg, b, refs[i])
        # every batch ran as its graph, none fell back to plain launches
        assert ctx.work_stats()["graph_fallbacks"] == 0


def test_two_frames_in_flight(tpcca, torch_cuda, row_x):
    """Two contexts fed alternately (two frames in flight on one GPU, as the
    pipelined bench runs them): every frame's results are the oracle's."""
    torch = torch_cuda
    frames = [tpcgen.minbias_batch(seed=s, n_events=3) for s in (11, 12)]
    refs = [_parity.oracle_units(b, row_x) for b in frames]
    dev = [(_dev(torch, b.cl), _dev(torch, b.row)) for b in frames]
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as c0, tpcca.Context(row_x) as c1:
        ctxs = (c0, c1)
        for i in range(6):
            k = i % 2
            print(f"frame {i}: context {k}, {frames[k].n_clusters} clusters", flush=True)
            ctxs[k].run_batch(dev[k][0], dev[k][1], frames[k].units, device=True, graph=True)
            if i >= 4:
                # the other context's frame is still in flight here
                units, tracks, hits, asg = ctxs[k].get_batch_results()
                _parity.compare_batch(units, tracks, hits, asg, frames[k], refs[k])
        c0.sync()
        c1.sync()
        assert c0.work_stats()["graph_fallbacks"] == 0 and c1.work_stats()["graph_fallbacks"] == 0


def test_timed_graph_replays_give_the_same_results(tpcca, row_x):
    """Stage timing in graph mode (one graph per stage, events between)
    changes nothing in the results and reports every stage."""
    b = tpcgen.minbias_batch(seed=7, n_events=2)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(b.cl, b.row, b.units, graph=True)
        base = [a.copy() for a in ctx.get_batch_results()]
        ctx.set_timing(True)
        for _ in range(2):
            ctx.run_batch(b.cl, b.row, b.units, graph=True)
            ctx.sync()
            got = ctx.get_batch_results()
            st = ctx.stage_times()
            assert len(st) == 6 and all(v > 0 for v in st.values()), st
            for x, y in zip(base, got):
                assert x.tobytes() == y.tobytes()
        ctx.set_timing(False)
        ctx.run_batch(b.cl, b.row, b.units, graph=True)
        for x, y in zip(base, ctx.get_batch_results()):
            assert x.tobytes() == y.tobytes()


def test_batch_equals_sector_by_sector(tpcca, row_x):
    """A unit's results do not depend on the batch it runs in."""
    b = tpcgen.minbias_batch(seed=5, n_events=3)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(b.cl, b.row, b.units, graph=True)
        units, tracks, hits, asg = ctx.get_batch_results()
    with tpcca.Context(row_x) as ctx:
        for u in range(b.units.shape[0]):
            cl, row, slot, sec, _ = b.unit(u)
            ctx.load_sector(slot, sec, cl, row)
            ctx.run_all(slot, sec)
        ctx.sync()
        for u in range(b.units.shape[0]):
            cl, row, slot, sec, _ = b.unit(u)
            tr, h = ctx.get_tracks(slot, sec)
            ur = units[u]
            t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
            h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
            assert tr.tobytes() == tracks[t0:t0 + nt].tobytes()
            assert np.array_equal(h, hits[h0:h0 + nh])
            a = ctx.get_assignment(slot, sec, cl.shape[0])
            c0 = int(ur["cluster_begin"])
            assert np.array_equal(a, asg[c0:c0 + cl.shape[0]])


@pytest.mark.parametrize("knobs", [
    dict(fit_pool=16, fit_min_waves=0, grid_hits_per_bin=2, link_blocks_per_cu=8, fit_claims=1,
         fit_xcd_slices=0, link_stage=1, fit_long_first=20, fit_row_bands=30, fit_tail_units=50),
    dict(fit_pool=128, fit_min_waves=6, grid_hits_per_bin=1, link_blocks_per_cu=16, fit_claims=0,
         fit_xcd_slices=1, link_stage=2, fit_long_first=3, fit_row_bands=159),
    dict(fit_pool=32, fit_min_waves=4, fit_blocks_per_cu=2, grid_hits_per_bin=4, link_blocks_per_cu=32,
         fit_claims=1, fit_xcd_slices=1, fit_row_bands=7, fit_tail_units=40),
    # the row-synchronous fit: small chunks on few blocks, large chunks with
    # the claims in a kernel of their own
    dict(fit_rows=64, fit_blocks_per_cu=1),
    dict(fit_rows=1024, fit_claims=0, grid_hits_per_bin=2),
    dict(fit_rows=384),
    # neighbour tiles of 128 and 512 hits, fit blocks of 64 and 256 threads
    dict(link_tile=128, fit_block=64, fit_blocks_per_cu=10),
    dict(link_tile=512, fit_block=256, link_stage=1, fit_min_waves=4),
])
def test_schedule_does_not_change_results(tpcca, row_x, knobs):
    """Every launch schedule gives the default schedule's bytes and the oracle's results."""
    b = tpcgen.minbias_batch(seed=6, n_events=3)
    print(f"schedule {knobs}: {b.n_clusters} clusters", flush=True)
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(b.cl, b.row, b.units, graph=True)
        base = [a.copy() for a in ctx.get_batch_results()]
    with tpcca.Context(row_x) as ctx:
        ctx.set_tuning(**knobs)
        assert all(ctx.get_tuning()[k] == v for k, v in knobs.items())
        for graph in (False, True):
            ctx.run_batch(b.cl, b.row, b.units, graph=graph)
            got = ctx.get_batch_results()
            for x, y in zip(base, got):
                assert x.tobytes() == y.tobytes()
    refs = _parity.oracle_units(b, row_x, which={0, 20, 50})
    units, tracks, hits, asg = base
    for u in (0, 20, 50):
        ur = units[u]
        t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
        h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
        c0, n = int(ur["cluster_begin"]), int(b.units[u, 1])
        _parity.compare_tracks(tracks[t0:t0 + nt], hits[h0:h0 + nh], refs[u])
        assert np.array_equal(asg[c0:c0 + n], refs[u].assignment)


def _edge_units(row_x):
    rng = np.random.default_rng(9)
    units = []
    units.append(("empty", np.zeros((0, 4), np.float32), np.zeros(0, np.uint8)))
    units.append(("one", np.array([[row_x[5], 1.0, 20.0, 1.0]], np.float32), np.array([5], np.uint8)))
    # all clusters in one row
    k = 3000
    cl = np.stack([np.full(k, row_x[40]), rng.uniform(-20, 20, k), rng.uniform(0, 250, k), np.ones(k)], 1)
    units.append(("one row", cl.astype(np.float32), np.full(k, 40, np.uint8)))
    # only the edge rows (no links can form there)
    k = 500
    r = np.where(rng.random(k) < 0.5, 0, 158).astype(np.uint8)
    cl = np.stack([row_x[r], rng.uniform(-10, 10, k), rng.uniform(0, 250, k), np.ones(k)], 1)
    units.append(("edge rows", cl.astype(np.float32), r))
    # dense straight tracks with many exact duplicates (ties by ID), ragged size
    b = tpcgen.one_sector(seed=7, sigma=0.0)
    cl, row, _, _, _ = b.unit(0)
    dup = rng.choice(cl.shape[0], 777, replace=False)
    cl = np.concatenate([cl, cl[dup]])
    row = np.concatenate([row, row[dup]])
    units.append(("duplicates", cl, row))
    # a sector of a time frame: z' spans tens of metres
    tf = tpcgen.timeframe(seed=3, n_events=12)
    cl, row, _, _, _ = tf.unit(4)
    units.append(("timeframe sector", cl, row))
    return units


def test_edge_cases(tpcca, row_x):
    units = _edge_units(row_x)
    with tpcca.Context(row_x) as ctx:
        for k, (name, cl, row) in enumerate(units):
            ctx.load_sector(0, k, cl, row)
        ctx.run_all(0, -1)
        ctx.sync()
        for k, (name, cl, row) in enumerate(units):
            print(f"edge case {name}: {cl.shape[0]} clusters", flush=True)
            ref = oracle.run_sector(cl, row, row_x)
            _parity.compare_unit_stagewise(ctx, 0, k, cl, row, ref)


def test_invalid_clusters_are_reported(tpcca, row_x):
    b = tpcgen.one_sector(seed=1)
    cl, row, _, _, _ = b.unit(0)
    row = row.copy()
    row[17] = 200  # beyond the last pad row
    with tpcca.Context(row_x) as ctx:
        ctx.load_sector(0, 0, cl, row)
        ctx.run_all(0, 0)
        with pytest.raises(tpcca.TpccaError) as ei:
            ctx.sync()
        assert ei.value.status == tpcca.EINVAL
    cl2 = cl.copy()
    cl2[3, 0] += 1.0  # x off its row
    with tpcca.Context(row_x) as ctx:
        ctx.load_sector(0, 0, cl2, b.unit(0)[1])
        ctx.run_all(0, 0)
        with pytest.raises(tpcca.TpccaError):
            ctx.sync()


def test_units_beyond_the_24_bit_index_are_refused(tpcca, row_x):
    """n > 2^24 - 1 is EINVAL before anything is read (the buffers here hold
    only 64 clusters), and the context stays usable afterwards."""
    import ctypes
    b = tpcgen.one_sector(seed=1)
    cl, row, _, _, _ = b.unit(0)
    small_cl = np.ascontiguousarray(cl[:64], np.float32)
    small_row = np.ascontiguousarray(row[:64], np.uint8)
    with tpcca.Context(row_x) as ctx:
        st = tpcca.lib().tpcca_load_sector(ctx.h, 0, 0, small_cl.ctypes.data, small_row.ctypes.data, 1 << 24,
                                           tpcca.MEM_HOST)
        assert st == tpcca.EINVAL
        with pytest.raises(tpcca.TpccaError) as ei:
            ctx.run_batch(small_cl, small_row, [(0, 1 << 24, 0, 0)])
        assert ei.value.status == tpcca.EINVAL
        ctx.reset()
        ctx.load_sector(0, 0, cl, row)
        ctx.run_all(0, 0)
        ctx.sync()
        _parity.compare_unit_stagewise(ctx, 0, 0, cl, row, oracle.run_sector(cl, row, row_x))


def test_stage_order_and_arguments(tpcca, row_x):
    b = tpcgen.one_sector(seed=1)
    cl, row, _, _, _ = b.unit(0)
    with tpcca.Context(row_x) as ctx:
        with pytest.raises(tpcca.TpccaError) as ei:
            ctx.clean_links(0, 0)
        assert ei.value.status == tpcca.ESTATE
        ctx.load_sector(0, 0, cl, row)
        with pytest.raises(tpcca.TpccaError):
            ctx.load_sector(0, 0, cl, row)  # loaded twice
        with pytest.raises(tpcca.TpccaError):
            ctx.build_tracklets(0, 0)       # links not found yet
        with pytest.raises(tpcca.TpccaError):
            ctx.load_sector(0, 99, cl, row)  # no sector 99
        ctx.find_links(0, 0)
        with pytest.raises(tpcca.TpccaError):
            ctx.get_links(0, 0, cl.shape[0] + 1)
        ctx.clean_links(0, 0)
        ctx.build_tracklets(0, 0)
        ctx.select_tracks(0, 0)
        ctx.sync()


def test_fit_within_1e4_of_fp64_replay(tpcca, row_x):
    """GPU tracklets of a central event against the FP64 oracle replayed
    along the GPU's own decisions: the precision criterion of tests/_fp64.py
    (every tracklet within 0.1 sigma64, at most 0.5 % missing
    1e-4 max(|p64|, sigma64))."""
    from tests import _fp64
    b = tpcgen.central_event(seed=4, n_tracks=8000, keep_truth=False)
    checked = 0
    with tpcca.Context(row_x) as ctx:
        for u in (0, 13, 29):
            cl, row, slot, sec, _ = b.unit(u)
            ctx.load_sector(slot, sec, cl, row)
        ctx.run_all(0, -1)
        ctx.sync()
        for u in (0, 13, 29):
            cl, row, slot, sec, _ = b.unit(u)
            gt, ghb, gh = ctx.get_tracklets(slot, sec)
            st = _fp64.compare(cl, row, row_x, gt, ghb, gh)
            print(_fp64.summary(f"central event, unit {u}", st), flush=True)
            _fp64.check(st)
            checked += st["tracklets"]
    assert checked > 1500


def test_tile_size_is_fixed_once_units_are_loaded(tpcca, row_x):
    """The neighbour tile size sets the tile reservations of loaded units:
    changing it then is refused; after a reset it is accepted."""
    b = tpcgen.minbias_batch(seed=2, n_events=1)
    with tpcca.Context(row_x) as ctx:
        cl, row, slot, sec, _ = b.unit(0)
        ctx.load_sector(slot, sec, cl, row)
        with pytest.raises(tpcca.TpccaError):
            ctx.set_tuning(link_tile=128)
        ctx.set_tuning(link_tile=256, fit_block=64)  # the default tile: accepted
        ctx.reset()
        ctx.set_tuning(link_tile=512)
        ctx.load_sector(slot, sec, cl, row)
        ctx.run_all(slot, sec)
        ctx.sync()
        tr, h = ctx.get_tracks(slot, sec)
    ref = _parity.oracle_units(b, row_x, which={0})[0]
    _parity.compare_tracks(tr, h, ref)
    with tpcca.Context(row_x) as ctx:
        with pytest.raises(tpcca.TpccaError):
            ctx.set_tuning(link_tile=300)
        with pytest.raises(tpcca.TpccaError):
            ctx.set_tuning(fit_block=96)


def test_row_synchronous_fit_on_a_time_frame(tpcca, row_x):
    """The row-synchronous fit on a 32-event time frame (dense rows, z' over
    tens of metres) gives the per-lane fit's tracklets, tracks and
    assignment byte for byte, the same device work counts, and the oracle's
    results on three units."""
    tf = tpcgen.timeframe(seed=3, n_events=32)
    print(f"time frame: {tf.n_clusters} clusters in {tf.units.shape[0]} units", flush=True)
    out = {}
    for rows in (0, 384, 160):
        with tpcca.Context(row_x) as ctx:
            ctx.set_tuning(fit_rows=rows)
            ctx.run_batch(tf.cl, tf.row, tf.units, graph=True)
            res = [a.copy() for a in ctx.get_batch_results()]
            trk = {}
            for u in (0, 13, 35):
                _, _, slot, sec, _ = tf.unit(u)
                trk[u] = [a.copy() for a in ctx.get_tracklets(slot, sec)]
            w = ctx.work_stats()
        print(f"fit_rows={rows}: {w}", flush=True)
        out[rows] = (res, trk, w)
    base = out[0]
    for rows in (384, 160):
        res, trk, w = out[rows]
        for x, y in zip(base[0], res):
            assert x.tobytes() == y.tobytes()
        for u in trk:
            for x, y in zip(base[1][u], trk[u]):
                assert x.tobytes() == y.tobytes()
        for k in ("fit_steps", "fit_candidates", "fit_tests", "fit_updates", "tracklets", "tracks",
                  "track_hits", "graph_fallbacks"):
            assert w[k] == base[2][k], k
    refs = _parity.oracle_units(tf, row_x, which={0, 13, 35})
    units, tracks, hits, asg = out[384][0]
    for u in (0, 13, 35):
        ur = units[u]
        t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
        h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
        c0, n = int(ur["cluster_begin"]), int(tf.units[u, 1])
        _parity.compare_tracks(tracks[t0:t0 + nt], hits[h0:h0 + nh], refs[u])
        assert np.array_equal(asg[c0:c0 + n], refs[u].assignment)
