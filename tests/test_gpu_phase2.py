"""GPU parity of the measured workloads and of the second phase.

* the benchmark's own time frame (128 minimum-bias events, seed 0, 36 units,
  about 32.5 M clusters): every unit of the sector tracker bit for bit, the
  second phase (merging and refit, vertices, flags, compression) bit for bit,
  the decompression round trip of every hit, the FP64 criterion on a sample
  of tracklets;
* a batch of 64 minimum-bias events in one launch (2304 units, events of 10
  to 8000 tracks): the same per event, with the FP64 criterion on units of
  the smallest and the largest event;
* a central event: the second phase and the round trip.

The oracle's near-tie counts (decisions with a relative margin below 1e-6)
are printed; no exception to bit-exactness is needed.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import tpcgen
from tests import _fp64, _parity
from tests import _phase2_parity as p2p

pytestmark = pytest.mark.gpu

F32 = np.float32


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


def _oracle_units(batch, row_x, workers=16):
    def one(u):
        cl, row, _, _, _ = batch.unit(u)
        return oracle.run_sector(cl, row, row_x, precision=32)
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, range(batch.units.shape[0])))


def _round_trip(torch, ctx, batch, units, hits):
    """Decompress every segment on the GPU from the phase's records and
    residuals; compare with the quantised clusters and rows of the tracks'
    hits.  Returns (hits checked, mismatches)."""
    v = ctx.phase2_view()
    n = max(1, int(units["n_track_hits"].sum()))
    yq = torch.full((n,), -(2 ** 31), dtype=torch.int32, device="cuda")
    zq = torch.full((n,), -(2 ** 31), dtype=torch.int32, device="cuda")
    rows = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ctx.decompress(v.n_seg, v.seg_n_hits, v.seg_hit_begin, v.rec, v.res, yq, zq, rows)
    ctx.sync()
    yq_h, zq_h, rows_h = yq.cpu().numpy(), zq.cpu().numpy(), rows.cpu().numpy()
    q = np.float32(0.01)
    mism, checked = 0, 0
    # one run from cluster 0: the device hit positions are the batch-relative ones
    for u in range(batch.units.shape[0]):
        beg, nc, _, _ = (int(x) for x in batch.units[u])
        h0, nh = int(units["hit_begin"][u]), int(units["n_track_hits"][u])
        ids = hits[h0:h0 + nh]
        cl = batch.cl[beg:beg + nc]
        wy = np.rint(cl[ids, 1] / q).astype(np.int32)
        wz = np.rint(cl[ids, 2] / q).astype(np.int32)
        mism += int(np.count_nonzero(yq_h[h0:h0 + nh] != wy) + np.count_nonzero(zq_h[h0:h0 + nh] != wz)
                    + np.count_nonzero(rows_h[h0:h0 + nh] != batch.row[beg:beg + nc][ids]))
        checked += nh
    return checked, mism


def _fp64_sample(ctx, batch, row_x, units_idx, per_unit=400, seed=0):
    """FP64 criterion (tests/_fp64.py) on a sample of GPU tracklets."""
    stats = []
    for u in units_idx:
        cl, row, slot, sec, _ = batch.unit(int(u))
        gt, ghb, gh = ctx.get_tracklets(slot, sec)
        st = _fp64.compare(cl, row, row_x, gt, ghb, gh, max_tracklets=per_unit, seed=seed)
        print(_fp64.summary(f"unit {u} (slot {slot}, sector {sec})", st), flush=True)
        stats.append(st)
    dev = np.max([s["max_dev_sigma"] for s in stats], axis=0)
    n = sum(s["tracklets"] for s in stats)
    fails = sum(s["fail"] for s in stats)
    assert np.all(dev <= _fp64.MAX_DEV_SIGMA), dev
    assert fails <= _fp64.MAX_FAIL_FRAC * n, (fails, n)
    return n


def test_phase2_central_event(tpcca, torch_cuda, row_x):
    torch = torch_cuda
    b = tpcgen.central_event(seed=0, keep_truth=False)
    print(f"central event: {b.n_clusters} clusters", flush=True)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(dcl, drow, b.units, device=True, graph=True)
        ctx.phase2()
        ctx.sync()
        s = p2p.compare_slot(ctx, b, row_x, 0)
        units, tracks, hits, _ = ctx.get_batch_results()
        checked, mism = _round_trip(torch, ctx, b, units, hits)
    print(f"second phase, central event: {s}; round trip {checked} hits, {mism} mismatches", flush=True)
    assert mism == 0 and checked > 900000
    assert s["merges"] > 5000 and s["vertices"] >= 1


def test_bench_time_frame_parity(tpcca, torch_cuda, row_x):
    """The benchmark's time frame, as the benchmark runs it (device inputs,
    graph replay, the cached schedule): all 36 units equal the FP32 oracle, the second phase
    equals the oracle's, every hit survives the compression round trip, and
    a sample of tracklets meets the FP64 criterion."""
    torch = torch_cuda
    tf = tpcgen.timeframe(seed=0, n_events=128)
    print(f"benchmark time frame: {tf.n_clusters} clusters in {tf.units.shape[0]} units", flush=True)
    refs = _oracle_units(tf, row_x)
    print(f"oracle near-ties: {sum(r.near_ties for r in refs)}, min margin "
          f"{min(r.min_margin for r in refs):.2e}", flush=True)
    dcl, drow = _dev(torch, tf.cl), _dev(torch, tf.row)
    torch.cuda.synchronize()
    # the schedule the benchmark applies to this frame (its cached entry)
    from paper_1709_00618_amd import autotune
    entry = autotune.lookup(tf.n_clusters, len(tf.units))
    knobs = entry["knobs"] if entry else {}
    print(f"schedule: {knobs or 'default'}", flush=True)
    with tpcca.Context(row_x) as ctx:
        if knobs:
            ctx.set_tuning(**knobs)
        ctx.run_batch(dcl, drow, tf.units, device=True, graph=True)
        units, tracks, hits, asg = ctx.get_batch_results()
        _parity.compare_batch(units, tracks, hits, asg, tf, refs)
        print("sector tracker: all units bit-exact", flush=True)
        ctx.phase2()
        ctx.sync()
        s = p2p.compare_slot(ctx, tf, row_x, 0)
        print(f"second phase: {s}", flush=True)
        checked, mism = _round_trip(torch, ctx, tf, units, hits)
        print(f"round trip: {checked} hits, {mism} mismatches", flush=True)
        assert mism == 0 and checked > 2.5e7
        n = _fp64_sample(ctx, tf, row_x, units_idx=(0, 11, 17, 30), per_unit=300)
    assert n >= 1000
    assert s["vertices"] >= 100


def test_minbias_64_events_one_launch(tpcca, torch_cuda, row_x):
    """64 minimum-bias events (10 to 8000 tracks) in one launch: every unit
    equals the oracle, the second phase of every event equals the oracle's,
    and units of the smallest and the largest event meet the FP64
    criterion."""
    torch = torch_cuda
    b = tpcgen.minbias_batch(seed=0, n_events=64)
    mult = b.meta["multiplicity"]
    print(f"minimum-bias batch: {b.units.shape[0]} units, {b.n_clusters} clusters, tracks per event "
          f"{mult.min()}..{mult.max()}", flush=True)
    refs = _oracle_units(b, row_x)
    print(f"oracle near-ties: {sum(r.near_ties for r in refs)}", flush=True)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(dcl, drow, b.units, device=True, graph=True)
        units, tracks, hits, asg = ctx.get_batch_results()
        _parity.compare_batch(units, tracks, hits, asg, b, refs)
        ctx.phase2()
        ctx.sync()
        tot = {"finals": 0, "merges": 0, "vertices": 0, "near_ties": 0}
        for ev in range(64):
            s = p2p.compare_slot(ctx, b, row_x, ev, check_compression=(ev % 8 == 0))
            for k in tot:
                tot[k] += s[k]
        print(f"second phase over 64 events: {tot}", flush=True)
        checked, mism = _round_trip(torch, ctx, b, units, hits)
        assert mism == 0
        sizes = np.bincount(b.units[:, 2], weights=b.units[:, 1])
        big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
        pick = [u for u in range(b.units.shape[0]) if int(b.units[u, 2]) in (big, small) and b.units[u, 1] > 0]
        _fp64_sample(ctx, b, row_x, units_idx=pick[::6], per_unit=200)


def test_phase2_stage_errors(tpcca, row_x):
    """The phase needs every unit selected; getters need the phase."""
    b = tpcgen.minbias_batch(seed=9, n_events=1)
    with tpcca.Context(row_x) as ctx:
        with pytest.raises(tpcca.TpccaError):
            ctx.phase2()  # nothing loaded
        cl, row, slot, sec, _ = b.unit(3)
        ctx.load_sector(slot, sec, cl, row)
        ctx.find_links(slot, sec)
        with pytest.raises(tpcca.TpccaError):
            ctx.phase2()  # not selected yet
        with pytest.raises(tpcca.TpccaError):
            ctx.get_finals(slot)
        ctx.clean_links(slot, sec)
        ctx.build_tracklets(slot, sec)
        ctx.select_tracks(slot, sec)
        ctx.phase2()
        ctx.sync()
        f, h = ctx.get_finals(slot)
        tr, _ = ctx.get_tracks(slot, sec)
        assert f.shape[0] == tr.shape[0] and np.all(f["n_seg"] == 1)  # one sector: nothing to merge
    with pytest.raises(tpcca.TpccaError):
        tpcca.Context(row_x).set_phase2_params(max_sinphi=1.5)


def test_phase2_without_tracks_and_with_a_tiny_event(tpcca, torch_cuda, row_x):
    """Degenerate inputs of the second phase: units that yield no track at
    all (the per-lane loops and their longest-first orders get no items),
    then a single minimum-bias event of 68 tracks against the oracle."""
    rng = np.random.default_rng(5)
    k = 2000
    cl = np.stack([np.full(k, row_x[40]), rng.uniform(-20, 20, k), rng.uniform(0, 250, k), np.ones(k)],
                  1).astype(np.float32)
    row = np.full(k, 40, np.uint8)
    with tpcca.Context(row_x) as ctx:
        ctx.load_sector(0, 0, cl, row)
        ctx.load_sector(0, 1, cl, row)
        ctx.run_all(0, -1)
        ctx.phase2()
        ctx.sync()
        finals, hits = ctx.get_finals(0)
        assert finals.shape[0] == 0 and hits.shape[0] == 0
        assert ctx.get_vertices(0).shape[0] == 0
    torch = torch_cuda
    b = tpcgen.minbias_batch(seed=8, n_events=1)
    print(f"tiny event: {int(b.meta['multiplicity'][0])} tracks, {b.n_clusters} clusters", flush=True)
    dcl, drow = _dev(torch, b.cl), _dev(torch, b.row)
    torch.cuda.synchronize()
    with tpcca.Context(row_x) as ctx:
        ctx.run_batch(dcl, drow, b.units, device=True, graph=False)
        ctx.phase2()
        ctx.sync()
        s = p2p.compare_slot(ctx, b, row_x, 0)
    print(f"second phase, tiny event: {s}", flush=True)
    assert s["finals"] > 0
