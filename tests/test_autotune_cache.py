"""The schedule autotuner's cache and search (CPU only): size buckets, the
committed entry for the time frame on gfx950 (knobs that exist and are in
range), a store/lookup round trip, that the default schedule is the search's
first point, and the coordinate search on a timing model."""
import itertools
import json

from paper_1709_00618_amd import autotune, tpcca


def test_buckets():
    assert autotune.bucket(32_513_174, 36) == "cl2^24_u36"
    assert autotune.bucket(4_690, 1) == "cl2^12_u1"
    assert autotune.bucket(16_000_000, 2304) == "cl2^23_umany"
    assert autotune.bucket(0, 0) == "cl2^0_u1"


def test_committed_time_frame_entry_is_valid():
    e = autotune.lookup(32_513_174, 36, dev="gfx950")
    assert e is not None, "no cached schedule for the time frame on gfx950"
    fields = {k for k, _ in tpcca.Tuning._fields_}
    assert set(e["knobs"]) <= fields
    k = e["knobs"]
    assert k.get("link_stage", 0) in (0, 1, 2)
    assert k.get("fit_min_waves", 0) in (0, 4, 5, 6)
    assert 0 <= k.get("fit_blocks_per_cu", 0) <= 64 and 0 < k.get("fit_pool", 64) <= 4096
    for name, vals in autotune.SPACE.items():
        assert k.get(name, vals[0]) in vals or name not in k


def test_store_and_lookup_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "cache.json"
    monkeypatch.setattr(autotune, "CACHE", str(path))
    assert autotune.lookup(1 << 20, 36, dev="gfxTEST") is None
    autotune.store({"knobs": {"fit_pool": 128}, "ms": 1.0}, 1 << 20, 36, dev="gfxTEST", path=str(path))
    assert autotune.lookup((1 << 20) + 5, 30, dev="gfxTEST")["knobs"] == {"fit_pool": 128}
    assert json.load(open(path))["gfxTEST"]["cl2^20_u36"]["ms"] == 1.0


def test_default_schedule_is_in_the_space():
    names = list(autotune.SPACE)
    table = [(0.0, dict(zip(names, c))) for c in itertools.product(*(autotune.SPACE[n] for n in names))]
    assert autotune._default(table) is not None
    import ctypes
    d = tpcca.Tuning()
    tpcca.lib().tpcca_tuning_default(ctypes.byref(d))
    for k, v in autotune.DEFAULT.items():
        assert getattr(d, k) == v, k  # the schedule a new context starts with


class _ModelCtx:
    """Stands in for a context: run_batch 'takes' a time that is a sum of
    per-knob costs (minimum at a known point), measured by _time."""
    best = {"fit_block": 256, "fit_blocks_per_cu": 8, "fit_min_waves": 0, "fit_pool": 32, "link_stage": 1,
            "link_tile": 0}

    def __init__(self):
        self.knobs = {}
        self.calls = []

    def reset(self):
        pass

    def set_tuning(self, **kw):
        self.knobs = dict(kw)
        self.calls.append(dict(kw))

    def cost(self):
        return sum(0.0 if self.knobs.get(k) == v else 1.0 + 0.1 * autotune.SPACE[k].index(self.knobs.get(k, 0))
                   for k, v in self.best.items())

    def run_batch(self, *a, **k):
        pass

    def sync(self):
        pass


def test_coordinate_search_finds_a_separable_optimum(monkeypatch):
    ctx = _ModelCtx()
    monkeypatch.setattr(autotune, "_time", lambda c, run, reps: c.cost())
    best, table = autotune.tune(ctx, None, None, [0], log=None)
    assert best == ctx.best
    assert table[0][1] == ctx.best and table[0][0] == 0.0
    n_points = 1 + sum(len(v) - 1 for v in autotune.SPACE.values())
    assert len(table) == n_points  # each knob's values once, the default point once
    assert ctx.knobs == ctx.best  # the context is left on the best schedule
