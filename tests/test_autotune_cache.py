"""The schedule autotuner's cache (CPU only): size buckets, the committed
entry for the time frame on gfx950 (knobs that exist and are in range), a
store/lookup round trip, and that the default schedule is a point of the
search space (so the tuner always times it)."""
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
