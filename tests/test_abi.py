"""The C ABI library: it loads, exports what include/tpcca.h declares, and
its defaults agree with the oracle's reading (no GPU needed)."""
import os
import re

import numpy as np

import oracle
from paper_1709_00618_amd import tpcca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tpcca.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpcca_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tpcca.lib()
    names = _declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(tpcca.SYMBOLS)


def test_struct_layouts():
    import ctypes
    assert tpcca.TRACK_DTYPE.itemsize == 108
    assert ctypes.sizeof(tpcca.Params) == 22 * 4
    assert ctypes.sizeof(tpcca.Timeframe) == 13 * 8


def test_defaults_match_the_oracle_reading():
    g = tpcca.params_default()
    o = oracle.default_params()
    for name, _ in oracle.Params._fields_:
        assert np.float32(getattr(g, name)) == np.float32(getattr(o, name)), name
    assert g.grid_hits_per_bin >= 1


def test_phase2_defaults_match_the_oracle_reading():
    g = tpcca.phase2_params_default()
    o = oracle.default_p2params()
    for name, _ in oracle.P2Params._fields_:
        assert np.float32(getattr(g, name)) == np.float32(getattr(o, name)), name
    assert [n for n, _ in tpcca.Phase2Params._fields_] == [n for n, _ in oracle.P2Params._fields_]


def test_error_strings():
    for s in (tpcca.OK, tpcca.EINVAL, tpcca.ENOMEM, tpcca.ECAPACITY, tpcca.EDEVICE, tpcca.ESTATE,
              tpcca.EBUSY, tpcca.ENOTFOUND):
        assert tpcca.error_string(s) not in ("", "unknown status")
    assert tpcca.error_string(12345) == "unknown status"


def test_product_path_does_not_touch_the_oracle():
    """The package and its sources never import or link the oracle."""
    pkg = os.path.join(ROOT, "paper_1709_00618_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "tpcref" not in text and "import oracle" not in text, f


def test_allocation_free_entry_point_validates_on_the_host(row_x):
    """Bad units, capacities and sizes are refused before any device work:
    the pointers below are never dereferenced, so this runs without a GPU."""
    import ctypes
    L = tpcca.lib()
    geo = tpcca.Geometry(36, len(row_x), row_x.ctypes.data_as(ctypes.c_void_p))
    prm = tpcca.params_default()
    fake = ctypes.c_void_p(0x1000)  # stands for a device address; never read

    def call(n, sector=0, flags=tpcca.MEM_DEVICE, tracks_cap=None, hits_cap=None):
        n = np.asarray(n, np.int32)
        U = len(n)
        slot = np.zeros(U, np.int32)
        sec = np.full(U, sector, np.int32)
        begin = np.zeros(U, np.int64)
        bt = tpcca.Batch(U, slot.ctypes.data, sec.ctypes.data, begin.ctypes.data, n.ctypes.data,
                         fake, fake, flags)
        tot = int(n.clip(0).sum())
        tc = tot if tracks_cap is None else tracks_cap
        hc = tot if hits_cap is None else hits_cap
        nt, nh = ctypes.c_int64(-1), ctypes.c_int64(-1)
        return L.tpcca_run_batch_noalloc(ctypes.byref(geo), ctypes.byref(prm), 0, None, ctypes.byref(bt),
                                         fake, tc, fake, hc, fake, tot, fake, ctypes.byref(nt),
                                         ctypes.byref(nh))

    assert call([1 << 24]) == tpcca.EINVAL            # beyond the 24-bit unit-local index
    assert call([5, -1]) == tpcca.EINVAL
    assert call([5], sector=36) == tpcca.EINVAL
    assert call([5], flags=tpcca.MEM_HOST) == tpcca.EINVAL
    assert call([5], flags=tpcca.MEM_DEVICE | tpcca.BATCH_GRAPH) == tpcca.EINVAL
    assert call([300], tracks_cap=0) == tpcca.ECAPACITY
    assert call([300], hits_cap=299) == tpcca.ECAPACITY
    big = (1 << 24) - 1                                   # a legal unit, but beyond the fixed array
    assert call([big], tracks_cap=1 << 24) == tpcca.ENOMEM
