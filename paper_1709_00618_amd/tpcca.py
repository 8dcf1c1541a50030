"""ctypes binding of libtpcca.so (the gfx950 TPC sector tracker).

Argument marshalling only: every step of the tracker runs in the HIP kernels
of libtpcca.so.  The functions keep the C names (``tpcca_create`` ...); the
``Context`` and ``Server`` classes wrap them for numpy / torch callers.  There
is no fallback: if the shared library is missing or cannot be loaded, the
import of this module's ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpcca.so")

OK, EINVAL, ENOMEM, ECAPACITY, EDEVICE, ESTATE, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
MEM_HOST, MEM_DEVICE, BATCH_GRAPH = 0, 1, 2

c_i32, c_i64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p


class TpccaError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: status {status} ({error_string(status)}) {detail}".strip())


class Geometry(ctypes.Structure):
    _fields_ = [("n_sectors", c_i32), ("n_rows", c_i32), ("row_x", c_vp)]


class Params(ctypes.Structure):
    _fields_ = [
        ("n_rows", c_i32), ("link_wy", c_f32), ("link_wz", c_f32), ("link_chi2", c_f32),
        ("min_chain_hits", c_i32), ("kB", c_f32), ("err2_y", c_f32), ("err2_z", c_f32),
        ("max_sinphi", c_f32), ("seed_c22", c_f32), ("seed_c33", c_f32), ("seed_c44", c_f32),
        ("reset_c00", c_f32), ("reset_c11", c_f32), ("pick_nsig", c_f32), ("pick_win_max", c_f32),
        ("pick_chi2", c_f32), ("max_miss", c_i32), ("min_track_hits", c_i32), ("own_frac_pct", c_i32),
        ("refit_inflate", c_f32), ("grid_hits_per_bin", c_i32),
    ]


class Batch(ctypes.Structure):
    _fields_ = [("n_units", c_i32), ("slot", c_vp), ("sector", c_vp), ("begin", c_vp), ("n", c_vp),
                ("cl", c_vp), ("row", c_vp), ("flags", c_i32)]


class DeviceResults(ctypes.Structure):
    _fields_ = [("tracks", c_vp), ("hits", c_vp), ("assignment", c_vp), ("units", c_vp), ("n_units", c_i32)]


class WorkStats(ctypes.Structure):
    _fields_ = [("clusters", c_i64), ("tracklets", c_i64), ("tracks", c_i64), ("track_hits", c_i64),
                ("fit_steps", c_i64), ("fit_candidates", c_i64), ("fit_tests", c_i64),
                ("fit_updates", c_i64), ("fit_wave_iterations", c_i64), ("fit_ns", c_i64),
                ("fit_drain_ns", c_i64), ("graph_fallbacks", c_i64)]


class Tuning(ctypes.Structure):
    _fields_ = [("fit_pool", c_i32), ("fit_blocks_per_cu", c_i32), ("grid_hits_per_bin", c_i32),
                ("link_blocks_per_cu", c_i32), ("fit_min_waves", c_i32), ("fit_claims", c_i32),
                ("fit_xcd_slices", c_i32), ("link_stage", c_i32), ("fit_long_first", c_i32),
                ("fit_row_bands", c_i32), ("fit_tail_units", c_i32), ("fit_rows", c_i32),
                ("link_tile", c_i32), ("fit_block", c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timeframe(ctypes.Structure):
    _fields_ = [("n_units", c_i32), ("sector", c_vp), ("begin", c_vp), ("n", c_vp), ("cl", c_vp),
                ("row", c_vp), ("tracks", c_vp), ("tracks_cap", c_i64), ("hits", c_vp),
                ("hits_cap", c_i64), ("assignment", c_vp), ("units", c_vp), ("arrival_s", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", c_i32), ("done", c_i32), ("n_tracks", c_i64), ("n_hits", c_i64),
                ("arrival_s", ctypes.c_double), ("start_s", ctypes.c_double), ("end_s", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("rejected", c_i64), ("clusters_done", c_i64),
                ("tracks_done", c_i64), ("bytes_in_flight", c_i64), ("bytes_budget", c_i64),
                ("queue_depth", c_i32), ("batches_run", c_i32), ("busy_s", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double)]


class Phase2Params(ctypes.Structure):
    _fields_ = [
        ("sector_cos", c_f32), ("sector_sin", c_f32), ("max_sinphi", c_f32), ("merge_dz_ends", c_f32),
        ("merge_max_gap", c_i32), ("merge_wy", c_f32), ("merge_wz", c_f32), ("merge_chi2", c_f32),
        ("refit_inflate", c_f32), ("dca_steps", c_i32), ("vdrift", c_f32), ("vtx_gap_us", c_f32),
        ("vtx_min_tracks", c_i32), ("vtx_min_hits", c_i32), ("vtx_attach_us", c_f32), ("cmp_qy", c_f32),
        ("cmp_qz", c_f32), ("cmp_c22", c_f32), ("cmp_c33", c_f32), ("cmp_c44", c_f32), ("rej_qpt", c_f32),
        ("rej_looper_qpt", c_f32), ("rej_sinphi", c_f32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Phase2View(ctypes.Structure):
    _fields_ = [("n_seg", c_i32), ("n_final", c_i32), ("n_vertices", c_i32), ("pad_", c_i32),
                ("n_final_hits", c_i64), ("finals", c_vp), ("final_hits", c_vp), ("vertices", c_vp),
                ("flags", c_vp), ("rec", c_vp), ("res", c_vp), ("seg_n_hits", c_vp), ("seg_hit_begin", c_vp)]


FINAL_DTYPE = np.dtype([("slot", "i4"), ("sector", "i4"), ("status", "i4"), ("n_seg", "i4"), ("n_hits", "i4"),
                        ("ndf", "i4"), ("row_ref", "i4"), ("vertex", "i4"), ("z0_ok", "i4"), ("first_seg", "i4"),
                        ("hit_begin", "i8"), ("x_ref", "f4"), ("chi2", "f4"), ("p", "f4", 5), ("cov", "f4", 15),
                        ("z0", "f4"), ("t0", "f4"), ("z_conv", "f4"), ("pad_", "i4")])
VERTEX_DTYPE = np.dtype([("slot", "i4"), ("n_tracks", "i4"), ("first", "i4"), ("t0", "f4")])
assert FINAL_DTYPE.itemsize == 152 and VERTEX_DTYPE.itemsize == 16
FLAG_LOWPT, FLAG_LEG, FLAG_INCL = 1, 2, 4

TRACK_DTYPE = np.dtype([("x_ref", "f4"), ("p", "f4", 5), ("cov", "f4", 15), ("chi2", "f4"), ("ndf", "i4"),
                        ("n_hits", "i4"), ("hit_offset", "i4"), ("sector", "i4"), ("start_id", "i4")])
TRACKLET_DTYPE = np.dtype([("start_id", "i4"), ("n_chain", "i4"), ("status", "i4"), ("n_hits", "i4"),
                           ("n_pass1", "i4"), ("ndf", "i4"), ("row_ref", "i4"), ("row_out", "i4"),
                           ("x_ref", "f4"), ("chi2", "f4"), ("x_out", "f4"), ("p", "f4", 5), ("cov", "f4", 15),
                           ("p_out", "f4", 5), ("cov_out", "f4", 15)])
UNIT_RESULT_DTYPE = np.dtype([("slot", "i4"), ("sector", "i4"), ("n_clusters", "i4"), ("n_tracklets", "i4"),
                              ("n_tracks", "i4"), ("n_track_hits", "i4"), ("cluster_begin", "i8"),
                              ("track_begin", "i8"), ("hit_begin", "i8")])
assert TRACK_DTYPE.itemsize == 108 and TRACKLET_DTYPE.itemsize == 204 and UNIT_RESULT_DTYPE.itemsize == 48

# exported symbols (kept in step with include/tpcca.h)
SYMBOLS = (
    "tpcca_params_default", "tpcca_create", "tpcca_destroy", "tpcca_reset", "tpcca_load_sector",
    "tpcca_find_links", "tpcca_clean_links", "tpcca_build_tracklets", "tpcca_select_tracks", "tpcca_sync",
    "tpcca_get_links", "tpcca_get_tracklets", "tpcca_get_tracks", "tpcca_get_assignment", "tpcca_run_batch",
    "tpcca_get_batch_results", "tpcca_batch_totals", "tpcca_device_results", "tpcca_error_string",
    "tpcca_last_error", "tpcca_stage_times", "tpcca_set_timing", "tpcca_server_create",
    "tpcca_server_submit", "tpcca_server_poll", "tpcca_server_wait", "tpcca_server_release",
    "tpcca_server_stats", "tpcca_server_reset_stats", "tpcca_server_destroy", "tpcca_now",
    "tpcca_server_last_error",
    "tpcca_work_stats", "tpcca_set_tuning", "tpcca_get_tuning", "tpcca_server_set_tuning",
    "tpcca_tuning_default", "tpcca_run_batch_noalloc",
    "tpcca_phase2_params_default", "tpcca_set_phase2_params", "tpcca_phase2", "tpcca_get_finals",
    "tpcca_get_segment_links", "tpcca_get_vertices", "tpcca_get_flags", "tpcca_get_compressed",
    "tpcca_phase2_view", "tpcca_decompress",
)

_lib = None


def lib():
    """Load libtpcca.so (built by paper_1709_00618_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "tpcca_params_default": (None, [ctypes.POINTER(Params)]),
        "tpcca_create": (c_i32, [ctypes.POINTER(Geometry), ctypes.POINTER(Params), c_i32, c_vp, ctypes.c_size_t,
                                 ctypes.POINTER(c_vp)]),
        "tpcca_destroy": (c_i32, [c_vp]),
        "tpcca_reset": (c_i32, [c_vp]),
        "tpcca_load_sector": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_vp, c_i32, c_i32]),
        "tpcca_find_links": (c_i32, [c_vp, c_i32, c_i32]),
        "tpcca_clean_links": (c_i32, [c_vp, c_i32, c_i32]),
        "tpcca_build_tracklets": (c_i32, [c_vp, c_i32, c_i32]),
        "tpcca_select_tracks": (c_i32, [c_vp, c_i32, c_i32]),
        "tpcca_sync": (c_i32, [c_vp]),
        "tpcca_get_links": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_i32]),
        "tpcca_get_tracklets": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_i32, ctypes.POINTER(c_i32), c_vp, c_vp, c_i64,
                                        ctypes.POINTER(c_i64)]),
        "tpcca_get_tracks": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_i32, ctypes.POINTER(c_i32), c_vp, c_i64,
                                     ctypes.POINTER(c_i64)]),
        "tpcca_get_assignment": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_i32]),
        "tpcca_run_batch": (c_i32, [c_vp, ctypes.POINTER(Batch)]),
        "tpcca_get_batch_results": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64]),
        "tpcca_batch_totals": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                       ctypes.POINTER(c_i64)]),
        "tpcca_device_results": (c_i32, [c_vp, ctypes.POINTER(DeviceResults)]),
        "tpcca_error_string": (ctypes.c_char_p, [c_i32]),
        "tpcca_last_error": (ctypes.c_char_p, [c_vp]),
        "tpcca_stage_times": (c_i32, [c_vp, c_vp, c_i32]),
        "tpcca_set_timing": (c_i32, [c_vp, c_i32]),
        "tpcca_server_create": (c_i32, [ctypes.POINTER(Geometry), ctypes.POINTER(Params), c_i32, ctypes.c_size_t,
                                        c_i32, c_i32, ctypes.POINTER(c_vp)]),
        "tpcca_server_submit": (c_i32, [c_vp, ctypes.POINTER(Timeframe), ctypes.POINTER(ctypes.c_uint64)]),
        "tpcca_server_poll": (c_i32, [c_vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
        "tpcca_server_wait": (c_i32, [c_vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Result)]),
        "tpcca_server_release": (c_i32, [c_vp, ctypes.c_uint64]),
        "tpcca_server_stats": (c_i32, [c_vp, ctypes.POINTER(Stats)]),
        "tpcca_server_last_error": (ctypes.c_char_p, [c_vp]),
        "tpcca_server_reset_stats": (c_i32, [c_vp]),
        "tpcca_server_destroy": (c_i32, [c_vp]),
        "tpcca_now": (ctypes.c_double, []),
        "tpcca_work_stats": (c_i32, [c_vp, ctypes.POINTER(WorkStats)]),
        "tpcca_set_tuning": (c_i32, [c_vp, ctypes.POINTER(Tuning)]),
        "tpcca_server_set_tuning": (c_i32, [c_vp, ctypes.POINTER(Tuning)]),
        "tpcca_tuning_default": (None, [ctypes.POINTER(Tuning)]),
        "tpcca_get_tuning": (c_i32, [c_vp, ctypes.POINTER(Tuning)]),
        "tpcca_run_batch_noalloc": (c_i32, [ctypes.POINTER(Geometry), ctypes.POINTER(Params), c_i32, c_vp,
                                            ctypes.POINTER(Batch), c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
                                            ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
        "tpcca_phase2_params_default": (None, [ctypes.POINTER(Phase2Params)]),
        "tpcca_set_phase2_params": (c_i32, [c_vp, ctypes.POINTER(Phase2Params)]),
        "tpcca_phase2": (c_i32, [c_vp]),
        "tpcca_get_finals": (c_i32, [c_vp, c_i32, c_vp, c_i32, ctypes.POINTER(c_i32), c_vp, c_i64,
                                     ctypes.POINTER(c_i64)]),
        "tpcca_get_segment_links": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_i32]),
        "tpcca_get_vertices": (c_i32, [c_vp, c_i32, c_vp, c_i32, ctypes.POINTER(c_i32)]),
        "tpcca_get_flags": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_i32]),
        "tpcca_get_compressed": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_i32, c_vp, c_i64, ctypes.POINTER(c_i32),
                                         ctypes.POINTER(c_i64)]),
        "tpcca_phase2_view": (c_i32, [c_vp, ctypes.POINTER(Phase2View)]),
        "tpcca_decompress": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    }
    missing = [n for n in SYMBOLS if not hasattr(L, n)]
    if missing:
        raise ImportError(f"{LIB_PATH} lacks {missing}: rebuild it")
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def error_string(status: int) -> str:
    try:
        return lib().tpcca_error_string(status).decode()
    except Exception:  # the library may be what failed to load
        return "?"


def _p(a):
    if a is None:
        return None
    if isinstance(a, int):
        return c_vp(a)
    if hasattr(a, "data_ptr"):
        return c_vp(a.data_ptr())
    return c_vp(a.ctypes.data)


def params_default(**over) -> Params:
    p = Params()
    lib().tpcca_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def _check(status, where, ctx=None):
    if status != OK:
        detail = ""
        if ctx is not None:
            try:
                detail = lib().tpcca_last_error(ctx).decode()
            except Exception:
                pass
        raise TpccaError(status, where, detail)


class Context:
    """One tpcca_ctx: a device arena and a HIP stream."""

    def __init__(self, row_x, params: Params | None = None, device: int = 0, stream=None,
                 budget_bytes: int = 0, n_sectors: int = 36):
        L = lib()
        self.row_x = np.ascontiguousarray(row_x, np.float32)
        self.params = params or params_default(n_rows=self.row_x.shape[0])
        geo = Geometry(n_sectors, self.row_x.shape[0], _p(self.row_x))
        h = c_vp()
        _check(L.tpcca_create(ctypes.byref(geo), ctypes.byref(self.params), device, stream, budget_bytes,
                              ctypes.byref(h)), "tpcca_create")
        self.h = h
        self.R = self.row_x.shape[0]

    def close(self):
        if getattr(self, "h", None):
            lib().tpcca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # stages
    def reset(self):
        _check(lib().tpcca_reset(self.h), "tpcca_reset", self.h)

    def load_sector(self, slot, sector, cl, row, device=False):
        n = int(cl.shape[0])
        if not device:
            cl = np.ascontiguousarray(cl, np.float32)
            row = np.ascontiguousarray(row, np.uint8)
        st = lib().tpcca_load_sector(self.h, slot, sector, _p(cl) if n else None, _p(row) if n else None, n,
                                     MEM_DEVICE if device else MEM_HOST)
        _check(st, "tpcca_load_sector", self.h)

    def find_links(self, slot=-1, sector=-1):
        _check(lib().tpcca_find_links(self.h, slot, sector), "tpcca_find_links", self.h)

    def clean_links(self, slot=-1, sector=-1):
        _check(lib().tpcca_clean_links(self.h, slot, sector), "tpcca_clean_links", self.h)

    def build_tracklets(self, slot=-1, sector=-1):
        _check(lib().tpcca_build_tracklets(self.h, slot, sector), "tpcca_build_tracklets", self.h)

    def select_tracks(self, slot=-1, sector=-1):
        _check(lib().tpcca_select_tracks(self.h, slot, sector), "tpcca_select_tracks", self.h)

    def run_all(self, slot=-1, sector=-1):
        self.find_links(slot, sector)
        self.clean_links(slot, sector)
        self.build_tracklets(slot, sector)
        self.select_tracks(slot, sector)

    def sync(self):
        _check(lib().tpcca_sync(self.h), "tpcca_sync", self.h)

    # results
    def get_links(self, slot, sector, n, which=0):
        up = np.empty(n, np.int32)
        dn = np.empty(n, np.int32)
        _check(lib().tpcca_get_links(self.h, slot, sector, which, _p(up), _p(dn), n), "tpcca_get_links", self.h)
        return up, dn

    def get_tracklets(self, slot, sector):
        n = c_i32()
        nh = c_i64()
        st = lib().tpcca_get_tracklets(self.h, slot, sector, None, 0, ctypes.byref(n), None, None, 0,
                                       ctypes.byref(nh))
        if st not in (OK, ECAPACITY):
            _check(st, "tpcca_get_tracklets", self.h)
        out = np.zeros(n.value, TRACKLET_DTYPE)
        hb = np.zeros(n.value + 1, np.int64)
        hits = np.zeros(max(1, nh.value), np.int32)
        st = lib().tpcca_get_tracklets(self.h, slot, sector, _p(out), n.value, ctypes.byref(n), _p(hb), _p(hits),
                                       hits.shape[0], ctypes.byref(nh))
        _check(st, "tpcca_get_tracklets", self.h)
        return out, hb, hits[:nh.value]

    def get_tracks(self, slot, sector):
        n = c_i32()
        nh = c_i64()
        st = lib().tpcca_get_tracks(self.h, slot, sector, None, 0, ctypes.byref(n), None, 0, ctypes.byref(nh))
        if st not in (OK, ECAPACITY):
            _check(st, "tpcca_get_tracks", self.h)
        out = np.zeros(n.value, TRACK_DTYPE)
        hits = np.zeros(max(1, nh.value), np.int32)
        st = lib().tpcca_get_tracks(self.h, slot, sector, _p(out), n.value, ctypes.byref(n), _p(hits),
                                    hits.shape[0], ctypes.byref(nh))
        _check(st, "tpcca_get_tracks", self.h)
        return out, hits[:nh.value]

    def get_assignment(self, slot, sector, n):
        a = np.empty(n, np.int32)
        _check(lib().tpcca_get_assignment(self.h, slot, sector, _p(a), n), "tpcca_get_assignment", self.h)
        return a

    # batches
    def run_batch(self, cl, row, units, device=False, graph=False):
        """units: (U, 4) int array of (begin, n, slot, sector)."""
        units = np.asarray(units, np.int64)
        self._bt = (np.ascontiguousarray(units[:, 2], np.int32), np.ascontiguousarray(units[:, 3], np.int32),
                    np.ascontiguousarray(units[:, 0], np.int64), np.ascontiguousarray(units[:, 1], np.int32))
        if not device:
            cl = np.ascontiguousarray(cl, np.float32)
            row = np.ascontiguousarray(row, np.uint8)
        self._bt_in = (cl, row)
        b = Batch(units.shape[0], _p(self._bt[0]), _p(self._bt[1]), _p(self._bt[2]), _p(self._bt[3]),
                  _p(cl), _p(row), (MEM_DEVICE if device else MEM_HOST) | (BATCH_GRAPH if graph else 0))
        _check(lib().tpcca_run_batch(self.h, ctypes.byref(b)), "tpcca_run_batch", self.h)

    def batch_totals(self):
        nu, nc, nt, nh = c_i32(), c_i64(), c_i64(), c_i64()
        _check(lib().tpcca_batch_totals(self.h, ctypes.byref(nu), ctypes.byref(nc), ctypes.byref(nt),
                                        ctypes.byref(nh)), "tpcca_batch_totals", self.h)
        return nu.value, nc.value, nt.value, nh.value

    def get_batch_results(self, out=None):
        """(units, tracks, hits, assignment) of the last batch; `out` may hold
        four preallocated arrays of those dtypes (e.g. views of pinned host
        memory, for copies at link speed) with room for the results."""
        nu, nc, nt, nh = self.batch_totals()
        if out is not None:
            units, tracks, hits, asg = out
            assert units.shape[0] >= nu and tracks.shape[0] >= max(1, nt) and hits.shape[0] >= max(1, nh) \
                and asg.shape[0] >= max(1, nc), "result buffers too small"
        else:
            units = np.zeros(nu, UNIT_RESULT_DTYPE)
            tracks = np.zeros(max(1, nt), TRACK_DTYPE)
            hits = np.zeros(max(1, nh), np.int32)
            asg = np.zeros(max(1, nc), np.int32)
        _check(lib().tpcca_get_batch_results(self.h, _p(units), _p(tracks), tracks.shape[0], _p(hits),
                                             hits.shape[0], _p(asg), asg.shape[0]),
               "tpcca_get_batch_results", self.h)
        return units[:nu], tracks[:nt], hits[:nh], asg[:nc]

    def work_stats(self) -> dict:
        w = WorkStats()
        _check(lib().tpcca_work_stats(self.h, ctypes.byref(w)), "tpcca_work_stats", self.h)
        return {k: getattr(w, k) for k, _ in WorkStats._fields_}

    def device_results(self):
        d = DeviceResults()
        _check(lib().tpcca_device_results(self.h, ctypes.byref(d)), "tpcca_device_results", self.h)
        return d

    def set_tuning(self, **kw):
        t = Tuning()
        lib().tpcca_get_tuning(self.h, ctypes.byref(t))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(lib().tpcca_set_tuning(self.h, ctypes.byref(t)), "tpcca_set_tuning", self.h)

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().tpcca_get_tuning(self.h, ctypes.byref(t)), "tpcca_get_tuning", self.h)
        return t.as_dict()

    def set_timing(self, on=True):
        lib().tpcca_set_timing(self.h, 1 if on else 0)

    # second phase (merging and refit, vertices, compression, rejection flags)
    def set_phase2_params(self, **kw):
        q = phase2_params_default(**kw)
        _check(lib().tpcca_set_phase2_params(self.h, ctypes.byref(q)), "tpcca_set_phase2_params", self.h)

    def phase2(self):
        _check(lib().tpcca_phase2(self.h), "tpcca_phase2", self.h)

    def get_finals(self, slot):
        n, nh = c_i32(), c_i64()
        st = lib().tpcca_get_finals(self.h, slot, None, 0, ctypes.byref(n), None, 0, ctypes.byref(nh))
        if st not in (OK, ECAPACITY):
            _check(st, "tpcca_get_finals", self.h)
        out = np.zeros(max(1, n.value), FINAL_DTYPE)
        hits = np.zeros(max(1, nh.value), np.int32)
        _check(lib().tpcca_get_finals(self.h, slot, _p(out), out.shape[0], ctypes.byref(n), _p(hits), hits.shape[0],
                                      ctypes.byref(nh)), "tpcca_get_finals", self.h)
        return out[:n.value], hits[:nh.value]

    def get_segment_links(self, slot, sector, n):
        nx, pv, fo = (np.zeros(max(1, n), np.int32) for _ in range(3))
        _check(lib().tpcca_get_segment_links(self.h, slot, sector, _p(nx), _p(pv), _p(fo), n),
               "tpcca_get_segment_links", self.h)
        return nx[:n], pv[:n], fo[:n]

    def get_vertices(self, slot):
        n = c_i32()
        st = lib().tpcca_get_vertices(self.h, slot, None, 0, ctypes.byref(n))
        if st not in (OK, ECAPACITY):
            _check(st, "tpcca_get_vertices", self.h)
        out = np.zeros(max(1, n.value), VERTEX_DTYPE)
        _check(lib().tpcca_get_vertices(self.h, slot, _p(out), out.shape[0], ctypes.byref(n)), "tpcca_get_vertices",
               self.h)
        return out[:n.value]

    def get_flags(self, slot, sector, n):
        f = np.zeros(max(1, n), np.uint8)
        _check(lib().tpcca_get_flags(self.h, slot, sector, _p(f), n), "tpcca_get_flags", self.h)
        return f[:n]

    def get_compressed(self, slot, sector):
        ns, nh = c_i32(), c_i64()
        st = lib().tpcca_get_compressed(self.h, slot, sector, None, 0, None, 0, ctypes.byref(ns), ctypes.byref(nh))
        if st not in (OK, ECAPACITY):
            _check(st, "tpcca_get_compressed", self.h)
        rec = np.zeros((max(1, ns.value), 6), np.int32)
        res = np.zeros((max(1, nh.value), 4), np.int32)  # row step, y, z, 0
        _check(lib().tpcca_get_compressed(self.h, slot, sector, _p(rec), rec.shape[0], _p(res), res.shape[0],
                                          ctypes.byref(ns), ctypes.byref(nh)), "tpcca_get_compressed", self.h)
        return rec[:ns.value], np.ascontiguousarray(res[:nh.value, :3])

    def phase2_view(self) -> Phase2View:
        v = Phase2View()
        _check(lib().tpcca_phase2_view(self.h, ctypes.byref(v)), "tpcca_phase2_view", self.h)
        return v

    def decompress(self, n_seg, n_hits, hit_begin, rec, res, yq, zq, rows):
        """Device pointers (ints) or tensors; queued on the context's stream."""
        _check(lib().tpcca_decompress(self.h, n_seg, _p(n_hits), _p(hit_begin), _p(rec), _p(res), _p(yq), _p(zq),
                                      _p(rows)), "tpcca_decompress", self.h)

    STAGES = ("grid", "links", "clean", "chains", "fit", "select")

    def stage_times(self):
        ms = np.zeros(6, np.float32)
        n = lib().tpcca_stage_times(self.h, _p(ms), 6)
        return dict(zip(self.STAGES, ms[:n].tolist()))


def phase2_params_default(**over) -> Phase2Params:
    q = Phase2Params()
    lib().tpcca_phase2_params_default(ctypes.byref(q))
    for k, v in over.items():
        setattr(q, k, v)
    return q


NOALLOC_SCRATCH_BYTES = 64 << 20  # TPCCA_NOALLOC_SCRATCH_BYTES


def run_batch_noalloc(row_x, cl, row, units, tracks, hits, assignment, unit_results, params: Params | None = None,
                      device: int = 0, stream=None, n_sectors: int = 36):
    """tpcca_run_batch_noalloc: the whole tracker on device-resident inputs,
    every work buffer in the library's fixed device array, results written
    to the caller's device tensors (tracks: uint8 of n x 108 B, hits and
    assignment: int32, unit_results: uint8 of U x 48 B).  units: (U, 4)
    int array of (begin, n, slot, sector).  Returns (n_tracks, n_hits)."""
    row_x = np.ascontiguousarray(row_x, np.float32)
    params = params or params_default(n_rows=row_x.shape[0])
    geo = Geometry(n_sectors, row_x.shape[0], _p(row_x))
    units = np.asarray(units, np.int64).reshape(-1, 4)
    slot = np.ascontiguousarray(units[:, 2], np.int32)
    sector = np.ascontiguousarray(units[:, 3], np.int32)
    begin = np.ascontiguousarray(units[:, 0], np.int64)
    n = np.ascontiguousarray(units[:, 1], np.int32)
    b = Batch(units.shape[0], _p(slot), _p(sector), _p(begin), _p(n), _p(cl), _p(row), MEM_DEVICE)
    nt, nh = c_i64(), c_i64()
    st = lib().tpcca_run_batch_noalloc(
        ctypes.byref(geo), ctypes.byref(params), device, stream, ctypes.byref(b), _p(tracks),
        tracks.numel() // TRACK_DTYPE.itemsize, _p(hits), hits.numel(), _p(assignment), assignment.numel(),
        _p(unit_results), ctypes.byref(nt), ctypes.byref(nh))
    detail = ""
    if st == ENOMEM:
        detail = f"the units need more than the {NOALLOC_SCRATCH_BYTES >> 20} MiB allocation-free work array"
    if st != OK:
        raise TpccaError(st, "tpcca_run_batch_noalloc", detail)
    return nt.value, nh.value


def now() -> float:
    return float(lib().tpcca_now())
