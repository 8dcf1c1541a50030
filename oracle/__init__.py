"""Python access to the plain CPU oracle (TEST INFRASTRUCTURE).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``libtpcref.so`` built from
``tpcref.cpp`` with g++ (no contraction, no fast-math) and shares nothing with
the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpcref.cpp")
_HDR = os.path.join(_HERE, "tpcref.h")
_LIB_PATH = os.path.join(_HERE, "libtpcref.so")

CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32), ("link_wy", ctypes.c_float), ("link_wz", ctypes.c_float),
        ("link_chi2", ctypes.c_float), ("min_chain_hits", ctypes.c_int32), ("kB", ctypes.c_float),
        ("err2_y", ctypes.c_float), ("err2_z", ctypes.c_float), ("max_sinphi", ctypes.c_float),
        ("seed_c22", ctypes.c_float), ("seed_c33", ctypes.c_float), ("seed_c44", ctypes.c_float),
        ("reset_c00", ctypes.c_float), ("reset_c11", ctypes.c_float), ("pick_nsig", ctypes.c_float),
        ("pick_win_max", ctypes.c_float), ("pick_chi2", ctypes.c_float), ("max_miss", ctypes.c_int32),
        ("min_track_hits", ctypes.c_int32), ("own_frac_pct", ctypes.c_int32),
        ("refit_inflate", ctypes.c_float),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TRACKLET_DTYPE = np.dtype([
    ("start_id", "i4"), ("n_chain", "i4"), ("status", "i4"), ("n_hits", "i4"), ("n_pass1", "i4"),
    ("ndf", "i4"), ("row_ref", "i4"), ("row_out", "i4"), ("x_ref", "f8"), ("chi2", "f8"), ("x_out", "f8"),
    ("p", "f8", 5), ("cov", "f8", 15), ("p_out", "f8", 5), ("cov_out", "f8", 15)])


class _Stats(ctypes.Structure):
    _fields_ = [("decisions", ctypes.c_int64), ("near_ties", ctypes.c_int64), ("min_margin", ctypes.c_double),
                ("propagations", ctypes.c_int64), ("tests", ctypes.c_int64), ("updates", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.tpcref_params_default.argtypes = [ctypes.POINTER(Params)]
        L.tpcref_run.restype = vp
        L.tpcref_run.argtypes = [ctypes.POINTER(Params), vp, vp, vp, i32, i32, ctypes.POINTER(i32)]
        L.tpcref_free.argtypes = [vp]
        for f in ("tpcref_n_clusters", "tpcref_n_tracklets", "tpcref_n_tracks"):
            getattr(L, f).restype = i32
            getattr(L, f).argtypes = [vp]
        for f in ("tpcref_n_tracklet_hits", "tpcref_n_track_hits"):
            getattr(L, f).restype = i64
            getattr(L, f).argtypes = [vp]
        L.tpcref_get_links.argtypes = [vp, i32, vp, vp]
        L.tpcref_get_tracklets.argtypes = [vp, vp, vp, vp]
        L.tpcref_get_tracks.argtypes = [vp, vp, vp, vp]
        L.tpcref_get_assignment.argtypes = [vp, vp]
        L.tpcref_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.tpcref_refit.restype = i32
        L.tpcref_refit.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, i32, i32, i32, i32, vp, vp]
        L.tpcref_chi2.restype = i32
        L.tpcref_chi2.argtypes = [ctypes.POINTER(Params), i32, vp, vp, ctypes.c_double, ctypes.c_double, vp]
        L.tpcref_search_row.restype = i32
        L.tpcref_search_row.argtypes = [ctypes.POINTER(Params), i32, vp, vp, vp, i32, i32, vp, vp, ctypes.c_double]
        L.tpcref_select.restype = i32
        L.tpcref_select.argtypes = [ctypes.POINTER(Params), i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.tpcref_propagate.restype = i32
        L.tpcref_propagate.argtypes = [ctypes.POINTER(Params), i32, vp, vp, vp, ctypes.c_double]
        L.tpcref_update.restype = i32
        L.tpcref_update.argtypes = [ctypes.POINTER(Params), i32, vp, vp, ctypes.c_double, ctypes.c_double, vp]
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def default_params(**over) -> Params:
    p = Params()
    lib().tpcref_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


@dataclass
class SectorResult:
    up_raw: np.ndarray
    dn_raw: np.ndarray
    up: np.ndarray
    dn: np.ndarray
    tracklets: np.ndarray        # TRACKLET_DTYPE, ascending start_id
    tracklet_hit_begin: np.ndarray
    tracklet_hits: np.ndarray
    track_tracklet: np.ndarray   # accepted: index into tracklets
    track_hit_begin: np.ndarray
    track_hits: np.ndarray       # won hits
    assignment: np.ndarray
    decisions: int
    near_ties: int
    min_margin: float
    work: dict = None            # fit work: propagations, tests, updates

    @property
    def n_tracks(self) -> int:
        return int(self.track_tracklet.shape[0])

    def tracklet_hit_list(self, t):
        return self.tracklet_hits[self.tracklet_hit_begin[t]:self.tracklet_hit_begin[t + 1]]

    def track_hit_list(self, k):
        return self.track_hits[self.track_hit_begin[k]:self.track_hit_begin[k + 1]]


def run_sector(cl: np.ndarray, row: np.ndarray, row_x: np.ndarray, params: Params | None = None,
               precision: int = 32) -> SectorResult:
    L = lib()
    params = params or default_params()
    cl = np.ascontiguousarray(cl, np.float32)
    row = np.ascontiguousarray(row, np.uint8)
    row_x = np.ascontiguousarray(row_x, np.float32)
    n = cl.shape[0]
    err = ctypes.c_int32(0)
    h = L.tpcref_run(ctypes.byref(params), _ptr(row_x), _ptr(cl) if n else None,
                     _ptr(row) if n else None, n, precision, ctypes.byref(err))
    if not h:
        raise ValueError(f"oracle rejected the input (err {err.value})")
    try:
        up_raw = np.empty(n, np.int32); dn_raw = np.empty(n, np.int32)
        up = np.empty(n, np.int32); dn = np.empty(n, np.int32)
        L.tpcref_get_links(h, 0, _ptr(up_raw), _ptr(dn_raw))
        L.tpcref_get_links(h, 1, _ptr(up), _ptr(dn))
        T = L.tpcref_n_tracklets(h)
        tr = np.zeros(T, TRACKLET_DTYPE)
        tb = np.zeros(T + 1, np.int64)
        th = np.zeros(max(1, L.tpcref_n_tracklet_hits(h)), np.int32)
        L.tpcref_get_tracklets(h, _ptr(tr), _ptr(tb), _ptr(th))
        K = L.tpcref_n_tracks(h)
        ki = np.zeros(K, np.int32)
        kb = np.zeros(K + 1, np.int64)
        kh = np.zeros(max(1, L.tpcref_n_track_hits(h)), np.int32)
        L.tpcref_get_tracks(h, _ptr(ki), _ptr(kb), _ptr(kh))
        asg = np.empty(n, np.int32)
        if n:
            L.tpcref_get_assignment(h, _ptr(asg))
        st = _Stats()
        L.tpcref_get_stats(h, ctypes.byref(st))
    finally:
        L.tpcref_free(h)
    return SectorResult(up_raw, dn_raw, up, dn, tr, tb, th[:tb[-1]], ki, kb, kh[:kb[-1]], asg,
                        st.decisions, st.near_ties, st.min_margin,
                        {"propagations": st.propagations, "tests": st.tests, "updates": st.updates})


def refit(cl, row, row_x, hits, k0, n_chain, params=None, precision=64, with_margin=False):
    """Replay one tracklet's fit along its hit list at the given precision.
    with_margin: also return the smallest margin of the replay's sin phi tests."""
    L = lib()
    params = params or default_params()
    hits = np.ascontiguousarray(hits, np.int32)
    out = np.zeros(1, TRACKLET_DTYPE)
    mm = np.zeros(1, np.float64)
    rc = L.tpcref_refit(ctypes.byref(params), _ptr(np.ascontiguousarray(row_x, np.float32)),
                        _ptr(np.ascontiguousarray(cl, np.float32)), _ptr(np.ascontiguousarray(row, np.uint8)),
                        _ptr(hits), hits.shape[0], int(k0), int(n_chain), precision, _ptr(out), _ptr(mm))
    if with_margin:
        return rc, out[0], float(mm[0])
    return rc, out[0]


def chi2(state, cov, ym, zm, params=None, precision=64):
    """The 2-D chi^2 of a measurement against a state (the searches' pickup test)."""
    L = lib()
    params = params or default_params()
    s = np.ascontiguousarray(state, np.float64)
    c = np.ascontiguousarray(cov, np.float64)
    out = np.zeros(1, np.float64)
    rc = L.tpcref_chi2(ctypes.byref(params), precision, _ptr(s), _ptr(c), float(ym), float(zm), _ptr(out))
    return rc, float(out[0])


def search_row(cl, row, row_x, r, state, cov, zr=0.0, params=None, precision=32):
    """The hit the track-following search picks in row r (-1: none)."""
    L = lib()
    params = params or default_params()
    cl = np.ascontiguousarray(cl, np.float32)
    row = np.ascontiguousarray(row, np.uint8)
    s = np.ascontiguousarray(state, np.float64)
    c = np.ascontiguousarray(cov, np.float64)
    h = L.tpcref_search_row(ctypes.byref(params), precision, _ptr(np.ascontiguousarray(row_x, np.float32)),
                            _ptr(cl), _ptr(row), cl.shape[0], int(r), _ptr(s), _ptr(c), float(zr))
    if h == -2:
        raise ValueError("oracle rejected the input")
    return h


def select(n_clusters, n_hits, chi2_, start_id, status, hit_lists, params=None):
    """The selection alone: (accepted index per candidate or -1, assignment)."""
    L = lib()
    params = params or default_params()
    T = len(hit_lists)
    nh = np.ascontiguousarray(n_hits, np.int32)
    c2 = np.ascontiguousarray(chi2_, np.float32)
    sid = np.ascontiguousarray(start_id, np.int32)
    st = np.ascontiguousarray(status, np.int32)
    hb = np.zeros(T + 1, np.int64)
    hb[1:] = np.cumsum([len(h) for h in hit_lists])
    hits = np.ascontiguousarray(np.concatenate([np.asarray(h, np.int32) for h in hit_lists]) if T else
                                np.zeros(1, np.int32), np.int32)
    acc = np.zeros(max(T, 1), np.int32)
    asg = np.zeros(max(n_clusters, 1), np.int32)
    k = L.tpcref_select(ctypes.byref(params), int(n_clusters), T, _ptr(nh), _ptr(c2), _ptr(sid), _ptr(st),
                        _ptr(hb), _ptr(hits), _ptr(acc), _ptr(asg))
    if k < 0:
        raise ValueError("oracle rejected the candidates")
    return acc[:T], asg[:n_clusters]


def propagate(state, cov, x0, x1, params=None, precision=64):
    L = lib()
    params = params or default_params()
    s = np.array(state, np.float64).copy()
    c = np.array(cov, np.float64).copy()
    x = np.array([x0], np.float64)
    rc = L.tpcref_propagate(ctypes.byref(params), precision, _ptr(s), _ptr(c), _ptr(x), float(x1))
    return rc, s, c, float(x[0])


def update(state, cov, ym, zm, params=None, precision=64):
    L = lib()
    params = params or default_params()
    s = np.array(state, np.float64).copy()
    c = np.array(cov, np.float64).copy()
    chi2 = np.zeros(1, np.float64)
    rc = L.tpcref_update(ctypes.byref(params), precision, _ptr(s), _ptr(c), float(ym), float(zm), _ptr(chi2))
    return rc, s, c, float(chi2[0])


def cov_matrix(c15) -> np.ndarray:
    """Symmetric 5x5 from the 15-element lower triangle."""
    m = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            m[i, j] = m[j, i] = c15[k]
            k += 1
    return m


def cov_lower(m) -> np.ndarray:
    return np.array([m[i, j] for i in range(5) for j in range(i + 1)])
