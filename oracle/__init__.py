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
_SRCS = [_SRC, os.path.join(_HERE, "tpcphase2.cpp")]
_HDRS = [os.path.join(_HERE, h) for h in ("tpcref.h", "tpckf.h", "tpcphase2.h")]
_LIB_PATH = os.path.join(_HERE, "libtpcref.so")

CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(f) for f in _SRCS + _HDRS)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, "-o", tmp, *_SRCS])
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


# ------------------------------------------------------------ second phase ---
# Merging of sector segments and refit (Sec. 2), vertex times (Sec. 5),
# track-model compression and cluster rejection (Sec. 3): tpcphase2.cpp.

class P2Params(ctypes.Structure):
    _fields_ = [
        ("sector_cos", ctypes.c_float), ("sector_sin", ctypes.c_float), ("max_sinphi", ctypes.c_float),
        ("merge_dz_ends", ctypes.c_float),
        ("merge_max_gap", ctypes.c_int32), ("merge_wy", ctypes.c_float), ("merge_wz", ctypes.c_float),
        ("merge_chi2", ctypes.c_float), ("refit_inflate", ctypes.c_float), ("dca_steps", ctypes.c_int32),
        ("vdrift", ctypes.c_float), ("vtx_gap_us", ctypes.c_float), ("vtx_min_tracks", ctypes.c_int32),
        ("vtx_min_hits", ctypes.c_int32), ("vtx_attach_us", ctypes.c_float), ("cmp_qy", ctypes.c_float), ("cmp_qz", ctypes.c_float),
        ("cmp_c22", ctypes.c_float), ("cmp_c33", ctypes.c_float), ("cmp_c44", ctypes.c_float),
        ("rej_qpt", ctypes.c_float), ("rej_looper_qpt", ctypes.c_float), ("rej_sinphi", ctypes.c_float),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SEGMENT_DTYPE = np.dtype([("sector", "i4"), ("start_id", "i4"), ("n_hits", "i4"), ("pad_", "i4"),
                          ("x_ref", "f8"), ("p", "f8", 5), ("cov", "f8", 15)])
FINAL_DTYPE = np.dtype([
    ("status", "i4"), ("n_seg", "i4"), ("seg_begin", "i4"), ("sector", "i4"), ("n_hits", "i4"), ("ndf", "i4"),
    ("row_ref", "i4"), ("vertex", "i4"), ("x_ref", "f8"), ("chi2", "f8"), ("p", "f8", 5), ("cov", "f8", 15),
    ("z0", "f8"), ("t0", "f8"), ("z0_ok", "i4"), ("pad_", "i4"), ("z_conv", "f8")])
VERTEX_DTYPE = np.dtype([("t0", "f8"), ("n_tracks", "i4"), ("first", "i4")])
FLAG_LOWPT, FLAG_LEG, FLAG_INCL = 1, 2, 4

_p2_bound = False


def _lib2():
    global _p2_bound
    L = lib()
    if not _p2_bound:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P, Q = ctypes.POINTER(Params), ctypes.POINTER(P2Params)
        L.tpcref_p2params_default.argtypes = [Q]
        L.tpcref_phase2.restype = vp
        L.tpcref_phase2.argtypes = [P, Q, vp, i32, vp, vp, vp, i32, vp, vp, vp, i32, i32]
        L.tpcref_phase2_free.argtypes = [vp]
        L.tpcref_p2_n_final.restype = i32
        L.tpcref_p2_n_final.argtypes = [vp]
        L.tpcref_p2_n_vertices.restype = i32
        L.tpcref_p2_n_vertices.argtypes = [vp]
        L.tpcref_p2_n_final_hits.restype = i64
        L.tpcref_p2_n_final_hits.argtypes = [vp]
        L.tpcref_p2_links.argtypes = [vp, vp, vp, vp]
        L.tpcref_p2_finals.argtypes = [vp, vp, vp, vp, vp]
        L.tpcref_p2_vertices.argtypes = [vp, vp]
        L.tpcref_p2_flags.argtypes = [vp, vp]
        L.tpcref_p2_outer.argtypes = [vp, vp, vp, vp, vp]
        L.tpcref_p2_stats.argtypes = [vp, vp, vp, vp]
        L.tpcref_compress.restype = i32
        L.tpcref_compress.argtypes = [P, Q, vp, vp, vp, i32, vp, vp, vp, i32, vp, vp]
        L.tpcref_decompress.restype = i32
        L.tpcref_decompress.argtypes = [P, Q, vp, i32, vp, vp, vp, i32, vp, vp, vp]
        L.tpcref_rotate.restype = i32
        L.tpcref_rotate.argtypes = [P, i32, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.tpcref_chi2_5.restype = i32
        L.tpcref_chi2_5.argtypes = [i32, vp, vp, vp, vp]
        L.tpcref_z0.restype = i32
        L.tpcref_z0.argtypes = [P, Q, i32, vp, ctypes.c_double, ctypes.c_double, vp]
        L.tpcref_vertex_groups.restype = i32
        L.tpcref_vertex_groups.argtypes = [i32, vp, vp, ctypes.c_double, i32, vp, vp]
        _p2_bound = True
    return L


def default_p2params(**over) -> P2Params:
    q = P2Params()
    _lib2().tpcref_p2params_default(ctypes.byref(q))
    for k, v in over.items():
        setattr(q, k, v)
    return q


def segments_of(results) -> tuple:
    """Segments of one slot from per-sector oracle results (list indexed by
    sector; None for a sector without input): sector-major, ascending
    start_id within a sector.  Returns (segments, hit_begin, hits)."""
    segs, hl = [], []
    for s, res in enumerate(results):
        if res is None:
            continue
        for k in range(res.n_tracks):
            t = res.tracklets[res.track_tracklet[k]]
            h = res.track_hit_list(k)
            g = np.zeros((), SEGMENT_DTYPE)
            g["sector"], g["start_id"], g["n_hits"] = s, t["start_id"], h.shape[0]
            g["x_ref"], g["p"], g["cov"] = t["x_ref"], t["p"], t["cov"]
            segs.append(g)
            hl.append(np.asarray(h, np.int32))
    seg = np.array(segs, SEGMENT_DTYPE) if segs else np.zeros(0, SEGMENT_DTYPE)
    hb = np.zeros(len(hl) + 1, np.int64)
    hb[1:] = np.cumsum([h.shape[0] for h in hl])
    hits = np.concatenate(hl).astype(np.int32) if hl else np.zeros(0, np.int32)
    return seg, hb, hits


@dataclass
class Phase2Result:
    next: np.ndarray
    prev: np.ndarray
    final_of_seg: np.ndarray
    finals: np.ndarray          # FINAL_DTYPE, in the order of their innermost segment
    seg_order: np.ndarray
    hit_begin: np.ndarray
    hits: np.ndarray            # sector << 24 | cluster ID
    vertices: np.ndarray
    flags: np.ndarray           # per cluster of the slot
    out_x: np.ndarray
    out_p: np.ndarray
    out_cov: np.ndarray
    out_ok: np.ndarray
    pair_tests: int
    near_ties: int
    min_margin: float


def phase2(sector_cl, sector_row, row_x, seg, seg_hit_begin, seg_hits, params=None, p2=None,
           precision=32, brute=False) -> Phase2Result:
    """Second phase of one slot.  sector_cl / sector_row: lists (one entry
    per sector, 36 or fewer) of that sector's clusters and rows."""
    L = _lib2()
    params = params or default_params()
    p2 = p2 or default_p2params()
    ns = len(sector_cl)
    sb = np.zeros(ns + 1, np.int64)
    sb[1:] = np.cumsum([c.shape[0] for c in sector_cl])
    cl = np.ascontiguousarray(np.concatenate(sector_cl) if sb[-1] else np.zeros((1, 4)), np.float32)
    row = np.ascontiguousarray(np.concatenate(sector_row) if sb[-1] else np.zeros(1), np.uint8)
    seg = np.ascontiguousarray(seg, SEGMENT_DTYPE)
    hb = np.ascontiguousarray(seg_hit_begin, np.int64)
    hits = np.ascontiguousarray(seg_hits if len(seg_hits) else np.zeros(1), np.int32)
    n = seg.shape[0]
    h = L.tpcref_phase2(ctypes.byref(params), ctypes.byref(p2), _ptr(np.ascontiguousarray(row_x, np.float32)), ns,
                        _ptr(sb), _ptr(cl), _ptr(row), n, _ptr(seg) if n else None, _ptr(hb), _ptr(hits),
                        precision, 1 if brute else 0)
    if not h:
        raise ValueError("oracle rejected the second-phase input")
    try:
        nf = L.tpcref_p2_n_final(h)
        nv = L.tpcref_p2_n_vertices(h)
        nh = L.tpcref_p2_n_final_hits(h)
        nxt = np.zeros(max(n, 1), np.int32); prv = np.zeros(max(n, 1), np.int32); fos = np.zeros(max(n, 1), np.int32)
        L.tpcref_p2_links(h, _ptr(nxt), _ptr(prv), _ptr(fos))
        fin = np.zeros(max(nf, 1), FINAL_DTYPE)
        so = np.zeros(max(n, 1), np.int32)
        fb = np.zeros(nf + 1, np.int64)
        fh = np.zeros(max(nh, 1), np.int32)
        L.tpcref_p2_finals(h, _ptr(fin), _ptr(so), _ptr(fb), _ptr(fh))
        vt = np.zeros(max(nv, 1), VERTEX_DTYPE)
        if nv:
            L.tpcref_p2_vertices(h, _ptr(vt))
        fl = np.zeros(max(int(sb[-1]), 1), np.uint8)
        L.tpcref_p2_flags(h, _ptr(fl))
        ox = np.zeros(max(n, 1)); op = np.zeros((max(n, 1), 5)); oc = np.zeros((max(n, 1), 15))
        ok = np.zeros(max(n, 1), np.int32)
        L.tpcref_p2_outer(h, _ptr(ox), _ptr(op), _ptr(oc), _ptr(ok))
        pt = ctypes.c_int64(0); nt = ctypes.c_int64(0); mm = ctypes.c_double(0)
        L.tpcref_p2_stats(h, ctypes.byref(pt), ctypes.byref(nt), ctypes.byref(mm))
    finally:
        L.tpcref_phase2_free(h)
    return Phase2Result(nxt[:n], prv[:n], fos[:n], fin[:nf], so[:n], fb, fh[:nh], vt[:nv], fl[:int(sb[-1])],
                        ox[:n], op[:n], oc[:n], ok[:n], pt.value, nt.value, mm.value)


def compress(cl, row, row_x, seg, seg_hit_begin, seg_hits, params=None, p2=None):
    """Track-model compression of one sector's segments: (rec (n, 6) int32,
    res (hits, 3) int32)."""
    L = _lib2()
    params = params or default_params()
    p2 = p2 or default_p2params()
    seg = np.ascontiguousarray(seg, SEGMENT_DTYPE)
    n = seg.shape[0]
    nh = int(seg_hit_begin[-1])
    rec = np.zeros((max(n, 1), 6), np.int32)
    res = np.zeros((max(nh, 1), 3), np.int32)
    rc = L.tpcref_compress(ctypes.byref(params), ctypes.byref(p2), _ptr(np.ascontiguousarray(row_x, np.float32)),
                           _ptr(np.ascontiguousarray(cl, np.float32)), _ptr(np.ascontiguousarray(row, np.uint8)), n,
                           _ptr(seg) if n else None, _ptr(np.ascontiguousarray(seg_hit_begin, np.int64)),
                           _ptr(np.ascontiguousarray(seg_hits if nh else np.zeros(1), np.int32)), 32,
                           _ptr(rec), _ptr(res))
    if rc != 0:
        raise ValueError("oracle rejected the compression input")
    return rec[:n], res[:nh]


def decompress(row_x, n_hits, rec, res, params=None, p2=None):
    """(yq, zq, rows) of every hit from the records and residuals."""
    L = _lib2()
    params = params or default_params()
    p2 = p2 or default_p2params()
    n_hits = np.ascontiguousarray(n_hits, np.int32)
    nh = int(n_hits.sum())
    yq = np.zeros(max(nh, 1), np.int32); zq = np.zeros(max(nh, 1), np.int32); rows = np.zeros(max(nh, 1), np.uint8)
    rc = L.tpcref_decompress(ctypes.byref(params), ctypes.byref(p2), _ptr(np.ascontiguousarray(row_x, np.float32)),
                             n_hits.shape[0], _ptr(n_hits), _ptr(np.ascontiguousarray(rec, np.int32)),
                             _ptr(np.ascontiguousarray(res, np.int32)), 32, _ptr(yq), _ptr(zq), _ptr(rows))
    if rc != 0:
        raise ValueError("oracle rejected the decompression input")
    return yq[:nh], zq[:nh], rows[:nh]


def rotate(state, cov, x, cs, sn, params=None, precision=64):
    L = _lib2()
    params = params or default_params()
    s = np.array(state, np.float64).copy()
    c = np.array(cov, np.float64).copy()
    xx = np.array([x], np.float64)
    rc = L.tpcref_rotate(ctypes.byref(params), precision, float(cs), float(sn), _ptr(s), _ptr(c), _ptr(xx))
    return rc, s, c, float(xx[0])


def chi2_5(d, c1, c2, precision=64):
    L = _lib2()
    out = np.zeros(1)
    rc = L.tpcref_chi2_5(precision, _ptr(np.ascontiguousarray(d, np.float64)),
                         _ptr(np.ascontiguousarray(c1, np.float64)), _ptr(np.ascontiguousarray(c2, np.float64)),
                         _ptr(out))
    return rc, float(out[0])


def z0(state, x, zr=0.0, params=None, p2=None, precision=64):
    """z at the plane x = 0 of a state at plane x (z relative to zr)."""
    L = _lib2()
    params = params or default_params()
    p2 = p2 or default_p2params()
    out = np.zeros(1)
    rc = L.tpcref_z0(ctypes.byref(params), ctypes.byref(p2), precision,
                     _ptr(np.ascontiguousarray(state, np.float64)), float(x), float(zr), _ptr(out))
    return rc, float(out[0])


def vertex_groups(t0, key, gap, min_n):
    """FP32 grouping of t0 estimates: (group index per entry or -1, vertices)."""
    L = _lib2()
    n = len(t0)
    t = np.ascontiguousarray(t0, np.float64)
    k = np.ascontiguousarray(key, np.int64)
    g = np.zeros(max(n, 1), np.int32)
    v = np.zeros(max(n, 1), VERTEX_DTYPE)
    nv = L.tpcref_vertex_groups(n, _ptr(t), _ptr(k), float(gap), int(min_n), _ptr(g), _ptr(v))
    if nv < 0:
        raise ValueError("oracle rejected the input")
    return g[:n], v[:nv]
