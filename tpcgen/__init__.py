"""Seeded synthetic TPC inputs for the sector tracker (inputs only).

The C core (``tpcgen.c``) intersects FP64 helices with the pad-row planes of
36 sectors and emits FP32 clusters.  This wrapper builds the workloads the
tracker is measured on:

* ``one_sector``   - 200 primaries, phi inside sector 0, no noise, 1 sector;
* ``central_event``- 8000 primaries (5 % low-pT loopers), 1 % noise, 36 sectors;
* ``minbias_batch``- 64 events, multiplicity from an impact parameter drawn
  uniformly in area (overlap-area proxy for N_part), 36 sectors each;
* ``timeframe``    - minimum-bias events with Poisson arrival times at 50 kHz,
  z shifted by the drift velocity, clusters of all events mixed per sector;
* ``served_stream``- time-frame sizes log-uniform in [8, 256] events with
  Poisson arrivals equivalent to a 50 kHz interaction rate.

Everything returned is plain numpy.  Nothing here computes any part of the
tracking method.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpcgen.c")
_LIB_PATH = os.path.join(_HERE, "libtpcgen.so")

N_ROWS = 159
N_SECTORS = 36
VDRIFT_CM_PER_US = 2.58


def build(force: bool = False) -> str:
    """Compile the generator core with gcc (fast, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint64), ("event", ctypes.c_uint64),
        ("n_tracks", ctypes.c_int32), ("only_sector", ctypes.c_int32),
        ("looper_frac", ctypes.c_double), ("noise_frac", ctypes.c_double),
        ("sigma_y", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("pt_min", ctypes.c_double), ("pt_max", ctypes.c_double), ("pt_index", ctypes.c_double),
        ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double), ("phi_min", ctypes.c_double), ("phi_max", ctypes.c_double),
        ("looper_pt_min", ctypes.c_double), ("looper_pt_max", ctypes.c_double),
        ("looper_turns", ctypes.c_double), ("normal_turns", ctypes.c_double),
        ("bz", ctypes.c_double), ("zmax", ctypes.c_double), ("t0_us", ctypes.c_double),
        ("vdrift", ctypes.c_double), ("q_min", ctypes.c_double), ("q_max", ctypes.c_double),
    ]


TRUTH_DTYPE = np.dtype([("y", "f8"), ("z", "f8"), ("sinphi", "f8"), ("tanl", "f8"), ("qpt", "f8"),
                        ("track", "i4"), ("leg", "i4"), ("branch", "i4"), ("pad", "i4")])
TRACK_DTYPE = np.dtype([("pt", "f8"), ("eta", "f8"), ("phi0", "f8"), ("tanl", "f8"), ("kappa", "f8"),
                        ("charge", "i4"), ("looper", "i4"), ("side", "i4"), ("pad", "i4")])
assert TRUTH_DTYPE.itemsize == 56 and TRACK_DTYPE.itemsize == 56

_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.tpcgen_make_event.restype = ctypes.c_void_p
        _lib.tpcgen_make_event.argtypes = [ctypes.POINTER(_Cfg)]
        _lib.tpcgen_count.restype = ctypes.c_int64
        _lib.tpcgen_count.argtypes = [ctypes.c_void_p]
        _lib.tpcgen_count_signal.restype = ctypes.c_int64
        _lib.tpcgen_count_signal.argtypes = [ctypes.c_void_p]
        _lib.tpcgen_n_tracks.restype = ctypes.c_int32
        _lib.tpcgen_n_tracks.argtypes = [ctypes.c_void_p]
        _lib.tpcgen_copy.restype = ctypes.c_int
        _lib.tpcgen_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        _lib.tpcgen_free.argtypes = [ctypes.c_void_p]
        _lib.tpcgen_cfg_default.argtypes = [ctypes.POINTER(_Cfg)]
        _lib.tpcgen_row_x.argtypes = [ctypes.c_int, ctypes.c_void_p]
        _lib.tpcgen_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.c_int64, ctypes.c_void_p]
        _lib.tpcgen_uniform.restype = ctypes.c_double
        _lib.tpcgen_uniform.argtypes = [ctypes.c_uint64] * 5
        _lib.tpcgen_hash.restype = ctypes.c_uint64
        _lib.tpcgen_hash.argtypes = [ctypes.c_uint64] * 5
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def row_x() -> np.ndarray:
    """FP32 pad-row radii: x_i = 85 + i*162/158 cm, evaluated in FP64, rounded once."""
    out = np.empty(N_ROWS, np.float32)
    _L().tpcgen_row_x(N_ROWS, _p(out))
    return out


def uniform(seed, stream, a, b, draw) -> float:
    return float(_L().tpcgen_uniform(seed, stream, a, b, draw))


def permutation(seed: int, stream: int, key: int, n: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    if n:
        _L().tpcgen_permutation(seed, stream, key, n, _p(out))
    return out


# --------------------------------------------------------------- events ---
@dataclass
class Event:
    """One event's clusters grouped by sector (sector_begin has 37 entries)."""
    cl: np.ndarray          # (N, 4) float32: x, y, z, q in the sector frame
    row: np.ndarray         # (N,) uint8 pad row
    sector: np.ndarray      # (N,) uint8
    sector_begin: np.ndarray  # (37,) int64
    truth: np.ndarray | None  # (N,) TRUTH_DTYPE
    tracks: np.ndarray        # (T,) TRACK_DTYPE
    n_signal: int
    t0_us: float = 0.0


def make_event(seed=0, stream=0, event=0, n_tracks=200, only_sector=-1, looper_frac=0.0,
               noise_frac=0.0, sigma=0.1, phi_range=None, t0_us=0.0, bz=0.5, pt_min=0.1,
               pt_max=20.0, eta_max=0.9, eta_min=None, want_truth=True, normal_turns=0.5) -> Event:
    L = _L()
    c = _Cfg()
    L.tpcgen_cfg_default(ctypes.byref(c))
    c.seed, c.stream, c.event = seed, stream, event
    c.n_tracks = int(n_tracks)
    c.only_sector = int(only_sector)
    c.looper_frac = looper_frac
    c.noise_frac = noise_frac
    c.sigma_y = c.sigma_z = sigma
    c.t0_us = t0_us
    c.bz = bz
    c.pt_min, c.pt_max, c.eta_max = pt_min, pt_max, eta_max
    c.eta_min = -eta_max if eta_min is None else eta_min
    c.normal_turns = normal_turns
    if phi_range is not None:
        c.phi_min, c.phi_max = phi_range
    h = L.tpcgen_make_event(ctypes.byref(c))
    if not h:
        raise MemoryError("tpcgen_make_event failed")
    try:
        n = L.tpcgen_count(h)
        ns = L.tpcgen_count_signal(h)
        nt = L.tpcgen_n_tracks(h)
        cl = np.empty((n, 4), np.float32)
        row = np.empty(n, np.uint8)
        sec = np.empty(n, np.uint8)
        truth = np.empty(n, TRUTH_DTYPE) if want_truth else None
        sb = np.empty(N_SECTORS + 1, np.int64)
        tracks = np.empty(nt, TRACK_DTYPE)
        L.tpcgen_copy(h, _p(cl), _p(row), _p(sec), _p(truth) if truth is not None else None, _p(sb), _p(tracks))
    finally:
        L.tpcgen_free(h)
    return Event(cl, row, sec, sb, truth, tracks, int(ns), t0_us)


# ---------------------------------------------------------------- batch ---
UNIT_FIELDS = ("begin", "n", "slot", "sector")


@dataclass
class Batch:
    """Clusters of many (slot, sector) units, concatenated.

    units[u] = (begin, n, slot, sector): unit u's clusters are cl[begin:begin+n].
    Cluster IDs are local to a unit (0..n-1), i.e. positions inside its slice.
    """
    cl: np.ndarray
    row: np.ndarray
    units: np.ndarray  # (U, 4) int64
    truth: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self) -> int:
        return int(self.cl.shape[0])

    def unit(self, u: int):
        b, n, slot, sec = (int(v) for v in self.units[u])
        t = self.truth[b:b + n] if self.truth is not None else None
        return self.cl[b:b + n], self.row[b:b + n], slot, sec, t


def _concat_units(parts, keep_truth):
    """parts: list of (slot, sector, cl, row, truth)."""
    n = sum(p[2].shape[0] for p in parts)
    cl = np.empty((n, 4), np.float32)
    row = np.empty(n, np.uint8)
    truth = np.empty(n, TRUTH_DTYPE) if keep_truth else None
    units = np.empty((len(parts), 4), np.int64)
    off = 0
    for u, (slot, sec, c, r, t) in enumerate(parts):
        k = c.shape[0]
        cl[off:off + k] = c
        row[off:off + k] = r
        if keep_truth:
            truth[off:off + k] = t
        units[u] = (off, k, slot, sec)
        off += k
    return cl, row, units, truth


def event_units(ev: Event, slot: int, shuffle_key=None, seed=0, stream=0, sectors=None):
    """Split an event into per-sector units; optionally shuffle each unit's order."""
    parts = []
    secs = range(N_SECTORS) if sectors is None else sectors
    for s in secs:
        b, e = int(ev.sector_begin[s]), int(ev.sector_begin[s + 1])
        c, r = ev.cl[b:e], ev.row[b:e]
        t = ev.truth[b:e] if ev.truth is not None else None
        if shuffle_key is not None and e > b:
            perm = permutation(seed, stream, (shuffle_key << 8) | s, e - b)
            c, r = c[perm], r[perm]
            t = t[perm] if t is not None else None
        parts.append((slot, s, c, r, t))
    return parts


STREAM_ONE_SECTOR = 1
STREAM_CENTRAL = 2
STREAM_MINBIAS = 3
STREAM_TIMEFRAME = 4
STREAM_SERVED = 5


def one_sector(seed=0, n_tracks=200, sigma=0.1, shuffle=True, bz=0.5, eta_max=0.9, eta_min=0.0,
               pt_min=0.1, pt_max=20.0) -> Batch:
    """200 primaries with phi inside sector 0 (its 20 deg at the vertex), no noise.
    Sector 0 is on the A side, so eta is drawn in [0, 0.9): every helix heads
    into the one sector that is tracked."""
    ev = make_event(seed=seed, stream=STREAM_ONE_SECTOR, event=0, n_tracks=n_tracks, only_sector=0,
                    sigma=sigma, phi_range=(0.0, 20.0 * math.pi / 180.0), bz=bz, eta_max=eta_max,
                    eta_min=eta_min, pt_min=pt_min, pt_max=pt_max)
    parts = event_units(ev, 0, shuffle_key=0 if shuffle else None, seed=seed,
                        stream=STREAM_ONE_SECTOR, sectors=[0])
    cl, row, units, truth = _concat_units(parts, True)
    return Batch(cl, row, units, truth, {"workload": "one_sector", "tracks": ev.tracks, "seed": seed})


def central_event(seed=0, n_tracks=8000, slot=0, shuffle=True, keep_truth=True, event=0) -> Batch:
    """8000 primaries (5 % loopers with pT in [0.07, 0.185] GeV, 2 turns), 1 % noise."""
    ev = make_event(seed=seed, stream=STREAM_CENTRAL, event=event, n_tracks=n_tracks, looper_frac=0.05,
                    noise_frac=0.01, want_truth=keep_truth)
    parts = event_units(ev, slot, shuffle_key=event if shuffle else None, seed=seed, stream=STREAM_CENTRAL)
    cl, row, units, truth = _concat_units(parts, keep_truth)
    return Batch(cl, row, units, truth, {"workload": "central_event", "tracks": ev.tracks, "seed": seed})


def minbias_multiplicity(seed: int, stream: int, event: int, n_central=8000) -> int:
    """N_tracks from an impact parameter uniform in area: u = b / 2R_A has pdf 2u;
    the overlap area of two discs, normalised to 1 at u = 0, scales 8000."""
    u = math.sqrt(uniform(seed, stream, event, 0xB0B0, 0))
    frac = (2.0 / math.pi) * (math.acos(u) - u * math.sqrt(max(0.0, 1.0 - u * u)))
    return max(10, int(round(n_central * frac)))


def _minbias_event(seed, stream, event, t0_us=0.0, keep_truth=False):
    n = minbias_multiplicity(seed, stream, event)
    return make_event(seed=seed, stream=stream, event=event, n_tracks=n, looper_frac=0.05,
                      noise_frac=0.01, t0_us=t0_us, want_truth=keep_truth)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _pmap(fn, items):
    """Generate events in threads: the C core releases the GIL."""
    with ThreadPoolExecutor(_workers()) as ex:
        return list(ex.map(fn, items))


def minbias_batch(seed=0, n_events=64, keep_truth=False, shuffle=True) -> Batch:
    """64 minimum-bias events x 36 sectors, one unit per (event, sector)."""
    parts = []
    mult = []
    evs = _pmap(lambda e: _minbias_event(seed, STREAM_MINBIAS, e, keep_truth=keep_truth), range(n_events))
    for e, ev in enumerate(evs):
        mult.append(ev.tracks.shape[0])
        parts += event_units(ev, e, shuffle_key=e if shuffle else None, seed=seed, stream=STREAM_MINBIAS)
    cl, row, units, truth = _concat_units(parts, keep_truth)
    return Batch(cl, row, units, truth, {"workload": "minbias_batch", "multiplicity": np.array(mult), "seed": seed})


def arrival_times_us(seed: int, stream: int, key: int, n: int, rate_khz: float = 50.0) -> np.ndarray:
    """Poisson arrivals: exponential gaps of mean 1/rate, starting from 0."""
    gaps = np.array([-math.log(1.0 - uniform(seed, stream, key, 0xA77, i)) for i in range(n)])
    return np.cumsum(gaps) * (1000.0 / rate_khz)


def timeframe(seed=0, n_events=128, tf_index=0, slot=0, keep_truth=False, shuffle=True,
              stream=STREAM_TIMEFRAME, event_pool=None) -> Batch:
    """Continuous-readout time frame: n_events minimum-bias events with Poisson
    arrival times (50 kHz => mean 5 per 100 us); z' = z - sign(z) * v_drift * t0;
    the clusters of all events are mixed per sector (one unit per sector)."""
    t0 = arrival_times_us(seed, stream, tf_index, n_events)
    per_sector = [[] for _ in range(N_SECTORS)]
    per_sector_truth = [[] for _ in range(N_SECTORS)]
    per_sector_row = [[] for _ in range(N_SECTORS)]
    if event_pool is None:
        evs = _pmap(lambda i: _minbias_event(seed, stream, (tf_index << 16) | i, t0_us=float(t0[i]),
                                             keep_truth=keep_truth), range(n_events))
    for i in range(n_events):
        eid = (tf_index << 16) | i
        if event_pool is not None:
            ev = event_pool[eid % len(event_pool)]
            shift = VDRIFT_CM_PER_US * t0[i]
        else:
            ev = evs[i]
            shift = 0.0
        for s in range(N_SECTORS):
            b, e = int(ev.sector_begin[s]), int(ev.sector_begin[s + 1])
            c = ev.cl[b:e]
            if shift:
                c = c.copy()
                c[:, 2] -= np.float32(shift) if s < 18 else -np.float32(shift)
            per_sector[s].append(c)
            per_sector_row[s].append(ev.row[b:e])
            if keep_truth and ev.truth is not None:
                t = ev.truth[b:e].copy()
                t["pad"] = i  # event index inside the frame
                per_sector_truth[s].append(t)
    parts = []
    for s in range(N_SECTORS):
        c = np.concatenate(per_sector[s]) if per_sector[s] else np.zeros((0, 4), np.float32)
        r = np.concatenate(per_sector_row[s]) if per_sector_row[s] else np.zeros(0, np.uint8)
        t = np.concatenate(per_sector_truth[s]) if keep_truth and per_sector_truth[s] else None
        if shuffle and c.shape[0]:
            perm = permutation(seed, stream, (tf_index << 8) | s | (1 << 40), c.shape[0])
            c, r = c[perm], r[perm]
            t = t[perm] if t is not None else None
        parts.append((slot, s, c, r, t))
    cl, row, units, truth = _concat_units(parts, keep_truth and all(p[4] is not None for p in parts))
    return Batch(cl, row, units, truth, {"workload": "timeframe", "n_events": n_events, "t0_us": t0,
                                         "seed": seed, "tf_index": tf_index})


def minbias_pool(seed=0, n=64, stream=STREAM_SERVED):
    """A pool of minimum-bias events at t0 = 0 from which served time frames are composed."""
    return _pmap(lambda e: _minbias_event(seed, stream, e), range(n))


def served_stream(seed=0, n_tf=100, rate_khz=50.0, min_events=8, max_events=256):
    """Sizes log-uniform in [8, 256] events and Poisson TF arrivals at the rate
    that carries 50 kHz of interactions: lambda_TF = 50 kHz / E[size]."""
    lo, hi = math.log(min_events), math.log(max_events)
    sizes = np.array([int(round(math.exp(lo + (hi - lo) * uniform(seed, STREAM_SERVED, i, 0x512E, 0))))
                      for i in range(n_tf)])
    # E[size] for log-uniform on [a, b]: (b - a) / ln(b / a)
    mean_size = (max_events - min_events) / (hi - lo)
    tf_rate_khz = rate_khz / mean_size
    arrivals = arrival_times_us(seed, STREAM_SERVED, 0x7F, n_tf, tf_rate_khz)
    return sizes, arrivals, mean_size
