"""Per-slot runs of the CPU oracle (sector tracker, then the second phase)
shared by the second-phase pins and the GPU parity tests."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def slot_arrays(cl, row, units, truth=None, slot=None):
    """Per-sector lists (36 entries) of clusters, rows and truth of one slot
    of a batch (units (begin, n, slot, sector)); sectors without input get
    empty arrays."""
    cls = [np.zeros((0, 4), np.float32) for _ in range(36)]
    rows = [np.zeros(0, np.uint8) for _ in range(36)]
    trs = [None] * 36
    for b, n, sl, s in units:
        if slot is not None and sl != slot:
            continue
        cls[s], rows[s] = cl[b:b + n], row[b:b + n]
        if truth is not None:
            trs[s] = truth[b:b + n]
    return cls, rows, trs


def event_arrays(ev):
    """Per-sector lists of a tpcgen Event (clusters already grouped by sector)."""
    sb = ev.sector_begin
    cls = [ev.cl[sb[s]:sb[s + 1]] for s in range(36)]
    rows = [ev.row[sb[s]:sb[s + 1]] for s in range(36)]
    trs = [ev.truth[sb[s]:sb[s + 1]] if ev.truth is not None else None for s in range(36)]
    return cls, rows, trs


def sector_results(cls, rows, row_x, params=None, precision=32, workers=8):
    def one(s):
        return oracle.run_sector(cls[s], rows[s], row_x, params, precision) if cls[s].shape[0] else None
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, range(36)))


def run_slot(cls, rows, row_x, params=None, p2=None, precision=32, brute=False, results=None):
    """(per-sector results, segments, hit_begin, hits, second-phase result)"""
    res = results if results is not None else sector_results(cls, rows, row_x, params, precision)
    seg, hb, hits = oracle.segments_of(res)
    r = oracle.phase2(cls, rows, row_x, seg, hb, hits, params, p2, precision, brute)
    return res, seg, hb, hits, r
