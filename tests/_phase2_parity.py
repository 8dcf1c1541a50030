"""Element-by-element comparison of the GPU's second phase with the FP32
oracle (oracle/tpcphase2.cpp) for one slot.

The oracle gets the slot's segments in the GPU's order (units of the slot in
load order, tracks of a unit in ascending start ID), built from the oracle's
own sector results, which the phase-1 parity tests show equal to the GPU's.
Integer results (merge links, final-track composition and hits, vertex
membership, flags, compression records and residuals) must be identical and
every FP32 quantity bit-identical (the oracle's FP32 values are held exactly
by its doubles).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
from tests._parity import Mismatch, _eq

F32 = np.float32


def sector_results(batch, row_x, slot, workers=16):
    """Oracle results of the slot's units, indexed by sector, and per-sector
    cluster / row arrays (36 entries)."""
    units = [u for u in range(batch.units.shape[0]) if int(batch.units[u, 2]) == slot]
    cls = [np.zeros((0, 4), np.float32) for _ in range(36)]
    rows = [np.zeros(0, np.uint8) for _ in range(36)]
    for u in units:
        cl, row, _, sec, _ = batch.unit(u)
        cls[sec], rows[sec] = cl, row

    def one(s):
        return oracle.run_sector(cls[s], rows[s], row_x, precision=32) if cls[s].shape[0] else None
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(one, range(36)))
    order = [int(batch.units[u, 3]) for u in units]
    return res, cls, rows, order


def _n_tracks(res, s):
    return res[s].n_tracks if res[s] is not None else 0


def oracle_slot(res, cls, rows, order, row_x):
    """Second phase of the oracle on the slot's segments in unit order."""
    segs, hbs, hits_l = [], [], []
    for s in order:
        r = res[s]
        if r is None:  # a unit without clusters
            continue
        sg, hb, h = oracle.segments_of([None] * s + [r])
        segs.append(sg)
        hbs.append(hb)
        hits_l.append(h)
    seg = np.concatenate(segs) if segs else np.zeros(0, oracle.SEGMENT_DTYPE)
    hb = np.zeros(seg.shape[0] + 1, np.int64)
    hb[1:] = np.cumsum(seg["n_hits"]) if seg.shape[0] else []
    hits = np.concatenate(hits_l).astype(np.int32) if hits_l else np.zeros(0, np.int32)
    p2 = oracle.phase2(cls, rows, row_x, seg, hb, hits, precision=32)
    # key of every segment: sector << 24 | index among its unit's tracks
    keys = np.concatenate([(s << 24) + np.arange(_n_tracks(res, s)) for s in order]).astype(np.int64) \
        if seg.shape[0] else np.zeros(0, np.int64)
    return seg, hb, hits, p2, keys


def compare_slot(ctx, batch, row_x, slot, check_compression=True):
    """Phase-2 outputs of one slot against the oracle; returns a summary."""
    res, cls, rows, order = sector_results(batch, row_x, slot)
    seg, hb, hits, r, keys = oracle_slot(res, cls, rows, order, row_x)
    # merge links per unit
    off = 0
    for s in order:
        n = _n_tracks(res, s)
        nx, pv, fo = ctx.get_segment_links(slot, s, n)
        want_n = np.where(r.next[off:off + n] >= 0, keys[np.maximum(r.next[off:off + n], 0)], -1)
        want_p = np.where(r.prev[off:off + n] >= 0, keys[np.maximum(r.prev[off:off + n], 0)], -1)
        _eq(f"sector {s} merge next", nx, want_n)
        _eq(f"sector {s} merge prev", pv, want_p)
        _eq(f"sector {s} final of segment", fo, r.final_of_seg[off:off + n])
        off += n
    # final tracks
    gf, gh = ctx.get_finals(slot)
    rf = r.finals
    _eq("final count", gf.shape[0], rf.shape[0])
    for f in ("status", "n_seg", "sector", "n_hits", "ndf", "row_ref", "vertex", "z0_ok"):
        _eq(f"final {f}", gf[f], rf[f])
    _eq("final innermost segment", gf["first_seg"], keys[r.seg_order[rf["seg_begin"]]] if rf.shape[0] else [])
    _eq("final hit offsets", gf["hit_begin"], r.hit_begin[:-1])
    _eq("final hits", gh, r.hits)
    for f in ("x_ref", "chi2", "p", "cov", "z0", "t0", "z_conv"):
        _eq(f"final {f}", gf[f], rf[f].astype(F32))
    # vertices
    gv = ctx.get_vertices(slot)
    _eq("vertex count", gv.shape[0], r.vertices.shape[0])
    _eq("vertex t0", gv["t0"], r.vertices["t0"].astype(F32))
    _eq("vertex tracks", gv["n_tracks"], r.vertices["n_tracks"])
    _eq("vertex first", gv["first"], r.vertices["first"])
    # rejection flags
    sb = np.zeros(37, np.int64)
    sb[1:] = np.cumsum([c.shape[0] for c in cls])
    for s in order:
        n = cls[s].shape[0]
        _eq(f"sector {s} flags", ctx.get_flags(slot, s, n), r.flags[sb[s]:sb[s] + n])
    # compression
    if check_compression:
        for s in order:
            sg, shb, sh = oracle.segments_of([None] * s + [res[s]])
            rec, rs = oracle.compress(cls[s], rows[s], row_x, sg, shb, sh)
            grec, grs = ctx.get_compressed(slot, s)
            _eq(f"sector {s} compression records", grec, rec)
            _eq(f"sector {s} compression residuals", grs, rs)
    return {"segments": int(seg.shape[0]), "finals": int(rf.shape[0]), "merges": int((r.next >= 0).sum()),
            "vertices": int(r.vertices.shape[0]), "flagged": int((r.flags != 0).sum()),
            "near_ties": int(r.near_ties), "min_margin": float(r.min_margin),
            "tracker_near_ties": int(sum(x.near_ties for x in res if x is not None))}


__all__ = ["Mismatch", "compare_slot", "sector_results", "oracle_slot"]
