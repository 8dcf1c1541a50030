"""Element-by-element comparison of GPU results with the FP32 oracle.

Links, tracklet hit lists, track hit lists and the cluster assignment must
be identical (integer results); every FP32 fit quantity must be bit-identical
too, because both sides run the same IEEE operation sequence (the oracle's
FP32 values are stored as doubles, which holds them exactly).
"""
import numpy as np

import oracle

F32 = np.float32


class Mismatch(AssertionError):
    pass


def _eq(name, a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape or not np.array_equal(a, b):
        bad = None
        if a.shape == b.shape:
            idx = np.nonzero(a.reshape(-1) != b.reshape(-1))[0]
            bad = (idx.shape[0], idx[:5].tolist())
        raise Mismatch(f"{name}: shapes {a.shape} vs {b.shape}, differing {bad}")


def compare_tracklets(gt, ghb, ghits, ref):
    rt = ref.tracklets
    _eq("tracklet count", gt.shape[0], rt.shape[0])
    for f in ("start_id", "n_chain", "status", "n_hits", "n_pass1", "ndf", "row_ref", "row_out"):
        _eq(f"tracklet {f}", gt[f], rt[f])
    _eq("tracklet hit offsets", ghb, ref.tracklet_hit_begin)
    _eq("tracklet hits", ghits, ref.tracklet_hits)
    for f in ("x_ref", "chi2", "x_out", "p", "cov", "p_out", "cov_out"):
        _eq(f"tracklet {f}", gt[f], rt[f].astype(F32))


def compare_tracks(gtr, ghits, ref):
    _eq("track count", gtr.shape[0], ref.n_tracks)
    src = ref.tracklets[ref.track_tracklet]
    _eq("track start_id", gtr["start_id"], src["start_id"])
    _eq("track p", gtr["p"], src["p"].astype(F32))
    _eq("track cov", gtr["cov"], src["cov"].astype(F32))
    _eq("track chi2", gtr["chi2"], src["chi2"].astype(F32))
    _eq("track x_ref", gtr["x_ref"], src["x_ref"].astype(F32))
    _eq("track ndf", gtr["ndf"], src["ndf"])
    _eq("track n_hits", gtr["n_hits"], np.diff(ref.track_hit_begin))
    _eq("track hit_offset", gtr["hit_offset"], ref.track_hit_begin[:-1])
    _eq("track hits", ghits, ref.track_hits)


def compare_unit_stagewise(ctx, slot, sector, cl, row, ref):
    n = cl.shape[0]
    up, dn = ctx.get_links(slot, sector, n, which=0)
    _eq("raw up", up, ref.up_raw)
    _eq("raw down", dn, ref.dn_raw)
    up, dn = ctx.get_links(slot, sector, n, which=1)
    _eq("clean up", up, ref.up)
    _eq("clean down", dn, ref.dn)
    gt, ghb, gh = ctx.get_tracklets(slot, sector)
    compare_tracklets(gt, ghb, gh, ref)
    gtr, ghits = ctx.get_tracks(slot, sector)
    compare_tracks(gtr, ghits, ref)
    _eq("assignment", ctx.get_assignment(slot, sector, n), ref.assignment)


def compare_batch(units, tracks, hits, asg, batch, refs):
    """Whole-batch outputs against per-unit oracle runs (refs[u] or None)."""
    for u in range(batch.units.shape[0]):
        if refs[u] is None:
            continue
        ur = units[u]
        ref = refs[u]
        b, n = int(batch.units[u, 0]), int(batch.units[u, 1])
        _eq(f"unit {u} n_clusters", ur["n_clusters"], n)
        _eq(f"unit {u} n_tracklets", ur["n_tracklets"], ref.tracklets.shape[0])
        t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
        h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
        compare_tracks(tracks[t0:t0 + nt], hits[h0:h0 + nh], ref)
        _eq(f"unit {u} assignment", asg[int(ur["cluster_begin"]):int(ur["cluster_begin"]) + n], ref.assignment)


def oracle_units(batch, row_x, which=None, params=None):
    refs = []
    for u in range(batch.units.shape[0]):
        if which is not None and u not in which:
            refs.append(None)
            continue
        cl, row, _, _, _ = batch.unit(u)
        refs.append(oracle.run_sector(cl, row, row_x, params, precision=32))
    return refs
