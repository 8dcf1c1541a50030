"""Monte-Carlo truth matching shared by the quality tests.

A truth segment is one generating track's crossings of one sector on one
(half-turn, branch) leg: the maximal runs of consecutive rows.  A segment is
findable if it spans at least ``min_rows`` consecutive rows on the outgoing
branch of the first half-turn with |sin phi| <= ``max_sin`` throughout (the
paper's findable notion, Sec. 2 Fig. 3 caption, scaled to one sector: long
enough and inside the acceptance of the seeding windows).
"""
import numpy as np


def segment_keys(truth):
    return (truth["track"].astype(np.int64) * 8 + truth["leg"].astype(np.int64) * 2
            + truth["branch"].astype(np.int64))


def findable_segments(truth, row, min_rows=10, max_sin=0.85):
    """{(key, first_row): sorted array of cluster ids}"""
    out = {}
    sig = np.nonzero(truth["track"] >= 0)[0]
    keys = segment_keys(truth)
    order = np.lexsort((row[sig], keys[sig]))
    ids = sig[order]
    k = keys[ids]
    starts = np.r_[0, np.nonzero(np.diff(k))[0] + 1, ids.shape[0]]
    for a, b in zip(starts[:-1], starts[1:]):
        run_ids = ids[a:b]
        if truth["leg"][run_ids[0]] != 0 or truth["branch"][run_ids[0]] != 0:
            continue
        rr = row[run_ids].astype(np.int64)
        cuts = np.nonzero(np.diff(rr) != 1)[0] + 1
        for seg in np.split(run_ids, cuts):
            if seg.shape[0] >= min_rows and np.all(np.abs(truth["sinphi"][seg]) <= max_sin):
                out[(int(k[a]), int(row[seg[0]]))] = np.sort(seg)
    return out


def match_tracks(truth, row, track_hits, min_rows=10, max_sin=0.85, purity=0.9):
    """track_hits: list of arrays of cluster ids (one per accepted track).
    Returns dict with findable, found, exact, fakes, clones and pure labels."""
    keys = segment_keys(truth)
    seg = findable_segments(truth, row, min_rows, max_sin)
    by_cluster = {}
    for fk, ids in seg.items():
        for i in ids:
            by_cluster[int(i)] = fk
    found = {}
    fakes = 0
    exact = 0
    labels = []
    for t, hits in enumerate(track_hits):
        lab = keys[hits]
        lab = np.where(truth["track"][hits] >= 0, lab, -1)
        vals, cnt = np.unique(lab, return_counts=True)
        j = int(np.argmax(cnt))
        if vals[j] < 0 or cnt[j] < purity * hits.shape[0]:
            fakes += 1
            labels.append(None)
            continue
        labels.append(int(vals[j]))
        fks = {by_cluster.get(int(h)) for h in hits} - {None}
        for fk in fks:
            ids = seg[fk]
            if np.intersect1d(ids, hits).shape[0] * 2 >= ids.shape[0]:
                found.setdefault(fk, []).append(t)
                if np.array_equal(np.sort(hits), ids):
                    exact += 1
    clones = sum(len(v) - 1 for v in found.values())
    return {"findable": len(seg), "found": len(found), "exact": exact, "fakes": fakes,
            "clones": clones, "tracks": len(track_hits), "segments": seg, "matched": found,
            "labels": labels}
