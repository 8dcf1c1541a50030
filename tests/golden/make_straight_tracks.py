"""Writes ``straight_tracks_b0.txt``: a hand-built sector of eight straight
tracks without magnetic field and without noise, and the result the tracker
must give on it, fixed by construction (not by running any tracker).

Why these values (Sec. 2, Fig. 1): hits of one track lie exactly on a
straight line, so every middle-row hit links to its own track's hits in the
rows next to it (Fig. 1a) and the chains are the tracks (Fig. 1b).  Edge rows
(0 and 158) get no links of their own, so the reciprocal links of a track run
from row 1 to row 157; track following (Fig. 1c) adds row 158 outward and
row 0 inward.  With the field off, the fit estimates a line: y, z at the
innermost row are the line's, sin(phi) = s / sqrt(1 + s^2) and tan(lambda) =
t / sqrt(1 + s^2) for dy/dx = s and dz/dx = t, and q/pT keeps its seed value
0 (nothing couples it to the measurements when the curvature constant is 0).
Each track is accepted with all 159 of its clusters; tracks are listed by
ascending ID of their chain's first cluster (the row-1 hit).

Run from the repository root: python tests/golden/make_straight_tracks.py
"""
import os

import numpy as np

N_ROWS = 159
# (dy/dx, dz/dx) of tracks from the origin; slopes keep them inside sector 0
# (|y| <= x tan 10 deg) and at least 3 cm apart in y or z on every row
TRACKS = [(-0.12, 0.10), (-0.08, 0.60), (-0.04, -0.30), (0.00, 0.25),
          (0.04, 0.80), (0.08, -0.70), (0.12, 0.40), (0.02, -0.05)]


def row_x():
    return (85.0 + np.arange(N_ROWS, dtype=np.float64) * (162.0 / 158.0)).astype(np.float32)


def main():
    rx = row_x()
    cl = []
    for k, (s, t) in enumerate(TRACKS):
        for r in range(N_ROWS):
            x = float(rx[r])
            cl.append((k, r, x, s * x, t * x))
    # a fixed relabelling so that IDs do not follow the tracks
    perm = np.random.default_rng(20171009).permutation(len(cl))
    cl = [cl[i] for i in perm]
    lines = ["# Straight tracks, field off, no noise: clusters and the result fixed by construction",
             "# (Sec. 2, Fig. 1a-c; see make_straight_tracks.py for why each value holds).",
             "# params: defaults with kB = 0",
             "# cluster: id row x y z (FP32 values, printed with 9 significant digits)"]
    for i, (k, r, x, y, z) in enumerate(cl):
        lines.append(f"cluster {i} {r} {np.float32(x):.9g} {np.float32(y):.9g} {np.float32(z):.9g}")
    # expected tracks: ascending start ID (the row-1 hit)
    exp = []
    for k, (s, t) in enumerate(TRACKS):
        ids = [i for i, c in enumerate(cl) if c[0] == k]
        start = next(i for i in ids if cl[i][1] == 1)
        x0 = float(rx[0])
        c = 1.0 / np.sqrt(1.0 + s * s)
        exp.append((start, k, s * x0, t * x0, s * c, t * c))
    exp.sort()
    lines.append("# track: start_id n_hits row_ref row_out x_ref y z sin_phi tan_lambda q_pt")
    for start, k, y, z, sp, tl in exp:
        lines.append(f"track {start} {N_ROWS} 0 {N_ROWS - 1} {float(rx[0]):.9g} {y:.9g} {z:.9g} "
                     f"{sp:.9g} {tl:.9g} 0")
    lines.append("# assignment: cluster id -> index of its track in the list above")
    order = {k: j for j, (_, k, *_rest) in enumerate(exp)}
    lines.append("assignment " + " ".join(str(order[c[0]]) for c in cl))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "straight_tracks_b0.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}: {len(cl)} clusters, {len(exp)} tracks")


if __name__ == "__main__":
    main()
