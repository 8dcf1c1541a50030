"""Benchmark of the gfx950 TPC sector tracker (one MI355X).

Headline value: tracked TPC clusters per second of the batched form on a
continuous-readout time frame (128 minimum-bias Pb-Pb events, Poisson
arrivals at 50 kHz, z shifted by the drift velocity, clusters mixed per
sector: about 32.5 M clusters), inputs resident in HBM, all stages replayed
as one captured HIP graph per step, two time frames in flight (two
contexts fed alternately, as the online farm processes several events in
parallel per GPU; each step is one whole frame).  The same frame with one
frame in flight is reported beside it ("sequential").

Also reported on the same JSON line:
  per_event   - the plain path, one launch per kernel per central Pb-Pb
                event (36 sectors, ~1.07 M clusters), and the ratio to it;
  served      - the continuous-batching server on time frames of 8-256
                events (log-uniform) at Poisson arrivals, host-resident
                inputs, p50 / p99 latency (see --served-tfs);
  stages      - per-stage HIP-event times of one instrumented pass;
  roofline    - the neighbour-finding kernel against HBM peak, and the
                Kalman-fit kernel timing;
  cpu_baseline- the plain CPU oracle on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3     # published vector FP32 (packed); 78.6 without packed FP32
LINK_BYTES_PER_CLUSTER = 16  # read y, z (8 B) + write up, down (8 B)
# algorithmic bytes of the fit per candidate examined, per update and per row step
FIT_BYTES_PER_ITEM = 8
# random 8-B loads over 2 GiB, each one 128-B line (profiles/memory_ceilings_random_access.md)
RANDOM_LINE_CEILING_GPS = 53.5
# FP32 operations of the fit per counted event (fma = 2, div / sqrt = 1):
FIT_FLOPS = {
    "fit_steps": 154,       # propagation: 52 state + 102 covariance
    "fit_tests": 20,        # chi2 of a searched hit
    "fit_updates": 130,     # Kalman update: gain, state, covariance, chi2
    "fit_candidates": 5,    # window candidate: residuals and squared distance
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--events", type=int, default=128, help="events per time frame")
    ap.add_argument("--served-tfs", type=int, default=1000, help="time frames per served load level (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3")
    ap.add_argument("--retune", action="store_true", help="re-run the schedule autotuner")
    ap.add_argument("--summarize-profile", nargs=4, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="write the profiles/ summaries from rocprofv3 outputs of --profile runs")
    ap.add_argument("--sq-dir", default=None, help="with --summarize-profile: an SQ counter pass to add")
    ap.add_argument("--summary-name", default=None,
                    help="with --summarize-profile: write profiles/<name>.md and leave the traffic file "
                         "(the bench line's counters) alone")
    ap.add_argument("--fit-rows", type=int, default=0,
                    help="with --profile: the row-synchronous fit with chunks of this many tracklets "
                         "(tuning knob fit_rows; 0: the schedule as tuned)")
    ap.add_argument("--ceilings", action="store_true",
                    help="run the random-access microbenchmark and write its summary under profiles/")
    ap.add_argument("--profile-pipelined", action="store_true",
                    help="short run for rocprofv3: 4 warm-up + 8 time frames with two in flight")
    ap.add_argument("--summarize-pipelined", nargs=2, metavar=("TRACE_DIR", "COMMAND"),
                    help="write the overlap summary of a --profile-pipelined kernel trace under profiles/")
    return ap.parse_args()


def main():
    args = parse()
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile, sq_dir=args.sq_dir, out_name=args.summary_name)
        return
    if args.ceilings:
        ceilings()
        return
    if args.summarize_pipelined:
        summarize_pipelined(*args.summarize_pipelined)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only (--gpus 1); sectors and time frames are independent "
              "units, so several GPUs would each run a server of their own on separate frames",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import tpcgen
    from paper_1709_00618_amd import tpcca

    tpcca.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rx = tpcgen.row_x()

    if args.profile_pipelined:
        profile_pipelined(rx)
        return
    if args.profile:
        args.steps, args.warmup, args.served_tfs = min(args.steps, 3), 1, 0
        args.no_cpu_baseline = True
        # a plain device copy of known size: the reference that scales the
        # FETCH_SIZE / WRITE_SIZE counters of the profiled kernels
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst

    # measured copy bandwidth (read + write of a 1 GiB device copy), the
    # streaming ceiling beside the published 8 TB/s
    copy_gbs = None
    if not args.profile:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        a.fill_(1)
        bcp = torch.empty_like(a)
        for _ in range(3):
            bcp.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            bcp.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * (1 << 30) * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
        del a, bcp

    # ------------------------------------------------------------ inputs
    t = time.time()
    tf = tpcgen.timeframe(seed=0, n_events=args.events)
    log(f"time frame: {tf.n_clusters} clusters in {tf.units.shape[0]} sector units "
        f"({time.time() - t:.1f} s to generate)")
    dcl = torch.from_numpy(tf.cl).cuda()
    drow = torch.from_numpy(tf.row).cuda()
    ev = tpcgen.central_event(seed=0, keep_truth=False)
    ecl = torch.from_numpy(ev.cl).cuda()
    erow = torch.from_numpy(ev.row).cuda()
    torch.cuda.synchronize()

    # ------------------------------------------------- batched (headline)
    ctx = tpcca.Context(rx, device=0)
    ctx2 = None if args.profile else tpcca.Context(rx, device=0)  # second frame in flight
    from paper_1709_00618_amd import autotune
    if args.profile:  # never tune under a profiler
        entry = autotune.lookup(tf.n_clusters, len(tf.units))
        knobs, knob_src = (entry["knobs"], "cache") if entry else (ctx.get_tuning(), "default")
        if args.fit_rows:
            knobs, knob_src = dict(knobs, fit_rows=args.fit_rows), knob_src + " + fit_rows"
        ctx.set_tuning(**knobs)
    else:
        # the schedule is tuned with two frames in flight, as the headline runs
        knobs, knob_src = autotune.tuned(ctx, dcl, drow, tf.units, tf.n_clusters, log=log, retune=args.retune,
                                         ctx2=ctx2)
    log(f"schedule ({knob_src}): {knobs}")
    # the captured graph carries HIP event nodes at the stage boundaries, on
    # the stream the kernels run on: every timed replay times its own stages
    ctx.set_timing(True)
    for _ in range(args.warmup):
        ctx.run_batch(dcl, drow, tf.units, device=True, graph=True)
        ctx.sync()
    torch.cuda.synchronize()
    stage_runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run_batch(dcl, drow, tf.units, device=True, graph=True)
        ctx.sync()
        stage_runs.append(ctx.stage_times())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.set_timing(False)
    nu, ncl, ntr, nhits = ctx.batch_totals()
    work = ctx.work_stats()
    batched = ncl / dt
    log(f"batched time frame: {dt * 1e3:.2f} ms/step, {batched / 1e9:.3f} G clusters/s, "
        f"{ntr} tracks, {nhits} assigned clusters; work {work}")
    stages = {k: float(np.mean([s[k] for s in stage_runs])) for k in stage_runs[0]}
    log("stage ms (timed replays): " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))

    # ------------------------------ pipelined: two time frames in flight
    # two contexts, each with its own stream and buffers, fed alternately:
    # one frame's early stages fill the GPU while the other's fit drains
    in_flight, pipe_dt = 1, dt
    if not args.profile:
        pipe = [ctx, ctx2]
        for i in range(2 * args.warmup):
            pipe[i % 2].run_batch(dcl, drow, tf.units, device=True, graph=True)
        for c in pipe:
            c.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            pipe[i % 2].run_batch(dcl, drow, tf.units, device=True, graph=True)
        for c in pipe:
            c.sync()
        torch.cuda.synchronize()
        pipe_dt = (time.perf_counter() - t0) / args.steps
        in_flight = 2
        # both contexts tracked the same frame: same totals and work counts
        assert ctx2.batch_totals() == (nu, ncl, ntr, nhits), "pipelined frame totals differ"
        w2 = ctx2.work_stats()
        assert all(w2[k] == work[k] for k in ("tracklets", "fit_steps", "fit_updates", "track_hits")), \
            "pipelined work counts differ"
        ctx2.close()
        log(f"pipelined (2 frames in flight): {pipe_dt * 1e3:.2f} ms/frame, "
            f"{ncl / pipe_dt / 1e9:.3f} G clusters/s")
    value = ncl / pipe_dt

    # -------------------------------- second phase on the resident frame
    # merging of the sector segments and refit (Sec. 2), vertex times
    # (Sec. 5), rejection flags and track-model compression (Sec. 3), run on
    # the tracks the frame's batch left in HBM (no host transfer)
    phase2 = None
    if not args.profile:
        phase2 = bench_phase2(ctx, dcl, drow, tf, args, log)
    else:
        # two calls of the second phase on the frame just tracked (their
        # kernels are the k_p2_* dispatches of the profile)
        for _ in range(2):
            ctx.phase2()
            ctx.sync()

    # --------------------------------------------- per-event plain path
    pe = tpcca.Context(rx, device=0)

    def per_event_step():
        pe.reset()
        for u in range(ev.units.shape[0]):
            b, n, slot, sec = (int(v) for v in ev.units[u])
            pe.load_sector(slot, sec, ecl[b:b + n], erow[b:b + n], device=True)
        pe.run_all(0, -1)
        pe.sync()

    for _ in range(args.warmup):
        per_event_step()
    pe_steps = max(args.steps, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(pe_steps):
        per_event_step()
    torch.cuda.synchronize()
    pe_dt = (time.perf_counter() - t0) / pe_steps
    per_event = ev.n_clusters / pe_dt
    log(f"per-event plain: {pe_dt * 1e3:.2f} ms/event, {per_event / 1e9:.3f} G clusters/s")
    pe.close()

    # ------------------------------------------ host-resident bases
    # inputs in pinned host memory (the library copies them in), every
    # result (tracks, hits, assignment) copied back into pinned host buffers:
    # the basis of the served path, for the plain per-event path and for the
    # batched frame (one in flight)
    host_res = None
    if not args.profile:
        keep = []

        def pinned(n, dtype):
            dtype = np.dtype(dtype)
            t = torch.empty(max(1, n) * dtype.itemsize, dtype=torch.uint8, pin_memory=True)
            keep.append(t)
            return t.numpy().view(dtype)

        def host_in(b):
            hc = pinned(b.cl.shape[0] * 4, np.float32).reshape(-1, 4)
            hc[:] = b.cl
            hr = pinned(b.row.shape[0], np.uint8)
            hr[:] = b.row
            return hc, hr

        def host_out(n_cl, n_units):
            # accepted tracks own disjoint sets of >= 10 hits
            return (pinned(n_units, tpcca.UNIT_RESULT_DTYPE), pinned(n_cl // 10 + n_units + 1, tpcca.TRACK_DTYPE),
                    pinned(n_cl, np.int32), pinned(n_cl, np.int32))

        def timed(step, n):
            for _ in range(args.warmup):
                step()
            t0 = time.perf_counter()
            for _ in range(n):
                step()
            return (time.perf_counter() - t0) / n

        ev_in, ev_out = host_in(ev), host_out(ev.n_clusters, ev.units.shape[0])
        he = tpcca.Context(rx, device=0)
        he_dt = timed(lambda: (he.run_batch(ev_in[0], ev_in[1], ev.units, device=False, graph=False),
                               he.get_batch_results(out=ev_out)), pe_steps)
        he.close()
        tf_in, tf_out = host_in(tf), host_out(tf.n_clusters, tf.units.shape[0])
        hb_dt = timed(lambda: (ctx.run_batch(tf_in[0], tf_in[1], tf.units, device=False, graph=True),
                               ctx.get_batch_results(out=tf_out)), max(5, args.steps // 2))
        host_res = {"per_event": {"value": round(ev.n_clusters / he_dt, 1), "ms_per_event": round(he_dt * 1e3, 4)},
                    "batched": {"value": round(ncl / hb_dt, 1), "ms_per_step": round(hb_dt * 1e3, 4),
                                "in_flight": 1},
                    "batched_over_per_event": round((ncl / hb_dt) / (ev.n_clusters / he_dt), 3),
                    "unit": "clusters/s",
                    "basis": "pinned host inputs and outputs: H2D + all stages + D2H of tracks, hits, assignment"}
        log(f"host-resident: per-event {he_dt * 1e3:.2f} ms, batched frame {hb_dt * 1e3:.2f} ms "
            f"({host_res['batched_over_per_event']}x)")
        del keep, ev_in, ev_out, tf_in, tf_out

    # ------------------------------------- time against frame size
    # device-resident, one frame in flight: t = a + b N over frames of
    # 8 .. 128 events (the paper's linear dependence on the input size)
    lin = None
    if not args.profile:
        pts = []
        for k in (8, 16, 32, 64):
            tk = tpcgen.timeframe(seed=0, n_events=k)
            kcl, krow = torch.from_numpy(tk.cl).cuda(), torch.from_numpy(tk.row).cuda()
            torch.cuda.synchronize()
            for _ in range(2):
                ctx.run_batch(kcl, krow, tk.units, device=True, graph=True)
                ctx.sync()
            t0 = time.perf_counter()
            for _ in range(5):
                ctx.run_batch(kcl, krow, tk.units, device=True, graph=True)
                ctx.sync()
            pts.append((tk.n_clusters, (time.perf_counter() - t0) / 5 * 1e3))
            del kcl, krow
        pts.append((ncl, dt * 1e3))
        xs, ys = np.array([p[0] for p in pts], float), np.array([p[1] for p in pts], float)
        b_, a_ = np.polyfit(xs, ys, 1)
        r2 = 1.0 - float(np.sum((ys - (a_ + b_ * xs)) ** 2) / max(1e-30, np.sum((ys - ys.mean()) ** 2)))
        lin = {"points_clusters_ms": [[int(x), round(y, 4)] for x, y in pts], "a_ms": round(float(a_), 4),
               "b_ns_per_cluster": round(float(b_) * 1e6, 5), "r2": round(r2, 5)}
        log(f"time vs size: t = {a_:.3f} ms + {b_ * 1e6:.4f} ns x N (r2 {r2:.4f})")

    # ---------------------------------- 64 minimum-bias events, one launch
    mb64 = None
    if not args.profile:
        mb64 = bench_minbias64(rx, tpcca, torch, args, log, knobs)

    # the headline context is not needed any more: closed before the server
    # starts, so that its stream does not share a hardware queue with the
    # lanes' streams (HIP gives a process four by default)
    ctx.close()

    # ------------------------------------------------------------ served
    served = None
    if args.served_tfs > 0:
        from paper_1709_00618_amd import serving
        served = serving.bench_served(rx, n_tf=args.served_tfs, log=log)

    # ---------------------------------------------------------- roofline
    # dominant kernel: the Kalman fit.  What binds it is the memory system's
    # handling of random accesses (one 128-B line per 8-B load, partial-line
    # stores, memory-side atomics): quoted against HBM with its algorithmic
    # bytes (8 B, the y and z of a hit, per candidate examined and per
    # update, and 8 B per row step for the bin pair of the row), its
    # measured traffic beside them, its line fetches against the measured
    # random-load ceiling, and its arithmetic against the FP32 peak
    traffic = measured_traffic()
    fit_ms = stages["fit"]
    flops = sum(FIT_FLOPS[k] * work[k] for k in FIT_FLOPS)
    fit_tf = flops / (fit_ms * 1e-3) / 1e12
    fit_alg = FIT_BYTES_PER_ITEM * (work["fit_candidates"] + work["fit_updates"] + work["fit_steps"])
    fit_gbs = fit_alg / (fit_ms * 1e-3) / 1e9
    fit_lines = (traffic.get("k_kf_fetch") or 0) / 128.0
    random_access = {"ceiling_G_lines_per_s": RANDOM_LINE_CEILING_GPS,
                     "achieved_G_lines_per_s": (round(fit_lines / (fit_ms * 1e-3) / 1e9, 2) if fit_lines else None),
                     "frac": (round(fit_lines / (fit_ms * 1e-3) / 1e9 / RANDOM_LINE_CEILING_GPS, 4)
                              if fit_lines else None),
                     "basis": "FETCH_SIZE of the committed counter pass / 128 B per line, over the fit's time "
                              "(null when the kernel sources changed since the pass)"}
    roofline = {"kernel": "k_kf (tracklet fit and track following)", "bound": "hbm",
                "binding_resource": "random 128-B line fetches, partial stores and atomics (see random_access)",
                "achieved": round(fit_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(fit_gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get("k_kf"),
                "algorithmic_bytes": int(fit_alg),
                "bytes_basis": "8 B per candidate examined, per update and per row step (device work counters)",
                "random_access": random_access,
                "alu": {"achieved": round(fit_tf, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(fit_tf / FP32_PEAK_TFLOPS, 4), "flops_per_launch": int(flops),
                        "flops_per_step": round(flops / max(1, work["fit_steps"]), 1)},
                "lane_use": round(work["fit_steps"] / max(1, 64 * work["fit_wave_iterations"]), 4),
                "valu_busy": (round(measured_valu_busy()["k_kf"], 4)
                              if "k_kf" in measured_valu_busy() else None),
                "ms": round(fit_ms, 4)}
    link_ms = stages["links"]
    link_bytes = LINK_BYTES_PER_CLUSTER * ncl
    link_gbs = link_bytes / (link_ms * 1e-3) / 1e9
    roofline_links = {"kernel": "k_links (CA neighbour finding)", "bound": "hbm", "achieved": round(link_gbs, 1),
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(link_gbs / HBM_PEAK_GBS, 4),
                      "traffic": traffic.get("k_links"), "bytes_per_cluster": LINK_BYTES_PER_CLUSTER,
                      "ms": round(link_ms, 4),
                      "valu_busy": (round(measured_valu_busy()["k_links"], 4)
                                    if "k_links" in measured_valu_busy() else None),
                      "copy_gbs": round(copy_gbs, 1) if copy_gbs else None,
                      "frac_of_copy": round(link_gbs / copy_gbs, 4) if copy_gbs else None}

    # ------------------------------------------------------ cpu baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ev, rx, args.cpu_seconds)

    out = {
        "metric": "tracked TPC clusters/s on 1 MI355X (batched time frame; served and per-event beside)",
        "value": round(value, 1),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(pipe_dt * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded helices, tpcgen)",
        "config": {"workload": f"continuous-readout time frame: {args.events} min-bias Pb-Pb events at 50 kHz, "
                               f"36 sector units, {ncl} clusters, device-resident, graph replay, "
                               f"{in_flight} frame(s) in flight",
                   "clusters": ncl, "units": nu, "tracks": ntr, "assigned_clusters": nhits,
                   "in_flight": in_flight},
        "tracks_per_s": round(ntr / pipe_dt, 1),
        "sequential": {"value": round(batched, 1), "unit": "clusters/s", "ms_per_step": round(dt * 1e3, 4),
                       "in_flight": 1},
        "schedule": {"knobs": knobs, "source": knob_src},
        "work": work,
        "per_event": {"workload": f"central Pb-Pb event, 8000 tracks, {ev.n_clusters} clusters, one launch per "
                                  "kernel per event, device-resident",
                      "value": round(per_event, 1), "unit": "clusters/s", "ms_per_event": round(pe_dt * 1e3, 4)},
        "batched_over_per_event": round(value / per_event, 3),
        "host_resident": host_res,
        "served_over_per_event": (round(served["capacity"]["clusters_per_s"] / host_res["per_event"]["value"], 3)
                                  if served and host_res else None),
        "phase2": phase2,
        "batched_minbias64": mb64,
        "linear_scaling": lin,
        "served": served,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": roofline,
        "roofline_links": roofline_links,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_timeframe128.json")
KERNEL_SOURCES = ("paper_1709_00618_amd/csrc/tpcca_kernels.hip", "paper_1709_00618_amd/csrc/tpcca_internal.h",
                  "paper_1709_00618_amd/csrc/tpcca_kf.h", "paper_1709_00618_amd/csrc/tpcca_dev.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_valu_busy():
    """Kernel -> VALU busy fraction from the committed SQ pass, while the
    kernel sources still hash to the profiled ones."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("source_hash") != kernel_source_hash():
        return {}
    return {k: v["valu_busy"] for k, v in t.get("kernels", {}).items() if "valu_busy" in v}


def measured_traffic():
    """HBM bytes per launch of each kernel from the committed counter passes,
    only while the kernel sources are the ones the counters were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return {}
    out = {k: v["bytes"] for k, v in t["kernels"].items()}
    for k, v in t["kernels"].items():
        if "fetch_size" in v:
            out[k + "_fetch"] = v["fetch_size"]
    return out


def summarize_profile(trace_dir, fetch_dir, write_dir, command, sq_dir=None, out_name=None):
    """Turn the rocprofv3 outputs of `bench.py --profile` (a kernel trace and
    FETCH_SIZE / WRITE_SIZE passes) into the committed summaries: per-kernel
    durations of the time-frame dispatches and counter bytes scaled by the
    plain 1 GiB device copy that the profile run makes first."""
    import csv
    import glob

    def one(d, pat):
        fs = glob.glob(os.path.join(d, "**", pat), recursive=True)
        assert fs, f"no {pat} under {d}"
        return fs[0]

    def short(name):
        n = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()
        return n.replace("tpcca::", "")

    tf_n = 4  # bench.py --profile: 1 warm-up + 3 timed replays of the time frame

    def tf_end(ids_names):
        # the time-frame replays come first; each ends with k_output
        outs = sorted(i for i, n in ids_names if short(n) == "k_output")
        return outs[tf_n - 1] if len(outs) >= tf_n else max(i for i, _ in ids_names)

    # kernel trace: split at the last dispatch of the time-frame replays
    rows = sorted(csv.DictReader(open(one(trace_dir, "*kernel_trace.csv"))), key=lambda r: int(r["Dispatch_Id"]))
    end_tr = tf_end([(int(r["Dispatch_Id"]), r["Kernel_Name"]) for r in rows])
    per, per_o = {}, {}
    for r in rows:
        (per if int(r["Dispatch_Id"]) <= end_tr else per_o).setdefault(short(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["| kernel | TF dispatches | avg us (TF) | share | other dispatches | avg us (other) |",
             "|---|---|---|---|---|---|"]
    tf_tot = {k: sum(v) for k, v in per.items() if k.startswith("k_")}
    total = sum(tf_tot.values())
    for k in sorted(tf_tot, key=lambda k: -tf_tot[k]):
        a, b = per[k], per_o.get(k, [])
        lines.append(f"| {k} | {len(a)} | {np.mean(a):.1f} | {100 * tf_tot[k] / total:.1f}% | {len(b)} | "
                     f"{(np.mean(b) if b else 0):.1f} |")

    def counters(d, name):
        vals = {}
        for r in csv.DictReader(open(one(d, "*counter_collection.csv"))):
            if r["Counter_Name"] != name:
                continue
            vals.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        end = tf_end([(k, v[0]) for k, v in vals.items()])
        return [vals[k] + [k <= end] for k in sorted(vals)]

    out = {"source_hash": kernel_source_hash(), "command": command, "kernels": {}}
    fac = {}
    for cname, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        seq = counters(d, cname)
        # the calibration copy: 1 GiB read and written; first dispatches before any tracker kernel
        cal = []
        for name, v, _ in seq:
            if "tpcca" in name:
                break
            cal.append((name, v))
        # the copies (0.5 GiB of FETCH, 1 GiB of WRITE each); the fill before
        # them reads nothing
        big = [v for name, v in cal if v > 0.1 * (1 << 20)]  # KiB
        fac[cname] = (1 << 20) / float(np.median(big)) if big else 1.0
        byk = {}
        for name, v, in_tf in seq:
            # the time frame's kernels, and the second phase's (run on it after the replays)
            if "tpcca" in name and (in_tf or short(name).startswith("k_p2")):
                byk.setdefault(short(name), []).append(v * 1024.0 * fac[cname])
        for k, v in byk.items():
            e = out["kernels"].setdefault(k, {})
            e[cname.lower()] = float(np.mean(v))
    for k, e in out["kernels"].items():
        e["bytes"] = e.get("fetch_size", 0.0) + e.get("write_size", 0.0)
    out["factor"] = fac
    # a templated kernel is also reported under its plain name (the variant
    # the profiled schedule ran)
    for k in list(out["kernels"]):
        if "<" in k:
            out["kernels"].setdefault(k.split("<")[0], out["kernels"][k])
    if not out_name:
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
    md = ["# Kernel trace and HBM traffic: batched time frame (128 events, 32.5 M clusters)"
          + (f" — {out_name}" if out_name else ""), "",
          "Command (run from the repository root; `$R` = repository root):", "", "```", command, "```", "",
          "`bench.py --profile`: a 1 GiB device copy (counter calibration), then 1 warm-up + 3 timed graph "
          "replays of the time frame (the TF dispatches below), then two calls of the second phase on that frame "
          "(its `k_p2_*` kernels and the radix sort) and the per-event path (other dispatches).", "",
          "## Durations (kernel trace)", ""] + lines + ["",
          f"Sum of TF kernel time over {tf_n} replays: {total / 1e3:.2f} ms ({total / tf_n / 1e3:.2f} ms per replay).",
          "", "## HBM traffic per TF dispatch (FETCH_SIZE + WRITE_SIZE, scaled by the copy)", "",
          f"Scale factors (1 GiB / counter reading of the copy): FETCH {fac['FETCH_SIZE']:.4f}, "
          f"WRITE {fac['WRITE_SIZE']:.4f}.", "",
          "| kernel | fetch MB | write MB | total MB |", "|---|---|---|---|"]
    for k in sorted(out["kernels"], key=lambda k: -out["kernels"][k]["bytes"]):
        if "<" not in k and any(q.startswith(k + "<") for q in out["kernels"]):
            continue  # alias of a templated kernel's variant
        e = out["kernels"][k]
        md.append(f"| {k} | {e.get('fetch_size', 0) / 1e6:.1f} | {e.get('write_size', 0) / 1e6:.1f} | "
                  f"{e['bytes'] / 1e6:.1f} |")
    if sq_dir:
        # instruction counters per wave of the TF dispatches (summed over the chip)
        per_k = {}
        sq_rows = list(csv.DictReader(open(one(sq_dir, "*counter_collection.csv"))))
        end_sq = tf_end([(int(r["Dispatch_Id"]), r["Kernel_Name"]) for r in sq_rows])
        for r in sq_rows:
            if "tpcca" not in r["Kernel_Name"] or int(r["Dispatch_Id"]) > end_sq:
                continue
            d = per_k.setdefault(short(r["Kernel_Name"]), {})
            d.setdefault(int(r["Dispatch_Id"]), {}).setdefault(r["Counter_Name"], 0.0)
            d[int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
        md += ["", "## Instruction counters per wave (SQ pass, TF dispatches)", "",
               "| kernel | waves | VALU | SALU | LDS | VMEM rd | VMEM wr | waiting % of wave cycles |",
               "|---|---|---|---|---|---|---|---|"]
        rows_sq = []
        for k, d in per_k.items():
            ds = [d[x] for x in sorted(d)]
            avg = {c: float(np.mean([x.get(c, 0.0) for x in ds])) for c in ds[0]}
            w = max(1.0, avg.get("SQ_WAVES", 1.0))
            rows_sq.append((tf_tot.get(k, 0.0), k, w, avg))
            # VALU busy: wave64 VALU instructions take 4 cycles of a SIMD;
            # against the kernel's traced duration on 1024 SIMDs at 2.4 GHz
            dur_us = float(np.mean(per[k])) if k in per else 0.0
            if dur_us > 0:
                e = out["kernels"].setdefault(k, {})
                e["valu_busy"] = 4.0 * avg.get("SQ_INSTS_VALU", 0.0) / (1024 * dur_us * 1e-6 * 2.4e9)
                e["sq"] = {c: v for c, v in avg.items()}
        # refresh the file with the SQ figures (and the plain-name aliases)
        for k in list(out["kernels"]):
            if "<" in k:
                out["kernels"][k.split("<")[0]] = out["kernels"][k]
        if not out_name:
            with open(TRAFFIC_FILE, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)
        for _, k, w, a in sorted(rows_sq, reverse=True):
            md.append(f"| {k} | {w:.0f} | {a.get('SQ_INSTS_VALU', 0) / w:.0f} | {a.get('SQ_INSTS_SALU', 0) / w:.0f} | "
                      f"{a.get('SQ_INSTS_LDS', 0) / w:.0f} | {a.get('SQ_INSTS_VMEM_RD', 0) / w:.0f} | "
                      f"{a.get('SQ_INSTS_VMEM_WR', 0) / w:.0f} | "
                      f"{100 * a.get('SQ_WAIT_ANY', 0) / max(1.0, a.get('SQ_WAVE_CYCLES', 1)):.0f} |")
    # the second phase's kernels (two calls on the time frame, after the replays)
    p2 = {k: v for k, v in per_o.items() if k.startswith("k_p2") or "rocprim" in k}
    if p2:
        p2_tot = {k: sum(v) for k, v in p2.items()}
        md += ["", "## Second phase on the time frame (two calls)", "",
               "| kernel | dispatches | avg us | share | fetch MB | write MB |", "|---|---|---|---|---|---|"]
        for k in sorted(p2_tot, key=lambda k: -p2_tot[k]):
            e = out["kernels"].get(k, {})
            name = "radix sort (hipCUB / rocPRIM)" if "rocprim" in k else k
            md.append(f"| {name} | {len(p2[k])} | {np.mean(p2[k]):.1f} | {100 * p2_tot[k] / sum(p2_tot.values()):.1f}% | "
                      f"{e.get('fetch_size', 0) / 1e6:.1f} | {e.get('write_size', 0) / 1e6:.1f} |")
        md.append(f"Sum per call: {sum(p2_tot.values()) / 2e3:.2f} ms of kernel time.")
    md += ["", f"Kernel sources hash: `{out['source_hash']}` (bench.py reports traffic only while it matches)."]
    path = os.path.join(ROOT, "profiles", (out_name or "tracker_timeframe128_kernel_trace") + ".md")
    with open(path, "w") as f:
        f.write("\n".join(md) + "\n")
    print(f"wrote {path}" + ("" if out_name else f" and {TRAFFIC_FILE}"))


def profile_pipelined(rx):
    """Two contexts fed alternately with the time frame (cached schedule):
    4 warm-up frames, then 8 frames; for a kernel trace of the overlap."""
    import torch

    import tpcgen
    from paper_1709_00618_amd import autotune, tpcca

    tf = tpcgen.timeframe(seed=0, n_events=128)
    dcl, drow = torch.from_numpy(tf.cl).cuda(), torch.from_numpy(tf.row).cuda()
    torch.cuda.synchronize()
    entry = autotune.lookup(tf.n_clusters, len(tf.units))
    ctxs = [tpcca.Context(rx, device=0) for _ in range(2)]
    for c in ctxs:
        if entry:
            c.set_tuning(**entry["knobs"])
    for i in range(4):
        ctxs[i % 2].run_batch(dcl, drow, tf.units, device=True, graph=True)
    for c in ctxs:
        c.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(8):
        ctxs[i % 2].run_batch(dcl, drow, tf.units, device=True, graph=True)
    for c in ctxs:
        c.sync()
    log(f"8 frames, two in flight: {(time.perf_counter() - t0) / 8 * 1e3:.2f} ms/frame")
    for c in ctxs:
        c.close()


def summarize_pipelined(trace_dir, command):
    """Overlap of the two frames' kernels in a --profile-pipelined trace: the
    window after the 4 warm-up frames, how long the GPU runs at least one
    and at least two tracker kernels, and the idle gaps."""
    import csv
    import glob

    fs = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    assert fs, f"no kernel trace under {trace_dir}"
    rows = [r for r in csv.DictReader(open(fs[0])) if "tpcca" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    outs = [r for r in rows if "k_output" in r["Kernel_Name"]]
    t_begin = int(outs[3]["End_Timestamp"])
    win = [r for r in rows if int(r["Start_Timestamp"]) >= t_begin]
    t_end = max(int(r["End_Timestamp"]) for r in win)
    ev = sorted([(int(r["Start_Timestamp"]), 1) for r in win] + [(int(r["End_Timestamp"]), -1) for r in win])
    busy = both = idle = 0
    cur, last, gaps = 0, ev[0][0], []
    for t, d in ev:
        if cur >= 1:
            busy += t - last
        if cur >= 2:
            both += t - last
        if cur == 0 and t > last:
            gaps.append(t - last)
        cur += d
        last = t
    span = t_end - t_begin
    per_q = {}
    for r in win:
        per_q.setdefault(r["Queue_Id"], 0)
        per_q[r["Queue_Id"]] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    md = ["# Overlap of two time frames in flight (128 events, 32.5 M clusters each)", "",
          "Command (run from the repository root; `$R` = repository root):", "", "```", command, "```", "",
          "`bench.py --profile-pipelined`: two contexts fed alternately, 4 warm-up frames, then 8 frames "
          "(the window below starts at the end of the 4th warm-up frame).", "",
          f"- window: {span / 1e6:.2f} ms for 8 frames = {span / 8e6:.2f} ms per frame",
          f"- at least one tracker kernel running: {busy / 1e6:.2f} ms ({100 * busy / span:.1f} %)",
          f"- at least two (both frames) running: {both / 1e6:.2f} ms ({100 * both / span:.1f} %)",
          f"- idle gaps: {len(gaps)}, total {sum(gaps) / 1e3:.1f} us, largest {max(gaps, default=0) / 1e3:.1f} us",
          "- kernel time per queue (each frame's kernels run longer when they share the GPU): " +
          ", ".join(f"queue {q}: {v / 1e6:.2f} ms" for q, v in sorted(per_q.items())), ""]
    path = os.path.join(ROOT, "profiles", "pipelined_timeframe128_overlap.md")
    with open(path, "w") as f:
        f.write("\n".join(md))
    print(f"wrote {path}")


def ceilings():
    """Random-access ceilings of the GPU (paper_1709_00618_amd/membench, a
    measurement tool built here with hipcc, not part of the library): the
    rates that bound the fit and the selection."""
    import subprocess

    from paper_1709_00618_amd import build as gpu_build
    exe = gpu_build.build_membench()
    out = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=300)
    text = out.stdout.decode(errors="replace")
    print(text, end="", flush=True)
    if out.returncode != 0:
        sys.exit(out.returncode)
    write_ceilings(text)


def write_ceilings(text):
    """profiles/memory_ceilings_random_access.md from the output of membench."""
    md = ["# Random-access ceilings of one MI355X", "",
          "Command (run from the repository root): `python3 bench.py --ceilings` (runs "
          "`paper_1709_00618_amd/membench`, which `--ceilings` builds from "
          "`paper_1709_00618_amd/csrc/membench.hip`; it is a measurement tool, not part of the library).", "",
          "256 x 32 blocks of 256 threads; random addresses over the table size in brackets "
          "(2 GiB where none is given); one warm launch, the rate of 5 timed launches. "
          "`wg scope`: workgroup-scope atomics, each XCD on a region of its own. The last line "
          "maps each block of a 8192-block launch to the XCD it ran on (hardware register XCC_ID).",
          "", "```", text.rstrip(), "```", ""]
    path = os.path.join(ROOT, "profiles", "memory_ceilings_random_access.md")
    with open(path, "w") as f:
        f.write("\n".join(md))
    print(f"wrote {path}")


def _entropy_bits(v):
    """Zeroth-order empirical entropy (bits per symbol) of an integer array."""
    v = np.asarray(v, np.int64).ravel()
    if v.size == 0:
        return 0.0
    _, c = np.unique(v, return_counts=True)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def bench_phase2(ctx, dcl, drow, tf, args, log):
    """The second phase on the frame the context tracked last: its time per
    call (the kernels and one wait for the number of final tracks), what it
    produced, and the entropy of the track-model residuals against that of
    the stored coordinates."""
    ctx.run_batch(dcl, drow, tf.units, device=True, graph=True)
    ctx.sync()
    for _ in range(2):
        ctx.phase2()
        ctx.sync()
    reps = max(5, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.phase2()
        ctx.sync()
    p2_dt = (time.perf_counter() - t0) / reps
    finals, _ = ctx.get_finals(0)
    verts = ctx.get_vertices(0)
    units, _, hits, _ = ctx.get_batch_results()
    nseg = int(units["n_tracks"].sum())
    flags = np.concatenate([ctx.get_flags(0, int(u[3]), int(u[1])) for u in tf.units])
    # entropy: stored (quantised) coordinates of every cluster against the
    # track model (rows steps and residuals of the clusters on tracks, the
    # first cluster of a segment stored as it is plus its three FP32 values)
    q = np.float32(0.01)
    yq_all = np.rint(tf.cl[:, 1] / q).astype(np.int64)
    zq_all = np.rint(tf.cl[:, 2] / q).astype(np.int64)
    h_abs = _entropy_bits(yq_all) + _entropy_bits(zq_all) + _entropy_bits(tf.row)
    res_all, rec_all = [], []
    for u in tf.units:
        rec, res = ctx.get_compressed(0, int(u[3]))
        rec_all.append(rec)
        res_all.append(res)
    rec = np.concatenate(rec_all)
    res = np.concatenate(res_all)
    first = np.zeros(res.shape[0], bool)
    # the first hit of each segment holds zeros: locate them from the segments' hit counts
    seg_nh = np.concatenate([ctx.get_tracks(0, int(u[3]))[0]["n_hits"] for u in tf.units])
    first[np.r_[0, np.cumsum(seg_nh)[:-1]]] = True
    rest = res[~first]
    h_model_hit = _entropy_bits(rest[:, 0]) + _entropy_bits(rest[:, 1]) + _entropy_bits(rest[:, 2])
    n_on = int(res.shape[0])
    n_off = int(tf.n_clusters) - n_on
    bits_abs = h_abs * tf.n_clusters
    bits_model = h_model_hit * (n_on - nseg) + nseg * (h_abs + 96.0) + n_off * h_abs
    out = {
        "workload": "the resident 128-event time frame's accepted tracks (sector segments)",
        "ms": round(p2_dt * 1e3, 4),
        "segments": nseg, "final_tracks": int(finals.shape[0]),
        "merged_segments": int(nseg - finals.shape[0]),
        "refit_failures": int((finals["status"] != 0).sum()),
        "vertices": int(verts.shape[0]), "events_in_frame": int(len(tf.meta["t0_us"])),
        "tracks_with_vertex": int((finals["vertex"] >= 0).sum()),
        "flagged_clusters": {"low_pt": int(((flags & 1) != 0).sum()), "looper_leg": int(((flags & 2) != 0).sum()),
                             "inclined": int(((flags & 4) != 0).sum()), "any": int((flags != 0).sum()),
                             "of": int(tf.n_clusters)},
        "compression": {"bits_per_cluster_stored_coordinates": round(h_abs, 3),
                        "bits_per_track_hit_model": round(h_model_hit, 3),
                        "bits_per_cluster_with_model": round(bits_model / tf.n_clusters, 3),
                        "gain": round(bits_abs / bits_model, 3),
                        "basis": "zeroth-order empirical entropy of the frame's symbols; 0.01 cm steps"},
    }
    log(f"second phase: {out}")
    return out


def bench_minbias64(rx, tpcca, torch, args, log, knobs):
    """64 minimum-bias events (10 to 8000 tracks) as one batch of 2304 units
    in one launch per kernel (graph replay), one and two batches in flight,
    against the same events one launch sequence per event, and the oracle
    on a sample of the units."""
    import tpcgen
    b = tpcgen.minbias_batch(seed=0, n_events=64)
    dcl = torch.from_numpy(b.cl).cuda()
    drow = torch.from_numpy(b.row).cuda()
    torch.cuda.synchronize()
    cx = [tpcca.Context(rx, device=0), tpcca.Context(rx, device=0)]
    for c in cx:
        c.set_tuning(**knobs)
    for _ in range(args.warmup):
        cx[0].run_batch(dcl, drow, b.units, device=True, graph=True)
        cx[0].sync()
    steps = max(args.steps, 10)
    t0 = time.perf_counter()
    for _ in range(steps):
        cx[0].run_batch(dcl, drow, b.units, device=True, graph=True)
        cx[0].sync()
    one_dt = (time.perf_counter() - t0) / steps
    _, ncl, ntr, _ = cx[0].batch_totals()
    for i in range(2 * args.warmup):
        cx[i % 2].run_batch(dcl, drow, b.units, device=True, graph=True)
    for c in cx:
        c.sync()
    t0 = time.perf_counter()
    for i in range(steps):
        cx[i % 2].run_batch(dcl, drow, b.units, device=True, graph=True)
    for c in cx:
        c.sync()
    two_dt = (time.perf_counter() - t0) / steps
    # the same events, one plain launch sequence per event
    pe = cx[0]
    slots = np.unique(b.units[:, 2])

    def per_event_pass():
        for ev in slots:
            pe.reset()
            for u in np.nonzero(b.units[:, 2] == ev)[0]:
                beg, n, slot, sec = (int(v) for v in b.units[u])
                pe.load_sector(slot, sec, dcl[beg:beg + n], drow[beg:beg + n], device=True)
            pe.run_all(int(ev), -1)
            pe.sync()
    per_event_pass()
    t0 = time.perf_counter()
    for _ in range(3):
        per_event_pass()
    pe_dt = (time.perf_counter() - t0) / 3
    for c in cx:
        c.close()
    # the oracle on every 9th unit, 16 threads
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    sample = list(range(0, b.units.shape[0], 9))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        done = sum(ex.map(lambda u: (oracle.run_sector(b.unit(u)[0], b.unit(u)[1], rx, precision=32),
                                     int(b.units[u, 1]))[1], sample))
    or_dt = time.perf_counter() - t0
    out = {"workload": f"64 minimum-bias Pb-Pb events ({int(b.meta['multiplicity'].min())}.."
                       f"{int(b.meta['multiplicity'].max())} tracks), {b.units.shape[0]} units, {ncl} clusters, "
                       "one launch per kernel (graph replay), device-resident",
           "units": int(b.units.shape[0]), "clusters": int(ncl), "tracks": int(ntr),
           "value": round(ncl / two_dt, 1), "unit": "clusters/s", "ms": round(two_dt * 1e3, 4), "in_flight": 2,
           "one_in_flight": {"value": round(ncl / one_dt, 1), "ms": round(one_dt * 1e3, 4)},
           "per_event": {"value": round(ncl / pe_dt, 1), "ms_for_64_events": round(pe_dt * 1e3, 3),
                         "basis": "the same 64 events, one launch sequence per event"},
           "batched_over_per_event": round(pe_dt / two_dt, 3),
           "oracle": {"value": round(done / or_dt, 1), "unit": "clusters/s", "cores": cores,
                      "sample": f"every 9th unit ({len(sample)} units, {done} clusters), FP32 oracle, "
                                f"{or_dt:.1f} s"}}
    log(f"64 minimum-bias events: {out}")
    return out


def cpu_baseline(ev, rx, seconds):
    """The plain oracle, as it stands, over the sectors of the central event
    on a thread pool of the host's cores until `seconds` of wall time."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    cores = max(1, min(16, os.cpu_count() or 1))
    units = list(range(ev.units.shape[0]))
    done_cl = 0
    t0 = time.perf_counter()
    rounds = 0
    with ThreadPoolExecutor(cores) as ex:
        while True:
            def run(u):
                cl, row, _, _, _ = ev.unit(u)
                oracle.run_sector(cl, row, rx, precision=32)
                return cl.shape[0]
            done_cl += sum(ex.map(run, units))
            rounds += 1
            if time.perf_counter() - t0 >= seconds:
                break
    dt = time.perf_counter() - t0
    # one thread, the 36 sectors in turn
    t1 = time.perf_counter()
    near, decisions = 0, 0
    for u in units:
        cl, row, _, _, _ = ev.unit(u)
        r = oracle.run_sector(cl, row, rx, precision=32)
        near += r.near_ties
        decisions += r.decisions
    st_dt = time.perf_counter() - t1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(done_cl / dt, 1), "unit": "clusters/s", "cores": cores, "kind": "oracle",
            "single_thread": round(ev.n_clusters / st_dt, 1), "nproc": os.cpu_count(), "cpu_model": model,
            "near_ties": {"decisions": int(decisions), "margin_below_1e-6": int(near),
                          "note": "the oracle's count on this event; the GPU path needed no exception"},
            "sample": f"{rounds} pass(es) over the 36 sectors of one central Pb-Pb event "
                      f"({ev.n_clusters} clusters), FP32 oracle, one sector per thread, {dt:.1f} s wall"}


if __name__ == "__main__":
    main()
