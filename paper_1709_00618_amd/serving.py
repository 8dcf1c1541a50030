"""Python driver of the continuous-batching time-frame server in libtpcca.so.

``Server`` marshals time frames (numpy or pinned torch host tensors) into
``tpcca_server_submit`` and collects results; the queueing, admission by
device-memory budget, packing of sector units into lane batches and the GPU
work all happen in the C++/HIP library.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import tpcca


class Frame:
    """A time frame in host memory plus its output buffers."""

    def __init__(self, cl, row, units, pinned=False):
        import torch

        units = np.asarray(units, np.int64)
        self.n_units = units.shape[0]
        self.sector = np.ascontiguousarray(units[:, 3], np.int32)
        self.begin = np.ascontiguousarray(units[:, 0], np.int64)
        self.n = np.ascontiguousarray(units[:, 1], np.int32)
        self.n_clusters = int(self.n.sum())
        if pinned:
            self.cl_t = torch.empty((cl.shape[0], 4), dtype=torch.float32, pin_memory=True)
            self.cl_t.numpy()[:] = cl
            self.row_t = torch.empty(row.shape[0], dtype=torch.uint8, pin_memory=True)
            self.row_t.numpy()[:] = row
            self.cl_ptr, self.row_ptr = self.cl_t.data_ptr(), self.row_t.data_ptr()
        else:
            self.cl_np = np.ascontiguousarray(cl, np.float32)
            self.row_np = np.ascontiguousarray(row, np.uint8)
            self.cl_ptr, self.row_ptr = self.cl_np.ctypes.data, self.row_np.ctypes.data


class Outputs:
    """Result buffers of one request.  pinned=True places them in page-locked
    host memory (torch), so that the server's device-to-host copies run
    asynchronously at link speed instead of being staged through a bounce
    buffer while the lane's thread waits."""

    def __init__(self, max_clusters, max_units, min_track_hits=10, pinned=False):
        self._keep = []

        def buf(n, dtype):
            dtype = np.dtype(dtype)
            if not pinned:
                return np.zeros(n, dtype)
            import torch

            t = torch.zeros(n * dtype.itemsize, dtype=torch.uint8, pin_memory=True)
            self._keep.append(t)
            return t.numpy().view(dtype)

        self.tracks = buf(max_clusters // min_track_hits + max_units + 1, tpcca.TRACK_DTYPE)
        self.hits = buf(max(1, max_clusters), np.int32)
        self.assignment = buf(max(1, max_clusters), np.int32)
        self.units = np.zeros(max(1, max_units), tpcca.UNIT_RESULT_DTYPE)


class Server:
    def __init__(self, row_x, params=None, device=0, budget_bytes=64 << 30, n_streams=3, max_queue=64):
        L = tpcca.lib()
        self.row_x = np.ascontiguousarray(row_x, np.float32)
        self.params = params or tpcca.params_default(n_rows=self.row_x.shape[0])
        geo = tpcca.Geometry(36, self.row_x.shape[0], ctypes.c_void_p(self.row_x.ctypes.data))
        h = ctypes.c_void_p()
        st = L.tpcca_server_create(ctypes.byref(geo), ctypes.byref(self.params), device, budget_bytes,
                                   n_streams, max_queue, ctypes.byref(h))
        if st != tpcca.OK:
            raise tpcca.TpccaError(st, "tpcca_server_create")
        self.h = h
        self._keep = {}

    def submit(self, frame: Frame, out: Outputs, arrival_s: float = 0.0) -> int:
        tf = tpcca.Timeframe(frame.n_units, frame.sector.ctypes.data, frame.begin.ctypes.data,
                             frame.n.ctypes.data, frame.cl_ptr, frame.row_ptr, out.tracks.ctypes.data,
                             out.tracks.shape[0], out.hits.ctypes.data, out.hits.shape[0],
                             out.assignment.ctypes.data, out.units.ctypes.data, arrival_s)
        rid = ctypes.c_uint64()
        st = tpcca.lib().tpcca_server_submit(self.h, ctypes.byref(tf), ctypes.byref(rid))
        if st != tpcca.OK:
            raise tpcca.TpccaError(st, "tpcca_server_submit")
        self._keep[rid.value] = (frame, out)
        return rid.value

    def wait(self, rid: int, timeout_s: float = 600.0) -> tpcca.Result:
        r = tpcca.Result()
        st = tpcca.lib().tpcca_server_wait(self.h, rid, timeout_s, ctypes.byref(r))
        if st != tpcca.OK:
            raise tpcca.TpccaError(st, "tpcca_server_wait")
        return r

    def poll(self, rid: int) -> tpcca.Result:
        r = tpcca.Result()
        st = tpcca.lib().tpcca_server_poll(self.h, rid, ctypes.byref(r))
        if st != tpcca.OK:
            raise tpcca.TpccaError(st, "tpcca_server_poll")
        return r

    def release(self, rid: int):
        tpcca.lib().tpcca_server_release(self.h, rid)
        self._keep.pop(rid, None)

    def stats(self) -> tpcca.Stats:
        s = tpcca.Stats()
        tpcca.lib().tpcca_server_stats(self.h, ctypes.byref(s))
        return s

    def reset_stats(self):
        tpcca.lib().tpcca_server_reset_stats(self.h)

    def set_tuning(self, **kw):
        """Launch schedule of every lane's context from its next batch on."""
        t = tpcca.Tuning()
        tpcca.lib().tpcca_tuning_default(ctypes.byref(t))
        for k, v in kw.items():
            setattr(t, k, int(v))
        st = tpcca.lib().tpcca_server_set_tuning(self.h, ctypes.byref(t))
        if st != tpcca.OK:
            raise tpcca.TpccaError(st, "tpcca_server_set_tuning")

    def last_error(self) -> str:
        t = tpcca.lib().tpcca_server_last_error(self.h)
        return t.decode(errors="replace") if t else ""

    def close(self):
        if getattr(self, "h", None):
            tpcca.lib().tpcca_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def unit_results(frame: Frame, out: Outputs):
    """Per unit: (tracks, hits, assignment) views of a completed request."""
    res = []
    for u in range(frame.n_units):
        ur = out.units[u]
        t0, nt = int(ur["track_begin"]), int(ur["n_tracks"])
        h0, nh = int(ur["hit_begin"]), int(ur["n_track_hits"])
        c0, n = int(ur["cluster_begin"]), int(frame.n[u])
        res.append((out.tracks[t0:t0 + nt], out.hits[h0:h0 + nh], out.assignment[c0:c0 + n]))
    return res


def _run_stream(srv: Server, frames, outs, order, arrivals_s, log=None):
    """Submit frames[order[i]] at arrivals_s[i] (seconds from now); recycle
    output buffers as requests complete.  Returns wall time and clusters."""
    free = list(range(len(outs)))
    inflight = []  # (rid, out index)
    t0 = tpcca.now()
    total = 0
    for i, k in enumerate(order):
        target = t0 + arrivals_s[i]
        while True:
            now = tpcca.now()
            if now >= target:
                break
            time.sleep(min(0.002, target - now))
        while not free:
            rid, oi = inflight.pop(0)
            _finish(srv, rid)
            free.append(oi)
        oi = free.pop()
        rid = srv.submit(frames[k], outs[oi], arrival_s=target)
        inflight.append((rid, oi))
        total += frames[k].n_clusters
    for rid, oi in inflight:
        _finish(srv, rid)
    return tpcca.now() - t0, total


def _finish(srv, rid):
    r = srv.wait(rid)
    srv.release(rid)
    if r.status != tpcca.OK:
        raise tpcca.TpccaError(r.status, f"served request {rid}", srv.last_error())


def bench_served(row_x, n_tf=48, ring=8, n_streams=3, seed=0, log=print):
    """Served time frames: sizes log-uniform in [8, 256] events, Poisson
    arrivals equivalent to 50 kHz.  A ring of `ring` distinct frames (built
    from a pool of minimum-bias events shifted to Poisson arrival times) is
    replayed in the arrival sequence.  Reports the closed-loop capacity, the
    nominal-rate run and runs at 0.5 / 0.8 / 0.95 of capacity."""
    import tpcgen

    t = time.time()
    pool = tpcgen.minbias_pool(seed=seed, n=64)
    sizes, arrivals_us, mean_size = tpcgen.served_stream(seed=seed, n_tf=n_tf)
    frames = []
    for i in range(min(ring, n_tf)):
        tf = tpcgen.timeframe(seed=seed, n_events=int(sizes[i]), tf_index=i, event_pool=pool,
                              stream=tpcgen.STREAM_SERVED)
        frames.append(Frame(tf.cl, tf.row, tf.units, pinned=True))
    del pool
    order = [i % len(frames) for i in range(n_tf)]
    maxc = max(f.n_clusters for f in frames)
    outs = [Outputs(maxc, 36, pinned=True) for _ in range(8)]  # at most 8 frames outstanding
    log(f"served: {len(frames)} distinct frames, {[f.n_clusters for f in frames]} clusters, "
        f"built in {time.time() - t:.1f} s")
    res = {"workload": f"time frames of {tpcgen.N_SECTORS} sector units, 8-256 events log-uniform "
                       f"(ring of {len(frames)} distinct frames replayed), host-resident pinned inputs and outputs",
           "n_streams": n_streams, "tfs_per_level": n_tf, "outputs": "pinned host", "max_outstanding": len(outs),
           "warmup_tfs": len(frames) + min(n_tf, 200)}
    with Server(row_x, n_streams=n_streams) as srv:
        # the lanes keep two or more frames in flight: the schedule tuned for
        # that on a time frame of the median served size, if cached
        from . import autotune
        med = sorted(f.n_clusters for f in frames)[len(frames) // 2]
        entry = autotune.lookup(med, tpcgen.N_SECTORS)
        if entry:
            srv.set_tuning(**entry["knobs"])
            res["schedule"] = entry["knobs"]
        # warm-up: every frame once, then a closed-loop pass over the ring
        # (the lanes' buffers grow to the batches they form and their graphs
        # are captured; the measured runs start in the steady state)
        _run_stream(srv, frames, outs, list(range(len(frames))), [0.0] * len(frames))
        n_warm = min(n_tf, 200)
        _run_stream(srv, frames, outs, [i % len(frames) for i in range(n_warm)], [0.0] * n_warm)
        srv.reset_stats()
        wall, tot = _run_stream(srv, frames, outs, order, [0.0] * n_tf)
        st = srv.stats()
        cap = tot / wall
        cap_tf = n_tf / wall
        res["capacity"] = {"clusters_per_s": round(cap, 1), "tf_per_s": round(cap_tf, 2),
                           "p50_ms": round(st.p50_ms, 3), "p99_ms": round(st.p99_ms, 3), "batches": st.batches_run}
        log(f"served capacity: {cap / 1e9:.3f} G clusters/s, {cap_tf:.1f} TF/s")
        levels = []
        arr_s = np.asarray(arrivals_us) * 1e-6
        nominal_rate = n_tf / arr_s[-1] if arr_s[-1] > 0 else float("inf")
        for name, rho in (("nominal_50kHz", None), ("rho_0.5", 0.5), ("rho_0.8", 0.8), ("rho_0.95", 0.95)):
            a = arr_s if rho is None else arr_s * (nominal_rate / (rho * cap_tf))
            srv.reset_stats()
            wall, tot = _run_stream(srv, frames, outs, order, list(a))
            st = srv.stats()
            lv = {"level": name, "offered_tf_per_s": round(n_tf / a[-1], 2) if a[-1] > 0 else None,
                  "sustained_clusters_per_s": round(tot / wall, 1), "p50_ms": round(st.p50_ms, 3),
                  "p99_ms": round(st.p99_ms, 3), "mean_ms": round(st.mean_ms, 3)}
            levels.append(lv)
            log(f"served {name}: {lv}")
        res["levels"] = levels
    return res
