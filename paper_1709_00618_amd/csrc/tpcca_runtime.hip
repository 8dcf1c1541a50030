// Host runtime of the gfx950 sector tracker: contexts, device arenas, the
// stage calls of the C ABI and the batched (graph-replayed) path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "tpcca.h"
#include "tpcca_internal.h"
#include "tpcca_kernels.h"
#include "tpcca_phase2.h"
#include "tpcca_runtime.h"

using namespace tpcca;

namespace {

enum UnitState { kLoaded = 1, kLinked = 2, kCleaned = 3, kTracklets = 4, kSelected = 5 };

struct UnitHost {
  int32_t slot, sector, n;
  int32_t state;
  int32_t run;
};

int64_t bins_cap_of(int64_t n, int hpb, int R) { return n / hpb + 2 * (int64_t)(R + 1) + 1; }
int64_t trk_cap_of(int64_t n, int min_chain) { return n / std::max(1, min_chain) + 1; }
int64_t tile_cap_of(int64_t n, int R, int tile) { return n / tile + R + 2; }

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct tpcca_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, allocated = 0;
  tpcca_params_t params;
  ParamsDev P;
  int R = 0;
  int n_sectors = 36;
  std::vector<float> row_x;

  std::vector<UnitDev> units;
  std::vector<UnitHost> uh;
  std::vector<Chunk> chunks;
  std::vector<int32_t> unit_chunk0;  // first chunk of each unit
  std::vector<RunHost> runs;
  std::map<std::pair<int, int>, int> index;
  int64_t n_total = 0, bins_total = 0, trk_total = 0, tiles_total = 0, in_used = 0;
  bool tables_dirty = true;
  std::vector<int> pending_runs;  // runs launched since the last sync

  // device buffers
  DevBuf row_x_d, units_d, chunks_d, runs_d, rowtab, row_cnt, row_fill, chunk_hist, rtmp, zmm, binbeg, yz, sid, up,
      dn, upc, dnc, flag, starts, tiles, sval, tofg, kf_order, kf_tmp, band_tmp, srow, cinfo, trk_start, trk_unit, unit_tbegin, trk, trk_hits, owner, accv, wonmask, accx,
      tracks, hits_out, assign, unit_res, scan_tmp, zo_tmp, zo_cnt, kf_chunks, in_cl, in_row;
  Bufs B{};

  // graph replay of the batch path: the graphs captured for the last few
  // launch-capacity buckets, so that batches of recurring sizes (a server
  // lane's mix of frames) replay without a new capture
  struct GraphEntry {
    hipGraphExec_t exec[6] = {};  // whole sequence, or the six timed segments
    RunHost cap{};                // the capacities the graph was captured for
    int gen = -1;                 // buffer generation its kernel arguments belong to
    bool timing = false;          // holds the stage events
    uint64_t used = 0;            // last replay (least recently used is replaced)
  };
  static constexpr int kGraphCache = 8;
  GraphEntry graphs[kGraphCache];
  uint64_t graph_clock = 0;
  int generation = 0;  // bumped when buffers move or launch shapes change

  bool timing = false;
  hipEvent_t ev[7] = {};
  float stage_ms[6] = {};
  bool have_times = false;
  bool capturing = false;       // a graph capture is in progress
  int64_t graph_fallbacks = 0;  // batches run without a graph after a failed capture

  std::string last_error;

  // second phase (Sec. 2 merging and refit, Sec. 5 vertices, Sec. 3
  // compression and rejection)
  tpcca_phase2_params_t p2params{};
  DevBuf p2units, p2seg_begin, p2seg_unit, p2seg_nh, p2seg_hb, p2seg_fpos, p2seg_rows, p2seg_zin, p2seg_zout, p2seg_out,
      p2zmm, p2unit_nz, p2unit_bbase, p2bin_cnt, p2bin_beg, p2bin_seg, p2bin_rz, p2hrec, p2seg_flag, p2pairs, p2best_b, p2best_a, p2next, p2prev, p2final_of, p2final_start,
      p2final_nhits, p2final_hbeg, p2finals, p2final_hits, p2vkey0, p2vkey1, p2vval0, p2vval1, p2gstart,
      p2group_pos, p2vertices, p2slot_first, p2slot_vbeg, p2slot_vend, p2flags, p2rec, p2res, p2scan, p2cnt,
      p2sort_tmp, p2order, p2lenh;
  P2Bufs P2{};
  bool p2_done = false;
  P2Counts p2c{};
  std::vector<int32_t> p2_slot_value;  // compact slot index -> slot
};

// --------------------------------------------------------------- errors ---
// Destroys one cached batch graph.
static void drop_graph(tpcca_ctx::GraphEntry &e) {
  for (auto &g : e.exec) {
    if (g) hipGraphExecDestroy(g);
    g = nullptr;
  }
  e.gen = -1;
}

// Destroys the captured batch graphs; the next graph run captures again.
static void drop_graphs(tpcca_ctx *c) {
  for (auto &e : c->graphs) drop_graph(e);
}

static bool same_capacities(const RunHost &a, const RunHost &b) {
  return a.u1 == b.u1 && a.c1 == b.c1 && a.cl1 == b.cl1 && a.bin1 == b.bin1 && a.trk_cap == b.trk_cap &&
         a.tile1 == b.tile1 && a.dense == b.dense;
}

static int dev_err(tpcca_ctx *c, hipError_t e, const char *what) {
  if (c) {
    c->last_error = std::string(what) + ": " + hipGetErrorString(e);
  }
  return TPCCA_EDEVICE;
}
#define RCCHK(call)                  \
  do {                               \
    int rc_ = (call);                \
    if (rc_ != TPCCA_OK) return rc_; \
  } while (0)

#define HIPCHK(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return dev_err((ctx), e_, #call); \
  } while (0)

// Copy in stream order on the context's own (non-blocking) stream and wait
// for it: no library call touches the legacy stream, which other threads'
// graph captures forbid.
static int copy_sync(tpcca_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return TPCCA_OK;
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TPCCA_OK;
}

// Grow a device buffer to at least `bytes` (x1.25 headroom), preserving the
// first `keep` bytes.  Budget-checked.
static int ensure(tpcca_ctx *c, DevBuf &b, size_t bytes, size_t keep) {
  if (bytes <= b.bytes) return TPCCA_OK;
  size_t nb = std::max(bytes, b.bytes + b.bytes / 4);
  nb = (nb + 255) & ~(size_t)255;
  if (c->allocated - b.bytes + nb > c->budget) {
    nb = bytes;
    if (c->allocated - b.bytes + nb > c->budget) {
      c->last_error = "device budget exceeded";
      return TPCCA_ENOMEM;
    }
  }
  // allocation and release may synchronise the device: never during another
  // context's graph capture
  std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->last_error = std::string("hipMalloc: ") + hipGetErrorString(e);
    return TPCCA_ENOMEM;
  }
  if (b.p && keep) {
    e = hipMemcpyAsync(p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return dev_err(c, e, "hipMemcpyAsync(grow)");
  }
  if (b.p) {
    hipStreamSynchronize(c->stream);
    hipFree(b.p);
  }
  c->allocated = c->allocated - b.bytes + nb;
  b.p = p;
  b.bytes = nb;
  c->generation++;
  return TPCCA_OK;
}

template <typename T>
static T *ptr(DevBuf &b) {
  return static_cast<T *>(b.p);
}

static void refresh_bufs(tpcca_ctx *c);

// Every work and output buffer of a run: (member of tpcca_ctx, field of
// Bufs, element type, element count, elements kept when it grows).  The
// counts use R (rows), N (clusters), U (units), NB (bin-begin entries),
// T (tracklet slots), NC (chunks), NTILE (row tiles) and NSCAN (scan tiles);
// the kept counts keepN, keepU, keepB, keepT and keepTiles.  The tables the
// host writes (units, chunks, runs) are sized separately.
#define TPCCA_WORK_BUFFERS(X)                                                   \
  X(rowtab, rowtab, RowTab, U * (R + 1), keepU * (R + 1))                        \
  X(row_cnt, row_cnt, int32_t, U * (R + 1), keepU * (R + 1))                     \
  X(row_fill, row_fill, int32_t, U * (R + 1), 0)                                 \
  X(chunk_hist, chunk_hist, int32_t, NC * (R + 1), 0)                            \
  X(rtmp, rtmp, int4, N, 0)                                                      \
  X(zmm, zmm, int32_t, 2 * U, 2 * keepU)                                         \
  X(binbeg, binbeg, int32_t, NB, keepB)                                          \
  X(yz, yz, float2, N, keepN)                                                    \
  X(sid, sid, int32_t, N, keepN)                                                 \
  X(srow, srow, uint8_t, N, keepN)                                               \
  X(cinfo, cinfo, int2, N, keepN)                                                \
  X(up, up, int32_t, N, keepN)                                                   \
  X(dn, dn, int32_t, N, keepN)                                                   \
  X(upc, upc, int32_t, N, keepN)                                                 \
  X(dnc, dnc, int32_t, N, keepN)                                                 \
  X(flag, flag, int32_t, N, keepN)                                               \
  X(starts, starts, int2, N, 0)                                                  \
  X(tiles, tiles, int4, NTILE, keepTiles)                                        \
  X(owner, owner, unsigned long long, N, keepN)                                  \
  X(trk_start, trk_start, int32_t, T, keepT)                                     \
  X(kf_order, kf_order, int32_t, T, keepT)                                       \
  X(kf_tmp, kf_tmp, int32_t, T, 0)                                               \
  X(band_tmp, band_tmp, int32_t, 3 * U * (R + 1), 0)                             \
  X(sval, sval, uint8_t, N, keepN)                                               \
  X(tofg, tofg, int32_t, N, keepN)                                               \
  X(trk_unit, trk_unit, int32_t, T, keepT)                                       \
  X(unit_tbegin, unit_tbegin, int32_t, U + 1, keepU)                             \
  X(trk, trk, tpcca_tracklet_t, T, keepT)                                        \
  X(trk_hits, trk_hits, int32_t, T * (size_t)slot_stride(R), keepT * (size_t)slot_stride(R)) \
  X(accv, accv, unsigned long long, T + 1, 0)                                    \
  X(wonmask, wonmask, unsigned long long, 4 * T, 0)                              \
  X(accx, accx, unsigned long long, T + 1, 0)                                    \
  X(scan_tmp, scan_tmp, int64_t, NSCAN, 0)                                      \
  X(zo_tmp, zo_tmp, int2, T, 0)                                                  \
  X(zo_cnt, zo_cnt, int64_t, T / 16 + 2 * U + 2, 0)                              \
  X(kf_chunks, kf_chunks, int4, T / 64 + U + 2, 0)
#define TPCCA_OUTPUT_BUFFERS(X)                                                 \
  X(tracks, tracks, tpcca_track_t, T, keepT)                                     \
  X(hits_out, hits_out, int32_t, N, keepN)                                       \
  X(assign, assign, int32_t, N, keepN)                                           \
  X(unit_res, unit_res, tpcca_unit_result_t, U, keepU)

// The count variables of the buffer table for the given capacities.
#define TPCCA_BUFFER_COUNTS(R_, n_cl, n_units, n_bins, n_trk, n_chunks)                          \
  const int R = (R_);                                                                          \
  const size_t N = (size_t)std::max<int64_t>((n_cl), 1), U = (size_t)std::max<int64_t>((n_units), 1); \
  const size_t NB = (size_t)std::max<int64_t>((n_bins), 1), T = (size_t)std::max<int64_t>((n_trk), 1); \
  const size_t NC = (size_t)std::max<int64_t>((n_chunks), 1);                                  \
  const size_t NTILE = N / kTileMin + U * (R + 2) + 1;                                            \
  const size_t NSCAN = std::max(NB / kScanTile + 2, std::max(2 * NC + 2, T / kScanTile + 2));

static void refresh_bufs(tpcca_ctx *c) {
  Bufs &B = c->B;
  B.row_x = ptr<float>(c->row_x_d);
  B.units = ptr<UnitDev>(c->units_d);
  B.chunks = ptr<Chunk>(c->chunks_d);
  B.runs = ptr<RunDev>(c->runs_d);
#define REF(buf, field, type, count, keepc) B.field = ptr<type>(c->buf);
  TPCCA_WORK_BUFFERS(REF)
  TPCCA_OUTPUT_BUFFERS(REF)
#undef REF
  B.ids_tmp = nullptr;
}

// Size every work buffer for the given capacities (at least the loaded units).
static int ensure_work(tpcca_ctx *c, int64_t n_cl, int64_t n_units, int64_t n_bins, int64_t n_trk,
                       int64_t n_chunks) {
  TPCCA_BUFFER_COUNTS(c->R, n_cl, n_units, n_bins, n_trk, n_chunks)
  const size_t keepN = (size_t)c->n_total, keepU = c->units.size(), keepB = (size_t)c->bins_total,
               keepT = (size_t)c->trk_total, keepTiles = (size_t)c->tiles_total;
  int rc;
#define ENS(buf, field, type, count, keepc)                                                    \
  if ((rc = ensure(c, c->buf, (size_t)(count) * sizeof(type), (size_t)(keepc) * sizeof(type))) != TPCCA_OK) \
    return rc;
  ENS(units_d, units, UnitDev, U, 0)
  ENS(chunks_d, chunks, Chunk, NC, 0)
  ENS(runs_d, runs, RunDev, U + 1, c->runs.size())
  TPCCA_WORK_BUFFERS(ENS)
  TPCCA_OUTPUT_BUFFERS(ENS)
#undef ENS
  refresh_bufs(c);
  return TPCCA_OK;
}

static int upload_tables(tpcca_ctx *c) {
  if (!c->tables_dirty) return TPCCA_OK;
  if (!c->units.empty())
    HIPCHK(c, hipMemcpyAsync(c->units_d.p, c->units.data(), c->units.size() * sizeof(UnitDev),
                             hipMemcpyHostToDevice, c->stream));
  if (!c->chunks.empty())
    HIPCHK(c, hipMemcpyAsync(c->chunks_d.p, c->chunks.data(), c->chunks.size() * sizeof(Chunk),
                             hipMemcpyHostToDevice, c->stream));
  // host vectors may be modified by later loads before the copy runs
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->tables_dirty = false;
  return TPCCA_OK;
}

static int write_run(tpcca_ctx *c, int run) {
  const RunHost &h = c->runs[run];
  RunDev d{};
  d.u0 = h.u0;
  d.u1 = h.u1;
  d.c0 = h.c0;
  d.c1 = h.c1;
  d.cl0 = h.cl0;
  d.cl1 = h.cl1;
  d.bin0 = h.bin0;
  d.bin1 = h.bin1;
  d.trk0 = h.trk0;
  d.trk_cap = h.trk_cap;
  d.tile0 = h.tile0;
  d.tile1 = h.tile1;
  // pageable source: the copy completes before return
  RCCHK(copy_sync(c, ptr<RunDev>(c->runs_d) + run, &d, sizeof(d), hipMemcpyHostToDevice));
  return TPCCA_OK;
}

static RunHost make_run(tpcca_ctx *c, int u0, int u1) {
  RunHost h{};
  h.u0 = u0;
  h.u1 = u1;
  h.c0 = c->unit_chunk0[u0];
  h.c1 = c->unit_chunk0[u1];
  h.cl0 = c->units[u0].cl_begin;
  const UnitDev &L = c->units[u1 - 1];
  h.cl1 = L.cl_begin + L.n;
  h.bin0 = c->units[u0].bin_base;
  h.bin1 = L.bin_base + bins_cap_of(L.n, c->P.hits_per_bin, c->R);
  h.trk0 = c->units[u0].trk_base;
  h.trk_cap = (int32_t)(L.trk_base + trk_cap_of(L.n, c->P.min_chain) - h.trk0);
  h.tile0 = c->units[u0].tile_base;
  h.tile1 = (int32_t)(L.tile_base + tile_cap_of(L.n, c->R, link_tile_of(c->P)));
  h.dense = (int64_t)(h.cl1 - h.cl0) / ((int64_t)(u1 - u0) * (c->R + 1)) >= 1024 ? 1 : 0;
  return h;
}

// Units matching (slot, sector), grouped into maximal index ranges.
static std::vector<std::pair<int, int>> select_ranges(tpcca_ctx *c, int slot, int sector) {
  std::vector<std::pair<int, int>> out;
  int a = -1;
  for (int u = 0; u <= (int)c->uh.size(); ++u) {
    bool m = u < (int)c->uh.size() && (slot < 0 || c->uh[u].slot == slot) &&
             (sector < 0 || c->uh[u].sector == sector);
    if (m && a < 0) a = u;
    if (!m && a >= 0) {
      out.push_back({a, u});
      a = -1;
    }
  }
  return out;
}

// Stage boundary k (events 0..6 bracket the six timed segments).
static void record_event(tpcca_ctx *c, int k) {
  if (c->timing && !c->capturing) (void)hipEventRecord(c->ev[k], c->stream);
}

// The six timed segments: 0 grid, 1 links, 2 clean, 3 chains, 4 fit,
// 5 selection.  Stage calls map to segments 1 -> {0, 1}, 2 -> {2},
// 3 -> {3, 4}, 4 -> {5}.
static hipError_t launch_segment(tpcca_ctx *c, int run, const RunHost &h, int seg) {
  hipStream_t s = c->stream;
  switch (seg) {
    case 0: return launch_grid(c->B, c->P, run, h, s);
    case 1: return launch_links(c->B, c->P, run, h, s);
    case 2: return launch_clean(c->B, c->P, run, h, s);
    case 3: return launch_chains(c->B, c->P, run, h, s);
    case 4: return launch_kf(c->B, c->P, run, h, s);
    default: return launch_select(c->B, c->P, run, h, s);
  }
}
static const int kSegFirst[5] = {0, 0, 2, 3, 5};  // first segment of stage 1..4
static const int kSegEnd[5] = {0, 2, 3, 5, 6};    // one past its last

// Launch stages [first, last] (1 = grid + links, 2 = clean, 3 = tracklets,
// 4 = selection) for one run.
static int launch_stages(tpcca_ctx *c, int run, const RunHost &h, int first, int last) {
  hipError_t e = hipSuccess;
  if (first == 1) record_event(c, 0);
  for (int seg = kSegFirst[first]; seg < kSegEnd[last] && e == hipSuccess; ++seg) {
    e = launch_segment(c, run, h, seg);
    record_event(c, seg + 1);
  }
  if (e != hipSuccess) return dev_err(c, e, "kernel launch");
  if (c->timing && first == 1 && last == 4) c->have_times = true;
  return TPCCA_OK;
}

static int stage_call(tpcca_ctx *c, int slot, int sector, int stage) {
  if (!c) return TPCCA_EINVAL;
  auto ranges = select_ranges(c, slot, sector);
  if (ranges.empty()) return TPCCA_ESTATE;
  if (stage == 1) {
    for (auto &r : ranges)
      for (int u = r.first; u < r.second; ++u)
        if (c->uh[u].state != kLoaded) return TPCCA_ESTATE;
    int rc = ensure_work(c, c->n_total, (int64_t)c->units.size(), c->bins_total, c->trk_total,
                         (int64_t)c->chunks.size());
    if (rc != TPCCA_OK) return rc;
    if ((rc = upload_tables(c)) != TPCCA_OK) return rc;
    for (auto &r : ranges) {
      const int run = (int)c->runs.size();
      c->runs.push_back(make_run(c, r.first, r.second));
      if ((rc = ensure_work(c, c->n_total, (int64_t)c->units.size(), c->bins_total, c->trk_total,
                            (int64_t)c->chunks.size())) != TPCCA_OK)
        return rc;
      if ((rc = write_run(c, run)) != TPCCA_OK) return rc;
      if ((rc = launch_stages(c, run, c->runs[run], 1, 1)) != TPCCA_OK) return rc;
      for (int u = r.first; u < r.second; ++u) {
        c->uh[u].state = kLinked;
        c->uh[u].run = run;
      }
      c->pending_runs.push_back(run);
    }
    return TPCCA_OK;
  }
  // later stages act on whole runs
  std::vector<int> runs;
  for (auto &r : ranges)
    for (int u = r.first; u < r.second; ++u)
      if (std::find(runs.begin(), runs.end(), c->uh[u].run) == runs.end()) runs.push_back(c->uh[u].run);
  for (int run : runs) {
    if (run < 0) return TPCCA_ESTATE;
    const RunHost &h = c->runs[run];
    for (int u = h.u0; u < h.u1; ++u)
      if (c->uh[u].state != stage) return TPCCA_ESTATE;
  }
  for (int run : runs) {
    const RunHost &h = c->runs[run];
    int rc = launch_stages(c, run, h, stage, stage);
    if (rc != TPCCA_OK) return rc;
    for (int u = h.u0; u < h.u1; ++u) c->uh[u].state = stage + 1;
  }
  return TPCCA_OK;
}

static int check_errors(tpcca_ctx *c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int rc = TPCCA_OK;
  for (int run : c->pending_runs) {
    RunDev d;
    RCCHK(copy_sync(c, &d, ptr<RunDev>(c->runs_d) + run, sizeof(d), hipMemcpyDeviceToHost));
    if (d.err & 2) {
      c->last_error = "internal error: inconsistent fit order";
      rc = TPCCA_EDEVICE;
    } else if (d.err) {
      c->last_error = "invalid cluster (row out of range, non-finite value, or x off its row)";
      rc = TPCCA_EINVAL;
    }
  }
  c->pending_runs.clear();
  if (c->timing && c->have_times) {
    for (int k = 0; k < 6; ++k) hipEventElapsedTime(&c->stage_ms[k], c->ev[k], c->ev[k + 1]);
  }
  return rc;
}

static int find_unit(tpcca_ctx *c, int slot, int sector) {
  auto it = c->index.find({slot, sector});
  return it == c->index.end() ? -1 : it->second;
}

static int load_unit(tpcca_ctx *c, int32_t slot, int32_t sector, const tpcca_cluster_t *cl,
                     const uint8_t *row, int32_t n, int32_t flags, bool defer_copy) {
  if (!c || n < 0 || slot < 0 || sector < 0 || sector >= c->n_sectors) return TPCCA_EINVAL;
  if (n > 0 && (!cl || !row)) return TPCCA_EINVAL;
  if (n > 0xFFFFFF) {
    c->last_error = "a unit holds at most 2^24 - 1 clusters";
    return TPCCA_EINVAL;
  }
  if (c->index.count({slot, sector})) return TPCCA_ESTATE;
  if (c->n_total + n > (int64_t)0x7FFFFFFF) return TPCCA_ENOMEM;
  // the grid's bin table is addressed with 32-bit indices
  if (c->bins_total + bins_cap_of(n, c->P.hits_per_bin, c->R) > (int64_t)0x7FFFFFFF) return TPCCA_ENOMEM;
  UnitDev U{};
  U.n = n;
  U.slot = slot;
  U.sector = sector;
  U.cl_begin = (int32_t)c->n_total;
  U.bin_base = c->bins_total;
  U.trk_base = (int32_t)c->trk_total;
  U.tile_base = (int32_t)c->tiles_total;
  if ((flags & 1) == TPCCA_MEM_DEVICE) {
    U.cl = reinterpret_cast<const float4 *>(cl);
    U.row = row;
  } else if (n > 0) {
    float4 *old_cl = ptr<float4>(c->in_cl);
    uint8_t *old_row = ptr<uint8_t>(c->in_row);
    int rc = ensure(c, c->in_cl, (size_t)(c->in_used + n) * sizeof(float4),
                    (size_t)c->in_used * sizeof(float4));
    if (rc != TPCCA_OK) return rc;
    rc = ensure(c, c->in_row, (size_t)(c->in_used + n), (size_t)c->in_used);
    if (rc != TPCCA_OK) return rc;
    if (old_cl && old_cl != ptr<float4>(c->in_cl)) {
      // staged units recorded addresses in the old buffers: rebase them
      for (auto &V : c->units) {
        if (V.cl >= old_cl && V.cl < old_cl + c->in_used) {
          V.row = ptr<uint8_t>(c->in_row) + (V.row - old_row);
          V.cl = ptr<float4>(c->in_cl) + (V.cl - old_cl);
        }
      }
      c->tables_dirty = true;
    }
    float4 *dcl = ptr<float4>(c->in_cl) + c->in_used;
    uint8_t *drow = ptr<uint8_t>(c->in_row) + c->in_used;
    if (!defer_copy) {
      HIPCHK(c, hipMemcpyAsync(dcl, cl, (size_t)n * sizeof(float4), hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(drow, row, (size_t)n, hipMemcpyHostToDevice, c->stream));
    }
    U.cl = dcl;
    U.row = drow;
    c->in_used += n;
  }
  const int u = (int)c->units.size();
  c->units.push_back(U);
  c->uh.push_back({slot, sector, n, kLoaded, -1});
  for (int32_t b = 0; b < n; b += kChunk) c->chunks.push_back({u, b, std::min(kChunk, n - b), 0});
  c->unit_chunk0.push_back((int32_t)c->chunks.size());
  c->index[{slot, sector}] = u;
  c->n_total += n;
  c->bins_total += bins_cap_of(n, c->P.hits_per_bin, c->R);
  c->trk_total += trk_cap_of(n, c->P.min_chain);
  c->tiles_total += tile_cap_of(n, c->R, link_tile_of(c->P));
  c->tables_dirty = true;
  return TPCCA_OK;
}

// Device copy of the parameters with the default launch schedule.
static ParamsDev params_dev(const tpcca_params_t &p) {
  ParamsDev P{};
  P.n_rows = p.n_rows;
  P.wy = p.link_wy;
  P.wz = p.link_wz;
  P.link_chi2 = p.link_chi2;
  P.min_chain = p.min_chain_hits;
  P.kB = p.kB;
  P.ery = p.err2_y;
  P.erz = p.err2_z;
  P.max_sin = p.max_sinphi;
  P.c22 = p.seed_c22;
  P.c33 = p.seed_c33;
  P.c44 = p.seed_c44;
  P.r00 = p.reset_c00;
  P.r11 = p.reset_c11;
  P.nsig = p.pick_nsig;
  P.wmax = p.pick_win_max;
  P.pick_chi2 = p.pick_chi2;
  P.max_miss = p.max_miss;
  P.min_hits = p.min_track_hits;
  P.own_pct = p.own_frac_pct;
  P.inflate = p.refit_inflate;
  P.hits_per_bin = p.grid_hits_per_bin;
  P.kf_pool = 64;
  P.kf_claims = 1;
  return P;
}

// The argument checks tpcca_create applies to a geometry and parameters.
static bool setup_valid(const tpcca_geometry_t *geo, const tpcca_params_t *params) {
  if (!geo || !params || !geo->row_x) return false;
  if (geo->n_rows < 3 || geo->n_rows > kMaxRows || params->n_rows != geo->n_rows) return false;
  return !(geo->n_sectors < 1 || params->grid_hits_per_bin < 1 || params->min_chain_hits < 2 ||
           params->min_track_hits < 1 || params->max_miss < 1);
}

// ===================================================================== ABI
extern "C" {

void tpcca_params_default(tpcca_params_t *p) {
  if (!p) return;
  p->n_rows = 159;
  p->link_wy = 2.0f;
  p->link_wz = 2.0f;
  p->link_chi2 = 0.2f;
  p->min_chain_hits = 3;
  p->kB = (float)(-0.5 * 0.299792458e-2);
  p->err2_y = 0.01f;
  p->err2_z = 0.01f;
  p->max_sinphi = 0.95f;
  p->seed_c22 = 0.25f;
  p->seed_c33 = 0.25f;
  p->seed_c44 = 400.0f;
  p->reset_c00 = 1.0f;
  p->reset_c11 = 1.0f;
  p->pick_nsig = 3.0f;
  p->pick_win_max = 4.0f;
  p->pick_chi2 = 16.0f;
  p->max_miss = 10;
  p->min_track_hits = 10;
  p->own_frac_pct = 90;
  p->refit_inflate = 100.0f;
  p->grid_hits_per_bin = 1;
}

const char *tpcca_error_string(int s) {
  switch (s) {
    case TPCCA_OK: return "ok";
    case TPCCA_EINVAL: return "invalid argument or cluster";
    case TPCCA_ENOMEM: return "device memory budget exceeded";
    case TPCCA_ECAPACITY: return "output buffer too small";
    case TPCCA_EDEVICE: return "HIP runtime error";
    case TPCCA_ESTATE: return "stage called out of order or unit not loaded";
    case TPCCA_EBUSY: return "busy, retry later";
    case TPCCA_ENOTFOUND: return "unknown request";
  }
  return "unknown status";
}

const char *tpcca_last_error(tpcca_ctx_t *c) { return c ? c->last_error.c_str() : ""; }

int tpcca_create(const tpcca_geometry_t *geo, const tpcca_params_t *params, int device,
                 void *hip_stream, size_t budget, tpcca_ctx_t **out) {
  if (!out || !setup_valid(geo, params)) return TPCCA_EINVAL;
  *out = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return TPCCA_EDEVICE;
  tpcca_ctx *c = new tpcca_ctx();
  c->device = device;
  c->budget = budget ? budget : ((size_t)64 << 30);
  c->params = *params;
  c->R = geo->n_rows;
  c->n_sectors = geo->n_sectors;
  c->row_x.assign(geo->row_x, geo->row_x + geo->n_rows);
  c->P = params_dev(*params);
  tpcca_phase2_params_default(&c->p2params);
  std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return TPCCA_EDEVICE;
    }
    c->own_stream = true;
  }
  for (int k = 0; k < 7; ++k) hipEventCreate(&c->ev[k]);
  c->unit_chunk0.push_back(0);
  int rc = ensure(c, c->row_x_d, sizeof(float) * c->R, 0);
  if (rc == TPCCA_OK) rc = copy_sync(c, c->row_x_d.p, c->row_x.data(), sizeof(float) * c->R, hipMemcpyHostToDevice);
  if (rc != TPCCA_OK) {
    tpcca_destroy(c);
    return rc;
  }
  refresh_bufs(c);
  *out = c;
  return TPCCA_OK;
}

int tpcca_destroy(tpcca_ctx_t *c) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
  if (c->stream) hipStreamSynchronize(c->stream);
  drop_graphs(c);
  DevBuf *all[] = {&c->row_x_d, &c->units_d, &c->chunks_d, &c->runs_d, &c->rowtab, &c->row_cnt,
                   &c->row_fill, &c->chunk_hist, &c->rtmp,
                   &c->zmm, &c->binbeg, &c->yz, &c->sid, &c->up, &c->dn, &c->upc,
                   &c->dnc, &c->flag, &c->starts, &c->tiles, &c->sval, &c->tofg, &c->kf_order, &c->kf_tmp, &c->band_tmp, &c->srow, &c->cinfo, &c->trk_start, &c->trk_unit, &c->unit_tbegin, &c->trk,
                   &c->trk_hits, &c->owner, &c->accv, &c->wonmask, &c->accx, &c->tracks, &c->hits_out,
                   &c->assign, &c->unit_res, &c->scan_tmp, &c->zo_tmp, &c->zo_cnt, &c->kf_chunks, &c->in_cl, &c->in_row,
                   &c->p2units, &c->p2seg_begin, &c->p2seg_unit, &c->p2seg_nh, &c->p2seg_hb, &c->p2seg_fpos,
                   &c->p2seg_rows,
                   &c->p2seg_zin, &c->p2seg_zout, &c->p2seg_out, &c->p2zmm, &c->p2unit_nz, &c->p2unit_bbase, &c->p2bin_cnt, &c->p2bin_beg,
                   &c->p2bin_seg, &c->p2bin_rz, &c->p2hrec, &c->p2seg_flag, &c->p2pairs, &c->p2best_b, &c->p2best_a, &c->p2next, &c->p2prev, &c->p2final_of,
                   &c->p2final_start, &c->p2final_nhits, &c->p2final_hbeg, &c->p2finals, &c->p2final_hits,
                   &c->p2vkey0, &c->p2vkey1, &c->p2vval0, &c->p2vval1, &c->p2gstart, &c->p2group_pos,
                   &c->p2vertices, &c->p2slot_first, &c->p2slot_vbeg, &c->p2slot_vend, &c->p2flags, &c->p2rec,
                   &c->p2res, &c->p2scan, &c->p2cnt, &c->p2sort_tmp, &c->p2order, &c->p2lenh};
  for (DevBuf *b : all)
    if (b->p) hipFree(b->p);
  for (int k = 0; k < 7; ++k)
    if (c->ev[k]) hipEventDestroy(c->ev[k]);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
  return TPCCA_OK;
}

int tpcca_reset(tpcca_ctx_t *c) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->units.clear();
  c->uh.clear();
  c->chunks.clear();
  c->unit_chunk0.assign(1, 0);
  c->runs.clear();
  c->index.clear();
  c->pending_runs.clear();
  c->n_total = c->bins_total = c->trk_total = c->tiles_total = c->in_used = 0;
  c->tables_dirty = true;
  c->have_times = false;
  c->p2_done = false;
  return TPCCA_OK;
}

int tpcca_load_sector(tpcca_ctx_t *c, int32_t slot, int32_t sector, const tpcca_cluster_t *cl,
                      const uint8_t *row, int32_t n, int32_t flags) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = load_unit(c, slot, sector, cl, row, n, flags, false);
  if (rc == TPCCA_OK && (flags & 1) == TPCCA_MEM_HOST && n > 0) {
    // the caller may reuse pageable buffers on return
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return rc;
}

int tpcca_find_links(tpcca_ctx_t *c, int32_t slot, int32_t sector) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  return stage_call(c, slot, sector, 1);
}
int tpcca_clean_links(tpcca_ctx_t *c, int32_t slot, int32_t sector) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  return stage_call(c, slot, sector, kLinked);
}
int tpcca_build_tracklets(tpcca_ctx_t *c, int32_t slot, int32_t sector) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  return stage_call(c, slot, sector, kCleaned);
}
int tpcca_select_tracks(tpcca_ctx_t *c, int32_t slot, int32_t sector) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  return stage_call(c, slot, sector, kTracklets);
}

int tpcca_sync(tpcca_ctx_t *c) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  return check_errors(c);
}

int tpcca_get_links(tpcca_ctx_t *c, int32_t slot, int32_t sector, int32_t which, int32_t *up,
                    int32_t *down, int32_t n) {
  if (!c || !up || !down) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  const int u = find_unit(c, slot, sector);
  if (u < 0 || c->uh[u].state < kLinked || (which == 1 && c->uh[u].state < kCleaned))
    return TPCCA_ESTATE;
  if (n != c->uh[u].n) return TPCCA_EINVAL;
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  if (n == 0) return TPCCA_OK;
  int32_t *tmp = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
    HIPCHK(c, hipMalloc(&tmp, sizeof(int32_t) * 2 * (size_t)n));
  }
  const UnitDev &U = c->units[u];
  hipError_t e = launch_links_by_id(c->B, which ? c->B.upc : c->B.up, which ? c->B.dnc : c->B.dn,
                                    tmp, tmp + n, U.cl_begin, n, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(up, tmp, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(down, tmp + n, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  {
    std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
    hipFree(tmp);
  }
  if (e != hipSuccess) return dev_err(c, e, "get_links");
  return TPCCA_OK;
}

// tracklet range [t0, t1) of a unit (valid once tracklets were built)
static int unit_tracklets(tpcca_ctx *c, int u, int32_t *t0, int32_t *t1) {
  const int run = c->uh[u].run;
  const RunHost &h = c->runs[run];
  int32_t tb[2];
  RCCHK(copy_sync(c, &tb[0], ptr<int32_t>(c->unit_tbegin) + u, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (u + 1 < h.u1) {
    RCCHK(copy_sync(c, &tb[1], ptr<int32_t>(c->unit_tbegin) + u + 1, sizeof(int32_t),
                        hipMemcpyDeviceToHost));
  } else {
    RunDev d;
    RCCHK(copy_sync(c, &d, ptr<RunDev>(c->runs_d) + run, sizeof(d), hipMemcpyDeviceToHost));
    tb[1] = d.trk0 + d.n_trk;
  }
  *t0 = tb[0];
  *t1 = tb[1];
  return TPCCA_OK;
}

int tpcca_get_tracklets(tpcca_ctx_t *c, int32_t slot, int32_t sector, tpcca_tracklet_t *out,
                        int32_t cap, int32_t *n_out, int64_t *hit_begin, int32_t *hits,
                        int64_t hits_cap, int64_t *n_hits_out) {
  if (!c || !n_out) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  const int u = find_unit(c, slot, sector);
  if (u < 0 || c->uh[u].state < kTracklets) return TPCCA_ESTATE;
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  int32_t t0, t1;
  if ((rc = unit_tracklets(c, u, &t0, &t1)) != TPCCA_OK) return rc;
  const int T = t1 - t0;
  std::vector<tpcca_tracklet_t> trk(T);
  if (T > 0)
    RCCHK(copy_sync(c, trk.data(), ptr<tpcca_tracklet_t>(c->trk) + t0, sizeof(tpcca_tracklet_t) * T,
                        hipMemcpyDeviceToHost));
  int64_t nh = 0;
  for (auto &t : trk) nh += t.n_hits;
  *n_out = T;
  if (n_hits_out) *n_hits_out = nh;
  if (cap < T || (hits && hits_cap < nh)) return TPCCA_ECAPACITY;
  if (out && T) std::memcpy(out, trk.data(), sizeof(tpcca_tracklet_t) * T);
  if (hits || hit_begin) {
    const UnitDev &U = c->units[u];
    std::vector<int32_t> sid(U.n);
    if (U.n)
      RCCHK(copy_sync(c, sid.data(), ptr<int32_t>(c->sid) + U.cl_begin, sizeof(int32_t) * U.n,
                          hipMemcpyDeviceToHost));
    const int Rs = slot_stride(c->R);
    std::vector<int32_t> slots((size_t)T * Rs);
    if (T)
      RCCHK(copy_sync(c, slots.data(), ptr<int32_t>(c->trk_hits) + (int64_t)t0 * Rs,
                          sizeof(int32_t) * slots.size(), hipMemcpyDeviceToHost));
    int64_t off = 0;
    for (int t = 0; t < T; ++t) {
      if (hit_begin) hit_begin[t] = off;
      const int n1 = trk[t].n_pass1, ne = trk[t].n_hits - trk[t].n_pass1;
      const int32_t *hl = slots.data() + (size_t)t * Rs;
      for (int j = 0; j < trk[t].n_hits; ++j) {
        // slots hold the unit-local sorted index in their low 24 bits
        const int32_t v = j < ne ? hl[n1 + ne - 1 - j] : hl[j - ne];
        if (hits) hits[off] = sid[(uint32_t)v & 0xFFFFFFu];
        ++off;
      }
    }
    if (hit_begin) hit_begin[T] = off;
  }
  return TPCCA_OK;
}

int tpcca_get_tracks(tpcca_ctx_t *c, int32_t slot, int32_t sector, tpcca_track_t *out, int32_t cap,
                     int32_t *n_out, int32_t *hits, int64_t hits_cap, int64_t *n_hits_out) {
  if (!c || !n_out) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  const int u = find_unit(c, slot, sector);
  if (u < 0 || c->uh[u].state < kSelected) return TPCCA_ESTATE;
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  tpcca_unit_result_t r;
  RCCHK(copy_sync(c, &r, ptr<tpcca_unit_result_t>(c->unit_res) + u, sizeof(r), hipMemcpyDeviceToHost));
  *n_out = r.n_tracks;
  if (n_hits_out) *n_hits_out = r.n_track_hits;
  if (cap < r.n_tracks || (hits && hits_cap < r.n_track_hits)) return TPCCA_ECAPACITY;
  if (out && r.n_tracks)
    RCCHK(copy_sync(c, out, ptr<tpcca_track_t>(c->tracks) + r.track_begin,
                        sizeof(tpcca_track_t) * r.n_tracks, hipMemcpyDeviceToHost));
  if (hits && r.n_track_hits)
    RCCHK(copy_sync(c, hits, ptr<int32_t>(c->hits_out) + r.hit_begin, sizeof(int32_t) * r.n_track_hits,
                        hipMemcpyDeviceToHost));
  return TPCCA_OK;
}

int tpcca_get_assignment(tpcca_ctx_t *c, int32_t slot, int32_t sector, int32_t *a, int32_t n) {
  if (!c || !a) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  const int u = find_unit(c, slot, sector);
  if (u < 0 || c->uh[u].state < kSelected) return TPCCA_ESTATE;
  if (n != c->uh[u].n) return TPCCA_EINVAL;
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  if (n)
    RCCHK(copy_sync(c, a, ptr<int32_t>(c->assign) + c->units[u].cl_begin, sizeof(int32_t) * n,
                        hipMemcpyDeviceToHost));
  return TPCCA_OK;
}

// ---------------------------------------------------------------- batch ---
static int64_t bucket(int64_t v) {
  int64_t b = 1024;
  while (b < v) b += b / 2;
  return b;
}

int tpcca_run_batch(tpcca_ctx_t *c, const tpcca_batch_t *bt) {
  if (!c || !bt || bt->n_units < 0) return TPCCA_EINVAL;
  if (bt->n_units > 0 && (!bt->slot || !bt->sector || !bt->begin || !bt->n)) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = tpcca_reset(c);
  if (rc != TPCCA_OK) return rc;
  const bool host = (bt->flags & 1) == TPCCA_MEM_HOST;
  const bool graph = (bt->flags & TPCCA_BATCH_GRAPH) != 0;
  int64_t lo = INT64_MAX, hi = 0, tot = 0;
  for (int u = 0; u < bt->n_units; ++u) {
    if (bt->n[u] < 0 || bt->n[u] > 0xFFFFFF || bt->begin[u] < 0) {
      c->last_error = "a unit holds 0 .. 2^24 - 1 clusters at a non-negative offset";
      return TPCCA_EINVAL;
    }
    if (bt->n[u] == 0) continue;
    lo = std::min<int64_t>(lo, bt->begin[u]);
    hi = std::max<int64_t>(hi, bt->begin[u] + bt->n[u]);
    tot += bt->n[u];
  }
  if (tot > 0 && (!bt->cl || !bt->row)) return TPCCA_EINVAL;
  const tpcca_cluster_t *cl_base = bt->cl;
  const uint8_t *row_base = bt->row;
  if (host && tot > 0) {
    // one copy of the batch's input span
    const int64_t span = hi - lo;
    if ((rc = ensure(c, c->in_cl, (size_t)span * sizeof(float4), 0)) != TPCCA_OK) return rc;
    if ((rc = ensure(c, c->in_row, (size_t)span, 0)) != TPCCA_OK) return rc;
    HIPCHK(c, hipMemcpyAsync(c->in_cl.p, bt->cl + lo, (size_t)span * sizeof(float4),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->in_row.p, bt->row + lo, (size_t)span, hipMemcpyHostToDevice, c->stream));
    cl_base = reinterpret_cast<const tpcca_cluster_t *>(ptr<float4>(c->in_cl)) - lo;
    row_base = ptr<uint8_t>(c->in_row) - lo;
  }
  for (int u = 0; u < bt->n_units; ++u) {
    rc = load_unit(c, bt->slot[u], bt->sector[u], cl_base + bt->begin[u], row_base + bt->begin[u],
                   bt->n[u], TPCCA_MEM_DEVICE, true);
    if (rc != TPCCA_OK) return rc;
  }
  if (c->units.empty()) return TPCCA_OK;
  // capacities: graphs are captured for buckets so that they are replayed
  const int U = (int)c->units.size();
  int64_t capN = c->n_total, capU = U, capB = c->bins_total, capT = c->trk_total,
          capC = (int64_t)c->chunks.size();
  if (graph) {
    capN = bucket(capN);
    capU = bucket(capU);
    capB = bucket(capB);
    capT = bucket(capT);
    capC = bucket(capC);
  }
  rc = ensure_work(c, capN, capU, capB, capT, capC);
  if (rc == TPCCA_ENOMEM && graph) {
    // the rounded-up capacities do not fit the budget: use the exact ones
    // (the graph is then re-captured whenever the sizes change)
    capN = c->n_total;
    capU = U;
    capB = c->bins_total;
    capT = c->trk_total;
    capC = (int64_t)c->chunks.size();
    rc = ensure_work(c, capN, capU, capB, capT, capC);
  }
  if (rc != TPCCA_OK) return rc;
  if ((rc = upload_tables(c)) != TPCCA_OK) return rc;
  c->runs.push_back(make_run(c, 0, U));
  if ((rc = write_run(c, 0)) != TPCCA_OK) return rc;
  for (int u = 0; u < U; ++u) {
    c->uh[u].run = 0;
    c->uh[u].state = kSelected;
  }
  c->pending_runs.push_back(0);
  if (!graph) return launch_stages(c, 0, c->runs[0], 1, 4);
  RunHost capr = c->runs[0];
  capr.u1 = (int32_t)capU;
  capr.c1 = (int32_t)capC;
  capr.cl1 = (int32_t)capN;
  capr.bin1 = capB;
  capr.trk_cap = (int32_t)capT;
  capr.tile1 = (int32_t)(capN / link_tile_of(c->P) + capU * (c->R + 2) + 1);
  tpcca_ctx::GraphEntry *ge = nullptr;
  for (auto &e : c->graphs)
    if (e.exec[0] && e.gen == c->generation && e.timing == c->timing && same_capacities(e.cap, capr)) ge = &e;
  if (!ge) {
    // a free or outdated entry, else the least recently replayed one
    ge = &c->graphs[0];
    for (auto &e : c->graphs) {
      if (!e.exec[0] || e.gen != c->generation) {
        ge = &e;
        break;
      }
      if (e.used < ge->used) ge = &e;
    }
    // its last replay has finished before it is destroyed (waiting on this
    // context's own stream, outside the lock that other contexts' captures
    // take)
    if (ge->exec[0]) HIPCHK(c, hipStreamSynchronize(c->stream));
    std::lock_guard<std::recursive_mutex> lock(tpcca::device_ops_lock());
    if (ge->exec[0]) drop_graph(*ge);
    // one graph of the whole sequence, or with timing on one graph per timed
    // segment (HIP events between the replays of the segments)
    const int nseg = c->timing ? 6 : 1;
    for (int k = 0; k < nseg; ++k) {
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      c->capturing = true;
      hipError_t le = hipSuccess;
      if (nseg == 1) {
        for (int seg = 0; seg < 6 && le == hipSuccess; ++seg) le = launch_segment(c, 0, capr, seg);
      } else {
        le = launch_segment(c, 0, capr, k);
      }
      c->capturing = false;
      // always end the capture, also after a failed launch
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (le != hipSuccess || e != hipSuccess) {
        // the capture was invalidated (for instance by a device-wide
        // synchronisation from a thread outside this library): run this
        // batch without a graph; a real launch error shows there again
        if (g) hipGraphDestroy(g);
        drop_graphs(c);
        (void)hipGetLastError();
        ++c->graph_fallbacks;
        return launch_stages(c, 0, c->runs[0], 1, 4);
      }
      e = hipGraphInstantiate(&ge->exec[k], g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        ge->exec[k] = nullptr;
        drop_graphs(c);  // also the segments captured before
        return dev_err(c, e, "hipGraphInstantiate");
      }
    }
    ge->cap = capr;
    ge->timing = c->timing;
    ge->gen = c->generation;
  }
  ge->used = ++c->graph_clock;
  if (!ge->timing) {
    HIPCHK(c, hipGraphLaunch(ge->exec[0], c->stream));
  } else {
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    for (int k = 0; k < 6; ++k) {
      HIPCHK(c, hipGraphLaunch(ge->exec[k], c->stream));
      HIPCHK(c, hipEventRecord(c->ev[k + 1], c->stream));
    }
  }
  c->have_times = ge->timing;
  return TPCCA_OK;
}

int tpcca_batch_totals(tpcca_ctx_t *c, int32_t *n_units, int64_t *n_clusters, int64_t *n_tracks,
                       int64_t *n_hits) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  if (n_units) *n_units = (int32_t)c->units.size();
  if (n_clusters) *n_clusters = c->n_total;
  int64_t nt = 0, nh = 0;
  for (size_t r = 0; r < c->runs.size(); ++r) {
    RunDev d;
    RCCHK(copy_sync(c, &d, ptr<RunDev>(c->runs_d) + r, sizeof(d), hipMemcpyDeviceToHost));
    bool selected = true;
    for (int u = c->runs[r].u0; u < c->runs[r].u1; ++u) selected &= c->uh[u].state >= kSelected;
    if (selected) {
      nt += d.n_acc;
      nh += d.n_acc_hits;
    }
  }
  if (n_tracks) *n_tracks = nt;
  if (n_hits) *n_hits = nh;
  return TPCCA_OK;
}

int tpcca_work_stats(tpcca_ctx_t *c, tpcca_work_stats_t *out) {
  if (!c || !out) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  std::memset(out, 0, sizeof(*out));
  out->clusters = c->n_total;
  out->graph_fallbacks = c->graph_fallbacks;
  for (size_t r = 0; r < c->runs.size(); ++r) {
    RunDev d;
    RCCHK(copy_sync(c, &d, ptr<RunDev>(c->runs_d) + r, sizeof(d), hipMemcpyDeviceToHost));
    int lo = kSelected;
    for (int u = c->runs[r].u0; u < c->runs[r].u1; ++u) lo = std::min(lo, c->uh[u].state);
    if (lo >= kTracklets) {
      out->tracklets += d.n_trk;
      out->fit_steps += (int64_t)d.kf_steps;
      out->fit_candidates += (int64_t)d.kf_cands;
      out->fit_tests += (int64_t)d.kf_tests;
      out->fit_updates += (int64_t)d.kf_updates;
      out->fit_wave_iterations += (int64_t)d.kf_iters;
      if (d.kf_t_end > d.kf_t_start && d.kf_t_start != ~0ull) {
        out->fit_ns += (int64_t)(d.kf_t_end - d.kf_t_start) * 10;  // 100 MHz clock
        if (d.kf_t_drain != ~0ull && d.kf_t_drain <= d.kf_t_end)
          out->fit_drain_ns += (int64_t)(d.kf_t_end - d.kf_t_drain) * 10;
      }
    }
    if (lo >= kSelected) {
      out->tracks += d.n_acc;
      out->track_hits += d.n_acc_hits;
    }
  }
  return TPCCA_OK;
}

int tpcca_get_batch_results(tpcca_ctx_t *c, tpcca_unit_result_t *units, tpcca_track_t *tracks,
                            int64_t tracks_cap, int32_t *hits, int64_t hits_cap, int32_t *assignment,
                            int64_t n_clusters) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  const int U = (int)c->units.size();
  for (int u = 0; u < U; ++u)
    if (c->uh[u].state < kSelected) return TPCCA_ESTATE;
  std::vector<tpcca_unit_result_t> ur(U);
  if (U)
    RCCHK(copy_sync(c, ur.data(), c->unit_res.p, sizeof(tpcca_unit_result_t) * U, hipMemcpyDeviceToHost));
  int64_t nt = 0, nh = 0;
  for (auto &r : ur) {
    nt += r.n_tracks;
    nh += r.n_track_hits;
  }
  if ((tracks && tracks_cap < nt) || (hits && hits_cap < nh) || (assignment && n_clusters < c->n_total))
    return TPCCA_ECAPACITY;
  // batch-relative offsets
  int64_t to = 0, ho = 0;
  for (int u = 0; u < U; ++u) {
    if (tracks && ur[u].n_tracks)
      HIPCHK(c, hipMemcpyAsync(tracks + to, ptr<tpcca_track_t>(c->tracks) + ur[u].track_begin,
                               sizeof(tpcca_track_t) * ur[u].n_tracks, hipMemcpyDeviceToHost, c->stream));
    if (hits && ur[u].n_track_hits)
      HIPCHK(c, hipMemcpyAsync(hits + ho, ptr<int32_t>(c->hits_out) + ur[u].hit_begin,
                               sizeof(int32_t) * ur[u].n_track_hits, hipMemcpyDeviceToHost, c->stream));
    ur[u].track_begin = to;
    ur[u].hit_begin = ho;
    to += ur[u].n_tracks;
    ho += ur[u].n_track_hits;
  }
  if (assignment && c->n_total)
    HIPCHK(c, hipMemcpyAsync(assignment, c->assign.p, sizeof(int32_t) * c->n_total, hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (units && U) std::memcpy(units, ur.data(), sizeof(tpcca_unit_result_t) * U);
  return TPCCA_OK;
}

int tpcca_device_results(tpcca_ctx_t *c, tpcca_device_results_t *out) {
  if (!c || !out) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  int rc = check_errors(c);
  if (rc != TPCCA_OK) return rc;
  out->tracks = ptr<tpcca_track_t>(c->tracks);
  out->hits = ptr<int32_t>(c->hits_out);
  out->assignment = ptr<int32_t>(c->assign);
  out->units = ptr<tpcca_unit_result_t>(c->unit_res);
  out->n_units = (int32_t)c->units.size();
  return TPCCA_OK;
}

void tpcca_tuning_default(tpcca_tuning_t *t) {
  if (!t) return;
  *t = tpcca_tuning_t{};
  t->fit_pool = 64;
  t->fit_claims = 1;
}

int tpcca_set_tuning(tpcca_ctx_t *c, const tpcca_tuning_t *t) {
  if (!c || !t) return TPCCA_EINVAL;
  if (!tpcca::tuning_valid(t, c->R)) return TPCCA_EINVAL;
  // the grid layout and the tile reservations of loaded units depend on
  // hits per bin and the tile size
  if (t->grid_hits_per_bin && !c->units.empty() && t->grid_hits_per_bin != c->P.hits_per_bin)
    return TPCCA_ESTATE;
  if (!c->units.empty() && (t->link_tile ? t->link_tile : kTile) != link_tile_of(c->P)) return TPCCA_ESTATE;
  c->P.kf_min_waves = t->fit_min_waves;
  c->P.kf_claims = t->fit_claims;
  c->P.kf_xcd = t->fit_xcd_slices;
  c->P.link_stage = t->link_stage;
  c->P.kf_split = t->fit_long_first;
  c->P.kf_bands = t->fit_row_bands;
  c->P.kf_tail = t->fit_tail_units;
  c->P.kf_rows = t->fit_rows;
  c->P.link_tile = t->link_tile;
  c->P.kf_block = t->fit_block;
  c->P.kf_pool = t->fit_pool ? t->fit_pool : 64;
  c->P.kf_blocks_per_cu = t->fit_blocks_per_cu;
  c->P.link_blocks_per_cu = t->link_blocks_per_cu;
  if (t->grid_hits_per_bin) {
    c->P.hits_per_bin = t->grid_hits_per_bin;
    c->params.grid_hits_per_bin = t->grid_hits_per_bin;
  }
  c->generation++;  // launch shapes changed: the cached graphs are captured again
  return TPCCA_OK;
}

int tpcca_get_tuning(tpcca_ctx_t *c, tpcca_tuning_t *t) {
  if (!c || !t) return TPCCA_EINVAL;
  t->fit_pool = c->P.kf_pool;
  t->fit_blocks_per_cu = c->P.kf_blocks_per_cu;
  t->grid_hits_per_bin = c->P.hits_per_bin;
  t->link_blocks_per_cu = c->P.link_blocks_per_cu;
  t->fit_min_waves = c->P.kf_min_waves;
  t->fit_claims = c->P.kf_claims;
  t->fit_xcd_slices = c->P.kf_xcd;
  t->link_stage = c->P.link_stage;
  t->fit_long_first = c->P.kf_split;
  t->fit_row_bands = c->P.kf_bands;
  t->fit_tail_units = c->P.kf_tail;
  t->fit_rows = c->P.kf_rows;
  t->link_tile = c->P.link_tile;
  t->fit_block = c->P.kf_block;
  return TPCCA_OK;
}

int tpcca_set_timing(tpcca_ctx_t *c, int32_t enable) {
  if (!c) return TPCCA_EINVAL;
  c->timing = enable != 0;
  return TPCCA_OK;
}

int tpcca_stage_times(tpcca_ctx_t *c, float *ms, int32_t cap) {
  if (!c || !ms) return TPCCA_EINVAL;
  if (!c->have_times) return 0;
  int n = std::min(cap, 6);
  for (int k = 0; k < n; ++k) ms[k] = c->stage_ms[k];
  return n;
}

}  // extern "C"

// ------------------------------------------------------ allocation-free ---
// Device memory of tpcca_run_batch_noalloc: the run tables and every work
// buffer are carved from this array.  Each device the library runs on holds
// its own copy until the process ends.  In host code the name stands for a
// host-side shadow, not a device address: the device address is looked up
// once per device with hipGetSymbolAddress and only that address is used.
static __device__ __align__(256) unsigned char noalloc_scratch[TPCCA_NOALLOC_SCRATCH_BYTES];

namespace {

struct NoallocDevice {
  std::mutex mu;                      // one call at a time per device
  unsigned char *scratch = nullptr;   // device address of noalloc_scratch
  std::vector<unsigned char> tables;  // host image of the run tables
};

NoallocDevice &noalloc_device(int dev) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<NoallocDevice>> devs;
  std::lock_guard<std::mutex> lock(mu);
  auto &d = devs[dev];
  if (!d) d.reset(new NoallocDevice());
  return *d;
}

// Lays out the run tables (row radii, the run, units, chunks: one block at
// the start, written by one copy) and every work buffer from `base`, 256-B
// aligned; base = nullptr only sizes them.  Returns {table bytes, total bytes}.
std::pair<size_t, size_t> noalloc_layout(unsigned char *base, int R_, int64_t n_cl, int64_t n_units,
                                         int64_t n_bins, int64_t n_trk, int64_t n_chunks, Bufs &B) {
  TPCCA_BUFFER_COUNTS(R_, n_cl, n_units, n_bins, n_trk, n_chunks)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char *p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  B.row_x = reinterpret_cast<float *>(take(sizeof(float) * (size_t)R));
  B.runs = reinterpret_cast<RunDev *>(take(sizeof(RunDev)));
  B.units = reinterpret_cast<UnitDev *>(take(sizeof(UnitDev) * U));
  B.chunks = reinterpret_cast<Chunk *>(take(sizeof(Chunk) * NC));
  const size_t table_bytes = off;
#define CARVE(buf, field, type, count, keepc) B.field = reinterpret_cast<type *>(take((size_t)(count) * sizeof(type)));
  TPCCA_WORK_BUFFERS(CARVE)
#undef CARVE
  B.ids_tmp = nullptr;
  return {table_bytes, off};
}

}  // namespace

extern "C" int tpcca_run_batch_noalloc(const tpcca_geometry_t *geo, const tpcca_params_t *params,
                                       int device, void *hip_stream, const tpcca_batch_t *bt,
                                       tpcca_track_t *tracks, int64_t tracks_cap, int32_t *hits,
                                       int64_t hits_cap, int32_t *assignment, int64_t n_assignment,
                                       tpcca_unit_result_t *units, int64_t *n_tracks_out,
                                       int64_t *n_hits_out) {
  if (!setup_valid(geo, params) || !bt || bt->n_units < 0) return TPCCA_EINVAL;
  if ((bt->flags & 1) != TPCCA_MEM_DEVICE || (bt->flags & TPCCA_BATCH_GRAPH)) return TPCCA_EINVAL;
  const int U = bt->n_units;
  if (U > 0 && (!bt->slot || !bt->sector || !bt->begin || !bt->n || !units)) return TPCCA_EINVAL;
  const int R = geo->n_rows;
  const ParamsDev P = params_dev(*params);
  // capacities, exactly as a context reserves them for these units
  int64_t n_total = 0, bins_total = 0, trk_total = 0, tiles_total = 0, n_chunks = 0;
  for (int u = 0; u < U; ++u) {
    const int64_t n = bt->n[u];
    if (n < 0 || n > 0xFFFFFF || bt->begin[u] < 0 || bt->slot[u] < 0 || bt->sector[u] < 0 ||
        bt->sector[u] >= geo->n_sectors)
      return TPCCA_EINVAL;
    n_total += n;
    bins_total += bins_cap_of(n, P.hits_per_bin, R);
    trk_total += trk_cap_of(n, P.min_chain);
    tiles_total += tile_cap_of(n, R, link_tile_of(P));
    n_chunks += (n + kChunk - 1) / kChunk;
  }
  if (n_total > 0 && (!bt->cl || !bt->row)) return TPCCA_EINVAL;
  if (n_total > 0 && (!tracks || !hits || !assignment)) return TPCCA_EINVAL;
  if (tracks_cap < trk_total || hits_cap < n_total || n_assignment < n_total) return TPCCA_ECAPACITY;
  Bufs B{};
  const auto sz = noalloc_layout(nullptr, R, n_total, U, bins_total, trk_total, n_chunks, B);
  if (sz.second > (size_t)TPCCA_NOALLOC_SCRATCH_BYTES) return TPCCA_ENOMEM;
  if (U == 0) {
    if (n_tracks_out) *n_tracks_out = 0;
    if (n_hits_out) *n_hits_out = 0;
    return TPCCA_OK;
  }
  if (hipSetDevice(device) != hipSuccess) return TPCCA_EDEVICE;
  NoallocDevice &D = noalloc_device(device);
  std::lock_guard<std::mutex> lock(D.mu);
  if (!D.scratch) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return TPCCA_EDEVICE;
    }
    D.scratch = static_cast<unsigned char *>(p);
  }
  // host image of the tables, laid out as on the device
  D.tables.assign(sz.first, 0);
  Bufs H{};
  noalloc_layout(D.tables.data(), R, n_total, U, bins_total, trk_total, n_chunks, H);
  std::memcpy(const_cast<float *>(H.row_x), geo->row_x, sizeof(float) * (size_t)R);
  int64_t cl = 0, bins = 0, trk = 0, tiles = 0, ch = 0;
  for (int u = 0; u < U; ++u) {
    const int32_t n = bt->n[u];
    UnitDev &V = H.units[u];
    V.cl = reinterpret_cast<const float4 *>(bt->cl + bt->begin[u]);
    V.row = bt->row + bt->begin[u];
    V.bin_base = bins;
    V.cl_begin = (int32_t)cl;
    V.n = n;
    V.trk_base = (int32_t)trk;
    V.slot = bt->slot[u];
    V.sector = bt->sector[u];
    V.tile_base = (int32_t)tiles;
    for (int32_t b = 0; b < n; b += kChunk) H.chunks[ch++] = Chunk{u, b, std::min(kChunk, n - b), 0};
    cl += n;
    bins += bins_cap_of(n, P.hits_per_bin, R);
    trk += trk_cap_of(n, P.min_chain);
    tiles += tile_cap_of(n, R, link_tile_of(P));
  }
  RunHost h{};
  h.u0 = 0;
  h.u1 = U;
  h.c0 = 0;
  h.c1 = (int32_t)n_chunks;
  h.cl0 = 0;
  h.cl1 = (int32_t)n_total;
  h.bin0 = 0;
  h.bin1 = bins_total;
  h.trk0 = 0;
  h.trk_cap = (int32_t)trk_total;
  h.tile0 = 0;
  h.tile1 = (int32_t)tiles_total;
  h.dense = n_total / ((int64_t)U * (R + 1)) >= 1024 ? 1 : 0;
  RunDev &rd = H.runs[0];
  rd.u0 = h.u0;
  rd.u1 = h.u1;
  rd.c0 = h.c0;
  rd.c1 = h.c1;
  rd.cl0 = h.cl0;
  rd.cl1 = h.cl1;
  rd.bin0 = h.bin0;
  rd.bin1 = h.bin1;
  rd.trk0 = h.trk0;
  rd.trk_cap = h.trk_cap;
  rd.tile0 = h.tile0;
  rd.tile1 = h.tile1;
  noalloc_layout(D.scratch, R, n_total, U, bins_total, trk_total, n_chunks, B);
  B.tracks = tracks;
  B.hits_out = hits;
  B.assign = assignment;
  B.unit_res = units;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipMemcpyAsync(D.scratch, D.tables.data(), sz.first, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_grid(B, P, 0, h, s);
  if (e == hipSuccess) e = launch_links(B, P, 0, h, s);
  if (e == hipSuccess) e = launch_clean(B, P, 0, h, s);
  if (e == hipSuccess) e = launch_chains(B, P, 0, h, s);
  if (e == hipSuccess) e = launch_kf(B, P, 0, h, s);
  if (e == hipSuccess) e = launch_select(B, P, 0, h, s);
  RunDev out{};
  if (e == hipSuccess) e = hipMemcpyAsync(&out, B.runs, sizeof(RunDev), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return TPCCA_EDEVICE;
  }
  if (out.err) return (out.err & 2) ? TPCCA_EDEVICE : TPCCA_EINVAL;
  if (n_tracks_out) *n_tracks_out = out.n_acc;
  if (n_hits_out) *n_hits_out = out.n_acc_hits;
  return TPCCA_OK;
}

// ------------------------------------------------ internal (server) hooks ---
namespace tpcca {
std::recursive_mutex &device_ops_lock() {
  static std::recursive_mutex mu;
  return mu;
}
hipStream_t ctx_stream(tpcca_ctx *c) { return c->stream; }
bool tuning_valid(const tpcca_tuning_t *t, int n_rows) {
  return !(t->fit_pool < 0 || t->fit_pool > 4096 || t->fit_blocks_per_cu < 0 || t->grid_hits_per_bin < 0 ||
           t->link_blocks_per_cu < 0 || t->fit_min_waves < 0 || t->fit_claims < 0 || t->fit_claims > 1 ||
           t->fit_xcd_slices < 0 || t->fit_xcd_slices > 1 || t->link_stage < 0 || t->link_stage > 2 ||
           t->fit_long_first < 0 || t->fit_row_bands < 0 || t->fit_row_bands > n_rows ||
           t->fit_tail_units < 0 || t->fit_rows < 0 || (t->fit_rows > 0 && t->fit_rows < 64) ||
           t->fit_rows > 1024 ||
           !(t->link_tile == 0 || t->link_tile == 128 || t->link_tile == 256 || t->link_tile == 512) ||
           !(t->fit_block == 0 || t->fit_block == 64 || t->fit_block == 128 || t->fit_block == 256));
}
size_t ctx_allocated(tpcca_ctx *c) { return c->allocated; }
}  // namespace tpcca

// ========================================================= second phase ===
// Merging of the sector segments and refit (Sec. 2), vertex times (Sec. 5),
// track-model compression and rejection flags (Sec. 3) on the accepted
// tracks of every unit of a context.
namespace {

P2Params p2_dev(const tpcca_phase2_params_t &q) {
  P2Params d{};
  d.cs = q.sector_cos;
  d.sn = q.sector_sin;
  d.max_sin = q.max_sinphi;
  d.dz_ends = q.merge_dz_ends;
  d.max_gap = q.merge_max_gap;
  d.wy = q.merge_wy;
  d.wz = q.merge_wz;
  d.chi2 = q.merge_chi2;
  d.inflate = q.refit_inflate;
  d.dca_steps = q.dca_steps;
  d.vdrift = q.vdrift;
  d.gap_us = q.vtx_gap_us;
  d.vtx_min_tracks = q.vtx_min_tracks;
  d.vtx_min_hits = q.vtx_min_hits;
  d.attach_us = q.vtx_attach_us;
  d.qy = q.cmp_qy;
  d.qz = q.cmp_qz;
  d.c22 = q.cmp_c22;
  d.c33 = q.cmp_c33;
  d.c44 = q.cmp_c44;
  d.rej_qpt = q.rej_qpt;
  d.rej_looper = q.rej_looper_qpt;
  d.rej_sin = q.rej_sinphi;
  return d;
}

// the tracker's parameters with the phase's own |sin phi| limit
ParamsDev p2_prop_params(const tpcca_ctx *c) {
  ParamsDev P = c->P;
  P.max_sin = c->p2params.max_sinphi;
  return P;
}

bool p2_valid(const tpcca_phase2_params_t &q) {
  auto fin = [](float v) { return std::isfinite(v); };
  return fin(q.sector_cos) && fin(q.sector_sin) && q.max_sinphi > 0.0f && q.max_sinphi < 1.0f &&
         q.merge_dz_ends >= 0.0f && q.merge_max_gap >= 1 && q.merge_wy >= 0.0f && q.merge_wz >= 0.0f &&
         q.merge_chi2 >= 0.0f && q.refit_inflate > 0.0f && q.dca_steps >= 1 && q.dca_steps <= 1024 &&
         q.vdrift > 0.0f && q.vtx_gap_us >= 0.0f && q.vtx_min_tracks >= 1 && q.vtx_attach_us >= 0.0f &&
         q.cmp_qy > 0.0f && q.cmp_qz > 0.0f && q.cmp_c22 > 0.0f && q.cmp_c33 > 0.0f && q.cmp_c44 > 0.0f &&
         fin(q.rej_qpt) && fin(q.rej_looper_qpt) && fin(q.rej_sinphi);
}

int p2_ensure(tpcca_ctx *c, int64_t U, int64_t T, int64_t N, int64_t S) {
  U = std::max<int64_t>(U, 1);
  T = std::max<int64_t>(T, 1);
  N = std::max<int64_t>(N, 1);
  S = std::max<int64_t>(S, 1);
  const int64_t tiles = T / kP2Tile + 2 + N / kP2Tile;
  struct E {
    DevBuf *b;
    size_t bytes;
  } list[] = {
      {&c->p2units, sizeof(P2Unit) * U}, {&c->p2seg_begin, sizeof(int32_t) * (U + 1)},
      {&c->p2seg_unit, sizeof(int32_t) * T}, {&c->p2seg_nh, sizeof(int32_t) * T},
      {&c->p2seg_hb, sizeof(int64_t) * T}, {&c->p2seg_fpos, sizeof(int32_t) * T},
      {&c->p2seg_rows, sizeof(int2) * T},
      {&c->p2seg_zin, sizeof(float) * T}, {&c->p2seg_zout, sizeof(float) * T},
      {&c->p2seg_out, sizeof(P2Out) * T}, {&c->p2zmm, sizeof(int2) * U},
      {&c->p2unit_nz, sizeof(int32_t) * U}, {&c->p2unit_bbase, sizeof(int64_t) * U},
      {&c->p2bin_cnt, sizeof(int32_t) * p2_grid_cells(T, U, c->R)},
      {&c->p2bin_beg, sizeof(int32_t) * (p2_grid_cells(T, U, c->R) + U)},
      {&c->p2bin_seg, sizeof(int32_t) * T}, {&c->p2bin_rz, sizeof(int2) * T},
      {&c->p2hrec, sizeof(float4) * N}, {&c->p2seg_flag, sizeof(float4) * T},
      {&c->p2best_b, sizeof(unsigned long long) * T},
      {&c->p2best_a, sizeof(unsigned long long) * T}, {&c->p2next, sizeof(int32_t) * T},
      {&c->p2prev, sizeof(int32_t) * T}, {&c->p2final_of, sizeof(int32_t) * T},
      {&c->p2final_start, sizeof(int32_t) * T}, {&c->p2final_nhits, sizeof(int32_t) * T},
      {&c->p2final_hbeg, sizeof(int64_t) * T}, {&c->p2finals, sizeof(tpcca_final_t) * T},
      {&c->p2final_hits, sizeof(int32_t) * N}, {&c->p2vkey0, sizeof(unsigned long long) * T},
      {&c->p2vkey1, sizeof(unsigned long long) * T}, {&c->p2vval0, sizeof(int32_t) * T},
      {&c->p2vval1, sizeof(int32_t) * T}, {&c->p2gstart, sizeof(int32_t) * T},
      {&c->p2group_pos, sizeof(int32_t) * T}, {&c->p2vertices, sizeof(tpcca_vertex_t) * T},
      {&c->p2slot_first, sizeof(int32_t) * S}, {&c->p2slot_vbeg, sizeof(int32_t) * S},
      {&c->p2slot_vend, sizeof(int32_t) * S}, {&c->p2flags, (size_t)N},
      {&c->p2rec, sizeof(int32_t) * 6 * T}, {&c->p2res, sizeof(int32_t) * 4 * N},
      {&c->p2scan, sizeof(int64_t) * (tiles + 2)}, {&c->p2cnt, sizeof(P2Counts)},
      {&c->p2order, sizeof(int32_t) * T}, {&c->p2lenh, sizeof(int32_t) * 2 * 512},
  };
  for (auto &e : list) RCCHK(ensure(c, *e.b, e.bytes, 0));
  P2Bufs &Q = c->P2;
  Q.units = ptr<P2Unit>(c->p2units);
  Q.n_units = (int32_t)c->units.size();
  Q.seg_begin = ptr<int32_t>(c->p2seg_begin);
  Q.seg_unit = ptr<int32_t>(c->p2seg_unit);
  Q.seg_nh = ptr<int32_t>(c->p2seg_nh);
  Q.seg_hb = ptr<int64_t>(c->p2seg_hb);
  Q.seg_rows = ptr<int2>(c->p2seg_rows);
  Q.seg_zin = ptr<float>(c->p2seg_zin);
  Q.seg_zout = ptr<float>(c->p2seg_zout);
  Q.seg_out = ptr<P2Out>(c->p2seg_out);
  Q.zmm = ptr<int2>(c->p2zmm);
  Q.unit_nz = ptr<int32_t>(c->p2unit_nz);
  Q.unit_bbase = ptr<int64_t>(c->p2unit_bbase);
  Q.bin_cnt = ptr<int32_t>(c->p2bin_cnt);
  Q.bin_beg = ptr<int32_t>(c->p2bin_beg);
  Q.bin_seg = ptr<int32_t>(c->p2bin_seg);
  Q.bin_rz = ptr<int2>(c->p2bin_rz);
  Q.hrec = ptr<float4>(c->p2hrec);
  Q.seg_flag = ptr<float4>(c->p2seg_flag);
  Q.best_b = ptr<unsigned long long>(c->p2best_b);
  Q.best_a = ptr<unsigned long long>(c->p2best_a);
  Q.next = ptr<int32_t>(c->p2next);
  Q.prev = ptr<int32_t>(c->p2prev);
  Q.final_of = ptr<int32_t>(c->p2final_of);
  Q.seg_fpos = ptr<int32_t>(c->p2seg_fpos);
  Q.final_start = ptr<int32_t>(c->p2final_start);
  Q.final_nhits = ptr<int32_t>(c->p2final_nhits);
  Q.final_hbeg = ptr<int64_t>(c->p2final_hbeg);
  Q.finals = ptr<tpcca_final_t>(c->p2finals);
  Q.final_hits = ptr<int32_t>(c->p2final_hits);
  Q.vkey[0] = ptr<unsigned long long>(c->p2vkey0);
  Q.vkey[1] = ptr<unsigned long long>(c->p2vkey1);
  Q.vval[0] = ptr<int32_t>(c->p2vval0);
  Q.vval[1] = ptr<int32_t>(c->p2vval1);
  Q.gstart = ptr<int32_t>(c->p2gstart);
  Q.group_pos = ptr<int32_t>(c->p2group_pos);
  Q.vertices = ptr<tpcca_vertex_t>(c->p2vertices);
  Q.slot_first = ptr<int32_t>(c->p2slot_first);
  Q.slot_vbeg = ptr<int32_t>(c->p2slot_vbeg);
  Q.slot_vend = ptr<int32_t>(c->p2slot_vend);
  Q.flags = ptr<uint8_t>(c->p2flags);
  Q.rec = ptr<int32_t>(c->p2rec);
  Q.res = ptr<int32_t>(c->p2res);
  Q.scan_tmp = ptr<int64_t>(c->p2scan);
  Q.cnt = ptr<P2Counts>(c->p2cnt);
  Q.order = ptr<int32_t>(c->p2order);
  Q.len_hist = ptr<int32_t>(c->p2lenh);
  Q.len_cursor = Q.len_hist + 512;
  return TPCCA_OK;
}

int p2_side_of(int s) { return s < 18 ? 0 : 1; }

int p2_ready(tpcca_ctx *c) {
  if (!c) return TPCCA_EINVAL;
  if (!c->p2_done) return TPCCA_ESTATE;
  hipSetDevice(c->device);
  return check_errors(c);
}

}  // namespace

extern "C" {

void tpcca_phase2_params_default(tpcca_phase2_params_t *q) {
  if (!q) return;
  const double w = 20.0 * 3.14159265358979323846 / 180.0;
  q->sector_cos = (float)std::cos(w);
  q->sector_sin = (float)std::sin(w);
  q->max_sinphi = 0.99f;
  q->merge_dz_ends = 40.0f;
  q->merge_max_gap = 10;
  q->merge_wy = 4.0f;
  q->merge_wz = 4.0f;
  q->merge_chi2 = 50.0f;
  q->refit_inflate = 100.0f;
  q->dca_steps = 16;
  q->vdrift = 2.58f;
  q->vtx_gap_us = 0.1f;
  q->vtx_min_tracks = 3;
  q->vtx_min_hits = 20;
  q->vtx_attach_us = 0.25f;
  q->cmp_qy = 0.01f;
  q->cmp_qz = 0.01f;
  q->cmp_c22 = 1e-4f;
  q->cmp_c33 = 1e-4f;
  q->cmp_c44 = 1.0f;
  q->rej_qpt = 20.0f;
  q->rej_looper_qpt = 5.4f;
  q->rej_sinphi = 0.8f;
}

int tpcca_set_phase2_params(tpcca_ctx_t *c, const tpcca_phase2_params_t *q) {
  if (!c || !q || !p2_valid(*q)) return TPCCA_EINVAL;
  c->p2params = *q;
  return TPCCA_OK;
}

int tpcca_phase2(tpcca_ctx_t *c) {
  if (!c) return TPCCA_EINVAL;
  hipSetDevice(c->device);
  const int U = (int)c->units.size();
  if (U == 0) return TPCCA_ESTATE;
  for (int u = 0; u < U; ++u)
    if (c->uh[u].state < kSelected) return TPCCA_ESTATE;
  c->p2_done = false;
  // units: compact slot index and the neighbouring sectors of the same side
  std::map<int, int> slot_idx;
  c->p2_slot_value.clear();
  for (int u = 0; u < U; ++u) {
    if (!slot_idx.count(c->uh[u].slot)) {
      slot_idx[c->uh[u].slot] = (int)c->p2_slot_value.size();
      c->p2_slot_value.push_back(c->uh[u].slot);
    }
  }
  std::vector<P2Unit> pu(U);
  for (int u = 0; u < U; ++u) {
    const int s = c->uh[u].sector, side = p2_side_of(s);
    const int sp = side * 18 + ((s % 18) + 17) % 18, sn = side * 18 + ((s % 18) + 1) % 18;
    pu[u].slot = slot_idx[c->uh[u].slot];
    pu[u].sector = s;
    pu[u].prev = (s < 36 && sp < c->n_sectors && sp != s) ? find_unit(c, c->uh[u].slot, sp) : -1;
    pu[u].next = (s < 36 && sn < c->n_sectors && sn != s) ? find_unit(c, c->uh[u].slot, sn) : -1;
  }
  const int64_t T = std::max<int64_t>(c->trk_total, 1);
  const int S = (int)c->p2_slot_value.size();
  RCCHK(p2_ensure(c, U, T, c->n_total, S));
  RCCHK(copy_sync(c, c->p2units.p, pu.data(), sizeof(P2Unit) * U, hipMemcpyHostToDevice));
  const P2Params q = p2_dev(c->p2params);
  const ParamsDev P = p2_prop_params(c);
  hipError_t e = p2_launch_merge(c->B, c->P2, P, q, U, T, c->n_total, c->stream);
  if (e != hipSuccess) return dev_err(c, e, "second phase (merge)");
  RCCHK(copy_sync(c, &c->p2c, c->p2cnt.p, sizeof(P2Counts), hipMemcpyDeviceToHost));
  RCCHK(ensure(c, c->p2pairs, sizeof(int2) * (size_t)std::max<int64_t>(c->p2c.n_pairs, 1), 0));
  e = p2_launch_pairs(c->B, c->P2, P, q, T, ptr<int2>(c->p2pairs), c->p2c.n_pairs, c->stream);
  if (e != hipSuccess) return dev_err(c, e, "second phase (pairs, refit)");
  RCCHK(copy_sync(c, &c->p2c, c->p2cnt.p, sizeof(P2Counts), hipMemcpyDeviceToHost));
  const size_t tmp = p2_sort_tmp_bytes(c->p2c.n_cand);
  RCCHK(ensure(c, c->p2sort_tmp, std::max<size_t>(tmp, 256), 0));
  e = p2_launch_vertices(c->B, c->P2, P, q, c->p2c.n_final, c->p2c.n_cand, S, c->p2sort_tmp.p,
                         c->p2sort_tmp.bytes, c->stream);
  if (e != hipSuccess) return dev_err(c, e, "second phase (vertices)");
  e = p2_launch_finish(c->B, c->P2, P, q, c->p2c.n_seg, c->p2c.n_final, c->n_total, c->stream);
  if (e != hipSuccess) return dev_err(c, e, "second phase (flags, compression)");
  c->p2_done = true;
  return TPCCA_OK;
}

int tpcca_get_finals(tpcca_ctx_t *c, int32_t slot, tpcca_final_t *out, int32_t cap, int32_t *n_out,
                     int32_t *hits, int64_t hits_cap, int64_t *n_hits_out) {
  RCCHK(p2_ready(c));
  if (!n_out) return TPCCA_EINVAL;
  const int nf = c->p2c.n_final;
  std::vector<tpcca_final_t> all(nf);
  if (nf) RCCHK(copy_sync(c, all.data(), c->p2finals.p, sizeof(tpcca_final_t) * nf, hipMemcpyDeviceToHost));
  std::vector<int> mine;
  int64_t nh = 0;
  for (int f = 0; f < nf; ++f) {
    if (c->p2_slot_value[all[f].slot] != slot) continue;
    mine.push_back(f);
    nh += all[f].n_hits;
  }
  *n_out = (int32_t)mine.size();
  if (n_hits_out) *n_hits_out = nh;
  if (cap < (int32_t)mine.size() || (hits && hits_cap < nh)) return TPCCA_ECAPACITY;
  int64_t off = 0;
  for (size_t k = 0; k < mine.size(); ++k) {
    tpcca_final_t o = all[mine[k]];
    if (hits && o.n_hits)
      HIPCHK(c, hipMemcpyAsync(hits + off, ptr<int32_t>(c->p2final_hits) + o.hit_begin, sizeof(int32_t) * o.n_hits,
                               hipMemcpyDeviceToHost, c->stream));
    o.slot = slot;
    o.hit_begin = off;
    off += o.n_hits;
    if (out) out[k] = o;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TPCCA_OK;
}

int tpcca_get_segment_links(tpcca_ctx_t *c, int32_t slot, int32_t sector, int32_t *next, int32_t *prev,
                            int32_t *final_of, int32_t n) {
  RCCHK(p2_ready(c));
  const int u = find_unit(c, slot, sector);
  if (u < 0) return TPCCA_ESTATE;
  const int U = (int)c->units.size();
  std::vector<int32_t> sb(U + 1), su;
  RCCHK(copy_sync(c, sb.data(), c->p2seg_begin.p, sizeof(int32_t) * (U + 1), hipMemcpyDeviceToHost));
  const int g0 = sb[u], ng = sb[u + 1] - sb[u];
  if (n != ng) return TPCCA_EINVAL;
  if (ng == 0) return TPCCA_OK;
  std::vector<int32_t> nx(ng), pv(ng), fo(ng);
  RCCHK(copy_sync(c, nx.data(), ptr<int32_t>(c->p2next) + g0, sizeof(int32_t) * ng, hipMemcpyDeviceToHost));
  RCCHK(copy_sync(c, pv.data(), ptr<int32_t>(c->p2prev) + g0, sizeof(int32_t) * ng, hipMemcpyDeviceToHost));
  RCCHK(copy_sync(c, fo.data(), ptr<int32_t>(c->p2final_of) + g0, sizeof(int32_t) * ng, hipMemcpyDeviceToHost));
  // final index among the slot's finals: finals of earlier positions in the slot
  const int nf = c->p2c.n_final;
  std::vector<tpcca_final_t> all(nf);
  if (nf) RCCHK(copy_sync(c, all.data(), c->p2finals.p, sizeof(tpcca_final_t) * nf, hipMemcpyDeviceToHost));
  std::vector<int32_t> local(nf, -1);
  int k = 0;
  for (int f = 0; f < nf; ++f)
    if (c->p2_slot_value[all[f].slot] == slot) local[f] = k++;
  auto key = [&](int g) {
    if (g < 0) return -1;
    const int v = (int)(std::upper_bound(sb.begin(), sb.end(), g) - sb.begin()) - 1;
    return (int32_t)(((uint32_t)c->uh[v].sector << 24) | (uint32_t)(g - sb[v]));
  };
  for (int i = 0; i < ng; ++i) {
    if (next) next[i] = key(nx[i]);
    if (prev) prev[i] = key(pv[i]);
    if (final_of) final_of[i] = fo[i] >= 0 ? local[fo[i]] : -1;
  }
  return TPCCA_OK;
}

int tpcca_get_vertices(tpcca_ctx_t *c, int32_t slot, tpcca_vertex_t *out, int32_t cap, int32_t *n_out) {
  RCCHK(p2_ready(c));
  if (!n_out) return TPCCA_EINVAL;
  int32_t nv = 0;
  RCCHK(copy_sync(c, &nv, &c->P2.cnt->n_vtx, sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<tpcca_vertex_t> all(nv);
  if (nv) RCCHK(copy_sync(c, all.data(), c->p2vertices.p, sizeof(tpcca_vertex_t) * nv, hipMemcpyDeviceToHost));
  int32_t k = 0;
  for (auto &v : all) {
    if (c->p2_slot_value[v.slot] != slot) continue;
    if (out && k < cap) {
      out[k] = v;
      out[k].slot = slot;
    }
    ++k;
  }
  *n_out = k;
  return cap < k ? TPCCA_ECAPACITY : TPCCA_OK;
}

int tpcca_get_flags(tpcca_ctx_t *c, int32_t slot, int32_t sector, uint8_t *flags, int32_t n) {
  RCCHK(p2_ready(c));
  const int u = find_unit(c, slot, sector);
  if (u < 0) return TPCCA_ESTATE;
  if (!flags || n != c->uh[u].n) return TPCCA_EINVAL;
  if (n) RCCHK(copy_sync(c, flags, ptr<uint8_t>(c->p2flags) + c->units[u].cl_begin, (size_t)n, hipMemcpyDeviceToHost));
  return TPCCA_OK;
}

int tpcca_get_compressed(tpcca_ctx_t *c, int32_t slot, int32_t sector, int32_t *rec, int32_t seg_cap,
                         int32_t *res, int64_t hits_cap, int32_t *n_seg, int64_t *n_hits) {
  RCCHK(p2_ready(c));
  const int u = find_unit(c, slot, sector);
  if (u < 0) return TPCCA_ESTATE;
  if (!n_seg) return TPCCA_EINVAL;
  int32_t sb[2];
  RCCHK(copy_sync(c, sb, ptr<int32_t>(c->p2seg_begin) + u, sizeof(sb), hipMemcpyDeviceToHost));
  tpcca_unit_result_t r;
  RCCHK(copy_sync(c, &r, ptr<tpcca_unit_result_t>(c->unit_res) + u, sizeof(r), hipMemcpyDeviceToHost));
  *n_seg = sb[1] - sb[0];
  if (n_hits) *n_hits = r.n_track_hits;
  if ((rec && seg_cap < *n_seg) || (res && hits_cap < r.n_track_hits)) return TPCCA_ECAPACITY;
  if (rec && *n_seg)
    RCCHK(copy_sync(c, rec, ptr<int32_t>(c->p2rec) + 6 * (int64_t)sb[0], sizeof(int32_t) * 6 * (size_t)*n_seg,
                    hipMemcpyDeviceToHost));
  if (res && r.n_track_hits)
    RCCHK(copy_sync(c, res, ptr<int32_t>(c->p2res) + 4 * r.hit_begin, sizeof(int32_t) * 4 * (size_t)r.n_track_hits,
                    hipMemcpyDeviceToHost));
  return TPCCA_OK;
}

int tpcca_phase2_view(tpcca_ctx_t *c, tpcca_phase2_view_t *out) {
  RCCHK(p2_ready(c));
  if (!out) return TPCCA_EINVAL;
  RCCHK(copy_sync(c, &c->p2c, c->p2cnt.p, sizeof(P2Counts), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->n_seg = c->p2c.n_seg;
  out->n_final = c->p2c.n_final;
  out->n_vertices = c->p2c.n_cand > 0 ? c->p2c.n_vtx : 0;
  out->n_final_hits = c->p2c.n_final_hits;
  out->finals = ptr<tpcca_final_t>(c->p2finals);
  out->final_hits = ptr<int32_t>(c->p2final_hits);
  out->vertices = ptr<tpcca_vertex_t>(c->p2vertices);
  out->flags = ptr<uint8_t>(c->p2flags);
  out->rec = ptr<int32_t>(c->p2rec);
  out->res = ptr<int32_t>(c->p2res);
  out->seg_n_hits = ptr<int32_t>(c->p2seg_nh);
  out->seg_hit_begin = ptr<int64_t>(c->p2seg_hb);
  return TPCCA_OK;
}

int tpcca_decompress(tpcca_ctx_t *c, int32_t n_seg, const int32_t *n_hits, const int64_t *hit_begin,
                     const int32_t *rec, const int32_t *res, int32_t *yq, int32_t *zq, uint8_t *rows) {
  if (!c || n_seg < 0) return TPCCA_EINVAL;
  if (n_seg > 0 && (!n_hits || !hit_begin || !rec || !res || !yq || !zq || !rows)) return TPCCA_EINVAL;
  if (reinterpret_cast<uintptr_t>(res) & 15) return TPCCA_EINVAL;  // read as 16-B records
  hipSetDevice(c->device);
  const P2Params q = p2_dev(c->p2params);
  hipError_t e = p2_launch_decompress(p2_prop_params(c), q, ptr<float>(c->row_x_d), n_seg, n_hits, hit_begin, rec,
                                      res, yq, zq, rows, c->stream);
  if (e != hipSuccess) return dev_err(c, e, "decompress");
  return TPCCA_OK;
}

}  // extern "C"
