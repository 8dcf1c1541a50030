// Continuous-batching server of time frames.
//
// Sec. 5 of the paper plans to track whole time frames (~20 ms of continuous
// read-out) on the GPU, limited by GPU memory, slicing a frame like the
// sectors are sliced today when it does not fit.  Here a time frame is a set
// of sector units; the server:
//   * queues submitted frames (bounded queue, EBUSY when full),
//   * runs n_streams lanes, each a worker thread with its own context, HIP
//     stream and share of the device budget,
//   * lets every free lane pack the next units of all waiting frames, in
//     arrival order, up to its memory share (continuous batching: frames
//     arriving while others are on the GPU join the next batch of any lane;
//     a frame larger than a lane is sliced across batches by sector),
//   * copies each unit's inputs host -> device, replays the tracker graph,
//     copies tracks, hits and assignment back into the frame's buffers, and
//   * stamps the frame's latency when its last unit completes.
// Results of a unit do not depend on the batch it ran in: every stage works
// per unit and decisions compare per-unit cluster IDs only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "tpcca.h"
#include "tpcca_runtime.h"

namespace {

// Device bytes one cluster may need in a lane (inputs, work arrays, tracklet
// slots, outputs, and the growth headroom of buffers and graph buckets).
constexpr int64_t kBytesPerCluster = 800;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  tpcca_timeframe_t tf{};
  std::vector<int32_t> sector, n;
  std::vector<int64_t> begin;
  int next_unit = 0;
  int units_done = 0;
  int64_t track_cursor = 0, hit_cursor = 0, cl_total = 0;
  int status = TPCCA_OK;
  bool done = false;
  double arrival = 0, start = -1, end = 0;
  int64_t n_tracks = 0, n_hits = 0;
  std::vector<int64_t> cl_offset;  // unit -> offset in the assignment array
};

struct Item {
  std::shared_ptr<Request> req;
  int unit;
};

}  // namespace

struct tpcca_server {
  int device = 0;
  size_t budget = 0;
  int n_lanes = 1, max_queue = 64;
  int64_t lane_clusters = 0;
  tpcca_geometry_t geo{};
  std::vector<float> row_x;
  tpcca_params_t params{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;  // requests with units not yet taken
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<std::thread> lanes;
  std::atomic<bool> stop{false};
  uint64_t next_id = 1;
  // stats
  int64_t submitted = 0, completed = 0, rejected = 0, clusters_done = 0, tracks_done = 0;
  int64_t bytes_in_flight = 0;
  int32_t batches = 0;
  int active = 0;
  tpcca_tuning_t tuning{};  // launch schedule of the lanes' contexts
  int tuning_gen = 0;       // 0: none set (context defaults)
  double busy_since = 0, busy_total = 0;
  std::vector<double> latencies;
  std::string last_error;  // text of the last failed batch
  int lanes_up = 0, lanes_failed = 0;  // lanes whose context was (not) created
  int lane_create_status = TPCCA_OK;    // status of the first lane that failed
};

namespace {

void lane_main(tpcca_server *S, int lane) {
  hipSetDevice(S->device);
  tpcca_ctx_t *ctx = nullptr;
  const size_t lane_budget = S->budget / S->n_lanes;
  const int crc = tpcca_create(&S->geo, &S->params, S->device, nullptr, lane_budget, &ctx);
  {
    // server_create waits for every lane's verdict
    std::lock_guard<std::mutex> lk(S->mu);
    if (crc == TPCCA_OK) {
      S->lanes_up++;
    } else {
      if (S->lanes_failed++ == 0) S->lane_create_status = crc;
    }
  }
  S->cv_done.notify_all();
  if (crc != TPCCA_OK) return;
  hipStream_t st = tpcca::ctx_stream(ctx);
  int tuning_gen = 0;
  float4 *d_cl = nullptr;
  uint8_t *d_row = nullptr;
  int64_t d_cap = 0;
  std::vector<tpcca_unit_result_t> ur;
  std::vector<int32_t> bslot, bsector, bn;
  std::vector<int64_t> bbegin;
  for (;;) {
    std::vector<Item> items;
    int64_t ncl = 0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop.load() || !S->queue.empty(); });
      if (S->queue.empty() && S->stop.load()) break;
      // pack units of waiting frames in arrival order up to the lane share
      while (!S->queue.empty()) {
        auto &r = S->queue.front();
        while (r->next_unit < (int)r->n.size()) {
          const int u = r->next_unit;
          const int64_t k = r->n[u];
          if (!items.empty() && ncl + k > S->lane_clusters) break;
          items.push_back({r, u});
          ncl += k;
          r->next_unit++;
          if (r->start < 0) r->start = now_s();
        }
        if (r->next_unit < (int)r->n.size()) break;  // lane full
        S->queue.pop_front();
      }
      if (items.empty()) continue;
      if (S->active++ == 0) S->busy_since = now_s();
      S->bytes_in_flight += ncl * kBytesPerCluster;
    }
    int rc = TPCCA_OK;
    std::string fail_text;
    // a schedule set since this lane's last batch applies from this batch on
    {
      tpcca_tuning_t t{};
      bool apply = false;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->tuning_gen != tuning_gen) {
          t = S->tuning;
          tuning_gen = S->tuning_gen;
          apply = true;
        }
      }
      if (apply && (tpcca_reset(ctx) != TPCCA_OK || tpcca_set_tuning(ctx, &t) != TPCCA_OK)) {
        rc = TPCCA_EINVAL;
        fail_text = std::string("set_tuning: ") + tpcca_last_error(ctx);
      }
    }
    // inputs: one device span per batch, unit slices copied from the frames
    if (ncl > d_cap) {
      std::lock_guard<std::recursive_mutex> dlock(tpcca::device_ops_lock());
      if (d_cl) (void)hipFree(d_cl);
      if (d_row) (void)hipFree(d_row);
      d_cl = nullptr;
      d_row = nullptr;
      d_cap = std::max<int64_t>(ncl, d_cap + d_cap / 2);
      if (hipMalloc(&d_cl, d_cap * sizeof(float4)) != hipSuccess ||
          hipMalloc(&d_row, d_cap) != hipSuccess) {
        (void)hipGetLastError();
        if (d_cl) (void)hipFree(d_cl);
        if (d_row) (void)hipFree(d_row);
        d_cl = nullptr;
        d_row = nullptr;
        rc = TPCCA_ENOMEM;
        d_cap = 0;
      }
    }
    const int U = (int)items.size();
    bslot.resize(U);
    bsector.resize(U);
    bn.resize(U);
    bbegin.resize(U);
    int64_t off = 0;
    for (int i = 0; i < U && rc == TPCCA_OK; ++i) {
      Request &r = *items[i].req;
      const int u = items[i].unit;
      bslot[i] = i;  // distinct slot per unit inside the batch
      bsector[i] = r.sector[u];
      bn[i] = r.n[u];
      bbegin[i] = off;
      if (r.n[u] > 0) {
        if (hipMemcpyAsync(d_cl + off, r.tf.cl + r.begin[u], sizeof(float4) * r.n[u],
                           hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_row + off, r.tf.row + r.begin[u], r.n[u], hipMemcpyHostToDevice, st) !=
                hipSuccess)
          rc = TPCCA_EDEVICE;
      }
      off += r.n[u];
    }
    if (rc == TPCCA_OK) {
      tpcca_batch_t b{};
      b.n_units = U;
      b.slot = bslot.data();
      b.sector = bsector.data();
      b.begin = bbegin.data();
      b.n = bn.data();
      b.cl = reinterpret_cast<const tpcca_cluster_t *>(d_cl);
      b.row = d_row;
      b.flags = TPCCA_MEM_DEVICE | TPCCA_BATCH_GRAPH;
      rc = tpcca_run_batch(ctx, &b);
      if (rc != TPCCA_OK) fail_text = std::string("run_batch: ") + tpcca_last_error(ctx);
    } else {
      if (fail_text.empty()) fail_text = "input staging";
    }
    tpcca_device_results_t dr{};
    if (rc == TPCCA_OK) {
      rc = tpcca_device_results(ctx, &dr);  // synchronises
      if (rc != TPCCA_OK) fail_text = std::string("device_results: ") + tpcca_last_error(ctx);
    }
    if (rc == TPCCA_OK) {
      ur.resize(U);
      if (hipMemcpyAsync(ur.data(), dr.units, sizeof(tpcca_unit_result_t) * U, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        rc = TPCCA_EDEVICE;
        fail_text = "unit results copy";
      }
    }
    // outputs: reserve ranges in each frame's buffers, then copy
    std::vector<int64_t> tpos(U, 0), hpos(U, 0);
    std::vector<int> ok(U, 0);
    if (rc == TPCCA_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (int i = 0; i < U; ++i) {
        Request &r = *items[i].req;
        if (r.track_cursor + ur[i].n_tracks > r.tf.tracks_cap ||
            r.hit_cursor + ur[i].n_track_hits > r.tf.hits_cap) {
          r.status = TPCCA_ECAPACITY;
          continue;
        }
        tpos[i] = r.track_cursor;
        hpos[i] = r.hit_cursor;
        r.track_cursor += ur[i].n_tracks;
        r.hit_cursor += ur[i].n_track_hits;
        ok[i] = 1;
      }
    }
    for (int i = 0; i < U && rc == TPCCA_OK; ++i) {
      if (!ok[i]) continue;
      Request &r = *items[i].req;
      const int u = items[i].unit;
      hipError_t e = hipSuccess;
      if (ur[i].n_tracks && r.tf.tracks)
        e = hipMemcpyAsync(r.tf.tracks + tpos[i], dr.tracks + ur[i].track_begin,
                           sizeof(tpcca_track_t) * ur[i].n_tracks, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess && ur[i].n_track_hits && r.tf.hits)
        e = hipMemcpyAsync(r.tf.hits + hpos[i], dr.hits + ur[i].hit_begin,
                           sizeof(int32_t) * ur[i].n_track_hits, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess && r.n[u] && r.tf.assignment)
        e = hipMemcpyAsync(r.tf.assignment + r.cl_offset[u], dr.assignment + ur[i].cluster_begin,
                           sizeof(int32_t) * r.n[u], hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) {
        rc = TPCCA_EDEVICE;
        fail_text = std::string("result copy: ") + hipGetErrorString(e);
      }
    }
    if (rc == TPCCA_OK) {
      const hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        rc = TPCCA_EDEVICE;
        fail_text = std::string("result copy: ") + hipGetErrorString(e);
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (rc != TPCCA_OK)
        S->last_error = "lane " + std::to_string(lane) + ", batch of " + std::to_string(U) + " units, " +
                        std::to_string(ncl) + " clusters: " + fail_text;
      const double t = now_s();
      for (int i = 0; i < U; ++i) {
        Request &r = *items[i].req;
        const int u = items[i].unit;
        if (rc != TPCCA_OK) r.status = rc;
        if (r.tf.units) {
          tpcca_unit_result_t x = rc == TPCCA_OK ? ur[i] : tpcca_unit_result_t{};
          x.slot = 0;
          x.sector = r.sector[u];
          x.n_clusters = r.n[u];
          x.cluster_begin = r.cl_offset[u];
          x.track_begin = tpos[i];
          x.hit_begin = hpos[i];
          r.tf.units[u] = x;
        }
        if (rc == TPCCA_OK && ok[i]) {
          r.n_tracks += ur[i].n_tracks;
          r.n_hits += ur[i].n_track_hits;
          S->tracks_done += ur[i].n_tracks;
        }
        S->clusters_done += r.n[u];
        if (++r.units_done == (int)r.n.size()) {
          r.done = true;
          r.end = t;
          S->completed++;
          S->latencies.push_back(r.end - r.arrival);
        }
      }
      S->bytes_in_flight -= ncl * kBytesPerCluster;
      S->batches++;
      if (--S->active == 0) S->busy_total += t - S->busy_since;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  {
    std::lock_guard<std::recursive_mutex> dlock(tpcca::device_ops_lock());
    if (d_cl) hipFree(d_cl);
    if (d_row) hipFree(d_row);
  }
  tpcca_destroy(ctx);
  (void)lane;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0;
  std::sort(v.begin(), v.end());
  const double pos = q * (v.size() - 1);
  const size_t a = (size_t)pos;
  const size_t b = std::min(a + 1, v.size() - 1);
  return v[a] + (v[b] - v[a]) * (pos - a);
}

void fill_result(const Request &r, tpcca_result_t *res) {
  res->status = r.status;
  res->done = r.done ? 1 : 0;
  res->n_tracks = r.n_tracks;
  res->n_hits = r.n_hits;
  res->arrival_s = r.arrival;
  res->start_s = r.start;
  res->end_s = r.end;
}

}  // namespace

extern "C" {

double tpcca_now(void) { return now_s(); }

int tpcca_server_create(const tpcca_geometry_t *geo, const tpcca_params_t *params, int device,
                        size_t budget, int32_t n_streams, int32_t max_queue, tpcca_server_t **out) {
  if (!geo || !params || !out || !geo->row_x || n_streams < 1 || n_streams > 16 || max_queue < 1)
    return TPCCA_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return TPCCA_EDEVICE;
  auto *S = new tpcca_server();
  S->device = device;
  S->budget = budget ? budget : ((size_t)64 << 30);
  S->n_lanes = n_streams;
  S->max_queue = max_queue;
  S->row_x.assign(geo->row_x, geo->row_x + geo->n_rows);
  S->geo = *geo;
  S->geo.row_x = S->row_x.data();
  S->params = *params;
  S->lane_clusters = (int64_t)(S->budget / n_streams) / kBytesPerCluster;
  for (int l = 0; l < n_streams; ++l) S->lanes.emplace_back(lane_main, S, l);
  int failed = 0, status = TPCCA_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->lanes_up + S->lanes_failed == S->n_lanes; });
    failed = S->lanes_failed;
    status = S->lane_create_status;
  }
  if (failed) {
    // a lane without a context would leave its share of requests waiting
    // forever: stop the lanes that did start and report the first failure
    S->stop.store(true);
    S->cv_work.notify_all();
    for (auto &t : S->lanes) t.join();
    delete S;
    return status;
  }
  *out = S;
  return TPCCA_OK;
}

int tpcca_server_submit(tpcca_server_t *S, const tpcca_timeframe_t *tf, uint64_t *req_id) {
  if (!S || !tf || !req_id || tf->n_units < 0) return TPCCA_EINVAL;
  if (tf->n_units > 0 && (!tf->sector || !tf->begin || !tf->n)) return TPCCA_EINVAL;
  auto r = std::make_shared<Request>();
  r->tf = *tf;
  r->sector.assign(tf->sector, tf->sector + tf->n_units);
  r->begin.assign(tf->begin, tf->begin + tf->n_units);
  r->n.assign(tf->n, tf->n + tf->n_units);
  r->cl_offset.resize(tf->n_units);
  int64_t tot = 0;
  for (int u = 0; u < tf->n_units; ++u) {
    if (r->n[u] < 0 || r->begin[u] < 0 || r->sector[u] < 0 || r->sector[u] >= S->geo.n_sectors)
      return TPCCA_EINVAL;
    if (r->n[u] > S->lane_clusters) return TPCCA_ENOMEM;
    r->cl_offset[u] = tot;
    tot += r->n[u];
  }
  if (tot > 0 && (!tf->cl || !tf->row)) return TPCCA_EINVAL;
  r->cl_total = tot;
  r->arrival = tf->arrival_s > 0 ? tf->arrival_s : now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop.load()) return TPCCA_ESTATE;
    if ((int)S->queue.size() >= S->max_queue) {
      S->rejected++;
      return TPCCA_EBUSY;
    }
    r->id = S->next_id++;
    S->submitted++;
    S->all[r->id] = r;
    if (tf->n_units == 0) {
      r->done = true;
      r->start = r->end = now_s();
      S->completed++;
      S->latencies.push_back(r->end - r->arrival);
    } else {
      S->queue.push_back(r);
    }
    *req_id = r->id;
  }
  S->cv_work.notify_one();
  return TPCCA_OK;
}

int tpcca_server_poll(tpcca_server_t *S, uint64_t id, tpcca_result_t *res) {
  if (!S || !res) return TPCCA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return TPCCA_ENOTFOUND;
  fill_result(*it->second, res);
  return TPCCA_OK;
}

int tpcca_server_wait(tpcca_server_t *S, uint64_t id, double timeout_s, tpcca_result_t *res) {
  if (!S || !res) return TPCCA_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return TPCCA_ENOTFOUND;
  auto r = it->second;
  const auto dl = std::chrono::steady_clock::now() +
                  std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                      std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
  if (!S->cv_done.wait_until(lk, dl, [&] { return r->done; })) {
    fill_result(*r, res);
    return TPCCA_EBUSY;
  }
  fill_result(*r, res);
  return TPCCA_OK;
}

int tpcca_server_release(tpcca_server_t *S, uint64_t id) {
  if (!S) return TPCCA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return TPCCA_ENOTFOUND;
  if (!it->second->done) return TPCCA_ESTATE;
  S->all.erase(it);
  return TPCCA_OK;
}

const char *tpcca_server_last_error(tpcca_server_t *S) {
  static thread_local std::string copy;
  if (!S) return "";
  std::lock_guard<std::mutex> lk(S->mu);
  copy = S->last_error;
  return copy.c_str();
}

int tpcca_server_stats(tpcca_server_t *S, tpcca_stats_t *st) {
  if (!S || !st) return TPCCA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->rejected = S->rejected;
  st->clusters_done = S->clusters_done;
  st->tracks_done = S->tracks_done;
  st->bytes_in_flight = S->bytes_in_flight;
  st->bytes_budget = (int64_t)S->budget;
  st->queue_depth = (int32_t)S->queue.size();
  st->batches_run = S->batches;
  st->busy_s = S->busy_total + (S->active ? now_s() - S->busy_since : 0.0);
  st->p50_ms = percentile(S->latencies, 0.50) * 1e3;
  st->p99_ms = percentile(S->latencies, 0.99) * 1e3;
  double m = 0;
  for (double v : S->latencies) m += v;
  st->mean_ms = S->latencies.empty() ? 0 : m / S->latencies.size() * 1e3;
  return TPCCA_OK;
}

int tpcca_server_set_tuning(tpcca_server_t *S, const tpcca_tuning_t *t) {
  if (!S || !t || !tpcca::tuning_valid(t, S->geo.n_rows)) return TPCCA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  S->tuning = *t;
  ++S->tuning_gen;
  return TPCCA_OK;
}

int tpcca_server_reset_stats(tpcca_server_t *S) {
  if (!S) return TPCCA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  S->submitted = S->completed = S->rejected = S->clusters_done = S->tracks_done = 0;
  S->batches = 0;
  S->busy_total = 0;
  if (S->active) S->busy_since = now_s();
  S->latencies.clear();
  return TPCCA_OK;
}

int tpcca_server_destroy(tpcca_server_t *S) {
  if (!S) return TPCCA_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop.store(true);
  }
  S->cv_work.notify_all();
  for (auto &t : S->lanes) t.join();
  delete S;
  return TPCCA_OK;
}

}  // extern "C"
