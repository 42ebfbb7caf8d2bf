// Request loop over resident factorizations: continuous batching with
// memory admission (see include/mbf.h, "Serving").
//
// A dispatcher thread owns `nslots` HIP streams.  Submitted requests wait in
// a FIFO.  Whenever a slot is free, the dispatcher forms a batch from the
// oldest request and every queued request on the same (factor, precision),
// up to max_batch_rhs columns, reserves the batch's staging and workspace
// bytes from the server's device pool (admission: the batch waits while the
// pool cannot hold it), and enqueues on the slot's stream:
//   gather the requests' g columns into one contiguous block,
//   one mbf_apply over all columns (the factor is read once per batch),
//   scatter the result columns to each request's u,
//   an event marking completion.
// Batches on different slots overlap on the device.  Completion is observed
// by polling the events; a request's latency is completion - submission on
// the host clock.
//
// Graph mode (MBF_SERVER_GRAPHS): each slot keeps one fixed region of the
// pool for its staging blocks and workspace, sized for the largest batch it
// has run (grown when a larger one comes, which drops the slot's graphs; the
// regions of idle slots are given back when the pool cannot otherwise hold a
// growth).  The apply's launches for a (factor, precision, batch width) are
// captured once on the slot's stream into a HIP graph and replayed for every
// later batch of that kind; batch widths are rounded up to a power of two of
// at least 16 columns (within max_batch_rhs) so that few graphs serve every
// mix, the padding columns computing results nobody reads (the apply treats
// every column on its own).  Per batch the slot issues the gather copies, one
// graph launch and the scatter copies.
//
// Admission never fails a request that fits alone: when a batch of several
// requests exceeds the pool, trailing requests are left in the queue until
// the batch fits; only a request whose own staging and workspace exceed the
// whole budget completes with MBF_ERR_OOM.  A batch whose apply cannot be
// enqueued completes each of its requests with that error.  Records of
// completed requests are kept until polled (at most kMaxRecords; the oldest
// unpolled ones are dropped beyond that); the latency statistics keep the
// last kMaxLatencies completions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "device.h"
#include "factor.h"


namespace mbf {
namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t id;
  mbf_factor f;
  int prec;
  int64_t nrhs;
  const void* g;
  int64_t ldg;
  void* u;
  int64_t ldu;
  hipEvent_t ready;  // g is complete once this event has completed (null: already complete)
  clk::time_point t_submit;
};

struct Record {
  double latency_us;
  mbf_status st;
};

constexpr size_t kMaxRecords = (size_t)1 << 20;
constexpr size_t kMaxLatencies = (size_t)1 << 20;

// First-fit allocator over one device allocation (offsets 256-byte aligned).
struct Pool {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  bool init(size_t bytes) {
    size = bytes;
    if (hipMalloc((void**)&base, bytes) != hipSuccess) {
      base = nullptr;
      return false;
    }
    free_[0] = bytes;
    return true;
  }
  size_t alloc(size_t bytes) {  // returns SIZE_MAX when full
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        return off;
      }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

using GraphKey = std::tuple<uint64_t, int, int64_t>;  // factor serial, precision, batch width

constexpr size_t kMaxGraphsPerSlot = 256;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  mbf_status st = MBF_OK;  // status given to every request of the batch
  std::vector<Request> reqs;
  size_t off = 0, bytes = 0;  // the batch's reservation (direct launches)
  // graph mode: the slot's fixed region and its captured applies
  size_t fix_off = SIZE_MAX, fix_bytes = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
};

// Smallest power of two >= max(cols, 16), kept within max(max_rhs, cols).
int64_t batch_width(int64_t cols, int64_t max_rhs) {
  int64_t w = 16;
  while (w < cols) w *= 2;
  return std::max(cols, std::min(w, max_rhs));
}

}  // namespace

struct Server {
  int device = 0;
  Pool pool;
  std::vector<Slot> slots;
  int64_t max_batch_rhs = 256;
  bool use_graphs = false;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::map<uint64_t, Record> records;  // completed, not yet polled
  std::vector<double> latencies;       // ring of the last kMaxLatencies completions
  size_t lat_next = 0;
  uint64_t lat_count = 0;
  std::atomic<uint64_t> next_id{1};
  bool stop = false;
  std::string error;
  int64_t batches = 0, rhs_done = 0, requests_done = 0, max_concurrent = 0, graphs_captured = 0,
          graph_batches = 0;
  clk::time_point t_first{}, t_last{};
  std::thread th;

  size_t batch_bytes(const Request& r, int64_t nrhs) const {
    const DevFactor& F = r.f->dev;
    const size_t es = r.prec == MBF_C128 ? 16 : 8;
    const size_t io = (size_t)(F.nxi + F.nx) * (size_t)nrhs * es;
    return (io + 255) / 256 * 256 + workspace_bytes(F, r.prec, nrhs);
  }

  void complete(const Request& r, mbf_status st, clk::time_point now) {
    const double us = std::chrono::duration<double, std::micro>(now - r.t_submit).count();
    if (records.size() >= kMaxRecords) records.erase(records.begin());
    records[r.id] = Record{us, st};
    if (st != MBF_OK) return;
    if (latencies.size() < kMaxLatencies) {
      latencies.push_back(us);
    } else {
      latencies[lat_next] = us;
      lat_next = (lat_next + 1) % kMaxLatencies;
    }
    ++lat_count;
    rhs_done += r.nrhs;
    ++requests_done;
  }

  // Launch one batch on slot s; called with mu held.
  bool launch(Slot& s) {
    if (queue.empty()) return false;
    const Request head = queue.front();
    std::vector<size_t> take;
    int64_t cols = 0;
    for (size_t i = 0; i < queue.size(); ++i) {
      const Request& r = queue[i];
      if (r.f != head.f || r.prec != head.prec) continue;
      if (cols > 0 && cols + r.nrhs > max_batch_rhs) break;
      take.push_back(i);
      cols += r.nrhs;
    }
    // Leave trailing requests queued until the batch fits the pool.
    while (take.size() > 1 && batch_bytes(head, cols) > pool.size) {
      cols -= queue[take.back()].nrhs;
      take.pop_back();
    }
    if (batch_bytes(head, cols) > pool.size) {
      // the head request alone can never fit: it fails, the rest proceed
      error = "request larger than the server memory budget";
      complete(head, MBF_ERR_OOM, clk::now());
      queue.pop_front();
      return true;
    }
    // columns of the apply: the batch's own, or its graph width
    int64_t width = cols;
    if (use_graphs) {
      width = batch_width(cols, max_batch_rhs);
      if (batch_bytes(head, width) > pool.size) width = cols;
    }
    const size_t need = batch_bytes(head, width);
    size_t off;
    if (use_graphs) {
      if (s.fix_bytes < need) {
        // grow to the factorization's widest batch when every slot could hold
        // one that size, so that the region (and its graphs) stays put
        const size_t full = batch_bytes(head, batch_width(max_batch_rhs, max_batch_rhs));
        const bool roomy = full > need && full <= pool.size / slots.size();
        if (!(roomy && grow_region(s, full, false)) && !grow_region(s, need, true)) return false;  // admission: wait
      }
      off = s.fix_off;
    } else {
      off = pool.alloc(need);
      if (off == SIZE_MAX) return false;  // admission: wait for memory
    }
    const DevFactor& F = head.f->dev;
    const size_t es = head.prec == MBF_C128 ? 16 : 8;
    char* gb = pool.base + off;
    char* ub = gb + (size_t)F.nxi * width * es;
    const size_t io = (size_t)(F.nxi + F.nx) * (size_t)width * es;
    char* ws = pool.base + off + (io + 255) / 256 * 256;
    const size_t ws_bytes = need - (size_t)(ws - gb);
    s.reqs.clear();
    s.st = MBF_OK;
    hipGraphExec_t exec = nullptr;
    if (use_graphs) {
      // capture before this batch's copies are on the (idle) stream
      Error e = slot_graph(s, head, width, gb, ub, ws, ws_bytes, &exec);
      if (e.st != MBF_OK) {
        error = e.msg;
        s.st = e.st;
      }
    }
    int64_t c0 = 0;
    for (size_t k = 0; k < take.size(); ++k) {
      const Request& r = queue[take[k]];
      if (r.ready && hipStreamWaitEvent(s.stream, r.ready, 0) != hipSuccess) s.st = MBF_ERR_HIP;
      if (hipMemcpy2DAsync(gb + (size_t)c0 * F.nxi * es, (size_t)F.nxi * es, r.g, (size_t)r.ldg * es,
                           (size_t)F.nxi * es, (size_t)r.nrhs, hipMemcpyDeviceToDevice, s.stream) != hipSuccess)
        s.st = MBF_ERR_HIP;
      c0 += r.nrhs;
      s.reqs.push_back(r);
    }
    if (s.st == MBF_OK) {
      if (exec) {
        if (hipGraphLaunch(exec, s.stream) != hipSuccess) {
          error = "graph launch failed";
          s.st = MBF_ERR_HIP;
        }
        ++graph_batches;
      } else {
        Error e = launch_apply(F, head.prec, false, cols, gb, F.nxi, ub, F.nx, ws, ws_bytes, s.stream);
        if (e.st != MBF_OK) {
          error = e.msg;
          s.st = e.st;
        }
      }
    }
    if (s.st == MBF_OK) {
      c0 = 0;
      for (const Request& r : s.reqs) {
        if (hipMemcpy2DAsync(r.u, (size_t)r.ldu * es, ub + (size_t)c0 * F.nx * es, (size_t)F.nx * es,
                             (size_t)F.nx * es, (size_t)r.nrhs, hipMemcpyDeviceToDevice, s.stream) != hipSuccess)
          s.st = MBF_ERR_HIP;
        c0 += r.nrhs;
      }
    }
    if (s.st != MBF_OK && error.empty()) error = "batch enqueue failed";
    (void)hipEventRecord(s.done, s.stream);
    for (size_t k = take.size(); k-- > 0;) queue.erase(queue.begin() + (std::ptrdiff_t)take[k]);
    s.busy = true;
    s.off = off;
    s.bytes = use_graphs ? 0 : need;
    ++batches;
    return true;
  }

  // Graph mode: give slot s a fixed region of at least `need` bytes (its
  // graphs point into the old one and are dropped).  When the pool cannot
  // hold it and `evict` is set, the regions of idle slots are released too;
  // false when it does not fit (the batch waits).
  bool grow_region(Slot& s, size_t need, bool evict) {
    auto release = [&](Slot& t) {
      t.drop_graphs();
      if (t.fix_off != SIZE_MAX) pool.release(t.fix_off, t.fix_bytes);
      t.fix_off = SIZE_MAX;
      t.fix_bytes = 0;
    };
    release(s);
    size_t off = pool.alloc(need);
    if (off == SIZE_MAX && evict) {
      for (auto& t : slots)
        if (&t != &s && !t.busy) release(t);
      off = pool.alloc(need);
    }
    if (off == SIZE_MAX) return false;
    s.fix_off = off;
    s.fix_bytes = need;
    return true;
  }

  // Graph mode: the captured apply of `width` columns of the head request's
  // factorization from the slot's staging g block into its u block.
  Error slot_graph(Slot& s, const Request& head, int64_t width, char* gb, char* ub, char* ws, size_t ws_bytes,
                   hipGraphExec_t* exec) {
    const GraphKey key{head.f->serial, head.prec, width};
    auto it = s.graphs.find(key);
    if (it != s.graphs.end()) {
      *exec = it->second;
      return {MBF_OK, ""};
    }
    if (s.graphs.size() >= kMaxGraphsPerSlot) s.drop_graphs();
    const DevFactor& F = head.f->dev;
    if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return {MBF_ERR_HIP, "hipStreamBeginCapture failed"};
    Error e = launch_apply(F, head.prec, false, width, gb, F.nxi, ub, F.nx, ws, ws_bytes, s.stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s.stream, &g);
    if (e.st == MBF_OK && ec != hipSuccess) e = {MBF_ERR_HIP, "hipStreamEndCapture failed"};
    hipGraphExec_t x = nullptr;
    if (e.st == MBF_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess)
      e = {MBF_ERR_HIP, "hipGraphInstantiate failed"};
    if (g) (void)hipGraphDestroy(g);
    if (e.st != MBF_OK) return e;
    s.graphs[key] = x;
    ++graphs_captured;
    *exec = x;
    return {MBF_OK, ""};
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      // completions
      int64_t active = 0;
      for (auto& s : slots) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q != hipErrorNotReady) {
          const auto now = clk::now();
          if (q != hipSuccess && s.st == MBF_OK) {
            s.st = MBF_ERR_HIP;
            error = std::string("batch failed on the device: ") + hipGetErrorString(q);
          }
          for (const Request& r : s.reqs) complete(r, s.st, now);
          t_last = now;
          if (s.bytes) pool.release(s.off, s.bytes);
          s.busy = false;
          s.reqs.clear();
        } else {
          ++active;
        }
      }
      // admissions
      bool progressed = true;
      while (progressed && !queue.empty()) {
        progressed = false;
        for (auto& s : slots)
          if (!s.busy && launch(s)) {
            progressed = true;
            if (s.busy) ++active;
            break;
          }
      }
      max_concurrent = std::max(max_concurrent, active);
      if (stop && queue.empty() && active == 0) break;
      cv.notify_all();
      cv.wait_for(lk, std::chrono::microseconds(active ? 20 : 500));
    }
    cv.notify_all();
  }
};

}  // namespace mbf

using mbf::Server;
struct mbf_server_s : Server {};

extern "C" {

mbf_status mbf_server_create(size_t mem_budget, int32_t nslots, int64_t max_batch_rhs, uint32_t flags,
                             mbf_server* out) {
  if (!out || mem_budget == 0 || nslots <= 0 || nslots > 64 || max_batch_rhs <= 0 || (flags & ~MBF_SERVER_GRAPHS)) {
    mbf::set_error("invalid server arguments");
    return MBF_ERR_INVALID_ARG;
  }
  *out = nullptr;
  mbf_server_s* s = new mbf_server_s();
  (void)hipGetDevice(&s->device);
  if (!s->pool.init(mem_budget)) {
    delete s;
    mbf::set_error("server memory budget allocation failed");
    return MBF_ERR_OOM;
  }
  s->max_batch_rhs = max_batch_rhs;
  s->use_graphs = (flags & MBF_SERVER_GRAPHS) != 0;
  s->slots.resize(nslots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      mbf::set_error("stream/event creation failed");
      for (auto& q : s->slots) {
        if (q.stream) (void)hipStreamDestroy(q.stream);
        if (q.done) (void)hipEventDestroy(q.done);
      }
      (void)hipFree(s->pool.base);
      delete s;
      return MBF_ERR_HIP;
    }
  }
  s->th = std::thread([s]() { s->loop(); });
  *out = s;
  return MBF_OK;
}

mbf_status mbf_server_submit(mbf_server srv, mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg,
                             void* u, int64_t ldu, void* ready_event, uint64_t* id) {
  Server* s = srv;
  if (!s || !f || !g || !u || !id || nrhs <= 0 || p < 0 || p >= mbf::kNumPrec) {
    mbf::set_error("invalid submit arguments");
    return MBF_ERR_INVALID_ARG;
  }
  if (!(f->dev.prec_mask & (1u << p))) {
    mbf::set_error("precision not built for this factor");
    return MBF_ERR_UNSUPPORTED;
  }
  if (ldg < f->dev.nxi || ldu < f->dev.nx) {
    mbf::set_error("leading dimension too small");
    return MBF_ERR_INVALID_ARG;
  }
  mbf::Request r{s->next_id++, f, (int)p, nrhs, g, ldg, u, ldu, (hipEvent_t)ready_event, mbf::clk::now()};
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      mbf::set_error("server is shutting down");
      return MBF_ERR_BUSY;
    }
    if (s->requests_done == 0 && s->queue.empty()) s->t_first = r.t_submit;
    s->queue.push_back(r);
  }
  s->cv.notify_all();
  *id = r.id;
  return MBF_OK;
}

mbf_status mbf_server_poll(mbf_server srv, uint64_t id, int32_t* done, double* latency_us) {
  Server* s = srv;
  if (!s || !done) {
    mbf::set_error("invalid poll arguments");
    return MBF_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *done = 0;
  if (latency_us) *latency_us = 0.0;
  auto it = s->records.find(id);
  if (it == s->records.end()) {
    // still queued or in flight, or never issued / already reported
    bool pending = false;
    for (const auto& r : s->queue) pending = pending || r.id == id;
    for (const auto& sl : s->slots)
      for (const auto& r : sl.reqs) pending = pending || (sl.busy && r.id == id);
    if (pending) return MBF_OK;
    mbf::set_error("unknown request id (never issued, or its completion was already reported)");
    return MBF_ERR_INVALID_ARG;
  }
  const mbf::Record rec = it->second;
  s->records.erase(it);
  *done = 1;
  if (latency_us) *latency_us = rec.latency_us;
  if (rec.st != MBF_OK) {
    mbf::set_error(s->error.empty() ? "request failed" : s->error);
    return rec.st;
  }
  return MBF_OK;
}

mbf_status mbf_server_drain(mbf_server srv) {
  Server* s = srv;
  if (!s) return MBF_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&]() {
    if (!s->queue.empty()) return false;
    for (auto& sl : s->slots)
      if (sl.busy) return false;
    return true;
  });
  if (!s->error.empty()) {
    mbf::set_error(s->error);
    return MBF_ERR_HIP;
  }
  return MBF_OK;
}

mbf_status mbf_server_stats(mbf_server srv, mbf_server_stats_t* out) {
  Server* s = srv;
  if (!s || !out) return MBF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  std::vector<double> v = s->latencies;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) { return v.empty() ? 0.0 : v[std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5))]; };
  out->requests = s->requests_done;
  out->rhs = s->rhs_done;
  out->batches = s->batches;
  out->max_concurrent_batches = s->max_concurrent;
  out->graphs_captured = s->graphs_captured;
  out->graph_batches = s->graph_batches;
  out->p50_us = pct(0.50);
  out->p99_us = pct(0.99);
  out->mean_us = v.empty() ? 0.0 : [&]() { double t = 0; for (double x : v) t += x; return t / v.size(); }();
  out->wall_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
  return MBF_OK;
}

void mbf_server_destroy(mbf_server srv) {
  mbf_server_s* s = srv;
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  int prev = 0;
  const bool switch_dev = hipGetDevice(&prev) == hipSuccess && prev != s->device;
  if (switch_dev) (void)hipSetDevice(s->device);  // the side streams were made on the server's device
  for (auto& sl : s->slots) {
    (void)hipStreamSynchronize(sl.stream);
    sl.drop_graphs();
    mbf::release_side_streams(sl.stream);
    (void)hipStreamDestroy(sl.stream);
    (void)hipEventDestroy(sl.done);
  }
  (void)hipFree(s->pool.base);
  if (switch_dev) (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
