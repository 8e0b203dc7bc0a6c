// Continuous-batching server over resident grids (gp_serve_* in include/gp.h).
//
// Slots.  The server owns n slots (bounded by the memory budget).  A slot is a HIP
// stream plus fixed device buffers for `slot_points` points: inputs, outputs and a
// query workspace.  A request occupies one slot while it runs; requests larger than a
// slot are processed chunk by chunk on that slot (every point is independent, so
// chunking is exact).  Different slots run concurrently, so requests that arrive while
// others are on the GPU overlap with them on the device.
//
// Graphs.  For each (slot, kind, size bucket) the query pipeline is captured once into
// a hipGraph and replayed.  Buckets are powers of two from 1024 up to the slot size;
// a chunk of n points runs the graph of the smallest bucket >= n with the tail of the
// slot's input filled with NaN, which the filter leaves unpaired (no refinement work).
//
// A single server thread admits queued requests (FIFO) onto free slots, enqueues their
// copies and graph launches, and polls slot events to complete tickets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gp_internal.h"

namespace gp {
gp_status set_error(gp_status code, const char *fmt, ...);
gp_status run_query_tuned(const gp_grid *g, gp_kind kind, int64_t n, const double *px,
                          const double *py, int32_t *out_id, double *out_dist,
                          gp_precision prec, void *ws, size_t ws_bytes, hipStream_t s,
                          gp_stats *stats, const gp_tuning *t);
}  // namespace gp

using namespace gp;
using Clock = std::chrono::steady_clock;

namespace {

__global__ void k_fill_nan(double *x, double *y, int64_t lo, int64_t hi) {
  for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = __builtin_nan("");
    y[i] = __builtin_nan("");
  }
}

struct Request {
  uint64_t ticket;
  gp_kind kind;
  int64_t n;
  const double *px, *py;
  int32_t *out_id;
  double *out_dist;
  Clock::time_point t_submit;
  int done = 0;
  gp_status status = GP_OK;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  double *px = nullptr, *py = nullptr, *dist = nullptr;
  int32_t *id = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  unsigned long long *h_tests = nullptr;  // pinned: test count of each chunk
  int max_chunks = 0;
  std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;
  Request *req = nullptr;  // in flight
  int nchunks = 0;
};

}  // namespace

struct gp_server {
  const gp_grid *grid[3] = {nullptr, nullptr, nullptr};
  gp_serve_opts opts;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false, closed = false;
  std::thread th;
  // statistics
  std::vector<double> lat_us;
  int64_t completed = 0, failed = 0, points = 0, replays = 0;
  unsigned long long tests = 0;
  Clock::time_point t_first, t_last;
  bool any = false;
};

static int64_t bucket_for(int64_t n, int64_t cap) {
  int64_t b = 1024;
  while (b < n && b < cap) b <<= 1;
  return std::min(b, cap);
}

// Enqueue one chunk [lo, lo+m) of request r on slot sl.  Called by the server thread.
static gp_status enqueue_chunk(gp_server *srv, Slot &sl, Request *r, int64_t lo, int64_t m,
                               int chunk_idx) {
  const gp_serve_opts &o = srv->opts;
  const hipMemcpyKind in_kind = o.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind out_kind = o.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipStream_t s = sl.stream;
  const gp_grid *g = srv->grid[r->kind];
  const int64_t b = o.use_graphs ? bucket_for(m, o.slot_points) : m;
#define SV_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(GP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)
  SV_TRY(hipMemcpyAsync(sl.px, r->px + lo, (size_t)m * 8, in_kind, s));
  SV_TRY(hipMemcpyAsync(sl.py, r->py + lo, (size_t)m * 8, in_kind, s));
  if (b > m) {
    hipLaunchKernelGGL(k_fill_nan, dim3(256), dim3(256), 0, s, sl.px, sl.py, m, b);
    SV_TRY(hipGetLastError());
  }
  const gp_precision prec = (gp_precision)o.precision;
  Workspace w;
  workspace_layout(*(const Grid *)g, b, prec, sl.ws, &w);
  // A request's points spread over the grid's cells, so a small bucket has few points
  // per cell: keep work items to one wavefront and fewer points per lane there.
  gp_tuning tn = ((const Grid *)g)->tune[prec];
  tn.waves_per_item = 1;
  const int ppl_cap = b >= (1 << 20) ? 4 : b >= (1 << 17) ? 2 : 1;
  if (tn.points_per_lane > ppl_cap) tn.points_per_lane = ppl_cap;
  if (o.use_graphs) {
    auto key = std::make_pair((int)r->kind, b);
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
      hipGraph_t graph;
      SV_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      gp_status rc = run_query_tuned(g, r->kind, b, sl.px, sl.py, sl.id, sl.dist, prec, sl.ws,
                                     sl.ws_bytes, s, nullptr, &tn);
      hipError_t ec = hipStreamEndCapture(s, &graph);
      if (rc) return rc;
      SV_TRY(ec);
      hipGraphExec_t exec;
      SV_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(graph);
      it = sl.graphs.emplace(key, exec).first;
    }
    SV_TRY(hipGraphLaunch(it->second, s));
    srv->replays++;
  } else {
    gp_status rc = run_query_tuned(g, r->kind, b, sl.px, sl.py, sl.id, sl.dist, prec, sl.ws,
                                   sl.ws_bytes, s, nullptr, &tn);
    if (rc) return rc;
  }
  SV_TRY(hipMemcpyAsync(r->out_id + lo, sl.id, (size_t)m * 4, out_kind, s));
  if (r->kind == GP_P2P)
    SV_TRY(hipMemcpyAsync(r->out_dist + lo, sl.dist, (size_t)m * 8, out_kind, s));
  SV_TRY(hipMemcpyAsync(sl.h_tests + chunk_idx, w.tests, 8, hipMemcpyDeviceToHost, s));
#undef SV_TRY
  return GP_OK;
}

static void complete(gp_server *srv, Slot &sl, gp_status st) {
  Request *r = sl.req;
  auto now = Clock::now();
  std::lock_guard<std::mutex> lk(srv->mu);
  r->status = st;
  r->done = 1;
  if (st == GP_OK) {
    srv->completed++;
    srv->points += r->n;
    for (int c = 0; c < sl.nchunks; ++c) srv->tests += sl.h_tests[c];
    srv->lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
    if (!srv->any) { srv->t_first = r->t_submit; srv->any = true; }
    srv->t_last = now;
  } else {
    srv->failed++;
  }
  sl.req = nullptr;
  sl.nchunks = 0;
  srv->cv_done.notify_all();
}

static void server_loop(gp_server *srv) {
  // the device the grids live on (a new host thread starts on device 0)
  const gp_grid *g0 = srv->grid[GP_PIP] ? srv->grid[GP_PIP] : srv->grid[GP_P2P];
  (void)hipSetDevice(((const Grid *)g0)->device);
  for (;;) {
    bool busy = false;
    // completions
    for (Slot &sl : srv->slots) {
      if (!sl.req) continue;
      busy = true;
      hipError_t q = hipEventQuery(sl.done_ev);
      if (q == hipSuccess) complete(srv, sl, GP_OK);
      else if (q != hipErrorNotReady) {
        set_error(GP_E_HIP, "request failed on the device: %s", hipGetErrorString(q));
        complete(srv, sl, GP_E_HIP);
      }
    }
    // admissions: FIFO onto free slots
    for (Slot &sl : srv->slots) {
      if (sl.req) continue;
      Request *r = nullptr;
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->queue.empty()) break;
        r = srv->queue.front();
        srv->queue.pop_front();
      }
      sl.req = r;
      busy = true;
      const int64_t P = srv->opts.slot_points;
      const int nch = (int)((r->n + P - 1) / P);
      gp_status st = GP_OK;
      if (nch > sl.max_chunks) {
        unsigned long long *nt = nullptr;
        if (hipHostMalloc((void **)&nt, (size_t)nch * 8, hipHostMallocDefault) != hipSuccess) {
          st = set_error(GP_E_OOM, "pinned allocation failed");
        } else {
          if (sl.h_tests) (void)hipHostFree(sl.h_tests);
          sl.h_tests = nt;
          sl.max_chunks = nch;
        }
      }
      sl.nchunks = nch;
      for (int c = 0; c < nch && st == GP_OK; ++c) {
        const int64_t lo = (int64_t)c * P;
        st = enqueue_chunk(srv, sl, r, lo, std::min(P, r->n - lo), c);
      }
      if (st == GP_OK && hipEventRecord(sl.done_ev, sl.stream) != hipSuccess)
        st = set_error(GP_E_HIP, "hipEventRecord failed");
      if (st != GP_OK) {
        (void)hipStreamSynchronize(sl.stream);
        complete(srv, sl, st);
      }
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    const bool idle = !busy && srv->queue.empty();
    if (idle && srv->stopping) break;
    if (idle) srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

static void free_server(gp_server *srv) {
  for (Slot &sl : srv->slots) {
    for (auto &kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    (void)hipFree(sl.px);
    (void)hipFree(sl.py);
    (void)hipFree(sl.id);
    (void)hipFree(sl.dist);
    (void)hipFree(sl.ws);
    if (sl.h_tests) (void)hipHostFree(sl.h_tests);
  }
  for (auto &kv : srv->reqs) delete kv.second;
  delete srv;
}

extern "C" gp_status gp_serve_create(const gp_grid *pip_grid, const gp_grid *p2p_grid,
                                     const gp_serve_opts *opts, gp_server **out) {
  if (!out || !opts) return set_error(GP_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (!pip_grid && !p2p_grid) return set_error(GP_E_INVALID_ARG, "no grid given");
  if ((pip_grid && ((const Grid *)pip_grid)->kind != GP_PIP) ||
      (p2p_grid && ((const Grid *)p2p_grid)->kind != GP_P2P))
    return set_error(GP_E_INVALID_ARG, "grid kinds do not match their arguments");
  gp_serve_opts o = *opts;
  if (o.n_slots < 1 || o.n_slots > 16) return set_error(GP_E_INVALID_ARG, "n_slots must be 1..16");
  if (o.slot_points < 1024 || o.slot_points >= ((int64_t)1 << 30))
    return set_error(GP_E_INVALID_ARG, "slot_points must be in [1024, 2^30)");
  if (o.precision != GP_FP64 && o.precision != GP_MIXED)
    return set_error(GP_E_INVALID_ARG, "bad precision");
  if (o.max_queue <= 0) o.max_queue = 1 << 20;
  // device bytes one slot needs at full size
  size_t ws = 0;
  for (const gp_grid *g : {pip_grid, p2p_grid})
    if (g) {
      size_t b = 0;
      gp_status rc = gp_workspace_bytes(g, o.slot_points, (gp_precision)o.precision, &b);
      if (rc) return rc;
      ws = std::max(ws, b);
    }
  const size_t per_slot = ws + (size_t)o.slot_points * (8 + 8 + 4 + 8) + 4096;
  int n_slots = (int)std::min<int64_t>(o.n_slots, o.mem_budget / (int64_t)per_slot);
  if (n_slots < 1)
    return set_error(GP_E_OOM, "memory budget %lld below one slot (%zu bytes)",
                     (long long)o.mem_budget, per_slot);
  o.n_slots = n_slots;
  gp_server *srv = new gp_server();
  srv->grid[GP_PIP] = pip_grid;
  srv->grid[GP_P2P] = p2p_grid;
  srv->opts = o;
  srv->slots.resize(n_slots);
  for (Slot &sl : srv->slots) {
    const size_t P = (size_t)o.slot_points;
    bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&sl.px, P * 8) == hipSuccess && hipMalloc(&sl.py, P * 8) == hipSuccess &&
              hipMalloc(&sl.id, P * 4) == hipSuccess && hipMalloc(&sl.dist, P * 8) == hipSuccess &&
              hipMalloc(&sl.ws, ws) == hipSuccess;
    sl.ws_bytes = ws;
    if (!ok) {
      free_server(srv);
      return set_error(GP_E_OOM, "slot allocation failed");
    }
  }
  srv->th = std::thread(server_loop, srv);
  *out = srv;
  return GP_OK;
}

extern "C" gp_status gp_serve_submit(gp_server *srv, gp_kind kind, int64_t n, const double *px,
                                     const double *py, int32_t *out_id, double *out_dist,
                                     uint64_t *ticket) {
  if (!srv || !ticket) return set_error(GP_E_INVALID_ARG, "null argument");
  if (kind != GP_PIP && kind != GP_P2P) return set_error(GP_E_INVALID_ARG, "bad kind");
  if (!srv->grid[kind]) return set_error(GP_E_INVALID_ARG, "server has no grid of this kind");
  if (n < 0 || n >= ((int64_t)1 << 31)) return set_error(GP_E_CAPACITY, "n must be in [0, 2^31)");
  if (n > 0 && (!px || !py || !out_id || (kind == GP_P2P && !out_dist)))
    return set_error(GP_E_INVALID_ARG, "null point or output pointer");
  Request *r = new Request();
  r->kind = kind;
  r->n = n;
  r->px = px;
  r->py = py;
  r->out_id = out_id;
  r->out_dist = out_dist;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->closed || srv->stopping) {
    delete r;
    return set_error(GP_E_CLOSED, "server is shut down");
  }
  if ((int64_t)srv->queue.size() >= srv->opts.max_queue) {
    delete r;
    return set_error(GP_E_BUSY, "request queue is full");
  }
  r->ticket = srv->next_ticket++;
  srv->reqs[r->ticket] = r;
  *ticket = r->ticket;
  if (n == 0) {
    r->done = 1;
    srv->completed++;
    srv->lat_us.push_back(0.0);
    srv->cv_done.notify_all();
  } else {
    srv->queue.push_back(r);
    srv->cv_work.notify_one();
  }
  return GP_OK;
}

extern "C" gp_status gp_serve_poll(gp_server *srv, uint64_t ticket, int32_t *done) {
  if (!srv || !done) return set_error(GP_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(GP_E_NOT_FOUND, "unknown ticket");
  *done = it->second->done;
  return GP_OK;
}

extern "C" gp_status gp_serve_wait(gp_server *srv, uint64_t ticket, int64_t timeout_us) {
  if (!srv) return set_error(GP_E_INVALID_ARG, "null argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(GP_E_NOT_FOUND, "unknown ticket");
  Request *r = it->second;
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, [&] { return r->done != 0; });
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                    [&] { return r->done != 0; })) {
    return set_error(GP_E_TIMEOUT, "ticket %llu not complete", (unsigned long long)ticket);
  }
  gp_status st = r->status;
  if (st != GP_OK) set_error(st, "request %llu failed", (unsigned long long)ticket);
  return st;
}

extern "C" gp_status gp_serve_stats_get(gp_server *srv, gp_serve_stats *out) {
  if (!srv || !out) return set_error(GP_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  memset(out, 0, sizeof(*out));
  out->completed = srv->completed;
  out->failed = srv->failed;
  out->pending = (int64_t)srv->queue.size();
  for (const Slot &sl : srv->slots) out->in_flight += sl.req ? 1 : 0;
  out->points = srv->points;
  out->tests = (int64_t)srv->tests;
  out->graph_replays = srv->replays;
  std::vector<double> l = srv->lat_us;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      size_t k = (size_t)std::ceil(p * (double)l.size()) - 1;
      return l[std::min(k, l.size() - 1)];
    };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    double s = 0;
    for (double v : l) s += v;
    out->mean_us = s / (double)l.size();
    out->max_us = l.back();
  }
  if (srv->any) {
    double span = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
    if (span > 0) {
      out->points_per_s = (double)srv->points / span;
      out->tests_per_s = (double)srv->tests / span;
    }
  }
  return GP_OK;
}

extern "C" gp_status gp_serve_stats_reset(gp_server *srv) {
  if (!srv) return set_error(GP_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->lat_us.clear();
  srv->completed = srv->failed = srv->points = srv->replays = 0;
  srv->tests = 0;
  srv->any = false;
  return GP_OK;
}

extern "C" gp_status gp_serve_destroy(gp_server *srv) {
  if (!srv) return set_error(GP_E_INVALID_ARG, "null argument");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    srv->cv_work.notify_all();
  }
  if (srv->th.joinable()) srv->th.join();
  for (Slot &sl : srv->slots) (void)hipStreamSynchronize(sl.stream);
  free_server(srv);
  return GP_OK;
}
