// Continuous-batching server over resident grids (gp_serve_* in include/gp.h).
//
// Memory.  At creation the server takes one device arena of `mem_budget` bytes.  Every
// chunk of work (at most `slot_points` points of one request) runs in a block carved
// from the arena for its size bucket: the chunk's input and output buffers plus its
// query workspace, sized with gp_workspace_bytes for that bucket and grid.  Admission is
// by bytes: a chunk starts only when a stream is free AND its block fits in the arena
// (reusing an idle block of the same shape, else carving free space, else evicting
// idle blocks of other shapes, least recently used first).  A chunk whose stream is
// free but whose block does not fit waits for running chunks to return their blocks
// (counted in deferred_for_memory).
//
// Streams.  Up to n_slots chunks run at once, each on its own HIP stream.  Requests are
// cut into chunks of slot_points points (every point is independent, so chunking is
// exact) and chunks are admitted in FIFO order: the chunks of one large request spread
// over all free streams, and requests that arrive while others are on the GPU start as
// soon as a stream and memory free up, so their work overlaps on the device.
//
// Graphs.  A block captures its query pipeline into a hipGraph the first time it runs
// and replays it for every later chunk of its shape.  Buckets are powers of two from
// 1024 up to slot_points; a chunk of m points runs the graph of bucket b >= m with the
// tail [m, b) of its inputs filled with NaN, which the filter leaves unpaired (no
// refinement work).  Graphs capture the grid's kernel configuration at first use.
//
// One server thread admits chunks, enqueues their copies and graph launches, and polls
// the streams' events to complete chunks and tickets.  A ticket is released (its
// bookkeeping freed) by the gp_serve_wait that returns its completion or the
// gp_serve_poll that reports it done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

constexpr size_t kAlign = 256;
constexpr size_t kLatSamples = 1 << 16;  // latency samples kept for the percentiles

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

__global__ void k_fill_nan(double *x, double *y, int64_t lo, int64_t hi) {
  for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = __builtin_nan("");
    y[i] = __builtin_nan("");
  }
}

struct Request {
  uint64_t ticket = 0;
  gp_kind kind = GP_PIP;
  int64_t n = 0;
  const double *px = nullptr, *py = nullptr;
  int32_t *out_id = nullptr;
  double *out_dist = nullptr;
  Clock::time_point t_submit;
  int64_t issued = 0;      // points handed to chunks
  int64_t finished = 0;    // points of completed chunks
  int running = 0;         // chunks on the device
  bool waited_mem = false; // the current head chunk was already counted as deferred
  unsigned long long tests = 0;
  int done = 0;
  gp_status status = GP_OK;
};

// Device buffers of one chunk, carved from the arena: inputs, outputs, workspace.
struct Block {
  size_t off = 0, bytes = 0;
  gp_kind kind = GP_PIP;
  int64_t bucket = 0;
  double *px = nullptr, *py = nullptr, *dist = nullptr;
  int32_t *id = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipGraphExec_t graph = nullptr;
  uint64_t last_use = 0;
};

// A stream running at most one chunk.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  unsigned long long *h_tests = nullptr;  // pinned landing slot of the chunk's test count
  Request *req = nullptr;
  Block *blk = nullptr;
  int64_t m = 0;  // points of the running chunk
};

}  // namespace

struct gp_server {
  const gp_grid *grid[3] = {nullptr, nullptr, nullptr};
  gp_serve_opts opts;
  int device = 0;
  // server-thread state (no lock: only the server thread touches it after creation)
  std::vector<Lane> lanes;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_ranges;  // offset -> size, coalesced
  std::vector<Block *> idle;
  uint64_t use_clock = 0;
  unsigned long long *h_tests = nullptr;
  // shared state, under mu
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread th;
  // statistics, under mu
  std::vector<double> lat_us;  // ring of the most recent kLatSamples latencies
  size_t lat_next = 0;
  int64_t lat_total = 0;
  int64_t completed = 0, failed = 0, points = 0, replays = 0;
  unsigned long long tests = 0;
  int64_t cur_requests = 0, cur_chunks = 0, max_requests = 0, max_chunks = 0;
  int64_t deferred_mem = 0;
  int64_t bytes_in_use = 0, peak_bytes = 0;
  Clock::time_point t_first, t_last;
  bool any = false;
};

static int64_t bucket_for(int64_t n, int64_t cap) {
  int64_t b = 1024;
  while (b < n && b < cap) b <<= 1;
  return std::min(b, cap);
}

// Bytes of a block of bucket b for one grid: inputs, outputs, workspace.
static size_t block_bytes(const gp_server *srv, gp_kind kind, int64_t b, size_t *ws_bytes) {
  size_t ws = workspace_layout(*(const Grid *)srv->grid[kind], b, (gp_precision)srv->opts.precision,
                               nullptr, nullptr);
  if (ws_bytes) *ws_bytes = ws;
  size_t io = 2 * align_up((size_t)b * 8) + align_up((size_t)b * 4);
  if (kind == GP_P2P) io += align_up((size_t)b * 8);
  return io + align_up(ws);
}

// ------------------------------------------------------------------------- arena

static size_t arena_carve(gp_server *srv, size_t bytes) {
  for (auto it = srv->free_ranges.begin(); it != srv->free_ranges.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, sz = it->second;
    srv->free_ranges.erase(it);
    if (sz > bytes) srv->free_ranges.emplace(off + bytes, sz - bytes);
    return off;
  }
  return SIZE_MAX;
}

static void arena_release(gp_server *srv, size_t off, size_t bytes) {
  auto it = srv->free_ranges.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != srv->free_ranges.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    srv->free_ranges.erase(nx);
  }
  if (it != srv->free_ranges.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      srv->free_ranges.erase(it);
    }
  }
}

static void drop_block(gp_server *srv, Block *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  arena_release(srv, b->off, b->bytes);
  delete b;
}

// A block for a chunk of `kind` and bucket b: an idle one of the same shape, else new
// arena space, else space freed by evicting idle blocks (least recently used first).
// NULL when running chunks hold too much of the arena.
static Block *acquire_block(gp_server *srv, gp_kind kind, int64_t b) {
  Block *hit = nullptr;
  for (Block *x : srv->idle)
    if (x->kind == kind && x->bucket == b && (!hit || x->last_use > hit->last_use)) hit = x;
  if (hit) {
    srv->idle.erase(std::find(srv->idle.begin(), srv->idle.end(), hit));
    return hit;
  }
  size_t ws_bytes = 0;
  const size_t bytes = block_bytes(srv, kind, b, &ws_bytes);
  size_t off = arena_carve(srv, bytes);
  while (off == SIZE_MAX && !srv->idle.empty()) {
    auto lru = std::min_element(srv->idle.begin(), srv->idle.end(),
                                [](const Block *x, const Block *y) { return x->last_use < y->last_use; });
    Block *victim = *lru;
    srv->idle.erase(lru);
    drop_block(srv, victim);
    off = arena_carve(srv, bytes);
  }
  if (off == SIZE_MAX) return nullptr;
  Block *nb = new Block();
  nb->off = off;
  nb->bytes = bytes;
  nb->kind = kind;
  nb->bucket = b;
  char *p = srv->arena + off;
  auto take = [&](size_t sz) {
    char *q = p;
    p += align_up(sz);
    return q;
  };
  nb->px = (double *)take((size_t)b * 8);
  nb->py = (double *)take((size_t)b * 8);
  nb->id = (int32_t *)take((size_t)b * 4);
  if (kind == GP_P2P) nb->dist = (double *)take((size_t)b * 8);
  nb->ws = take(ws_bytes);
  nb->ws_bytes = ws_bytes;
  return nb;
}

// ------------------------------------------------------------------------- chunks

#define SV_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(GP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// Enqueue chunk [lo, lo+m) of request r on lane ln with block blk.  Server thread.
static gp_status enqueue_chunk(gp_server *srv, Lane &ln, Request *r, Block *blk, int64_t lo,
                               int64_t m) {
  const gp_serve_opts &o = srv->opts;
  const hipMemcpyKind in_kind = o.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind out_kind = o.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipStream_t s = ln.stream;
  const gp_grid *g = srv->grid[r->kind];
  const int64_t b = blk->bucket;
  const int64_t nq = o.use_graphs ? b : m;  // points the query runs on
  SV_TRY(hipMemcpyAsync(blk->px, r->px + lo, (size_t)m * 8, in_kind, s));
  SV_TRY(hipMemcpyAsync(blk->py, r->py + lo, (size_t)m * 8, in_kind, s));
  if (nq > m) {
    hipLaunchKernelGGL(k_fill_nan, dim3(256), dim3(256), 0, s, blk->px, blk->py, m, nq);
    SV_TRY(hipGetLastError());
  }
  const gp_precision prec = (gp_precision)o.precision;
  Workspace w;
  workspace_layout(*(const Grid *)g, nq, prec, blk->ws, &w);
  // A request's points spread over the grid's cells, so a small bucket has few points
  // per cell: keep work items to one wavefront and fewer points per lane there.
  gp_tuning tn = ((const Grid *)g)->tune[prec];
  tn.waves_per_item = 1;
  int ppl_cap = b >= (1 << 20) ? 4 : b >= (1 << 17) ? 2 : 1;
  if (ppl_cap > 2 && b < kFourPerLaneMinPointsPerCell * ((const Grid *)g)->ncells) ppl_cap = 2;
  if (tn.points_per_lane > ppl_cap) tn.points_per_lane = ppl_cap;
  if (b < kPersistentMinPoints) tn.persistent = 0;
  // with under 4 points per cell on average most items hold a few points: those run
  // vertex-parallel (lanes over edges or segments) instead of leaving most lanes idle
  if (tn.vp_points < 0 && (double)b < 4.0 * (double)((const Grid *)g)->ncells)
    tn.vp_points = 4;
  if (o.use_graphs) {
    if (!blk->graph) {
      hipGraph_t graph;
      SV_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      gp_status rc = run_query_tuned(g, r->kind, b, blk->px, blk->py, blk->id, blk->dist, prec,
                                     blk->ws, blk->ws_bytes, s, nullptr, &tn);
      hipError_t ec = hipStreamEndCapture(s, &graph);
      if (rc) return rc;
      SV_TRY(ec);
      hipGraphExec_t exec;
      hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      SV_TRY(ei);
      blk->graph = exec;
    }
    SV_TRY(hipGraphLaunch(blk->graph, s));
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->replays++;
  } else {
    gp_status rc = run_query_tuned(g, r->kind, m, blk->px, blk->py, blk->id, blk->dist, prec,
                                   blk->ws, blk->ws_bytes, s, nullptr, &tn);
    if (rc) return rc;
  }
  SV_TRY(hipMemcpyAsync(r->out_id + lo, blk->id, (size_t)m * 4, out_kind, s));
  if (r->kind == GP_P2P)
    SV_TRY(hipMemcpyAsync(r->out_dist + lo, blk->dist, (size_t)m * 8, out_kind, s));
  SV_TRY(hipMemcpyAsync(ln.h_tests, w.tests, 8, hipMemcpyDeviceToHost, s));
  SV_TRY(hipEventRecord(ln.done_ev, s));
  return GP_OK;
}
#undef SV_TRY

// Completion of the chunk on lane ln (status st): its block goes back to the idle
// list, and the request completes once all of its points are done.  Server thread.
static void finish_chunk(gp_server *srv, Lane &ln, gp_status st) {
  Request *r = ln.req;
  Block *blk = ln.blk;
  const unsigned long long t = st == GP_OK ? *ln.h_tests : 0ull;
  blk->last_use = ++srv->use_clock;
  srv->idle.push_back(blk);
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->cur_chunks--;
  srv->bytes_in_use -= (int64_t)blk->bytes;
  if (--r->running == 0) srv->cur_requests--;
  if (st != GP_OK) r->status = st;
  r->tests += t;
  r->finished += ln.m;
  if (r->finished == r->n) {
    r->done = 1;
    if (r->status == GP_OK) {
      srv->completed++;
      srv->points += r->n;
      srv->tests += r->tests;
      const double us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
      if (srv->lat_us.size() < kLatSamples) srv->lat_us.push_back(us);
      else srv->lat_us[srv->lat_next] = us;
      srv->lat_next = (srv->lat_next + 1) % kLatSamples;
      srv->lat_total++;
      if (!srv->any) { srv->t_first = r->t_submit; srv->any = true; }
      srv->t_last = now;
    } else {
      srv->failed++;
    }
    srv->cv_done.notify_all();
  }
  ln.req = nullptr;
  ln.blk = nullptr;
  ln.m = 0;
}

static Lane *free_lane(gp_server *srv) {
  for (Lane &ln : srv->lanes)
    if (!ln.req) return &ln;
  return nullptr;
}

// Admit chunks in FIFO order while a stream is free and the head chunk's block fits.
// Returns true when anything was admitted.  Server thread.
static bool admit(gp_server *srv) {
  bool any = false;
  for (;;) {
    Lane *ln = free_lane(srv);
    if (!ln) break;
    Request *r = nullptr;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      if (srv->queue.empty()) break;
      r = srv->queue.front();
    }
    const int64_t lo = r->issued;
    const int64_t m = std::min(srv->opts.slot_points, r->n - lo);
    Block *blk = acquire_block(srv, r->kind, bucket_for(m, srv->opts.slot_points));
    if (!blk) {
      if (!r->waited_mem) {
        r->waited_mem = true;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->deferred_mem++;
      }
      break;
    }
    r->waited_mem = false;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      r->issued += m;
      if (r->issued == r->n) srv->queue.pop_front();
      if (r->running++ == 0) srv->cur_requests++;
      srv->cur_chunks++;
      srv->bytes_in_use += (int64_t)blk->bytes;
      srv->max_requests = std::max(srv->max_requests, srv->cur_requests);
      srv->max_chunks = std::max(srv->max_chunks, srv->cur_chunks);
      srv->peak_bytes = std::max(srv->peak_bytes, srv->bytes_in_use);
    }
    ln->req = r;
    ln->blk = blk;
    ln->m = m;
    gp_status st = r->status == GP_OK ? enqueue_chunk(srv, *ln, r, blk, lo, m) : r->status;
    if (st != GP_OK) {
      (void)hipStreamSynchronize(ln->stream);
      finish_chunk(srv, *ln, st);
    }
    any = true;
  }
  return any;
}

static void server_loop(gp_server *srv) {
  (void)hipSetDevice(srv->device);  // a new host thread starts on device 0
  for (;;) {
    bool busy = false;
    for (Lane &ln : srv->lanes) {
      if (!ln.req) continue;
      busy = true;
      const hipError_t q = hipEventQuery(ln.done_ev);
      if (q == hipSuccess) {
        finish_chunk(srv, ln, GP_OK);
      } else if (q != hipErrorNotReady) {
        set_error(GP_E_HIP, "request failed on the device: %s", hipGetErrorString(q));
        finish_chunk(srv, ln, GP_E_HIP);
      }
    }
    if (admit(srv)) busy = true;
    std::unique_lock<std::mutex> lk(srv->mu);
    const bool running = srv->cur_chunks > 0;
    const bool idle = !running && srv->queue.empty();
    if (idle && srv->stopping) break;
    if (idle || (!running && !busy)) {
      srv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

static void free_server(gp_server *srv) {
  for (Lane &ln : srv->lanes) {
    if (ln.blk) srv->idle.push_back(ln.blk);
    if (ln.done_ev) (void)hipEventDestroy(ln.done_ev);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  for (Block *b : srv->idle) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    delete b;
  }
  srv->idle.clear();
  if (srv->arena) (void)hipFree(srv->arena);
  if (srv->h_tests) (void)hipHostFree(srv->h_tests);
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
  if (pip_grid && p2p_grid && ((const Grid *)pip_grid)->device != ((const Grid *)p2p_grid)->device)
    return set_error(GP_E_INVALID_ARG, "the two grids live on different devices");
  gp_serve_opts o = *opts;
  if (o.n_slots < 1 || o.n_slots > 16) return set_error(GP_E_INVALID_ARG, "n_slots must be 1..16");
  if (o.slot_points < 1024 || o.slot_points >= ((int64_t)1 << 30))
    return set_error(GP_E_INVALID_ARG, "slot_points must be in [1024, 2^30)");
  if (o.precision != GP_FP64 && o.precision != GP_MIXED)
    return set_error(GP_E_INVALID_ARG, "bad precision");
  if (o.mem_budget <= 0) return set_error(GP_E_INVALID_ARG, "mem_budget must be > 0");
  if (o.max_queue <= 0) o.max_queue = 1 << 20;
  gp_server *srv = new gp_server();
  srv->grid[GP_PIP] = pip_grid;
  srv->grid[GP_P2P] = p2p_grid;
  srv->opts = o;
  srv->device = ((const Grid *)(pip_grid ? pip_grid : p2p_grid))->device;
  // the largest block must fit: a chunk of slot_points points of either kind
  size_t need = 0;
  for (gp_kind k : {GP_PIP, GP_P2P})
    if (srv->grid[k]) need = std::max(need, block_bytes(srv, k, o.slot_points, nullptr));
  if ((size_t)o.mem_budget < need) {
    delete srv;
    return set_error(GP_E_OOM, "memory budget %lld below one chunk of slot_points (%zu bytes)",
                     (long long)o.mem_budget, need);
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != srv->device) {
    delete srv;
    return set_error(GP_E_INVALID_ARG, "the grids live on device %d; make it current",
                     srv->device);
  }
  srv->arena_bytes = (size_t)o.mem_budget / kAlign * kAlign;
  if (hipMalloc((void **)&srv->arena, srv->arena_bytes) != hipSuccess) {
    srv->arena = nullptr;
    free_server(srv);
    return set_error(GP_E_OOM, "arena of %zu bytes could not be allocated", srv->arena_bytes);
  }
  srv->free_ranges.emplace(0, srv->arena_bytes);
  srv->lanes.resize(o.n_slots);
  if (hipHostMalloc((void **)&srv->h_tests, (size_t)o.n_slots * 8, hipHostMallocDefault) !=
      hipSuccess) {
    srv->h_tests = nullptr;
    free_server(srv);
    return set_error(GP_E_OOM, "pinned allocation failed");
  }
  for (int i = 0; i < o.n_slots; ++i) {
    Lane &ln = srv->lanes[i];
    ln.h_tests = srv->h_tests + i;
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.done_ev, hipEventDisableTiming) != hipSuccess) {
      free_server(srv);
      return set_error(GP_E_HIP, "stream or event creation failed");
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
  if (srv->stopping) {
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
    srv->cv_done.notify_all();
  } else {
    srv->queue.push_back(r);
    srv->cv_work.notify_one();
  }
  return GP_OK;
}

// Forget a completed ticket.  Caller holds mu.
static void release_ticket(gp_server *srv, uint64_t ticket) {
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return;
  delete it->second;
  srv->reqs.erase(it);
}

extern "C" gp_status gp_serve_poll(gp_server *srv, uint64_t ticket, int32_t *done) {
  if (!srv || !done) return set_error(GP_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(GP_E_NOT_FOUND, "unknown ticket");
  *done = it->second->done;
  if (*done) release_ticket(srv, ticket);
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
  const gp_status st = r->status;
  release_ticket(srv, ticket);
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
  out->in_flight = srv->cur_requests;
  out->points = srv->points;
  out->tests = (int64_t)srv->tests;
  out->graph_replays = srv->replays;
  out->chunks_in_flight = srv->cur_chunks;
  out->max_in_flight = srv->max_requests;
  out->max_chunks_in_flight = srv->max_chunks;
  out->deferred_for_memory = srv->deferred_mem;
  out->bytes_in_use = srv->bytes_in_use;
  out->peak_bytes_in_use = srv->peak_bytes;
  out->arena_bytes = (int64_t)srv->arena_bytes;
  out->latency_samples = (int64_t)srv->lat_us.size();
  std::vector<double> l = srv->lat_us;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      size_t k = (size_t)std::ceil(p * (double)l.size());
      k = k == 0 ? 0 : k - 1;
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
    const double span = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
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
  srv->lat_next = 0;
  srv->lat_total = 0;
  srv->completed = srv->failed = srv->points = srv->replays = 0;
  srv->tests = 0;
  srv->max_requests = srv->cur_requests;
  srv->max_chunks = srv->cur_chunks;
  srv->deferred_mem = 0;
  srv->peak_bytes = srv->bytes_in_use;
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
  for (Lane &ln : srv->lanes) (void)hipStreamSynchronize(ln.stream);
  free_server(srv);
  return GP_OK;
}
