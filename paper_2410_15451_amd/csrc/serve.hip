// Batched and serving forms on one GPU.
//
// Both run many independent graph handles at once: worker threads, each with
// its own HIP stream (default priority), take work from a shared queue and
// drive the ordinary single-graph entry points on their stream.  The handles
// share nothing, so every result is the one the graph gets alone; the
// concurrency fills the GPU with several graphs' kernels while other workers
// wait on their own host synchronisations.
//
// Serving: tenant graphs are admitted against an HBM budget (an estimate of a
// handle's device footprint); update requests are queued with their arrival
// time and admitted to a free worker in arrival order, except that one graph
// never runs two requests at once (per-graph order is kept); latency is
// completion minus arrival, service time is completion minus start.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/leiden.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double k = (v.size() - 1) * p / 100.0;
  const size_t lo = (size_t)k, hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (k - lo);
}

// Device bytes of a handle holding n vertices and nnz directed entries with
// the given slack (CSR with its overflow room, state, per-level workspace,
// aggregation and batch buffers), rounded up.  Used for admission only.
uint64_t handle_bytes(uint32_t n, uint64_t nnz, double slack) {
  const double rows = (double)nnz * (1.0 + slack) * 1.5;  // slack rows plus the overflow area
  const double graph = rows * 8.0 + (double)n * 16.0;
  const double per_vertex = 420.0;                        // state, level arrays, lists, tracking
  const double per_entry = 2.0 * 12.0 + 4.0 + 8.0 / 64.0; // two level CSRs, scan room, marking items
  return (uint64_t)(graph + per_vertex * n + per_entry * (double)nnz) + (64ull << 20);
}

struct Request {
  uint32_t graph = 0;
  std::vector<uint32_t> del, ins;
  leiden_mode mode = LEIDEN_DF;
  leiden_opts opts{};
  Clock::time_point arrive, start, end;
  bool done = false;
  leiden_status status = LEIDEN_OK;
  std::vector<uint32_t> membership;
  double q = 0;
  leiden_stats stats{};
  char err[160] = {0};
};

struct Tenant {
  leiden_graph* g = nullptr;
  uint32_t n = 0;
  uint64_t bytes = 0;
  bool busy = false;
  bool live = false;
};

}  // namespace

struct leiden_server {
  int device = 0;
  uint64_t budget = 0, used = 0;
  std::deque<Tenant> tenants;  // deque: workers hold references while graphs are added
  std::deque<uint64_t> queue;  // waiting tickets in arrival order
  std::unordered_map<uint64_t, Request> req;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::vector<std::thread> workers;
  bool stop = false;
  // completed-request statistics
  std::vector<double> lat, svc;
  uint64_t completed = 0, failed = 0, edges = 0;
  bool any = false;
  Clock::time_point first_arrive, last_end;
};

namespace {

void worker_main(leiden_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // the oldest waiting request whose graph is idle
    auto pick = S->queue.end();
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
      if (!S->tenants[S->req[*it].graph].busy) {
        pick = it;
        break;
      }
    if (pick == S->queue.end()) {
      if (S->stop) break;
      S->work_cv.wait(lk);
      continue;
    }
    const uint64_t t = *pick;
    S->queue.erase(pick);
    Request& r = S->req[t];
    Tenant& tn = S->tenants[r.graph];
    tn.busy = true;
    r.start = Clock::now();
    r.membership.assign(tn.n, 0);
    lk.unlock();
    leiden_opts o = r.opts;
    o.stream = st;
    const uint64_t nd = r.del.size() / 2, ni = r.ins.size() / 3;
    r.status = leiden_update(tn.g, nd ? r.del.data() : nullptr, nd, ni ? r.ins.data() : nullptr, ni, 0, nullptr, 0,
                             r.mode, &o, r.membership.data(), 0, &r.q, &r.stats);
    if (r.status != LEIDEN_OK) std::snprintf(r.err, sizeof(r.err), "%s", leiden_last_error());
    lk.lock();
    r.end = Clock::now();
    r.done = true;
    tn.busy = false;
    if (r.status == LEIDEN_OK) {
      S->completed++;
      S->lat.push_back(ms_between(r.arrive, r.end));
      S->svc.push_back(ms_between(r.start, r.end));
      S->edges += nd + ni;
      S->last_end = std::max(S->last_end, r.end);
    } else {
      S->failed++;
    }
    S->done_cv.notify_all();
    S->work_cv.notify_all();
  }
  lk.unlock();
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

leiden_status leiden_server_footprint(uint32_t n, uint64_t nnz, double slack, uint64_t* bytes) {
  if (!bytes || !(slack >= 0.0)) return LEIDEN_EINVAL;
  *bytes = handle_bytes(n, nnz, slack);
  return LEIDEN_OK;
}

leiden_status leiden_server_create(int device, uint64_t hbm_budget_bytes, uint32_t workers, leiden_server** out) {
  if (!out || workers == 0 || workers > 64) return LEIDEN_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return LEIDEN_EDEVICE;
  auto* S = new leiden_server();
  S->device = device;
  S->budget = hbm_budget_bytes;
  for (uint32_t i = 0; i < workers; ++i) S->workers.emplace_back(worker_main, S);
  *out = S;
  return LEIDEN_OK;
}

void leiden_server_destroy(leiden_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->work_cv.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& tn : S->tenants)
    if (tn.live) leiden_graph_destroy(tn.g);
  delete S;
}

leiden_status leiden_server_add_graph(leiden_server* S, uint32_t n, uint64_t nnz, const int64_t* offsets,
                                      const uint32_t* cols, const uint32_t* w, int on_device, double slack,
                                      const leiden_opts* opts, uint32_t* graph_id) {
  if (!S || !graph_id) return LEIDEN_EINVAL;
  const uint64_t need = handle_bytes(n, nnz, slack);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->used + need > S->budget) return LEIDEN_ENOMEM;
    S->used += need;  // reserved while the handle is built
  }
  leiden_graph* g = nullptr;
  leiden_status st = leiden_graph_create(S->device, n, nnz, offsets, cols, w, on_device, slack, &g);
  if (st == LEIDEN_OK) st = leiden_static(g, opts, nullptr, 0, nullptr, nullptr);
  std::lock_guard<std::mutex> lk(S->mu);
  if (st != LEIDEN_OK) {
    S->used -= need;
    if (g) leiden_graph_destroy(g);
    return st;
  }
  Tenant tn;
  tn.g = g;
  tn.n = n;
  tn.bytes = need;
  tn.live = true;
  S->tenants.push_back(tn);
  *graph_id = (uint32_t)(S->tenants.size() - 1);
  return LEIDEN_OK;
}

leiden_status leiden_server_remove_graph(leiden_server* S, uint32_t graph_id) {
  if (!S) return LEIDEN_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  if (graph_id >= S->tenants.size() || !S->tenants[graph_id].live) return LEIDEN_EINVAL;
  for (uint64_t t : S->queue)
    if (S->req[t].graph == graph_id) return LEIDEN_ESTATE;
  while (S->tenants[graph_id].busy) S->done_cv.wait(lk);
  Tenant& tn = S->tenants[graph_id];
  leiden_graph_destroy(tn.g);
  tn.live = false;
  tn.g = nullptr;
  S->used -= tn.bytes;
  return LEIDEN_OK;
}

leiden_status leiden_server_submit(leiden_server* S, uint32_t graph_id, const uint32_t* del, uint64_t n_del,
                                   const uint32_t* ins, uint64_t n_ins, leiden_mode mode, const leiden_opts* opts,
                                   uint64_t* ticket) {
  if (!S || !ticket || (n_del && !del) || (n_ins && !ins)) return LEIDEN_EINVAL;
  Request r;
  r.arrive = Clock::now();
  r.graph = graph_id;
  r.mode = mode;
  if (opts) {
    r.opts = *opts;
  } else {
    leiden_default_opts(&r.opts);
  }
  r.opts.compute_modularity = 1;
  r.del.assign(del, del + 2 * n_del);
  r.ins.assign(ins, ins + 3 * n_ins);
  std::lock_guard<std::mutex> lk(S->mu);
  if (graph_id >= S->tenants.size() || !S->tenants[graph_id].live) return LEIDEN_EINVAL;
  const uint64_t t = S->next_ticket++;
  if (!S->any) {
    S->any = true;
    S->first_arrive = r.arrive;
  }
  S->req.emplace(t, std::move(r));
  S->queue.push_back(t);
  *ticket = t;
  S->work_cv.notify_one();
  return LEIDEN_OK;
}

leiden_status leiden_server_wait(leiden_server* S, uint64_t ticket, uint32_t* membership_out, double* q_out,
                                 leiden_stats* stats_out, double* latency_ms, double* service_ms) {
  if (!S) return LEIDEN_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->req.find(ticket);
  if (it == S->req.end()) return LEIDEN_EINVAL;
  while (!it->second.done) S->done_cv.wait(lk);
  Request r = std::move(it->second);
  S->req.erase(it);
  lk.unlock();
  if (membership_out && r.status == LEIDEN_OK)
    std::memcpy(membership_out, r.membership.data(), r.membership.size() * sizeof(uint32_t));
  if (q_out) *q_out = r.q;
  if (stats_out) *stats_out = r.stats;
  if (latency_ms) *latency_ms = ms_between(r.arrive, r.end);
  if (service_ms) *service_ms = ms_between(r.start, r.end);
  return r.status;
}

leiden_status leiden_server_get_stats(leiden_server* S, leiden_server_stats* out) {
  if (!S || !out) return LEIDEN_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = S->completed;
  out->failed = S->failed;
  out->waiting = S->queue.size();
  out->graphs = 0;
  for (auto& tn : S->tenants) out->graphs += tn.live ? 1 : 0;
  out->hbm_reserved = S->used;
  out->latency_p50_ms = percentile(S->lat, 50);
  out->latency_p99_ms = percentile(S->lat, 99);
  out->service_p50_ms = percentile(S->svc, 50);
  out->service_p99_ms = percentile(S->svc, 99);
  const double span = S->any && S->completed ? ms_between(S->first_arrive, S->last_end) : 0.0;
  out->updated_edges_per_s = span > 0 ? (double)S->edges / (span * 1e-3) : 0.0;
  return LEIDEN_OK;
}

// Batched form: `count` independent handles, `streams` worker threads.
leiden_status leiden_batch_run(leiden_graph* const* graphs, uint32_t count, const leiden_batch_item* items,
                               leiden_mode mode, const leiden_opts* opts, uint32_t streams,
                               uint32_t* const* memberships_out, double* q_out, leiden_status* status_out) {
  if (!graphs || (count && !memberships_out) || streams == 0 || streams > 64) return LEIDEN_EINVAL;
  leiden_opts base;
  leiden_default_opts(&base);
  if (opts) base = *opts;
  int device = 0;
  (void)hipGetDevice(&device);
  std::atomic<uint32_t> next{0};
  std::vector<leiden_status> st(count, LEIDEN_OK);
  auto body = [&]() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    leiden_opts o = base;
    o.stream = s;
    for (uint32_t i; (i = next.fetch_add(1)) < count;) {
      double q = 0;
      if (!items) {
        st[i] = leiden_static(graphs[i], &o, memberships_out[i], 0, &q, nullptr);
      } else {
        const leiden_batch_item& b = items[i];
        st[i] = leiden_update(graphs[i], b.del, b.n_del, b.ins, b.n_ins, 0, nullptr, 0, mode, &o, memberships_out[i],
                              0, &q, nullptr);
      }
      if (q_out) q_out[i] = q;
    }
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  };
  std::vector<std::thread> th;
  const uint32_t nt = std::min<uint32_t>(streams, std::max<uint32_t>(count, 1));
  for (uint32_t k = 0; k < nt; ++k) th.emplace_back(body);
  for (auto& t : th) t.join();
  leiden_status first = LEIDEN_OK;
  for (uint32_t i = 0; i < count; ++i) {
    if (status_out) status_out[i] = st[i];
    if (first == LEIDEN_OK && st[i] != LEIDEN_OK) first = st[i];
  }
  return first;
}

}  // extern "C"
