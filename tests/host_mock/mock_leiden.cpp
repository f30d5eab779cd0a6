// Host-only stand-in for the single-graph entry points that the batched and
// serving executors call.  A "graph" is a counter state; an update folds the
// batch into it and derives a membership from it, with a short random delay
// so that requests of different graphs overlap.  Results depend only on the
// graph's own sequence of requests, as with the real library, so a correct
// executor returns the same results alone and in a mix.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <thread>

#include <hip/hip_runtime.h>

#include "leiden.h"

struct mock_stream {
  int id;
};

struct leiden_graph {
  uint32_t n;
  uint64_t state;
  std::atomic<int> busy{0};
  bool overlapped = false;  // two calls on one graph at once
};

namespace {
thread_local std::string g_msg;
std::atomic<int> g_streams{0};

void jitter(uint64_t salt) {
  thread_local std::mt19937_64 rng(std::hash<std::thread::id>()(std::this_thread::get_id()) ^ salt);
  std::this_thread::sleep_for(std::chrono::microseconds(rng() % 400));
}

void fill(leiden_graph* g, uint32_t* out) {
  if (!out) return;
  for (uint32_t i = 0; i < g->n; ++i) out[i] = (uint32_t)((g->state * 0x9e3779b97f4a7c15ull + i * 31u) % g->n);
}

struct Busy {
  leiden_graph* g;
  explicit Busy(leiden_graph* x) : g(x) {
    if (g->busy.fetch_add(1) != 0) g->overlapped = true;
  }
  ~Busy() { g->busy.fetch_sub(1); }
};
}  // namespace

extern "C" {

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* c) {
  *c = 1;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new mock_stream{g_streams.fetch_add(1)};
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  g_streams.fetch_sub(1);
  return hipSuccess;
}

int mock_live_streams() { return g_streams.load(); }
int mock_graph_overlapped(leiden_graph* g) { return g->overlapped ? 1 : 0; }

leiden_status leiden_default_opts(leiden_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->deterministic = 1;
  return LEIDEN_OK;
}

leiden_status leiden_graph_create(int, uint32_t n, uint64_t nnz, const int64_t*, const uint32_t*, const uint32_t*, int,
                                  double, leiden_graph** out) {
  if (n == 0) return LEIDEN_EINVAL;
  auto* g = new leiden_graph();
  g->n = n;
  g->state = nnz;
  *out = g;
  return LEIDEN_OK;
}

void leiden_graph_destroy(leiden_graph* g) { delete g; }

leiden_status leiden_static(leiden_graph* g, const leiden_opts*, uint32_t* out, int, double* q, leiden_stats* st) {
  Busy b(g);
  jitter(g->state);
  g->state = g->state * 1000003u + 17u;
  fill(g, out);
  if (q) *q = (double)(g->state % 1000) / 1000.0;
  if (st) std::memset(st, 0, sizeof(*st));
  return LEIDEN_OK;
}

leiden_status leiden_update(leiden_graph* g, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                            int, const uint32_t*, int, leiden_mode mode, const leiden_opts*, uint32_t* out, int,
                            double* q, leiden_stats* st) {
  Busy b(g);
  jitter(g->state + n_ins);
  uint64_t h = g->state * 6364136223846793005ull + (uint64_t)mode;
  for (uint64_t k = 0; k < 2 * n_del; ++k) h = h * 31u + del[k];
  for (uint64_t k = 0; k < 3 * n_ins; ++k) h = h * 37u + ins[k];
  if (n_ins && ins[0] == 0xFFFFFFFFu) {
    g_msg = "invalid batch";
    return LEIDEN_EINVAL;
  }
  g->state = h;
  fill(g, out);
  if (q) *q = (double)(h % 1000) / 1000.0;
  if (st) std::memset(st, 0, sizeof(*st));
  return LEIDEN_OK;
}

const char* leiden_last_error(void) { return g_msg.c_str(); }

}  // extern "C"
