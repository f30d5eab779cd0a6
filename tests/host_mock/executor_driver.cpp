// Drives the batched and serving executors (serve.hip) against the host-only
// mock of the single-graph entry points, checking that every result equals
// the result of the same graph alone, that one graph never runs two requests
// at once, that failures stay with their request, that admission follows the
// budget and that every worker stream is released.  Exit status 0 on success.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include <hip/hip_runtime.h>

#include "leiden.h"

extern "C" int mock_live_streams();
extern "C" int mock_graph_overlapped(leiden_graph* g);

#define EXPECT(c)                                                    \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "FAILED %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

struct Req {
  uint32_t graph;
  std::vector<uint32_t> del, ins;
  leiden_mode mode;
};

static std::vector<uint32_t> run_alone(uint32_t n, uint64_t nnz, const std::vector<Req>& reqs, uint32_t gid,
                                       size_t upto) {
  leiden_graph* g = nullptr;
  EXPECT(leiden_graph_create(0, n, nnz, nullptr, nullptr, nullptr, 0, 0.2, &g) == LEIDEN_OK);
  EXPECT(leiden_static(g, nullptr, nullptr, 0, nullptr, nullptr) == LEIDEN_OK);
  std::vector<uint32_t> out(n);
  for (size_t k = 0; k <= upto; ++k) {
    const Req& r = reqs[k];
    if (r.graph != gid) continue;
    if (!r.ins.empty() && r.ins[0] == 0xFFFFFFFFu) continue;  // the failing request changes nothing
    EXPECT(leiden_update(g, r.del.data(), r.del.size() / 2, r.ins.data(), r.ins.size() / 3, 0, nullptr, 0, r.mode,
                         nullptr, out.data(), 0, nullptr, nullptr) == LEIDEN_OK);
  }
  leiden_graph_destroy(g);
  return out;
}

int main() {
  std::mt19937 rng(7);
  // --- serving ---
  const uint32_t G = 5;
  std::vector<uint32_t> ns = {100, 257, 64, 1000, 33};
  leiden_server* S = nullptr;
  EXPECT(leiden_server_create(0, 1ull << 40, 3, &S) == LEIDEN_OK);
  std::vector<uint32_t> ids(G);
  for (uint32_t k = 0; k < G; ++k)
    EXPECT(leiden_server_add_graph(S, ns[k], 10 * ns[k], nullptr, nullptr, nullptr, 0, 0.2, nullptr, &ids[k]) ==
           LEIDEN_OK);
  std::vector<Req> reqs;
  for (int r = 0; r < 60; ++r) {
    Req q;
    q.graph = rng() % G;
    q.mode = (leiden_mode)(rng() % 3);
    for (int e = 0; e < 4; ++e) q.del.push_back(rng() % 1000);
    for (int e = 0; e < 6; ++e) q.ins.push_back(rng() % 1000);
    if (r == 17) q.ins[0] = 0xFFFFFFFFu;  // fails in the library
    reqs.push_back(q);
  }
  std::vector<uint64_t> tickets;
  for (auto& q : reqs) {
    uint64_t t = 0;
    EXPECT(leiden_server_submit(S, ids[q.graph], q.del.data(), q.del.size() / 2, q.ins.data(), q.ins.size() / 3,
                                q.mode, nullptr, &t) == LEIDEN_OK);
    tickets.push_back(t);
  }
  // wait in a shuffled order
  std::vector<size_t> order(reqs.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::shuffle(order.begin(), order.end(), rng);
  std::vector<std::vector<uint32_t>> got(reqs.size());
  for (size_t k : order) {
    got[k].assign(ns[reqs[k].graph], 0);
    double lat = 0, svc = 0;
    const leiden_status st = leiden_server_wait(S, tickets[k], got[k].data(), nullptr, nullptr, &lat, &svc);
    EXPECT(st == (k == 17 ? LEIDEN_EINVAL : LEIDEN_OK));
    EXPECT(lat >= svc && svc >= 0);
  }
  EXPECT(leiden_server_wait(S, tickets[3], nullptr, nullptr, nullptr, nullptr, nullptr) == LEIDEN_EINVAL);
  leiden_server_stats ss;
  EXPECT(leiden_server_get_stats(S, &ss) == LEIDEN_OK);
  EXPECT(ss.completed == reqs.size() - 1 && ss.failed == 1 && ss.waiting == 0 && ss.graphs == G);
  for (size_t k = 0; k < reqs.size(); ++k) {
    if (k == 17) continue;
    EXPECT(got[k] == run_alone(ns[reqs[k].graph], 10 * ns[reqs[k].graph], reqs, reqs[k].graph, k));
  }
  // admission: the budget is the only limit; removing a graph returns its share
  leiden_server* T = nullptr;
  EXPECT(leiden_server_create(0, 1ull << 30, 2, &T) == LEIDEN_OK);
  uint32_t id = 0, admitted = 0;
  while (leiden_server_add_graph(T, 1u << 16, 1u << 20, nullptr, nullptr, nullptr, 0, 0.2, nullptr, &id) ==
         LEIDEN_OK) {
    ++admitted;
    EXPECT(admitted < 1000);
  }
  EXPECT(admitted >= 1);
  EXPECT(leiden_server_remove_graph(T, id) == LEIDEN_OK);
  EXPECT(leiden_server_add_graph(T, 1u << 16, 1u << 20, nullptr, nullptr, nullptr, 0, 0.2, nullptr, &id) == LEIDEN_OK);
  leiden_server_destroy(T);
  leiden_server_destroy(S);
  // --- batched ---
  const uint32_t B = 20;
  std::vector<leiden_graph*> gs(B), ref(B);
  std::vector<std::vector<uint32_t>> outs(B), expect(B);
  std::vector<uint32_t*> po(B);
  for (uint32_t k = 0; k < B; ++k) {
    const uint32_t n = 50 + 37 * k;
    EXPECT(leiden_graph_create(0, n, 7 * n, nullptr, nullptr, nullptr, 0, 0.2, &gs[k]) == LEIDEN_OK);
    EXPECT(leiden_graph_create(0, n, 7 * n, nullptr, nullptr, nullptr, 0, 0.2, &ref[k]) == LEIDEN_OK);
    outs[k].assign(n, 0);
    expect[k].assign(n, 0);
    po[k] = outs[k].data();
  }
  std::vector<double> q(B);
  std::vector<leiden_status> sts(B);
  EXPECT(leiden_batch_run(gs.data(), B, nullptr, LEIDEN_DF, nullptr, 4, po.data(), q.data(), sts.data()) ==
         LEIDEN_OK);
  for (uint32_t k = 0; k < B; ++k) {
    EXPECT(leiden_static(ref[k], nullptr, expect[k].data(), 0, nullptr, nullptr) == LEIDEN_OK);
    EXPECT(outs[k] == expect[k]);
  }
  std::vector<leiden_batch_item> items(B);
  std::vector<uint32_t> ins = {1, 2, 3, 4, 5, 6};
  for (auto& it : items) it = leiden_batch_item{nullptr, 0, ins.data(), 2};
  EXPECT(leiden_batch_run(gs.data(), B, items.data(), LEIDEN_DF, nullptr, 4, po.data(), q.data(), sts.data()) ==
         LEIDEN_OK);
  for (uint32_t k = 0; k < B; ++k) {
    EXPECT(leiden_update(ref[k], nullptr, 0, ins.data(), 2, 0, nullptr, 0, LEIDEN_DF, nullptr, expect[k].data(), 0,
                         nullptr, nullptr) == LEIDEN_OK);
    EXPECT(outs[k] == expect[k]);
    EXPECT(mock_graph_overlapped(gs[k]) == 0);
    leiden_graph_destroy(gs[k]);
    leiden_graph_destroy(ref[k]);
  }
  EXPECT(mock_live_streams() == 0);
  std::printf("OK\n");
  return 0;
}
