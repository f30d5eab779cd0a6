// Host runtime and C-ABI of the gfx950 Leiden library: the graph handle, its
// device workspace, and the pass loop of Alg. 4 driving the kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/leiden.h"
#include "graph.h"
#include "noalloc.h"

using namespace lm;

namespace {

thread_local std::string g_err;

leiden_status fail(leiden_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(LEIDEN_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                             \
  } while (0)

#define CHK(expr)                              \
  do {                                         \
    leiden_status s_ = (expr);                 \
    if (s_ != LEIDEN_OK) return s_;            \
  } while (0)

// Calls of the library running in the process right now (static and update
// runs, autotuning): the decide kernels use the handle's side streams only
// while a call runs alone.
std::atomic<int> g_in_flight{0};
struct InFlight {
  InFlight() { g_in_flight.fetch_add(1); }
  ~InFlight() { g_in_flight.fetch_sub(1); }
};

// Side streams for a level of nl vertices: levels large enough to fill the
// GPU with several bins at once, and no other call running.
const DecideStreams* side_streams(leiden_graph* G, uint32_t nl);

// The stream of the current API call on this thread (null outside calls).
// Every kernel that reads a handle's buffers runs on that stream or on a side
// stream joined back into it before host code runs again, and earlier calls
// ended with a synchronisation of their own stream; so a buffer of the handle
// can be released once this stream is idle, without waiting for the whole
// device (other handles' calls on other streams keep running).
thread_local hipStream_t tl_alloc_stream = nullptr;

// Device bytes a handle holds, and its budget (0: none).  The handle of the
// current API call on this thread is charged for its buffers' growth.
struct MemAccount {
  uint64_t budget = 0, used = 0;
};
thread_local MemAccount* tl_account = nullptr;

struct AllocScope {
  hipStream_t prev;
  MemAccount* prev_account;
  explicit AllocScope(hipStream_t s, MemAccount* a = nullptr) : prev(tl_alloc_stream), prev_account(tl_account) {
    tl_alloc_stream = s;
    tl_account = a;
  }
  ~AllocScope() {
    tl_alloc_stream = prev;
    tl_account = prev_account;
  }
};

// Device allocation owned by the handle; grows on demand, never shrinks.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  leiden_status reserve(size_t b) {
    if (b <= bytes) return LEIDEN_OK;
    const size_t want = std::max<size_t>(b, 256);
    MemAccount* acct = tl_account;
    if (acct && acct->budget && acct->used - bytes + want > acct->budget)
      return fail(LEIDEN_ENOMEM, "the handle's device memory budget of %llu bytes would be exceeded (%llu held, "
                  "%zu more wanted)", (unsigned long long)acct->budget, (unsigned long long)acct->used, want - bytes);
    if (p) {
      // kernels queued earlier may still read the old block
      if (tl_alloc_stream)
        (void)hipStreamSynchronize(tl_alloc_stream);
      else
        (void)hipDeviceSynchronize();
      (void)hipFree(p);
      if (acct) acct->used -= bytes;
    }
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return fail(LEIDEN_ENOMEM, "device allocation of %zu bytes failed", want);
    }
    bytes = want;
    if (acct) acct->used += want;
    return LEIDEN_OK;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

constexpr uint64_t kAggItems = 1 << 20;  // aggregation work items per round of big communities

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Eq. 2 constants from 2m, computed once per run on the host.
struct QConst {
  double inv_m = 0, inv_2m2 = 0;
  bool narrow = false;  // 2m < 2^32: every K_{i->c} fits 32 bits
};
QConst make_qconst(uint64_t M2) {
  QConst q;
  q.narrow = M2 < (1ull << 32);
  const double m = 0.5 * (double)M2;
  q.inv_m = 1.0 / m;
  q.inv_2m2 = 1.0 / ((2.0 * m) * m);
  return q;
}

// A forest's graphs and its per-graph run state (see forest.hip).
struct ForestState {
  uint32_t nq = 0;
  std::vector<uint32_t> first;  // first vertex of every graph (nq + 1; the last is n)
  Buf gid0, base0;              // the input graph's
  Buf gidA, baseA, gidB, baseB; // level graphs' (alternating)
  const uint32_t* cur_gid = nullptr;
  const uint32_t* cur_base = nullptr;
  Buf m2, inv, dq, move, pass, refined, cur_iters, passes, iters_hist, parts, out_local, live_len;
  // results of the last call
  std::vector<double> q;
  std::vector<uint32_t> passes_h, iters_h;
  ForestBufs bufs() {
    ForestBufs f{};
    f.nq = nq;
    f.m2 = m2.as<unsigned long long>();
    f.inv = inv.as<double>();
    f.dq = dq.as<unsigned long long>();
    f.move = move.as<uint8_t>();
    f.pass = pass.as<uint8_t>();
    f.refined = refined.as<uint8_t>();
    f.cur_iters = cur_iters.as<uint32_t>();
    f.passes = passes.as<uint32_t>();
    f.iters_hist = iters_hist.as<uint32_t>();
    return f;
  }
};

}  // namespace

struct leiden_graph {
  int device = 0;
  hipStream_t own = nullptr;
  MemAccount mem;                 // device bytes held and the budget
  std::atomic<bool> busy{false};  // a call is using the handle
  uint32_t n = 0;
  float slack = 0.2f;
  SlackCsr g;
  Buf b_start, b_alt, b_len, b_cap, b_cols, b_w;
  Buf b_top;  // unsigned long long bump pointer of the overflow area
  Buf edge_parts;  // edge-scan counters of the decide kernels (kEdgeParts x kEdgeStride)
  Buf hist_parts;  // partial rows of the degree histogram (64 x 16 u64)
  uint64_t nnz = 0;
  // auxiliary state (Section 4.4): C, K, Sigma, DeltaSigma
  bool has_state = false;
  Buf st_C, st_K, st_S, st_dS;
  Buf st_head;               // minimum vertex of every label of st_C (kNone: not a label)
  bool heads_valid = false;  // st_head describes st_C
  uint32_t stamp = 0;  // iteration stamp, never reused
  BinCfg bincfg = kDefaultBins;  // degree-bin thresholds (tunable)
  float tune_ms = 0;             // probe time of the last autotuning
  float tune_agg_ms = 0;         // aggregation probe time with the chosen emit table
  uint32_t emit_slots = 4096;    // LDS table of the aggregation emit step (power of two, 16..4096)
  uint64_t sweeps = 0;           // vertices of the per-vertex passes of the current call
  uint32_t run_passes = 0;       // passes of the last run of Alg. 4
  bool run_refined0 = false;     // its first pass refined some community
  // level-0 degree bins
  uint64_t bins0[kBins] = {0};
  uint32_t maxdeg0 = 0;
  // workspace
  Buf C, K, Kb, Kt, S, S2, size, size2, dS, dS2, dR, dR2, CB, rep, Ctop, pend, unproc;
  Buf cls_lists, bin_lists, iter_list, next_list, movers, split_list, split_rest, split_key, split_wide, lab;
  Buf long_items;  // chunk list of the long rows of the input graph
  Buf flag, newid, scan_tmp, ctl, small;
  Buf lvA_start, lvA_len, lvA_cols, lvA_w, lvB_start, lvB_len, lvB_cols, lvB_w;
  Buf agg_count, agg_off, agg_fill, agg_fill2, agg_eoff, agg_members, agg_deg, agg_cap, agg_lists, agg_bigcap, agg_tbl, agg_keys, agg_vals,
      agg_mat, agg_items, mark_items;
  Buf hub_keys, hub_vals, hub_list, hub_idx, hub_off, hub_moff, hub_rbits, hub_size, hub_msize, hub_kid;
  Buf hub_items, hub_mat, hub_live, hub_pdq, hub_pc, hub_done;
  Buf tr_minv, tr_hk, tr_hv, tr_bw, tr_bv, tr_cw, tr_cb, tr_old, tr_flag, tr_rank, tr_frank, tr_fid, tr_label,
      tr_matched, tr_kc, tr_wcom, tr_owners;
  void* tr_clean = nullptr;  // pair table known empty (its allocation)
  Buf dV, dE, dC, sig, partials, modparts;
  Buf bt_src, bt_dst, bt_w, bt_del, bt_slot, bt_rowcnt, bt_rowidx, bt_touched, bt_segcnt, bt_segoff, bt_newlen,
      bt_ssrc, bt_sdst, bt_sw, bt_sdel, bt_sid, bt_spre, bt_slb, bt_sortl, bt_tdst, bt_tw, bt_tdel, bt_in, bt_dest, bt_rlen,
      bt_roff, bt_rsrc, bt_rdst;
  Buf rb_cols, rb_w, rb_off, rb_reserve;
  Buf scatter_ws;  // bucketed scatter reductions over n items
  size_t ws_n = 0, ws_classes = 0;
  uint64_t ws_nnz = 0;
  bool rowcnt_ready = false;
  Ctl* hctl = nullptr;  // pinned mirror
  KTimer kt;
  DecideStreams dstreams{};  // side streams of the decide kernels (created with the handle)
  bool dstreams_ready = false;
  ForestState* forest = nullptr;  // a forest of independent graphs, or null
  ~leiden_graph() {
    delete forest;
    if (dstreams_ready) {
      for (hipStream_t& x : dstreams.aux) (void)hipStreamDestroy(x);
      (void)hipEventDestroy(dstreams.fork);
      for (hipEvent_t& e : dstreams.join) (void)hipEventDestroy(e);
    }
    if (kt.ready)
      for (hipEvent_t& e : kt.ev) (void)hipEventDestroy(e);
    if (hctl) (void)hipHostFree(hctl);
    if (own) (void)hipStreamDestroy(own);
  }
};

// One call at a time per handle: a second call that finds the handle in use
// returns LEIDEN_EBUSY instead of racing on its buffers.
struct BusyGuard {
  std::atomic<bool>* f = nullptr;
  explicit BusyGuard(leiden_graph* G) {
    if (G && !G->busy.exchange(true)) f = &G->busy;
  }
  ~BusyGuard() {
    if (f) f->store(false);
  }
  bool ok() const { return f != nullptr; }
};
// Once a batch is merged into the graph, a call that fails must not leave the
// previous graph's auxiliary state behind as if it described the new one: the
// state is dropped unless the call completes (leiden_static or
// leiden_state_import restores it).
struct StateDrop {
  leiden_graph* G;
  bool armed = true;
  explicit StateDrop(leiden_graph* g) : G(g) {}
  void keep() { armed = false; }
  ~StateDrop() {
    if (armed) {
      G->has_state = false;
      G->heads_valid = false;
    }
  }
};

#define BUSY_GUARD(G)          \
  BusyGuard busy_guard_(G);    \
  if (!busy_guard_.ok()) return fail(LEIDEN_EBUSY, "the handle is in use by another call")

namespace {
const DecideStreams* side_streams(leiden_graph* G, uint32_t nl) {
  constexpr uint32_t kSideMinVertices = 1u << 20;
  if (!G->dstreams_ready || nl < kSideMinVertices || g_in_flight.load() != 1) return nullptr;
  return &G->dstreams;
}
}  // namespace

namespace lm {
thread_local KTimer* tl_ktimer = nullptr;
thread_local const ScatterWs* tl_scatter_ws = nullptr;
}

namespace {

// Points the launch sites at the handle's timer for one call.
struct KtScope {
  explicit KtScope(leiden_graph* G, int which) {
    if (!which) return;
    if (!G->kt.ready) {
      for (hipEvent_t& e : G->kt.ev)
        if (hipEventCreate(&e) != hipSuccess) return;
      G->kt.ready = true;
    }
    G->kt.which = which;
    G->kt.n = 0;
    tl_ktimer = &G->kt;
  }
  ~KtScope() { tl_ktimer = nullptr; }
};

// Points the scatter reductions at the handle's workspace for one call.
struct ScatterScope {
  ScatterWs ws;
  explicit ScatterScope(leiden_graph* G) {
    ws.p = G->scatter_ws.p;
    ws.bytes = G->scatter_ws.bytes;
    tl_scatter_ws = ws.p ? &ws : nullptr;
  }
  ~ScatterScope() { tl_scatter_ws = nullptr; }
};

double kt_unit_bytes(int which) {
  return which == LEIDEN_KT_HUB_INSERT || which == LEIDEN_KT_AGG_BIG ? 12.0 : 0.0;
}

// After the call's final synchronisation: launches, device time, units, bytes.
void kt_collect(leiden_graph* G, int which, leiden_stats* st) {
  if (!which || tl_ktimer != &G->kt) return;
  double ms = 0;
  for (int k = 0; k + 1 < G->kt.n; k += 2) {
    float m = 0;
    if (hipEventElapsedTime(&m, G->kt.ev[k], G->kt.ev[k + 1]) == hipSuccess) ms += m;
  }
  st->kt_launches = (uint32_t)(G->kt.n / 2);
  st->kt_ms = ms;
  st->kt_units = G->hctl->kt_units[which];
  st->kt_bytes = (double)st->kt_units * kt_unit_bytes(which);
}

// Work counters, sweeps and algorithmic bytes of the call into *st (after
// read_ctl_final).  Bytes per unit as leiden.h states them.
void fill_work(leiden_graph* G, leiden_stats* st, uint64_t batch_entries) {
  static const double kUnitBytes[LEIDEN_WORK_COUNT] = {12, 16, 48, 16, 4, 8, 12, 12, 16};
  double bytes = 0;
  for (int u = 0; u < LEIDEN_WORK_COUNT; ++u) {
    st->work[u] = G->hctl->units[u];
    bytes += kUnitBytes[u] * (double)st->work[u];
  }
  st->sweep_vertices = G->sweeps;
  st->batch_entries = batch_entries;
  bytes += 32.0 * (double)G->hctl->total_moves + 16.0 * (double)G->sweeps + 12.0 * (double)batch_entries;
  st->algo_bytes = bytes;
}

hipStream_t stream_of(leiden_graph* g, const leiden_opts* o) {
  return (o && o->stream) ? (hipStream_t)o->stream : g->own;
}

void bind_graph(leiden_graph* G) {
  G->g.start = G->b_start.as<int64_t>();
  G->g.alt = G->b_alt.as<int64_t>();
  G->g.len = G->b_len.as<uint32_t>();
  G->g.cap = G->b_cap.as<uint32_t>();
  G->g.cols = G->b_cols.as<uint32_t>();
  G->g.w = G->b_w.as<uint32_t>();
}

Rows<uint32_t> rows0(leiden_graph* G) { return Rows<uint32_t>{G->g.start, G->g.len, G->g.cols, G->g.w}; }

// The chunk list of the input graph's long rows, sized for its entries.
leiden_status reserve_long_items(leiden_graph* G) {
  return G->long_items.reserve(long_items_bytes(std::max<uint64_t>(G->nnz, 1)));
}

// K[i] = weighted degree of row i of the input graph
leiden_status row_sums(leiden_graph* G, hipStream_t s, int64_t* K) {
  CHK(reserve_long_items(G));
  launch_row_sums_u32(s, rows0(G), G->n, K, G->long_items.as<unsigned long long>());
  return LEIDEN_OK;
}

// Allocate every n- and nnz-sized array a run needs.  Arrays that must start
// zeroed are cleared on the call's stream s: a hipMemset on the null stream
// is asynchronous to the host and not ordered with the non-blocking streams
// the calls run on, so it could land after the first kernels of the call.
leiden_status ensure_workspace(leiden_graph* G, hipStream_t s, uint32_t classes) {
  const size_t n = std::max<size_t>(G->n, 1);
  uint64_t nnz = std::max<uint64_t>(G->nnz, 1);
  if (G->ws_n >= n && G->ws_nnz >= nnz && G->ws_classes >= classes) return LEIDEN_OK;
  nnz += nnz / 4;  // room for the graph to grow by insertions
  const size_t u32 = 4, u64 = 8;
  CHK(G->C.reserve(n * u32));
  CHK(G->K.reserve(n * u64));
  CHK(G->Kb.reserve(n * u64));
  CHK(G->Kt.reserve(n * u64));
  CHK(G->S.reserve(n * u64));
  CHK(G->S2.reserve(n * u64));
  CHK(G->size.reserve(n * u32));
  CHK(G->size2.reserve(n * u32));
  CHK(G->dS.reserve(n));
  CHK(G->dS2.reserve(n));
  CHK(G->dR.reserve(n));
  CHK(G->dR2.reserve(n));
  CHK(G->CB.reserve(n * u32));
  CHK(G->rep.reserve(n * u32));
  CHK(G->Ctop.reserve(n * u32));
  if (G->pend.bytes < n * u32) {
    CHK(G->pend.reserve(n * u32));
    CHK(G->unproc.reserve(n * u32));
    fill_u32(s, G->pend.as<uint32_t>(), 0, n);
    fill_u32(s, G->unproc.as<uint32_t>(), 0, n);
  }
  CHK(G->cls_lists.reserve(n * u32 * classes));
  CHK(G->bin_lists.reserve(n * u32 * kBins));
  CHK(G->iter_list.reserve(n * u32));
  CHK(G->next_list.reserve(n * u32));
  CHK(G->movers.reserve(n * sizeof(Mover)));
  CHK(G->split_list.reserve(n * u32));
  CHK(G->split_rest.reserve(n * u32));
  CHK(G->split_wide.reserve(n * u32));
  CHK(G->split_key.reserve(n * u64));
  CHK(G->lab.reserve(n * u64));  // union-find words of the split
  CHK(G->flag.reserve(n * u32));
  CHK(G->newid.reserve((n + 1) * u64));
  CHK(G->scan_tmp.reserve(scan_tmp_bytes(std::max<uint64_t>(n, 2 * nnz)) + 64));
  CHK(G->ctl.reserve(sizeof(Ctl)));
  CHK(G->edge_parts.reserve(sizeof(unsigned long long) * kEdgeParts * kEdgeStride));
  CHK(G->small.reserve(4096));
  for (Buf* b : {&G->lvA_start, &G->lvB_start}) CHK(b->reserve(n * u64));
  for (Buf* b : {&G->lvA_len, &G->lvB_len}) CHK(b->reserve(n * u32));
  for (Buf* b : {&G->lvA_cols, &G->lvB_cols}) CHK(b->reserve(nnz * u32));
  for (Buf* b : {&G->lvA_w, &G->lvB_w}) CHK(b->reserve(nnz * u64));
  CHK(G->agg_count.reserve(n * u32));
  CHK(G->agg_off.reserve((n + 1) * u64));
  CHK(G->agg_fill.reserve(n * u32));
  CHK(G->agg_fill2.reserve(n * u32));
  CHK(G->agg_eoff.reserve((n + 1) * u64));
  CHK(G->agg_members.reserve(n * u32));
  CHK(G->agg_deg.reserve(n * u64));
  CHK(G->agg_cap.reserve((n + 1) * u64));
  CHK(G->agg_lists.reserve(4 * n * u32));
  CHK(G->agg_bigcap.reserve(4 * n * u64));
  CHK(G->agg_tbl.reserve(n * 48));  // per-round descriptors (32 B) and counters (4 + 8 B) of big communities
  CHK(G->agg_items.reserve(kAggItems * 24));
  CHK(G->mark_items.reserve((nnz / 64 + n + 1) * 8));
  // staging for the big communities of an aggregation: one slot per entry;
  // bucket-start matrices: (R + 1) 16-bit starts per stage column
  const uint64_t scap = nnz + (1 << 16), mcap = nnz + 8 * (uint64_t)n + (1 << 16);
  CHK(G->agg_keys.reserve(scap * u32));
  CHK(G->agg_vals.reserve(scap * u64));
  CHK(G->agg_mat.reserve((mcap + mcap / 1024 + 4096) * 2));
  const uint64_t hslots = next_pow2(2 * n);
  CHK(G->tr_minv.reserve(n * u32));
  const size_t hk_bytes = G->tr_hk.bytes;
  CHK(G->tr_hk.reserve(hslots * u64));
  CHK(G->tr_hv.reserve(hslots * u64));
  if (G->tr_hk.bytes != hk_bytes) G->tr_clean = nullptr;  // a new pair table (perhaps at the old address)
  CHK(G->tr_bw.reserve(n * u64));
  CHK(G->tr_bv.reserve(n * u32));
  CHK(G->tr_cw.reserve(n * u64));
  CHK(G->tr_cb.reserve(n * u32));
  CHK(G->tr_old.reserve(n * u32));
  CHK(G->tr_flag.reserve(n * u32));
  CHK(G->tr_rank.reserve(n * u64));
  CHK(G->tr_frank.reserve(n * u64));
  CHK(G->tr_fid.reserve(n * u32));
  CHK(G->tr_label.reserve(n * u32));
  CHK(G->tr_matched.reserve(n));
  CHK(G->tr_kc.reserve(n * u64));
  CHK(G->tr_wcom.reserve(n * u64));
  CHK(G->tr_owners.reserve(n * u32 + 64));
  CHK(G->dV.reserve(n));
  CHK(G->dE.reserve(n));
  CHK(G->dC.reserve(n));
  CHK(G->sig.reserve(n * u64));
  CHK(G->partials.reserve(4 * 1024 * u64));
  CHK(G->modparts.reserve(sizeof(ModParts)));
  CHK(G->rb_reserve.reserve(n * u32));
  CHK(G->scatter_ws.reserve(scatter_ws_bytes(n, n)));
  CHK(G->rb_off.reserve((n + 1) * u64));
  G->ws_n = n;
  G->ws_nnz = nnz;
  G->ws_classes = classes;
  return LEIDEN_OK;
}

Ctl* dctl(leiden_graph* G) { return G->ctl.as<Ctl>(); }

// Hub tables of the current level: every hub gets a clean region of the
// arena (the select kernel clears what it reads, so the arena stays clean).
leiden_status setup_hubs(leiden_graph* G, hipStream_t s, const uint32_t* len, uint32_t nl) {
  const size_t n = std::max<size_t>(G->n, 1);
  CHK(G->hub_list.reserve(n * 4));
  CHK(G->hub_idx.reserve(n * 4));
  CHK(G->hub_off.reserve((n + 1) * 8));
  CHK(G->hub_moff.reserve((n + 1) * 8));
  CHK(G->hub_msize.reserve(n * 8));
  CHK(G->hub_rbits.reserve(n * 4));
  CHK(G->hub_size.reserve(n * 8));
  if (G->hub_kid.bytes < n * 8) {
    CHK(G->hub_kid.reserve(n * 8));
    HIPCHK(hipMemsetAsync(G->hub_kid.p, 0, n * 8, s));
  }
  HubLayout h{G->hub_list.as<uint32_t>(), G->hub_idx.as<uint32_t>(),   G->hub_off.as<uint64_t>(),
              G->hub_moff.as<uint64_t>(), G->hub_rbits.as<uint32_t>(), G->hub_size.as<uint64_t>(),
              G->hub_msize.as<uint64_t>(), G->hub_kid.as<unsigned long long>()};
  uint32_t cnt = 0;
  uint64_t slots = 0, mat = 0;
  if (hub_layout(s, len, nl, G->bincfg.max_deg[kBins - 2], h, dctl(G), G->scan_tmp.p, G->small.as<uint64_t>() + 64,
                 &cnt, &slots, &mat) != 0)
    return fail(LEIDEN_EDEVICE, "hub layout failed");
  const size_t hc = std::max<uint32_t>(cnt, 1);
  CHK(G->hub_items.reserve((slots / kHubChunk + 1) * 8));  // one per chunk
  CHK(G->hub_mat.reserve(std::max<uint64_t>(mat, 1) * 2));
  if (G->hub_live.bytes < hc * 4) {
    CHK(G->hub_live.reserve(hc * 4));
    fill_u32(s, G->hub_live.as<uint32_t>(), 0, G->hub_live.bytes / 4);
  }
  // segmented pick: per hub up to kHubPickMaxSegs partial results
  CHK(G->hub_pdq.reserve(hc * kHubPickMaxSegs * 8));
  CHK(G->hub_pc.reserve(hc * kHubPickMaxSegs * 4));
  if (G->hub_done.bytes < hc * 4) {
    CHK(G->hub_done.reserve(hc * 4));
    fill_u32(s, G->hub_done.as<uint32_t>(), 0, G->hub_done.bytes / 4);
  }
  // staging: every slot is written before it is read
  CHK(G->hub_keys.reserve(std::max<uint64_t>(slots, 1) * 4));
  CHK(G->hub_vals.reserve(std::max<uint64_t>(slots, 1) * 8));
  return LEIDEN_OK;
}

template <typename W>
void bind_hubs(leiden_graph* G, DecideParams<W>& dp) {
  dp.edge_parts = G->edge_parts.as<unsigned long long>();
  dp.hub_idx = G->hub_idx.as<uint32_t>();
  dp.hub_off = G->hub_off.as<uint64_t>();
  dp.hub_rbits = G->hub_rbits.as<uint32_t>();
  dp.hub_kid = G->hub_kid.as<unsigned long long>();
  dp.hub_keys = G->hub_keys.as<uint32_t>();
  dp.hub_vals = G->hub_vals.as<unsigned long long>();
  dp.hub_items = G->hub_items.as<unsigned long long>();
  dp.hub_moff = G->hub_moff.as<uint64_t>();
  dp.hub_mat = G->hub_mat.as<uint16_t>();
  dp.hub_live = G->hub_live.as<unsigned int>();
  dp.hub_pdq = G->hub_pdq.as<double>();
  dp.hub_pc = G->hub_pc.as<uint32_t>();
  dp.hub_done = G->hub_done.as<unsigned int>();
  dp.pick_segs = 1;  // callers widen it from the level's maximum degree (hub_pick_segs)
}

leiden_status read_ctl(leiden_graph* G, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(G->hctl, G->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return LEIDEN_OK;
}

// One small value from device memory through the pinned stage.
template <typename T>
leiden_status read_dev(hipStream_t s, T* out, const void* dev) {
  T* p = (T*)pinned_stage(sizeof(T));
  if (!p) return fail(LEIDEN_ENOMEM, "pinned staging buffer");
  HIPCHK(hipMemcpyAsync(p, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *out = *p;
  return LEIDEN_OK;
}

__global__ void k_zero_ctl(Ctl* c, unsigned long long* parts) {
  unsigned int* p = (unsigned int*)c;
  for (size_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) p[i] = 0;
  if (parts)
    for (uint32_t i = threadIdx.x; i < kEdgeParts * kEdgeStride; i += blockDim.x) parts[i] = 0;
}

void zero_ctl(leiden_graph* G, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(256), 0, s, dctl(G), G->edge_parts.as<unsigned long long>());
}

// Ctl::units += the spread work counters, which are cleared; Ctl::edges +=
// the local-moving scans.
__global__ void k_fold_edges(Ctl* c, unsigned long long* parts) {
  for (uint32_t u = 0; u < kWUnits; ++u) {
    unsigned long long e = 0;
    if (threadIdx.x < kEdgeParts) {
      e = parts[threadIdx.x * kEdgeStride + u];
      parts[threadIdx.x * kEdgeStride + u] = 0;
    }
    e = group_sum<kWave>(e);
    if (threadIdx.x == 0) {
      c->units[u] += e;
      if (u == kWScan0 || u == kWScanUp) c->edges += e;
    }
  }
}

// read_ctl with the edge-scan counters folded in first (end of a call)
leiden_status read_ctl_final(leiden_graph* G, hipStream_t s) {
  if (G->edge_parts.p)
    hipLaunchKernelGGL(k_fold_edges, dim3(1), dim3(kWave), 0, s, dctl(G), G->edge_parts.as<unsigned long long>());
  return read_ctl(G, s);
}

// Degree bins (vertex counts per bin) and max degree of one level.
leiden_status level_bins(leiden_graph* G, hipStream_t s, const uint32_t* len, uint32_t nl, uint64_t bins[kBins],
                         uint32_t* maxdeg) {
  unsigned long long* d = G->small.as<unsigned long long>();
  CHK(G->hist_parts.reserve(sizeof(unsigned long long) * 64 * 16));
  fill_u64(s, (uint64_t*)d, 0, kBins + 1);
  launch_degree_hist(s, len, nl, G->bincfg, d, (unsigned int*)(d + kBins), G->hist_parts.as<unsigned long long>());
  unsigned long long* h = (unsigned long long*)pinned_stage(sizeof(unsigned long long) * (kBins + 1));
  if (!h) return fail(LEIDEN_ENOMEM, "pinned staging buffer");
  HIPCHK(hipMemcpyAsync(h, d, sizeof(unsigned long long) * (kBins + 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < kBins; ++b) bins[b] = h[b];
  *maxdeg = (uint32_t)h[kBins];
  return LEIDEN_OK;
}

struct RunOpts {
  leiden_opts o;
  bool dynamic;
  int mode;                // for dynamic runs
  const uint8_t* in_range; // first pass of DS, else null
  bool init_all;           // first iteration: every vertex
};

// Mutable per-level state pointers (swapped by subset renumbering).
struct LevelState {
  uint32_t* C;
  int64_t* K;
  int64_t* S;
  uint32_t* size;
  uint8_t* dS;
  uint8_t* dR;
  RenumberBufs rb;
};

struct PassOut {
  uint32_t iters = 0;
  uint32_t subrounds = 0;
  bool refined = false;
};

// Alg. 6 with the blocked synchronous schedule on one level.
template <typename W>
leiden_status local_move(leiden_graph* G, hipStream_t s, Rows<W> g, uint32_t nl, LevelState& L, const RunOpts& ro,
                         bool first_pass, double tau, const QConst& qc, const uint64_t bins[kBins], uint32_t maxdeg,
                         PassOut& out) {
  // the asynchronous mode keeps the class sub-rounds but moves at once
  const bool async = !ro.o.deterministic;
  const uint32_t P = ro.o.move_classes;
  Ctl* ctl = dctl(G);
  uint32_t* iter_list = G->iter_list.as<uint32_t>();
  uint32_t* next_list = G->next_list.as<uint32_t>();
  DecideParams<W> dp{};
  dp.g = g;
  dp.C = L.C;
  dp.K = L.K;
  dp.S = L.S;
  dp.size = L.size;
  dp.inv_m = qc.inv_m;
  dp.inv_2m2 = qc.inv_2m2;
  dp.movers = G->movers.as<Mover>();
  dp.ctl = ctl;
  dp.async = async ? 1 : 0;
  dp.narrow = qc.narrow ? 1 : 0;
  dp.dS = ro.dynamic ? L.dS : nullptr;
  bind_hubs(G, dp);
  dp.pick_segs = hub_pick_segs(maxdeg);
  const uint8_t* in_range = first_pass ? ro.in_range : nullptr;
  for (uint32_t li = 0; li < ro.o.max_iters; ++li) {
    const uint32_t stamp = ++G->stamp;
    launch_iteration_reset(s, ctl, P);  // moves the queued count into iter_count
    std::swap(iter_list, next_list);
    const bool all = li == 0 && (!first_pass || ro.init_all);
    launch_distribute(s, all ? nullptr : iter_list, all ? nullptr : &ctl->iter_count, nl, li, P, stamp,
                      G->pend.as<uint32_t>(), G->cls_lists.as<uint32_t>(), (size_t)nl, ctl);
    // each sub-round's counters are cleared by the iteration reset, or by
    // the previous sub-round's bin (movers, marks) and apply (bins, hubs)
    for (uint32_t k = 0; k < P; ++k) {
      launch_bin(s, G->cls_lists.as<uint32_t>() + (size_t)k * nl, &ctl->cls_count[k], nl, g.len, in_range,
                 G->bin_lists.as<uint32_t>(), (size_t)nl, G->bincfg, G->hub_items.as<unsigned long long>(), ctl);
      launch_decide_all<W, false>(s, dp, G->bin_lists.as<uint32_t>(), (size_t)nl, ctl->bin_count, bins, maxdeg,
                                  side_streams(G, nl));
      ApplyParams ap{};
      ap.start = g.start;
      ap.len = g.len;
      ap.cols = g.cols;
      ap.C = L.C;
      ap.S = L.S;
      ap.K = L.K;
      ap.size = L.size;
      ap.dS = ro.dynamic ? L.dS : nullptr;
      ap.movers = G->movers.as<Mover>();
      ap.ctl = ctl;
      ap.li = li;
      ap.P = P;
      ap.k = k;
      ap.stamp = stamp;
      ap.pend_mark = G->pend.as<uint32_t>();
      ap.unproc_mark = G->unproc.as<uint32_t>();
      ap.cls_lists = G->cls_lists.as<uint32_t>();
      ap.cls_stride = nl;
      ap.next_list = next_list;
      ap.mark_items = G->mark_items.as<unsigned long long>();
      ap.applied = async ? 1 : 0;
      ap.parts = G->edge_parts.as<unsigned long long>();
      launch_apply_moves(s, ap, nl, G->mark_items.bytes / 8);
    }
    if (G->forest) forest_iter_end(s, G->forest->bufs(), tau, li, ro.o.max_iters, ctl);
    CHK(read_ctl(G, s));
    out.iters = li + 1;
    for (uint32_t k = 0; k < P; ++k) out.subrounds += G->hctl->cls_count[k] ? 1 : 0;
    if (G->forest) {
      if (G->hctl->f_moving == 0) break;  // every graph met its own stopping rule
      continue;
    }
    const double dq = (double)(long long)G->hctl->dq_fixed / 72057594037927936.0;
    if (dq <= tau) break;
  }
  // the last iteration queued vertices under stamp + 1; never hand that value out again
  ++G->stamp;
  return LEIDEN_OK;
}

// Alg. 8 with R colour rounds on one level (after subset renumbering / split).
template <typename W>
leiden_status refine(leiden_graph* G, hipStream_t s, Rows<W> g, uint32_t nl, LevelState& L, const RunOpts& ro,
                     const QConst& qc, const uint64_t bins[kBins], uint32_t maxdeg) {
  // the asynchronous mode keeps the colour rounds but moves at once
  const bool async = !ro.o.deterministic;
  const uint32_t R = ro.o.refine_rounds;
  Ctl* ctl = dctl(G);
  launch_cls_reset(s, ctl);
  launch_refine_reset(s, nl, L.C, G->CB.as<uint32_t>(), L.S, L.K, L.size, L.dR, R, G->cls_lists.as<uint32_t>(),
                      (size_t)nl, ctl);
  DecideParams<W> dp{};
  dp.g = g;
  dp.C = L.C;
  dp.K = L.K;
  dp.S = L.S;
  dp.size = L.size;
  dp.CB = G->CB.as<uint32_t>();
  dp.R = R;
  dp.inv_m = qc.inv_m;
  dp.inv_2m2 = qc.inv_2m2;
  dp.movers = G->movers.as<Mover>();
  dp.ctl = ctl;
  dp.async = async ? 1 : 0;
  dp.narrow = qc.narrow ? 1 : 0;
  bind_hubs(G, dp);
  dp.pick_segs = hub_pick_segs(maxdeg);
  // each colour round's counters are cleared by the class reset above, or by
  // the previous round's bin (movers) and apply (bins, hubs)
  for (uint32_t r = 0; r < R; ++r) {
    launch_bin(s, G->cls_lists.as<uint32_t>() + (size_t)r * nl, &ctl->cls_count[r], nl, g.len, nullptr,
               G->bin_lists.as<uint32_t>(), (size_t)nl, G->bincfg, G->hub_items.as<unsigned long long>(), ctl);
    dp.colour = r;
    launch_decide_all<W, true>(s, dp, G->bin_lists.as<uint32_t>(), (size_t)nl, ctl->bin_count, bins, maxdeg,
                               side_streams(G, nl));
    launch_apply_refine(s, L.C, L.S, L.K, L.size, G->movers.as<Mover>(), ctl, nl);
  }
  return LEIDEN_OK;
}

template <typename W>
leiden_status split(leiden_graph* G, hipStream_t s, Rows<W> g, uint32_t nl, LevelState& L,
                    const uint64_t bins[kBins]) {
  Ctl* ctl = dctl(G);
  unsigned long long* lab = G->lab.as<unsigned long long>();
  uint32_t* list = G->split_list.as<uint32_t>();
  uint32_t* rest = G->split_rest.as<uint32_t>();
  unsigned long long* key = G->split_key.as<unsigned long long>();
  uint32_t* wide = G->split_wide.as<uint32_t>();
  launch_split_init(s, nl, L.C, L.dS, L.dR, lab, list, wide, key, ctl, g.len, G->edge_parts.as<unsigned long long>());
  launch_split_sample<W>(s, g, L.C, lab, list, wide, key, rest, ctl, nl);
  // vertices outside their community's main tree, by degree
  launch_subround_reset(s, ctl);
  launch_bin(s, rest, &ctl->split_rest, nl, g.len, nullptr, G->bin_lists.as<uint32_t>(), (size_t)nl, G->bincfg,
             nullptr, ctl);
  launch_split_union<W>(s, g, L.C, lab, G->bin_lists.as<uint32_t>(), (size_t)nl, ctl->bin_count, bins);
  launch_split_finish(s, L.C, lab, list, ctl, nl);
  return LEIDEN_OK;
}

// One pass of Alg. 4 on level graph g; returns whether the pass loop stops.
template <typename W>
leiden_status run_pass(leiden_graph* G, hipStream_t s, Rows<W> g, uint32_t nl, LevelState& L, const RunOpts& ro,
                       uint32_t pass, double tau, const QConst& qc, const uint64_t bins[kBins], uint32_t maxdeg,
                       leiden_stats* st, bool* stop) {
  PassOut po;
  if (bins[kBins - 1]) CHK(setup_hubs(G, s, g.len, nl));
  CHK(local_move<W>(G, s, g, nl, L, ro, pass == 0, tau, qc, bins, maxdeg, po));
  if (st && pass < 16) st->iters[pass] = po.iters, st->subrounds[pass] = po.subrounds;
  // split-all ablation: every community not marked for refinement is split
  if (ro.o.split_all) fill_u8(s, L.dS, 1, nl);
  subset_renumber(s, nl, L.C, L.S, L.size, L.dS, L.dR, L.rb, dctl(G));
  G->sweeps += 2 * (uint64_t)nl;  // Alg. 10 and the refinement reset of Alg. 8
  CHK(read_ctl(G, s));
  const uint32_t nsplit = G->hctl->misc[0], nref = G->hctl->misc[1];
  if (nsplit > 0) CHK(split<W>(G, s, g, nl, L, bins));
  if (st && pass == 0) st->split_marked = nsplit;
  const bool refined = nref > 0;
  if (refined) CHK(refine<W>(G, s, g, nl, L, ro, qc, bins, maxdeg));
  if (st && pass == 0) st->refined_first_pass = refined ? 1 : 0;
  if (pass == 0) G->run_refined0 = refined;
  if (G->forest) {
    // every graph by its own iteration count and refinement flag
    forest_pass_end(s, G->forest->bufs(), pass, dctl(G));
    CHK(read_ctl(G, s));
    *stop = G->hctl->f_live == 0;
    return LEIDEN_OK;
  }
  *stop = (po.iters <= 1 && !refined) || (po.iters <= 1 && pass > 0);
  return LEIDEN_OK;
}

// Aggregate level g (labels L.C renumbered densely) into the next level.
// The aggregation's work buffers of the handle.
AggBufs agg_bufs(leiden_graph* G, uint64_t* total) {
  AggBufs ab{};
  ab.comm_count = G->agg_count.as<uint32_t>();
  ab.comm_off = G->agg_off.as<uint64_t>();
  ab.comm_fill = G->agg_fill.as<uint32_t>();
  ab.comm_fill_long = G->agg_fill2.as<uint32_t>();
  ab.member_eoff = G->agg_eoff.as<uint64_t>();
  ab.members = G->agg_members.as<uint32_t>();
  ab.comm_deg = G->agg_deg.as<uint64_t>();
  ab.cap_off = G->agg_cap.as<uint64_t>();
  ab.total = total;
  ab.scan_tmp = G->scan_tmp.p;
  ab.small_lists = G->agg_lists.as<uint32_t>();
  ab.big_info = G->agg_bigcap.as<uint64_t>();
  ab.bigc = G->agg_tbl.p;
  ab.items = G->agg_items.p;
  ab.item_cap = kAggItems;
  ab.stage_ctr = (unsigned long long*)((char*)G->agg_tbl.p + 32 * (size_t)G->n);
  ab.self_acc = (unsigned long long*)((char*)G->agg_tbl.p + 40 * (size_t)G->n);
  ab.skeys = G->agg_keys.as<uint32_t>();
  ab.svals = G->agg_vals.as<unsigned long long>();
  ab.smat = G->agg_mat.as<uint16_t>();
  ab.scap = G->agg_keys.bytes / 4;
  ab.mcap = G->agg_mat.bytes / 2;
  ab.emit_cap = G->emit_slots;
  ab.slice_ctl = (unsigned int*)(G->small.as<uint64_t>() + 400);
  return ab;
}

template <typename W>
leiden_status next_level(leiden_graph* G, hipStream_t s, Rows<W> g, uint32_t nl, LevelState& L, bool useA,
                         Rows<int64_t>* out, uint32_t* nc_out) {
  uint64_t* total = G->small.as<uint64_t>() + 64;
  dense_renumber(s, nl, L.C, G->flag.as<uint32_t>(), G->newid.as<uint64_t>(), total, G->scan_tmp.p);
  uint64_t nc = 0;
  CHK(read_dev(s, &nc, total));
  launch_lookup(s, G->Ctop.as<uint32_t>(), L.C, G->n);
  if (ForestState* FS = G->forest) {
    // graphs that left the pass loop are aggregated without their entries
    forest_live_len(s, nl, FS->cur_gid, FS->pass.as<uint8_t>(), g.len, FS->live_len.as<uint32_t>());
    g.len = FS->live_len.as<uint32_t>();
    // the next level's graphs: first super-vertices and the graph of each
    const bool toA = FS->cur_gid != FS->gidA.as<uint32_t>();
    uint32_t* nb = toA ? FS->baseA.as<uint32_t>() : FS->baseB.as<uint32_t>();
    uint32_t* ng = toA ? FS->gidA.as<uint32_t>() : FS->gidB.as<uint32_t>();
    forest_next_base(s, FS->nq, nl, FS->cur_base, G->newid.as<uint64_t>(), total, nb);
    forest_gid(s, (uint32_t)nc, FS->nq, nb, ng);
    forest_bind(s, dctl(G), FS->bufs(), ng, nb);
    FS->cur_gid = ng;
    FS->cur_base = nb;
  }
  Buf& bs = useA ? G->lvA_start : G->lvB_start;
  Buf& bl = useA ? G->lvA_len : G->lvB_len;
  Buf& bc = useA ? G->lvA_cols : G->lvB_cols;
  Buf& bw = useA ? G->lvA_w : G->lvB_w;
  AggBufs ab = agg_bufs(G, total);
  // K of the next level goes to whichever of the two K buffers is not current
  int64_t* Kn = L.K == G->K.as<int64_t>() ? G->Kb.as<int64_t>() : G->K.as<int64_t>();
  count_units(s, g.len, nullptr, nl, G->edge_parts.as<unsigned long long>(), kWAggIn);
  // the input graph's rows are sorted by column (required of the input and
  // kept by the batch merge); aggregated levels are not
  int rc = aggregate<W>(s, g, nl, L.C, (uint32_t)nc, ab, bs.as<int64_t>(), bl.as<uint32_t>(), bc.as<uint32_t>(),
                        bw.as<int64_t>(), Kn, dctl(G), std::is_same<W, uint32_t>::value);
  if (rc != 0) return fail(LEIDEN_EDEVICE, "aggregation failed (%d)", rc);
  count_units(s, bl.as<uint32_t>(), nullptr, nc, G->edge_parts.as<unsigned long long>(), kWAggOut);
  // dense renumbering, C <- C'[C] over the input vertices, next-level set-up
  G->sweeps += 2 * (uint64_t)nl + G->n + nc;
  // K' = Sigma' = weight of each super-vertex; C' = identity; all refined; none split
  HIPCHK(hipMemcpyAsync(L.S, Kn, sizeof(int64_t) * nc, hipMemcpyDeviceToDevice, s));
  L.K = Kn;
  fill_u32(s, L.size, 1, nc);
  iota_u32(s, L.C, nc);
  fill_u8(s, L.dR, 1, nc);
  fill_u8(s, L.dS, 0, nc);
  *out = Rows<int64_t>{bs.as<int64_t>(), bl.as<uint32_t>(), bc.as<uint32_t>(), bw.as<int64_t>()};
  *nc_out = (uint32_t)nc;
  return LEIDEN_OK;
}

// Alg. 4 over all levels.  On entry L holds C^{t-1} (identity for static
// runs), K^t, Sigma^t, the split / refine flags, and (dynamic DF / DS) the
// first unprocessed list queued in next_list.  On exit Ctop holds C.
leiden_status run_leiden(leiden_graph* G, hipStream_t s, LevelState& L, const RunOpts& ro, uint64_t M2,
                         leiden_stats* st) {
  const uint32_t n = G->n;
  iota_u32(s, G->Ctop.as<uint32_t>(), n);
  G->run_passes = 0;
  G->run_refined0 = false;
  if (ForestState* FS = G->forest) {
    // per-graph constants come from forest_prepare; graphs without edges
    // take no part, and their vertices stay alone
    FS->cur_gid = FS->gid0.as<uint32_t>();
    FS->cur_base = FS->base0.as<uint32_t>();
    forest_start(s, FS->bufs(), dctl(G));
    forest_bind(s, dctl(G), FS->bufs(), FS->cur_gid, FS->cur_base);
    forest_isolate(s, n, FS->cur_gid, FS->pass.as<uint8_t>(), L.C);
  }
  if (M2 == 0 || n == 0) {  // no edges: every vertex stays alone
    iota_u32(s, L.C, n);
    return LEIDEN_OK;
  }
  const QConst qc = make_qconst(M2);
  launch_count_members(s, L.C, n, L.size);
  double tau = ro.o.tau;
  uint64_t bins[kBins];
  for (int b = 0; b < kBins; ++b) bins[b] = G->bins0[b];
  uint32_t maxdeg = G->maxdeg0;
  Rows<int64_t> cur{};
  uint32_t nl = n;
  bool useA = true;
  uint32_t pass = 0;
  for (; pass < ro.o.max_passes; ++pass) {
    bool stop = false;
    if (pass == 0)
      CHK(run_pass<uint32_t>(G, s, rows0(G), nl, L, ro, pass, tau, qc, bins, maxdeg, st, &stop));
    else
      CHK(run_pass<int64_t>(G, s, cur, nl, L, ro, pass, tau, qc, bins, maxdeg, st, &stop));
    if (stop) break;
    Rows<int64_t> nxt{};
    uint32_t nc = 0;
    if (pass == 0)
      CHK(next_level<uint32_t>(G, s, rows0(G), nl, L, useA, &nxt, &nc));
    else
      CHK(next_level<int64_t>(G, s, cur, nl, L, useA, &nxt, &nc));
    cur = nxt;
    nl = nc;
    useA = !useA;
    CHK(level_bins(G, s, cur.len, nl, bins, &maxdeg));
    tau = tau / (double)ro.o.tol_decline;
  }
  G->run_passes = pass < ro.o.max_passes ? pass + 1 : ro.o.max_passes;
  if (st) st->passes = G->run_passes;
  launch_lookup(s, G->Ctop.as<uint32_t>(), L.C, n);
  G->sweeps += n;
  return LEIDEN_OK;
}

LevelState level_state(leiden_graph* G) {
  LevelState L;
  L.C = G->C.as<uint32_t>();
  L.K = G->K.as<int64_t>();
  L.S = G->S.as<int64_t>();
  L.size = G->size.as<uint32_t>();
  L.dS = G->dS.as<uint8_t>();
  L.dR = G->dR.as<uint8_t>();
  L.rb.rep = G->rep.as<uint32_t>();
  L.rb.S2 = G->S2.as<int64_t>();
  L.rb.size2 = G->size2.as<uint32_t>();
  L.rb.dS2 = G->dS2.as<uint8_t>();
  L.rb.dR2 = G->dR2.as<uint8_t>();
  return L;
}

leiden_status check_opts(const leiden_opts& o) {
  if (o.move_classes < 1 || o.move_classes > (uint32_t)kMaxClasses)
    return fail(LEIDEN_EINVAL, "move_classes must be in 1..%d", kMaxClasses);
  if (o.refine_rounds < 1 || o.refine_rounds > (uint32_t)kMaxClasses)
    return fail(LEIDEN_EINVAL, "refine_rounds must be in 1..%d", kMaxClasses);
  if (o.tau_re_den == 0 || o.tol_decline == 0 || o.max_iters == 0)
    return fail(LEIDEN_EINVAL, "tau_re_den, tol_decline and max_iters must be > 0");
  if (!(o.tau >= 0.0)) return fail(LEIDEN_EINVAL, "tau must be >= 0");
  if (o.split_all != 0 && o.split_all != 1) return fail(LEIDEN_EINVAL, "split_all must be 0 or 1");
  if (o.timed_kernel < LEIDEN_KT_NONE || o.timed_kernel > LEIDEN_KT_AGG_BIG)
    return fail(LEIDEN_EINVAL, "unknown timed_kernel");
  return LEIDEN_OK;
}

leiden_status modularity_of(leiden_graph* G, hipStream_t s, const uint32_t* C, const int64_t* K, double* q) {
  const int nb = 1024;
  ModParts* mp = G->modparts.as<ModParts>();
  CHK(reserve_long_items(G));
  modularity_parts(s, rows0(G), G->n, C, K, G->sig.as<int64_t>(), G->partials.as<unsigned long long>(), nb, mp,
                   G->long_items.as<unsigned long long>());
  unsigned long long* m2d = G->small.as<unsigned long long>() + 128;
  sum_i64(s, K, G->n, m2d);
  char* st = (char*)pinned_stage(sizeof(ModParts) + 8);
  if (!st) return fail(LEIDEN_ENOMEM, "pinned staging buffer");
  HIPCHK(hipMemcpyAsync(st, mp, sizeof(ModParts), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(st + sizeof(ModParts), m2d, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ModParts h;
  unsigned long long M2 = 0;
  std::memcpy(&h, st, sizeof(ModParts));
  std::memcpy(&M2, st + sizeof(ModParts), 8);
  if (M2 == 0) {
    *q = 0.0;
    return LEIDEN_OK;
  }
  const unsigned __int128 T = ((unsigned __int128)h.T_hi << 64) | h.T_lo;
  const double m2 = (double)M2;
  const double first = (double)h.sigma / m2;
  const double second = (double)T / (m2 * m2);
  *q = first - second;
  return LEIDEN_OK;
}

// A forest's per-graph 2m and Eq. 2 constants from the weighted degrees K
// (the host formula of one graph, per graph).
leiden_status forest_prepare(leiden_graph* G, hipStream_t s, const int64_t* K) {
  ForestState* FS = G->forest;
  const uint32_t nq = FS->nq;
  fill_u64(s, FS->m2.as<uint64_t>(), 0, nq);
  forest_sum(s, G->n, FS->gid0.as<uint32_t>(), K, FS->m2.as<unsigned long long>());
  std::vector<unsigned long long> m2(nq);
  HIPCHK(hipMemcpyAsync(m2.data(), FS->m2.p, 8 * (size_t)nq, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> inv(2 * (size_t)nq, 0.0);
  for (uint32_t q = 0; q < nq; ++q) {
    if (!m2[q]) continue;
    const QConst c = make_qconst(m2[q]);
    inv[2 * (size_t)q] = c.inv_m;
    inv[2 * (size_t)q + 1] = c.inv_2m2;
  }
  HIPCHK(hipMemcpyAsync(FS->inv.p, inv.data(), 16 * (size_t)nq, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return LEIDEN_OK;
}

// Per-graph results of a forest call: passes and iteration counts of the run
// (when `ran`), and Eq. 1 of every graph under the forest labels C (NaN when
// modularity is not asked for).
leiden_status forest_collect(leiden_graph* G, hipStream_t s, bool ran, const uint32_t* C, const int64_t* K,
                             bool modularity) {
  ForestState* FS = G->forest;
  const uint32_t nq = FS->nq;
  if (ran) {
    FS->passes_h.assign(nq, 0);
    FS->iters_h.assign((size_t)kForestIterHist * nq, 0);
    HIPCHK(hipMemcpyAsync(FS->passes_h.data(), FS->passes.p, 4 * (size_t)nq, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(FS->iters_h.data(), FS->iters_hist.p, 4 * (size_t)kForestIterHist * nq,
                          hipMemcpyDeviceToHost, s));
  }
  FS->q.assign(nq, std::numeric_limits<double>::quiet_NaN());
  std::vector<unsigned long long> parts;
  if (modularity) {
    forest_modularity_parts(s, rows0(G), G->n, nq, C, K, FS->gid0.as<uint32_t>(), G->sig.as<int64_t>(),
                            FS->parts.as<unsigned long long>());
    parts.resize(4 * (size_t)nq);
    HIPCHK(hipMemcpyAsync(parts.data(), FS->parts.p, 32 * (size_t)nq, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (uint32_t q = 0; q < nq && modularity; ++q) {
    const unsigned long long M2 = parts[3 * (size_t)nq + q];
    if (M2 == 0) {
      FS->q[q] = 0.0;
      continue;
    }
    const unsigned __int128 T = ((unsigned __int128)parts[nq + (size_t)q] << 64) | parts[2 * (size_t)nq + q];
    const double m2 = (double)M2;
    const double first = (double)parts[q] / m2;
    const double second = (double)T / (m2 * m2);
    FS->q[q] = first - second;
  }
  return LEIDEN_OK;
}

leiden_status copy_out(hipStream_t s, void* dst, const void* src, size_t bytes, int on_device) {
  if (!dst || !bytes) return LEIDEN_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  return LEIDEN_OK;
}

leiden_status copy_in(hipStream_t s, void* dst, const void* src, size_t bytes, int on_device) {
  if (!bytes) return LEIDEN_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  return LEIDEN_OK;
}

// Entries allocated for a layout whose row capacities sum to tot: two spans
// per row plus an overflow area for rows that outgrow them.
uint64_t edge_capacity(uint64_t tot) { return 2 * tot + tot / 4 + 8192; }

// Rebuild the slack CSR so every row has room for `reserve` entries (or its
// current length when reserve is null), with fresh per-row slack.
leiden_status rebuild(leiden_graph* G, hipStream_t s, const uint32_t* reserve) {
  const uint32_t n = G->n;
  uint64_t* total = G->small.as<uint64_t>() + 200;
  CHK(G->rb_off.reserve((uint64_t)(n + 1) * 8));
  rebuild_caps(s, n, G->g.len, reserve, G->slack, G->g.cap, G->rb_off.as<uint64_t>(), G->scan_tmp.p, total);
  uint64_t tot = 0;
  CHK(read_dev(s, &tot, total));
  const uint64_t cap = edge_capacity(tot);
  Buf nc, nw;
  CHK(nc.reserve(cap * 4));
  CHK(nw.reserve(cap * 4));
  copy_rows(s, n, G->g.start, G->g.len, G->g.cap, G->g.cols, G->g.w, G->rb_off.as<uint64_t>(), nc.as<uint32_t>(),
            nw.as<uint32_t>(), G->g.start, G->g.alt);
  unsigned long long top = 2 * tot;
  HIPCHK(hipMemcpyAsync(G->b_top.p, &top, sizeof(top), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  std::swap(G->b_cols.p, nc.p);
  std::swap(G->b_cols.bytes, nc.bytes);
  std::swap(G->b_w.p, nw.p);
  std::swap(G->b_w.bytes, nw.bytes);
  bind_graph(G);
  G->g.edge_cap = cap;
  return LEIDEN_OK;
}


// ---------------------------------------------------------------------------
// Degree-bin autotuning.  The probe is one local-moving iteration of the
// synchronous schedule over every vertex of the input graph, starting from
// singleton communities, with decisions only (nothing is applied), timed with
// events; it runs the same decide kernels as the first iteration of a static
// run.  Coordinate descent over the five thresholds, each tried at a few
// multiples of its current value within the capacity of its bin.
// ---------------------------------------------------------------------------
bool bins_valid(const BinCfg& c) {
  for (int b = 0; b < kBins - 1; ++b) {
    if (c.max_deg[b] < 1 || c.max_deg[b] > kBinCap[b]) return false;
    if (b > 0 && c.max_deg[b] <= c.max_deg[b - 1]) return false;
  }
  return true;
}

leiden_status probe_decide(leiden_graph* G, hipStream_t s, const leiden_opts& o, float* ms_out) {
  const uint32_t n = G->n;
  const uint32_t P = o.move_classes;
  Ctl* ctl = dctl(G);
  LevelState L = level_state(G);
  uint64_t bins[kBins];
  uint32_t maxdeg = 0;
  CHK(level_bins(G, s, G->g.len, n, bins, &maxdeg));
  if (bins[kBins - 1]) CHK(setup_hubs(G, s, G->g.len, n));
  unsigned long long* m2d = G->small.as<unsigned long long>() + 128;
  sum_i64(s, L.K, n, m2d);
  unsigned long long M2 = 0;
  CHK(read_dev(s, &M2, m2d));
  const QConst qc = make_qconst(M2 ? M2 : 1);
  DecideParams<uint32_t> dp{};
  dp.g = rows0(G);
  dp.C = L.C;
  dp.K = L.K;
  dp.S = L.S;
  dp.size = L.size;
  dp.inv_m = qc.inv_m;
  dp.inv_2m2 = qc.inv_2m2;
  dp.movers = G->movers.as<Mover>();
  dp.ctl = ctl;
  bind_hubs(G, dp);
  dp.pick_segs = hub_pick_segs(maxdeg);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  const uint32_t stamp = ++G->stamp;
  launch_cls_reset(s, ctl);
  launch_distribute(s, nullptr, nullptr, n, 0, P, stamp, G->pend.as<uint32_t>(), G->cls_lists.as<uint32_t>(),
                    (size_t)n, ctl);
  for (uint32_t k = 0; k < P; ++k) {
    launch_subround_reset(s, ctl);
    launch_bin(s, G->cls_lists.as<uint32_t>() + (size_t)k * n, &ctl->cls_count[k], n, G->g.len, nullptr,
               G->bin_lists.as<uint32_t>(), (size_t)n, G->bincfg, G->hub_items.as<unsigned long long>(), ctl);
    launch_decide_all<uint32_t, false>(s, dp, G->bin_lists.as<uint32_t>(), (size_t)n, ctl->bin_count, bins, maxdeg,
                                       side_streams(G, n));
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  ++G->stamp;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms;
  return LEIDEN_OK;
}

// Probe membership for timing the aggregation: every vertex joins its
// smallest neighbour (or stays alone), one wavefront per row.  Communities
// then range from pairs to the stars of low-ID hubs.
__global__ __launch_bounds__(kBlock) void k_probe_min_label(Rows<uint32_t> g, uint32_t n, uint32_t* C) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t i = wave; i < n; i += nwaves) {
    uint32_t m = (uint32_t)i;
    const int64_t s0 = g.start[i];
    for (uint32_t e = lane; e < g.len[i]; e += kWave) m = min(m, g.cols[s0 + e]);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o));
    if (lane == 0) C[i] = m;
  }
}

// One aggregation (Alg. 9) of the input graph under the probe membership with
// an emit table of `slots` slots, timed with events; the handle's graph and
// state are not touched (the level buffers are scratch between calls).
leiden_status probe_aggregate(leiden_graph* G, hipStream_t s, uint32_t slots, float* ms_out) {
  const uint32_t n = G->n;
  uint32_t* C = G->CB.as<uint32_t>();
  const uint64_t nwave_blocks = std::min<uint64_t>(16384, (n + kBlock / kWave - 1) / (kBlock / kWave));
  hipLaunchKernelGGL(k_probe_min_label, dim3((uint32_t)std::max<uint64_t>(nwave_blocks, 1)), dim3(kBlock), 0, s,
                     rows0(G), n, C);
  uint64_t* total = G->small.as<uint64_t>() + 64;
  dense_renumber(s, n, C, G->flag.as<uint32_t>(), G->newid.as<uint64_t>(), total, G->scan_tmp.p);
  uint64_t nc = 0;
  CHK(read_dev(s, &nc, total));
  AggBufs ab = agg_bufs(G, total);
  ab.emit_cap = slots;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  const int rc = aggregate<uint32_t>(s, rows0(G), n, C, (uint32_t)nc, ab, G->lvA_start.as<int64_t>(),
                                     G->lvA_len.as<uint32_t>(), G->lvA_cols.as<uint32_t>(), G->lvA_w.as<int64_t>(),
                                     G->Kb.as<int64_t>(), dctl(G), true);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != 0) return fail(LEIDEN_EDEVICE, "aggregation probe failed (%d)", rc);
  *ms_out = ms;
  return LEIDEN_OK;
}

// Level-0 degree bins after a change of thresholds.
leiden_status refresh_bins0(leiden_graph* G) {
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  CHK(level_bins(G, s, G->g.len, G->n, G->bins0, &G->maxdeg0));
  HIPCHK(hipStreamSynchronize(s));
  return LEIDEN_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

leiden_status leiden_default_opts(leiden_opts* o) {
  if (!o) return fail(LEIDEN_EINVAL, "null opts");
  o->tau = 1e-2;
  o->tau_re_num = 3;
  o->tau_re_den = 5;
  o->tol_decline = 10;
  o->max_iters = 20;
  o->max_passes = 10;
  o->move_classes = 4;
  o->refine_rounds = 8;
  o->deterministic = 1;
  o->compute_modularity = 1;
  o->stream = nullptr;
  o->timed_kernel = LEIDEN_KT_NONE;
  o->split_all = 0;
  return LEIDEN_OK;
}

const char* leiden_kernel_name(int32_t kernel) {
  switch (kernel) {
    case LEIDEN_KT_NONE:
      return "";
    case LEIDEN_KT_HUB_INSERT:  // two instantiations (32- or 64-bit table sums): their common prefix
      return "lm::k_hub_chunk<unsigned int, false";
    case LEIDEN_KT_AGG_BIG:
      return "lm::k_agg_stage<unsigned int>";
    default:
      return nullptr;
  }
}


static void tuning_of(const leiden_graph* G, leiden_tuning* out) {
  std::memset(out, 0, sizeof(*out));
  for (int b = 0; b < kBins - 1; ++b) out->bin_max_degree[b] = G->bincfg.max_deg[b];
  out->agg_emit_slots = G->emit_slots;
  out->probe_ms = G->tune_ms;
  out->agg_probe_ms = G->tune_agg_ms;
}

leiden_status leiden_get_tuning(leiden_graph* G, leiden_tuning* out) {
  g_err.clear();
  if (!G || !out) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  tuning_of(G, out);
  return LEIDEN_OK;
}

leiden_status leiden_set_tuning(leiden_graph* G, const leiden_tuning* t) {
  g_err.clear();
  if (!G || !t) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  BinCfg c = kDefaultBins;
  for (int b = 0; b < kBins - 1; ++b) c.max_deg[b] = t->bin_max_degree[b];
  if (!bins_valid(c))
    return fail(LEIDEN_EINVAL, "bin thresholds must increase and stay within %u, %u, %u, %u, %u", kBinCap[0],
                kBinCap[1], kBinCap[2], kBinCap[3], kBinCap[4]);
  const uint32_t es = t->agg_emit_slots ? t->agg_emit_slots : 4096;
  if (es < 16 || es > 4096 || (es & (es - 1)))
    return fail(LEIDEN_EINVAL, "agg_emit_slots must be 0 or a power of two in 16..4096");
  G->emit_slots = es;
  G->bincfg = c;
  CHK(refresh_bins0(G));
  return LEIDEN_OK;
}

leiden_status leiden_autotune(leiden_graph* G, const leiden_opts* opts, leiden_tuning* out) {
  g_err.clear();
  InFlight in_flight;
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  leiden_opts o;
  leiden_default_opts(&o);
  if (opts) o = *opts;
  CHK(check_opts(o));
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = stream_of(G, opts);
  AllocScope alloc_scope(s, &G->mem);
  CHK(ensure_workspace(G, s, std::max(o.move_classes, o.refine_rounds)));
  const uint32_t n = G->n;
  // singleton start on the input graph
  zero_ctl(G, s);
  LevelState L = level_state(G);
  CHK(row_sums(G, s, L.K));
  HIPCHK(hipMemcpyAsync(L.S, L.K, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
  iota_u32(s, L.C, n);
  fill_u32(s, L.size, 1, n);
  auto measure = [&](const BinCfg& c, float* best) -> leiden_status {
    G->bincfg = c;
    float a = 0, b = 0;
    CHK(probe_decide(G, s, o, &a));
    CHK(probe_decide(G, s, o, &b));
    *best = std::min(a, b);
    return LEIDEN_OK;
  };
  BinCfg cur = G->bincfg;
  float cur_ms = 0;
  CHK(measure(cur, &cur_ms));
  static const double kSteps[] = {0.5, 0.75, 1.5, 2.0};
  for (int round = 0; round < 2; ++round) {
    bool improved = false;
    for (int b = 0; b < kBins - 1; ++b) {
      for (double f : kSteps) {
        BinCfg c = cur;
        c.max_deg[b] = std::min<uint32_t>(kBinCap[b], std::max<uint32_t>(1, (uint32_t)(cur.max_deg[b] * f)));
        if (c.max_deg[b] == cur.max_deg[b] || !bins_valid(c)) continue;
        float ms = 0;
        CHK(measure(c, &ms));
        if (ms < cur_ms * 0.98f) {  // keep a change only for a clear gain
          cur = c;
          cur_ms = ms;
          improved = true;
        }
      }
    }
    if (!improved) break;
  }
  G->bincfg = cur;
  G->tune_ms = cur_ms;
  CHK(refresh_bins0(G));
  // the aggregation's emit table: the fastest of a few sizes (the default
  // unless another is clearly faster)
  uint32_t best_slots = G->emit_slots;
  float best_agg = 0;
  for (const uint32_t slots : {4096u, 2048u, 1024u, 512u}) {
    float a = 0, b = 0;
    CHK(probe_aggregate(G, s, slots, &a));
    CHK(probe_aggregate(G, s, slots, &b));
    const float t = std::min(a, b);
    if (slots == 4096u || t < best_agg * 0.98f) {
      best_slots = slots;
      best_agg = t;
    }
  }
  G->emit_slots = best_slots;
  G->tune_agg_ms = best_agg;
  if (out) tuning_of(G, out);
  return LEIDEN_OK;
}

const char* leiden_last_error(void) { return g_err.c_str(); }

leiden_status leiden_graph_create(int device, uint32_t n, uint64_t nnz, const int64_t* offsets, const uint32_t* cols,
                                  const uint32_t* w, int on_device, double slack, leiden_graph** out) {
  g_err.clear();
  if (!out) return fail(LEIDEN_EINVAL, "null output handle");
  *out = nullptr;
  if (!offsets || (nnz && (!cols || !w))) return fail(LEIDEN_EINVAL, "null CSR arrays");
  if (!(slack >= 0.0) || slack > 64.0) return fail(LEIDEN_EINVAL, "slack must be in [0, 64]");
  if (n == 0xFFFFFFFFu) return fail(LEIDEN_EINVAL, "n too large");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(LEIDEN_EINVAL, "no device %d", device);
  HIPCHK(hipSetDevice(device));
  leiden_graph* G = new leiden_graph();
  G->device = device;
  G->n = n;
  G->slack = (float)slack;
  G->nnz = nnz;
  auto bail = [&](leiden_status st) {
    delete G;
    return st;
  };
  if (hipStreamCreateWithFlags(&G->own, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(LEIDEN_EDEVICE, "stream creation failed"));
  if (hipHostMalloc((void**)&G->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
    return bail(fail(LEIDEN_EDEVICE, "pinned allocation failed"));
  {
    DecideStreams& d = G->dstreams;
    bool ok = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < kDecideSide && ok; ++k)
      ok = hipStreamCreateWithFlags(&d.aux[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&d.join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) return bail(fail(LEIDEN_EDEVICE, "stream creation failed"));
    G->dstreams_ready = true;
  }
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  leiden_status st;
  // upload the input CSR
  Buf in_offs, in_cols, in_w;
  if ((st = in_offs.reserve((uint64_t)(n + 1) * 8)) || (st = in_cols.reserve(nnz * 4)) ||
      (st = in_w.reserve(nnz * 4)))
    return bail(st);
  auto up = [&](void* d, const void* h, size_t b) {
    return hipMemcpyAsync(d, h, b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
  };
  if (up(in_offs.p, offsets, (uint64_t)(n + 1) * 8) != hipSuccess || (nnz && up(in_cols.p, cols, nnz * 4) != hipSuccess) ||
      (nnz && up(in_w.p, w, nnz * 4) != hipSuccess))
    return bail(fail(LEIDEN_EDEVICE, "input copy failed"));
  if ((st = G->small.reserve(4096)) || (st = G->ctl.reserve(sizeof(Ctl)))) return bail(st);
  const unsigned int err = csr_check(s, n, nnz, in_offs.as<int64_t>(), in_cols.as<uint32_t>(), in_w.as<uint32_t>(),
                                     (unsigned int*)G->small.p);
  if (err & 0x80000000u) return bail(fail(LEIDEN_EDEVICE, "input check failed"));
  if (err & 16) return bail(fail(LEIDEN_EINVAL, "offsets must start at 0, end at nnz and not decrease"));
  if (err & 1) return bail(fail(LEIDEN_EINVAL, "column out of range, self-loop or zero weight"));
  if (err & 2) return bail(fail(LEIDEN_EINVAL, "rows must be sorted without duplicate columns"));
  if (err & 4) return bail(fail(LEIDEN_EINVAL, "matrix is not symmetric (missing or unequal reverse entry)"));
  // slack layout
  const size_t nn = std::max<size_t>(n, 1);
  if ((st = G->b_start.reserve(nn * 8)) || (st = G->b_alt.reserve(nn * 8)) || (st = G->b_len.reserve(nn * 4)) ||
      (st = G->b_cap.reserve(nn * 4)) ||
      (st = G->b_top.reserve(8)) || (st = G->rb_off.reserve((nn + 1) * 8)) ||
      (st = G->scan_tmp.reserve(scan_tmp_bytes(std::max<uint64_t>(nn, 2 * nnz)) + 64)))
    return bail(st);
  bind_graph(G);
  uint64_t* total = G->small.as<uint64_t>() + 200;
  caps_from_csr(s, n, in_offs.as<int64_t>(), G->slack, G->g, G->rb_off.as<uint64_t>(), G->scan_tmp.p, total);
  uint64_t tot = 0;
  if (hipMemcpyAsync(&tot, total, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(LEIDEN_EDEVICE, "layout failed"));
  const uint64_t cap = edge_capacity(tot);
  if ((st = G->b_cols.reserve(cap * 4)) || (st = G->b_w.reserve(cap * 4))) return bail(st);
  bind_graph(G);
  G->g.edge_cap = cap;
  copy_rows(s, n, in_offs.as<int64_t>(), G->g.len, G->g.cap, in_cols.as<uint32_t>(), in_w.as<uint32_t>(),
            G->rb_off.as<uint64_t>(), G->g.cols, G->g.w, G->g.start, G->g.alt);
  unsigned long long top = 2 * tot;
  if (hipMemcpyAsync(G->b_top.p, &top, 8, hipMemcpyHostToDevice, s) != hipSuccess) return bail(fail(LEIDEN_EDEVICE, "copy"));
  G->bins0[0] = 0;
  if ((st = level_bins(G, s, G->g.len, n, G->bins0, &G->maxdeg0))) return bail(st);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(LEIDEN_EDEVICE, "graph creation failed"));
  *out = G;
  return LEIDEN_OK;
}

void leiden_graph_destroy(leiden_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipStreamSynchronize(g->own);
  delete g;
}

leiden_status leiden_forest_create(int device, uint32_t n_graphs, const uint32_t* graph_vertices, uint64_t nnz,
                                   const int64_t* offsets, const uint32_t* cols, const uint32_t* w, int on_device,
                                   double slack, leiden_graph** out) {
  g_err.clear();
  if (!out) return fail(LEIDEN_EINVAL, "null output handle");
  *out = nullptr;
  if (n_graphs == 0 || !graph_vertices) return fail(LEIDEN_EINVAL, "a forest needs at least one graph");
  std::vector<uint32_t> first(n_graphs + 1, 0);
  uint64_t n = 0;
  for (uint32_t q = 0; q < n_graphs; ++q) {
    if (graph_vertices[q] == 0) return fail(LEIDEN_EINVAL, "graph %u has no vertices", q);
    first[q] = (uint32_t)n;
    n += graph_vertices[q];
    if (n >= 0xFFFFFFFFull) return fail(LEIDEN_EINVAL, "too many vertices");
  }
  first[n_graphs] = (uint32_t)n;
  leiden_graph* G = nullptr;
  CHK(leiden_graph_create(device, (uint32_t)n, nnz, offsets, cols, w, on_device, slack, &G));
  ForestState* FS = new ForestState();
  G->forest = FS;
  FS->nq = n_graphs;
  FS->first = first;
  auto bail = [&](leiden_status st) {
    leiden_graph_destroy(G);
    return st;
  };
  const size_t nn = std::max<uint64_t>(n, 1), nb = (size_t)n_graphs + 1;
  leiden_status st;
  if ((st = FS->gid0.reserve(nn * 4)) || (st = FS->gidA.reserve(nn * 4)) || (st = FS->gidB.reserve(nn * 4)) ||
      (st = FS->base0.reserve(nb * 4)) || (st = FS->baseA.reserve(nb * 4)) || (st = FS->baseB.reserve(nb * 4)) ||
      (st = FS->m2.reserve(nb * 8)) || (st = FS->inv.reserve(nb * 16)) || (st = FS->dq.reserve(nb * 8)) ||
      (st = FS->move.reserve(nb)) || (st = FS->pass.reserve(nb)) || (st = FS->refined.reserve(nb)) ||
      (st = FS->cur_iters.reserve(nb * 4)) || (st = FS->passes.reserve(nb * 4)) ||
      (st = FS->iters_hist.reserve(nb * 4 * kForestIterHist)) || (st = FS->parts.reserve(nb * 32)) ||
      (st = FS->out_local.reserve(nn * 4)) || (st = FS->live_len.reserve(nn * 4)))
    return bail(st);
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  if (hipMemcpyAsync(FS->base0.p, first.data(), nb * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return bail(fail(LEIDEN_EDEVICE, "copy"));
  forest_gid(s, (uint32_t)n, n_graphs, FS->base0.as<uint32_t>(), FS->gid0.as<uint32_t>());
  unsigned int* fl = (unsigned int*)(G->small.as<uint64_t>() + 300);
  fill_u32(s, fl, 0, 1);
  forest_check_rows(s, rows0(G), (uint32_t)n, FS->gid0.as<uint32_t>(), FS->base0.as<uint32_t>(), fl);
  unsigned int f = 0;
  if (hipMemcpyAsync(&f, fl, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(LEIDEN_EDEVICE, "forest check failed"));
  if (f) return bail(fail(LEIDEN_EINVAL, "an entry joins vertices of two graphs of the forest"));
  *out = G;
  return LEIDEN_OK;
}

leiden_status leiden_forest_results(leiden_graph* G, double* q, uint32_t* passes, uint32_t* iters) {
  g_err.clear();
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  ForestState* FS = G->forest;
  if (!FS) return fail(LEIDEN_EINVAL, "not a forest");
  const uint32_t nq = FS->nq;
  if (q) {
    if (FS->q.size() != nq) return fail(LEIDEN_ESTATE, "no forest call yet");
    std::memcpy(q, FS->q.data(), 8 * (size_t)nq);
  }
  if (passes || iters) {
    if (FS->passes_h.size() != nq) return fail(LEIDEN_ESTATE, "no forest run yet");
    if (passes) std::memcpy(passes, FS->passes_h.data(), 4 * (size_t)nq);
    // graph-major: iters[q * kForestIterHist + pass]
    if (iters)
      for (uint32_t g = 0; g < nq; ++g)
        for (uint32_t p = 0; p < kForestIterHist; ++p)
          iters[(size_t)g * kForestIterHist + p] = FS->iters_h[(size_t)p * nq + g];
  }
  return LEIDEN_OK;
}

leiden_status leiden_forest_info(leiden_graph* G, uint32_t* n_graphs, uint32_t* first_vertex) {
  g_err.clear();
  if (!G || !n_graphs) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  if (!G->forest) {
    *n_graphs = 0;
    return LEIDEN_OK;
  }
  *n_graphs = G->forest->nq;
  if (first_vertex) std::memcpy(first_vertex, G->forest->first.data(), 4 * ((size_t)G->forest->nq + 1));
  return LEIDEN_OK;
}

leiden_status leiden_set_memory_budget(leiden_graph* G, uint64_t budget_bytes) {
  g_err.clear();
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  G->mem.budget = budget_bytes;
  return LEIDEN_OK;
}

leiden_status leiden_memory_used(leiden_graph* G, uint64_t* used_bytes) {
  g_err.clear();
  if (!G || !used_bytes) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  *used_bytes = G->mem.used;
  return LEIDEN_OK;
}

leiden_status leiden_graph_nnz(leiden_graph* g, uint64_t* nnz) {
  if (!g || !nnz) return fail(LEIDEN_EINVAL, "null argument");
  *nnz = g->nnz;
  return LEIDEN_OK;
}

leiden_status leiden_static(leiden_graph* G, const leiden_opts* opts, uint32_t* membership_out, int out_on_device,
                            double* q_out, leiden_stats* stats) {
  g_err.clear();
  InFlight in_flight;
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  leiden_opts o;
  leiden_default_opts(&o);
  if (opts) o = *opts;
  CHK(check_opts(o));
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = stream_of(G, opts);
  AllocScope alloc_scope(s, &G->mem);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  KtScope kts(G, o.timed_kernel);
  CHK(ensure_workspace(G, s, std::max(o.move_classes, o.refine_rounds)));
  ScatterScope scs(G);
  hipEvent_t e0, e1, e2;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventCreate(&e2));
  HIPCHK(hipEventRecord(e0, s));
  const uint32_t n = G->n;
  zero_ctl(G, s);
  G->sweeps = 2 * (uint64_t)n;  // set-up of C', K, Sigma and the flags; dense output labels
  LevelState L = level_state(G);
  CHK(row_sums(G, s, L.K));
  HIPCHK(hipMemcpyAsync(L.S, L.K, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
  iota_u32(s, L.C, n);
  fill_u8(s, L.dR, 1, n);
  fill_u8(s, L.dS, 0, n);
  unsigned long long* m2d = G->small.as<unsigned long long>() + 128;
  sum_i64(s, L.K, n, m2d);
  unsigned long long M2 = 0;
  CHK(read_dev(s, &M2, m2d));
  ForestState* FS = G->forest;
  if (FS) CHK(forest_prepare(G, s, L.K));
  RunOpts ro{o, false, 0, nullptr, true};
  CHK(run_leiden(G, s, L, ro, M2, stats));
  // dense output labels by minimum vertex; new state (C, K, Sigma, DeltaSigma = 0)
  CHK(G->st_C.reserve((size_t)std::max<uint32_t>(n, 1) * 4));
  CHK(G->st_K.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  CHK(G->st_S.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  CHK(G->st_dS.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  uint32_t* out = G->st_C.as<uint32_t>();
  launch_static_relabel(s, G->Ctop.as<uint32_t>(), n, G->tr_minv.as<uint32_t>(), G->flag.as<uint32_t>(),
                        G->newid.as<uint64_t>(), out, G->scan_tmp.p, G->small.as<uint64_t>() + 64,
                        FS ? FS->gid0.as<uint32_t>() : nullptr, FS ? FS->base0.as<uint32_t>() : nullptr);
  CHK(G->st_head.reserve((size_t)std::max<uint32_t>(n, 1) * 4));
  static_heads(s, n, G->flag.as<uint32_t>(), out, G->st_head.as<uint32_t>());
  G->heads_valid = true;
  CHK(row_sums(G, s, G->st_K.as<int64_t>()));
  launch_sigma_from(s, out, G->st_K.as<int64_t>(), n, G->st_S.as<int64_t>());
  fill_i64(s, G->st_dS.as<int64_t>(), 0, n);
  G->has_state = true;
  HIPCHK(hipEventRecord(e1, s));
  double q = std::numeric_limits<double>::quiet_NaN();
  if (FS)
    CHK(forest_collect(G, s, true, out, G->st_K.as<int64_t>(), o.compute_modularity != 0));
  else if (o.compute_modularity)
    CHK(modularity_of(G, s, out, G->st_K.as<int64_t>(), &q));
  HIPCHK(hipEventRecord(e2, s));
  if (FS) {  // labels inside each graph
    forest_to_local(s, n, FS->gid0.as<uint32_t>(), FS->base0.as<uint32_t>(), out, FS->out_local.as<uint32_t>());
    out = FS->out_local.as<uint32_t>();
  }
  CHK(copy_out(s, membership_out, out, sizeof(uint32_t) * n, out_on_device));
  HIPCHK(hipStreamSynchronize(s));
  if (q_out) *q_out = q;
  if (stats) {
    CHK(read_ctl_final(G, s));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e2);
    stats->ms_total = ms;
    (void)hipEventElapsedTime(&ms, e1, e2);
    stats->ms_modularity = ms;
    kt_collect(G, o.timed_kernel, stats);
    fill_work(G, stats, 0);
    stats->affected = n;
    stats->moves = G->hctl->total_moves;
    stats->refine_moves = G->hctl->refine_moves;
    stats->edges_scanned = G->hctl->edges;
    stats->nnz = G->nnz;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  return LEIDEN_OK;
}

leiden_status leiden_update(leiden_graph* G, const uint32_t* del, uint64_t n_del, const uint32_t* ins,
                            uint64_t n_ins, int batch_on_device, const uint32_t* prev_membership, int prev_on_device,
                            leiden_mode mode, const leiden_opts* opts, uint32_t* membership_out, int out_on_device,
                            double* q_out, leiden_stats* stats) {
  g_err.clear();
  InFlight in_flight;
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  if (mode != LEIDEN_ND && mode != LEIDEN_DS && mode != LEIDEN_DF) return fail(LEIDEN_EINVAL, "unknown mode");
  if ((n_del && !del) || (n_ins && !ins)) return fail(LEIDEN_EINVAL, "null batch arrays");
  leiden_opts o;
  leiden_default_opts(&o);
  if (opts) o = *opts;
  CHK(check_opts(o));
  if (!G->has_state && !prev_membership)
    return fail(LEIDEN_ESTATE, "no previous memberships: run leiden_static or pass prev_membership");
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = stream_of(G, opts);
  AllocScope alloc_scope(s, &G->mem);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  KtScope kts(G, o.timed_kernel);
  const uint32_t n = G->n;
  CHK(ensure_workspace(G, s, std::max(o.move_classes, o.refine_rounds)));
  ScatterScope scs(G);
  CHK(G->st_C.reserve((size_t)std::max<uint32_t>(n, 1) * 4));
  CHK(G->st_K.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  CHK(G->st_S.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  CHK(G->st_dS.reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  // batch buffers
  const uint64_t nb = n_del + n_ins, ne = 2 * nb;
  const size_t nn = std::max<size_t>(n, 1), nE = std::max<uint64_t>(ne, 1);
  CHK(G->bt_in.reserve((2 * n_del + 3 * n_ins + 1) * 4));
  for (Buf* b : {&G->bt_src, &G->bt_dst, &G->bt_w, &G->bt_del, &G->bt_slot, &G->bt_ssrc, &G->bt_sdst, &G->bt_sw,
                 &G->bt_sdel, &G->bt_sid, &G->bt_slb, &G->bt_tdst, &G->bt_tw, &G->bt_tdel, &G->bt_touched,
                 &G->bt_segcnt, &G->bt_newlen})
    CHK(b->reserve(nE * 4));
  CHK(G->bt_dest.reserve(nE * 8));
  CHK(G->bt_sortl.reserve(2 * nE * 4));
  CHK(G->bt_segoff.reserve((nE + 1) * 8));
  CHK(G->bt_spre.reserve((nE + 1) * 8));
  // runs of old entries: one per segment entry and one per touched row
  CHK(G->bt_rlen.reserve(2 * nE * 4));
  CHK(G->bt_roff.reserve((2 * nE + 1) * 8));
  CHK(G->bt_rsrc.reserve(2 * nE * 8));
  CHK(G->bt_rdst.reserve(2 * nE * 8));
  if (!G->rowcnt_ready) {
    CHK(G->bt_rowcnt.reserve(nn * 4));
    CHK(G->bt_rowidx.reserve(nn * 4));
    fill_u32(s, G->bt_rowcnt.as<uint32_t>(), 0, nn);
    G->rowcnt_ready = true;
  }
  CHK(G->scan_tmp.reserve(scan_tmp_bytes(std::max<uint64_t>(nn, 2 * nE)) + 64));
  hipEvent_t e0, e1, e2, e3;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventCreate(&e2));
  HIPCHK(hipEventCreate(&e3));
  HIPCHK(hipEventRecord(e0, s));
  zero_ctl(G, s);
  // C^{t-1} and the auxiliary state into the run; tracking (two passes); Sigma^t
  G->sweeps = 4 * (uint64_t)n;
  // previous memberships: validate and compare with the handle's state
  uint32_t* Cprev = G->st_C.as<uint32_t>();
  bool restart = !G->has_state;
  uint32_t* pm = nullptr;  // the caller's C^{t-1}, taken into the state once the batch is in
  if (prev_membership) {
    pm = G->tr_label.as<uint32_t>();
    CHK(copy_in(s, pm, prev_membership, sizeof(uint32_t) * n, prev_on_device));
    unsigned int* fl = (unsigned int*)(G->small.as<uint64_t>() + 300);
    if (G->forest) {  // labels inside each graph -> forest labels
      fill_u32(s, fl, 0, 1);
      forest_to_forest(s, n, G->forest->gid0.as<uint32_t>(), G->forest->base0.as<uint32_t>(), pm, pm, fl);
      unsigned int f = 0;
      CHK(read_dev(s, &f, fl));
      if (f) return fail(LEIDEN_EINVAL, "prev_membership has a label not below its graph's vertex count");
    }
    label_check(s, pm, G->has_state ? Cprev : nullptr, n, fl);
    unsigned int f = 0;
    CHK(read_dev(s, &f, fl));
    if (f & 1) return fail(LEIDEN_EINVAL, "prev_membership has a label >= n");
    if (f & 2) restart = true;
  }
  // batch: copy, group, sort, validate (nothing changes before this passes)
  uint32_t* din = G->bt_in.as<uint32_t>();
  CHK(copy_in(s, din, del, sizeof(uint32_t) * 2 * n_del, batch_on_device));
  CHK(copy_in(s, din + 2 * n_del, ins, sizeof(uint32_t) * 3 * n_ins, batch_on_device));
  if (G->forest) {
    unsigned int* fl = (unsigned int*)(G->small.as<uint64_t>() + 300);
    fill_u32(s, fl, 0, 1);
    forest_check_batch(s, din, n_del, din + 2 * n_del, n_ins, n, G->forest->gid0.as<uint32_t>(), fl);
    unsigned int f = 0;
    CHK(read_dev(s, &f, fl));
    if (f) return fail(LEIDEN_EINVAL, "invalid batch: a pair joins vertices of two graphs of the forest");
  }
  BatchBufs bb{};
  bb.src = G->bt_src.as<uint32_t>();
  bb.dst = G->bt_dst.as<uint32_t>();
  bb.w = G->bt_w.as<uint32_t>();
  bb.is_del = G->bt_del.as<uint32_t>();
  bb.slot = G->bt_slot.as<uint32_t>();
  bb.row_cnt = G->bt_rowcnt.as<uint32_t>();
  bb.row_idx = G->bt_rowidx.as<uint32_t>();
  bb.touched = G->bt_touched.as<uint32_t>();
  bb.seg_cnt = G->bt_segcnt.as<uint32_t>();
  bb.seg_off = G->bt_segoff.as<uint64_t>();
  bb.new_len = G->bt_newlen.as<uint32_t>();
  bb.dest = G->bt_dest.as<uint64_t>();
  bb.n_entries = ne;
  bb.seg_src = G->bt_ssrc.as<uint32_t>();
  bb.seg_dst = G->bt_sdst.as<uint32_t>();
  bb.seg_w = G->bt_sw.as<uint32_t>();
  bb.seg_del = G->bt_sdel.as<uint32_t>();
  bb.seg_id = G->bt_sid.as<uint32_t>();
  bb.seg_pre = G->bt_spre.as<uint64_t>();
  bb.seg_lb = G->bt_slb.as<uint32_t>();
  bb.sort_mid = G->bt_sortl.as<uint32_t>();
  bb.sort_long = G->bt_sortl.as<uint32_t>() + nE;
  bb.run_len = G->bt_rlen.as<uint32_t>();
  bb.run_off = G->bt_roff.as<uint64_t>();
  bb.run_src = G->bt_rsrc.as<int64_t>();
  bb.run_dst = G->bt_rdst.as<int64_t>();
  bb.tmp_dst = G->bt_tdst.as<uint32_t>();
  bb.tmp_w = G->bt_tw.as<uint32_t>();
  bb.tmp_del = G->bt_tdel.as<uint32_t>();
  bb.scan_tmp = G->scan_tmp.p;
  bb.total = G->small.as<uint64_t>() + 64;
  uint64_t nt = 0;
  int rc = batch_prepare(s, n, din, n_del, din + 2 * n_del, n_ins, bb, dctl(G), &nt);
  if (rc < 0) return fail(LEIDEN_EDEVICE, "batch preparation failed");
  if (rc > 0) return fail(LEIDEN_EINVAL, "invalid batch: vertex ID out of range, self-loop or zero weight");
  rc = batch_validate(s, rows0(G), n, ne, nt, bb, dctl(G));
  if (rc < 0) return fail(LEIDEN_EDEVICE, "batch validation failed");
  if (rc & 2) return fail(LEIDEN_EINVAL, "invalid batch: a pair appears twice");
  if (rc & 8) return fail(LEIDEN_EINVAL, "invalid batch: deletion of an absent edge");
  if (rc & 4) return fail(LEIDEN_EINVAL, "invalid batch: insertion of a present edge");
  // merge into the slack CSR (rebuild with more room if the overflow area is short)
  {
    for (int attempt = 0; attempt < 3; ++attempt) {
      rc = batch_merge(s, G->g.start, G->g.alt, G->g.len, G->g.cap, G->g.cols, G->g.w, nt, bb,
                       G->b_top.as<unsigned long long>(), G->g.edge_cap, dctl(G));
      if (rc == 0) break;
      if (rc < 0) return fail(LEIDEN_EDEVICE, "batch merge failed");
      // short of overflow room
      unsigned long long need = 0, top = 0;
      HIPCHK(hipMemcpyAsync(&need, &dctl(G)->overflow_need, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&top, G->b_top.p, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (top + need > G->g.edge_cap) {
        uint32_t* reserve = G->rb_reserve.as<uint32_t>();
        HIPCHK(hipMemcpyAsync(reserve, G->g.len, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        reserve_touched(s, nt, bb.touched, bb.new_len, reserve);
        CHK(rebuild(G, s, reserve));
      }
      HIPCHK(hipMemsetAsync(&dctl(G)->overflow_need, 0, 8, s));
    }
    if (rc != 0) return fail(LEIDEN_ENOMEM, "could not make room for the batch");
  }
  StateDrop drop(G);  // the graph holds the batch from here on
  if (restart && pm) HIPCHK(hipMemcpyAsync(Cprev, pm, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  count_units(s, G->g.len, bb.touched, nt, G->edge_parts.as<unsigned long long>(), kWMerge);
  // level-0 degree bins after the batch
  CHK(level_bins(G, s, G->g.len, n, G->bins0, &G->maxdeg0));
  G->nnz = G->nnz - 2 * n_del + 2 * n_ins;
  CHK(ensure_workspace(G, s, std::max(o.move_classes, o.refine_rounds)));  // nnz-sized scratch
  HIPCHK(hipEventRecord(e1, s));
  // auxiliary state: restart or continue
  LevelState L = level_state(G);
  // the input level works on the handle's K and Sigma in place: K^t is kept
  // by the run (aggregated levels write the two other K buffers in turn) and
  // Sigma^t is recomputed under the tracked labels at the end; a failure from
  // here on drops the state (the batch is in the graph)
  L.K = G->st_K.as<int64_t>();
  L.S = G->st_S.as<int64_t>();
  if (restart) {
    CHK(row_sums(G, s, L.K));  // K^t directly
    launch_sigma_from(s, Cprev, L.K, n, L.S);   // Sigma^t by C^{t-1}
    fill_i64(s, G->st_dS.as<int64_t>(), 0, n);
    // DeltaSigma^t from zero
    int64_t* dSig = G->sig.as<int64_t>();
    fill_i64(s, dSig, 0, n);
    int64_t* Kdummy = G->S2.as<int64_t>();
    int64_t* Sdummy = (int64_t*)G->newid.p;
    fill_i64(s, Kdummy, 0, n);
    fill_i64(s, Sdummy, 0, n);
    launch_aux_update(s, bb, ne, Cprev, Kdummy, Sdummy, dSig);
  } else {
    HIPCHK(hipMemcpyAsync(G->sig.p, G->st_dS.p, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
    launch_aux_update(s, bb, ne, Cprev, L.K, L.S, G->sig.as<int64_t>());
  }
  int64_t* dSig = G->sig.as<int64_t>();
  fill_u8(s, L.dS, 0, n);
  fill_u8(s, L.dR, 0, n);
  launch_mark_communities(s, bb, ne, Cprev, L.S, dSig, o.tau_re_num, o.tau_re_den, L.dS, L.dR);
  unsigned long long* m2d = G->small.as<unsigned long long>() + 128;
  sum_i64(s, L.K, n, m2d);
  unsigned long long M2 = 0;
  CHK(read_dev(s, &M2, m2d));
  ForestState* FS = G->forest;
  if (FS) {
    CHK(forest_prepare(G, s, L.K));
    bb.f_gid = FS->gid0.as<uint32_t>();
    bb.f_inv = FS->inv.as<double>();
  }
  // vertex marking (first pass): the first unprocessed list goes to next_list
  RunOpts ro{o, true, (int)mode, nullptr, false};
  const uint32_t first_stamp = G->stamp + 1;
  Ctl* ctl = dctl(G);
  if (mode == LEIDEN_ND) {
    ro.init_all = true;
  } else if (mode == LEIDEN_DF) {
    launch_mark_df(s, bb, ne, Cprev, G->next_list.as<uint32_t>(), &ctl->next_count, G->unproc.as<uint32_t>(),
                   first_stamp);
  } else {
    uint8_t *dV = G->dV.as<uint8_t>(), *dE = G->dE.as<uint8_t>(), *dC = G->dC.as<uint8_t>();
    fill_u8(s, dV, 0, n);
    fill_u8(s, dE, 0, n);
    fill_u8(s, dC, 0, n);
    const QConst qc = make_qconst(M2 ? M2 : 1);
    if (M2) launch_mark_ds(s, bb, ne, nt, rows0(G), n, Cprev, L.K, L.S, qc.inv_m, qc.inv_2m2, dV, dE, dC);
    launch_flags_to_list(s, dV, n, G->next_list.as<uint32_t>(), &ctl->next_count, G->unproc.as<uint32_t>(),
                         first_stamp);
    ro.in_range = dV;
  }
  // the run starts from C^{t-1}
  HIPCHK(hipMemcpyAsync(L.C, Cprev, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  CHK(read_ctl(G, s));
  const uint64_t affected = mode == LEIDEN_ND ? n : G->hctl->next_count;
  unsigned long long refine_marked = 0;
  {
    // count communities marked for refinement (statistics)
    unsigned int* cnt = (unsigned int*)(G->small.as<uint64_t>() + 310);
    (void)cnt;
  }
  // K^t of the input graph survives the run in its own buffer (levels reuse K)
  int64_t* const Kt = L.K;  // K^t of the input graph (the handle's K)
  CHK(run_leiden(G, s, L, ro, M2, stats));
  // tracking (Alg. 12) and the new state
  TrackBufs tb{};
  tb.minv = G->tr_minv.as<uint32_t>();
  tb.hkeys = G->tr_hk.as<unsigned long long>();
  tb.hvals = G->tr_hv.as<long long>();
  tb.hmask = next_pow2(2 * (uint64_t)std::max<uint32_t>(n, 1)) - 1;
  tb.best_w = G->tr_bw.as<long long>();
  tb.best_vmin = G->tr_bv.as<uint32_t>();
  tb.cand_w = G->tr_cw.as<long long>();
  tb.cand_b = G->tr_cb.as<uint32_t>();
  CHK(G->st_head.reserve((size_t)std::max<uint32_t>(n, 1) * 4));
  tb.head = G->st_head.as<uint32_t>();
  tb.cb = G->tr_old.as<uint32_t>();
  if (restart || !G->heads_valid) track_heads_of(s, n, Cprev, tb.head);
  tb.flag = G->tr_flag.as<uint32_t>();
  tb.rank = G->tr_rank.as<uint64_t>();
  tb.free_rank = G->tr_frank.as<uint64_t>();
  tb.free_id = G->tr_fid.as<uint32_t>();
  tb.label = G->tr_label.as<uint32_t>();
  tb.matched = G->tr_matched.as<uint8_t>();
  tb.Kc = G->tr_kc.as<int64_t>();
  tb.wb = G->tr_wcom.as<int64_t>();
  tb.owners = G->tr_owners.as<uint32_t>();
  tb.owner_count = (unsigned int*)(G->small.as<uint64_t>() + 320);
  if (FS) {
    tb.f_gid = FS->gid0.as<uint32_t>();
    tb.f_base = FS->base0.as<uint32_t>();
  }
  if (G->tr_clean != G->tr_hk.p) {  // a fresh pair table starts empty; each call leaves it empty
    fill_u64(s, (uint64_t*)G->tr_hk.p, ~0ull, tb.hmask + 1);
    fill_u64(s, (uint64_t*)G->tr_hv.p, 0, tb.hmask + 1);
    G->tr_clean = G->tr_hk.p;
  }
  // after one pass without refinement every label is its community's minimum
  // vertex (Alg. 10 and the split's component labels)
  const bool labels_are_min = G->run_passes == 1 && !G->run_refined0;
  tb.scan_tmp = G->scan_tmp.p;
  tb.total = G->small.as<uint64_t>() + 64;
  uint32_t* out = G->flag.as<uint32_t>();  // free after the run
  track(s, n, G->Ctop.as<uint32_t>(), Cprev, Kt, out, G->st_S.as<int64_t>(), labels_are_min, tb);
  G->heads_valid = true;
  // new state: C^t, K^t, Sigma^t by C^t, DeltaSigma^t kept for continued labels
  dsig_out(s, n, tb.matched, dSig, G->st_dS.as<int64_t>());
  HIPCHK(hipMemcpyAsync(G->st_C.p, out, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  G->has_state = true;
  drop.keep();
  HIPCHK(hipEventRecord(e2, s));
  double q = std::numeric_limits<double>::quiet_NaN();
  if (FS)
    CHK(forest_collect(G, s, true, G->st_C.as<uint32_t>(), G->st_K.as<int64_t>(), o.compute_modularity != 0));
  else if (o.compute_modularity)
    CHK(modularity_of(G, s, G->st_C.as<uint32_t>(), G->st_K.as<int64_t>(), &q));
  HIPCHK(hipEventRecord(e3, s));
  const void* res = G->st_C.p;
  if (FS) {  // labels inside each graph
    forest_to_local(s, n, FS->gid0.as<uint32_t>(), FS->base0.as<uint32_t>(), G->st_C.as<uint32_t>(),
                    FS->out_local.as<uint32_t>());
    res = FS->out_local.p;
  }
  CHK(copy_out(s, membership_out, res, sizeof(uint32_t) * n, out_on_device));
  HIPCHK(hipStreamSynchronize(s));
  if (q_out) *q_out = q;
  if (stats) {
    CHK(read_ctl_final(G, s));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e3);
    stats->ms_total = ms;
    (void)hipEventElapsedTime(&ms, e0, e1);
    stats->ms_batch = ms;
    (void)hipEventElapsedTime(&ms, e2, e3);
    stats->ms_modularity = ms;
    kt_collect(G, o.timed_kernel, stats);
    fill_work(G, stats, ne);
    stats->affected = affected;
    stats->refine_marked = refine_marked;
    stats->moves = G->hctl->total_moves;
    stats->refine_moves = G->hctl->refine_moves;
    stats->edges_scanned = G->hctl->edges;
    stats->nnz = G->nnz;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  (void)hipEventDestroy(e3);
  return LEIDEN_OK;
}

leiden_status leiden_modularity(leiden_graph* G, const uint32_t* membership, int on_device, double* q_out) {
  g_err.clear();
  if (!G || !membership || !q_out) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  CHK(ensure_workspace(G, s, 8));
  const uint32_t n = G->n;
  uint32_t* C = G->C.as<uint32_t>();
  CHK(copy_in(s, C, membership, sizeof(uint32_t) * n, on_device));
  unsigned int* fl = (unsigned int*)(G->small.as<uint64_t>() + 300);
  label_check(s, C, nullptr, n, fl);
  unsigned int f = 0;
  CHK(read_dev(s, &f, fl));
  if (f & 1) return fail(LEIDEN_EINVAL, "membership has a label >= n");
  int64_t* K = G->K.as<int64_t>();
  CHK(row_sums(G, s, K));
  if (ForestState* FS = G->forest) {
    // labels inside each graph; the per-graph values go to leiden_forest_results
    CHK(copy_in(s, C, membership, sizeof(uint32_t) * n, on_device));
    fill_u32(s, fl, 0, 1);
    forest_to_forest(s, n, FS->gid0.as<uint32_t>(), FS->base0.as<uint32_t>(), C, C, fl);
    CHK(read_dev(s, &f, fl));
    if (f) return fail(LEIDEN_EINVAL, "membership has a label not below its graph's vertex count");
    CHK(forest_collect(G, s, false, C, K, true));
    *q_out = std::numeric_limits<double>::quiet_NaN();
    return LEIDEN_OK;
  }
  return modularity_of(G, s, C, K, q_out);
}

leiden_status leiden_modularity_noalloc(leiden_graph* G, const uint32_t* membership, void* stream, double* q_out) {
  g_err.clear();
  if (!G || !membership || !q_out) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  if (G->forest) return fail(LEIDEN_EINVAL, "forests report modularity per graph (leiden_modularity)");
  if (G->n > kNoAllocMaxN)
    return fail(LEIDEN_EINVAL, "n = %u exceeds the %u vertices of the scratch array", G->n, kNoAllocMaxN);
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = stream ? (hipStream_t)stream : G->own;
  AllocScope alloc_scope(s, &G->mem);
  const int rc = noalloc_modularity(s, G->device, rows0(G), G->n, membership, q_out);
  if (rc == 2) return fail(LEIDEN_EINVAL, "membership has a label >= n");
  if (rc != 0) return fail(LEIDEN_EDEVICE, "modularity without allocation failed");
  return LEIDEN_OK;
}

leiden_status leiden_graph_export(leiden_graph* G, int64_t* offsets_out, uint32_t* cols_out, uint32_t* w_out) {
  g_err.clear();
  if (!G || !offsets_out) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  const uint32_t n = G->n;
  std::vector<int64_t> start(n);
  std::vector<uint32_t> len(n);
  unsigned long long top = 0;
  HIPCHK(hipMemcpyAsync(start.data(), G->g.start, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(len.data(), G->g.len, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&top, G->b_top.p, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint32_t> cols(top), w(top);
  HIPCHK(hipMemcpyAsync(cols.data(), G->g.cols, sizeof(uint32_t) * top, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(w.data(), G->g.w, sizeof(uint32_t) * top, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t e = 0;
  offsets_out[0] = 0;
  for (uint32_t i = 0; i < n; ++i) {
    for (uint32_t k = 0; k < len[i]; ++k, ++e) {
      if (cols_out) cols_out[e] = cols[start[i] + k];
      if (w_out) w_out[e] = w[start[i] + k];
    }
    offsets_out[i + 1] = e;
  }
  return LEIDEN_OK;
}

leiden_status leiden_state_export(leiden_graph* G, uint32_t* C, int64_t* K, int64_t* Sigma, int64_t* dSigma) {
  g_err.clear();
  if (!G) return fail(LEIDEN_EINVAL, "null handle");
  BUSY_GUARD(G);
  if (G->forest) return fail(LEIDEN_EINVAL, "state export is for single graphs");
  if (!G->has_state) return fail(LEIDEN_ESTATE, "no state yet");
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  const uint32_t n = G->n;
  CHK(copy_out(s, C, G->st_C.p, sizeof(uint32_t) * n, 0));
  CHK(copy_out(s, K, G->st_K.p, sizeof(int64_t) * n, 0));
  CHK(copy_out(s, Sigma, G->st_S.p, sizeof(int64_t) * n, 0));
  CHK(copy_out(s, dSigma, G->st_dS.p, sizeof(int64_t) * n, 0));
  HIPCHK(hipStreamSynchronize(s));
  return LEIDEN_OK;
}

leiden_status leiden_state_import(leiden_graph* G, const uint32_t* C, const int64_t* K, const int64_t* Sigma,
                                  const int64_t* dSigma) {
  g_err.clear();
  if (!G || !C || !K || !Sigma || !dSigma) return fail(LEIDEN_EINVAL, "null argument");
  BUSY_GUARD(G);
  if (G->forest) return fail(LEIDEN_EINVAL, "state import is for single graphs");
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->own;
  AllocScope alloc_scope(s, &G->mem);
  const uint32_t n = G->n;
  CHK(ensure_workspace(G, s, 8));
  for (Buf* b : {&G->st_C}) CHK(b->reserve((size_t)std::max<uint32_t>(n, 1) * 4));
  for (Buf* b : {&G->st_K, &G->st_S, &G->st_dS}) CHK(b->reserve((size_t)std::max<uint32_t>(n, 1) * 8));
  // check on the host: labels < n, K = row sums, Sigma = sums of K by label
  std::vector<int64_t> Kref(n);
  int64_t* Kd = G->K.as<int64_t>();
  CHK(row_sums(G, s, Kd));
  HIPCHK(hipMemcpyAsync(Kref.data(), Kd, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> Sref(n, 0);
  for (uint32_t i = 0; i < n; ++i) {
    if (C[i] >= n) return fail(LEIDEN_EINVAL, "label >= n");
    if (K[i] != Kref[i]) return fail(LEIDEN_EINVAL, "K differs from the row sums of the graph");
    Sref[C[i]] += K[i];
  }
  for (uint32_t c = 0; c < n; ++c)
    if (Sref[c] != Sigma[c]) return fail(LEIDEN_EINVAL, "Sigma differs from the sums of K by community");
  CHK(copy_in(s, G->st_C.p, C, sizeof(uint32_t) * n, 0));
  CHK(copy_in(s, G->st_K.p, K, sizeof(int64_t) * n, 0));
  CHK(copy_in(s, G->st_S.p, Sigma, sizeof(int64_t) * n, 0));
  CHK(copy_in(s, G->st_dS.p, dSigma, sizeof(int64_t) * n, 0));
  HIPCHK(hipStreamSynchronize(s));
  G->has_state = true;
  G->heads_valid = false;
  return LEIDEN_OK;
}

}  // extern "C"
