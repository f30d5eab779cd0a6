// Kernel parameter blocks and host launchers of the gfx950 Leiden library.
#pragma once

#include "common.h"
#include "leiden.h"

namespace lm {

template <typename W>
struct DecideParams {
  Rows<W> g;
  const uint32_t* C;     // current community of each vertex
  const int64_t* K;      // weighted degree
  const int64_t* S;      // total weight of each community
  const uint32_t* size;  // members of each community label
  const uint32_t* CB;    // community bound (refinement)
  uint32_t colour;       // refinement round
  uint32_t R;            // refinement rounds
  double inv_m, inv_2m2; // 1/m and 1/(2 m^2)
  const uint32_t* list;  // vertices of this bin
  const unsigned int* count;
  Mover* movers;
  Ctl* ctl;
  unsigned long long* edge_parts;  // edge scans, kEdgeParts counters kEdgeStride apart
  int async;             // 1: moves are applied at once against the live state
  int narrow;            // 1: 2m < 2^32, so every K_{i->c} fits 32 bits (narrower LDS tables)
  uint8_t* dS;           // split flags for asynchronous local moves (dynamic runs) or null
  // hub bin: a hub of degree L has nch = ceil(L / kHubChunk) chunks; chunk k
  // owns staging slots [k * kHubChunk, (k + 1) * kHubChunk) of the hub's
  // region, holding its distinct communities sorted by bucket (2^rbits
  // buckets of about kHubBucket communities each), and column k of the hub's
  // (R + 1) x nch matrix of bucket starts within the chunk (row R: the
  // chunk's total).
  const uint32_t* hub_idx;   // vertex -> hub index (hubs only)
  const uint64_t* hub_off;   // hub index -> first staging slot
  const uint64_t* hub_moff;  // hub index -> first matrix entry
  const uint32_t* hub_rbits; // hub index -> log2 of its bucket count
  unsigned long long* hub_kid;  // hub index -> K_{i->d} accumulator (kept zero between uses)
  uint32_t* hub_keys;
  unsigned long long* hub_vals;
  uint16_t* hub_mat;
  unsigned int* hub_live;    // hub index -> 1 while the hub takes part in the sub-round (kept zero between uses)
  // pick in segments: per hub and segment the best candidate, and a
  // completion counter per hub (kept zero between uses)
  uint32_t pick_segs;
  double* hub_pdq;
  uint32_t* hub_pc;
  unsigned int* hub_done;
  unsigned long long* hub_items;  // (hub vertex, chunk) work items of the current sub-round
};

// Work counters of a call (the units of the method's data access), spread
// over kEdgeParts copies: each block adds to copy blockIdx.x % kEdgeParts,
// each copy on its own 256-byte line, folded into Ctl::units at the end of a
// call.  Thousands of blocks that finish together and all add to one address
// queue on it (atomics on one address are serialised device-wide): one
// shared counter cost the small-degree decide kernel about 90 of its 127 µs.
constexpr uint32_t kEdgeParts = 64, kEdgeStride = 32;
enum WorkUnit : uint32_t {
  kWScan0 = 0,      // local-moving row entries scanned on the input graph
  kWScanUp = 1,     // local-moving row entries scanned on aggregated graphs
  kWDecided = 2,    // local-moving decisions (vertices evaluated)
  kWRefScan = 3,    // refinement row entries scanned
  kWMarks = 4,      // row entries of movers (neighbours re-marked)
  kWSplit = 5,      // row entries of vertices in split communities
  kWAggIn = 6,      // row entries read by aggregation
  kWAggOut = 7,     // super-edges written by aggregation
  kWMerge = 8,      // entries of rows rewritten by a batch merge (new lengths)
  kWUnits = 9
};
__device__ inline void add_units(unsigned long long* parts, uint32_t unit, unsigned long long e) {
  if (e && parts) atomicAdd(&parts[(blockIdx.x % kEdgeParts) * kEdgeStride + unit], e);
}
// local-moving scans of a level with weight type W
template <typename W>
__device__ inline void add_edges(unsigned long long* parts, unsigned long long e) {
  add_units(parts, sizeof(W) == 4 ? kWScan0 : kWScanUp, e);
}

// Hub layout of one level: a hub (degree above the last LDS bin) of degree
// L gets nch = ceil(L / kHubChunk) chunks of staging slots and R =
// pow2(ceil(L / kHubBucket)) buckets (at most 2^kHubMaxRbits), with an
// (R + 1) x nch matrix of 16-bit bucket starts.
constexpr uint32_t kHubChunk = 2048, kHubSlots = 4096;
constexpr uint32_t kHubBucketBits = 10, kHubBucket = 1u << kHubBucketBits;
// At most 256 buckets per hub: every chunk writes R + 1 scattered 16-bit
// bucket starts (one column of the matrix), and the smaller counter array
// leaves room for a third block per CU; the pick's groups just get larger.
constexpr uint32_t kHubMaxRbits = 8;
struct HubLayout {
  uint32_t* list;       // hubs of the level
  uint32_t* idx;        // vertex -> hub index (valid for hubs)
  uint64_t* off;        // hub index -> staging offset (count + 1)
  uint64_t* moff;       // hub index -> matrix offset (count + 1)
  uint32_t* rbits;      // hub index -> log2 of the bucket count
  uint64_t* size_tmp;   // scratch (count)
  uint64_t* msize_tmp;  // scratch (count)
  unsigned long long* kid;
};
// fills list / idx / off / moff / rbits for the level; returns the hub count,
// the staging slots and the matrix entries needed
int hub_layout(hipStream_t s, const uint32_t* len, uint32_t nl, uint32_t hub_above, HubLayout& h, Ctl* ctl,
               void* scan_tmp, uint64_t* total_dev, uint32_t* count_out, uint64_t* slots_out,
               uint64_t* mat_out);

struct ApplyParams {
  const int64_t* start;
  const uint32_t* len;
  const uint32_t* cols;
  uint32_t* C;
  int64_t* S;
  const int64_t* K;
  uint32_t* size;
  uint8_t* dS;  // split flags (dynamic runs) or null
  const Mover* movers;
  Ctl* ctl;
  uint32_t li, P, k, stamp;
  uint32_t* pend_mark;
  uint32_t* unproc_mark;
  uint32_t* cls_lists;
  size_t cls_stride;
  uint32_t* next_list;
  unsigned long long* mark_items;  // (mover, chunk) marking work items of the sub-round
  int applied;         // 1: the decide kernels already moved the vertices (asynchronous mode)
  unsigned long long* parts;  // work counters (WorkUnit) or null
};

// move.hip
void launch_distribute(hipStream_t s, const uint32_t* in_list, const unsigned int* in_count, uint32_t n_upper,
                       uint32_t li, uint32_t P, uint32_t stamp, uint32_t* pend_mark, uint32_t* cls_lists,
                       size_t stride, Ctl* ctl);
// Segments of the hub pick (kernel grid y): one per bucket of the level's
// longest row, at most kHubPickMaxSegs.
constexpr uint32_t kHubPickMaxSegs = 16;
inline uint32_t hub_pick_segs(uint32_t maxdeg) {
  const uint32_t units = maxdeg / kHubBucket + 1;
  uint32_t s = 1;
  while (s < units && s < kHubPickMaxSegs) s <<= 1;
  return s;
}

// hub_items (may be NULL): hubs also queue their row chunks for the hub kernels
void launch_bin(hipStream_t s, const uint32_t* list, const unsigned int* count, uint32_t n_upper, const uint32_t* len,
                const uint8_t* in_range, uint32_t* bin_lists, size_t stride, const BinCfg& cfg,
                unsigned long long* hub_items, Ctl* ctl);
// Side streams of a sub-round's decide kernels: the degree bins read the same
// state and only append movers, so their kernels can run side by side
// (forked from and joined back into the call's stream by events).  Only used
// while no other call of the process is running: the streams then outnumber
// the hardware queues, and event waits that several threads submit into
// shared in-order queues can wait on each other in a cycle.
constexpr int kDecideSide = 2;
struct DecideStreams {
  hipStream_t aux[kDecideSide];
  hipEvent_t fork, join[kDecideSide];
};
// maxdeg: largest degree of the level (sizes the hub kernels); ds may be null
// (everything on s)
template <typename W, bool REFINE>
void launch_decide_all(hipStream_t s, DecideParams<W> p, uint32_t* bin_lists, size_t stride, unsigned int* bin_counts,
                       const uint64_t* bin_upper, uint32_t maxdeg, const DecideStreams* ds);
// long_rows: the level has rows longer than the wavefront path handles
// items_upper: upper bound of the marking work items (entries / 64 + vertices)
void launch_apply_moves(hipStream_t s, const ApplyParams& p, uint32_t n_upper, uint64_t items_upper);
void launch_apply_refine(hipStream_t s, uint32_t* C, int64_t* S, const int64_t* K, uint32_t* size,
                         const Mover* movers, Ctl* ctl, uint32_t n_upper);
void launch_subround_reset(hipStream_t s, Ctl* ctl);
void launch_iteration_reset(hipStream_t s, Ctl* ctl, uint32_t P);
void launch_cls_reset(hipStream_t s, Ctl* ctl);

// prims.hip
void fill_u32(hipStream_t s, uint32_t* p, uint32_t v, size_t n);
// work counter `unit` (WorkUnit) += sum of len[i] (idx null) or len[idx[i]], i < n
void count_units(hipStream_t s, const uint32_t* len, const uint32_t* idx, uint64_t n, unsigned long long* parts,
                 uint32_t unit);
void fill_u8(hipStream_t s, uint8_t* p, uint8_t v, size_t n);
void fill_i64(hipStream_t s, int64_t* p, int64_t v, size_t n);
void iota_u32(hipStream_t s, uint32_t* p, size_t n);
// exclusive scan of n values (u32 in, u64 out); writes the total to *total (device) if non-null
void exclusive_scan_u32(hipStream_t s, const uint32_t* in, uint64_t* out, size_t n, uint64_t* total, void* tmp);
// Pinned host memory of at least `bytes` owned by the calling thread (NULL on
// failure); valid until its next call on this thread.
void* pinned_stage(size_t bytes);
size_t scan_tmp_bytes(size_t n);
void exclusive_scan_u64(hipStream_t s, const uint64_t* in, uint64_t* out, size_t n, uint64_t* total, void* tmp);

// scatter.hip: block-privatised scatter reductions over i < n
// Scatter reductions over keys below key_range (the output length).  With a
// workspace of scatter_ws_bytes(n, key_range) set in tl_scatter_ws, large
// inputs take the bucketed path (no global atomics).
struct ScatterWs {
  void* p;
  size_t bytes;
};
extern thread_local const ScatterWs* tl_scatter_ws;
size_t scatter_ws_bytes(uint64_t n, uint64_t key_range);
void scatter_add_i64(hipStream_t s, const uint32_t* key, const int64_t* val, uint64_t n, int64_t* out,
                     uint64_t key_range);
void scatter_add_u32_to_u64(hipStream_t s, const uint32_t* key, const uint32_t* val, uint64_t n, uint64_t* out,
                            uint64_t key_range);
void scatter_count(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out, uint64_t key_range);
void scatter_min_index(hipStream_t s, const uint32_t* key, uint64_t n, uint32_t* out, uint64_t key_range);

// phases.hip
void fill_u64(hipStream_t s, uint64_t* p, uint64_t v, size_t n);
// bins_out / maxdeg_out are added to; parts: 64 x 16 u64 of scratch
void launch_degree_hist(hipStream_t s, const uint32_t* len, uint32_t n, const BinCfg& cfg, unsigned long long* bins_out,
                        unsigned int* maxdeg_out, unsigned long long* parts);
// Rows of more than kWaveRowMax entries are summed in chunks of kRowChunk
// entries by whole blocks (kLongGrid of them); items holds the chunk list:
// long_items_bytes(nnz) bytes for a graph of nnz entries.
constexpr uint32_t kWaveRowMax = 1024, kRowChunk = 4096;
constexpr int kLongGrid = 1024;
inline size_t long_items_bytes(uint64_t nnz) { return (size_t)(nnz / kRowChunk + nnz / kWaveRowMax + 2) * 8; }
void launch_row_sums_u32(hipStream_t s, Rows<uint32_t> g, uint32_t n, int64_t* K, unsigned long long* items);
void launch_count_members(hipStream_t s, const uint32_t* C, uint32_t n, uint32_t* size);
void launch_sigma_from(hipStream_t s, const uint32_t* C, const int64_t* K, uint32_t n, int64_t* S);

struct RenumberBufs {
  uint32_t* rep;
  int64_t* S2;
  uint32_t* size2;
  uint8_t* dS2;
  uint8_t* dR2;
};
void subset_renumber(hipStream_t s, uint32_t n, uint32_t* C, int64_t*& S, uint32_t*& size, uint8_t*& dS,
                     uint8_t*& dR, RenumberBufs& b, Ctl* ctl);

// lab: one 64-bit union-find word per vertex (community << 32 | parent)
void launch_split_init(hipStream_t s, uint32_t n, const uint32_t* C, const uint8_t* dS, const uint8_t* dR,
                       unsigned long long* lab, uint32_t* list, uint32_t* wide, unsigned long long* main_key,
                       Ctl* ctl, const uint32_t* len, unsigned long long* parts);
template <typename W>
void launch_split_sample(hipStream_t s, Rows<W> g, const uint32_t* C, unsigned long long* lab, const uint32_t* list,
                         const uint32_t* wide, unsigned long long* main_key, uint32_t* rest, Ctl* ctl,
                         uint32_t n_upper);
template <typename W>
void launch_split_union(hipStream_t s, Rows<W> g, const uint32_t* C, unsigned long long* lab,
                        const uint32_t* bin_lists, size_t stride, const unsigned int* bin_counts,
                        const uint64_t* bin_upper);
void launch_split_finish(hipStream_t s, uint32_t* C, unsigned long long* lab, const uint32_t* list, Ctl* ctl,
                         uint32_t n_upper);

void launch_refine_reset(hipStream_t s, uint32_t n, uint32_t* C, uint32_t* CB, int64_t* S, const int64_t* K,
                         uint32_t* size, const uint8_t* dR, uint32_t R, uint32_t* col_lists, size_t stride,
                         Ctl* ctl);

// dense renumber: flag (u32[n]) scratch, newid (u64[n]) scratch; returns count on device in *total
void dense_renumber(hipStream_t s, uint32_t n, uint32_t* C, uint32_t* flag, uint64_t* newid, uint64_t* total,
                    void* scan_tmp);
void launch_lookup(hipStream_t s, uint32_t* Ctop, const uint32_t* C, uint32_t n);

struct AggBufs {
  uint32_t* comm_count;   // members per community
  uint64_t* comm_off;     // member offsets (n + 1)
  uint32_t* comm_fill;
  uint32_t* comm_fill_long; // members with long rows per community (placed at the back of its range)
  uint64_t* member_eoff;    // entry offsets of the members in member order (n + 1)
  uint32_t* members;
  uint64_t* comm_deg;     // total degree per community
  uint64_t* cap_off;      // super-row capacity offsets (n + 1)
  uint64_t* total;        // device scalars
  void* scan_tmp;
  uint32_t* small_lists;  // communities per class (small, large medium, big, medium), n each
  uint64_t* big_info;     // (member begin, member end, capacity, entries) of each big community, 4 n
  void* bigc;             // per-round descriptors of big communities (32 B each, n)
  void* items;            // per-round work items (24 B each, item_cap)
  uint64_t item_cap;
  unsigned long long* stage_ctr; // per-round stage columns and staging slots used (n)
  unsigned long long* self_acc;  // per-round own-key sums (n)
  uint32_t* skeys;               // staging slots (scap)
  unsigned long long* svals;
  uint16_t* smat;                // bucket-start matrices (mcap entries)
  size_t scap, mcap;
  uint32_t emit_cap;             // slots of the emit kernel's LDS table (power of two, 16..4096)
  unsigned int* slice_ctl;       // 9 words: offsets of the stage-item lists
};
// sorted_rows: every row of g is sorted by column (then large communities are
// staged by XCD slices of the column range)
template <typename W>
int aggregate(hipStream_t s, Rows<W> g, uint32_t n, const uint32_t* C, uint32_t nc, AggBufs& b, int64_t* out_start,
              uint32_t* out_len, uint32_t* out_cols, int64_t* out_w, int64_t* Kout, Ctl* ctl, bool sorted_rows);

void launch_static_relabel(hipStream_t s, const uint32_t* C, uint32_t n, uint32_t* minv, uint32_t* flag,
                           uint64_t* rank, uint32_t* out, void* scan_tmp, uint64_t* total, const uint32_t* fgid = nullptr,
                           const uint32_t* fbase = nullptr);

struct ModParts {
  unsigned long long sigma;
  unsigned long long T_hi, T_lo;
};
// partials: 4 * nblocks words; items: the long-row chunk list (as for the row sums)
void modularity_parts(hipStream_t s, Rows<uint32_t> g, uint32_t n, const uint32_t* C, const int64_t* K, int64_t* Sig,
                      unsigned long long* partials, int nblocks, ModParts* out_dev, unsigned long long* items);

struct TrackBufs {
  uint32_t* head;             // in: minimum vertex of every old label (kNone: not a label); out: those of the new labels
  uint32_t* cb;               // per old label: the current community of its head
  uint32_t* minv;
  unsigned long long* hkeys;  // pair table (empty between calls)
  long long* hvals;
  uint64_t hmask;
  int64_t* Kc;                // per vertex: its weight if its pair is (its old label, cb of it)
  int64_t* wb;                // per old label: weight of its common pair
  uint32_t* owners;           // slots of the rare pairs
  unsigned int* owner_count;
  long long* best_w;
  uint32_t* best_vmin;
  long long* cand_w;
  uint32_t* cand_b;
  uint32_t* flag;
  uint64_t* rank;
  uint64_t* free_rank;
  uint32_t* free_id;
  uint32_t* label;
  uint8_t* matched;
  void* scan_tmp;
  uint64_t* total;
  // a forest's graph of each vertex and first vertex of each graph (null for
  // one graph): every graph draws fresh labels from its own ID range
  const uint32_t* f_gid;
  const uint32_t* f_base;
};
// out: tracked labels; S_out: Sigma^t by tracked label.  labels_are_min:
// every label of Ccur is its community's minimum vertex (saves a scatter).
void track(hipStream_t s, uint32_t n, const uint32_t* Ccur, const uint32_t* Cprev, const int64_t* K, uint32_t* out,
           int64_t* S_out, bool labels_are_min, TrackBufs& b);
// head[label] = minimum vertex of the community of each label of C
void track_heads_of(hipStream_t s, uint32_t n, const uint32_t* C, uint32_t* head);
// heads of dense static labels (flag: minimum vertices, out: their labels)
void static_heads(hipStream_t s, uint32_t n, const uint32_t* flag, const uint32_t* out, uint32_t* head);

// forest.hip: per-graph state of a forest run (see the file's header).
constexpr uint32_t kForestIterHist = 16;  // passes whose iteration counts are kept per graph
struct ForestBufs {
  uint32_t nq;
  unsigned long long* m2;    // per graph 2m
  double* inv;               // per graph 1/m, 1/(2 m^2)
  unsigned long long* dq;    // per graph gain sum of the current iteration (2^56 fixed point)
  uint8_t* move;             // per graph: still iterating local moving
  uint8_t* pass;             // per graph: still in the pass loop
  uint8_t* refined;          // per graph: refined a community in the current pass
  uint32_t* cur_iters;       // per graph iterations of the current pass
  uint32_t* passes;          // per graph passes of the run
  uint32_t* iters_hist;      // kForestIterHist x nq iteration counts
};
void forest_gid(hipStream_t s, uint32_t n, uint32_t nq, const uint32_t* base, uint32_t* gid);
void forest_next_base(hipStream_t s, uint32_t nq, uint32_t nl, const uint32_t* base, const uint64_t* newid,
                      const uint64_t* total, uint32_t* next);
void forest_check_rows(hipStream_t s, Rows<uint32_t> g, uint32_t n, const uint32_t* gid, const uint32_t* base,
                       unsigned int* flags);
void forest_check_batch(hipStream_t s, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                        uint32_t n, const uint32_t* gid, unsigned int* flags);
void forest_to_forest(hipStream_t s, uint32_t n, const uint32_t* gid, const uint32_t* base, const uint32_t* local,
                      uint32_t* out, unsigned int* flags);
void forest_to_local(hipStream_t s, uint32_t n, const uint32_t* gid, const uint32_t* base, const uint32_t* in,
                     uint32_t* out);
void forest_sum(hipStream_t s, uint32_t n, const uint32_t* gid, const int64_t* x, unsigned long long* out);
void forest_modularity_parts(hipStream_t s, Rows<uint32_t> g, uint32_t n, uint32_t nq, const uint32_t* C,
                             const int64_t* K, const uint32_t* gid, int64_t* Sig, unsigned long long* parts);
void forest_start(hipStream_t s, const ForestBufs& f, Ctl* ctl);
void forest_iter_end(hipStream_t s, const ForestBufs& f, double tau, uint32_t li, uint32_t max_iters, Ctl* ctl);
void forest_pass_end(hipStream_t s, const ForestBufs& f, uint32_t pass, Ctl* ctl);
void forest_bind(hipStream_t s, Ctl* ctl, const ForestBufs& f, const uint32_t* gid, const uint32_t* base);
void forest_isolate(hipStream_t s, uint32_t n, const uint32_t* gid, const uint8_t* pass, uint32_t* C);
void forest_live_len(hipStream_t s, uint32_t n, const uint32_t* gid, const uint8_t* pass, const uint32_t* len,
                     uint32_t* out);

// Per-launch timing of one kernel with HIP events on the launch stream.  The
// runtime points tl_ktimer at the handle's timer for the duration of a call
// that asks for it; launch sites bracket the kernel with kt_mark.
constexpr int kKtMaxLaunches = 1024;
struct KTimer {
  int which = 0;  // leiden_kernel being timed
  int n = 0;      // events recorded (two per launch)
  bool ready = false;
  hipEvent_t ev[2 * kKtMaxLaunches];
};
extern thread_local KTimer* tl_ktimer;
inline void kt_mark(int which, hipStream_t s) {
  KTimer* t = tl_ktimer;
  if (t && t->which == which && t->n < 2 * kKtMaxLaunches) (void)hipEventRecord(t->ev[t->n++], s);
}

// batch.hip
struct BatchBufs {
  // directed entries in arrival order (2 per undirected update)
  uint32_t* src;
  uint32_t* dst;
  uint32_t* w;
  uint32_t* is_del;
  uint32_t* slot;      // rank of the entry inside its row segment
  // per vertex
  uint32_t* row_cnt;   // entries per source row (kept zero between batches)
  uint32_t* row_idx;   // position of a touched row in `touched`
  // per touched row
  uint32_t* touched;
  uint32_t* seg_cnt;
  uint64_t* seg_off;   // nt + 1
  uint32_t* new_len;
  uint64_t* dest;      // span that receives the merged row in the slack CSR
  uint64_t n_entries;  // directed entries (2 per update)
  // entries grouped by row and sorted by destination
  uint32_t* seg_src;
  uint32_t* seg_dst;
  uint32_t* seg_w;     // deletions: weight in G^{t-1} after validation
  uint32_t* seg_del;
  uint32_t* seg_id;
  uint64_t* seg_pre;   // exclusive prefix of seg_del (ne + 1)
  uint32_t* seg_lb;    // position of the entry's destination in the old row (lower bound)
  uint32_t* sort_mid;  // touched rows whose segment the LDS sort takes
  uint32_t* sort_long; // touched rows whose segment the merge sort takes
  uint32_t* tmp_dst;   // merge-sort scratch for long segments
  uint32_t* tmp_w;
  uint32_t* tmp_del;
  // old entries move in runs with one shift each: run i of touched row t lies
  // between its segment entries; ne + nt runs
  uint32_t* run_len;
  uint64_t* run_off;   // exclusive prefix of run_len (ne + nt + 1)
  int64_t* run_src;    // first old entry of the run
  int64_t* run_dst;    // its place in the merged row
  void* scan_tmp;
  uint64_t* total;
  // a forest's graph of each vertex and per-graph Eq. 2 constants (null for one graph)
  const uint32_t* f_gid;
  const double* f_inv;
};
int batch_prepare(hipStream_t s, uint32_t n, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                  BatchBufs& b, Ctl* ctl, uint64_t* n_touched_host);
int batch_validate(hipStream_t s, Rows<uint32_t> g, uint32_t n, uint64_t n_entries, uint64_t n_touched, BatchBufs& b,
                   Ctl* ctl);
// applies the validated batch; returns 1 if the overflow area is exhausted (nothing written)
int batch_merge(hipStream_t s, int64_t* start, int64_t* alt, uint32_t* len, uint32_t* cap, uint32_t* cols,
                uint32_t* w, uint64_t n_touched, BatchBufs& b, unsigned long long* edge_top, uint64_t edge_cap,
                Ctl* ctl);
void launch_aux_update(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev, int64_t* K,
                       int64_t* S, int64_t* dSig);
void launch_mark_communities(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev,
                             const int64_t* S, int64_t* dSig, uint32_t num, uint32_t den, uint8_t* dS, uint8_t* dR);
void launch_mark_df(hipStream_t s, const BatchBufs& b, uint64_t n_entries, const uint32_t* Cprev, uint32_t* list,
                    unsigned int* count, uint32_t* mark, uint32_t stamp);
void launch_mark_ds(hipStream_t s, const BatchBufs& b, uint64_t n_entries, uint64_t n_touched, Rows<uint32_t> g,
                    uint32_t n, const uint32_t* Cprev, const int64_t* K, const int64_t* S, double inv_m,
                    double inv_2m2, uint8_t* dV, uint8_t* dE, uint8_t* dC);
void launch_flags_to_list(hipStream_t s, const uint8_t* flags, uint32_t n, uint32_t* list, unsigned int* count,
                          uint32_t* mark, uint32_t stamp);

}  // namespace lm
