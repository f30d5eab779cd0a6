/*
 * leiden.h - C-ABI of the MI355X (gfx950) Static / ND / DS / DF Leiden library.
 *
 * The calls follow the problem statement of "Heuristic-based Dynamic Leiden
 * Algorithm for Efficient Tracking of Communities on Evolving Graphs" (Sahu):
 * Static Leiden takes a graph G (Section 5.1.5); the dynamic ND, DS and DF
 * algorithms (Alg. 1, 2, 3) take the updated graph G^t, the batch update
 * (deletions Delta^{t-} and insertions Delta^{t+}, Section 3.5), the previous
 * memberships C^{t-1} and the auxiliary state K^{t-1}, Sigma^{t-1} and
 * DeltaSigma^{t-1}, and return C^t with the new auxiliary state.  Here the
 * graph handle owns G^t on the device together with that auxiliary state
 * (Section 4.4), and applies each batch to its own copy of the graph.
 *
 * Conventions
 *   - Vertex IDs are uint32 in [0, n); edge weights are uint32 > 0; the graph
 *     is undirected and stored with both directions of every edge.
 *   - Pointer arguments are host or device memory as the `*_on_device`
 *     argument of the call says (1 = device memory of the handle's GPU).
 *   - Every call is ordered on opts->stream (a hipStream_t; NULL means the
 *     handle's own stream) and returns after its outputs are complete.
 *   - The caller owns every buffer it passes; the library copies what it
 *     needs before returning.  The handle owns all device memory it allocates.
 *   - Every call returns a leiden_status; leiden_last_error() gives a message
 *     for the calling thread.  A failed call leaves the handle's graph and
 *     state as they were, except an update that fails after its batch is in
 *     the graph (see leiden_update).
 *   - One call at a time per handle: a call that finds the handle in use by
 *     another thread returns LEIDEN_EBUSY and does nothing.  Different
 *     handles are independent.
 */
#ifndef LEIDEN_MI355X_H
#define LEIDEN_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LEIDEN_OK = 0,
  LEIDEN_EINVAL = -1,  /* invalid argument or batch */
  LEIDEN_ENOMEM = -2,  /* device memory exhausted */
  LEIDEN_EDEVICE = -3, /* HIP runtime error */
  LEIDEN_ESTATE = -4,  /* handle has no state for the request (e.g. update before any run) */
  LEIDEN_EBUSY = -5    /* another call is using the handle (one call at a time per handle) */
} leiden_status;

typedef enum {
  LEIDEN_ND = 0, /* Naive-dynamic: every vertex affected (Alg. 1) */
  LEIDEN_DS = 1, /* Delta-screening (Alg. 2) */
  LEIDEN_DF = 2  /* Dynamic Frontier (Alg. 3) */
} leiden_mode;

/* Kernels that a call can time (leiden_opts.timed_kernel), with the unit of
 * work each one counts and the algorithmic bytes per unit: the data the
 * method has to touch, not what the kernel actually moves. */
typedef enum {
  LEIDEN_KT_NONE = 0,
  /* Local moving (Alg. 6) of the hub-degree bin on the input graph: one unit
   * per scanned row entry, 12 bytes (neighbour ID, edge weight and the
   * neighbour's community, 4 bytes each). */
  LEIDEN_KT_HUB_INSERT = 1,
  /* Aggregation (Alg. 9) of the large communities of the input graph: one
   * unit per member row entry read, 12 bytes (neighbour ID, edge weight and
   * the neighbour's community). */
  LEIDEN_KT_AGG_BIG = 2
} leiden_kernel;
/* (LEIDEN_KT_HUB_INSERT is the kernel that sums chunks of hub rows by
 * community in LDS and stages each chunk's distinct communities sorted by
 * hash bucket; LEIDEN_KT_AGG_BIG is the kernel that does the same for 2048-
 * entry stages of a large community's member rows.  leiden_kernel_name gives
 * their profiler names.) */

/* Parameters (defaults from Section 5.1.2). */
typedef struct {
  double tau;             /* initial iteration tolerance, 1e-2 */
  uint32_t tau_re_num;    /* refinement tolerance tau_re = num / den, 3 / 5 */
  uint32_t tau_re_den;
  uint32_t tol_decline;   /* TOLERANCE_DECLINE_FACTOR, 10 */
  uint32_t max_iters;     /* MAX_ITERATIONS per pass, 20 */
  uint32_t max_passes;    /* MAX_PASSES, 10 */
  uint32_t move_classes;  /* vertex classes of the synchronous local-moving sub-rounds, 4 (1..32) */
  uint32_t refine_rounds; /* colour rounds of the synchronous refinement, 8 (1..32) */
  int32_t deterministic;  /* 1: synchronous schedule, bit-exact and reproducible */
  int32_t compute_modularity; /* 1: fill *q_out with Eq. 1 of the result; 0: NaN */
  void* stream;           /* hipStream_t or NULL */
  int32_t timed_kernel;   /* a leiden_kernel to time with HIP events on the stream, or LEIDEN_KT_NONE */
  int32_t split_all;      /* 1: split every community not marked for refinement (the ablation of
                             Section 4.3), 0: only the communities marked to be split (default) */
} leiden_opts;

/* Work counters of a call (leiden_stats.work), in the units of the data the
 * method has to touch, with the bytes each unit stands for in
 * leiden_stats.algo_bytes. */
typedef enum {
  LEIDEN_W_SCAN0 = 0,       /* local-moving row entries scanned on the input graph: 12 B
                               (neighbour ID, weight, the neighbour's community) */
  LEIDEN_W_SCAN_UP = 1,     /* the same on aggregated graphs: 16 B (64-bit weights) */
  LEIDEN_W_DECIDED = 2,     /* local-moving decisions: 48 B (row offset, C, K, Sigma and size of the
                               own community, candidate Sigma/size, C write) */
  LEIDEN_W_REFINE_SCAN = 3, /* refinement row entries scanned: 16 B (+ the neighbour's bound) */
  LEIDEN_W_MARKS = 4,       /* row entries of moved vertices (neighbours re-marked, Alg. 6): 4 B */
  LEIDEN_W_SPLIT = 5,       /* row entries of vertices in communities being split (Alg. 7): 8 B */
  LEIDEN_W_AGG_IN = 6,      /* row entries read by aggregation (Alg. 9): 12 B */
  LEIDEN_W_AGG_OUT = 7,     /* super-edges written by aggregation: 12 B */
  LEIDEN_W_MERGE = 8,       /* entries of the rows a batch rewrites: 16 B (read and write, ID and weight) */
  LEIDEN_WORK_COUNT = 9
} leiden_work;

/* Per-call statistics. */
typedef struct {
  uint32_t passes;
  uint32_t iters[16];        /* local-moving iterations per pass */
  uint32_t subrounds[16];    /* non-empty class sub-rounds per pass */
  uint64_t affected;         /* vertices marked affected before the first pass */
  uint64_t split_marked;     /* communities split in the first pass */
  uint64_t refine_marked;    /* communities marked for refinement by the batch */
  uint64_t moves;            /* local-moving moves, all passes */
  uint64_t refine_moves;     /* refinement moves, all passes */
  uint64_t edges_scanned;    /* local-moving edge scans, all passes */
  int32_t refined_first_pass;
  int32_t pad_;
  double ms_total;           /* device time of the whole call */
  double ms_batch;           /* batch validation and graph update */
  double ms_modularity;      /* final modularity */
  uint64_t nnz;              /* directed entries of the graph after the call */
  /* the kernel named by leiden_opts.timed_kernel: each launch is bracketed by
   * two events recorded on the call's stream */
  uint32_t kt_launches;      /* launches of that kernel in the call */
  uint32_t kt_pad_;
  double kt_ms;              /* their summed device time */
  uint64_t kt_units;         /* work units they processed (see leiden_kernel) */
  double kt_bytes;           /* algorithmic bytes of those units */
  uint64_t work[LEIDEN_WORK_COUNT]; /* work counters, indexed by leiden_work */
  uint64_t sweep_vertices;   /* vertices of the passes over per-vertex arrays (Alg. 4 set-up and
                                look-ups, Alg. 10, Alg. 8 reset, Alg. 12): 16 B each */
  uint64_t batch_entries;    /* directed batch entries: 12 B each */
  /* algorithmic bytes of the call: every work counter, the moves (32 B each:
   * Sigma and size of two communities), the sweeps and the batch entries
   * times their bytes */
  double algo_bytes;
} leiden_stats;

typedef struct leiden_graph leiden_graph;

/* Degree-bin thresholds of a handle.  Local moving and refinement decide a
 * vertex of degree d in the first bin b with d <= bin_max_degree[b] (bins:
 * 8 lanes and 16 table slots per vertex, 32 / 64, 64 / 256, a block with 1024
 * slots, a block with 4096 slots); longer rows are hubs, split into chunks.
 * The thresholds must increase and stay within 15, 63, 255, 1023 and 4095 (a
 * bin's table must hold every distinct community of its rows).  They decide
 * only which kernel evaluates a vertex, never the result (memberships are
 * identical for every valid setting).  Defaults: the capacities 15, 63,
 * 255, 1023, 4095. */
typedef struct {
  uint32_t bin_max_degree[5];
  /* Slots of the LDS table in which the aggregation (Alg. 9) sums a group of
   * a large community's neighbouring communities: a power of two in
   * 16..4096, or 0 for 4096.  A group with more distinct neighbours than the
   * table is split in halves by hash bits until each part fits; smaller
   * tables only take that path more often and never change the result. */
  uint32_t agg_emit_slots;
  double probe_ms; /* time of the autotuning probe with these thresholds (0 if never tuned) */
  double agg_probe_ms; /* time of the aggregation probe with this emit table (0 if never tuned) */
} leiden_tuning;

leiden_status leiden_get_tuning(leiden_graph* g, leiden_tuning* out);
/* LEIDEN_EINVAL if the thresholds are not increasing or exceed the limits, or
 * agg_emit_slots is not 0 or a power of two in 16..4096. */
leiden_status leiden_set_tuning(leiden_graph* g, const leiden_tuning* t);
/* Choose the thresholds for this graph by measurement: coordinate descent
 * over each threshold at 1/2, 3/4, 3/2 and 2 times its value, timing one
 * decide-only local-moving iteration over every vertex from singleton
 * communities (on opts->stream); then the aggregation's emit table
 * (agg_emit_slots) among 4096, 2048, 1024 and 512 slots, timing one
 * aggregation of the graph under a probe membership (every vertex with its
 * smallest neighbour).  Keeps the fastest setting in the handle and returns
 * it in *out (may be NULL).  The handle's graph and state are unchanged. */
leiden_status leiden_autotune(leiden_graph* g, const leiden_opts* opts, leiden_tuning* out);

/* Symbol of a leiden_kernel as profilers list it (NULL for an unknown value).
 * For LEIDEN_KT_HUB_INSERT it is the prefix common to the kernel's two
 * instantiations (32-bit table sums when 2m < 2^32, else 64-bit). */
const char* leiden_kernel_name(int32_t kernel);

/* Fill *opts with the defaults above. */
leiden_status leiden_default_opts(leiden_opts* opts);

/* Create a handle on GPU `device` holding the undirected graph given as a CSR
 * with both directions of every edge: offsets int64[n+1], cols uint32[nnz],
 * w uint32[nnz] (the graph of Section 3 with integer weights).  Each row
 * must be sorted by column; unsorted rows, duplicate entries, self-loops,
 * zero weights, IDs >= n or an asymmetric matrix give LEIDEN_EINVAL.  `slack`
 * >= 0 reserves room per row for future insertions (fraction of the row
 * length); each row holds two spans of that capacity on the device (a batch
 * writes the updated row into the spare one), so the handle takes about
 * 2 (1 + slack) nnz entries of 8 bytes.  *out receives the handle. */
leiden_status leiden_graph_create(int device, uint32_t n, uint64_t nnz, const int64_t* offsets,
                                  const uint32_t* cols, const uint32_t* w, int on_device, double slack,
                                  leiden_graph** out);

void leiden_graph_destroy(leiden_graph* g);

/* Number of directed entries currently held. */
leiden_status leiden_graph_nnz(leiden_graph* g, uint64_t* nnz);

/* Device memory of a handle: the graph, its auxiliary state and the working
 * buffers that calls grow on demand (they are kept for later calls).
 * leiden_memory_used gives the bytes held now.  A budget above 0 bounds
 * them: a call that would grow the handle past it returns LEIDEN_ENOMEM
 * (with the batch rules of leiden_update below); 0, the default, means no
 * bound.  Lowering the budget frees nothing. */
leiden_status leiden_set_memory_budget(leiden_graph* g, uint64_t budget_bytes);
leiden_status leiden_memory_used(leiden_graph* g, uint64_t* used_bytes);

/* Static Leiden (Alg. 4 with every vertex affected and every community
 * marked for refinement).  membership_out: uint32[n], dense labels ordered
 * by each community's minimum vertex.  Sets the handle's state (C, K, Sigma,
 * DeltaSigma = 0) for later updates.  q_out, stats may be NULL. */
leiden_status leiden_static(leiden_graph* g, const leiden_opts* opts, uint32_t* membership_out, int out_on_device,
                            double* q_out, leiden_stats* stats);

/* Dynamic Leiden (Alg. 1 / 2 / 3 followed by Alg. 4 and Alg. 12).
 * del: n_del undirected pairs (u, v) as uint32[2 * n_del], each pair once,
 * each an existing edge; ins: n_ins undirected (u, v, w) as uint32[3 * n_ins],
 * each an absent pair, w > 0.  A self-loop, an ID >= n, a repeated pair, a
 * deletion of an absent edge or an insertion of a present one gives
 * LEIDEN_EINVAL and changes nothing.  A failure after the batch is in the
 * graph (device memory, the memory budget, a HIP error) keeps the updated
 * graph and drops the auxiliary state: the next update then returns
 * LEIDEN_ESTATE unless it passes prev_membership, and leiden_static or
 * leiden_state_import restore the state.  prev_membership: uint32[n] C^{t-1} with
 * labels < n, or NULL for the handle's last result; a membership that differs
 * from the last result restarts Sigma from K and DeltaSigma from zero.
 * membership_out: uint32[n] C^t with tracked labels. */
leiden_status leiden_update(leiden_graph* g, const uint32_t* del, uint64_t n_del, const uint32_t* ins,
                            uint64_t n_ins, int batch_on_device, const uint32_t* prev_membership,
                            int prev_on_device, leiden_mode mode, const leiden_opts* opts,
                            uint32_t* membership_out, int out_on_device, double* q_out, leiden_stats* stats);

/* Modularity (Eq. 1) of membership (uint32[n], labels < n) on the handle's
 * current graph. */
leiden_status leiden_modularity(leiden_graph* g, const uint32_t* membership, int on_device, double* q_out);

/* leiden_modularity for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same value, computed without any allocation.  membership: device
 * uint32[n] (labels < n, else LEIDEN_EINVAL); stream: hipStream_t or NULL
 * for the handle's own; *q_out: host double.  The scratch memory is a fixed
 * device array of the library (about 32 MiB per GPU, held until the process
 * ends) shared by every call on that GPU, so n must not exceed 4,194,304
 * (2^22; else LEIDEN_EINVAL) and calls that overlap on one GPU race: issue
 * them from one thread or one stream at a time.  The call returns after
 * its work on `stream` is complete. */
leiden_status leiden_modularity_noalloc(leiden_graph* g, const uint32_t* membership, void* stream, double* q_out);

/* Copy the current graph to host memory as a CSR with sorted rows:
 * offsets_out int64[n+1], cols_out uint32[nnz], w_out uint32[nnz] (size them
 * with leiden_graph_nnz). */
leiden_status leiden_graph_export(leiden_graph* g, int64_t* offsets_out, uint32_t* cols_out, uint32_t* w_out);

/* Copy the auxiliary state to host memory: C uint32[n], K int64[n],
 * Sigma int64[n], DeltaSigma int64[n] (any may be NULL).  LEIDEN_ESTATE
 * before the first run. */
leiden_status leiden_state_export(leiden_graph* g, uint32_t* C, int64_t* K, int64_t* Sigma, int64_t* dSigma);

/* Replace the auxiliary state (host memory, all four arrays, length n):
 * resumes a run saved by leiden_state_export on a handle holding the same
 * graph.  K must equal the row sums of the graph and Sigma the sums of K by
 * community, else LEIDEN_EINVAL. */
leiden_status leiden_state_import(leiden_graph* g, const uint32_t* C, const int64_t* K, const int64_t* Sigma,
                                  const int64_t* dSigma);

/* Message of the last failed call on this thread ("" if none). */
const char* leiden_last_error(void);

/* ---------------------------------------------------------------------------
 * Batched form: many independent graphs at once.  `streams` worker threads,
 * each with its own HIP stream, take the handles in order and run the
 * single-graph call on them, so each result equals the one the graph gets
 * alone.  items == NULL: leiden_static on every handle; otherwise
 * leiden_update with items[i] (host batch arrays as for leiden_update, same
 * mode and opts for all).  memberships_out[i]: host uint32[n_i] (entries may
 * be NULL); q_out (may be NULL): double[count]; status_out (may be NULL):
 * per-graph status.  Returns the first failure's status, else LEIDEN_OK.
 * opts->stream is ignored.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * Forest form: many independent graphs held as one block-diagonal graph, so
 * that each phase of Alg. 4 (local moving, refinement, aggregation) and of
 * the dynamic steps (Alg. 1-3, 7, 12) runs as one launch over all of them.
 * Every graph gets the result it gets alone: its own 1/m in Eq. 2, its own
 * stopping rules of Alg. 6 and Alg. 4 (gain sum, iteration count, refinement
 * flag), and schedules hashed on its own vertex IDs.
 *
 * leiden_forest_create: graph q has graph_vertices[q] >= 1 vertices (host
 * array); its vertices are the forest vertices first_q .. first_q +
 * graph_vertices[q] - 1 with first_q the sum of the earlier counts.  The
 * CSR is the forest's (n = sum of the counts; rules as leiden_graph_create);
 * an entry joining two graphs gives LEIDEN_EINVAL.  The handle works with
 * leiden_static, leiden_update, leiden_modularity, leiden_set_tuning,
 * leiden_autotune and leiden_graph_export, with these differences:
 *  - memberships in and out are labels inside each graph (vertex v of graph
 *    q has its label in 0 .. graph_vertices[q] - 1; static labels are dense
 *    per graph, ordered by minimum vertex);
 *  - batch pairs name forest vertices, and a pair joining two graphs gives
 *    LEIDEN_EINVAL;
 *  - q_out receives NaN; Eq. 1 of every graph, and the passes and iteration
 *    counts of the last run, come from leiden_forest_results;
 *  - leiden_state_export / leiden_state_import and
 *    leiden_modularity_noalloc give LEIDEN_EINVAL.
 * leiden_graph_destroy releases it.
 * ------------------------------------------------------------------------- */
leiden_status leiden_forest_create(int device, uint32_t n_graphs, const uint32_t* graph_vertices, uint64_t nnz,
                                   const int64_t* offsets, const uint32_t* cols, const uint32_t* w, int on_device,
                                   double slack, leiden_graph** out);

/* Per-graph results of the last leiden_static / leiden_update /
 * leiden_modularity call on a forest (each pointer may be NULL):
 * q: double[n_graphs] Eq. 1 (NaN when compute_modularity was 0);
 * passes: uint32[n_graphs] passes of Alg. 4 (0 for a graph without edges);
 * iters: uint32[n_graphs][16] local-moving iterations of the first 16
 * passes.  LEIDEN_ESTATE before the first call. */
leiden_status leiden_forest_results(leiden_graph* g, double* q, uint32_t* passes, uint32_t* iters);

/* *n_graphs: graphs of a forest (0 for a single graph); first_vertex (may be
 * NULL): uint32[n_graphs + 1] first forest vertex of every graph, then n. */
leiden_status leiden_forest_info(leiden_graph* g, uint32_t* n_graphs, uint32_t* first_vertex);

typedef struct {
  const uint32_t* del; /* uint32[n_del][2] */
  uint64_t n_del;
  const uint32_t* ins; /* uint32[n_ins][3] */
  uint64_t n_ins;
} leiden_batch_item;

leiden_status leiden_batch_run(leiden_graph* const* graphs, uint32_t count, const leiden_batch_item* items,
                               leiden_mode mode, const leiden_opts* opts, uint32_t streams,
                               uint32_t* const* memberships_out, double* q_out, leiden_status* status_out);

/* ---------------------------------------------------------------------------
 * Serving form: device-resident tenant graphs receiving streams of update
 * batches.  A server owns `workers` threads with one HIP stream each.
 * Requests wait in arrival order and start as soon as a worker is free,
 * except that one graph never runs two requests at once (per-graph order is
 * kept).  Each request is a DF / DS / ND update (leiden_update) whose result
 * equals the one its graph gets alone.
 * ------------------------------------------------------------------------- */
typedef struct leiden_server leiden_server;

typedef struct {
  uint64_t completed, failed, waiting;
  uint32_t graphs, pad_;
  uint64_t hbm_reserved;      /* admitted graphs' estimated device bytes */
  double latency_p50_ms;      /* completion minus arrival */
  double latency_p99_ms;
  double service_p50_ms;      /* completion minus start */
  double service_p99_ms;
  double updated_edges_per_s; /* undirected updates of completed requests over first arrival to last completion */
} leiden_server_stats;

/* workers: 1..64.  hbm_budget_bytes bounds the admitted graphs' estimated
 * device footprint. */
leiden_status leiden_server_create(int device, uint64_t hbm_budget_bytes, uint32_t workers, leiden_server** out);
/* Waits for running requests, then frees every graph and the server. */
void leiden_server_destroy(leiden_server* s);
/* *bytes: the estimated device footprint the admission charges for a graph
 * of n vertices and nnz directed entries held with the given slack. */
leiden_status leiden_server_footprint(uint32_t n, uint64_t nnz, double slack, uint64_t* bytes);
/* Admit a graph (arguments as leiden_graph_create) and run leiden_static on
 * it (opts may be NULL).  LEIDEN_ENOMEM when its estimated footprint does not
 * fit in what is left of the budget; *graph_id receives its ID. */
leiden_status leiden_server_add_graph(leiden_server* s, uint32_t n, uint64_t nnz, const int64_t* offsets,
                                      const uint32_t* cols, const uint32_t* w, int on_device, double slack,
                                      const leiden_opts* opts, uint32_t* graph_id);
/* Free a graph with no waiting requests (LEIDEN_ESTATE otherwise) and return
 * its share of the budget. */
leiden_status leiden_server_remove_graph(leiden_server* s, uint32_t graph_id);
/* Queue an update of graph_id (host batch arrays, copied before returning).
 * *ticket identifies the request. */
leiden_status leiden_server_submit(leiden_server* s, uint32_t graph_id, const uint32_t* del, uint64_t n_del,
                                   const uint32_t* ins, uint64_t n_ins, leiden_mode mode, const leiden_opts* opts,
                                   uint64_t* ticket);
/* Block until the request is done; returns its status and fills the outputs
 * (membership_out: host uint32[n] of its graph; any output may be NULL).
 * Each ticket can be waited for once. */
leiden_status leiden_server_wait(leiden_server* s, uint64_t ticket, uint32_t* membership_out, double* q_out,
                                 leiden_stats* stats_out, double* latency_ms, double* service_ms);
leiden_status leiden_server_get_stats(leiden_server* s, leiden_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* LEIDEN_MI355X_H */
