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
 *     state as they were (updates are transactional).
 *   - Calls on one handle must not overlap; different handles are independent.
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
  LEIDEN_ESTATE = -4   /* handle has no state for the request (e.g. update before any run) */
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
  LEIDEN_KT_HUB_INSERT = 1
} leiden_kernel;
/* (LEIDEN_KT_HUB_INSERT is the kernel that sums chunks of hub rows by
 * community in LDS and merges them into per-hub tables.) */

/* Parameters (defaults from Section 5.1.2). */
typedef struct {
  double tau;             /* initial iteration tolerance, 1e-2 */
  uint32_t tau_re_num;    /* refinement tolerance tau_re = num / den, 3 / 5 */
  uint32_t tau_re_den;
  uint32_t tol_decline;   /* TOLERANCE_DECLINE_FACTOR, 10 */
  uint32_t max_iters;     /* MAX_ITERATIONS per pass, 20 */
  uint32_t max_passes;    /* MAX_PASSES, 10 */
  uint32_t move_classes;  /* vertex classes of the synchronous local-moving sub-rounds, 8 (1..32) */
  uint32_t refine_rounds; /* colour rounds of the synchronous refinement, 8 (1..32) */
  int32_t deterministic;  /* 1: synchronous schedule, bit-exact and reproducible */
  int32_t compute_modularity; /* 1: fill *q_out with Eq. 1 of the result; 0: NaN */
  void* stream;           /* hipStream_t or NULL */
  int32_t timed_kernel;   /* a leiden_kernel to time with HIP events on the stream, or LEIDEN_KT_NONE */
  int32_t pad_;
} leiden_opts;

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
} leiden_stats;

typedef struct leiden_graph leiden_graph;

/* Symbol of a leiden_kernel as profilers list it (NULL for an unknown value). */
const char* leiden_kernel_name(int32_t kernel);

/* Fill *opts with the defaults above. */
leiden_status leiden_default_opts(leiden_opts* opts);

/* Create a handle on GPU `device` holding the undirected graph given as a CSR
 * with both directions of every edge: offsets int64[n+1], cols uint32[nnz],
 * w uint32[nnz] (the graph of Section 3 with integer weights).  Each row
 * must be sorted by column; unsorted rows, duplicate entries, self-loops,
 * zero weights, IDs >= n or an asymmetric matrix give LEIDEN_EINVAL.  `slack`
 * >= 0 reserves room per row for future insertions (fraction of the row
 * length).  *out receives the handle. */
leiden_status leiden_graph_create(int device, uint32_t n, uint64_t nnz, const int64_t* offsets,
                                  const uint32_t* cols, const uint32_t* w, int on_device, double slack,
                                  leiden_graph** out);

void leiden_graph_destroy(leiden_graph* g);

/* Number of directed entries currently held. */
leiden_status leiden_graph_nnz(leiden_graph* g, uint64_t* nnz);

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
 * LEIDEN_EINVAL and changes nothing.  prev_membership: uint32[n] C^{t-1} with
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

#ifdef __cplusplus
}
#endif

#endif /* LEIDEN_MI355X_H */
