/*
 * CPU oracle for the Static / Naive-dynamic (ND) / Delta-screening (DS) /
 * Dynamic Frontier (DF) Leiden method of "Heuristic-based Dynamic Leiden
 * Algorithm for Efficient Tracking of Communities on Evolving Graphs" (Sahu).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path; the two meet only through the
 * seeded input generators.
 *
 * Plain, slow, single-threaded C++17.  Every step follows the paper's
 * algorithms in their order and notation; steps that have a plain definition
 * (modularity, connected components, renumbering, aggregation, overlap
 * tracking) compute that definition directly.
 *
 * Two schedules of the vertex-parallel loops:
 *   SEQ    - one thread sweeping vertices in ascending ID, reading and writing
 *            live state: the paper's asynchronous algorithm run on one thread.
 *   JACOBI - blocked synchronous sub-rounds that decide against a snapshot and
 *            apply all decisions together; the reference for the deterministic
 *            GPU mode.  Its class, min-label and colour-round rules are readings
 *            of this project, not the paper's: parity unpinned against the paper
 *            (pinned only against invariants and the SEQ schedule).
 *
 * Readings where the paper is silent or ambiguous (each also listed in the
 * design notes):
 *   - integer edge weights, int64 K / Sigma sums; delta-modularity (Eq. 2) in
 *     binary64 with one fixed operation order and no fused multiply-add;
 *   - candidate communities are the neighbour communities other than the
 *     current one; equal gains go to the lowest community ID; a vertex moves
 *     only on a strictly positive gain;
 *   - the community marked for splitting in the local-moving phase is the
 *     source community of the moving vertex;
 *   - the per-iteration gain sum is an int64 fixed-point sum (2^56 scale);
 *   - the subset-renumber representative is the minimum member vertex;
 *   - split labels are the minimum vertex of each connected component;
 *   - the iteration count returned by the local-moving phase is the number of
 *     iterations executed; the pass loop breaks as its pseudocode states;
 *   - vertex marking functions apply to the first pass only;
 *   - markCommunities flags are indexed by community; a marked community's
 *     cumulative change is reset to zero; the tolerance is a rational num/den;
 *   - tracking picks the exact maximum-overlap community (ties to the lowest
 *     minimum vertex, then the lowest old ID) and gives unmatched communities
 *     the smallest IDs that were not previous labels;
 *   - static output labels are dense, ordered by each community's minimum
 *     vertex; a graph without edges yields singleton communities.
 */
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>
#include <vector>

namespace {

using i64 = int64_t;
using u64 = uint64_t;
using u32 = uint32_t;
using u8 = uint8_t;
using u128 = unsigned __int128;

const u32 kEmpty = 0xFFFFFFFFu;

}  // namespace

extern "C" {

typedef struct {
  double tau;           /* initial iteration tolerance (Section 5.1.2: 1e-2) */
  uint32_t tau_re_num;  /* refinement tolerance as num/den (0.6 = 3/5) */
  uint32_t tau_re_den;
  uint32_t tol_decline; /* TOLERANCE_DECLINE_FACTOR (10) */
  uint32_t max_iters;   /* MAX_ITERATIONS per pass (20) */
  uint32_t max_passes;  /* MAX_PASSES (10) */
  int32_t schedule;     /* 0 = SEQ, 1 = JACOBI */
  uint32_t move_classes;  /* JACOBI: vertex classes per local-moving iteration (4) */
  uint32_t refine_rounds; /* JACOBI: colour rounds of the refinement (8) */
  int32_t split_all;      /* 1: split every community not marked for refinement (Section 4.3's
                             comparison with selective splitting), 0: selective (default) */
} oracle_opts;

typedef struct {
  uint32_t passes;
  uint32_t iters[16];
  uint32_t subrounds[16];
  uint64_t affected;       /* vertices marked affected before the first pass */
  uint64_t split_marked;   /* communities split-marked and not refined, first pass */
  uint64_t refine_marked;  /* communities marked for refinement by markCommunities */
  uint64_t moves;          /* local-moving moves over all passes */
  uint64_t refine_moves;   /* refinement moves over all passes */
  uint64_t edges_scanned;  /* local-moving edge scans over all passes */
  int32_t refined_first_pass;
  int32_t m2_zero;
} oracle_stats;

}  // extern "C"

namespace {

struct Graph {
  u32 n = 0;
  std::vector<i64> offs;  // n + 1
  std::vector<u32> cols;
  std::vector<i64> w;
};

Graph graph_from(u32 n, const int64_t* offs, const uint32_t* cols, const uint32_t* w) {
  Graph g;
  g.n = n;
  g.offs.assign(offs, offs + n + 1);
  i64 nnz = offs[n];
  g.cols.assign(cols, cols + nnz);
  g.w.resize(nnz);
  for (i64 e = 0; e < nnz; ++e) g.w[e] = (i64)w[e];
  return g;
}

/* ---------------------------------------------------------------------------
 * Eq. 2: delta-modularity of moving i from community d to community c.
 *   dQ = (K_{i->c} - K_{i->d}) / m  -  K_i (K_i + Sigma_c - Sigma_d) / (2 m^2)
 * The integer parts are exact; the float part is evaluated in one fixed order,
 * each product and difference rounded on its own.
 * ------------------------------------------------------------------------- */
struct Consts {
  i64 M2;  // 2m = sum of K_i
  double m, inv_m, inv_2m2;
};

Consts make_consts(i64 M2) {
  Consts k;
  k.M2 = M2;
  k.m = 0.5 * (double)M2;
  k.inv_m = 1.0 / k.m;
  k.inv_2m2 = 1.0 / ((2.0 * k.m) * k.m);
  return k;
}

double delta_modularity(i64 Kic, i64 Kid, i64 Ki, i64 Sc, i64 Sd, const Consts& k) {
  double a = (double)(Kic - Kid);
  double b = (double)(Ki + Sc - Sd);
  double first = a * k.inv_m;
  double kb = (double)Ki * b;
  double second = kb * k.inv_2m2;
  return first - second;
}

/* Per-iteration gain sum as an int64 fixed-point number with 2^56 scale. */
const double kTwo56 = 72057594037927936.0;
i64 gain_to_fixed(double dq) { return (i64)(dq * kTwo56); }
double fixed_to_gain(i64 s) { return (double)s / kTwo56; }

/* Optional record of a run for the tests (never read by the algorithm): every
 * local-moving move (pass, iteration, vertex, source and target community,
 * gain), and for every pass of Alg. 4 its iteration count, tolerance, whether
 * a community was refined, and the communities of the input vertices given by
 * the pass's local-moving labels (the refinement bounds) and by its refined
 * labels. */
struct Trace {
  u32 pass = 0;
  std::vector<u32> move_rec;  // 5 per move: pass, iteration, vertex, from, to
  std::vector<double> move_dq;
  std::vector<u32> pass_rec;  // 4 per pass: iterations, refined, level vertices, moves
  std::vector<double> pass_tau;
  std::vector<std::vector<u32>> bound_proj, refined_proj;
  void move(u32 li, u32 v, u32 from, u32 to, double dq) {
    move_rec.insert(move_rec.end(), {pass, li, v, from, to});
    move_dq.push_back(dq);
  }
};
thread_local Trace* g_trace = nullptr;

/* MurmurHash3 32-bit finaliser (Appleby): hashes vertex IDs into the classes
 * of the synchronous schedules. */
u32 fmix32(u32 h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
/* Class of vertex v in iteration t of the blocked synchronous local-moving
 * schedule, and its colour for the synchronous refinement rounds. */
u32 move_class(u32 v, u32 t, u32 P) { return fmix32(v + t * 0x9e3779b9u) % P; }
u32 refine_colour(u32 v, u32 R) { return fmix32(v) % R; }

/* The paper's collision-free hashtable: a dense value array indexed by
 * community plus the list of keys that are set. */
struct Table {
  std::vector<i64> val;
  std::vector<u8> has;
  std::vector<u32> keys;
  explicit Table(u32 n) : val(n, 0), has(n, 0) {}
  void add(u32 c, i64 w) {
    if (!has[c]) {
      has[c] = 1;
      keys.push_back(c);
    }
    val[c] += w;
  }
  i64 get(u32 c) const { return has[c] ? val[c] : 0; }
  void clear() {
    for (u32 c : keys) {
      val[c] = 0;
      has[c] = 0;
    }
    keys.clear();
  }
};

/* scanCommunities (Alg. 6): H[C[j]] += w over the edges of i, skipping the
 * self-loop unless `self`. */
u64 scan_communities(Table& H, const Graph& G, const std::vector<u32>& C, u32 i, bool self) {
  for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) {
    u32 j = G.cols[e];
    if (!self && j == i) continue;
    H.add(C[j], G.w[e]);
  }
  return (u64)(G.offs[i + 1] - G.offs[i]);
}

/* scanBounded (Alg. 8): as scanCommunities but only neighbours inside the
 * community bound of i. */
void scan_bounded(Table& H, const Graph& G, const std::vector<u32>& CB, const std::vector<u32>& C, u32 i,
                  bool self) {
  for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) {
    u32 j = G.cols[e];
    if (!self && j == i) continue;
    if (CB[i] != CB[j]) continue;
    H.add(C[j], G.w[e]);
  }
}

struct Choice {
  bool found = false;
  u32 c = 0;
  double dq = 0.0;
};

/* Best community linked to i: the largest Eq. 2 gain over the neighbour
 * communities other than d, equal gains to the lowest ID.  `allow` filters
 * candidates (used by the synchronous refinement). */
template <class Allow>
Choice best_community(const Table& H, u32 d, i64 Ki, const std::vector<i64>& S, const Consts& k, Allow allow) {
  Choice best;
  i64 Kid = H.get(d);
  for (u32 c : H.keys) {
    if (c == d || !allow(c)) continue;
    double dq = delta_modularity(H.val[c], Kid, Ki, S[c], S[d], k);
    if (!best.found || dq > best.dq || (dq == best.dq && c < best.c)) {
      best.found = true;
      best.c = c;
      best.dq = dq;
    }
  }
  return best;
}

struct Level {
  Graph G;               // G'
  std::vector<u32> C;    // C'
  std::vector<i64> K;    // K'
  std::vector<i64> S;    // Sigma'
  std::vector<u32> size; // members per community label (exact isolation test)
  std::vector<u8> dS;    // communities marked to be split
  std::vector<u8> dR;    // communities marked to be refined
};

struct MoveResult {
  u32 iterations = 0;
  u32 subrounds = 0;
  u64 moves = 0;
  u64 edges = 0;
};

/* Alg. 6, SEQ schedule: one sweep per iteration in ascending vertex order,
 * pruning with the unprocessed flags. */
MoveResult move_seq(Level& L, std::vector<u8>& unprocessed, const std::vector<u8>* in_range, bool dynamic,
                    double tau, const Consts& k, u32 max_iters) {
  MoveResult r;
  u32 n = L.G.n;
  Table H(n);
  for (u32 li = 0; li < max_iters; ++li) {
    i64 dQ = 0;
    r.subrounds++;
    for (u32 i = 0; i < n; ++i) {
      if (!unprocessed[i]) continue;
      unprocessed[i] = 0;  // prune
      if (in_range && !(*in_range)[i]) continue;
      r.edges += scan_communities(H, L.G, L.C, i, false);
      u32 d = L.C[i];
      Choice ch = best_community(H, d, L.K[i], L.S, k, [](u32) { return true; });
      H.clear();
      if (!ch.found || !(ch.dq > 0.0)) continue;
      L.S[d] -= L.K[i];
      L.S[ch.c] += L.K[i];
      L.size[d] -= 1;
      L.size[ch.c] += 1;
      L.C[i] = ch.c;
      dQ += gain_to_fixed(ch.dq);
      r.moves++;
      if (g_trace) g_trace->move(li, i, d, ch.c, ch.dq);
      for (i64 e = L.G.offs[i]; e < L.G.offs[i + 1]; ++e) unprocessed[L.G.cols[e]] = 1;
      if (dynamic) L.dS[d] = 1;
    }
    r.iterations = li + 1;
    if (fixed_to_gain(dQ) <= tau) break;
  }
  return r;
}

/* Alg. 6, JACOBI schedule (blocked).  Iteration t hashes the vertices into
 * P classes, class_t(v) = fmix32(v + t * 0x9e3779b9) mod P, and runs one
 * sub-round per class in ascending class order: the class's pending vertices
 * decide against the state at the start of the sub-round, then all their
 * moves are applied together (Jacobi inside a class, Gauss-Seidel across
 * classes, as the ascending sweep of the sequential loop is across vertices).
 * A mover's neighbour in a later class joins that class's sub-round of the
 * same iteration; any other neighbour is marked unprocessed for t + 1, as the
 * sequential sweep does for vertices it has already passed.  A vertex alone in
 * its community does not move to another singleton community of higher label
 * (two singletons of one class would otherwise swap forever). */
MoveResult move_jacobi(Level& L, std::vector<u8>& unprocessed, const std::vector<u8>* in_range, bool dynamic,
                       double tau, const Consts& k, u32 max_iters, u32 P) {
  MoveResult r;
  u32 n = L.G.n;
  Table H(n);
  std::vector<u8> pending_flag(n, 0);
  struct Move {
    u32 i, c;
    double dq;
  };
  for (u32 li = 0; li < max_iters; ++li) {
    i64 dQ = 0;
    std::vector<std::vector<u32>> pending(P);
    auto cls = [&](u32 v) { return move_class(v, li, P); };
    for (u32 i = 0; i < n; ++i)
      if (unprocessed[i]) {
        pending[cls(i)].push_back(i);
        pending_flag[i] = 1;
        unprocessed[i] = 0;
      }
    for (u32 kc = 0; kc < P; ++kc) {
      std::vector<u32> active;
      active.swap(pending[kc]);
      if (active.empty()) continue;
      r.subrounds++;
      std::vector<Move> moves;
      for (u32 i : active) {
        pending_flag[i] = 0;  // processed in this iteration
        if (in_range && !(*in_range)[i]) continue;
        r.edges += scan_communities(H, L.G, L.C, i, false);
        u32 d = L.C[i];
        Choice ch = best_community(H, d, L.K[i], L.S, k, [](u32) { return true; });
        H.clear();
        if (!ch.found || !(ch.dq > 0.0)) continue;
        if (L.size[d] == 1 && L.size[ch.c] == 1 && ch.c > d) continue;  // min-label rule
        moves.push_back({i, ch.c, ch.dq});
      }
      for (const Move& mv : moves) {
        u32 d = L.C[mv.i];
        L.S[d] -= L.K[mv.i];
        L.S[mv.c] += L.K[mv.i];
        L.size[d] -= 1;
        L.size[mv.c] += 1;
        L.C[mv.i] = mv.c;
        dQ += gain_to_fixed(mv.dq);
        if (dynamic) L.dS[d] = 1;
        if (g_trace) g_trace->move(li, mv.i, d, mv.c, mv.dq);
      }
      r.moves += moves.size();
      for (const Move& mv : moves) {
        for (i64 e = L.G.offs[mv.i]; e < L.G.offs[mv.i + 1]; ++e) {
          u32 j = L.G.cols[e];
          u32 kj = cls(j);
          if (kj > kc) {
            if (!pending_flag[j]) {
              pending_flag[j] = 1;
              pending[kj].push_back(j);
            }
          } else {
            unprocessed[j] = 1;
          }
        }
      }
    }
    r.iterations = li + 1;
    if (fixed_to_gain(dQ) <= tau) break;
  }
  return r;
}

/* Alg. 10: each community takes the ID of its minimum member vertex; Sigma',
 * the member counts and the split/refine flags move with the label, and
 * labels left without members are dropped. */
void subset_renumber(Level& L) {
  u32 n = L.G.n;
  std::vector<u32> rep(n, kEmpty);
  for (u32 i = 0; i < n; ++i) {
    u32 c = L.C[i];
    if (rep[c] == kEmpty) rep[c] = i;
  }
  std::vector<i64> S2(n, 0);
  std::vector<u32> size2(n, 0);
  std::vector<u8> dS2(n, 0), dR2(n, 0);
  for (u32 c = 0; c < n; ++c) {
    u32 r = rep[c];
    if (r == kEmpty) continue;
    S2[r] = L.S[c];
    size2[r] = L.size[c];
    dS2[r] = L.dS[c];
    dR2[r] = L.dR[c];
  }
  for (u32 i = 0; i < n; ++i) L.C[i] = rep[L.C[i]];
  L.S.swap(S2);
  L.size.swap(size2);
  L.dS.swap(dS2);
  L.dR.swap(dR2);
}

/* Alg. 7 by its definition: every community marked to be split and not marked
 * to be refined is replaced by the connected components of the subgraph its
 * vertices induce, each labelled by its minimum vertex.  Returns the number
 * of communities split-marked. */
u64 split_communities(Level& L, bool split_all) {
  u32 n = L.G.n;
  std::vector<u32> out = L.C;
  std::vector<u8> seen(n, 0);
  std::vector<u32> queue;
  std::vector<u8> counted(n, 0);
  u64 marked = 0;
  for (u32 s = 0; s < n; ++s) {
    u32 c = L.C[s];
    if (!((split_all || L.dS[c]) && !L.dR[c])) continue;
    if (!counted[c]) {
      counted[c] = 1;
      marked++;
    }
    if (seen[s]) continue;
    // s is the smallest unvisited vertex of c, hence the minimum of its component
    queue.clear();
    queue.push_back(s);
    seen[s] = 1;
    for (size_t q = 0; q < queue.size(); ++q) {
      u32 u = queue[q];
      out[u] = s;
      for (i64 e = L.G.offs[u]; e < L.G.offs[u + 1]; ++e) {
        u32 j = L.G.cols[e];
        if (j == u || L.C[j] != c || seen[j]) continue;
        seen[j] = 1;
        queue.push_back(j);
      }
    }
  }
  L.C.swap(out);
  return marked;
}

/* Alg. 8.  First every vertex whose bound is marked for refinement becomes a
 * singleton.  Then isolated vertices of refined bounds may join the best
 * sub-community inside their bound.  SEQ: one ascending sweep with live state
 * (the paper's CAS guard always succeeds on one thread).  JACOBI: R rounds by
 * vertex colour fmix32(v) mod R; in round r only colour-r isolated vertices
 * move, and only into communities that cannot move in the same round (two or
 * more members, or a singleton whose vertex has another colour); decisions use
 * the state at the start of the round.  Either way every vertex gets one
 * chance.  Returns whether any vertex lies in a refined bound. */
bool refine(Level& L, const std::vector<u32>& CB, const Consts& k, bool jacobi, u32 R, u64* moves_out) {
  u32 n = L.G.n;
  bool any = false;
  for (u32 i = 0; i < n; ++i) {
    if (!L.dR[CB[i]]) continue;
    any = true;
    L.C[i] = i;
    L.S[i] = L.K[i];
    L.size[i] = 1;
  }
  if (!any) return false;
  Table H(n);
  u64 moves = 0;
  if (!jacobi) {
    for (u32 i = 0; i < n; ++i) {
      u32 c = L.C[i];
      if (!L.dR[CB[i]] || L.size[c] != 1) continue;
      scan_bounded(H, L.G, CB, L.C, i, false);
      Choice ch = best_community(H, c, L.K[i], L.S, k, [](u32) { return true; });
      H.clear();
      if (!ch.found || !(ch.dq > 0.0)) continue;
      if (ch.c == c || L.C[ch.c] != ch.c) continue;
      L.S[c] -= L.K[i];
      L.S[ch.c] += L.K[i];
      L.size[c] -= 1;
      L.size[ch.c] += 1;
      L.C[i] = ch.c;
      moves++;
    }
  } else {
    struct Move {
      u32 i, c;
    };
    for (u32 r = 0; r < R; ++r) {
      std::vector<Move> mv;
      for (u32 i = 0; i < n; ++i) {
        u32 c = L.C[i];
        if (!L.dR[CB[i]] || L.size[c] != 1 || refine_colour(i, R) != r) continue;
        scan_bounded(H, L.G, CB, L.C, i, false);
        const std::vector<u32>& size = L.size;
        Choice ch = best_community(H, c, L.K[i], L.S, k,
                                   [&](u32 t) { return size[t] >= 2 || refine_colour(t, R) != r; });
        H.clear();
        if (!ch.found || !(ch.dq > 0.0)) continue;
        mv.push_back({i, ch.c});
      }
      for (const Move& m : mv) {
        u32 c = L.C[m.i];
        L.S[c] -= L.K[m.i];
        L.S[m.c] += L.K[m.i];
        L.size[c] -= 1;
        L.size[m.c] += 1;
        L.C[m.i] = m.c;
      }
      moves += mv.size();
    }
  }
  if (moves_out) *moves_out += moves;
  return true;
}

/* Renumber communities densely in ascending label order; returns the count. */
u32 renumber_dense(std::vector<u32>& C, u32 n) {
  std::vector<u32> id(n, kEmpty);
  for (u32 i = 0; i < n; ++i) id[C[i]] = 0;
  u32 next = 0;
  for (u32 c = 0; c < n; ++c)
    if (id[c] != kEmpty) id[c] = next++;
  for (u32 i = 0; i < n; ++i) C[i] = id[C[i]];
  return next;
}

/* Alg. 9 by its definition: w''(c, d) = sum of w_ij over all CSR entries with
 * C[i] = c and C[j] = d, self-loops included; rows sorted by d. */
Graph aggregate(const Graph& G, const std::vector<u32>& C, u32 nc) {
  std::vector<std::tuple<u32, u32, i64>> t;
  t.reserve(G.cols.size());
  for (u32 i = 0; i < G.n; ++i)
    for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) t.emplace_back(C[i], C[G.cols[e]], G.w[e]);
  std::sort(t.begin(), t.end());
  Graph A;
  A.n = nc;
  A.offs.assign(nc + 1, 0);
  for (size_t a = 0; a < t.size();) {
    size_t b = a;
    i64 sum = 0;
    while (b < t.size() && std::get<0>(t[b]) == std::get<0>(t[a]) && std::get<1>(t[b]) == std::get<1>(t[a]))
      sum += std::get<2>(t[b++]);
    A.cols.push_back(std::get<1>(t[a]));
    A.w.push_back(sum);
    A.offs[std::get<0>(t[a]) + 1]++;
    a = b;
  }
  for (u32 c = 0; c < nc; ++c) A.offs[c + 1] += A.offs[c];
  return A;
}

std::vector<i64> row_sums(const Graph& G) {
  std::vector<i64> K(G.n, 0);
  for (u32 i = 0; i < G.n; ++i)
    for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) K[i] += G.w[e];
  return K;
}

/* Eq. 1 by its definition: Q = sum_c [sigma_c / 2m - (Sigma_c / 2m)^2], with
 * sigma the weight of CSR entries inside a community (a self-loop entry
 * counted once) and Sigma_c the total weight of the entries leaving c's
 * vertices.  Integer sums are exact; the final expression is
 * sigma/2m - T/(2m)^2 with T = sum_c Sigma_c^2 as a 128-bit integer. */
struct QParts {
  i64 sigma = 0;
  u128 T = 0;
  i64 M2 = 0;
};

QParts modularity_parts(const Graph& G, const std::vector<u32>& C) {
  QParts p;
  std::vector<i64> Sig(G.n, 0);
  for (u32 i = 0; i < G.n; ++i)
    for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) {
      i64 w = G.w[e];
      p.M2 += w;
      Sig[C[i]] += w;
      if (C[i] == C[G.cols[e]]) p.sigma += w;
    }
  for (u32 c = 0; c < G.n; ++c) p.T += (u128)(u64)Sig[c] * (u128)(u64)Sig[c];
  return p;
}

double modularity_value(const QParts& p) {
  if (p.M2 == 0) return 0.0;
  double m2 = (double)p.M2;
  double first = (double)p.sigma / m2;
  double second = (double)p.T / (m2 * m2);
  return first - second;
}

/* Alg. 12 by its stated purpose: each old community b picks the current
 * community with the largest overlap (total K^t of shared vertices; ties to
 * the community with the lowest minimum vertex, so the result does not depend
 * on how current communities are labelled); each current community takes,
 * among the old communities that picked it, the one with the largest overlap
 * (ties to the lowest old ID).  The
 * remaining current communities, in ascending order of their minimum vertex,
 * take the smallest IDs that were not previous labels.  `matched` receives the
 * old labels that were kept. */
std::vector<u32> track(const std::vector<u32>& Ccur, const std::vector<u32>& Cprev, const std::vector<i64>& K,
                       std::vector<u8>* matched) {
  u32 n = (u32)Ccur.size();
  std::map<std::pair<u32, u32>, i64> overlap;
  for (u32 i = 0; i < n; ++i) overlap[{Cprev[i], Ccur[i]}] += K[i];
  std::map<u32, u32> min_vertex;  // current community -> its minimum vertex
  for (u32 i = 0; i < n; ++i)
    if (!min_vertex.count(Ccur[i])) min_vertex[Ccur[i]] = i;
  std::map<u32, std::pair<u32, i64>> best_of_old;  // b -> (c, w)
  for (const auto& kv : overlap) {
    u32 b = kv.first.first, c = kv.first.second;
    i64 w = kv.second;
    auto it = best_of_old.find(b);
    if (it == best_of_old.end() || w > it->second.second ||
        (w == it->second.second && min_vertex[c] < min_vertex[it->second.first]))
      best_of_old[b] = {c, w};
  }
  std::map<u32, std::pair<u32, i64>> best_for_cur;  // c -> (b, w)
  for (const auto& kv : best_of_old) {
    u32 b = kv.first, c = kv.second.first;
    i64 w = kv.second.second;
    auto it = best_for_cur.find(c);
    if (it == best_for_cur.end() || w > it->second.second) best_for_cur[c] = {b, w};
  }
  std::vector<u8> is_old(n, 0);
  for (u32 i = 0; i < n; ++i) is_old[Cprev[i]] = 1;
  std::map<u32, u32> label;
  if (matched) matched->assign(n, 0);
  for (const auto& kv : best_for_cur) {
    label[kv.first] = kv.second.first;
    if (matched) (*matched)[kv.second.first] = 1;
  }
  u32 next_free = 0;
  std::vector<u32> out(n);
  for (u32 i = 0; i < n; ++i) {
    u32 c = Ccur[i];
    auto it = label.find(c);
    if (it == label.end()) {
      while (is_old[next_free]) ++next_free;
      label[c] = next_free++;
      it = label.find(c);
    }
    out[i] = it->second;
  }
  return out;
}

/* Static output labels: dense IDs in ascending order of each community's
 * minimum vertex. */
std::vector<u32> relabel_by_min_vertex(const std::vector<u32>& C) {
  u32 n = (u32)C.size();
  std::vector<u32> id(n, kEmpty);
  std::vector<u32> out(n);
  u32 next = 0;
  for (u32 i = 0; i < n; ++i) {
    if (id[C[i]] == kEmpty) id[C[i]] = next++;
    out[i] = id[C[i]];
  }
  return out;
}

/* Vertex marking functions F passed to Alg. 4. */
struct Marking {
  std::vector<u8> affected;     // isAffected(i)
  std::vector<u8> in_range;     // inAffectedRange(i)
  bool range_all = true;        // inAffectedRange == 1 for every vertex
};

/* Alg. 4: the pass loop. */
std::vector<u32> leiden(const Graph& G0, const std::vector<u32>& Cprev, const std::vector<i64>& Kt,
                        const std::vector<i64>& St, std::vector<u8> dS, std::vector<u8> dR, const Marking& F,
                        bool dynamic, const oracle_opts& o, oracle_stats* st) {
  u32 n = G0.n;
  std::vector<u32> C(n);
  for (u32 i = 0; i < n; ++i) C[i] = i;
  i64 M2 = 0;
  for (i64 x : Kt) M2 += x;
  if (M2 == 0) {  // no edges: every vertex stays alone
    if (st) st->m2_zero = 1;
    return C;
  }
  const Consts k = make_consts(M2);
  const bool jacobi = o.schedule == 1;
  Level L;
  L.G = G0;
  L.C = Cprev;
  L.K = Kt;
  L.S = St;
  L.size.assign(n, 0);
  for (u32 i = 0; i < n; ++i) L.size[Cprev[i]]++;
  L.dS = std::move(dS);
  L.dR = std::move(dR);
  std::vector<u8> unprocessed = F.affected;
  double tau = o.tau;
  std::vector<u32> CB;  // C'_B: the refinement bounds of the current pass
  u32 lp = 0;
  for (; lp < o.max_passes; ++lp) {
    const std::vector<u8>* in_range = (lp == 0 && !F.range_all) ? &F.in_range : nullptr;
    if (g_trace) g_trace->pass = lp;
    MoveResult mr = jacobi ? move_jacobi(L, unprocessed, in_range, dynamic, tau, k, o.max_iters, o.move_classes)
                           : move_seq(L, unprocessed, in_range, dynamic, tau, k, o.max_iters);
    if (st) {
      if (lp < 16) {
        st->iters[lp] = mr.iterations;
        st->subrounds[lp] = mr.subrounds;
      }
      st->moves += mr.moves;
      st->edges_scanned += mr.edges;
    }
    u32 li = mr.iterations;
    subset_renumber(L);
    u64 split_marked = split_communities(L, o.split_all != 0);
    if (st && lp == 0) st->split_marked = split_marked;
    CB = L.C;
    u64 rmoves = 0;
    bool refined = refine(L, CB, k, jacobi, o.refine_rounds, &rmoves);
    if (st) {
      st->refine_moves += rmoves;
      if (lp == 0) st->refined_first_pass = refined ? 1 : 0;
    }
    if (g_trace) {
      g_trace->pass_rec.insert(g_trace->pass_rec.end(), {li, refined ? 1u : 0u, L.G.n, (u32)mr.moves});
      g_trace->pass_tau.push_back(tau);
      std::vector<u32> pb(n), pr(n);
      for (u32 v = 0; v < n; ++v) {
        pb[v] = CB[C[v]];
        pr[v] = L.C[C[v]];
      }
      g_trace->bound_proj.push_back(std::move(pb));
      g_trace->refined_proj.push_back(std::move(pr));
    }
    if (li <= 1 && !refined) break;
    if (li <= 1 && lp > 0) break;
    u32 nc = renumber_dense(L.C, L.G.n);
    for (u32 v = 0; v < n; ++v) C[v] = L.C[C[v]];
    L.G = aggregate(L.G, L.C, nc);
    L.K = row_sums(L.G);
    L.S = L.K;
    L.size.assign(nc, 1);
    L.C.resize(nc);
    for (u32 c = 0; c < nc; ++c) L.C[c] = c;
    unprocessed.assign(nc, 1);
    L.dR.assign(nc, 1);
    L.dS.assign(nc, 0);
    tau = tau / (double)o.tol_decline;
  }
  if (st) st->passes = lp < o.max_passes ? lp + 1 : o.max_passes;
  for (u32 v = 0; v < n; ++v) C[v] = L.C[C[v]];
  return C;
}

oracle_opts default_opts() {
  oracle_opts o;
  o.tau = 1e-2;
  o.tau_re_num = 3;
  o.tau_re_den = 5;
  o.tol_decline = 10;
  o.max_iters = 20;
  o.max_passes = 10;
  o.schedule = 1;
  o.move_classes = 4;
  o.refine_rounds = 8;
  o.split_all = 0;
  return o;
}

struct Entry {
  u32 i, j;
  i64 w;
};

}  // namespace

extern "C" {

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1 };

void oracle_default_opts(oracle_opts* o) { *o = default_opts(); }

double oracle_delta_modularity(int64_t Kic, int64_t Kid, int64_t Ki, int64_t Sc, int64_t Sd, int64_t M2) {
  return delta_modularity(Kic, Kid, Ki, Sc, Sd, make_consts(M2));
}

/* Eq. 1 on a CSR with int64 weights; also returns sigma, 2m and T (hi, lo). */
double oracle_modularity64(uint32_t n, const int64_t* offs, const uint32_t* cols, const int64_t* w,
                           const uint32_t* C, int64_t* sigma_out, int64_t* m2_out, uint64_t* T_out) {
  Graph G;
  G.n = n;
  G.offs.assign(offs, offs + n + 1);
  G.cols.assign(cols, cols + offs[n]);
  G.w.assign(w, w + offs[n]);
  std::vector<u32> c(C, C + n);
  QParts p = modularity_parts(G, c);
  if (sigma_out) *sigma_out = p.sigma;
  if (m2_out) *m2_out = p.M2;
  if (T_out) {
    T_out[0] = (u64)(p.T >> 64);
    T_out[1] = (u64)p.T;
  }
  return modularity_value(p);
}

double oracle_modularity(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w,
                         const uint32_t* C) {
  Graph G = graph_from(n, offs, cols, w);
  std::vector<u32> c(C, C + n);
  return modularity_value(modularity_parts(G, c));
}

/* Alg. 9 on a CSR with int64 weights and dense labels C < nc.  Call once with
 * null outputs to learn the entry count. */
int64_t oracle_aggregate(uint32_t n, const int64_t* offs, const uint32_t* cols, const int64_t* w, const uint32_t* C,
                         uint32_t nc, int64_t* offs_out, uint32_t* cols_out, int64_t* w_out) {
  Graph G;
  G.n = n;
  G.offs.assign(offs, offs + n + 1);
  G.cols.assign(cols, cols + offs[n]);
  G.w.assign(w, w + offs[n]);
  std::vector<u32> c(C, C + n);
  Graph A = aggregate(G, c, nc);
  if (offs_out) {
    std::memcpy(offs_out, A.offs.data(), sizeof(int64_t) * (nc + 1));
    std::memcpy(cols_out, A.cols.data(), sizeof(uint32_t) * A.cols.size());
    std::memcpy(w_out, A.w.data(), sizeof(int64_t) * A.w.size());
  }
  return (int64_t)A.cols.size();
}

/* Split one partition by Alg. 7's definition (all communities with
 * split[c] = 1 and refine[c] = 0). */
void oracle_split(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w, uint32_t* C,
                  const uint8_t* split, const uint8_t* refine_flags) {
  Level L;
  L.G = graph_from(n, offs, cols, w);
  L.C.assign(C, C + n);
  L.dS.assign(split, split + n);
  L.dR.assign(refine_flags, refine_flags + n);
  split_communities(L, false);
  std::memcpy(C, L.C.data(), sizeof(uint32_t) * n);
}

/* Recording of runs for the tests: oracle_trace_enable(1) starts a fresh
 * record on the calling thread (0 drops it); the runs that follow append to
 * it; the readers below copy it out. */
void oracle_trace_enable(int on) {
  static thread_local Trace t;
  t = Trace();
  g_trace = on ? &t : nullptr;
}

/* Moves in order: rec[5k..5k+4] = pass, iteration (0-based), vertex of the
 * pass's level graph, source and target community; dq[k] = its gain.
 * Returns the move count (copies at most cap). */
int64_t oracle_trace_moves(uint32_t* rec, double* dq, int64_t cap) {
  if (!g_trace) return 0;
  int64_t cnt = (int64_t)g_trace->move_dq.size();
  for (int64_t k = 0; k < std::min(cnt, cap); ++k) {
    for (int f = 0; f < 5; ++f) rec[5 * k + f] = g_trace->move_rec[5 * k + f];
    dq[k] = g_trace->move_dq[k];
  }
  return cnt;
}

/* Passes in order: rec[4p..4p+3] = local-moving iterations, refined (0/1),
 * vertices of the level graph, local-moving moves; tau[p] = the pass's
 * tolerance.  Returns the pass count (copies at most cap). */
uint32_t oracle_trace_passes(uint32_t* rec, double* tau, uint32_t cap) {
  if (!g_trace) return 0;
  uint32_t cnt = (uint32_t)g_trace->pass_tau.size();
  for (uint32_t p = 0; p < std::min(cnt, cap); ++p) {
    for (int f = 0; f < 4; ++f) rec[4 * p + f] = g_trace->pass_rec[4 * p + f];
    tau[p] = g_trace->pass_tau[p];
  }
  return cnt;
}

/* Communities of the input vertices after pass p: which = 0 by the pass's
 * local-moving labels (the refinement bounds), 1 by its refined labels.
 * out: uint32[n] of the input graph.  Returns 0, or -1 for no such pass. */
int oracle_trace_projection(uint32_t p, int which, uint32_t* out) {
  if (!g_trace || p >= g_trace->bound_proj.size()) return -1;
  const std::vector<u32>& v = which ? g_trace->refined_proj[p] : g_trace->bound_proj[p];
  std::memcpy(out, v.data(), sizeof(uint32_t) * v.size());
  return 0;
}

/* Static Leiden: Alg. 4 with C^{t-1} = identity, Sigma = K, every community
 * marked for refinement (Alg. 5, static branch), every vertex affected, no
 * split marking and no tracking.  Output labels are dense, ordered by minimum
 * vertex. */
int oracle_static(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w, const oracle_opts* opts,
                  uint32_t* C_out, double* q_out, oracle_stats* st) {
  oracle_opts o = opts ? *opts : default_opts();
  if (st) std::memset(st, 0, sizeof(*st));
  Graph G = graph_from(n, offs, cols, w);
  std::vector<i64> K = row_sums(G);
  std::vector<u32> Cprev(n);
  for (u32 i = 0; i < n; ++i) Cprev[i] = i;
  Marking F;
  F.affected.assign(n, 1);
  F.range_all = true;
  if (st) st->affected = n;
  std::vector<u32> C = leiden(G, Cprev, K, K, std::vector<u8>(n, 0), std::vector<u8>(n, 1), F, false, o, st);
  C = relabel_by_min_vertex(C);
  std::memcpy(C_out, C.data(), sizeof(uint32_t) * n);
  if (q_out) *q_out = modularity_value(modularity_parts(G, C));
  return ORACLE_OK;
}

/* Batch application G^{t-1} -> G^t with set semantics (Section 3.5): the
 * deleted pairs must exist, the inserted pairs must be absent, no self-loops,
 * IDs < n, no pair twice in the batch.  Also returns each deleted edge's
 * weight in G^{t-1}.  The caller sizes the outputs for
 * nnz - 2 n_del + 2 n_ins entries. */
int oracle_apply_batch(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w,
                       const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins, int64_t* offs_out,
                       uint32_t* cols_out, uint32_t* w_out, uint32_t* del_w_out) {
  // directed batch entries (src, dst, weight, index in the batch, is deletion)
  struct Upd {
    u32 s, d, w;
    u64 k;
    bool del;
  };
  std::vector<Upd> ups;
  ups.reserve(2 * (n_del + n_ins));
  for (u64 k = 0; k < n_del + n_ins; ++k) {
    bool is_del = k < n_del;
    u32 u = is_del ? del[2 * k] : ins[3 * (k - n_del)];
    u32 v = is_del ? del[2 * k + 1] : ins[3 * (k - n_del) + 1];
    u32 ww = is_del ? 0 : ins[3 * (k - n_del) + 2];
    if (u >= n || v >= n || u == v) return ORACLE_EINVAL;
    if (!is_del && ww == 0) return ORACLE_EINVAL;
    ups.push_back({u, v, ww, k, is_del});
    ups.push_back({v, u, ww, k, is_del});
  }
  std::sort(ups.begin(), ups.end(), [](const Upd& a, const Upd& b) { return a.s != b.s ? a.s < b.s : a.d < b.d; });
  for (size_t x = 1; x < ups.size(); ++x)
    if (ups[x].s == ups[x - 1].s && ups[x].d == ups[x - 1].d) return ORACLE_EINVAL;  // pair twice in the batch
  // validate against G^{t-1}: deletions present, insertions absent
  for (const Upd& u : ups) {
    const uint32_t* b = cols + offs[u.s];
    const uint32_t* e = cols + offs[u.s + 1];
    const uint32_t* p = std::lower_bound(b, e, u.d);
    bool present = p != e && *p == u.d;
    if (u.del != present) return ORACLE_EINVAL;
    if (u.del && del_w_out && u.s < u.d) del_w_out[u.k] = w[p - cols];
  }
  // rebuild each row as a set: old entries minus deletions plus insertions
  size_t x = 0;
  i64 out = 0;
  offs_out[0] = 0;
  for (u32 i = 0; i < n; ++i) {
    std::map<u32, u32> row;
    for (i64 e = offs[i]; e < offs[i + 1]; ++e) row[cols[e]] = w[e];
    for (; x < ups.size() && ups[x].s == i; ++x) {
      if (ups[x].del)
        row.erase(ups[x].d);
      else
        row[ups[x].d] = ups[x].w;
    }
    for (const auto& kv : row) {
      cols_out[out] = kv.first;
      w_out[out] = kv.second;
      ++out;
    }
    offs_out[i + 1] = out;
  }
  return ORACLE_OK;
}

}  // extern "C"

namespace {

/* Front-end of ND / DS / DF Leiden (Alg. 1, 2, 3 before their call of
 * leiden): Alg. 11 updateWeights and updateChanges, Alg. 5 markCommunities
 * and the vertex marking functions of the chosen mode. */
struct Prepared {
  std::vector<u32> Cp;
  std::vector<i64> K, S, dSig;
  std::vector<u8> dS, dR;
  Marking F;
};

int prepare_update(const Graph& G, const uint32_t* del, uint64_t n_del, const uint32_t* ins, uint64_t n_ins,
                   const uint32_t* C_prev, const int64_t* K_prev, const int64_t* S_prev, const int64_t* dS_prev,
                   int32_t mode, const oracle_opts& o, Prepared& P) {
  u32 n = G.n;
  if (mode < 0 || mode > 2) return ORACLE_EINVAL;
  for (u32 i = 0; i < n; ++i)
    if (C_prev[i] >= n) return ORACLE_EINVAL;
  P.Cp.assign(C_prev, C_prev + n);
  const std::vector<u32>& Cp = P.Cp;
  // both directed entries of every undirected update
  std::vector<Entry> dels, inss;
  for (u64 k = 0; k < n_del; ++k) {
    u32 u = del[3 * k], v = del[3 * k + 1];
    i64 ww = del[3 * k + 2];
    dels.push_back({u, v, ww});
    dels.push_back({v, u, ww});
  }
  for (u64 k = 0; k < n_ins; ++k) {
    u32 u = ins[3 * k], v = ins[3 * k + 1];
    i64 ww = ins[3 * k + 2];
    inss.push_back({u, v, ww});
    inss.push_back({v, u, ww});
  }
  // Alg. 11 updateWeights: K^t and Sigma^t from the previous values and the batch
  P.K.assign(K_prev, K_prev + n);
  P.S.assign(S_prev, S_prev + n);
  std::vector<i64>& K = P.K;
  std::vector<i64>& S = P.S;
  for (const Entry& x : dels) {
    K[x.i] -= x.w;
    S[Cp[x.i]] -= x.w;
  }
  for (const Entry& x : inss) {
    K[x.i] += x.w;
    S[Cp[x.i]] += x.w;
  }
  // Alg. 11 updateChanges: deletions and insertions both add to DeltaSigma
  P.dSig.assign(dS_prev, dS_prev + n);
  std::vector<i64>& dSig = P.dSig;
  for (const Entry& x : dels) dSig[Cp[x.i]] += x.w;
  for (const Entry& x : inss) dSig[Cp[x.i]] += x.w;
  // Alg. 5 markCommunities (dynamic branch)
  P.dS.assign(n, 0);
  P.dR.assign(n, 0);
  for (const Entry& x : dels)
    if (Cp[x.i] == Cp[x.j]) P.dS[Cp[x.i]] = 1;
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<Entry>& list = pass == 0 ? dels : inss;
    for (const Entry& x : list) {
      u32 c = Cp[x.i];
      if (c != Cp[x.j]) continue;
      // DeltaSigma[c] / Sigma[c] > num / den, compared exactly
      if ((u128)(u64)dSig[c] * o.tau_re_den > (u128)(u64)std::max<i64>(S[c], 0) * o.tau_re_num) P.dR[c] = 1;
    }
  }
  for (u32 c = 0; c < n; ++c)
    if (P.dR[c]) dSig[c] = 0;  // a community marked for refinement restarts its cumulative change
  // Vertex marking functions F (Alg. 1, 2, 3)
  Marking& F = P.F;
  i64 M2 = 0;
  for (i64 x : K) M2 += x;
  if (mode == 0) {
    F.affected.assign(n, 1);
    F.range_all = true;
  } else if (mode == 2) {
    std::vector<u8> dV(n, 0);
    for (const Entry& x : dels)
      if (Cp[x.i] == Cp[x.j]) dV[x.i] = 1;
    for (const Entry& x : inss)
      if (Cp[x.i] != Cp[x.j]) dV[x.i] = 1;
    F.affected = dV;
    F.range_all = true;
  } else {
    std::vector<u8> dV(n, 0), dE(n, 0), dC(n, 0);
    for (const Entry& x : dels)
      if (Cp[x.i] == Cp[x.j]) {
        dV[x.i] = 1;
        dE[x.i] = 1;
        dC[Cp[x.j]] = 1;
      }
    // insertions grouped by source vertex
    std::map<u32, std::vector<std::pair<u32, i64>>> by_src;
    for (const Entry& x : inss) by_src[x.i].push_back({x.j, x.w});
    if (M2 > 0) {
      Consts k = make_consts(M2);
      Table H(n);
      for (const auto& kv : by_src) {
        u32 i = kv.first;
        for (const auto& jw : kv.second)
          if (Cp[i] != Cp[jw.first]) H.add(Cp[jw.first], jw.second);
        if (H.keys.empty()) continue;  // only intra-community insertions: ignored
        // best community: Eq. 2 with K_{i->c} = H[c], K_{i->d} = 0
        u32 d = Cp[i];
        Choice best;
        for (u32 c : H.keys) {
          double dq = delta_modularity(H.val[c], 0, K[i], S[c], S[d], k);
          if (!best.found || dq > best.dq || (dq == best.dq && c < best.c)) {
            best.found = true;
            best.c = c;
            best.dq = dq;
          }
        }
        H.clear();
        dV[i] = 1;
        dE[i] = 1;
        dC[best.c] = 1;
      }
    }
    for (u32 i = 0; i < n; ++i) {
      if (dE[i])
        for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) dV[G.cols[e]] = 1;
      if (dC[Cp[i]]) dV[i] = 1;
    }
    F.affected = dV;
    F.in_range = dV;
    F.range_all = false;
  }
  return ORACLE_OK;
}

}  // namespace

extern "C" {

/* The update front-end alone: K^t, Sigma^t (by C^{t-1}), DeltaSigma^t after
 * the refinement resets, the split / refine community flags and the
 * affected / in-range vertex flags. */
int oracle_prepare(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w, const uint32_t* del,
                   uint64_t n_del, const uint32_t* ins, uint64_t n_ins, const uint32_t* C_prev,
                   const int64_t* K_prev, const int64_t* S_prev, const int64_t* dS_prev, int32_t mode,
                   const oracle_opts* opts, int64_t* K_out, int64_t* S_out, int64_t* dS_out, uint8_t* split_out,
                   uint8_t* refine_out, uint8_t* affected_out, uint8_t* in_range_out) {
  oracle_opts o = opts ? *opts : default_opts();
  Graph G = graph_from(n, offs, cols, w);
  Prepared P;
  int rc = prepare_update(G, del, n_del, ins, n_ins, C_prev, K_prev, S_prev, dS_prev, mode, o, P);
  if (rc != ORACLE_OK) return rc;
  std::memcpy(K_out, P.K.data(), sizeof(int64_t) * n);
  std::memcpy(S_out, P.S.data(), sizeof(int64_t) * n);
  std::memcpy(dS_out, P.dSig.data(), sizeof(int64_t) * n);
  std::memcpy(split_out, P.dS.data(), n);
  std::memcpy(refine_out, P.dR.data(), n);
  std::memcpy(affected_out, P.F.affected.data(), n);
  for (u32 i = 0; i < n; ++i) in_range_out[i] = P.F.range_all ? 1 : P.F.in_range[i];
  return ORACLE_OK;
}

/* ND / DS / DF Leiden (Alg. 1, 2, 3) on the updated graph G^t.
 * del: n_del undirected (u, v, w) with w the weight the edge had in G^{t-1};
 * ins: n_ins undirected (u, v, w).  Both are expanded to the two directed
 * entries of each pair.  State in: C^{t-1}, K^{t-1}, Sigma^{t-1},
 * DeltaSigma^{t-1}; state out: C^t (tracked labels), K^t, Sigma^t (recomputed
 * from C^t), DeltaSigma^t (kept for labels that continue an old community,
 * zero elsewhere).  mode: 0 = ND, 1 = DS, 2 = DF. */
int oracle_update(uint32_t n, const int64_t* offs, const uint32_t* cols, const uint32_t* w, const uint32_t* del,
                  uint64_t n_del, const uint32_t* ins, uint64_t n_ins, const uint32_t* C_prev,
                  const int64_t* K_prev, const int64_t* S_prev, const int64_t* dS_prev, int32_t mode,
                  const oracle_opts* opts, uint32_t* C_out, int64_t* K_out, int64_t* S_out, int64_t* dS_out,
                  double* q_out, oracle_stats* st) {
  oracle_opts o = opts ? *opts : default_opts();
  if (st) std::memset(st, 0, sizeof(*st));
  Graph G = graph_from(n, offs, cols, w);
  Prepared P;
  int rc = prepare_update(G, del, n_del, ins, n_ins, C_prev, K_prev, S_prev, dS_prev, mode, o, P);
  if (rc != ORACLE_OK) return rc;
  if (st) {
    for (u32 c = 0; c < n; ++c) st->refine_marked += P.dR[c];
    for (u32 i = 0; i < n; ++i) st->affected += P.F.affected[i];
  }
  std::vector<u32> C = leiden(G, P.Cp, P.K, P.S, P.dS, P.dR, P.F, true, o, st);
  // Alg. 12: keep community IDs across snapshots
  std::vector<u8> matched;
  std::vector<u32> Ct = track(C, P.Cp, P.K, &matched);
  std::vector<i64> St(n, 0);
  for (u32 i = 0; i < n; ++i) St[Ct[i]] += P.K[i];
  std::memcpy(C_out, Ct.data(), sizeof(uint32_t) * n);
  if (K_out) std::memcpy(K_out, P.K.data(), sizeof(int64_t) * n);
  if (S_out) std::memcpy(S_out, St.data(), sizeof(int64_t) * n);
  if (dS_out)
    for (u32 c = 0; c < n; ++c) dS_out[c] = matched[c] ? P.dSig[c] : 0;
  if (q_out) *q_out = modularity_value(modularity_parts(G, Ct));
  return ORACLE_OK;
}

/* Alg. 10 alone (for tests): relabels C in place and moves Sigma and the
 * split / refine flags with the labels. */
void oracle_subset_renumber(uint32_t n, uint32_t* C, int64_t* S, uint8_t* split, uint8_t* refine_flags) {
  Level L;
  L.G.n = n;
  L.C.assign(C, C + n);
  L.S.assign(S, S + n);
  L.size.assign(n, 0);
  for (u32 i = 0; i < n; ++i) L.size[C[i]]++;
  L.dS.assign(split, split + n);
  L.dR.assign(refine_flags, refine_flags + n);
  subset_renumber(L);
  std::memcpy(C, L.C.data(), sizeof(uint32_t) * n);
  std::memcpy(S, L.S.data(), sizeof(int64_t) * n);
  std::memcpy(split, L.dS.data(), n);
  std::memcpy(refine_flags, L.dR.data(), n);
}

/* Alg. 12 alone (for tests). */
void oracle_track(uint32_t n, const uint32_t* C_cur, const uint32_t* C_prev, const int64_t* K, uint32_t* out) {
  std::vector<u32> cc(C_cur, C_cur + n), cp(C_prev, C_prev + n);
  std::vector<i64> kk(K, K + n);
  std::vector<u32> r = track(cc, cp, kk, nullptr);
  std::memcpy(out, r.data(), sizeof(uint32_t) * n);
}

uint32_t oracle_move_class(uint32_t v, uint32_t t, uint32_t P) { return move_class(v, t, P); }
uint32_t oracle_refine_colour(uint32_t v, uint32_t R) { return refine_colour(v, R); }

}  // extern "C"
