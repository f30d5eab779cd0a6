#!/usr/bin/env python3
"""Benchmark of the MI355X Leiden path on one GPU.

Workload (the 4M-vertex R-MAT configuration): R-MAT with 2^22 vertices and
2^26 samples, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), self-loops and
duplicates removed, seeded vertex permutation, unit weights.  After a static
run, a stream of Dynamic Frontier (DF) updates of 1e-3 |E| undirected updates
each (80% insertions of absent pairs, 20% deletions of existing edges).

A step is one DF-Leiden update through the C-ABI with its batch already in
HBM: batch validation and merge into the device CSR, the auxiliary-state
update, community and vertex marking, every pass of local moving, splitting,
refinement and aggregation, and tracking.  value = |E^t| / step time
(directed entries of the updated graph per second, the paper's "runtime on
the entire updated graph").  Modularity is computed once outside the timed
steps.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s static & DF-Leiden update (1 GPU, % HBM roofline); p50/p99 update latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(scale, frac, reps, seed):
    """The oracle (single-threaded CPU, pinned to one core) on a bounded
    sample: R-MAT at `scale` with the same recipe, its own static run
    (untimed), then `reps` DF updates of frac*|E| timed around the algorithm
    only.  (On the 2^22 graph itself the oracle's own static run, which the
    DF updates start from, takes minutes of CPU time: beyond the sample's
    budget, so a smaller graph of the same recipe stands in.)"""
    import numpy as np

    import oracle
    from paper_2410_15451_amd import inputs
    pinned = False
    try:
        os.sched_setaffinity(0, {min(os.sched_getaffinity(0))})
        pinned = True
    except (AttributeError, OSError):
        pass
    g = inputs.rmat(scale, seed=seed)
    C0, _, _ = oracle.static(g)
    st = oracle.initial_state(g, C0)
    keys = g.undirected_keys()
    batches = inputs.random_batch_stream(g.n, keys, inputs.batch_size_for(g.nnz, frac), reps, seed=seed + 1000)
    edges = 0
    tsum = 0.0
    cur_keys = keys
    for dels, ins in batches:
        cur_keys = inputs.keys_after_batch(cur_keys, dels, ins)
        gt = inputs.csr_from_undirected(g.n, cur_keys >> np.uint64(32), cur_keys & np.uint64(0xFFFFFFFF))
        dw = np.concatenate([dels, np.ones((dels.shape[0], 1), np.uint32)], 1)
        t = time.perf_counter()
        _, st, _, _ = oracle.update(gt, dw, ins, st, "df")
        tsum += time.perf_counter() - t
        edges += gt.nnz
    return {"value": edges / tsum, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "R-MAT scale %d (same recipe, |E|=%d), %d DF updates of %g|E| after an untimed oracle static "
                      "run; single-threaded C++ oracle%s, %.1f s timed; not the 2^22 graph: the oracle's static run "
                      "there, which the updates start from, takes minutes" % (
                          scale, g.nnz, reps, frac, " pinned to one core" if pinned else "", tsum),
            "host": host_info()}


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = 0
    try:
        mem = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 2**30
    except (ValueError, OSError):
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count(), "ram_gib": round(mem, 1)}


def kernel_source_digest():
    """Digest of the library sources: a stored counter reading is only
    reported while it still describes the same code."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2410_15451_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(scope, workload, field):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor)
    from the committed rocprofv3 counter summary: per launch of a kernel or
    per step of a whole call (`scope`), or None when there is none for the
    current library source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    r = rec.get(scope, {}).get(workload)
    if not r or r.get("source_digest") != kernel_source_digest():
        return None
    return r.get(field)


def call_roofline(stats, ms, scope, workload):
    """Whole-call roofline: the algorithmic bytes the library counts on the
    device (work counters times their bytes per unit) over the call time."""
    algo = sum(s["algo_bytes"] for s in stats) / len(stats)
    achieved = algo / (ms * 1e-3) / 1e9
    work = {k: sum(s["work"][k] for s in stats) / len(stats) for k in stats[0]["work"]}
    for k in ("moves", "sweep_vertices", "batch_entries"):
        work[k] = sum(s[k] for s in stats) / len(stats)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": stored_traffic(scope, workload, "hbm_bytes_per_step"),
            "scope": scope, "algo_bytes_per_call": algo, "ms_per_call": ms, "work_per_call": work}


def run_forest(args, binding, inputs):
    """Batched form: args.graphs kNN-style graphs (vertex counts log-uniform in
    1e3..2e5, 15 near neighbours in a 16-d point cloud, weights 1..100), made on
    the GPU and held as forests of at most args.forest_entries entries, each a
    single block-diagonal handle whose every phase is one launch for all its
    graphs.  Static Leiden on every forest, then one DF update of 1e-3 |E_q|
    per graph.  A sample runs one graph per handle (the same library, one
    graph at a time) for the speedup and identical memberships (the oracle
    check of the same graphs is a GPU test)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    sizes = inputs.forest_sizes(args.graphs, 1000, 200000, seed=inputs.BASE_SEED + 4)
    chunks, cur, est = [], [], 0
    for q, nq in enumerate(sizes):
        if cur and est + 25 * int(nq) > args.forest_entries:
            chunks.append(cur)
            cur, est = [], 0
        cur.append(q)
        est += 25 * int(nq)
    chunks.append(cur)
    rng = np.random.default_rng(inputs.BASE_SEED + 8)
    ssample = set(int(x) for x in rng.choice(args.graphs, min(args.single_sample, args.graphs), replace=False))
    keep = ssample
    host = {}
    tot = {"entries": 0, "entries_after": 0, "static_s": 0.0, "update_s": 0.0, "gen_s": 0.0, "updates": 0}
    tunes = []
    log("forest: %d graphs, %d vertices, %d forests" % (args.graphs, int(sizes.sum()), len(chunks)))
    for c, qs in enumerate(chunks):
        t0 = time.time()
        sz = sizes[qs]
        offs, cols, w = inputs.knn_forest_torch(sz, dev, seed=inputs.BASE_SEED + 5 + qs[0],
                                                progress=lambda k: log("forest %d: %d graphs made" % (c, k)))
        first = np.concatenate([[0], np.cumsum(sz.astype(np.int64))])
        dels, ins = inputs.forest_batch_torch(offs, cols, first, args.frac, seed=inputs.BASE_SEED + 600 + c)
        torch.cuda.synchronize()
        F = binding.Forest(sz, offs, cols, w)
        nnz = int(cols.numel())
        dh, ih = dels.cpu().numpy().astype(np.int64), ins.cpu().numpy().astype(np.int64)
        for k, q in enumerate(qs):
            if q in keep:
                g = inputs.forest_graph(offs, cols, w, first, k)
                md = (dh[:, 0] >= first[k]) & (dh[:, 0] < first[k + 1])
                mi = (ih[:, 0] >= first[k]) & (ih[:, 0] < first[k + 1])
                d = (dh[md] - first[k]).astype(np.uint32)
                i = ih[mi].copy()
                i[:, :2] -= first[k]
                host[q] = {"g": g, "d": d, "i": i.astype(np.uint32)}
        del offs, cols, w
        torch.cuda.empty_cache()
        tot["gen_s"] += time.time() - t0
        tune = F.autotune()  # degree-bin thresholds and the aggregation's emit table for this forest
        F.static(compute_modularity=0)  # warm-up: workspace
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r0 = F.static(compute_modularity=0)
        tb = time.perf_counter()
        empty2, empty3 = np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32)
        F.update(empty2, empty3, mode="df", compute_modularity=0)  # warm-up: batch buffers
        torch.cuda.synchronize()
        tc = time.perf_counter()
        r1 = F.update(dels, ins, mode="df", compute_modularity=0)
        td = time.perf_counter()
        qF = F.modularity(r1.membership)
        C0, C1 = r0.membership, r1.membership
        for k, q in enumerate(qs):
            if q in keep:
                host[q]["C0"] = C0[first[k]:first[k + 1]].copy()
                host[q]["C1"] = C1[first[k]:first[k + 1]].copy()
                host[q]["q1"] = float(qF[k])
        tot["entries"] += nnz
        tot["entries_after"] += F.nnz
        tot["updates"] += int(dels.shape[0] + ins.shape[0])
        tot["static_s"] += tb - ta
        tot["update_s"] += td - tc
        _, fpasses, _ = F.results()
        st = r1.stats
        log("forest %d: %d graphs, %d entries, static %.1f ms, update %.1f ms (%d updates; device %.1f ms, batch %.1f ms, "
            "passes %d (graphs with more than one: %d), iters %s, affected %d, moves %d, scanned %d)"
            % (c, len(qs), nnz, (tb - ta) * 1e3, (td - tc) * 1e3, dels.shape[0] + ins.shape[0], st["ms_total"], st["ms_batch"],
               st["passes"], int((fpasses > 1).sum()), st["iters"], st["affected"], st["moves"],
               st["edges_scanned"]))
        log("forest %d: update work %s, subrounds %s; tuning %s" % (c, st["work"], st["subrounds"], tune))
        tunes.append(tune)
        F.close()
        del dels, ins
        torch.cuda.empty_cache()
    # the same library one graph per handle, on a sample
    s_static = s_update = 0.0
    s_entries = 0
    same = True
    for q in sorted(ssample):
        h = host[q]
        G = binding.Graph.from_csr(h["g"])
        G.static(compute_modularity=0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r0 = G.static(compute_modularity=0)
        tb = time.perf_counter()
        G.update(np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32), mode="df", compute_modularity=0)
        tc = time.perf_counter()
        r1 = G.update(h["d"], h["i"], mode="df", compute_modularity=0)
        td = time.perf_counter()
        s_static += tb - ta
        s_update += td - tc
        s_entries += h["g"].nnz
        same &= bool(np.array_equal(r0.membership, h["C0"]) and np.array_equal(r1.membership, h["C1"]))
        G.close()
    log("one graph at a time: %d graphs, static %.1f ms, update %.1f ms" % (len(ssample), s_static * 1e3,
                                                                            s_update * 1e3))
    forest_rate = tot["entries_after"] / tot["update_s"]
    single_rate = s_entries / s_update if s_update > 0 else float("nan")
    return {"metric": "edges/s, DF-Leiden update of every graph of a kNN forest (1 GPU)",
            "value": forest_rate, "unit": "edges/s", "n_gpus": 1, "higher_is_better": True,
            "data": "synthetic", "dtype": "int64+f64", "vs_baseline": None,
            "config": {"workload": "knn_forest_%d" % args.graphs, "graphs": args.graphs,
                       "vertices": int(sizes.sum()), "entries": tot["entries"], "n_range": [1000, 200000],
                       "forests": len(chunks), "max_forest_entries": args.forest_entries,
                       "update_frac": args.frac, "mode": "df", "deterministic": True},
            "static_edges_per_s": tot["entries"] / tot["static_s"], "static_s": tot["static_s"],
            "update_s": tot["update_s"], "batch_undirected_updates": tot["updates"],
            "generate_s": tot["gen_s"],
            "one_graph_at_a_time": {"graphs": len(ssample), "entries": s_entries, "static_s": s_static,
                                    "update_s": s_update,
                                    "static_edges_per_s": s_entries / s_static if s_static > 0 else None,
                                    "update_edges_per_s": single_rate},
            "speedup_update_vs_one_at_a_time": forest_rate / single_rate,
            "speedup_static_vs_one_at_a_time": (tot["entries"] / tot["static_s"]) / (s_entries / s_static),
            "identical_memberships_sample": bool(same), "autotuned": tunes}


def run_stability(args, binding, inputs):
    """Stability experiment of Section 4.1: from the static result on G^0,
    delete a random batch (G^1), then insert the same edges back (G^2 = G^0),
    updating the communities each time; report the share of vertices whose
    community ID on G^2 equals the one of the static run on G^0, for batch
    sizes 1e-7 .. 1e-1 |E| and the three dynamic modes (tracking keeps IDs)."""
    import numpy as np
    g = inputs.rmat(args.scale, seed=inputs.BASE_SEED + 2)
    keys = g.undirected_keys()
    G = binding.Graph.from_csr(g)
    C0 = G.static().membership.copy()
    st0 = G.state()
    out = {}
    for mode in ("nd", "ds", "df"):
        row = {}
        for k, f in enumerate((1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1)):
            nb = max(1, inputs.batch_size_for(g.nnz, f))
            dels, _ = inputs.random_batch(g.n, keys, nb, seed=1300 + k, ins_frac=0.0)
            ins = np.concatenate([dels, np.ones((dels.shape[0], 1), np.uint32)], axis=1)
            G.set_state(*st0)
            t = time.perf_counter()
            G.update(dels, np.zeros((0, 3), np.uint32), mode=mode)
            r = G.update(np.zeros((0, 2), np.uint32), ins, mode=mode)
            dt = time.perf_counter() - t
            row["%g" % f] = {"match": float(np.mean(r.membership == C0)), "two_updates_ms": dt * 1e3}
            log("stability %s f=%g match %.3f" % (mode, f, row["%g" % f]["match"]))
        out[mode] = row
    G.close()
    return {"metric": "stability: share of vertices keeping their static community ID after delete + re-insert",
            "value": out["df"]["%g" % 1e-3]["match"], "unit": "fraction", "n_gpus": 1, "higher_is_better": True,
            "data": "synthetic", "dtype": "int64+f64",
            "config": {"workload": "rmat%d_stability" % args.scale, "n": g.n, "nnz": g.nnz,
                       "value_is": "df at 1e-3 |E|"},
            "match_by_mode_and_fraction": out,
            "paper_context": "the paper reports DF Leiden with tracking keeping 84% to 44% for 1e-7 to 0.1 |E|"}


def chunglu_modularity(offs, cols, w, C, n):
    """Eq. 1 of membership C recomputed with torch on the device, rows taken
    in chunks (an independent check of the library's value)."""
    import torch
    C = C.to(torch.int64)
    deg = offs[1:] - offs[:-1]
    K = torch.zeros(n, dtype=torch.int64, device=offs.device)
    intra = 0
    step = 1 << 22
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        a, b = int(offs[r0]), int(offs[r1])
        src = torch.repeat_interleave(torch.arange(r0, r1, device=offs.device), deg[r0:r1])
        ww = w[a:b].to(torch.int64)
        K[r0:r1] = torch.zeros(r1 - r0, dtype=torch.int64, device=offs.device).index_add_(0, src - r0, ww)
        same = C[src] == C[cols[a:b].to(torch.int64)]
        intra += int(ww[same].sum())
    S = torch.zeros(n, dtype=torch.int64, device=offs.device).index_add_(0, C, K)
    m2 = int(K.sum())
    ssq = float((S.to(torch.float64) ** 2).sum())
    return intra / m2 - ssq / float(m2) ** 2


def run_chunglu(args, binding, inputs):
    """The large single graph: a Chung-Lu graph (exponent 2.1, largest
    expected degree 10^6, mean degree 40, weights 1..16) of --cl-vertices
    vertices made on the device; static Leiden, then DF Leiden over batch
    sizes 1e-7 .. 1e-1 |E| (80% insertions / 20% deletions), each size once
    in the deterministic and once in the asynchronous mode, on the evolving
    graph.  Reports time and modularity per (fraction, mode); the static
    result's modularity is checked against a recomputation with torch."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    n = args.cl_vertices
    t0 = time.time()
    offs, cols, w = inputs.chung_lu_torch(n, inputs.BASE_SEED + 60, dev)
    torch.cuda.synchronize()
    nnz = cols.numel()
    maxdeg = int((offs[1:] - offs[:-1]).max())
    log("chung-lu: n=%d nnz=%d maxdeg=%d (%.1f s)" % (n, nnz, maxdeg, time.time() - t0))
    # the update pool first, while the library holds no memory yet
    fracs = (1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1)
    E = nnz // 2
    sizes = [max(1, int(round(f * E))) for f in fracs]
    n_ins = [int(round(0.8 * b)) for b in sizes]
    n_del = [b - i for b, i in zip(sizes, n_ins)]
    t = time.time()
    dels, ins = inputs.update_pool_torch(offs, cols, 2 * sum(n_del), 2 * sum(n_ins), inputs.BASE_SEED + 61,
                                         w_range=(1, 16))
    log("update pool: %d deletions, %d insertions (%.1f s)" % (dels.shape[0], ins.shape[0], time.time() - t))
    torch.cuda.empty_cache()
    G = binding.Graph(offs, cols, w)
    out = torch.zeros(n, dtype=torch.int32, device=dev)
    G.static(out=out)  # the first run also allocates the workspace
    torch.cuda.synchronize()
    t = time.perf_counter()
    rs = G.static(out=out)
    torch.cuda.synchronize()
    t_static = time.perf_counter() - t
    log("static: %.1f ms, passes %d, q=%.6f" % (t_static * 1e3, rs.stats["passes"], rs.q))
    q_check = chunglu_modularity(offs, cols, w, out, n)
    log("static modularity recomputed with torch: %.9f (library %.9f)" % (q_check, rs.q))
    assert int(out.min()) >= 0 and int(out.max()) < n
    assert abs(q_check - rs.q) < 1e-9, (q_check, rs.q)
    del offs, cols, w
    torch.cuda.empty_cache()
    pd = pi = 0
    rows = {}
    for f, nd, ni in zip(fracs, n_del, n_ins):
        for mode, det in (("deterministic", 1), ("asynchronous", 0)):
            d = torch.from_numpy(dels[pd:pd + nd].view(np.int32)).to(dev)
            i = torch.from_numpy(ins[pi:pi + ni].view(np.int32)).to(dev)
            pd += nd
            pi += ni
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = G.update(d, i, mode="df", out=out, deterministic=det)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            rows.setdefault("%g" % f, {})[mode] = {"ms": dt * 1e3, "q": r.q, "passes": r.stats["passes"],
                                                  "affected": r.stats["affected"], "updates": nd + ni}
            log("df %s f=%g (%d updates): %.1f ms, q=%.6f, affected %d" % (mode, f, nd + ni, dt * 1e3, r.q,
                                                                        r.stats["affected"]))
            del d, i
    G.close()
    return {"metric": "large single graph: DF Leiden update time over batch sizes", "value": rows["0.001"]["deterministic"]["ms"],
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int64+f64",
            "config": {"workload": "chunglu_df_sweep", "n": n, "nnz": nnz, "max_degree": maxdeg, "gamma": 2.1,
                       "weights": "1..16", "value_is": "deterministic DF update at 1e-3 |E|"},
            "static_ms": t_static * 1e3, "static_q": rs.q, "static_q_torch": q_check, "by_fraction": rows}


def run_temporal(args, binding, inputs):
    """Temporal replay (the paper's real-world dynamic experiment with a
    synthetic stream): 90% of the edges preloaded, static Leiden, then 100
    consecutive insertion batches of B = f |E_T| edges with DF Leiden (the
    cumulative DeltaSigma carries across batches); B for f in 1e-5, 1e-4,
    1e-3.  Reports time per batch and the final modularity beside a static
    run on the final graph."""
    import numpy as np
    g0, stream = inputs.temporal_stream(args.scale)
    ET = g0.nnz // 2 + stream.shape[0]
    out = {}
    for f in (1e-5, 1e-4, 1e-3):
        B = max(1, int(round(f * ET)))
        nb = min(100, stream.shape[0] // B)
        G = binding.Graph.from_csr(g0)
        G.static()
        empty = np.zeros((0, 2), np.uint32)
        ts = []
        for k in range(nb):
            t = time.perf_counter()
            r = G.update(empty, stream[k * B:(k + 1) * B], mode="df")
            ts.append(time.perf_counter() - t)
        q_dyn = r.q
        q_static = G.static().q
        out["%g" % f] = {"batch_edges": B, "batches": nb, "ms_per_batch": 1e3 * float(np.mean(ts)),
                         "p99_ms": 1e3 * percentile(ts, 99), "q_df": q_dyn, "q_static_final": q_static}
        log("temporal f=%g: B=%d, %.2f ms/batch, q %.5f vs static %.5f" % (f, B, out["%g" % f]["ms_per_batch"],
                                                                        q_dyn, q_static))
        G.close()
    return {"metric": "temporal replay: DF Leiden time per insertion batch", "value": out["%g" % 1e-4]["ms_per_batch"],
            "unit": "ms/batch", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int64+f64",
            "config": {"workload": "rmat%d_temporal" % args.scale, "n": g0.n, "edges_total": ET,
                       "preload": 0.9, "value_is": "f = 1e-4"},
            "by_fraction": out}


def run_ablation(args, binding, inputs):
    """Refinement and split ablations of Sections 4.2 and 4.3: the same DF
    update stream replayed from one static result with the refinement
    threshold tau_re = 0.1 .. 0.9, and with every community that is not
    refined split (split-all) instead of only the marked ones; reports the
    mean update time and the final modularity of each setting."""
    import numpy as np
    g = inputs.rmat(args.scale, seed=inputs.BASE_SEED + 2)
    nb = inputs.batch_size_for(g.nnz, args.frac)
    nbat = 10
    batches = inputs.random_batch_stream(g.n, g.undirected_keys(), nb, nbat, seed=inputs.BASE_SEED + 2 + 2000)
    settings = [("tau_re=%d/10" % k, {"tau_re": (k, 10)}) for k in range(1, 10)]
    settings.append(("split_all (tau_re=6/10)", {"split_all": 1}))
    out = {}
    for name, kw in settings:
        G = binding.Graph.from_csr(g)  # the same graph and static result for every setting
        G.static()
        ts = []
        for d, i in batches:
            t = time.perf_counter()
            r = G.update(d, i, mode="df", **kw)
            ts.append(time.perf_counter() - t)
        out[name] = {"ms_per_update": 1e3 * float(np.mean(ts)), "q_final": r.q}
        log("ablation %s: %.2f ms/update, q %.5f" % (name, out[name]["ms_per_update"], r.q))
        G.close()
    return {"metric": "ablation: DF update time and final modularity per refinement / split setting",
            "value": out["tau_re=6/10"]["ms_per_update"], "unit": "ms/update", "n_gpus": 1,
            "higher_is_better": False, "data": "synthetic", "dtype": "int64+f64",
            "config": {"workload": "rmat%d_ablation" % args.scale, "n": g.n, "nnz": g.nnz,
                       "batch_undirected_updates": nb, "updates": nbat, "value_is": "tau_re = 0.6"},
            "by_setting": out}


def run_serving(args, binding, inputs):
    """Serving form: tenant R-MAT graphs (by default scales 20, 20, 21, 21, 22,
    22, 23, 23; edge factor 16; unit weights; made on the GPU) in a server with
    args.streams workers.  Admission: a budget that holds seven of the eight
    estimated footprints refuses the eighth; the measured server admits all.
    Requests: target graph uniform, B = round(exp(U[ln 1e2, ln 1e6]))
    undirected updates (80% insertions of absent pairs, 20% deletions of
    existing edges, consecutive slices of per-tenant pools, so every request
    is valid in its graph's order), DF update each.  Capacity = 1 / the mean
    service time of back-to-back requests; then Poisson arrivals at each of
    args.loads times the capacity.  Latency = completion - arrival, service =
    completion - start; updated edges/s = undirected updates over first
    arrival to last completion."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    scales = [int(x) for x in args.tenant_scales.split(",")]
    loads = [float(x) for x in args.loads.split(",")]
    nreq = args.requests
    nwarm = args.warm_requests
    rng = np.random.default_rng(inputs.BASE_SEED + 6)
    total = nwarm + nreq * len(loads)
    targets = rng.integers(0, len(scales), total)
    bsz = np.round(np.exp(rng.uniform(np.log(1e2), np.log(1e6), total))).astype(np.int64)
    n_del = np.round(0.2 * bsz).astype(np.int64)
    n_ins = bsz - n_del
    t0 = time.time()
    tenants = []
    for k, sc in enumerate(scales):
        offs, cols, w = inputs.rmat_torch(sc, inputs.BASE_SEED + 50 + k, dev)
        mine = targets == k
        d, i = inputs.update_pool_torch(offs, cols, int(n_del[mine].sum()), int(n_ins[mine].sum()),
                                        seed=inputs.BASE_SEED + 60 + k)
        torch.cuda.synchronize()
        tenants.append({"n": offs.numel() - 1, "offs": offs, "cols": cols, "w": w, "dels": d, "ins": i, "d0": 0,
                        "i0": 0})
        log("serving: tenant %d (scale %d): %d entries, pools %d / %d" % (k, sc, cols.numel(), d.shape[0],
                                                                          i.shape[0]))
    log("serving: tenants made in %.1f s" % (time.time() - t0))
    reqs = []
    for r in range(total):
        t = tenants[int(targets[r])]
        d = t["dels"][t["d0"]:t["d0"] + int(n_del[r])]
        i = t["ins"][t["i0"]:t["i0"] + int(n_ins[r])]
        t["d0"] += d.shape[0]
        t["i0"] += i.shape[0]
        reqs.append((int(targets[r]), d, i))
    # admission: a budget that holds the seven smallest footprints refuses the largest
    est = [binding.server_footprint(t["n"], int(t["cols"].numel()), 0.2) for t in tenants]
    order = np.argsort(est)
    budget7 = int(sum(est[j] for j in order[:7]) + (64 << 20))
    srvA = binding.Server(hbm_budget_bytes=budget7, workers=args.streams)
    admitted, refused = 0, 0
    for j in order:
        t = tenants[j]
        try:
            srvA.add_graph_device(t["n"], t["offs"], t["cols"], t["w"])
            admitted += 1
        except binding.LeidenError:
            refused += 1
    srvA.close()
    del srvA
    srv = binding.Server(hbm_budget_bytes=int(sum(est) + (1 << 30)), workers=args.streams)
    ids = [srv.add_graph_device(t["n"], t["offs"], t["cols"], t["w"]) for t in tenants]
    for t in tenants:
        del t["offs"], t["cols"], t["w"]
    torch.cuda.empty_cache()
    # warm-up and single-stream capacity: back-to-back requests
    svc0 = []
    for r in range(nwarm):
        tg, d, i = reqs[r]
        _, la, sv = srv.wait(srv.submit(ids[tg], d, i, mode="df"))
        svc0.append(sv)
    mean_svc = float(np.mean(svc0[len(svc0) // 5:]))
    capacity = 1e3 / mean_svc
    log("serving: %d warm-up requests, mean service %.2f ms, capacity %.1f req/s" % (nwarm, mean_svc, capacity))
    res = []
    base = nwarm
    for load in loads:
        lam = load * capacity
        gaps = rng.exponential(1.0 / lam, nreq)
        tickets = []
        start = time.perf_counter()
        due = start
        for k in range(nreq):
            due += gaps[k]
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            tg, d, i = reqs[base + k]
            tickets.append(srv.submit(ids[tg], d, i, mode="df"))
            if (k + 1) % 100 == 0:
                log("serving: load %.1f: %d requests submitted" % (load, k + 1))
        lat, svc = [], []
        for k, tk in enumerate(tickets):
            _, la, sv = srv.wait(tk)
            lat.append(la)
            svc.append(sv)
            if (k + 1) % 100 == 0:
                log("serving: load %.1f: %d requests done" % (load, k + 1))
        wall = time.perf_counter() - start
        upd = int(sum(reqs[base + k][1].shape[0] + reqs[base + k][2].shape[0] for k in range(nreq)))
        res.append({"load": load, "offered_req_per_s": lam, "requests": nreq,
                    "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
                    "service_ms": {"p50": percentile(svc, 50), "p99": percentile(svc, 99)},
                    "updated_edges_per_s": upd / wall})
        log("serving: load %.1f: latency p50 %.2f p99 %.2f ms, service p50 %.2f p99 %.2f ms, %.3g updated edges/s"
            % (load, res[-1]["latency_ms"]["p50"], res[-1]["latency_ms"]["p99"], res[-1]["service_ms"]["p50"],
               res[-1]["service_ms"]["p99"], res[-1]["updated_edges_per_s"]))
        base += nreq
    st = srv.stats()
    srv.close()
    top = res[-1]
    return {"metric": "serving: p50/p99 update latency and sustained updated edges/s (1 GPU)",
            "value": top["updated_edges_per_s"], "unit": "updated_edges/s", "n_gpus": 1, "higher_is_better": True,
            "data": "synthetic", "dtype": "int64+f64", "vs_baseline": None,
            "config": {"workload": "rmat_tenants_serving", "scales": scales, "edge_factor": 16,
                       "warm_up_requests": nwarm, "requests_per_load": nreq, "loads": loads,
                       "batch_sizes": "round(exp(U[ln 1e2, ln 1e6])) undirected updates, 80/20",
                       "workers": args.streams, "mode": "df", "deterministic": True},
            "latency_ms": top["latency_ms"], "service_ms": top["service_ms"], "per_load": res,
            "single_stream_capacity_req_per_s": capacity, "mean_service_ms_back_to_back": mean_svc,
            "admission": {"budget_bytes": budget7, "admitted": admitted, "refused": refused,
                          "estimates_bytes": est},
            "completed": st["completed"], "failed": st["failed"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--frac", type=float, default=1e-3)
    ap.add_argument("--mode", default="df", choices=["nd", "ds", "df"])
    ap.add_argument("--context-steps", type=int, default=3, help="ND / DS / static steps for the ratio context")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-scale", type=int, default=20)
    ap.add_argument("--cpu-reps", type=int, default=24)
    ap.add_argument("--timed-kernel", default="agg_big", help="kernel timed with HIP events for the roofline")
    ap.add_argument("--workload", default="rmat",
                    choices=["rmat", "forest", "serving", "stability", "temporal", "ablation", "chunglu"],
                    help="rmat: the 4M-vertex R-MAT DF stream (default); forest: 4,096 kNN graphs as "
                         "block-diagonal forests; "
                         "serving: tenant R-MAT graphs under a Poisson stream of update requests; chunglu: the "
                         "large single Chung-Lu graph, DF over batch sizes 1e-7..1e-1 |E|")
    ap.add_argument("--graphs", type=int, default=4096, help="forest: number of kNN graphs")
    ap.add_argument("--forest-entries", type=float, default=1.2e9, help="forest: most entries of one forest")
    ap.add_argument("--single-sample", type=int, default=128, help="forest: graphs also run one at a time")
    ap.add_argument("--streams", type=int, default=4, help="serving: worker streams")
    ap.add_argument("--requests", type=int, default=500, help="serving: measured requests per load")
    ap.add_argument("--warm-requests", type=int, default=50, help="serving: back-to-back warm-up requests")
    ap.add_argument("--loads", default="0.3,0.5,0.7,0.9", help="serving: offered loads (fractions of capacity)")
    ap.add_argument("--tenant-scales", default="20,20,21,21,22,22,23,23", help="serving: R-MAT scales of the tenants")
    ap.add_argument("--cl-vertices", type=int, default=50_000_000, help="chunglu: vertices of the large graph")
    ap.add_argument("--marker", type=int, default=0,
                    help="launch a spin kernel right before and after the timed static run and the timed "
                         "update steps (profile windows 0 and 1)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (reference for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_15451_amd import binding, inputs
    if args.workload == "forest":
        print(json.dumps(run_forest(args, binding, inputs)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args, binding, inputs)), flush=True)
        return
    if args.workload == "stability":
        print(json.dumps(run_stability(args, binding, inputs)), flush=True)
        return
    if args.workload == "temporal":
        print(json.dumps(run_temporal(args, binding, inputs)), flush=True)
        return
    if args.workload == "ablation":
        print(json.dumps(run_ablation(args, binding, inputs)), flush=True)
        return
    if args.workload == "chunglu":
        print(json.dumps(run_chunglu(args, binding, inputs)), flush=True)
        return
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    if args.calib_copy_mib:
        x = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB" % args.calib_copy_mib)
        del x, y

    t0 = time.time()
    g = inputs.rmat(args.scale, seed=inputs.BASE_SEED + 2)
    log("graph: n=%d nnz=%d maxdeg=%d (%.1f s)" % (g.n, g.nnz, int(g.degrees().max()), time.time() - t0))
    nb = inputs.batch_size_for(g.nnz, args.frac)
    ctx = args.context_steps
    total_batches = args.warmup + args.steps + 3 * ctx
    batches = inputs.random_batch_stream(g.n, g.undirected_keys(), nb, total_batches,
                                         seed=inputs.BASE_SEED + 2 + 1000)
    dev_batches = [(torch.from_numpy(d.view(np.int32)).to(dev), torch.from_numpy(i.view(np.int32)).to(dev))
                   for d, i in batches]
    G = binding.Graph.from_csr(g)
    out = torch.zeros(g.n, dtype=torch.int32, device=dev)
    opts = dict(stream=sp, compute_modularity=0)

    # static Leiden (twice: the first run also allocates the workspace)
    G.static(out=out, **opts)
    torch.cuda.synchronize()
    if args.marker:
        torch.cuda._sleep(1000)
    t = time.perf_counter()
    rs = G.static(out=out, **opts)
    torch.cuda.synchronize()
    t_static = time.perf_counter() - t
    if args.marker:
        torch.cuda._sleep(1000)
        torch.cuda.synchronize()
    q_static = G.modularity(out)
    log("static: %.2f ms, passes %d, iters %s, q=%.5f" % (t_static * 1e3, rs.stats["passes"], rs.stats["iters"],
                                                          q_static))
    bi = 0

    def run_update(mode, **kw):
        nonlocal bi
        d, i = dev_batches[bi]
        bi += 1
        ta = time.perf_counter()
        r = G.update(d, i, mode=mode, out=out, **opts, **kw)
        return time.perf_counter() - ta, r

    for _ in range(args.warmup):
        run_update(args.mode)
    torch.cuda.synchronize()
    lat, edges, stats = [], 0, []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if args.marker:
        torch.cuda._sleep(1000)
    ev0.record(stream)
    tw = time.perf_counter()
    for k in range(args.steps):
        dt, r = run_update(args.mode, timed_kernel=args.timed_kernel)
        lat.append(dt)
        edges += r.stats["nnz"]
        stats.append(r.stats)
        if args.marker and (k + 1) % 5 == 0:  # progress under a profiler (slow, serialised dispatches)
            log("step %d done" % (k + 1))
    ev1.record(stream)
    if args.marker:
        torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw
    dev_ms = ev0.elapsed_time(ev1)
    T = max(wall, dev_ms / 1e3)
    value = edges / T
    q_dyn = G.modularity(out)
    log("%s: %d steps, %.3f ms/step, p50 %.3f ms, p99 %.3f ms, q=%.5f" % (
        args.mode, args.steps, T / args.steps * 1e3, percentile(lat, 50) * 1e3, percentile(lat, 99) * 1e3, q_dyn))

    # context: ND / DS updates and a static recompute on the evolving graph
    context = {}
    for mode in [m for m in ("nd", "ds") if m != args.mode and ctx]:
        ts = [run_update(mode)[0] for _ in range(ctx)]
        context[mode + "_ms"] = 1e3 * sum(ts) / len(ts)
    if ctx:
        # the asynchronous mode on the same stream (not reproducible, faster)
        ts = [run_update(args.mode, deterministic=0)[0] for _ in range(ctx)]
        context["async_" + args.mode + "_ms"] = 1e3 * sum(ts) / len(ts)
    ts = []
    for _ in range(ctx):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        G.static(out=out, **opts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - ta)
    context["static_ms"] = 1e3 * sum(ts) / len(ts) if ts else t_static * 1e3
    context[args.mode + "_ms"] = T / args.steps * 1e3
    for m in ("nd", "ds", "df"):
        if m + "_ms" in context:
            context["speedup_%s_vs_static" % m] = context["static_ms"] / context[m + "_ms"]
    context["paper_speedup_vs_static_64core_epyc"] = {"nd": 3.9, "ds": 4.4, "df": 6.1}

    mean = {k: sum(s[k] for s in stats) / len(stats) for k in ("ms_total", "ms_batch", "edges_scanned", "moves",
                                                                 "affected", "passes")}
    workload = "rmat%d_%s_update_%g" % (args.scale, args.mode, args.frac)
    # whole-call rooflines (the DF update step and the static run): device
    # work counters times their algorithmic bytes, over the measured time
    roof = call_roofline(stats, T / args.steps * 1e3, "update", workload)
    roof_static = call_roofline([rs.stats], t_static * 1e3, "static", "rmat%d_static" % args.scale)
    # a single kernel inside the step, timed with HIP events on its stream:
    # algorithmic bytes per launch over its average launch time
    launches = sum(s["kt_launches"] for s in stats)
    kt_ms = sum(s["kt_ms"] for s in stats)
    kt_bytes = sum(s["kt_bytes"] for s in stats)
    kname = binding.kernel_name(args.timed_kernel)
    kroof = None
    if launches and kt_ms > 0:
        achieved = kt_bytes / (kt_ms * 1e-3) / 1e9
        kroof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(kname, workload, "hbm_bytes_per_launch"),
                 "kernel": kname, "launches": launches, "avg_launch_ms": kt_ms / launches,
                 "bytes_per_launch": kt_bytes / launches,
                 "units_per_launch": sum(s["kt_units"] for s in stats) / launches,
                 "share_of_step": kt_ms / (T * 1e3)}
    line = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": T / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": workload, "n": g.n, "nnz": g.nnz,
                   "batch_undirected_updates": nb, "mode": args.mode, "deterministic": True},
        "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
        "static_edges_per_s": g.nnz / t_static, "static_ms": t_static * 1e3,
        "batch_edges_per_s": 2 * nb * args.steps / T,
        "modularity": {"static": q_static, "after_updates": q_dyn},
        "step_stats_mean": mean, "context": context, "roofline": roof, "roofline_static": roof_static,
        "roofline_kernel": kroof,
    }
    if args.cpu_baseline:
        t = time.time()
        line["cpu_baseline"] = cpu_baseline(args.cpu_scale, args.frac, args.cpu_reps, inputs.BASE_SEED + 2)
        log("cpu baseline: %.3g edges/s (%.1f s)" % (line["cpu_baseline"]["value"], time.time() - t))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
