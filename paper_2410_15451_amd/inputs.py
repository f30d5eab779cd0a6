"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module builds graphs and edge-update batches only.  It contains none of the
community-detection method: no modularity, no local moving, no refinement, no
aggregation.  Both the HIP path and the CPU oracle receive exactly the arrays made
here, so the two sides never disagree about their inputs.

Graph format (host, numpy):
  ``Csr(n, offs, cols, w)`` - an undirected graph stored with both directions of
  every edge (the paper's convention of adding reverse edges, Section 5.1.4),
  ``offs`` int64[n+1], ``cols`` uint32[nnz] sorted inside each row, ``w`` uint32[nnz]
  with w > 0, no duplicate entries.

Batch format: deletions ``uint32[nd, 2]`` (each undirected pair once) and insertions
``uint32[ni, 3]`` as (u, v, w) (each undirected pair once, w > 0), following the
batch update definition of Section 3.5 (deletions are existing edges, insertions
are absent pairs, no vertex is added or removed).

Workload recipes (the paper's SuiteSparse and SNAP graphs are not available; these
stand in for them):
  * planted partition: n vertices in equal blocks, each pair is an edge with
    probability p_in (same block) or p_out (different blocks), unit weights;
  * R-MAT: 2^scale vertices, edge_factor * 2^scale samples with quadrant
    probabilities (a, b, c, d), self-loops and duplicates dropped, a seeded vertex
    permutation, unit weights;
  * Chung-Lu power law (stands in for the paper's largest graphs): expected
    degrees W (i + i0)^(-1/(gamma - 1)) with the largest one and the mean
    fixed, endpoint pairs drawn proportionally to them, self-loops and
    duplicates dropped, weights uniform in 1..16, a seeded permutation;
  * random batch (Section 5.1.4): a fraction of |E| undirected updates, 80%
    insertions of uniform absent pairs and 20% deletions of uniform existing edges;
  * kNN-style graphs for the batched form: points from a 16-d standard normal,
    quantised to integers so distances are exact on every machine; buckets by
    the sign pattern of ceil(log2(n / 512)) random projections; in each bucket
    the 32 nearest points of every point, of which 15 chosen uniformly become
    its neighbours; symmetrised by union; weight
    clamp(1 + floor(100 exp(-d^2 / D)), 1, 100) with D the median neighbour d^2;
    many such graphs with vertex counts log-uniform in a range;
  * kNN-style forests at full size (4,096 graphs of 10^3..2*10^5 vertices) are
    made on the device by ``knn_forest_torch`` with the same point and weight
    recipe, except that the 32 candidates of a point are the nearest among the
    64 points around it in the order of (bucket, a random projection) rather
    than among its whole bucket, and the weight is 1 + floor(99 D / (D + d^2))
    (integer arithmetic);
  * Chung-Lu at full size (the large single graph: 5*10^7 vertices, about
    2*10^9 entries) is made on the device by ``chung_lu_torch`` with the same
    recipe (endpoint pairs drawn in chunks);
  * serving tenants: R-MAT graphs by the recipe above made on the device by
    ``rmat_torch`` (torch random streams), and per tenant one pool of distinct
    edges to delete and distinct absent pairs to insert whose prefixes make
    a valid stream of batches;
  * temporal stream (stands in for the SNAP temporal graphs of the paper's
    real-world experiment): the distinct undirected edges of an R-MAT graph in
    a seeded random arrival order; the first 90% form the initial graph and
    the rest arrive as consecutive insertion batches.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASE_SEED = 2410154510


@dataclass
class Csr:
    n: int
    offs: np.ndarray  # int64[n+1]
    cols: np.ndarray  # uint32[nnz]
    w: np.ndarray  # uint32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.cols.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offs)

    def undirected_keys(self) -> np.ndarray:
        """Sorted uint64 keys u*2^32+v of the undirected edges with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.uint64), np.diff(self.offs))
        dst = self.cols.astype(np.uint64)
        m = src < dst
        return np.sort((src[m] << np.uint64(32)) | dst[m])


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def csr_from_undirected(n: int, u, v, w=None) -> Csr:
    """Build the symmetric CSR of an undirected edge list (each pair given once).

    Pairs must be distinct and free of self-loops; rows come out sorted.
    """
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    if w is None:
        w = np.ones(u.shape[0], dtype=np.uint32)
    w = np.asarray(w, dtype=np.uint32)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    key = (src << np.uint64(32)) | dst
    order = np.argsort(key, kind="stable")
    src = src[order]
    dst = dst[order].astype(np.uint32)
    ww = ww[order]
    counts = np.bincount(src.astype(np.int64), minlength=n) if n > 0 else np.zeros(0, np.int64)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    return Csr(n, offs, dst, ww)


def csr_from_edges(n: int, edges) -> Csr:
    """Small helper for hand-written test graphs: ``edges`` is [(u, v)] or [(u, v, w)]."""
    if len(edges) == 0:
        return Csr(n, np.zeros(n + 1, np.int64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    arr = np.asarray(edges, dtype=np.int64)
    u, v = arr[:, 0], arr[:, 1]
    w = arr[:, 2] if arr.shape[1] > 2 else np.ones(len(arr), np.int64)
    return csr_from_undirected(n, u, v, w)


def planted_partition(n: int = 1000, blocks: int = 10, p_in: float = 0.1, p_out: float = 0.005,
                      seed: int = BASE_SEED + 1) -> Csr:
    """Planted-partition graph: block(v) = floor(v / (n / blocks))."""
    rng = rng_for(seed)
    iu, ju = np.triu_indices(n, k=1)
    bs = n // blocks
    same = (iu // bs) == (ju // bs)
    p = np.where(same, p_in, p_out)
    keep = rng.random(iu.shape[0]) < p
    return csr_from_undirected(n, iu[keep], ju[keep])


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = BASE_SEED + 2, permute: bool = True) -> Csr:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale samples.

    Each sample picks one quadrant per level with probabilities (a, b, c, 1-a-b-c);
    self-loops and duplicate pairs are dropped, the result is symmetrised and the
    vertex IDs are shuffled by a seeded permutation; unit weights.
    """
    rng = rng_for(seed)
    n = 1 << scale
    m = edge_factor * n
    src = np.zeros(m, dtype=np.uint32)
    dst = np.zeros(m, dtype=np.uint32)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        r = rng.random(m, dtype=np.float32)
        bit = np.uint32(1 << (scale - 1 - lvl))
        sb = r >= ab
        db = ((r >= a) & (r < ab)) | (r >= abc)
        src |= sb.astype(np.uint32) * bit
        dst |= db.astype(np.uint32) * bit
        del r, sb, db
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo = np.minimum(src, dst).astype(np.uint64)
    hi = np.maximum(src, dst).astype(np.uint64)
    del src, dst, keep
    key = np.unique((lo << np.uint64(32)) | hi)
    del lo, hi
    u = (key >> np.uint64(32)).astype(np.uint32)
    v = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    del key
    if permute:
        perm = rng.permutation(n).astype(np.uint32)
        u, v = perm[u], perm[v]
    return csr_from_undirected(n, u, v)


def chung_lu_weights(n: int, avg_degree: float, max_degree: float, gamma: float = 2.1):
    """Expected degrees w_i = W (i + i0)^(-1/(gamma-1)), i = 0..n-1, with W and
    i0 chosen so that w_0 = max_degree and the sum of w is avg_degree * n (the
    sum taken as the integral of the power law over [i0, n + i0], solved by
    bisection on i0)."""
    a = 1.0 / (gamma - 1.0)
    target = float(avg_degree) * n

    def total(i0):
        W = max_degree * i0 ** a
        if abs(1.0 - a) < 1e-12:
            return W * (np.log(n + i0) - np.log(i0))
        return W * ((n + i0) ** (1.0 - a) - i0 ** (1.0 - a)) / (1.0 - a)

    lo, hi = 1e-9, 1e12
    for _ in range(200):  # total(i0) grows with i0
        mid = np.sqrt(lo * hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    i0 = np.sqrt(lo * hi)
    W = max_degree * i0 ** a
    return W * (np.arange(n, dtype=np.float64) + i0) ** (-a)


def chung_lu(n: int, avg_degree: float = 40.0, max_degree: float = 1e6, gamma: float = 2.1, wmax: int = 16,
             seed: int = BASE_SEED + 3) -> Csr:
    """Power-law graph of the Chung-Lu model: avg_degree * n / 2 endpoint pairs,
    each endpoint drawn with probability proportional to its expected degree
    (chung_lu_weights); self-loops and repeated pairs dropped, so the largest
    degrees end somewhat below max_degree; weights uniform in 1..wmax per
    undirected edge; a seeded vertex permutation."""
    rng = rng_for(seed)
    w = chung_lu_weights(n, avg_degree, max_degree, gamma)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(avg_degree * n / 2))
    u = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1).astype(np.uint64)
    v = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1).astype(np.uint64)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.unique((np.minimum(u, v) << np.uint64(32)) | np.maximum(u, v))
    del u, v, keep
    ww = rng.integers(1, wmax + 1, size=key.shape[0], dtype=np.int64).astype(np.uint32)
    perm = rng.permutation(n).astype(np.uint32)
    a = perm[(key >> np.uint64(32)).astype(np.int64)]
    b = perm[(key & np.uint64(0xFFFFFFFF)).astype(np.int64)]
    return csr_from_undirected(n, a, b, ww)


def random_batch(n: int, existing_keys: np.ndarray, n_updates: int, seed: int,
                 ins_frac: float = 0.8, w_range=(1, 1)):
    """Random batch update of ``n_updates`` undirected updates (Section 5.1.4).

    ``existing_keys`` are the sorted u*2^32+v keys (u < v) of the current graph.
    Returns (deletions uint32[nd,2], insertions uint32[ni,3]); deletions are distinct
    existing edges, insertions are distinct absent pairs without self-loops.
    """
    rng = rng_for(seed)
    n_ins = int(round(n_updates * ins_frac))
    n_del = int(n_updates) - n_ins
    n_del = min(n_del, existing_keys.shape[0])
    if n_del > 0:
        pick = rng.choice(existing_keys.shape[0], size=n_del, replace=False)
        dk = existing_keys[np.sort(pick)]
    else:
        dk = np.zeros(0, np.uint64)
    dels = np.stack([(dk >> np.uint64(32)).astype(np.uint32),
                     (dk & np.uint64(0xFFFFFFFF)).astype(np.uint32)], axis=1)
    got = np.zeros(0, np.uint64)
    max_pairs = n * (n - 1) // 2 - existing_keys.shape[0]
    n_ins = min(n_ins, max_pairs)
    while got.shape[0] < n_ins:
        want = (n_ins - got.shape[0]) * 2 + 16
        u = rng.integers(0, n, size=want, dtype=np.uint64)
        v = rng.integers(0, n, size=want, dtype=np.uint64)
        ok = u != v
        u, v = u[ok], v[ok]
        k = (np.minimum(u, v) << np.uint64(32)) | np.maximum(u, v)
        # keep the first occurrence of each new key, in draw order
        _, first = np.unique(k, return_index=True)
        k = k[np.sort(first)]
        pos = np.searchsorted(existing_keys, k)
        pos = np.minimum(pos, max(existing_keys.shape[0] - 1, 0))
        present = existing_keys[pos] == k if existing_keys.shape[0] else np.zeros(k.shape, bool)
        k = k[~present]
        k = k[~np.isin(k, got)]
        got = np.concatenate([got, k])[:n_ins]
    lo, hi = w_range
    ww = rng.integers(lo, hi + 1, size=got.shape[0], dtype=np.int64).astype(np.uint32)
    ins = np.stack([(got >> np.uint64(32)).astype(np.uint32),
                    (got & np.uint64(0xFFFFFFFF)).astype(np.uint32), ww], axis=1)
    return dels.astype(np.uint32).reshape(-1, 2), ins.astype(np.uint32).reshape(-1, 3)


def random_batch_stream(n: int, existing_keys: np.ndarray, n_updates: int, count: int, seed: int,
                        ins_frac: float = 0.8, w_range=(1, 1)):
    """``count`` consecutive batches of ``n_updates`` each, valid when applied in order.

    All deletions are distinct edges of the starting graph and all insertions
    distinct pairs absent from it, so no batch touches a pair an earlier batch
    changed.  Returns a list of (deletions, insertions)."""
    dels, ins = random_batch(n, existing_keys, n_updates * count, seed, ins_frac, w_range)
    rng = rng_for(seed + 7)
    dels = dels[rng.permutation(dels.shape[0])]
    ins = ins[rng.permutation(ins.shape[0])]
    nd, ni = dels.shape[0] // count, ins.shape[0] // count
    return [(dels[k * nd:(k + 1) * nd], ins[k * ni:(k + 1) * ni]) for k in range(count)]


def keys_after_batch(existing_keys: np.ndarray, dels: np.ndarray, ins: np.ndarray) -> np.ndarray:
    """Edge-key bookkeeping for generating a stream of batches (sorted result)."""
    dk = (np.minimum(dels[:, 0], dels[:, 1]).astype(np.uint64) << np.uint64(32)) | \
        np.maximum(dels[:, 0], dels[:, 1]).astype(np.uint64)
    ik = (np.minimum(ins[:, 0], ins[:, 1]).astype(np.uint64) << np.uint64(32)) | \
        np.maximum(ins[:, 0], ins[:, 1]).astype(np.uint64)
    keep = ~np.isin(existing_keys, dk, assume_unique=True)
    return np.sort(np.concatenate([existing_keys[keep], ik]))


def batch_size_for(nnz_directed: int, frac: float) -> int:
    """Number of undirected updates for a batch of ``frac * |E|`` (|E| counts directed entries)."""
    return max(1, int(round(frac * nnz_directed)))


def knn_graph(n: int, k: int = 15, dim: int = 16, cand: int = 32, seed: int = BASE_SEED + 4) -> Csr:
    """kNN-style graph on n random points (recipe in the module docstring)."""
    rng = rng_for(seed)
    X = np.round(rng.standard_normal((n, dim)) * 256.0).astype(np.int64)
    nproj = max(0, int(np.ceil(np.log2(max(n, 1) / 512.0))))
    if nproj:
        R = rng.standard_normal((dim, nproj))
        bits = (X.astype(np.float64) @ R) > 0
        bucket = (bits * (1 << np.arange(nproj))).sum(axis=1)
    else:
        bucket = np.zeros(n, np.int64)
    order = np.argsort(bucket, kind="stable")
    starts = np.searchsorted(bucket[order], np.arange((1 << nproj) + 1))
    us, vs, ds = [], [], []
    for b in range(1 << nproj):
        idx = order[starts[b]:starts[b + 1]]
        m = idx.shape[0]
        if m < 2:
            continue
        P = X[idx]
        sq = (P * P).sum(axis=1)
        D2 = sq[:, None] + sq[None, :] - 2 * (P @ P.T)  # exact in int64
        np.fill_diagonal(D2, np.iinfo(np.int64).max // (m + 1))  # never among the nearest; no overflow below
        c = min(cand, m - 1)
        # the c nearest of each point, ties to the lower index
        key = D2 * m + np.arange(m)[None, :]
        near = np.argpartition(key, c - 1, axis=1)[:, :c] if c < m else np.argsort(key, axis=1)[:, :c]
        pick = min(k, c)
        sel = np.argsort(rng.random((m, c)), axis=1)[:, :pick]
        nb = np.take_along_axis(near, sel, axis=1)
        us.append(np.repeat(idx, pick))
        vs.append(idx[nb.reshape(-1)])
        ds.append(np.take_along_axis(D2, nb, axis=1).reshape(-1))
    if not us:
        return csr_from_undirected(n, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    u = np.concatenate(us).astype(np.int64)
    v = np.concatenate(vs).astype(np.int64)
    d2 = np.concatenate(ds)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = lo * n + hi
    key, first = np.unique(key, return_index=True)  # union of both directions
    d2 = d2[first]
    Dm = float(np.median(d2)) if d2.shape[0] else 1.0
    w = np.clip(1 + np.floor(100.0 * np.exp(-d2.astype(np.float64) / max(Dm, 1.0))), 1, 100).astype(np.uint32)
    return csr_from_undirected(n, (key // n).astype(np.uint32), (key % n).astype(np.uint32), w)


def knn_forest(count: int, n_min: int = 1000, n_max: int = 200000, seed: int = BASE_SEED + 4):
    """``count`` kNN-style graphs with vertex counts log-uniform in [n_min, n_max]."""
    rng = rng_for(seed)
    ns = np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), count))).astype(np.int64)
    return [knn_graph(int(x), seed=seed + 1 + i) for i, x in enumerate(ns)]


def knn_graph_torch(n: int, seed: int, device, k: int = 15, dim: int = 16, cand: int = 32, window: int = 32):
    """kNN-style graph made with torch on ``device`` (recipe in the module
    docstring); returns (offs int64[n+1], cols int32[nnz], w int32[nnz]) tensors
    on the device (int32 holds the uint32 values of this size range)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    X = torch.round(torch.randn((n, dim), generator=g, device=device, dtype=f64) * 256.0)
    nproj = max(0, int(np.ceil(np.log2(max(n, 1) / 512.0))))
    R = torch.randn((dim, nproj + 1), generator=g, device=device, dtype=f64)
    P = X @ R
    bucket = torch.zeros(n, dtype=torch.int64, device=device)
    for b in range(nproj):
        bucket |= (P[:, b] > 0).to(torch.int64) << b
    # order by bucket, then by the last projection inside the bucket
    proj_rank = torch.argsort(P[:, nproj], stable=True)
    order = proj_rank[torch.argsort(bucket[proj_rank], stable=True)]
    bs = bucket[order]
    offs_w = torch.cat([torch.arange(-window, 0, device=device), torch.arange(1, window + 1, device=device)])
    pos = torch.arange(n, device=device)
    jpos = pos[:, None] + offs_w[None, :]
    ok = (jpos >= 0) & (jpos < n)
    jpos = jpos.clamp(0, max(n - 1, 0))
    ok &= bs[jpos] == bs[:, None]
    i_id = order
    j_id = order[jpos]
    d2 = ((X[i_id][:, None, :] - X[j_id]) ** 2).sum(dim=2)  # exact: integer values below 2^53
    big = float(2 ** 52)
    key = torch.where(ok, d2 * (2 * window) + torch.arange(2 * window, device=device, dtype=f64)[None, :], big)
    c = min(cand, 2 * window)
    near = torch.topk(key, c, dim=1, largest=False).indices
    near_ok = torch.gather(key, 1, near) < big
    pick = min(k, c)
    rnd = torch.rand((n, c), generator=g, device=device, dtype=f64)
    rnd = torch.where(near_ok, rnd, 2.0)
    sel = torch.topk(rnd, pick, dim=1, largest=False).indices
    nb = torch.gather(near, 1, sel)
    valid = torch.gather(near_ok, 1, sel)
    u = i_id[:, None].expand(-1, pick)[valid]
    v = torch.gather(j_id, 1, nb)[valid]
    dd = torch.gather(d2, 1, nb)[valid].to(torch.int64)
    lo, hi = torch.minimum(u, v), torch.maximum(u, v)
    ekey = lo * n + hi
    ekey, perm = torch.sort(ekey, stable=True)
    dd = dd[perm]
    first = torch.ones_like(ekey, dtype=torch.bool)
    if ekey.numel() > 1:
        first[1:] = ekey[1:] != ekey[:-1]
    ekey, dd = ekey[first], dd[first]
    D = int(torch.median(dd).item()) if dd.numel() else 1
    D = max(D, 1)
    w = 1 + (99 * D) // (D + dd)
    lo, hi = ekey // n, ekey % n
    src = torch.cat([lo, hi])
    dst = torch.cat([hi, lo])
    ww = torch.cat([w, w])
    o2 = torch.argsort(src * n + dst)
    src, dst, ww = src[o2], dst[o2], ww[o2]
    offs = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offs[1:] = torch.cumsum(torch.bincount(src, minlength=n), 0)
    return offs, dst.to(torch.int32), ww.to(torch.int32)


def rmat_torch(scale: int, seed: int, device, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19):
    """R-MAT graph by the recipe of ``rmat`` made with torch on ``device``
    (its own random streams, so not the same graph as ``rmat`` with the same
    seed); returns (offs int64[n+1], cols int32[nnz], w int32[nnz]) tensors."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = 1 << scale
    m = edge_factor * n
    src = torch.zeros(m, dtype=torch.int64, device=device)
    dst = torch.zeros(m, dtype=torch.int64, device=device)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        r = torch.rand(m, generator=g, device=device)
        bit = 1 << (scale - 1 - lvl)
        src |= (r >= ab).to(torch.int64) * bit
        dst |= (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64) * bit
        del r
    keep = src != dst
    lo = torch.minimum(src, dst)[keep]
    hi = torch.maximum(src, dst)[keep]
    del src, dst, keep
    key = torch.unique(lo * n + hi)
    del lo, hi
    perm = torch.randperm(n, generator=g, device=device)
    u, v = perm[key // n], perm[key % n]
    del key
    s2 = torch.cat([u, v])
    d2 = torch.cat([v, u])
    del u, v
    order = torch.argsort(s2 * n + d2)
    s2, d2 = s2[order], d2[order]
    offs = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offs[1:] = torch.cumsum(torch.bincount(s2, minlength=n), 0)
    return offs, d2.to(torch.int32), torch.ones_like(d2, dtype=torch.int32)


def chung_lu_torch(n: int, seed: int, device, avg_degree: float = 40.0, max_degree: float = 1e6,
                   gamma: float = 2.1, wmax: int = 16, chunk: int = 1 << 26):
    """Chung-Lu graph by the recipe of ``chung_lu`` made with torch on
    ``device`` (its own random streams, so not the same graph as
    ``chung_lu`` with the same seed): round(avg_degree * n / 2) endpoint
    pairs drawn in chunks, self-loops and repeated pairs dropped, weights
    uniform in 1..wmax per undirected edge, a seeded vertex permutation.
    The endpoint distribution and the permutation are made on the host (a
    floating-point prefix sum on the device need not repeat bit for bit from
    one process to the next), so the same seed gives the same graph in every
    process.
    Returns (offs int64[n+1], cols int32[nnz], w int32[nnz]) tensors."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cdf_h = np.cumsum(chung_lu_weights(n, avg_degree, max_degree, gamma))
    cdf_h /= cdf_h[-1]
    cdf = torch.from_numpy(cdf_h).to(device)
    del cdf_h
    m = int(round(avg_degree * n / 2))
    keys = []
    for a in range(0, m, chunk):
        c = min(chunk, m - a)
        u = torch.searchsorted(cdf, torch.rand(c, generator=g, device=device, dtype=torch.float64), right=True)
        v = torch.searchsorted(cdf, torch.rand(c, generator=g, device=device, dtype=torch.float64), right=True)
        u.clamp_(max=n - 1)
        v.clamp_(max=n - 1)
        keep = u != v
        lo, hi = torch.minimum(u, v)[keep], torch.maximum(u, v)[keep]
        del u, v, keep
        keys.append(torch.unique(lo * n + hi))
        del lo, hi
    del cdf
    key = torch.unique(torch.cat(keys))
    del keys
    ww = torch.randint(1, wmax + 1, (key.numel(),), generator=g, device=device, dtype=torch.int32)
    perm = torch.from_numpy(np.random.default_rng(int(seed)).permutation(n)).to(device)
    a, b = perm[key // n], perm[key % n]
    del key, perm
    # both directions, sorted by (row, column)
    rk = torch.cat([a * n + b, b * n + a])
    del a, b
    ww = torch.cat([ww, ww])
    rk, order = torch.sort(rk)
    ww = ww[order]
    del order
    src = rk // n
    offs = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offs[1:] = torch.cumsum(torch.bincount(src, minlength=n), 0)
    del src
    cols = (rk % n).to(torch.int32)
    del rk
    return offs, cols, ww


def update_pool_torch(offs, cols, n_del: int, n_ins: int, seed: int, w_range=(1, 1)):
    """Distinct existing edges to delete (n_del, uniform) and distinct absent
    pairs to insert (n_ins, uniform endpoints, weights uniform in w_range) for
    a graph on the device; any prefix of each, taken in order, is a valid
    stream of batches (Section 5.1.4).  Returns host numpy arrays
    (uint32[n_del, 2], uint32[n_ins, 3])."""
    import torch

    dev = offs.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    n = offs.numel() - 1
    src = torch.repeat_interleave(torch.arange(n, device=dev), offs[1:] - offs[:-1])
    dst = cols.to(torch.int64)
    up = src < dst
    u, v = src[up], dst[up]
    del src, dst, up
    keys = torch.sort(u * n + v).values
    n_del = min(n_del, keys.numel())
    pick = torch.randperm(keys.numel(), generator=g, device=dev)[:n_del]
    dk = keys[pick]
    dels = torch.stack([dk // n, dk % n], 1)
    got = []
    have = 0
    seen = torch.zeros(0, dtype=torch.int64, device=dev)
    while have < n_ins:
        want = 2 * (n_ins - have) + 16
        a = torch.randint(0, n, (want,), generator=g, device=dev)
        b = torch.randint(0, n, (want,), generator=g, device=dev)
        lo, hi = torch.minimum(a, b), torch.maximum(a, b)
        k = (lo * n + hi)[lo != hi]
        pos = torch.searchsorted(keys, k).clamp(max=max(keys.numel() - 1, 0))
        k = k[keys[pos] != k]
        ks, ko = torch.sort(k, stable=True)
        first = torch.ones_like(ks, dtype=torch.bool)
        first[1:] = ks[1:] != ks[:-1]
        k = k[torch.sort(ko[first]).values]  # first occurrences, in draw order
        if seen.numel():
            k = k[~torch.isin(k, seen)]
        k = k[:n_ins - have]
        got.append(k)
        seen = torch.cat([seen, k])
        have += k.numel()
    k = torch.cat(got) if got else torch.zeros(0, dtype=torch.int64, device=dev)
    wv = torch.randint(w_range[0], w_range[1] + 1, (k.numel(),), generator=g, device=dev)
    ins = torch.stack([k // n, k % n, wv], 1)
    return dels.cpu().numpy().astype(np.uint32), ins.cpu().numpy().astype(np.uint32)


def forest_sizes(count: int, n_min: int = 1000, n_max: int = 200000, seed: int = BASE_SEED + 4) -> np.ndarray:
    """Vertex counts log-uniform in [n_min, n_max] (uint32[count])."""
    rng = rng_for(seed)
    return np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), count))).astype(np.uint32)


def knn_forest_torch(sizes, device, seed: int = BASE_SEED + 5, progress=None):
    """The block-diagonal CSR of kNN-style graphs with the given vertex counts,
    made on ``device``: (offs int64[N+1], cols int32[nnz], w int32[nnz]) with
    graph q on vertices first_q .. first_q + sizes[q] - 1 (graph q from seed +
    q).  ``progress(q)`` is called after every 256 graphs."""
    import torch

    offs_l, cols_l, w_l = [], [], []
    vbase, ebase = 0, 0
    for q, nq in enumerate(np.asarray(sizes, np.int64)):
        o, c, w = knn_graph_torch(int(nq), seed + q, device)
        offs_l.append(o[:-1] + ebase)
        cols_l.append(c + vbase)
        w_l.append(w)
        vbase += int(nq)
        ebase += int(c.numel())
        if progress and (q + 1) % 256 == 0:
            progress(q + 1)
    offs_l.append(torch.tensor([ebase], dtype=torch.int64, device=device))
    return torch.cat(offs_l), torch.cat(cols_l), torch.cat(w_l)


def forest_batch_torch(offs, cols, first, frac: float, seed: int, ins_frac: float = 0.8, w_range=(1, 100)):
    """A random batch (Section 5.1.4) for every graph of a forest CSR on the
    device: graph q gets max(1, round(frac * |E_q|)) undirected updates,
    ins_frac of them insertions of distinct absent pairs of its own vertices
    (uniform endpoints, weights uniform in w_range) and the rest deletions of
    distinct existing edges (uniform).  Returns (deletions int32[nd, 2],
    insertions int32[ni, 3]) in forest vertex IDs on the device."""
    import torch

    dev = offs.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    first_t = torch.as_tensor(np.asarray(first, np.int64), device=dev)
    nq = first_t.numel() - 1
    N = int(first_t[-1])
    sizes = first_t[1:] - first_t[:-1]
    deg = offs[1:] - offs[:-1]
    src = torch.repeat_interleave(torch.arange(N, device=dev), deg)
    dst = cols.to(torch.int64)
    up = src < dst
    u, v = src[up], dst[up]
    del src, dst
    vg = torch.repeat_interleave(torch.arange(nq, device=dev), sizes)
    eg = vg[u]
    e_cnt = torch.bincount(eg, minlength=nq)
    nb = torch.clamp(torch.round(frac * 2 * e_cnt.to(torch.float64)), min=1).to(torch.int64)
    n_ins = torch.round(nb.to(torch.float64) * ins_frac).to(torch.int64)
    n_del = torch.minimum(nb - n_ins, e_cnt)
    # deletions: the first n_del[q] edges of graph q in a random order
    r = torch.randint(0, 1 << 40, (u.numel(),), generator=g, device=dev)
    order = torch.argsort(eg * (1 << 40) + r)
    seg0 = torch.cumsum(e_cnt, 0) - e_cnt
    rank = torch.arange(u.numel(), device=dev) - seg0[eg[order]]
    pick = order[rank < n_del[eg[order]]]
    dels = torch.stack([u[pick], v[pick]], 1)
    # insertions: candidate pairs in draw order, minus self-loops, present
    # edges and repeats; the first n_ins[q] of graph q
    ekeys = torch.sort(u * N + v).values
    del u, v, eg, order, r
    cand = 2 * n_ins + 16
    cg = torch.repeat_interleave(torch.arange(nq, device=dev), cand)
    a = first_t[cg] + (torch.rand(cg.numel(), generator=g, device=dev, dtype=torch.float64) * sizes[cg]).to(torch.int64)
    b = first_t[cg] + (torch.rand(cg.numel(), generator=g, device=dev, dtype=torch.float64) * sizes[cg]).to(torch.int64)
    a = torch.minimum(a, first_t[cg] + sizes[cg] - 1)
    b = torch.minimum(b, first_t[cg] + sizes[cg] - 1)
    lo, hi = torch.minimum(a, b), torch.maximum(a, b)
    k = lo * N + hi
    ok = lo != hi
    pos = torch.searchsorted(ekeys, k).clamp(max=max(ekeys.numel() - 1, 0))
    if ekeys.numel():
        ok &= ekeys[pos] != k
    ks, ko = torch.sort(k, stable=True)
    firstocc = torch.ones_like(ks, dtype=torch.bool)
    firstocc[1:] = ks[1:] != ks[:-1]
    keep = torch.zeros_like(ok)
    keep[ko] = firstocc
    ok &= keep
    csum = torch.cumsum(ok.to(torch.int64), 0)
    seg = torch.cumsum(cand, 0) - cand
    before = torch.where(seg > 0, csum[(seg - 1).clamp(min=0)], torch.zeros_like(seg))
    rk = csum - 1 - before[cg]
    ok &= rk < n_ins[cg]
    wv = torch.randint(w_range[0], w_range[1] + 1, (int(ok.sum()),), generator=g, device=dev)
    ins = torch.stack([lo[ok], hi[ok], wv], 1)
    return dels.to(torch.int32).contiguous(), ins.to(torch.int32).contiguous()


def forest_graph(offs, cols, w, first, q: int) -> Csr:
    """Graph q of a forest CSR (host numpy or torch arrays) as a Csr with its own vertex IDs."""
    a, b = int(first[q]), int(first[q + 1])
    o = np.asarray(offs[a:b + 1].cpu() if hasattr(offs, "cpu") else offs[a:b + 1], np.int64)
    e0, e1 = int(o[0]), int(o[-1])
    c = cols[e0:e1]
    ww = w[e0:e1]
    c = np.asarray(c.cpu() if hasattr(c, "cpu") else c).astype(np.int64) - a
    ww = np.asarray(ww.cpu() if hasattr(ww, "cpu") else ww).astype(np.uint32)
    return Csr(b - a, o - e0, c.astype(np.uint32), ww)


def forest_csr(graphs):
    """The block-diagonal forest CSR of host Csr graphs: (sizes uint32[q], Csr)."""
    sizes = np.array([g.n for g in graphs], np.uint32)
    first = np.zeros(len(graphs) + 1, np.int64)
    np.cumsum(sizes, out=first[1:])
    offs, cols, w = [np.zeros(1, np.int64)], [], []
    e = 0
    for g, f in zip(graphs, first):
        offs.append(g.offs[1:] + e)
        cols.append(g.cols.astype(np.int64) + f)
        w.append(g.w)
        e += g.nnz
    return sizes, Csr(int(first[-1]), np.concatenate(offs), np.concatenate(cols).astype(np.uint32),
                      np.concatenate(w).astype(np.uint32))


def temporal_stream(scale: int, seed: int = BASE_SEED + 7, preload: float = 0.9):
    """(initial Csr with the first `preload` share of the edges, remaining
    edges as uint32[m, 3] insertions (u, v, 1) in arrival order)."""
    g = rmat(scale, seed=seed)
    keys = g.undirected_keys()
    order = rng_for(seed + 1).permutation(keys.shape[0])
    keys = keys[order]
    k0 = int(round(preload * keys.shape[0]))
    first = np.sort(keys[:k0])
    g0 = csr_from_undirected(g.n, (first >> np.uint64(32)).astype(np.uint32),
                             (first & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    rest = keys[k0:]
    ins = np.stack([(rest >> np.uint64(32)).astype(np.uint32), (rest & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                    np.ones(rest.shape[0], np.uint32)], axis=1)
    return g0, ins
