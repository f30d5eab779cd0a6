"""Forest form: many independent graphs in one block-diagonal handle.

Every phase runs as one launch over all graphs, and every graph must still
get exactly the result it gets alone: memberships (labels inside each graph),
modularity, passes and per-pass iteration counts, in the deterministic mode,
for static runs and for ND / DS / DF updates with tracking.  A sample of
graphs is also compared with the oracle directly.
"""
import numpy as np
import pytest

from paper_2410_15451_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lm():
    from paper_2410_15451_amd import binding
    binding.lib()
    return binding


def _mixed_graphs():
    """Graphs of different shapes and sizes, including degenerate ones."""
    gs = [
        inputs.planted_partition(),
        inputs.rmat(9, seed=301),
        inputs.csr_from_edges(1, []),                       # one vertex, no edge
        inputs.knn_graph(1500, seed=302),
        inputs.csr_from_edges(2, [(0, 1, 7)]),              # one edge
        inputs.csr_from_edges(5, []),                       # no edges at all
        inputs.rmat(11, seed=303),
        inputs.planted_partition(600, 6, 0.08, 0.01, seed=304),
        inputs.chung_lu(3000, avg_degree=12, max_degree=400, seed=305),
    ]
    return gs


def _forest(lm, gs):
    sizes, F = inputs.forest_csr(gs)
    return lm.Forest(sizes, F.offs, F.cols, F.w), sizes


def _split(C, sizes):
    first = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
    return [C[first[q]:first[q + 1]] for q in range(len(sizes))]


def _check_alone(lm, Fh, gs, rF, singles):
    """The forest's per-graph results equal every graph's result alone."""
    qF, passes, iters = Fh.results()
    parts = _split(rF.membership, Fh.sizes)
    for k, (g, r) in enumerate(zip(gs, singles)):
        assert np.array_equal(parts[k], r.membership), (k, int((parts[k] != r.membership).sum()))
        assert qF[k] == r.q, (k, qF[k], r.q)
        assert passes[k] == r.stats["passes"], (k, passes[k], r.stats["passes"])
        it = [int(x) for x in iters[k]]
        assert it[:len(r.stats["iters"])] == list(r.stats["iters"]), (k, it, r.stats["iters"])
        assert not any(it[len(r.stats["iters"]):]), (k, it)
    assert np.isnan(rF.q)


def test_forest_static_equals_alone(lm, orc):
    gs = _mixed_graphs()
    Fh, sizes = _forest(lm, gs)
    rF = Fh.static()
    singles = [lm.Graph.from_csr(g).static() for g in gs]
    _check_alone(lm, Fh, gs, rF, singles)
    parts = _split(rF.membership, sizes)
    for k in (0, 3, 6, 8):
        C, q, st = orc.static(gs[k])
        assert np.array_equal(parts[k], C) and singles[k].q == q, k
    # Eq. 1 per graph through leiden_modularity
    qm = Fh.modularity(rF.membership)
    assert np.array_equal(qm, Fh.results()[0])


@pytest.mark.parametrize("mode", ["nd", "ds", "df"])
def test_forest_updates_equal_alone(lm, orc, mode):
    gs = _mixed_graphs()
    Fh, sizes = _forest(lm, gs)
    first = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
    Gs = [lm.Graph.from_csr(g) for g in gs]
    rF = Fh.static()
    for G in Gs:
        G.static()
    cur = list(gs)
    states = [orc.initial_state(g, orc.static(g)[0]) if k in (0, 6) else None for k, g in enumerate(gs)]
    for b, frac in enumerate((1e-3, 1e-2, 5e-2)):
        dels_all, ins_all, per = [], [], []
        for k, g in enumerate(cur):
            if g.nnz == 0 or g.n < 8:
                per.append((np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32)))
                continue
            nb = max(1, inputs.batch_size_for(g.nnz, frac))
            d, i = inputs.random_batch(g.n, g.undirected_keys(), nb, seed=400 + 20 * b + k, w_range=(1, 9))
            per.append((d, i))
            dels_all.append(d.astype(np.int64) + first[k])
            i2 = i.astype(np.int64)
            i2[:, :2] += first[k]
            ins_all.append(i2)
        dF = np.concatenate(dels_all).astype(np.uint32)
        iF = np.concatenate(ins_all).astype(np.uint32)
        rF = Fh.update(dF, iF, mode=mode)
        singles = [G.update(d, i, mode=mode) for G, (d, i) in zip(Gs, per)]
        _check_alone(lm, Fh, gs, rF, singles)
        parts = _split(rF.membership, sizes)
        for k in (0, 6):  # a sample against the oracle
            gt, dw = orc.apply_batch(cur[k], *per[k])
            C1, states[k], q1, _ = orc.update(gt, dw, per[k][1], states[k], mode)
            assert np.array_equal(parts[k], C1), (mode, b, k)
        cur = [orc.apply_batch(g, d, i)[0] for g, (d, i) in zip(cur, per)]


def test_forest_knn_sample_against_oracle(lm, orc):
    """A forest of kNN-style graphs made on the device (the batched workload's
    generator), static and one DF batch, checked graph by graph against the
    oracle on every fourth graph."""
    import torch
    sizes = inputs.forest_sizes(24, 1000, 20000, seed=inputs.BASE_SEED + 311)
    offs, cols, w = inputs.knn_forest_torch(sizes, "cuda", seed=inputs.BASE_SEED + 312)
    Fh = lm.Forest(sizes, offs, cols.view(torch.int32), w)
    first = Fh.first
    gs = [inputs.forest_graph(offs, cols, w, first, q) for q in range(len(sizes))]
    del offs, cols, w
    rF = Fh.static()
    parts = _split(rF.membership, sizes)
    qF, passes, _ = Fh.results()
    sample = list(range(0, len(gs), 4))
    for k in sample:
        C, q, st = orc.static(gs[k])
        assert np.array_equal(parts[k], C) and qF[k] == q and passes[k] == st["passes"], k
    # one DF batch of 1e-3 |E| per graph
    dl, il, per = [], [], []
    for k, g in enumerate(gs):
        nb = max(1, inputs.batch_size_for(g.nnz, 1e-3))
        d, i = inputs.random_batch(g.n, g.undirected_keys(), nb, seed=500 + k, w_range=(1, 100))
        per.append((d, i))
        dl.append(d.astype(np.int64) + first[k])
        i2 = i.astype(np.int64)
        i2[:, :2] += first[k]
        il.append(i2)
    rU = Fh.update(np.concatenate(dl).astype(np.uint32), np.concatenate(il).astype(np.uint32), mode="df")
    partsU = _split(rU.membership, sizes)
    qU = Fh.results()[0]
    for k in sample:
        C0 = orc.static(gs[k])[0]
        gt, dw = orc.apply_batch(gs[k], *per[k])
        C1, _, q1, _ = orc.update(gt, dw, per[k][1], orc.initial_state(gs[k], C0), "df")
        assert np.array_equal(partsU[k], C1) and qU[k] == q1, k


def test_forest_invalid_inputs(lm):
    gs = [inputs.rmat(8, seed=321), inputs.rmat(8, seed=322)]
    sizes, F = inputs.forest_csr(gs)
    # an entry joining the two graphs
    bad = inputs.csr_from_undirected(F.n, *_undirected_with_cross(F))
    with pytest.raises(lm.LeidenError):
        lm.Forest(sizes, bad.offs, bad.cols, bad.w)
    with pytest.raises(lm.LeidenError):
        lm.Forest(np.array([F.n - 1, 0], np.uint32), F.offs, F.cols, F.w)  # an empty graph
    Fh = lm.Forest(sizes, F.offs, F.cols, F.w)
    r = Fh.static()
    # a batch pair across graphs
    with pytest.raises(lm.LeidenError):
        Fh.update(np.zeros((0, 2), np.uint32), np.array([[0, gs[0].n, 3]], np.uint32))
    # a previous label outside its graph
    prev = r.membership.copy()
    prev[gs[0].n] = gs[1].n
    with pytest.raises(lm.LeidenError):
        Fh.update(np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32), prev=prev)
    # the state is unchanged by the refused calls
    r2 = Fh.update(np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32))
    assert np.array_equal(r2.membership, r.membership)
    with pytest.raises(lm.LeidenError):
        Fh.state()


def _undirected_with_cross(F):
    src = np.repeat(np.arange(F.n), np.diff(F.offs))
    m = src < F.cols
    u, v, w = list(src[m]), list(F.cols[m]), list(F.w[m])
    # a pair between vertex 0 of graph 0 and the last vertex (graph 1) that is not an edge yet
    u.append(0)
    v.append(F.n - 1)
    w.append(1)
    return np.array(u), np.array(v), np.array(w)


def _oracle_graph(job):
    """Oracle static run and one DF update (worker process)."""
    import oracle
    g, d, i = job
    C0, q0, st0 = oracle.static(g)
    gt, dw = oracle.apply_batch(g, d, i)
    C1, _, q1, _ = oracle.update(gt, dw, i, oracle.initial_state(g, C0), "df")
    return C0, q0, st0["passes"], C1, q1


def test_forest_knn_4096_sample_against_oracle(lm):
    """64 graphs of the 4,096-graph kNN workload (the same vertex counts and
    seeds as the benchmark's forests, chosen as its sample is), run as one
    forest: static, then a DF update of 1e-3 |E_q| per graph, every graph
    against the oracle.  A graph's result in a forest does not depend on the
    other graphs (the tests above), so these are the results the graphs get
    in the full workload."""
    import multiprocessing as mp

    import torch
    sizes_all = inputs.forest_sizes(4096, 1000, 200000, seed=inputs.BASE_SEED + 4)
    rng = np.random.default_rng(inputs.BASE_SEED + 9)
    sample = sorted(int(x) for x in rng.choice(4096, 64, replace=False))
    gs = []
    for q in sample:
        o, c, w = inputs.knn_graph_torch(int(sizes_all[q]), inputs.BASE_SEED + 5 + q, "cuda")
        gs.append(inputs.Csr(int(sizes_all[q]), o.cpu().numpy(), c.cpu().numpy().view(np.uint32),
                             w.cpu().numpy().view(np.uint32)))
    sizes, F = inputs.forest_csr(gs)
    Fh = lm.Forest(sizes, F.offs, F.cols, F.w)
    first = Fh.first.astype(np.int64)
    rF = Fh.static()
    qF, passes, _ = Fh.results()
    per, dl, il = [], [], []
    for k, g in enumerate(gs):
        nb = max(1, inputs.batch_size_for(g.nnz, 1e-3))
        d, i = inputs.random_batch(g.n, g.undirected_keys(), nb, seed=inputs.BASE_SEED + 700 + k, w_range=(1, 100))
        per.append((d, i))
        dl.append(d.astype(np.int64) + first[k])
        i2 = i.astype(np.int64)
        i2[:, :2] += first[k]
        il.append(i2)
    rU = Fh.update(np.concatenate(dl).astype(np.uint32), np.concatenate(il).astype(np.uint32), mode="df")
    qU = Fh.results()[0]
    with mp.get_context("fork").Pool(8) as pool:
        outs = pool.map(_oracle_graph, [(g, d, i) for g, (d, i) in zip(gs, per)])
    C0s, C1s = _split(rF.membership, sizes), _split(rU.membership, sizes)
    for k, (C0, q0, p0, C1, q1) in enumerate(outs):
        assert np.array_equal(C0s[k], C0) and qF[k] == q0 and passes[k] == p0, (k, sample[k])
        assert np.array_equal(C1s[k], C1) and qU[k] == q1, (k, sample[k])
