"""Batched and serving forms (several graphs at once on one GPU).

Both forms run independent graph handles concurrently, so every result must
equal the result of the same graph run alone, bit for bit in the
deterministic mode; a sample is also checked against the oracle.
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


def _batches_for(gs, frac, seed):
    out = []
    for k, g in enumerate(gs):
        nb = max(1, inputs.batch_size_for(g.nnz, frac))
        out.append(inputs.random_batch(g.n, g.undirected_keys(), nb, seed=seed + k, w_range=(1, 100)))
    return out


def test_batched_equals_one_graph_at_a_time(lm, orc):
    gs = inputs.knn_forest(12, 1000, 6000, seed=inputs.BASE_SEED + 70)
    A = [lm.Graph.from_csr(g) for g in gs]
    B = [lm.Graph.from_csr(g) for g in gs]
    Cs, qs = lm.batch_run(A, streams=4)
    for k, (g, Gb) in enumerate(zip(gs, B)):
        r = Gb.static()
        assert np.array_equal(Cs[k], r.membership) and qs[k] == r.q, k
    for k in (0, 7):  # a sample against the oracle
        C, q, _ = orc.static(gs[k])
        assert np.array_equal(Cs[k], C) and qs[k] == q
    batches = _batches_for(gs, 2e-3, seed=71)
    Cu, qu = lm.batch_run(A, batches, mode="df", streams=4)
    for k, (Gb, (d, i)) in enumerate(zip(B, batches)):
        r = Gb.update(d, i, mode="df")
        assert np.array_equal(Cu[k], r.membership) and qu[k] == r.q, k
    gt, dw = orc.apply_batch(gs[3], *batches[3])
    C1, _, q1, _ = orc.update(gt, dw, batches[3][1], orc.initial_state(gs[3], orc.static(gs[3])[0]), "df")
    assert np.array_equal(Cu[3], C1) and qu[3] == q1


def test_server_results_equal_alone(lm, orc):
    gs = [inputs.rmat(s, seed=80 + s) for s in (9, 10, 11, 12)]
    streams = []
    for k, g in enumerate(gs):
        keys = g.undirected_keys()
        seq = []
        for b, nb in enumerate((5, 50, 300)):
            d, i = inputs.random_batch(g.n, keys, nb, seed=90 + 10 * k + b)
            seq.append((d, i))
            keys = inputs.keys_after_batch(keys, d, i)
        streams.append(seq)
    srv = lm.Server(hbm_budget_bytes=8 << 30, workers=3)
    ids = [srv.add_graph(g) for g in gs]
    # interleave the graphs' requests; modes vary per graph
    modes = ["df", "ds", "nd", "df"]
    tickets = []
    for b in range(3):
        for k in range(len(gs)):
            d, i = streams[k][b]
            tickets.append((k, b, srv.submit(ids[k], d, i, mode=modes[k])))
    got = {}
    for k, b, t in tickets:
        r, lat, svc = srv.wait(t)
        assert lat >= svc >= 0
        got[(k, b)] = r
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["failed"] == 0 and st["waiting"] == 0
    assert st["latency_p99_ms"] >= st["latency_p50_ms"] > 0
    # each graph alone, same requests in the same order
    for k, g in enumerate(gs):
        G = lm.Graph.from_csr(g)
        G.static()
        for b in range(3):
            d, i = streams[k][b]
            r = G.update(d, i, mode=modes[k])
            assert np.array_equal(got[(k, b)].membership, r.membership) and got[(k, b)].q == r.q, (k, b)
    # a sample against the oracle: two graphs' whole request chains
    for k in (1, 3):
        C0, _, _ = orc.static(gs[k])
        st, cur = orc.initial_state(gs[k], C0), gs[k]
        for b in range(3):
            d, i = streams[k][b]
            gt, dw = orc.apply_batch(cur, d, i)
            C1, st, q1, _ = orc.update(gt, dw, i, st, modes[k])
            assert np.array_equal(got[(k, b)].membership, C1) and got[(k, b)].q == q1, (k, b)
            cur = gt
    for gid in ids:
        srv.remove_graph(gid)
    assert srv.stats()["hbm_reserved"] == 0
    srv.close()


def test_server_admission_budget(lm):
    g = inputs.rmat(12, seed=5)
    small = lm.Server(hbm_budget_bytes=1 << 20, workers=1)
    with pytest.raises(lm.LeidenError):
        small.add_graph(g)
    small.close()
    srv = lm.Server(hbm_budget_bytes=4 << 30, workers=2)
    a = srv.add_graph(g)
    used = srv.stats()["hbm_reserved"]
    assert used > 0
    # admit until the budget is exhausted: the next graph is rejected, nothing else changes
    admitted = [a]
    while True:
        try:
            admitted.append(srv.add_graph(g))
        except lm.LeidenError:
            break
        assert len(admitted) < 10000
    assert srv.stats()["hbm_reserved"] == used * len(admitted) <= 4 << 30
    srv.remove_graph(admitted.pop())
    admitted.append(srv.add_graph(g))  # room again
    srv.close()
