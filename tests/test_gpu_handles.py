"""Handle rules of the C-ABI: the device-memory budget of a handle and one
call at a time per handle (LEIDEN_EBUSY)."""
import threading
import time

import numpy as np
import pytest

from paper_2410_15451_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lm():
    from paper_2410_15451_amd import binding
    binding.lib()
    return binding


def test_memory_budget(lm, orc):
    """A call that would grow the handle past its budget returns
    LEIDEN_ENOMEM and changes nothing; without the bound the same calls give
    the oracle's results."""
    g = inputs.rmat(14, seed=171)
    G = lm.Graph.from_csr(g)
    used0 = G.memory_used()
    assert used0 > 8 * g.nnz  # the slack CSR: columns and weights, two spans
    G.set_memory_budget(used0 + 4096)
    with pytest.raises(lm.LeidenError) as e:
        G.static()
    assert e.value.code == lm.LEIDEN_ENOMEM
    assert G.memory_used() <= used0 + 4096
    with pytest.raises(lm.LeidenError) as e:  # no state was set
        G.update(np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32))
    assert e.value.code == lm.LEIDEN_ESTATE
    G.set_memory_budget(0)
    r = G.static()
    C0, q0, _ = orc.static(g)
    assert np.array_equal(r.membership, C0) and r.q == q0
    used1 = G.memory_used()
    assert used1 > used0
    # the batch buffers do not fit a budget of what the handle holds now
    dels, ins = inputs.random_batch(g.n, g.undirected_keys(), 500, seed=172)
    G.set_memory_budget(used1)
    with pytest.raises(lm.LeidenError) as e:
        G.update(dels, ins, mode="df")
    assert e.value.code == lm.LEIDEN_ENOMEM
    offs, cols, w = G.export()
    assert np.array_equal(offs, g.offs) and np.array_equal(cols, g.cols) and np.array_equal(w, g.w)
    G.set_memory_budget(0)
    r1 = G.update(dels, ins, mode="df")
    gt, dw = orc.apply_batch(g, dels, ins)
    C1, _, q1, _ = orc.update(gt, dw, ins, orc.initial_state(g, C0), "df")
    assert np.array_equal(r1.membership, C1) and r1.q == q1
    G.close()


def test_one_call_at_a_time(lm, orc):
    """Static runs on one thread and modularity calls on another, on the same
    handle: calls that find the handle in use get LEIDEN_EBUSY, every other
    call returns the right value."""
    g = inputs.rmat(16, seed=173)
    G = lm.Graph.from_csr(g)
    r = G.static()
    C = r.membership.copy()
    q = G.modularity(C)
    stop = threading.Event()
    errors = []

    def runner():
        try:
            while not stop.is_set():
                try:
                    rs = G.static()
                    if not np.array_equal(rs.membership, C):
                        errors.append("static result changed")
                except lm.LeidenError as ex:
                    if ex.code != lm.LEIDEN_EBUSY:
                        errors.append(str(ex))
                time.sleep(0.002)  # room for the other thread's calls
        except Exception as ex:  # noqa: BLE001 - reported below
            errors.append(repr(ex))

    t = threading.Thread(target=runner)
    t.start()
    busy = ok = 0
    try:
        for _ in range(4000):
            try:
                assert G.modularity(C) == q
                ok += 1
            except lm.LeidenError as ex:
                assert ex.code == lm.LEIDEN_EBUSY, str(ex)
                busy += 1
            if busy >= 10 and ok >= 10:
                break
            time.sleep(0.0005)
    finally:
        stop.set()
        t.join()
    assert not errors, errors[:3]
    assert busy > 0 and ok > 0, (busy, ok)
    G.close()
