"""The allocation-free modularity entry point (leiden_modularity_noalloc)
against the allocating one (leiden_modularity) on the same inputs: equal
values, two calls in a row with the second on a smaller graph (the shared
scratch array keeps the first call's contents), label and size errors."""
import numpy as np
import pytest

from paper_2410_15451_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_modularity_matches_allocating_call():
    import torch

    from paper_2410_15451_amd import binding
    dev = torch.device("cuda:0")
    big = inputs.rmat(16, seed=21)
    small = inputs.planted_partition()
    rng = np.random.default_rng(4)
    for g, k in ((big, 300), (small, 10), (big, big.n)):
        G = binding.Graph.from_csr(g)
        C = rng.integers(0, k, size=g.n).astype(np.uint32)
        Cd = torch.from_numpy(C.view(np.int32)).to(dev)
        q_alloc = G.modularity(C)
        q_na = G.modularity_noalloc(Cd)
        assert q_na == q_alloc, (g.n, k, q_na, q_alloc)
        # on the static result too, on a caller stream
        out = torch.zeros(g.n, dtype=torch.int32, device=dev)
        r = G.static(out=out)
        s = torch.cuda.current_stream()
        assert G.modularity_noalloc(out, stream=s.cuda_stream) == r.q
        bad = Cd.clone()
        bad[g.n // 2] = g.n
        with pytest.raises(binding.LeidenError) as ei:
            G.modularity_noalloc(bad)
        assert ei.value.code == binding.LEIDEN_EINVAL
        G.close()


def test_noalloc_modularity_size_limit():
    import torch

    from paper_2410_15451_amd import binding
    n = (1 << 22) + 1
    g = inputs.csr_from_edges(n, [(0, 1), (1, 2)])
    G = binding.Graph.from_csr(g)
    C = torch.zeros(n, dtype=torch.int32, device=torch.device("cuda:0"))
    with pytest.raises(binding.LeidenError) as ei:
        G.modularity_noalloc(C)
    assert ei.value.code == binding.LEIDEN_EINVAL
    assert G.modularity(np.zeros(n, np.uint32)) == 0.0
    G.close()
