"""sssp_solve_noalloc (the entry point for callers that cannot allocate) against sssp_solve through
the C ABI: bit-exact distances and equal phase counts on two calls in a row, the second on a
smaller graph (the scratch array keeps the first call's contents), for each static criterion; a
graph too large for the array is rejected before any device work."""
import numpy as np
import pytest

import graphgen as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("crit", [6, 2, 4, 1, 5])
def test_noalloc_matches_solve_on_two_calls(B, crit):
    big = G.er(60013, 12, 1, (1 << 20) - 1, 71)      # several scan blocks and relax chunks, ragged tail
    small = G.rmat(11, 16, 1, 1 << 16, 72)
    for g in (big, small):
        print("noalloc case", g.name, crit, flush=True)
        dg = B.DeviceGraph.from_graph(g)
        srcs = [0, int(G.sources(g, 1, 73)[0])]
        for s in srcs:
            ref = B.solve(dg, s, crit)
            got = B.solve_noalloc(dg, s, crit)
            assert np.array_equal(got.dist_u64(), ref.dist_u64()), (g.name, s, crit)
            assert got.phases == ref.phases, (g.name, s, crit, got.phases, ref.phases)
        dg.close()


def test_noalloc_rejects_what_it_cannot_do(B):
    g = G.er(1 << 22, 2, 1, (1 << 20) - 1, 74)         # needs more scratch than the array holds
    dg = B.DeviceGraph.from_graph(g)
    with pytest.raises(B.SsspError) as e:
        B.solve_noalloc(dg, 0, B.STATIC_OR)
    assert e.value.code == -4 and "scratch" in str(e.value)
    dg.close()
    small = B.DeviceGraph.from_graph(G.er(1000, 4, 1, 100, 75))
    with pytest.raises(B.SsspError) as e:
        B.solve_noalloc(small, 0, B.SIMPLE_OR)
    assert e.value.code == -4
    with pytest.raises(B.SsspError) as e:
        B.solve_noalloc(small, 1000, B.STATIC_OR)
    assert e.value.code == -1
    r = B.solve_noalloc(small, 0, B.STATIC_OR)        # still works after the rejections
    assert np.array_equal(r.dist_u64(), B.solve(small, 0, B.STATIC_OR).dist_u64())
