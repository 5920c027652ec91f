"""The clairvoyant ORACLE criterion (Section 3) on the GPU, pinned per vertex.

With d[v] = dist(s, v) as the criterion, v is settled in phase 1 + hop(v), where hop(v) is the
fewest edges over minimum-cost paths (induction on phases: the last edge of a fewest-edge shortest
path is relaxed at the end of the phase that settles its tail). The oracle's Dijkstra computes
dist and hop with lexicographic (cost, hops) keys, so the GPU's settle phase of every vertex, and
its phase count 1 + max hop, are fixed in advance. The reference distances given to the GPU come
from the oracle.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


def check(B, g, src):
    ref, hops = O.dijkstra(g, src)
    r = B.solve_oracle(B.DeviceGraph.from_graph(g), src, ref)
    assert np.array_equal(r.dist_u64(), ref), g.name
    reach = ref != np.uint64(O.INF_INT)
    po = r.phase_of.cpu().numpy().astype(np.int64)
    assert r.phases == 1 + int(hops[reach].max()), g.name
    assert np.array_equal(po[reach], hops[reach].astype(np.int64) + 1), g.name
    assert (po[~reach] == 0).all()
    return r


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_oracle_settles_each_vertex_at_its_hop_count(B, seed):
    for g in (G.er(3000, 6, 1, 1000, seed), G.rmat(11, 8, 1, 1 << 16, seed), G.grid(31, 17, 1, 40, seed),
              G.random_small(400, 1600, 5, seed), G.path(300, [1 + (i * 7) % 11 for i in range(299)])):
        check(B, g, int(G.sources(g, 1, seed)[0]))


def test_oracle_needs_fewer_phases_than_every_criterion(B):
    g = G.er(20000, 8, 1, 1 << 16, 9)
    r = check(B, g, 0)
    dg = B.DeviceGraph.from_graph(g)
    for crit in (B.STATIC_OR, B.SIMPLE_OR, B.FULL_OR, B.DIJK):
        assert B.solve(dg, 0, crit).phases >= r.phases


def test_oracle_full_size_random_graph(B):
    """The headline graph: 2^22 vertices, out-degree 16."""
    check(B, G.config_er_large(seed=1), 0)


def test_wrong_reference_is_reported(B):
    g = G.er(5000, 6, 1, 1000, 4)
    with pytest.raises(B.SsspError, match="ORACLE reference"):
        B.solve_oracle(B.DeviceGraph.from_graph(g), 0, np.zeros(g.n, np.uint64))
