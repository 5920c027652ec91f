"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Distances must be bit-exact (all arithmetic is integer). Phase counts, the phase in which each
vertex settles, the summed fringe sizes and the number of relaxations towards non-settled targets
are unique under the phase-start snapshot semantics (Section 3) and must match exactly.
Delta-stepping: distances exact, rounds and buckets exact under the round rules stated in the oracle.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O

pytestmark = pytest.mark.gpu

CRITS = [("DIJK", O.DIJK), ("IN_STATIC", O.IN_STATIC), ("OUT_STATIC", O.OUT_STATIC),
         ("IN_SIMPLE", O.IN_SIMPLE), ("OUT_SIMPLE", O.OUT_SIMPLE), ("IN_FULL", O.IN_FULL),
         ("OUT_WEAK", O.OUT_WEAK), ("OUT_FULL", O.OUT_FULL), ("STATIC_OR", O.STATIC_OR),
         ("SIMPLE_OR", O.SIMPLE_OR), ("FULL_OR", O.FULL_OR), ("IN_FULL|OUT_WEAK", O.IN_FULL | O.OUT_WEAK),
         ("DIJK|OUT_STATIC", O.DIJK | O.OUT_STATIC), ("IN_STATIC|OUT_FULL", O.IN_STATIC | O.OUT_FULL)]


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


def check_phased(B, g, src, crit, label=""):
    dg = B.DeviceGraph.from_graph(g)
    ref = O.phased(g, src, crit)
    r = B.solve_ex(dg, src, crit, phase_of=True, trace_cap=ref.phases + 4)
    got = r.dist_u64()
    assert np.array_equal(got, ref.dist), "%s: distances differ at %d vertices" % (label, int((got != ref.dist).sum()))
    assert r.phases == ref.phases, "%s: phases %d != oracle %d" % (label, r.phases, ref.phases)
    po = r.phase_of.cpu().numpy().view(np.uint32)
    assert np.array_equal(po, ref.phase_of), "%s: settle phases differ" % label
    st = r.stats
    assert st["sum_f"] == ref.sum_f, label
    assert st["n_reach"] == ref.n_reach and st["m_reach"] == ref.m_reach, label
    assert st["relax_edges"] == ref.relax_edges, label
    assert np.array_equal(r.trace["fringe"], ref.trace_f), label
    assert np.array_equal(r.trace["settled"], ref.trace_s), label
    assert np.array_equal(r.trace["min_d"], ref.trace_mind), label
    dg.close()
    return r


def small_cases():
    out = []
    for s in range(60):
        x = G.u64_stream(s, 21, 3)
        n = 1 + int(x[0] % np.uint64(40))
        m = int(x[1] % np.uint64(5 * n + 1))
        wmax = [1, 4, 100, 0xFFFFFFFF][int(x[2] % np.uint64(4))]
        out.append(G.random_small(n, m, wmax, 100 + s))
    return out


def test_hand_traces_all_criteria(B):
    import json, os
    fix = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_traces.json")))
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        for name, c in CRITS:
            check_phased(B, g, 0, c, "%s/%s" % (key, name))


def test_random_multigraphs_all_criteria(B):
    # zero weights, self-loops, parallel edges, unreachable parts, weights up to 2^32-1
    for g in small_cases():
        src = int(G.u64_stream(7, 3, 1)[0] % np.uint64(g.n))
        for name, c in CRITS:
            check_phased(B, g, src, c, "%s/%s" % (g.name, name))


@pytest.mark.parametrize("name,c", CRITS)
def test_config_small_er16k(B, name, c):
    check_phased(B, G.config_small(), 0, c, "er16k/" + name)


@pytest.mark.parametrize("maker", [
    lambda: G.er(1 << 15, 16, 1, (1 << 20) - 1, 5),
    lambda: G.rmat(14, 16, 1, (1 << 20) - 1, 6),
    lambda: G.grid(96, 80, 1, 1 << 16, 7),
    lambda: G.er(5000, 3, 1, 7, 8),          # many ties, sparse: unreachable vertices
])
def test_medium_graphs_key_criteria(B, maker):
    g = maker()
    src = int(G.sources(g, 1, 3)[0])
    for name, c in [("STATIC_OR", O.STATIC_OR), ("SIMPLE_OR", O.SIMPLE_OR), ("FULL_OR", O.FULL_OR),
                    ("IN_STATIC", O.IN_STATIC), ("OUT_WEAK", O.OUT_WEAK), ("DIJK", O.DIJK)]:
        check_phased(B, g, src, c, "%s/%s" % (g.name, name))


def test_edge_cases(B):
    one = G.from_edges(1, [])
    r = B.solve(B.DeviceGraph.from_graph(one), 0, O.STATIC_OR)
    assert r.phases == 1 and list(r.dist_u64()) == [0]
    loop = G.from_edges(2, [(0, 0, 5), (1, 0, 3)])  # self-loop on the source, vertex 1 unreachable
    check_phased(B, loop, 0, O.FULL_OR, "selfloop")
    sink = G.from_edges(4, [(1, 2, 1), (2, 3, 1)])  # source without out-edges
    check_phased(B, sink, 0, O.STATIC_OR, "sink-source")
    heavy = G.from_edges(3, [(0, 1, 0xFFFFFFFF), (1, 2, 0xFFFFFFFF), (0, 2, 0xFFFFFFFF)])
    r = check_phased(B, heavy, 0, O.SIMPLE_OR, "max-weights")
    assert int(r.dist_u64()[2]) == 0xFFFFFFFF


def test_repeat_runs_are_identical(B):
    g = G.rmat(13, 16, 1, 1000, 9)
    dg = B.DeviceGraph.from_graph(g)
    a = B.solve_ex(dg, 0, O.STATIC_OR, phase_of=True, trace_cap=4096)
    b = B.solve_ex(dg, 0, O.STATIC_OR, phase_of=True, trace_cap=4096)
    assert np.array_equal(a.dist_u64(), b.dist_u64())
    assert np.array_equal(a.trace, b.trace)
    assert np.array_equal(a.phase_of.cpu().numpy(), b.phase_of.cpu().numpy())


def test_static_minima_on_device(B):
    g = G.random_small(300, 1500, 1000, 4)
    mi, mo = B.DeviceGraph.from_graph(g).minima()
    rmi, rmo = O.static_minima(g)
    assert np.array_equal(mi.cpu().numpy().view(np.uint32), rmi)
    assert np.array_equal(mo.cpu().numpy().view(np.uint32), rmo)


def skewed_rows_graph():
    """CSR with the row shapes the minOut pass must get right: a 5000-edge row, a run of 200
    empty rows, rows ending on a 64-row boundary, and n not a multiple of 64."""
    n = 1000
    deg = np.zeros(n, np.int64)
    deg[:64] = 3                # one full window of short rows
    deg[64:264] = 0             # a run of empty rows across windows
    deg[300] = 5000             # one long row inside a window
    deg[301:999] = (np.arange(301, 999) % 7)
    deg[999] = 65               # the last row, in a partial window
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.uint64)
    m = int(rp[-1])
    x = G.u64_stream(9, 11, 2 * m)
    col = (x[:m] % n).astype(np.uint32)
    w = (1 + x[m:] % 1000000).astype(np.uint32)
    return G.Graph(n, rp, col, w, "skewed_rows")


def test_static_minima_skewed_rows(B):
    for g in (skewed_rows_graph(), G.rmat(12, 16, 1, (1 << 20) - 1, 4)):
        mi, mo = B.DeviceGraph.from_graph(g).minima()
        rmi, rmo = O.static_minima(g)
        assert np.array_equal(mi.cpu().numpy().view(np.uint32), rmi), g.name
        assert np.array_equal(mo.cpu().numpy().view(np.uint32), rmo), g.name


def test_rows_sorted_on_first_dynamic_solve(B):
    """Rows stay in input order until a solve first needs the dynamic criteria's cursors, which sorts
    them by weight in place: rows given heaviest edge first, static solves before and after the sort,
    the static minima and every criterion stay exact against the oracle."""
    g0 = G.er(4000, 12, 1, 1 << 20, 71)
    col, w = g0.col.copy(), g0.w.copy()
    for v in range(g0.n):  # each row heaviest edge first
        b, e = int(g0.row_ptr[v]), int(g0.row_ptr[v + 1])
        o = np.argsort(-w[b:e].astype(np.int64), kind="stable")
        col[b:e], w[b:e] = col[b:e][o], w[b:e][o]
    g = G.Graph(g0.n, g0.row_ptr.copy(), col, w, "er4000_rows_heaviest_first")
    dg = B.DeviceGraph.from_graph(g)
    rmi, rmo = O.static_minima(g)
    src = int(G.sources(g, 1, 72)[0])
    for c in (O.STATIC_OR, O.SIMPLE_OR, O.STATIC_OR, O.FULL_OR, O.IN_STATIC):
        mi, mo = dg.minima()
        assert np.array_equal(mi.cpu().numpy().view(np.uint32), rmi)
        assert np.array_equal(mo.cpu().numpy().view(np.uint32), rmo)
        ref = O.phased(g, src, c)
        r = B.solve(dg, src, c)
        assert np.array_equal(r.dist_u64(), ref.dist), c
        assert r.phases == ref.phases, (c, r.phases, ref.phases)
    dg.close()


def star_with_heavy_chain(n, seed):
    """Vertex 0 reaches every other vertex v by one edge of seeded weight w(v) in [1, 2^20], and
    every v in 1 .. n-2 has one more out-edge, to v + 1, of weight 2^31 (the last row is empty).
    No path through a heavy edge is shorter, so dist(v) = w(v) in closed form."""
    leaves = n - 1
    w0 = (G.u64_stream(seed, 5, leaves) % np.uint64(1 << 20) + np.uint64(1)).astype(np.uint32)
    rp = np.empty(n + 1, np.uint64)
    rp[0] = 0
    rp[1:n] = np.uint64(leaves) + np.arange(n - 1, dtype=np.uint64)  # rows 1 .. n-2 hold one edge each
    rp[n] = rp[n - 1]
    col = np.concatenate([np.arange(1, n, dtype=np.uint32), np.arange(2, n, dtype=np.uint32)])
    w = np.concatenate([w0, np.full(max(n - 2, 0), 1 << 31, np.uint32)])
    dist = np.concatenate([np.zeros(1, np.uint64), w0.astype(np.uint64)])
    return G.Graph(n, rp, col, w, "star%d_heavy_chain" % n), dist


def star_delta_rounds(dist, delta):
    """Delta-stepping's rounds on that star (delta <= 2^31): bucket 0 takes a light round from the
    source, a second one if some leaf is light, and its heavy round; every other bucket holding a
    leaf takes one light round (its leaves have no light edge) and one heavy round."""
    w0 = dist[1:]
    later = np.unique(w0[w0 >= np.uint64(delta)] // np.uint64(delta))
    return 2 + int(bool((w0 < np.uint64(delta)).any())) + 2 * len(later)


def test_star_with_heavy_chain_small_matches_oracle(B):
    """The construction of the largest-size test below, small enough for the oracle: its closed-form
    distances and its two phases (the source, then every leaf) are the oracle's."""
    g, dist = star_with_heavy_chain(3001, 81)
    assert int(g.row_ptr[-1]) == len(g.col) == 2 * 3001 - 3
    dg = B.DeviceGraph.from_graph(g)
    for c in (O.STATIC_OR, O.IN_STATIC, O.SIMPLE_OR):
        ref = O.phased(g, 0, c)
        assert np.array_equal(ref.dist, dist) and ref.phases == 2, c
        r = B.solve(dg, 0, c)
        assert np.array_equal(r.dist_u64(), dist) and r.phases == 2, c
    # Delta-stepping: with Delta = 2^21 every star edge is light (3 rounds, one bucket); with 2^19
    # and 2^18 the leaves spread over several buckets
    for delta, rounds in ((1 << 21, 3), (1 << 19, 5), (1 << 18, 9)):
        assert star_delta_rounds(dist, delta) == rounds
        ref = O.delta_step(g, 0, [delta])
        assert np.array_equal(ref.dist, dist) and ref.rounds == rounds, delta
        r = B.delta_step(dg, 0, delta)
        assert np.array_equal(r.dist_u64(), dist) and r.phases == rounds, delta
    dg.close()


def test_largest_vertex_count(B):
    """n = 2^26 - 1, the largest vertex count the library accepts, on the star with a heavy chain
    (134 M edges): distances exact against the closed form, two phases, with the default launch
    shape, keyed queue arrays and the one-workgroup form, with the SIMPLE criteria (their first
    solve sorts the rows), in a batch, and Delta-stepping's rounds."""
    n = (1 << 26) - 1
    g, dist = star_with_heavy_chain(n, 82)
    dg = B.DeviceGraph.from_graph(g)
    del g
    keyed = dict(scan_blocks=1024, relax_blocks=2048, chunk=256, use_graph=0, queue=2, single=0)
    try:
        for shape, c in ((None, O.STATIC_OR), (keyed, O.STATIC_OR), (dict(keyed, single=1), O.STATIC_OR),
                         (dict(keyed, single=0), O.SIMPLE_OR)):
            if shape:
                dg.set_launch(**shape)
            r = B.solve(dg, 0, c)
            assert r.phases == 2, (shape, c)
            assert np.array_equal(r.dist_u64(), dist), (shape, c)
        for delta in (1 << 21, 1 << 19):  # with 2^19 some leaf weighs 2^20: a third bucket
            r = B.delta_step(dg, 0, delta)
            assert r.phases == star_delta_rounds(dist, delta), delta
            assert np.array_equal(r.dist_u64(), dist), delta
        # the batched form: two queries on this graph (teams of workgroups, as it has more than
        # 2^20 edges) beside a small one (one workgroup)
        small = G.er(1000, 8, 1, 1000, 85)
        sdg = B.DeviceGraph.from_graph(small)
        dists, phases = B.solve_batch([dg, sdg, dg], [0, 3, 0], O.STATIC_OR)
        ref = O.phased(small, 3, O.STATIC_OR)
        assert [int(x) for x in phases] == [2, ref.phases, 2]
        assert np.array_equal(B.to_u64(dists[1]), ref.dist)
        assert np.array_equal(B.to_u64(dists[0]), dist) and np.array_equal(B.to_u64(dists[2]), dist)
        sdg.close()
    finally:
        dg.close()


def star_with_heavy_rows(n, heavy, seed):
    """Vertex 0 reaches every other vertex v by one edge of seeded weight w(v) in [1, 2^20], and
    every v >= 1 has `heavy` more out-edges, to (v + k) mod n for k = 1 .. heavy, of weight 2^31:
    m = (n - 1)(heavy + 1), and dist(v) = w(v) in closed form."""
    w0 = (G.u64_stream(seed, 6, n - 1) % np.uint64(1 << 20) + np.uint64(1)).astype(np.uint32)
    rp = np.empty(n + 1, np.uint64)
    rp[0] = 0
    rp[1:] = np.uint64(n - 1) + np.uint64(heavy) * np.arange(n, dtype=np.uint64)
    m = int(rp[-1])
    col = np.empty(m, np.uint32)
    col[: n - 1] = np.arange(1, n, dtype=np.uint32)
    hv = col[n - 1:].reshape(n - 1, heavy)
    ks = np.arange(1, heavy + 1, dtype=np.uint64)
    for r0 in range(0, n - 1, 1 << 18):  # rows in blocks, to keep the temporaries small
        r1 = min(r0 + (1 << 18), n - 1)
        t = np.arange(r0 + 1, r1 + 1, dtype=np.uint64)[:, None] + ks[None, :]
        t[t >= n] -= np.uint64(n)
        hv[r0:r1] = t
    w = np.full(m, 1 << 31, np.uint32)
    w[: n - 1] = w0
    dist = np.concatenate([np.zeros(1, np.uint64), w0.astype(np.uint64)])
    return G.Graph(n, rp, col, w, "star%d_heavy%d" % (n, heavy)), dist


def test_star_with_heavy_rows_small_matches_oracle(B):
    """The construction of the many-edges test below, small enough for the oracle: closed-form
    distances and two phases are the oracle's, and the library's."""
    g, dist = star_with_heavy_rows(1001, 7, 83)
    assert int(g.row_ptr[-1]) == len(g.col) == 1000 * 8
    for c in (O.STATIC_OR, O.IN_STATIC):
        ref = O.phased(g, 0, c)
        assert np.array_equal(ref.dist, dist) and ref.phases == 2, c
        r = B.solve(B.DeviceGraph.from_graph(g), 0, c)
        assert np.array_equal(r.dist_u64(), dist) and r.phases == 2, c


def test_more_than_2_31_edges(B):
    """m = 129 * 2^24 = 2,164,260,864 edges (above 2^31, below the 2^32 limit) on n = 2^24 + 1
    vertices: edge indices past the signed 32-bit range in graph creation (minima, packing) and in
    relax; distances exact against the closed form, two phases, default and keyed launch shapes."""
    n = (1 << 24) + 1
    g, dist = star_with_heavy_rows(n, 128, 84)
    assert int(g.row_ptr[-1]) > (1 << 31)
    dg = B.DeviceGraph.from_graph(g)
    del g
    try:
        for shape in (None, dict(scan_blocks=1024, relax_blocks=2048, chunk=256, use_graph=0, queue=2, single=0)):
            if shape:
                dg.set_launch(**shape)
            r = B.solve(dg, 0, O.STATIC_OR)
            assert r.phases == 2, shape
            assert np.array_equal(r.dist_u64(), dist), shape
    finally:
        dg.close()


def check_delta(B, g, src, deltas):
    dg = B.DeviceGraph.from_graph(g)
    ref = O.delta_step(g, src, deltas, trace_cap=0)
    r = B.delta_step_ex(dg, src, deltas)
    got = r.dist_u64()
    assert np.array_equal(got, ref.dist), "delta %s: distances differ" % (deltas,)
    assert r.phases == ref.rounds, "delta %s: rounds %d != %d" % (deltas, r.phases, ref.rounds)
    assert r.stats["buckets"] == ref.buckets
    dg.close()


def test_delta_stepping_small(B):
    for g in small_cases()[:30]:
        for deltas in ([1], [3], [1000], [1 << 40], [2, 50, 7]):
            check_delta(B, g, 0, deltas)


@pytest.mark.parametrize("delta", [1 << 12, 1 << 14, 1 << 16])
def test_delta_stepping_medium(B, delta):
    for g in (G.er(1 << 14, 16, 1, (1 << 20) - 1, 3), G.rmat(13, 16, 1, (1 << 20) - 1, 4),
              G.grid(64, 64, 1, 1 << 16, 5)):
        check_delta(B, g, int(G.sources(g, 1, 1)[0]), [delta])


def test_invalid_arguments_rejected(B):
    g = G.config_small()
    dg = B.DeviceGraph.from_graph(g)
    with pytest.raises(B.SsspError):
        B.solve(dg, g.n, O.STATIC_OR)        # source out of range
    with pytest.raises(B.SsspError):
        B.solve(dg, 0, 0)                    # empty criterion
    with pytest.raises(B.SsspError):
        B.solve(dg, 0, 1 << 9)               # unknown bit
    with pytest.raises(B.SsspError):
        B.delta_step(dg, 0, 0)               # zero bucket width
    r = B.solve(dg, 0, O.STATIC_OR)          # the handle still works afterwards
    assert r.phases > 1


def test_graph_replay_matches_stream_launches(B):
    """Phases replayed from a captured HIP graph give the same results as plain launches, on every
    replay, with eager solves in between."""
    g = G.rmat(14, 16, 1, 1 << 16, 12)
    dg = B.DeviceGraph.from_graph(g)
    ref = O.phased(g, 0, O.STATIC_OR)
    for use_graph in (0, 1, 1, 0, 1, 1):
        dg.set_launch(use_graph=use_graph)
        r = B.solve_ex(dg, 0, O.STATIC_OR, phase_of=True)
        assert np.array_equal(r.dist_u64(), ref.dist)
        assert r.phases == ref.phases and r.stats["sum_f"] == ref.sum_f
        assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of)
    for use_graph in (1, 0, 1):
        dg.set_launch(use_graph=use_graph)
        r = B.delta_step_ex(dg, 0, [1 << 12])
        rd = O.delta_step(g, 0, [1 << 12])
        assert np.array_equal(r.dist_u64(), rd.dist) and r.phases == rd.rounds


@pytest.mark.parametrize("cfg", [dict(scan_blocks=1, relax_blocks=1, chunk=256),
                                 dict(scan_blocks=7, relax_blocks=3, chunk=1024),
                                 dict(scan_blocks=4096, relax_blocks=4096, chunk=512)])
def test_launch_shapes_do_not_change_results(B, cfg):
    g = G.er(20000, 12, 1, 5000, 13)
    dg = B.DeviceGraph.from_graph(g)
    dg.set_launch(**cfg)
    for c in (O.STATIC_OR, O.FULL_OR):
        check_phased(B, g, 0, c, str(cfg))


def test_settle_buffer_overflow_path(B):
    """One phase settles thousands of vertices with out-edges inside a single scan block, more than
    the per-block LDS collection buffer holds, so part of them take the direct append path."""
    k = 60000
    edges = [(0, 1 + i, 1) for i in range(k)] + [(1 + i, 1 + k + i, 1 + (i % 5)) for i in range(k)]
    g = G.from_edges(1 + 2 * k, edges, "two-level-star")
    dg = B.DeviceGraph.from_graph(g)
    dg.set_launch(scan_blocks=8)  # about 15000 vertices per block
    ref = O.phased(g, 0, O.STATIC_OR)
    r = B.solve_ex(dg, 0, O.STATIC_OR, phase_of=True)
    assert np.array_equal(r.dist_u64(), ref.dist) and r.phases == ref.phases
    assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of)
    rd = B.delta_step_ex(dg, 0, [1 << 20])
    od = O.delta_step(g, 0, [1 << 20])
    assert np.array_equal(rd.dist_u64(), od.dist) and rd.phases == od.rounds


def test_scratch_rebuilt_after_launch_change(B):
    """Changing the scan grid rebuilds the per-solve scratch; every solve kind still works after it."""
    g = G.er(3000, 6, 1, 300, 14)
    dg = B.DeviceGraph.from_graph(g)
    od = O.delta_step(g, 0, [64])
    op = O.phased(g, 0, O.FULL_OR)
    for sb in (3, 11, 3):
        r = B.delta_step_ex(dg, 0, [64])
        assert np.array_equal(r.dist_u64(), od.dist) and r.phases == od.rounds
        r = B.solve(dg, 0, O.FULL_OR)
        assert np.array_equal(r.dist_u64(), op.dist) and r.phases == op.phases
        dg.set_launch(scan_blocks=sb)


def small_batch():
    graphs = [G.er(1 << 10, 6, 1, 1 << 16, 31), G.grid(40, 30, 1, 1 << 16, 32), G.rmat(10, 16, 1, 1 << 16, 33),
              G.er(3000, 20, 1, 100, 34), G.random_small(200, 900, 50, 35), G.from_edges(1, [])]
    queries = []
    for i, g in enumerate(graphs):
        for s in range(5 if g.n > 1 else 1):
            queries.append((i, int(G.u64_stream(i, s, 1)[0] % np.uint64(g.n))))
    return graphs, queries


@pytest.mark.parametrize("crit", [O.STATIC_OR, O.IN_STATIC, O.OUT_STATIC, O.DIJK])
@pytest.mark.parametrize("cfg", [None, dict(block=256, split=4, blocks=3), dict(block=1024, split=1000, blocks=64),
                                 dict(team_edges=1, team_size=4), dict(team_edges=3000, team_size=3, block=256, split=4),
                                 dict(team_edges=1, team_size=64, block=1024)])
def test_batched_matches_oracle(B, crit, cfg):
    """The batched launch against the oracle, one workgroup per query and (team_edges) with teams
    of workgroups sharing a query: odd team sizes, more members than a small query has fringe
    entries, the degree split inside a team member."""
    graphs, queries = small_batch()
    dgs = [B.DeviceGraph.from_graph(g) for g in graphs]
    dists, phases = B.solve_batch([dgs[i] for i, _ in queries], [s for _, s in queries], crit, cfg=cfg)
    for (i, s), d, ph in zip(queries, dists, phases):
        ref = O.phased(graphs[i], s, crit)
        assert np.array_equal(B.to_u64(d), ref.dist), (graphs[i].name, s)
        assert int(ph) == ref.phases, (graphs[i].name, s, int(ph), ref.phases)


def test_batched_rejects_dynamic_criteria(B):
    graphs, queries = small_batch()
    dg = B.DeviceGraph.from_graph(graphs[0])
    with pytest.raises(B.SsspError):
        B.solve_batch([dg], [0], O.FULL_OR)


def test_autotuners_keep_results(B):
    g = G.rmat(12, 16, 1, 1 << 16, 36)
    dg = B.DeviceGraph.from_graph(g)
    cfg, ms = B.autotune(dg, 0, O.STATIC_OR)
    assert ms > 0 and cfg["chunk"] in (256, 512)
    check_phased(B, g, 0, O.STATIC_OR, "after autotune")
    graphs, queries = small_batch()
    dgs = [B.DeviceGraph.from_graph(x) for x in graphs]
    bcfg, bms = B.autotune_batch([dgs[i] for i, _ in queries], [s for _, s in queries], O.STATIC_OR)
    assert bms > 0 and bcfg["block"] in (256, 512, 1024)
    dists, phases = B.solve_batch([dgs[i] for i, _ in queries], [s for _, s in queries], O.STATIC_OR)
    for (i, s), d in zip(queries, dists):
        assert np.array_equal(B.to_u64(d), O.dijkstra(graphs[i], s)[0])


STATIC_CRITS = [O.STATIC_OR, O.IN_STATIC, O.OUT_STATIC, O.DIJK, O.DIJK | O.OUT_STATIC, O.DIJK | O.IN_STATIC]


@pytest.mark.parametrize("cfg", [dict(scan_blocks=1), dict(scan_blocks=2), dict(scan_blocks=5, relax_blocks=3, chunk=1024),
                                 dict(scan_blocks=64, use_graph=1), dict(scan_blocks=4096, chunk=512)])
def test_queue_arrays_match_oracle(B, cfg):
    """Static criteria with keyed queue arrays, with per-block queue arrays (on by default) and with
    the dense scan: every observable of the oracle, on graphs whose vertex counts are not multiples
    of a block's span (keyed: rebuild launches are not phases, so the phase-indexed trace and
    settle phases must still equal the oracle's).
    With one or two scan blocks each block owns thousands of vertices, so its slots fill with
    tombstones and are compacted over several steps, many times per solve (one block cannot hold
    the 20011-vertex graph's state window and takes the dense scan there). On the random graph
    two thirds of the vertices are queued at the peak, far above the 3/8 at which identify switches
    to the dense scan, so solves switch over and back, rebuilding the arrays."""
    graphs = [G.er(20011, 10, 1, 5000, 41), G.rmat(13, 16, 1, 1 << 16, 42), G.grid(97, 61, 1, 1 << 16, 43),
              G.random_small(300, 1500, 0xFFFFFFFF, 44)]
    peak = O.phased(graphs[0], 0, O.STATIC_OR, trace_cap=1 << 16).trace_f.max()
    assert 8 * peak >= 3 * graphs[0].n and 5 * peak < 4 * graphs[0].n
    for g in graphs:
        refs = {c: O.phased(g, 0, c) for c in STATIC_CRITS}
        for queue in (2, 1, 0):
            dg = B.DeviceGraph.from_graph(g)
            dg.set_launch(queue=queue, **cfg)
            for c in STATIC_CRITS:
                ref = refs[c]
                r = B.solve_ex(dg, 0, c, phase_of=True, trace_cap=ref.phases + 4)
                label = (g.name, queue, cfg, c)
                assert np.array_equal(r.dist_u64(), ref.dist), label
                assert r.phases == ref.phases and r.stats["sum_f"] == ref.sum_f, label
                assert r.stats["relax_edges"] == ref.relax_edges, label
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), label
                assert np.array_equal(r.trace["settled"], ref.trace_s), label
            dg.close()


DYN_CRITS = [O.SIMPLE_OR, O.IN_SIMPLE, O.OUT_SIMPLE, O.CRIT["IN_SIMPLE"] | O.OUT_STATIC,
             O.IN_STATIC | O.OUT_SIMPLE, O.DIJK | O.OUT_SIMPLE, O.FULL_OR, O.IN_FULL | O.OUT_WEAK]


@pytest.mark.parametrize("cfg", [dict(scan_blocks=1), dict(scan_blocks=5, relax_blocks=3, chunk=1024),
                                 dict(scan_blocks=64, use_graph=1), dict(scan_blocks=4096, chunk=512)])
def test_queue_arrays_dynamic_criteria_match_oracle(B, cfg):
    """Dynamic criteria on the queue arrays (term pass over the entries and the vertices flagged
    new, identify with the IN flag and the dynamic OUT threshold) against the dense scan and the
    oracle: every observable, on graphs whose vertex counts are not multiples of a block's span.
    The random graph's peak queue passes the dense-scan threshold, so the term pass also runs
    after dense phases, when the entries are stale and it takes every queued vertex."""
    graphs = [G.er(20011, 10, 1, 5000, 46), G.rmat(13, 16, 1, 1 << 16, 47), G.grid(97, 61, 1, 1 << 16, 48),
              G.random_small(300, 1500, 0xFFFFFFFF, 49)]
    for g in graphs:
        crits = DYN_CRITS
        refs = {c: O.phased(g, 0, c) for c in crits}
        for queue in (1, 0, 2):
            dg = B.DeviceGraph.from_graph(g)
            dg.set_launch(queue=queue, **cfg)
            for c in crits:
                ref = refs[c]
                r = B.solve_ex(dg, 0, c, phase_of=True, trace_cap=ref.phases + 4)
                label = (g.name, queue, cfg, c)
                assert np.array_equal(r.dist_u64(), ref.dist), label
                assert r.phases == ref.phases and r.stats["sum_f"] == ref.sum_f, label
                assert r.stats["relax_edges"] == ref.relax_edges, label
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), label
                assert np.array_equal(r.trace["settled"], ref.trace_s), label
                assert np.array_equal(r.trace["min_d"], ref.trace_mind), label
            dg.close()


def test_queue_arrays_survive_solve_kind_changes(B):
    """Queue-array solves interleaved with dense, dynamic, Delta-stepping and other-source solves
    on one handle: each starts from a clean state."""
    g = G.er(5000, 8, 1, 1000, 45)
    dg = B.DeviceGraph.from_graph(g)
    srcs = [0, 17, 4999]
    refs = {s: O.phased(g, s, O.STATIC_OR) for s in srcs}
    full = O.phased(g, 0, O.FULL_OR)
    dl = O.delta_step(g, 0, [256])
    for step in range(3):
        for s in srcs:
            r = B.solve(dg, s, O.STATIC_OR)
            assert np.array_equal(r.dist_u64(), refs[s].dist) and r.phases == refs[s].phases, (step, s)
        r = B.solve(dg, 0, O.FULL_OR)
        assert np.array_equal(r.dist_u64(), full.dist) and r.phases == full.phases
        r = B.delta_step_ex(dg, 0, [256])
        assert np.array_equal(r.dist_u64(), dl.dist) and r.phases == dl.rounds
        dg.set_launch(queue=(step + 2) % 3)


def test_single_workgroup_solves_match_oracle(B):
    """Launch option `single`: sssp_solve with a static criterion runs in one workgroup of the batched
    kernel; distances and phase counts equal the oracle's, also on repeated calls with other sources
    (the scratch stays on the graph). Dynamic criteria and sssp_solve_ex ignore the option."""
    graphs = [G.grid(61, 53, 1, 1 << 16, 51), G.er(3000, 6, 1, 500, 52), G.rmat(12, 16, 1, 1 << 16, 53),
              G.random_small(200, 800, 0xFFFFFFFF, 54), G.from_edges(1, [])]
    for g in graphs:
        dg = B.DeviceGraph.from_graph(g)
        dg.set_launch(single=1)
        srcs = [0] if g.m == 0 else [int(x) for x in G.sources(g, 2, 55)]
        for src in srcs:
            for c in STATIC_CRITS:
                ref = O.phased(g, src, c)
                r = B.solve(dg, src, c)
                assert np.array_equal(r.dist_u64(), ref.dist), (g.name, src, c)
                assert r.phases == ref.phases, (g.name, src, c, r.phases, ref.phases)
        ref = O.phased(g, 0, O.SIMPLE_OR)
        r = B.solve(dg, 0, O.SIMPLE_OR)
        assert np.array_equal(r.dist_u64(), ref.dist) and r.phases == ref.phases
        ref = O.phased(g, 0, O.STATIC_OR)
        r = B.solve_ex(dg, 0, O.STATIC_OR, phase_of=True)
        assert np.array_equal(r.dist_u64(), ref.dist) and r.stats["sum_f"] == ref.sum_f
        dg.close()


def expected_switch(trace_f, phases, num, den, batch=16):
    """The switch phase of sssp_solve_switch as its header documents it, from the static-only
    oracle trace (the first stage is that solve): the host checks |F| at the start of the last
    phase of batch b - 1 after queuing batch b; the first check at or below num/den of the largest
    earlier check (and below it) ends the first stage after batch b. None: no switch before F empties."""
    peak, b = 0, 0
    while True:
        if b >= 1:
            last = batch * b - 1
            if last >= phases:  # the solve had ended: header shows done
                return None
            f = int(trace_f[last])
            if peak and f < peak and f * den <= peak * num:
                return batch * (b + 1)
            peak = max(peak, f)
        b += 1


def test_switched_solve_matches_oracle_replay(B):
    """sssp_solve_switch: static phases, then the second criterion from the documented batch
    boundary on; every observable equals the oracle's replay of the recorded criterion sequence,
    distances equal Dijkstra's, and the switch phase equals the one computed from the oracle's
    static-only trace."""
    graphs = [G.er(20011, 10, 1, 5000, 61), G.rmat(13, 16, 1, 1 << 16, 62), G.grid(97, 61, 1, 1 << 16, 63),
              G.er(5000, 3, 1, 7, 64)]
    for g in graphs:
        dg = B.DeviceGraph.from_graph(g)
        dj, _ = O.dijkstra(g, 0)
        base = O.phased(g, 0, O.STATIC_OR, trace_cap=1 << 20)
        for then in (O.CRIT["IN_SIMPLE"] | O.OUT_STATIC, O.SIMPLE_OR, O.FULL_OR):
            for num, den in ((1, 2), (1, 3), (1, 1)):
                r = B.solve_switch(dg, 0, O.STATIC_OR, then, (num, den), phase_of=True, trace_cap=g.n + 4)
                label = (g.name, then, num, den)
                assert np.array_equal(r.dist_u64(), dj), label
                crit = np.asarray(r.trace["criterion"])
                k = expected_switch(base.trace_f, base.phases, num, den)
                if k is None or k >= r.phases:
                    assert (crit == O.STATIC_OR).all(), label
                else:
                    assert (crit[:k] == O.STATIC_OR).all() and (crit[k:] == then).all(), (label, k)
                rep = O.phased(g, 0, 0, crit_seq=crit.astype(np.uint32))
                assert r.phases == rep.phases and r.stats["sum_f"] == rep.sum_f, label
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), rep.phase_of), label
        for bad in ((O.SIMPLE_OR, O.STATIC_OR, 1, 2), (O.STATIC_OR, 0, 1, 2), (O.STATIC_OR, O.SIMPLE_OR, 0, 2),
                    (O.STATIC_OR, O.SIMPLE_OR, 3, 2), (O.IN_STATIC, O.OUT_STATIC, 1, 2)):
            with pytest.raises(B.SsspError):
                B.solve_switch(dg, 0, bad[0], bad[1], (bad[2], bad[3]))
        dg.close()


@pytest.mark.parametrize("cfg", [dict(use_graph=1), dict(queue=0), dict(use_graph=1, queue=0, scan_blocks=7)])
def test_switched_solve_launch_shapes(B, cfg):
    """The switched solve with captured six-phase graphs in the second stage (which starts at a
    16-phase boundary, mostly not a multiple of six) and with the dense scan in the first stage."""
    g = G.er(20011, 10, 1, 5000, 65)
    dg = B.DeviceGraph.from_graph(g)
    dg.set_launch(**cfg)
    dj, _ = O.dijkstra(g, 0)
    base = O.phased(g, 0, O.STATIC_OR, trace_cap=1 << 20)
    then = O.CRIT["IN_SIMPLE"] | O.OUT_STATIC
    for num, den in ((1, 2), (1, 4)):
        r = B.solve_switch(dg, 0, O.STATIC_OR, then, (num, den), phase_of=True, trace_cap=g.n + 4)
        crit = np.asarray(r.trace["criterion"])
        k = expected_switch(base.trace_f, base.phases, num, den)
        assert k is not None and 0 < k < r.phases, (cfg, k)
        assert (crit[:k] == O.STATIC_OR).all() and (crit[k:] == then).all(), (cfg, k)
        rep = O.phased(g, 0, 0, crit_seq=crit.astype(np.uint32))
        assert np.array_equal(r.dist_u64(), dj) and r.phases == rep.phases, cfg
        assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), rep.phase_of), cfg
    dg.close()


def test_max_weight_minima_every_static_path(B):
    """A real static minimum of 2^32 - 1 is not an empty edge set (hand traces MAXW_IN, MAXW_OUT):
    queue arrays, the dense scan, the one-workgroup kernel and the batched kernel all settle the
    hand-derived sets and reach the oracle's distances; the single-query batch counts its phases."""
    import json, os
    fix = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_traces.json")))
    for key in ("MAXW_IN", "MAXW_OUT"):
        ent = fix["graphs"][key]
        g = G.from_edges(ent["n"], ent["edges"])
        for name, sets in ent["phases"].items():
            c = {"IN_STATIC": O.IN_STATIC, "OUT_STATIC": O.OUT_STATIC, "STATIC_OR": O.STATIC_OR}[name]
            for queue in (2, 1, 0):
                dg = B.DeviceGraph.from_graph(g)
                dg.set_launch(queue=queue)
                r = B.solve_ex(dg, 0, c, phase_of=True)
                po = r.phase_of.cpu().numpy().view(np.uint32)
                got = [[v for v in range(g.n) if po[v] == p] for p in range(1, r.phases + 1)]
                assert got == sets, (key, name, queue, got)
                assert [int(x) for x in r.dist_u64()] == ent["dist"], (key, name, queue)
                dg.set_launch(single=1)
                r = B.solve(dg, 0, c)
                assert [int(x) for x in r.dist_u64()] == ent["dist"] and r.phases == len(sets), (key, name)
                dg.close()
            dg = B.DeviceGraph.from_graph(g)
            dists, phases = B.solve_batch([dg, dg], [0, 0], c)
            for d, ph in zip(dists, phases):
                assert [int(x) for x in B.to_u64(d)] == ent["dist"] and int(ph) == len(sets), (key, name)
            dg.close()


def test_delta_stepping_hand_traces(B):
    """The hand-traced Delta-stepping runs (tests/golden/delta_hand_traces.json) on the GPU: distances,
    rounds and buckets as traced by hand, and the per-round frontier sizes of the trace."""
    import json, os
    fix = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "delta_hand_traces.json")))
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        dg = B.DeviceGraph.from_graph(g)
        r = B.delta_step_ex(dg, 0, [ent["delta"]], trace_cap=64)
        assert [int(x) for x in r.dist_u64()] == ent["dist"], key
        assert r.phases == ent["rounds"] and r.stats["buckets"] == ent["buckets"], (key, r.phases)
        light = [len(f) for b in ent["frontiers"] for f in b]
        got = [int(s) for s, k in zip(r.trace["settled"], r.trace["criterion"]) if int(k) != 2]
        assert got == light, (key, got, light)
        dg.close()


APPROX = [("DIJK|IN_APPROX", O.DIJK | O.IN_APPROX), ("DIJK|OUT_APPROX", O.DIJK | O.OUT_APPROX),
          ("DIJK|IN_APPROX|OUT_APPROX", O.DIJK | O.IN_APPROX | O.OUT_APPROX), ("OUT_APPROX", O.OUT_APPROX)]


def check_approx(B, g, src, crit, k, label):
    dg = B.DeviceGraph.from_graph(g)
    ref = O.phased(g, src, crit, approx_k=k)
    r = B.solve_approx(dg, src, crit, k, phase_of=True, trace_cap=ref.phases + 4)
    assert np.array_equal(r.dist_u64(), ref.dist), label
    assert r.phases == ref.phases, (label, r.phases, ref.phases)
    assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), label
    assert r.stats["sum_f"] == ref.sum_f and r.stats["relax_edges"] == ref.relax_edges, label
    assert np.array_equal(r.trace["settled"], ref.trace_s), label
    dg.close()


def test_approximate_criteria_match_oracle(B):
    """sssp_solve_approx (the GPU evaluates the kept minima in closed form from each neighbour's settle
    phase) against the oracle (which maintains them as the paper describes: lowered on U -> F, changes
    counted on F -> S, recomputed every k-th change): hand traces, random multigraphs, medium graphs,
    k in {0, 1, 2, 5}."""
    import json, os
    fix = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "approx_hand_traces.json")))
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        c = {"DIJK|IN_APPROX": O.DIJK | O.IN_APPROX, "DIJK|OUT_APPROX": O.DIJK | O.OUT_APPROX}[ent["criterion"]]
        for k, sets in ent["phases"].items():
            dg = B.DeviceGraph.from_graph(g)
            r = B.solve_approx(dg, 0, c, int(k), phase_of=True)
            po = r.phase_of.cpu().numpy().view(np.uint32)
            assert [[v for v in range(g.n) if po[v] == p] for p in range(1, r.phases + 1)] == sets, (key, k)
            dg.close()
    for g in small_cases()[:30]:
        for name, c in APPROX:
            for k in (0, 1, 3):
                check_approx(B, g, 0, c, k, "%s/%s/k%d" % (g.name, name, k))
    for g in [G.er(1 << 14, 8, 1, 1000, 61), G.rmat(13, 16, 1, 1 << 16, 62), G.grid(61, 47, 1, 1 << 16, 63)]:
        src = int(G.sources(g, 1, 64)[0])
        for name, c in APPROX[:3]:
            for k in (0, 1, 2, 5):
                check_approx(B, g, src, c, k, "%s/%s/k%d" % (g.name, name, k))


def test_approximate_rejects_other_bits(B):
    dg = B.DeviceGraph.from_graph(G.er(100, 3, 1, 10, 65))
    for c in (0, O.STATIC_OR, O.IN_APPROX | O.IN_FULL):
        with pytest.raises(B.SsspError):
            B.solve_approx(dg, 0, c, 2)
