"""Pins for the CPU oracle (no GPU): brute force, closed forms, hand traces, invariants.

Each test pins the oracle to something other than itself:
  * Bellman-Ford brute force on random tiny multigraphs (Section 2 problem definition);
  * closed forms for paths, out-stars and unit-weight grids;
  * hand-derived per-phase settled sets (tests/golden/hand_traces.json) for the criteria of
    Section 3 (equations crit:in, crit:out, crit:outweak, crit:instatic, crit:outstatic,
    crit:insimple, crit:outsimple);
  * the ORACLE lower bound of Section 3 (a vertex can be correct no earlier than one phase
    after its predecessor on a minimum-hop shortest path), label setting (every reachable
    vertex settled exactly once), and the Delta-stepping closed forms.
"""
import json
import os

import numpy as np
import pytest

import graphgen as G
import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ALL_CRITS = list(O.CRIT.items()) + [("STATIC_OR", O.STATIC_OR), ("SIMPLE_OR", O.SIMPLE_OR),
                                   ("FULL_OR", O.FULL_OR), ("IN_FULL|OUT_WEAK", O.IN_FULL | O.OUT_WEAK)]


def small_graphs(count, seed0=0):
    for s in range(count):
        x = G.u64_stream(seed0 + s, 5, 3)
        n = 2 + int(x[0] % np.uint64(30))
        m = int(x[1] % np.uint64(4 * n + 1))
        wmax = [1, 3, 10, 1000][int(x[2] % np.uint64(4))]
        yield G.random_small(n, m, wmax, seed0 + s)


def test_dijkstra_equals_bellman_ford_on_random_multigraphs():
    for g in small_graphs(400):
        src = 0
        d, hops = O.dijkstra(g, src)
        bf = O.bellman_ford(g, src)
        assert np.array_equal(d, bf), g.name
        # every reachable vertex != src has a tight in-edge; no edge can be relaxed further
        for u in range(g.n):
            for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                v, c = int(g.col[e]), int(g.w[e])
                if d[u] != O.INF:
                    assert int(d[v]) <= int(d[u]) + c


def test_hops_are_minimum_edge_counts_among_shortest_paths():
    # brute force: BFS-like layered relaxation counting edges (k-edge-limited shortest paths)
    for g in small_graphs(120, 1000):
        d, hops = O.dijkstra(g, 0)
        n = g.n
        best = [None] * n  # best[v] = cost with <= k edges
        best[0] = 0
        first_k = {0: 0}
        for k in range(1, n + 1):
            nb = list(best)
            for u in range(n):
                if best[u] is None:
                    continue
                for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                    v, c = int(g.col[e]), int(g.w[e])
                    if nb[v] is None or best[u] + c < nb[v]:
                        nb[v] = best[u] + c
            best = nb
            for v in range(n):
                if v not in first_k and best[v] is not None and best[v] == int(d[v]):
                    first_k[v] = k
        for v in range(n):
            if d[v] == O.INF:
                assert hops[v] == 0xFFFFFFFF
            else:
                assert hops[v] == first_k[v]


def test_path_graph_closed_form():
    ws = [3, 1, 4, 1, 5, 9, 2, 6]
    g = G.path(len(ws) + 1, ws)
    d, _ = O.dijkstra(g, 0)
    assert list(d) == list(np.cumsum([0] + ws))
    for name, c in ALL_CRITS:
        # only one vertex is ever queued on a path, so every criterion needs n phases
        assert O.phased(g, 0, c, check=True, dist_ref=d).phases == g.n, name


def test_out_star_closed_form():
    ws = [7, 3, 3, 9, 1, 7, 7]
    g = G.out_star(len(ws), ws)
    d, _ = O.dijkstra(g, 0)
    assert list(d[1:]) == ws
    for name, c in ALL_CRITS:
        r = O.phased(g, 0, c, check=True, dist_ref=d)
        if c == O.DIJK:
            assert r.phases == 1 + len(set(ws)), name  # one phase per distinct leaf distance
        else:
            assert r.phases == 2, name  # leaves have a single in-edge from S / no out-edges


@pytest.mark.parametrize("W,H", [(1, 1), (5, 1), (6, 4), (9, 9)])
def test_unit_grid_manhattan_closed_form(W, H):
    g = G.grid(W, H, 1, 1, 3)
    for src in {0, (H // 2) * W + W // 2}:
        d, hops = O.dijkstra(g, src)
        sx, sy = src % W, src // W
        expect = [abs(x - sx) + abs(y - sy) for y in range(H) for x in range(W)]
        assert list(d) == expect
        assert list(hops) == expect
        for name, c in ALL_CRITS:
            # every vertex at distance k settles in phase k + 1 under every criterion
            r = O.phased(g, src, c, check=True, dist_ref=d)
            assert r.phases == 1 + max(expect), name
            assert list(r.phase_of) == [1 + e for e in expect], name


def test_hand_traces():
    fix = json.load(open(os.path.join(HERE, "golden", "hand_traces.json")))
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        d, _ = O.dijkstra(g, 0)
        assert [int(x) for x in d] == ent["dist"], key
        for name, sets in ent["phases"].items():
            c = O.CRIT.get(name) or {"STATIC_OR": O.STATIC_OR, "SIMPLE_OR": O.SIMPLE_OR,
                                     "FULL_OR": O.FULL_OR}[name]
            r = O.phased(g, 0, c, check=True, dist_ref=d)
            got = [[v for v in range(ent["n"]) if r.phase_of[v] == p] for p in range(1, r.phases + 1)]
            assert got == sets, (key, name)


def test_invariants_on_random_graphs():
    """check mode asserts, on every snapshot: DIJK-set inside each criterion's set (completeness),
    X-STATIC => X-SIMPLE => (OUTWEAK =>) X, and certified vertices correct (soundness)."""
    for g in small_graphs(250, 5000):
        d, hops = O.dijkstra(g, 0)
        n_reach, m_reach = O.reach_stats(g, d)
        lower = 1 + int(hops[d != O.INF].max())
        distinct = len(set(int(x) for x in d[d != O.INF]))
        for name, c in ALL_CRITS:
            r = O.phased(g, 0, c, check=True, dist_ref=d)
            assert r.n_reach == n_reach and r.m_reach == m_reach
            assert int(r.trace_s.sum()) == n_reach  # label setting: each vertex settled once
            assert lower <= r.phases <= n_reach, name
            assert r.sum_f >= n_reach
            if c == O.DIJK:
                # with zero weights, equal distances may still need separate phases
                assert r.phases >= distinct
        r = O.phased(g, 0, O.DIJK)
        if g.w.size == 0 or int(g.w.min()) >= 1:
            assert r.phases == distinct


def test_trace_counts_respect_strength_chain():
    g = G.er(300, 4, 1, 100, 11)
    d, _ = O.dijkstra(g, 0)
    r = O.phased(g, 0, O.STATIC_OR, check=True, dist_ref=d)
    cnt = r.trace_counts  # columns in bit order DIJK, IN_STATIC, OUT_STATIC, IN_SIMPLE, ...
    assert (cnt[:, 1] <= cnt[:, 3]).all() and (cnt[:, 3] <= cnt[:, 5]).all()
    assert (cnt[:, 2] <= cnt[:, 4]).all() and (cnt[:, 4] <= cnt[:, 6]).all() and (cnt[:, 6] <= cnt[:, 7]).all()
    assert (cnt[:, 0] >= 1).all()


def test_stronger_criteria_take_no_more_phases_on_er():
    # not a theorem pointwise across runs, but on these seeds the measured order must hold
    g = G.er(2000, 8, 1, 1000, 3)
    ph = {name: O.phased(g, 0, c).phases for name, c in ALL_CRITS}
    assert ph["FULL_OR"] <= ph["STATIC_OR"] and ph["IN_FULL"] <= ph["IN_STATIC"]
    assert ph["DIJK"] > ph["STATIC_OR"]


def test_crit_seq_replays_fixed_criterion():
    g = G.er(500, 6, 1, 50, 4)
    a = O.phased(g, 0, O.STATIC_OR)
    b = O.phased(g, 0, 0, crit_seq=[O.STATIC_OR])
    assert a.phases == b.phases and np.array_equal(a.phase_of, b.phase_of)


def test_delta_stepping_closed_forms():
    for g in small_graphs(150, 9000):
        if g.w.size and int(g.w.min()) == 0:
            continue
        d, hops = O.dijkstra(g, 0)
        reach = d != O.INF
        distinct = len(set(int(x) for x in d[reach]))
        r1 = O.delta_step(g, 0, [1])
        assert np.array_equal(r1.dist, d)
        assert r1.rounds == 2 * distinct  # one (empty) light round + one heavy round per distance
        big = int(d[reach].max()) + 1
        rb = O.delta_step(g, 0, [big])
        assert np.array_equal(rb.dist, d)
        assert rb.rounds == int(hops[reach].max()) + 2  # synchronous Bellman-Ford + heavy round
        for delta in (2, 7, 100):
            assert np.array_equal(O.delta_step(g, 0, [delta]).dist, d)


def test_delta_stepping_variable_widths_keep_distances():
    g = G.er(3000, 6, 1, 1 << 16, 8)
    d, _ = O.dijkstra(g, 0)
    seq = [1 << 12, 1 << 16, 1 << 14, 1 << 12, 1 << 16]
    r = O.delta_step(g, 0, seq, trace_cap=64)
    assert np.array_equal(r.dist, d)
    assert list(r.trace_delta[:5]) == seq


def test_static_minima_match_definition():
    g = G.random_small(25, 80, 50, 3)
    mi, mo = O.static_minima(g)
    for v in range(g.n):
        outs = [int(g.w[e]) for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1]))]
        ins = [int(g.w[e]) for u in range(g.n) for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1]))
               if int(g.col[e]) == v]
        assert mo[v] == (min(outs) if outs else 0xFFFFFFFF)
        assert mi[v] == (min(ins) if ins else 0xFFFFFFFF)


def test_config_small_static_or_runs_and_is_sound():
    g = G.config_small()
    d, hops = O.dijkstra(g, 0)
    r = O.phased(g, 0, O.STATIC_OR, check=True, dist_ref=d)
    assert r.n_reach == int((d != O.INF).sum()) > 0.99 * g.n  # a few vertices have no in-edge
    assert 1 + int(hops[d != O.INF].max()) <= r.phases < 1000


def test_delta_stepping_hand_traces():
    """Hand-traced Delta-stepping runs (tests/golden/delta_hand_traces.json): buckets needing several
    light rounds, a vertex re-relaxed inside its bucket, and light rounds that discover or lower a
    vertex at or past the window end, which must not join the bucket's next light round."""
    fix = json.load(open(os.path.join(HERE, "golden", "delta_hand_traces.json")))
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        r = O.delta_step(g, 0, [ent["delta"]], trace_cap=16)
        assert [int(x) for x in r.dist] == ent["dist"], key
        assert [int(x) for x in O.dijkstra(g, 0)[0]] == ent["dist"], key
        assert r.rounds == ent["rounds"] and r.buckets == ent["buckets"], (key, r.rounds, r.buckets)
        assert r.light_relax == ent["light_relax"] and r.heavy_relax == ent["heavy_relax"], key
        assert r.sum_frontier == ent["sum_frontier"] == sum(len(f) for b in ent["frontiers"] for f in b), key
        assert r.rounds == sum(len(b) for b in ent["frontiers"]) + r.buckets, key


def test_approximate_criteria_hand_traces():
    """Approximate criteria (Section 3, closing paragraphs) against hand-traced runs
    (tests/golden/approx_hand_traces.json) for several recomputation intervals k; k = 1 recomputes at
    every change, so it must also equal the exact IN (full) / OUT-WEAK run."""
    fix = json.load(open(os.path.join(HERE, "golden", "approx_hand_traces.json")))
    names = {"DIJK|IN_APPROX": (O.DIJK | O.IN_APPROX, O.IN_FULL),
             "DIJK|OUT_APPROX": (O.DIJK | O.OUT_APPROX, O.OUT_WEAK)}
    for key, ent in fix["graphs"].items():
        g = G.from_edges(ent["n"], ent["edges"])
        d, _ = O.dijkstra(g, 0)
        assert [int(x) for x in d] == ent["dist"], key
        c, exact = names[ent["criterion"]]
        for k, sets in ent["phases"].items():
            r = O.phased(g, 0, c, check=True, dist_ref=d, approx_k=int(k))
            got = [[v for v in range(ent["n"]) if r.phase_of[v] == p] for p in range(1, r.phases + 1)]
            assert got == sets, (key, k, got)
        ex = O.phased(g, 0, exact)
        assert list(ex.phase_of) == list(O.phased(g, 0, c, approx_k=1).phase_of), key


def test_approximate_criteria_invariants():
    """On random multigraphs and every k: sound (check mode compares each settled distance with
    Dijkstra), complete, at least as strong as the static criterion (DIJK and X-STATIC imply
    X-APPROX on every snapshot, asserted in check mode), k = 1 equal to the exact IN (full) /
    OUT-WEAK criteria, and phases between the ORACLE bound and the reachable vertex count."""
    for g in small_graphs(150, 12000):
        d, hops = O.dijkstra(g, 0)
        lower = 1 + int(hops[d != O.INF].max())
        n_reach = int((d != O.INF).sum())
        for c, exact in ((O.DIJK | O.IN_APPROX, O.IN_FULL), (O.DIJK | O.OUT_APPROX, O.OUT_WEAK),
                         (O.DIJK | O.IN_APPROX | O.OUT_APPROX, O.IN_FULL | O.OUT_WEAK)):
            for k in (0, 1, 2, 5):
                r = O.phased(g, 0, c | O.IN_STATIC | O.OUT_STATIC, check=True, dist_ref=d, approx_k=k)
                assert lower <= r.phases <= n_reach
                r = O.phased(g, 0, c, check=True, dist_ref=d, approx_k=k)
                assert lower <= r.phases <= n_reach
            assert list(O.phased(g, 0, c, approx_k=1).phase_of) == list(O.phased(g, 0, exact).phase_of)
