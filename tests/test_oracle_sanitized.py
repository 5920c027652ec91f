"""The CPU oracle and the input generators under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_main.c drives oracle.c and graphgen/gen.c, built with gcc -fsanitize=address,undefined
(host code only), over the hand-traced graphs, 400 random multigraphs (zero weights, self-loops,
parallel edges, unreachable parts), the Delta-stepping closed forms (Delta = 1 and Delta above the
largest distance) and generated random, R-MAT and grid graphs. A sanitizer report ends the run with
a non-zero status; every printed figure must equal the ordinary -O2 build's.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen as G
import oracle as O


HERE = os.path.dirname(os.path.abspath(__file__))
CRITS = [1, 2, 4, 8, 16, 32, 64, 128, 6, 24, 160, 96, 769]  # same list and order as the driver (769: approx, k 2)


def fnv(data: bytes) -> int:
    h = 14695981039346656037
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("san") / "orc_san")
    return O.build_sanitized(exe)


def graph_block(g, src, deltas):
    lines = ["G %d %d %d %d %s" % (g.n, g.m, src, len(deltas), " ".join(str(int(d)) for d in deltas))]
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            lines.append("%d %d %d" % (u, int(g.col[e]), int(g.w[e])))
    return "\n".join(lines)


def expected_line(g, src, deltas):
    d, _ = O.dijkstra(g, src)
    n_reach = int((d != O.INF).sum())
    parts = ["OK", str(g.n), str(g.m), str(src), str(fnv(d.astype("<u8").tobytes())), str(n_reach)]
    for c in CRITS:
        r = O.phased(g, src, c, approx_k=2)
        parts += [str(r.phases), str(r.sum_f)]
    for dl in deltas:
        r = O.delta_step(g, src, [int(dl)])
        parts += [str(r.rounds), str(r.buckets)]
    return " ".join(parts)


def run_driver(exe, text):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, "sanitized oracle failed (status %d):\n%s" % (p.returncode, p.stderr[-3000:])
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-3000:]
    return p.stdout.splitlines()


def test_oracle_under_sanitizers(driver):
    cases = []
    fix = json.load(open(os.path.join(HERE, "golden", "hand_traces.json")))
    for ent in fix["graphs"].values():
        cases.append((G.from_edges(ent["n"], ent["edges"]), 0, [1, 2, 5]))
    dfix = json.load(open(os.path.join(HERE, "golden", "delta_hand_traces.json")))
    for ent in dfix["graphs"].values():
        cases.append((G.from_edges(ent["n"], ent["edges"]), 0, [ent["delta"]]))
    for s in range(400):
        x = G.u64_stream(s, 5, 3)
        n = 2 + int(x[0] % np.uint64(30))
        m = int(x[1] % np.uint64(4 * n + 1))
        wmax = [1, 3, 10, 1000, 0xFFFFFFFF][int(x[2] % np.uint64(5))]
        g = G.random_small(n, m, wmax, 31000 + s)
        deltas = [3]
        if s % 3 == 0 and (g.w.size == 0 or int(g.w.min()) >= 1):  # Delta closed forms
            d, _ = O.dijkstra(g, 0)
            reach = d != O.INF
            deltas = [1, int(d[reach].max()) + 1]
        cases.append((g, 0, deltas))
    text = "\n".join(graph_block(g, s, dl) for g, s, dl in cases) + "\n"
    out = run_driver(driver, text)
    assert len(out) == len(cases)
    for (g, s, dl), line in zip(cases, out):
        assert line == expected_line(g, s, dl), g.name


def test_generators_under_sanitizers(driver):
    specs = [("E", 3000, 8, 1, 1000, 3), ("R", 11, 16, 1, 1 << 16, 4), ("D", 41, 29, 1, 1 << 16, 5)]
    text = "\n".join(" ".join(str(x) for x in sp) for sp in specs) + "\n"
    out = run_driver(driver, text)
    assert len(out) == 2 * len(specs)
    for i, (kind, a, b, wlo, whi, seed) in enumerate(specs):
        g = G.er(a, b, wlo, whi, seed) if kind == "E" else G.rmat(a, b, wlo, whi, seed) if kind == "R" \
            else G.grid(a, b, wlo, whi, seed)
        h = fnv(g.row_ptr.astype("<u8").tobytes() + g.col.astype("<u4").tobytes() + g.w.astype("<u4").tobytes())
        assert out[2 * i] == "GEN %d" % h, kind
        src = int(G.sources(g, 1, seed)[0])
        assert out[2 * i + 1] == expected_line(g, src, []), kind
