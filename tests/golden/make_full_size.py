"""Write the oracle's expected values for the full-size workloads (calls only oracle/ and graphgen).

usage: python tests/golden/make_full_size.py JOB [JOB ...]
  JOB = <graph>:<what>[:<sources>], graph in {er16k, er22, er23, rmat22, grid2048}, what in
  {dist, STATIC_OR, IN_STATIC, OUT_STATIC, SIMPLE_OR, FULL_OR, IN_FULL|OUT_WEAK, delta12, delta14, delta16};
  sources = comma-separated indices into the graph's source list (default: all of them).
  JOB = batch writes the per-query expectations of the 512-query batch workload.
Each job writes tests/golden/full/<graph>_<what>_s<source>.json with, for `dist`, a SHA-256 of the
little-endian uint64 distance array, 256 sampled (vertex, distance) pairs and the reach counts; for
a criterion, phases / summed fringe sizes / relaxations and the distance SHA-256; for deltaK
(Delta = 2^K), rounds, buckets and the distance SHA-256. The batch job writes batch_c4.json: per
query (graph index, source, n) the distance SHA-256, the reach counts and the IN_STATIC|OUT_STATIC
phase count.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as G  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full")

GRAPHS = {
    "er16k": lambda: G.config_small(seed=1),
    "er22": lambda: G.config_er_large(seed=1),
    "er23": lambda: G.config_er_large(seed=1, log2n=23),
    "rmat22": lambda: G.config_rmat(seed=1),
    "grid2048": lambda: G.config_grid(seed=1),
}
CRITS = {"STATIC_OR": O.STATIC_OR, "SIMPLE_OR": O.SIMPLE_OR, "FULL_OR": O.FULL_OR,
         "IN_FULL|OUT_WEAK": O.IN_FULL | O.OUT_WEAK}


def sources_for(name, g):
    """Source 0 on the random graphs; on R-MAT and the grid the 8 seeded sources the benchmark uses."""
    if name.startswith("er"):
        return [0]
    return [int(s) for s in G.sources(g, 8, 11)]


def sha(d):
    return hashlib.sha256(np.ascontiguousarray(d).astype("<u8").tobytes()).hexdigest()


def file_tag(what):
    return what.replace("|", "_")


def run(job):
    if job == "batch":
        return run_batch()
    parts = job.split(":")
    gname, what = parts[0], parts[1]
    g = GRAPHS[gname]()
    srcs = sources_for(gname, g)
    if len(parts) > 2:
        srcs = [srcs[int(i)] for i in parts[2].split(",")]
    for src in srcs:
        t = time.time()
        rec = {"graph": gname, "source": src, "n": g.n, "m": g.m}
        if what == "dist":
            d, hops = O.dijkstra(g, src)
            reach = d != O.INF
            rec["sha256"] = sha(d)
            idx = np.linspace(0, g.n - 1, 256).astype(np.int64)
            rec["sample"] = [[int(i), int(d[i])] for i in idx]
            rec["n_reach"], rec["m_reach"] = O.reach_stats(g, d)
            rec["max_hop"] = int(hops[reach].max())
        elif what.startswith("delta"):
            r = O.delta_step(g, src, [1 << int(what[5:])])
            rec.update(rounds=r.rounds, buckets=r.buckets, dist_sha256=sha(r.dist))
        else:
            c = CRITS.get(what) or O.CRIT[what]
            r = O.phased(g, src, c, trace_cap=0)
            rec.update(criterion=what, phases=r.phases, sum_f=r.sum_f, relax_edges=r.relax_edges,
                       improving=r.improving, n_reach=r.n_reach, m_reach=r.m_reach, dist_sha256=sha(r.dist))
        rec["oracle_seconds"] = round(time.time() - t, 1)
        os.makedirs(OUT, exist_ok=True)
        path = os.path.join(OUT, "%s_%s_s%d.json" % (gname, file_tag(what), src))
        json.dump(rec, open(path, "w"), indent=1)
        print("wrote", path, rec.get("phases", rec.get("rounds", "")), rec["oracle_seconds"], "s", flush=True)


def run_batch():
    t = time.time()
    graphs, queries = G.batch_workload(seed=7)
    recs = []
    for gi, src in queries:
        g = graphs[gi]
        d, _ = O.dijkstra(g, src)
        r = O.phased(g, src, O.STATIC_OR, trace_cap=0)
        assert np.array_equal(r.dist, d)
        n_reach, m_reach = O.reach_stats(g, d)
        recs.append({"graph": gi, "source": src, "n": g.n, "m": g.m, "sha256": sha(d), "n_reach": n_reach,
                     "m_reach": m_reach, "phases": r.phases})
    rec = {"workload": "batch_workload(seed=7): 64 graphs, 8 sources each", "criterion": "STATIC_OR",
           "queries": recs, "oracle_seconds": round(time.time() - t, 1)}
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, "batch_c4.json")
    json.dump(rec, open(path, "w"), indent=0)
    print("wrote", path, len(recs), rec["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    for j in sys.argv[1:]:
        run(j)
