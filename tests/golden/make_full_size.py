"""Write the oracle's expected values for the full-size workloads (calls only oracle/ and graphgen).

usage: python tests/golden/make_full_size.py JOB [JOB ...]
  JOB = <graph>:<what>, graph in {er22, rmat22, grid2048}, what in
  {dist, STATIC_OR, IN_STATIC, OUT_STATIC, SIMPLE_OR, FULL_OR, delta12, delta14, delta16}.
Each job writes tests/golden/full/<graph>_<what>_s<source>.json with, for `dist`, a SHA-256 of the
little-endian uint64 distance array, 256 sampled (vertex, distance) pairs and the reach counts; for
a criterion, phases / summed fringe sizes / relaxations; for deltaK (Delta = 2^K), rounds and buckets.
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
    "er22": lambda: G.config_er_large(seed=1),
    "rmat22": lambda: G.config_rmat(seed=1),
    "grid2048": lambda: G.config_grid(seed=1),
}


def sources_for(name, g):
    if name == "er22":
        return [0]
    return [int(s) for s in G.sources(g, 2, 11)]


def run(job):
    gname, what = job.split(":")
    g = GRAPHS[gname]()
    for src in sources_for(gname, g):
        t = time.time()
        rec = {"graph": gname, "source": src, "n": g.n, "m": g.m}
        if what == "dist":
            d, hops = O.dijkstra(g, src)
            reach = d != O.INF
            rec["sha256"] = hashlib.sha256(d.astype("<u8").tobytes()).hexdigest()
            idx = np.linspace(0, g.n - 1, 256).astype(np.int64)
            rec["sample"] = [[int(i), int(d[i])] for i in idx]
            rec["n_reach"], rec["m_reach"] = O.reach_stats(g, d)
            rec["max_hop"] = int(hops[reach].max())
        elif what.startswith("delta"):
            r = O.delta_step(g, src, [1 << int(what[5:])])
            rec.update(rounds=r.rounds, buckets=r.buckets)
        else:
            c = {"STATIC_OR": O.STATIC_OR, "SIMPLE_OR": O.SIMPLE_OR, "FULL_OR": O.FULL_OR}.get(what) or O.CRIT[what]
            r = O.phased(g, src, c, trace_cap=0)
            rec.update(criterion=what, phases=r.phases, sum_f=r.sum_f, relax_edges=r.relax_edges,
                       n_reach=r.n_reach, m_reach=r.m_reach)
        rec["oracle_seconds"] = round(time.time() - t, 1)
        os.makedirs(OUT, exist_ok=True)
        path = os.path.join(OUT, "%s_%s_s%d.json" % (gname, what, src))
        json.dump(rec, open(path, "w"), indent=1)
        print("wrote", path, rec.get("phases", rec.get("rounds", "")), rec["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    for j in sys.argv[1:]:
        run(j)
