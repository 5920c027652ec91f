"""Phase-scaling study (the method's own measurements, on the GPU): phases and summed fringe
sizes of the phased algorithm for every criterion, including the clairvoyant ORACLE, on uniform
random graphs and R-MAT (Kronecker) graphs with m/n = 10 and near-continuous uniform weights, for
growing n; least-squares fits phases = b * n^c (ORACLE also a * log2 n) and sum|F| = b * n^c, the
forms the paper fits to its simulations (Section 4, tables of phases and of summed |F|).

    python -m paper_1903_12085_amd.study [--log2n-max 22] [--seeds 3] [--out study.json]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding as B


def fit_power(ns, ys):
    """(b, c) of y = b * n^c by least squares on logs."""
    c, lb = np.polyfit(np.log(np.asarray(ns, float)), np.log(np.asarray(ys, float)), 1)
    return float(math.exp(lb)), float(c)


def fit_log2(ns, ys):
    """a of y = a * log2 n by least squares through the origin."""
    x = np.log2(np.asarray(ns, float))
    y = np.asarray(ys, float)
    return float((x @ y) / (x @ x))


CRITERIA = {"out_static": B.OUT_STATIC, "in_static": B.IN_STATIC, "static_or": B.STATIC_OR,
            "out_simple": B.OUT_SIMPLE, "in_simple": B.IN_SIMPLE, "simple_or": B.SIMPLE_OR,
            "out": B.OUT_FULL, "in": B.IN_FULL, "full_or": B.FULL_OR}


def make_graph(family, lg, seed, degree):
    """Uniform: every vertex gets `degree` distinct random targets; Kronecker: R-MAT with the
    paper's initiator (.57, .19, .19, .05) and `degree` sampled edges per vertex. Weights uniform
    in [1, 2^20) (near-continuous, as the paper's real weights)."""
    import graphgen as G
    if family == "uniform":
        return G.er(1 << lg, degree, 1, (1 << 20) - 1, seed)
    return G.rmat(lg, degree, 1, (1 << 20) - 1, seed)


def run(family="uniform", log2n_min=12, log2n_max=22, seeds=3, degree=10, log=print):
    import graphgen as G
    rows = []
    for lg in range(log2n_min, log2n_max + 1):
        for seed in range(1, seeds + 1):
            t = time.time()
            g = make_graph(family, lg, 1000 + seed, degree)
            dg = B.DeviceGraph.from_graph(g)
            src = int(G.sources(g, 1, 1000 + seed)[0])  # a vertex with out-edges
            row = {"family": family, "log2n": lg, "n": g.n, "m": g.m, "seed": 1000 + seed, "source": src}
            for name, crit in CRITERIA.items():
                r = B.solve_ex(dg, src, crit)
                row[name] = {"phases": r.phases, "sum_f": int(r.stats["sum_f"])}
            ref = B.solve(dg, src, B.STATIC_OR).dist
            r = B.solve_oracle(dg, src, ref, phase_of=False)
            row["oracle"] = {"phases": r.phases, "sum_f": int(r.stats["sum_f"])}
            rows.append(row)
            log("%s n=2^%d seed %d: %s (%.1fs)" % (family, lg, seed,
                                                    {k: row[k]["phases"] for k in list(CRITERIA) + ["oracle"]},
                                                    time.time() - t))
            del dg
    fits = {}
    ns = [r["n"] for r in rows]
    for name in list(CRITERIA) + ["oracle"]:
        ph = [r[name]["phases"] for r in rows]
        sf = [r[name]["sum_f"] for r in rows]
        fits[name] = {"phases_b_c": fit_power(ns, ph), "sum_f_b_c": fit_power(ns, sf)}
        if name == "oracle":
            fits[name]["phases_a_log2n"] = fit_log2(ns, ph)
    return rows, fits


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--log2n-min", type=int, default=12)
    ap.add_argument("--log2n-max", type=int, default=22)
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--families", default="uniform,kronecker")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    res = {}
    for fam in args.families.split(","):
        rows, fits = run(fam, args.log2n_min, args.log2n_max, args.seeds)
        res[fam] = {"rows": rows, "fits": fits}
        print(fam, json.dumps({k: {"phases": [round(x, 3) for x in v["phases_b_c"]],
                                   "sum_f": [round(x, 3) for x in v["sum_f_b_c"]]} for k, v in fits.items()}))
    if args.out:
        json.dump(res, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
